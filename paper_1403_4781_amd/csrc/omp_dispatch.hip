// Dispatch from a runtime tile choice to the instantiated fused-OMP kernels.
#include "omp_kernel.h"

namespace smdl_omp {
#define SMDL_OMP_TILE(EM, SM, G, TT) \
    extern template hipError_t launch_one<EM, SM, G, TT>(const OmpArgs&, int, int, hipStream_t);
#include "omp_table.inc"
#undef SMDL_OMP_TILE
}  // namespace smdl_omp

namespace {

struct TileEntry {
    int EM, SM, G, TT;
    hipError_t (*fn)(const OmpArgs&, int, int, hipStream_t);
    size_t (*lds)(int, int);
};

const TileEntry kTiles[] = {
#define SMDL_OMP_TILE(EM, SM, G, TT) \
    {EM, SM, G, TT, &smdl_omp::launch_one<EM, SM, G, TT>, &smdl_omp::omp_lds_size<SM, G, TT>},
#include "omp_table.inc"
#undef SMDL_OMP_TILE
};

// Smallest instantiated (EM, SM) that covers Kpad / lanes entries and s steps.
const TileEntry* find_tile(OmpTile t, int Kpad, int s) {
    if (t.lanes != 16 && t.lanes != 32 && t.lanes != 64) return nullptr;
    if (Kpad % (4 * t.lanes) != 0) return nullptr;
    const int E = Kpad / t.lanes;
    const TileEntry* best = nullptr;
    for (const TileEntry& e : kTiles) {
        if (e.G != t.lanes || e.TT != t.tt || e.EM < E || e.SM < s) continue;
        if (!best || e.EM < best->EM || (e.EM == best->EM && e.SM < best->SM)) best = &e;
    }
    return best;
}

}  // namespace

// LDS of the instantiation that serves (t, maxKpad, s) with signal copies of m_copy floats;
// 0 when there is none.
size_t omp_lds_bytes(OmpTile t, int maxKpad, int s, int m_copy) {
    const TileEntry* e = find_tile(t, maxKpad, s);
    return e ? e->lds(maxKpad, m_copy) : 0;
}

// A tile is usable when it is instantiated for (Kpad, s) and its LDS (alpha0 staging and the
// greedy-loop slots) fits in the 160 KB of a gfx950 workgroup.
bool omp_tile_supported(OmpTile t, int Kpad, int s) {
    const TileEntry* e = find_tile(t, Kpad, s);
    return e != nullptr && e->lds(Kpad, 0) <= SMDL_LDS_BYTES;
}

bool omp_y_lds(OmpTile t, int maxKpad, int s, int m, const float* const* Ys, int n_sets) {
    if (m % 4) return false;
    for (int i = 0; i < n_sets; ++i)
        if (reinterpret_cast<uintptr_t>(Ys[i]) & 15) return false;
    const TileEntry* e = find_tile(t, maxKpad, s);
    return e != nullptr && e->lds(maxKpad, m) <= SMDL_LDS_BYTES;
}

hipError_t launch_omp(OmpTile t, int maxKpad, int maxS, const OmpArgs& a, int max_items, int n_cu,
                      hipStream_t st) {
    const TileEntry* e = find_tile(t, maxKpad, maxS);
    if (!e || e->lds(maxKpad, a.y_lds ? a.m : 0) > SMDL_LDS_BYTES || a.max_kpad != maxKpad)
        return hipErrorInvalidValue;
    return e->fn(a, max_items, n_cu, st);
}

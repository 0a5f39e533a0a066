// OMP coding with no device allocation: the variant of smdl_omp_code for callers that cannot
// allocate (code under HIP graph capture, tight serving loops).  Its scratch memory (the packed
// dictionary fragments, the Gram matrix and the launch descriptors) is one file-scope device
// array per GPU, sized for the library's largest dictionary; its device address is taken once
// per device when a handle is created, and only that address is used on the host.
#include <cmath>
#include <cstring>

#include "smdl_api_internal.h"

namespace {

// Layout of the scratch array: the launch descriptors (and the work counter) and the atom
// exponents first, then the
// packed fragments (mpad x Kpad floats), their FP16 split (hi and lo, mpad x Kpad halves each),
// then the Gram matrix (Kpad rows of gld floats).
constexpr size_t DESC_BYTES = 4096;
constexpr size_t AEXP_BYTES = (size_t)SMDL_MAX_K * 4;                  // 4 KiB
constexpr size_t FRAG_BYTES = (size_t)SMDL_MAX_M * SMDL_MAX_K * 4;     // 1 MiB
constexpr size_t F16_BYTES = (size_t)SMDL_MAX_M * SMDL_MAX_K * 2 * 2;  // 1 MiB
constexpr size_t GRAM_BYTES = (size_t)SMDL_MAX_K * SMDL_MAX_K * 4;     // 4 MiB (gld <= 1024)
constexpr size_t SCRATCH_BYTES = DESC_BYTES + AEXP_BYTES + FRAG_BYTES + F16_BYTES + GRAM_BYTES;

__device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
void* g_scratch[MAX_DEVICES] = {};   // device address of `scratch` on each GPU (set up once)

struct Descs {
    PackDesc pd;
    GramDesc gd;
    OmpDesc od;
};
static_assert(sizeof(Descs) <= DESC_BYTES / 2, "descriptor block too large");

// The descriptors come in as kernel arguments and are stored into the scratch array, so that no
// host-to-device copy is queued.
__global__ void store_descs_kernel(Descs v, Descs* dst) {
    if (threadIdx.x == 0) *dst = v;
}

}  // namespace

// Called by smdl_create with h->device current: the device address of this GPU's scratch array.
smdl_status noalloc_setup(smdl_t h) {
    if (h->device < 0 || h->device >= MAX_DEVICES) return h->fail(SMDL_E_ARG, "device index too large");
    if (g_scratch[h->device]) return SMDL_OK;
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return h->hip(e != hipSuccess ? e : hipErrorInvalidSymbol, "scratch address");
    g_scratch[h->device] = p;
    return SMDL_OK;
}

extern "C" smdl_status smdl_omp_code_noalloc(smdl_t h, const float* D, int m, int K, const float* Y, int64_t N,
                                             int s_max, float eps, smdl_codes X, float* res_norm) {
    if (!h) return SMDL_E_ARG;
    h->err.clear();
    smdl_status st = check_dims(h, m, K, s_max);
    if (st != SMDL_OK) return st;
    if (N < 0) return h->fail(SMDL_E_ARG, "N must be >= 0");
    if (!(eps >= 0.f) || std::isinf(eps)) return h->fail(SMDL_E_ARG, "eps must be finite and >= 0");
    if ((st = check_codes(h, X, N, s_max)) != SMDL_OK) return st;
    if (N == 0) return SMDL_OK;
    if (!D || !Y) return h->fail(SMDL_E_ARG, "null pointer");
    if (N > (int64_t)INT32_MAX * 16) return h->fail(SMDL_E_SHAPE, "N too large");
    if (h->device < 0 || h->device >= MAX_DEVICES || !g_scratch[h->device])
        return h->fail(SMDL_E_STATE, "scratch memory of this device was not set up");
    const int mpad = pad64(m), Kpad = pad64(K), gld = gram_ld(Kpad);
    const size_t frag_bytes = (size_t)mpad * Kpad * 4, gram_bytes = (size_t)Kpad * gld * 4;
    if (frag_bytes > FRAG_BYTES || gram_bytes > GRAM_BYTES)
        return h->fail(SMDL_E_SHAPE, "dictionary too large for the fixed scratch memory (m <= 256, K <= 1024)");
    (void)hipSetDevice(h->device);
    unsigned char* base = static_cast<unsigned char*>(g_scratch[h->device]);
    Descs* dd = reinterpret_cast<Descs*>(base);
    int* queue = reinterpret_cast<int*>(base + DESC_BYTES / 2);   // work counter (zeroed by the launch)
    int32_t* aexp = reinterpret_cast<int32_t*>(base + DESC_BYTES);
    float4* frag = reinterpret_cast<float4*>(base + DESC_BYTES + AEXP_BYTES);
    uint16_t* fhi = reinterpret_cast<uint16_t*>(base + DESC_BYTES + AEXP_BYTES + FRAG_BYTES);
    uint16_t* flo = fhi + (size_t)mpad * Kpad;
    float* gram = reinterpret_cast<float*>(base + DESC_BYTES + AEXP_BYTES + FRAG_BYTES + F16_BYTES);

    const OmpTile tile = choose_tile(h, Kpad, s_max, false);
    if (!omp_tile_supported(tile, Kpad, s_max)) return h->fail(SMDL_E_UNSUPPORTED, "no OMP tile for this shape");
    const int T = 16 * tile.tt;
    Descs v;
    std::memset(&v, 0, sizeof(v));
    v.pd = PackDesc{D, frag, fhi, flo, aexp, K, Kpad};
    v.gd = GramDesc{frag, gram, Kpad, gld};
    v.od = OmpDesc{D, fhi, flo, aexp, gram, Y, N, 0, K, Kpad, s_max, gld};
    hipError_t e;
    hipLaunchKernelGGL(store_descs_kernel, dim3(1), dim3(64), 0, h->stream, v, dd);
    if ((e = hipGetLastError()) != hipSuccess) return h->hip(e, "descriptors");
    if ((e = launch_pack_dict_m(&dd->pd, 1, Kpad, m, mpad / 64, h->stream)) != hipSuccess) return h->hip(e, "pack");
    if ((e = launch_gram_batched(&dd->gd, 1, Kpad, mpad / 64, h->stream)) != hipSuccess) return h->hip(e, "gram");
    OmpArgs a{};
    a.desc = &dd->od;
    a.items = nullptr;
    a.n_items = (int)((N + T - 1) / T);
    a.queue = queue;
    a.max_kpad = Kpad;
    a.y_lds = omp_y_lds(tile, Kpad, s_max, m, &Y, 1) ? 1 : 0;
    a.m = m;
    a.mchunks = mpad / 64;
    a.eps2 = eps > 0.f ? eps * eps : 0.f;
    a.tau = SMDL_TAU;
    a.dep_tol = SMDL_DEP_TOL;
    a.idx = X.idx;
    a.coef = X.coef;
    a.nnz = X.nnz;
    a.res = res_norm;
    a.s_out = X.s_max;
    if ((e = launch_omp(tile, Kpad, s_max, a, a.n_items, h->n_cu, h->stream)) != hipSuccess) return h->hip(e, "omp launch");
    // under graph capture the work is only recorded; otherwise the call returns when it is done
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    if ((e = hipStreamIsCapturing(h->stream, &cap)) != hipSuccess) return h->hip(e, "capture status");
    if (cap != hipStreamCaptureStatusNone || (h->flags & SMDL_ASYNC)) return SMDL_OK;
    return h->hip(hipStreamSynchronize(h->stream), "omp");
}

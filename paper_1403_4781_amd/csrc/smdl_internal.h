// Internal declarations shared by the HIP translation units of libsmdl (gfx950 only).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "smdl.h"

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// Hard limits of the kernels (checked on the host before any launch).
constexpr int SMDL_MAX_M = 256;
constexpr int SMDL_MAX_K = 1024;
constexpr int SMDL_MAX_S = 16;
constexpr int SMDL_MAX_COMPOSED = 64;   // atoms of a composed code (s_1 s_2)
// LDS one gfx950 workgroup may use (static + dynamic), minus a margin for static variables.
constexpr size_t SMDL_LDS_BYTES = 160 * 1024 - 256;

// Dictionaries are padded to Kpad atoms (multiple of 64) and m to mpad (multiple of 64) with
// zeros.  The packed "fragment" layout feeds the 16x16x4 FP32 MFMA directly: for m-chunk c
// (64 rows), atom block b (16 atoms), sub-step q (0..3) and lane l, the float4 at index
// ((c * Kpad/16 + b) * 4 + q) * 64 + l holds D[atom 16b + l%16][row 64c + 16(l/16) + 4q .. +3].
inline int pad64(int x) { return (x + 63) / 64 * 64; }

// Row stride (floats) of the Gram matrices of one launch whose largest padded width is maxKpad:
// the next power of two, at least 256.  Every instantiated OMP tile reads G-row spans of
// EM * G <= this many floats, so the row loads need no bounds guard; columns past Kpad are zero.
inline int gram_ld(int maxKpad) {
    int ld = 256;
    while (ld < maxKpad) ld *= 2;
    return ld;
}

// FP16 split fragments of a dictionary for the correlations of the OMP kernel: atom k is scaled by
// 2^-aexp[k] (aexp[k] = the exponent that brings max_r |D[r][k]| into [0.5, 1); 0 for a zero
// atom) and split as hi = fp16(v), lo = fp16(v - hi).  For row block kb (16 rows), atom block b
// (16 atoms) and lane l, the four halves at ((kb * Kpad/16 + b) * 64 + l) * 4 are the rows
// 16 kb + 4 (l/16) .. + 3 of atom 16 b + l%16: the A operand of v_mfma_f32_16x16x16_f16.
inline int pad16(int x) { return (x + 15) / 16 * 16; }

// One dictionary and the signals coded against it.
struct OmpDesc {
    const float* D;       // the dictionary, K rows of m floats (explicit residuals)
    const void* fhi;      // FP16 split fragments, hi and lo halves (mpad x Kpad halves each)
    const void* flo;
    const int32_t* aexp;  // Kpad atom exponents of the split
    const float* gram;    // Kpad rows of gld floats, row-major Gram matrix (zero outside K x K)
    const float* Y;       // signals (m floats each)
    int64_t n;            // number of signals in this set
    int64_t out0;         // output row of signal 0 of this set
    int K, Kpad, s, gld;
};

// A tile of up to T signals of one descriptor.
struct OmpItem {
    int32_t desc;
    int32_t count;
    int64_t first;
};

struct OmpArgs {
    const OmpDesc* desc;     // descriptors (device)
    const OmpItem* items;    // work items (device); NULL = one descriptor, item i covers T*i..
    int n_items;             // number of items (or, with items == NULL, ceil(n / T))
    int* queue;              // unused (the persistent grid strides over the items)
    const int32_t* sig_list; // gather mode: signals to code are sig_list[0 .. *list_count)
    const int32_t* list_count;
    int m, mchunks;
    float eps2, tau, dep_tol;
    int32_t* idx;
    float* coef;
    int32_t* nnz;
    float* res;              // optional
    int s_out;               // ELL row stride of the output
    int max_kpad;            // widest padded dictionary of the launch (LDS layout)
    int y_lds;               // 1: copy each item's signals into LDS ahead of use (needs m % 4 == 0
                             // and 16-byte aligned signal arrays; see omp_y_lds)
};

// Tile configuration of the OMP kernel.
struct OmpTile {
    int lanes;   // lanes per signal: 16, 32, 64
    int tt;      // work item = 16 * tt signals
};

// Launchers (return hipError_t of the launch).
hipError_t launch_pack_dict_m(const void* dev_pack_desc, int n_dict, int max_kpad, int m,
                              int mchunks, hipStream_t st);
hipError_t launch_gram_batched(const void* dev_gram_desc, int n_dict, int max_kpad, int mchunks,
                               hipStream_t st);
bool omp_tile_supported(OmpTile t, int Kpad, int s);
// The fused OMP kernel on a persistent grid (work group b takes items b, b + grid, ...).  max_items bounds the
// number of work items (the exact count may live on the device, a.list_count).
hipError_t launch_omp(OmpTile t, int maxKpad, int maxS, const OmpArgs& a, int max_items, int n_cu,
                      hipStream_t st);
// LDS of the instantiation serving (t, maxKpad, s) with signal copies of m floats (0: none).
size_t omp_lds_bytes(OmpTile t, int maxKpad, int s, int m_copy);
// Whether the signal copies into LDS can be used: m % 4 == 0, every signal array 16-byte aligned
// and the tile's LDS with the copies within a work group's limit.
bool omp_y_lds(OmpTile t, int maxKpad, int s, int m, const float* const* Ys, int n_sets);

// Batched dictionary helpers (descriptor arrays live in device memory).
struct PackDesc {
    const float* D;   // m x K column-major
    float4* dfrag;
    void* fhi;        // FP16 split fragments (see OmpDesc), mpad x Kpad halves each
    void* flo;
    int32_t* aexp;    // Kpad atom exponents
    int K, Kpad;
};
struct GramDesc {
    const float4* dfrag;
    float* G;             // Kpad rows of ld floats; columns Kpad .. ld-1 are written as zeros
    int Kpad, ld;
};

// MOD descriptors.
struct ModDesc {
    const float* Y;          // signals of this set (m each), contiguous
    const int32_t* idx;      // ELL codes of this set
    const float* coef;
    const int32_t* nnz;
    int64_t n;               // signals
    int64_t atom0;           // first global atom id of this dictionary
    float* D;                // m x K dictionary (in/out)
    double* A;               // Kpad x Kpad FP64 workspace (products)
    double* W;               // (Kpad + m) x Kpad FP64 workspace (factorisation)
    double* Ld;              // Kpad x 32 FP64: the factored 32 x 32 diagonal blocks (multi-work-group solve)
    int K, Kpad;
    int s_stride;            // ELL row stride
    int pad_;
};

// The MOD chain for n_desc dictionaries.  arena: the products workspace M = [A; B] of every
// descriptor (arena_len doubles, the descriptors' A pointers inside it); with chunks > 1 every
// atom's products are split over that many blocks and part holds (chunks - 1) x arena_len
// doubles of partial sums.  solver: 0 picks the factorisation by the number of dictionaries,
// 1 forces the multi-work-group panels, 2 one work group per dictionary.  bcnt, bbase: NULL, or
// (fixed-order mode) two int32 arrays of mod_csc_blocks(max_n) x total_atoms entries each.
hipError_t launch_mod(const ModDesc* dev_desc, int n_desc, int m, int total_atoms, int64_t max_n, int32_t* cnt,
                      int32_t* fill, int32_t* ptr, int32_t* list_sig, float* list_coef, int32_t* status,
                      int max_kpad, double* arena, double* part, int64_t arena_len, int chunks, int solver,
                      int32_t* bcnt, int32_t* bbase, hipStream_t st);
// Blocks of the fixed-order code transpose (per-block counts and bases) for sets of at most max_n
// signals.
int64_t mod_csc_blocks(int64_t max_n);

// Misc kernels.
// *bad (zeroed by the caller) becomes 1 when any of the n floats at x is not finite.
hipError_t launch_check_finite(const float* x, int64_t n, int32_t* bad, hipStream_t st);
// out[:, n] = Y[:, perm[n]] for n < N; an entry outside [0, n_src) writes zeros and sets *bad.
hipError_t launch_gather_columns(const float* Y, const int64_t* perm, int64_t N, int64_t n_src, int m,
                                 float* out, int32_t* bad, hipStream_t st);
hipError_t launch_init_from_columns_batched(const void* dev_init_desc, int n_dict, int max_k,
                                            int m, hipStream_t st);
struct InitDesc {
    const float* Y;
    float* D;
    int K, pad_;
};
hipError_t launch_code_scales(const float* coef, const int32_t* nnz, int s_stride,
                              const int64_t* offsets_dev, int L, double* scales, hipStream_t st);
// Proposition 1 composition of Algorithm 1's codes (compose_codes_kernel); ls * ms <= 64,
// ls * ms <= os <= 64; *bad is set when perm holds an entry outside [0, N).
hipError_t launch_compose_codes(const int32_t* lidx, const float* lcoef, const int32_t* lnnz, int ls,
                                const int32_t* midx, const float* mcoef, const int32_t* mnnz, int ms,
                                const int64_t* offs_dev, const int64_t* aoff_dev, int L, const double* scales,
                                const int64_t* perm, int64_t N, int K, int32_t* oidx, float* ocoef, int32_t* onnz,
                                int os, int32_t* bad, hipStream_t st);
hipError_t launch_pool_scale(const float* Dloc, const int64_t* atom_off_dev, int L, int m,
                             const double* scales, float* Ytil, int64_t total_atoms,
                             hipStream_t st);
hipError_t launch_zero_i32(int32_t* p, int64_t n, hipStream_t st);
hipError_t launch_fill_codes(int32_t* idx, float* coef, int32_t* nnz, int64_t N, int s_stride,
                             hipStream_t st);

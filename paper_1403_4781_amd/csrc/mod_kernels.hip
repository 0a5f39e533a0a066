// MOD dictionary update (least squares D = Y X^T (X X^T)^{-1}) for one or many dictionaries.
//
//  1. csc_count / scan / csc_fill: transpose the ELL codes into per-atom lists of
//     (signal, coefficient) so that every atom's products can be gathered without atomics
//     on global memory (per-block counts in LDS, one global atomic per atom and block).
//  2. mod_products: one block per atom a (and per chunk of a long list): column a of
//     A = X X^T (FP64, LDS) and column a of B = Y X^T (FP64 register accumulation over the
//     atom's list), written below each other as column a of the augmented matrix
//     M = [A; B] ((Kpad + m) x Kpad, FP64); the chunks' partial columns are added in order.
//  3. chol_factor: one block per dictionary: blocked FP64 Cholesky of A with the B rows carried
//     along (they end as Z = B L^{-T}), MFMA trailing updates, a ridge retry when a pivot is
//     rejected.  Atoms no signal uses get an identity diagonal (their column of A is zero) and
//     keep their value.
//  4. tri_solve: D L = Z by block columns (MFMA products, small triangular blocks), one block
//     per dictionary; mod_normalize: unit normalisation of the solved atoms.
#include <algorithm>

#include "smdl_internal.h"

namespace {

constexpr double PIV_TOL = 1e-12;
constexpr double RIDGE = 1e-10;

__device__ __forceinline__ int desc_of(const int64_t* __restrict__ starts, int n_desc, int64_t i) {
    int lo = 0, hi = n_desc - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (starts[mid] <= i) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// grid.y = descriptor; threads stride over that descriptor's signals.
// Entries with an atom index outside [0, K) or a count outside [0, s_stride] are skipped
// everywhere and flagged in status[8*t + 3] (the host turns that into SMDL_E_ARG).
__device__ __forceinline__ int clamp_nnz(int k, int s) { return k < 0 ? 0 : (k > s ? s : k); }

// Signals per block of the transpose kernels; each block counts its entries per atom in LDS and
// touches the global counters once per atom, so that many entries of one atom do not contend.
constexpr int CSC_SIG = 1024;

__global__ __launch_bounds__(256) void csc_count_kernel(const ModDesc* __restrict__ md, int32_t* __restrict__ cnt,
                                                        int32_t* __restrict__ status, int32_t* __restrict__ bcnt,
                                                        int total_atoms, int spb) {
    const ModDesc d = md[blockIdx.y];
    __shared__ int32_t hist[SMDL_MAX_K];
    const int tid = threadIdx.x;
    for (int a = tid; a < d.K; a += 256) hist[a] = 0;
    __syncthreads();
    const int64_t n0 = (int64_t)blockIdx.x * spb, n1 = min(d.n, n0 + (int64_t)spb);
    bool bad = false;
    for (int64_t n = n0 + tid; n < n1; n += 256) {
        const int k0 = d.nnz[n];
        const int k = clamp_nnz(k0, d.s_stride);
        bad |= k != k0;
        for (int i = 0; i < k; ++i) {
            const int ix = d.idx[n * d.s_stride + i];
            if (ix < 0 || ix >= d.K) { bad = true; continue; }
            atomicAdd(&hist[ix], 1);
        }
    }
    if (bad) atomicOr(&status[8 * blockIdx.y + 3], 1);
    __syncthreads();
    for (int a = tid; a < d.K; a += 256) {
        if (hist[a]) atomicAdd(&cnt[d.atom0 + a], hist[a]);
        // fixed-order mode: this block's count of every atom (zeros included)
        if (bcnt) bcnt[(int64_t)blockIdx.x * total_atoms + d.atom0 + a] = hist[a];
    }
}

// Fixed-order mode: the first list position of block b's entries of every atom, the blocks in
// order after the atom's list start (one thread per atom).
__global__ void csc_block_base_kernel(const int32_t* __restrict__ ptr, const int32_t* __restrict__ bcnt,
                                      int32_t* __restrict__ bbase, int total_atoms, int nblk) {
    const int ga = blockIdx.x * blockDim.x + threadIdx.x;
    if (ga >= total_atoms) return;
    int32_t run = ptr[ga];
    for (int b = 0; b < nblk; ++b) {
        bbase[(int64_t)b * total_atoms + ga] = run;
        run += bcnt[(int64_t)b * total_atoms + ga];
    }
}

// Exclusive scan of cnt[0..total) into ptr[0..total]; single block of 1024 threads.  Wave w
// owns the contiguous chunk [w C, (w + 1) C), C = 64 r, read as r rows of 64 consecutive entries
// (coalesced; all r loads issued at once when r <= SCAN_CAP, else row after row): each row is
// scanned across the wave with shuffles and the row totals carried; one barrier then adds the
// totals of the earlier waves.
constexpr int SCAN_CAP = 64;
__device__ __forceinline__ int32_t wave_incl_scan(int32_t x, int lane) {
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int32_t y = __shfl_up(x, off, 64);
        if (lane >= off) x += y;
    }
    return x;
}
__global__ __launch_bounds__(1024) void scan_kernel(const int32_t* __restrict__ cnt, int total,
                                                    int32_t* __restrict__ ptr) {
    __shared__ int32_t wtot[16];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int r = (total + 1023) / 1024;                 // rows of 64 per wave
    const int64_t c0 = (int64_t)wave * 64 * r;
    int32_t carry = 0;
    int32_t v[SCAN_CAP];
    if (r <= SCAN_CAP) {
#pragma unroll
        for (int i = 0; i < SCAN_CAP; ++i) {
            const int64_t k = c0 + 64 * i + lane;
            v[i] = (i < r && k < total) ? cnt[k] : 0;
        }
#pragma unroll
        for (int i = 0; i < SCAN_CAP; ++i) {
            if (i < r) {
                const int32_t inc = wave_incl_scan(v[i], lane);
                const int32_t tot = __shfl(inc, 63, 64);
                v[i] = carry + inc - v[i];               // exclusive, within the wave's chunk
                carry += tot;
            }
        }
    } else {
        for (int i = 0; i < r; ++i) {
            const int64_t k = c0 + 64 * i + lane;
            const int32_t x = k < total ? cnt[k] : 0;
            carry += __shfl(wave_incl_scan(x, lane), 63, 64);
        }
    }
    if (lane == 0) wtot[wave] = carry;
    __syncthreads();
    int32_t base = 0;
    for (int w = 0; w < wave; ++w) base += wtot[w];
    if (r <= SCAN_CAP) {
#pragma unroll
        for (int i = 0; i < SCAN_CAP; ++i) {
            const int64_t k = c0 + 64 * i + lane;
            if (i < r && k < total) ptr[k] = base + v[i];
        }
    } else {
        int32_t run = base;
        for (int i = 0; i < r; ++i) {
            const int64_t k = c0 + 64 * i + lane;
            const int32_t x = k < total ? cnt[k] : 0;
            const int32_t inc = wave_incl_scan(x, lane);
            if (k < total) ptr[k] = run + inc - x;
            run += __shfl(inc, 63, 64);
        }
    }
    if (threadIdx.x == 1023) {
        int32_t all = 0;
        for (int w = 0; w < 16; ++w) all += wtot[w];
        ptr[total] = all;
    }
}

// Each block takes CSC_FILL_SIG signals, one per thread.  One LDS atomic per entry counts the
// entries of each atom and gives the entry its rank among them; a scan of the counts gives each
// atom's local start, and one global atomic per atom with entries reserves a contiguous range of
// that atom's list.  The entries are staged in LDS grouped by atom, then written out in staging
// order: each atom's run of the block's entries goes out as consecutive stores (scattered 4-byte
// stores moved several times their bytes through the caches).
// Fixed-order mode (FIXED): the entries are ranked slot by slot, and within a slot by signal.
// In slot i each signal has at most one entry; it sets its bit in its atom's 256-bit mask (an
// LDS OR, whose result does not depend on the order of the ORs), and its rank is the atom's
// entries of the earlier slots plus the set bits below its own.  The block's run of each atom
// starts at bbase (the atom's list start plus the entries of the earlier blocks, from the
// per-block counts), so the lists are the same on every run.
constexpr int CSC_FILL_SIG = 256;
template <bool FIXED>
__global__ __launch_bounds__(CSC_FILL_SIG) void csc_fill_kernel(const ModDesc* __restrict__ md,
                                                                const int32_t* __restrict__ ptr,
                                                                int32_t* __restrict__ fill,
                                                                const int32_t* __restrict__ bbase,
                                                                int total_atoms,
                                                                int32_t* __restrict__ list_sig,
                                                                float* __restrict__ list_coef) {
    constexpr int NT = CSC_FILL_SIG;
    constexpr int AP = SMDL_MAX_K / NT;          // atoms per thread in the scan
    constexpr int MW = NT / 32;                  // mask words per atom (fixed-order mode)
    const ModDesc d = md[blockIdx.y];
    __shared__ int32_t cnt[SMDL_MAX_K];          // entries per atom, then the atom's local start
    __shared__ int32_t gpos[SMDL_MAX_K];         // list position of the atom's first entry
    __shared__ int32_t wsum[NT / 64];
    __shared__ int32_t st_sig[NT * SMDL_MAX_S];
    __shared__ float st_coef[NT * SMDL_MAX_S];
    __shared__ uint16_t st_atom[NT * SMDL_MAX_S];
    __shared__ uint32_t amask[FIXED ? SMDL_MAX_K * MW : 1];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    for (int a = tid; a < SMDL_MAX_K; a += NT) cnt[a] = 0;
    if constexpr (FIXED)
        for (int w = tid; w < SMDL_MAX_K * MW; w += NT) amask[w] = 0u;
    // this thread's signal and its entries (at most SMDL_MAX_S)
    const int64_t n = (int64_t)blockIdx.x * NT + tid;
    const int k = n < d.n ? clamp_nnz(d.nnz[n], min(d.s_stride, SMDL_MAX_S)) : 0;
    int ix[SMDL_MAX_S];
    float cf[SMDL_MAX_S];
#pragma unroll
    for (int i = 0; i < SMDL_MAX_S; ++i) {
        ix[i] = -1;
        cf[i] = 0.f;
        if (i < k) {
            ix[i] = d.idx[n * d.s_stride + i];
            cf[i] = d.coef[n * d.s_stride + i];
        }
    }
    __syncthreads();
    int rank[SMDL_MAX_S];
    if constexpr (FIXED) {
        const int S = min(d.s_stride, SMDL_MAX_S);   // the same for the whole block
        const int wd = tid >> 5;
        const uint32_t bit = 1u << (tid & 31);
#pragma unroll
        for (int i = 0; i < SMDL_MAX_S; ++i) {
            rank[i] = -1;
            if (i >= S) continue;
            const bool ok = i < k && ix[i] >= 0 && ix[i] < d.K;
            if (ok) atomicOr(&amask[ix[i] * MW + wd], bit);
            __syncthreads();
            int tot = 0;
            bool lead = false;
            if (ok) {
                const uint32_t* mk = &amask[ix[i] * MW];
                int below = __popc(mk[wd] & (bit - 1u));
                for (int w = 0; w < wd; ++w) below += __popc(mk[w]);
                rank[i] = cnt[ix[i]] + below;
                lead = below == 0;                   // the atom's lowest signal in this slot
                if (lead)
                    for (int w = wd; w < MW; ++w) tot += __popc(mk[w]);
            }
            __syncthreads();                         // every rank is read
            if (lead) {
                cnt[ix[i]] += tot;
                for (int w = 0; w < MW; ++w) amask[ix[i] * MW + w] = 0u;
            }
            __syncthreads();
        }
    } else {
#pragma unroll
        for (int i = 0; i < SMDL_MAX_S; ++i) {
            const bool ok = i < k && ix[i] >= 0 && ix[i] < d.K;
            rank[i] = ok ? atomicAdd(&cnt[ix[i]], 1) : -1;
        }
    }
    __syncthreads();
    // reserve the ranges; exclusive scan of the counts (thread t: atoms AP t .. AP t + AP - 1)
    int c[AP], run = 0;
#pragma unroll
    for (int q = 0; q < AP; ++q) {
        const int a = AP * tid + q;
        c[q] = cnt[a];
        if (a < d.K && c[q] > 0) {
            if constexpr (FIXED)
                gpos[a] = bbase[(int64_t)blockIdx.x * total_atoms + d.atom0 + a];
            else
                gpos[a] = ptr[d.atom0 + a] + atomicAdd(&fill[d.atom0 + a], c[q]);
        }
        run += c[q];
    }
    int inc = run;                               // inclusive scan over the wave
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int v = __shfl_up(inc, off, 64);
        if (lane >= off) inc += v;
    }
    if (lane == 63) wsum[wave] = inc;
    __syncthreads();
    int base = inc - run;
    for (int w = 0; w < wave; ++w) base += wsum[w];
#pragma unroll
    for (int q = 0; q < AP; ++q) {
        cnt[AP * tid + q] = base;
        base += c[q];
    }
    const int total = wsum[0] + wsum[1] + wsum[2] + wsum[3];
    __syncthreads();
#pragma unroll
    for (int i = 0; i < SMDL_MAX_S; ++i) {
        if (rank[i] >= 0) {
            const int p = cnt[ix[i]] + rank[i];
            st_sig[p] = (int32_t)n;
            st_coef[p] = cf[i];
            st_atom[p] = (uint16_t)ix[i];
        }
    }
    __syncthreads();
    for (int p = tid; p < total; p += NT) {
        const int a = st_atom[p];
        const int dst = gpos[a] + (p - cnt[a]);
        list_sig[dst] = st_sig[p];
        list_coef[dst] = st_coef[p];
    }
}

// mod_products_kernel's LDS: the A column, the B row sums and the staged list entries.
constexpr int MP_STAGE = 512;                // list entries staged per pass
constexpr int MP_LDS = SMDL_MAX_K * 8 + 256 * 8 + MP_STAGE * 8;

// One block per (atom a, descriptor, chunk c): the products over chunk c of the P equal parts of
// atom a's list.  Chunk 0 writes column a of M = [A; B] (FP64) in place; chunk c > 0 writes the
// same column of copy c - 1 of the M arena in `part` (sum_reduce_kernel adds the copies in a
// fixed order).  Long lists (many signals per atom) are so spread over P blocks.
// Fixed-order mode (FIXED): the A column is summed in list order without atomics.  Each round
// takes 256 / SP entries x SP support slots, one (entry, slot) pair per thread, keyed SP entry + slot;
// a pair sets its key's bit in its target atom's 256-bit mask and takes the minimum of its key
// in the target's owner word (dynamic LDS, 9 words per atom); the owner adds the round's values
// of that target in key order.  B is in list order in both modes.
template <bool FIXED>
__global__ __launch_bounds__(256) void mod_products_kernel(const ModDesc* __restrict__ md, int m,
                                                           const int32_t* __restrict__ ptr,
                                                           const int32_t* __restrict__ list_sig,
                                                           const float* __restrict__ list_coef,
                                                           const double* __restrict__ arena, double* __restrict__ part,
                                                           int64_t arena_len) {
    const ModDesc d = md[blockIdx.y];
    const int a = blockIdx.x;
    const int c = blockIdx.z, P = gridDim.z;
    if (a >= d.Kpad) return;
    static_assert(SMDL_MAX_S <= 16, "16 support slots per list entry");
    constexpr int PSTAGE = MP_STAGE;
    constexpr int PB = 8;                    // signal loads in flight per thread
    __shared__ double colA[SMDL_MAX_K];
    __shared__ double partB[256];            // groups x mcov = 256 row sums
    __shared__ int32_t s_sig[PSTAGE];
    __shared__ float s_cf[PSTAGE];
    extern __shared__ uint32_t amask[];      // fixed-order mode: Kpad x 8 mask words, Kpad owners
    __shared__ double vbuf[FIXED ? 256 : 1];
    const int tid = threadIdx.x;
    for (int l = tid; l < d.Kpad; l += 256) colA[l] = 0.0;
    int32_t* owner = reinterpret_cast<int32_t*>(amask + 8 * d.Kpad);   // fixed-order mode: Kpad
    if constexpr (FIXED) {
        for (int w = tid; w < d.Kpad * 8; w += 256) amask[w] = 0u;
        for (int l = tid; l < d.Kpad; l += 256) owner[l] = 0x7fffffff;
    }
    __syncthreads();
    const int64_t ld = d.Kpad + m;
    double* out = (c == 0 ? d.A : part + (int64_t)(c - 1) * arena_len + (d.A - arena)) + (int64_t)a * ld;
    const int mcov = m <= 32 ? 32 : (m <= 64 ? 64 : (m <= 128 ? 128 : 256));
    const int groups = 256 / mcov;
    const int r = tid % mcov, grp = tid / mcov;
    if (a < d.K) {
        const int64_t ga = d.atom0 + a;
        const int lb = ptr[ga], le = ptr[ga + 1];
        const int len = (le - lb + P - 1) / P;
        const int b = min(le, lb + c * len), e = min(le, b + len);
        // the entries in passes of PSTAGE, staged in LDS
        double acc = 0.0;
        for (int p0 = b; p0 < e; p0 += PSTAGE) {
            const int cnt = min(PSTAGE, e - p0);
            __syncthreads();                                  // the previous pass is read
            for (int q = tid; q < cnt; q += 256) {
                s_sig[q] = list_sig[p0 + q];
                s_cf[q] = list_coef[p0 + q];
            }
            __syncthreads();
            // A column: every entry (n, x_na) adds x_na * x_nl at every atom l of signal n; the
            // block's lanes take (entry, support slot) pairs, SP slots per entry (s_stride rounded
            // up to a power of two, at most 16) and 256 / SP entries per round, the loads of UA
            // rounds issued before their adds
            constexpr int UA = 4;
            const int lsp = d.s_stride <= 1 ? 0 : 32 - __clz(d.s_stride - 1);
            const int SP = 1 << lsp, ER = 256 >> lsp;
            const int slot = tid & (SP - 1), eq = tid >> lsp;
            for (int q0 = 0; q0 < cnt; q0 += ER * UA) {
                int lv[UA], kv[UA];
                float cv[UA];
                double xv[UA];
#pragma unroll
                for (int u = 0; u < UA; ++u) {
                    const int q = q0 + ER * u + eq;
                    lv[u] = -1;
                    kv[u] = 0;
                    cv[u] = 0.f;
                    xv[u] = 0.0;
                    if (q < cnt) {
                        const int64_t n = s_sig[q];
                        kv[u] = d.nnz[n];
                        if (slot < d.s_stride) {
                            lv[u] = d.idx[n * d.s_stride + slot];
                            cv[u] = d.coef[n * d.s_stride + slot];
                        }
                        xv[u] = s_cf[q];
                    }
                }
#pragma unroll
                for (int u = 0; u < UA; ++u) {
                    const bool ok = slot < clamp_nnz(kv[u], d.s_stride) && lv[u] >= 0 && lv[u] < d.K;
                    if constexpr (FIXED) {
                        // one round: mark, then the lowest key of each target adds in key order
                        const int wd = tid >> 5;
                        const uint32_t bit = 1u << (tid & 31);
                        if (ok) {
                            vbuf[tid] = xv[u] * (double)cv[u];
                            atomicOr(&amask[lv[u] * 8 + wd], bit);
                            atomicMin(&owner[lv[u]], tid);
                        }
                        __syncthreads();
                        // the owner (lowest key) of each target adds its values, then clears the
                        // target's mask and owner word for the next round; any other pair reads
                        // the lowest key or the cleared word, neither of which is its own key
                        if (ok && owner[lv[u]] == tid) {
                            uint32_t* mk = &amask[lv[u] * 8];
                            double acc = colA[lv[u]];
                            for (int w = wd; w < 8; ++w) {
                                uint32_t b = mk[w];
                                while (b) {
                                    acc += vbuf[32 * w + __builtin_ctz(b)];
                                    b &= b - 1u;
                                }
                                mk[w] = 0u;
                            }
                            colA[lv[u]] = acc;
                            owner[lv[u]] = 0x7fffffff;
                        }
                        __syncthreads();
                    } else {
                        if (ok) atomicAdd(&colA[lv[u]], xv[u] * (double)cv[u]);
                    }
                }
            }
            // B column: rows split over threads, entries over groups of threads, PB signal
            // loads in flight per thread (the sum keeps the order of the entries)
            if (r < m) {
                int q = grp;
                for (; q + (PB - 1) * groups < cnt; q += PB * groups) {
                    float yv[PB];
#pragma unroll
                    for (int u = 0; u < PB; ++u) yv[u] = d.Y[(int64_t)s_sig[q + u * groups] * m + r];
#pragma unroll
                    for (int u = 0; u < PB; ++u) acc += (double)s_cf[q + u * groups] * (double)yv[u];
                }
                for (; q < cnt; q += groups) acc += (double)s_cf[q] * (double)d.Y[(int64_t)s_sig[q] * m + r];
            }
        }
        partB[grp * mcov + r] = acc;
    } else {
        partB[grp * mcov + r] = 0.0;
    }
    __syncthreads();
    for (int l = tid; l < d.Kpad; l += 256) out[l] = colA[l];
    for (int rr = tid; rr < m; rr += 256) {
        double sm = 0.0;
        for (int q = 0; q < groups; ++q) sm += partB[q * mcov + rr];
        out[d.Kpad + rr] = sm;
    }
}

// arena[f] += sum_{c < P - 1} part[c * len + f], in order of c.
__global__ void sum_reduce_kernel(double* __restrict__ arena, const double* __restrict__ part, int64_t len, int nparts) {
    for (int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; f < len; f += (int64_t)gridDim.x * blockDim.x) {
        double v = arena[f];
        for (int c = 0; c < nparts; ++c) v += part[(int64_t)c * len + f];
        arena[f] = v;
    }
}

// ------------------------------------------------------------------------------------------
// FP64 Cholesky factorisation of the augmented matrix [A; B] (one block per dictionary)
// ------------------------------------------------------------------------------------------
// status[8*t + 0] = unused atoms (this call), [1] |= ridge used, [2] |= failed, [3] |= bad codes,
// [4] = failed in this call (read by the solve and normalisation kernels), [5] = a pivot of the
// multi-work-group factorisation was rejected in this call (the dictionary is factored again by
// this kernel).  The caller zeroes the status array before a sequence of updates.
//
// W (column-major, ld = Kpad + m) holds [A; B]; A = L L^T is factored in place and the B rows are
// carried along as extra rows of every panel, so that they end as Z = B L^{-T} (the forward half
// of D A = B).  Right-looking, panel width FB = 16 (the unrolled register factorisation of a
// 32-wide diagonal block does not fit in a 512-thread block's registers):
//   (i)   the 16 x 16 diagonal block: one row per lane of wave 0, each finished column broadcast
//         through LDS; the reciprocals of the diagonal are kept;
//   (ii)  every row below it (A rows and B rows) solves x L_kk^T = w right-looking (depth 16,
//         no divisions); A rows are also written transposed (W[i*ld + j] = L[i][j], j < i),
//         which the backward substitution reads contiguously;
//   (iii) the trailing lower triangle of A and the trailing B rows are updated on the FP64
//         matrix cores (v_mfma_f64_16x16x4f64, 16 x 16 tiles, the panel from LDS when it fits),
//         oriented so that consecutive lanes touch consecutive rows of W; each wave takes its
//         tiles four at a time with all their old values requested first.
constexpr int FB = 16;
constexpr int CT = 512;
constexpr int PR = 1168;                     // panel rows kept in LDS (16 x 1168 doubles = 146 KB);
                                             // 1168 = 16 mod 32 puts the four k-groups of an MFMA
                                             // operand read on alternating halves of the banks

typedef double f64x4 __attribute__((ext_vector_type(4)));

// FP64 global accesses at a 32-bit byte offset from a uniform base (W stays below 4 GiB: Kpad,
// m <= 1024 + 256): one VGPR per address instead of a 64-bit pair.
__device__ __forceinline__ double gld(const double* base, uint32_t off) {
    return *(const __attribute__((address_space(1))) double*)(reinterpret_cast<const char*>(base) + off);
}
__device__ __forceinline__ void gst(double* base, uint32_t off, double v) {
    *(__attribute__((address_space(1))) double*)(reinterpret_cast<char*>(base) + off) = v;
}

__device__ __forceinline__ double readlane_f64(double v, int lane) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), lane);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
    return __longlong_as_double(((long long)(unsigned)hi << 32) | (unsigned)lo);
}

// retry_only: factor only the dictionaries whose multi-work-group factorisation rejected a pivot
// (status[8*t + 5]), from the products again, with the ridge retry of this kernel.
__global__ __launch_bounds__(CT) void chol_factor_kernel(const ModDesc* __restrict__ md, int m,
                                                         int32_t* __restrict__ status, int retry_only) {
    if (retry_only && !status[8 * blockIdx.x + 5]) return;
    const ModDesc d = md[blockIdx.x];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int Kp = d.Kpad;
    const int ld = Kp + m;
    const double* P = d.A;
    double* W = d.W;
    __shared__ double LdT[FB][FB + 1];       // LdT[c][r] = L[kb + r][kb + c]
    __shared__ double rdiag[FB];             // 1 / L[kb + c][kb + c]
    __shared__ double colb[FB];              // column broadcast of the diagonal factorisation
    __shared__ double panel[FB * PR];        // panel[c * PR + row - r0]
    __shared__ double diag0[SMDL_MAX_K];
    __shared__ unsigned char active[SMDL_MAX_K];
    __shared__ int s_fail, s_failed_final;
    __shared__ double s_red[CT / 64];
    __shared__ int s_cnt[CT / 64];
    int32_t* st = status + 8 * blockIdx.x;

    double mx = 0.0;
    int unused = 0;
    for (int a = tid; a < Kp; a += CT) {
        const double v = P[(int64_t)a * ld + a];
        active[a] = v > 0.0;
        if (v > mx) mx = v;
        if (a < d.K && !(v > 0.0)) ++unused;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        mx = fmax(mx, __shfl_xor(mx, off, 64));
        unused += __shfl_xor(unused, off, 64);
    }
    if (lane == 0) {
        s_red[wave] = mx;
        s_cnt[wave] = unused;
    }
    if (tid == 0) s_failed_final = 0;
    __syncthreads();
    if (tid == 0) {
        double a = 0.0;
        int c = 0;
        for (int w = 0; w < CT / 64; ++w) {
            a = fmax(a, s_red[w]);
            c += s_cnt[w];
        }
        s_red[0] = a;
        st[0] = c;
        st[4] = 0;
    }
    __syncthreads();
    const double maxdiag = s_red[0];

    for (int attempt = 0; attempt < 2; ++attempt) {
        const double lam = attempt == 0 ? 0.0 : RIDGE * maxdiag;
        // W = [A (+ lam I on active atoms, identity diagonal on unused ones); B], sixteen loads
        // in flight per thread
        const int total = Kp * ld;
        for (int f0 = tid; f0 < total; f0 += 16 * CT) {
            double v[16];
#pragma unroll
            for (int u = 0; u < 16; ++u) {
                const int f = f0 + u * CT;
                v[u] = f < total ? P[f] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < 16; ++u) {
                const int f = f0 + u * CT;
                if (f < total) {
                    const int col = f / ld, row = f - col * ld;
                    double x = v[u];
                    if (row == col) x = active[col] ? x + lam : 1.0;
                    W[f] = x;
                }
            }
        }
        for (int a = tid; a < Kp; a += CT) diag0[a] = active[a] ? P[(int64_t)a * ld + a] + lam : 1.0;
        if (tid == 0) s_fail = 0;
        __syncthreads();

        for (int kb = 0; kb < Kp; kb += FB) {
            // (i) diagonal block, staged through LdT (LdT[c][r] = block entry (r, c), r >= c);
            // lane i < FB of wave 0 holds row i in registers
            for (int f = tid; f < FB * FB; f += CT) {
                const int c = f / FB, r = f % FB;
                LdT[c][r] = r >= c ? gld(W, 8u * (uint32_t)((kb + c) * ld + kb + r)) : 0.0;
            }
            __syncthreads();
            if (wave == 0) {
                // Entries above a row's diagonal (c > lane) are don't-care values: updating them
                // unconditionally avoids one lane mask per column; they are never read.  Lanes
                // FB..63 repeat lanes 0..FB-1.
                const int li = lane & (FB - 1);
                double a[FB];
#pragma unroll
                for (int c = 0; c < FB; ++c) a[c] = LdT[c][li];
                bool bad = false;
#pragma unroll
                for (int j = 0; j < FB; ++j) {
                    const double djj = readlane_f64(a[j], j);
                    const bool b = !(djj > PIV_TOL * diag0[kb + j]);
                    bad |= b;
                    const double dj = b ? 1.0 : sqrt(djj);
                    const double rd = 1.0 / dj;
                    a[j] *= rd;                           // lane j: d_j; lanes i > j: L[i][j]
                    colb[li] = a[j];
                    if (lane == 0) rdiag[j] = rd;
#pragma unroll
                    for (int c = j + 1; c < FB; ++c) a[c] = fma(-a[j], colb[c], a[c]);
                }
                if (lane == 0 && bad) s_fail = 1;
                if (lane < FB) {
#pragma unroll
                    for (int c = 0; c < FB; ++c) LdT[c][lane] = a[c];
                }
            }
            __syncthreads();
            // the factored block back to W: column kb + c gets L[., kb + c] below the diagonal
            // and, above it, the mirror W[i*ld + j] = L[i][j] (j < i) of row kb + c
            for (int f = tid; f < FB * FB; f += CT) {
                const int c = f / FB, r = f % FB;
                gst(W, 8u * (uint32_t)((kb + c) * ld + kb + r), r >= c ? LdT[c][r] : LdT[r][c]);
            }
            __syncthreads();
            if (s_fail) break;
            // (ii) rows below the block (the rest of A, then B): x L_kk^T = w
            const int r0 = kb + FB;
            const int R = ld - r0;
            const bool in_lds = (R + 15) / 16 * 16 <= PR;
            for (int rr = tid; rr < R; rr += CT) {
                const int i = r0 + rr;
                double x[FB];
#pragma unroll
                for (int c = 0; c < FB; ++c) x[c] = gld(W, 8u * (uint32_t)((kb + c) * ld + i));
#pragma unroll
                for (int c = 0; c < FB; ++c) {
                    x[c] *= rdiag[c];
#pragma unroll
                    for (int c2 = c + 1; c2 < FB; ++c2) x[c2] = fma(-x[c], LdT[c][c2], x[c2]);
                    __asm__ volatile("" ::: "memory");     // keep column c's LDS reads in this step
                }
#pragma unroll
                for (int c = 0; c < FB; ++c) gst(W, 8u * (uint32_t)((kb + c) * ld + i), x[c]);
                if (i < Kp) {
#pragma unroll
                    for (int c = 0; c < FB; ++c) gst(W, 8u * (uint32_t)(i * ld + kb + c), x[c]);   // mirror
                }
                if (in_lds) {
#pragma unroll
                    for (int c = 0; c < FB; ++c) panel[c * PR + rr] = x[c];
                }
            }
            __syncthreads();
            // (iii) trailing update: lower triangle of the A block (tiles ib >= jb) and the B rows
            // (tiles ib >= TA), T[row][col] -= sum_k X[row][k] X[col][k] over the panel columns
            const int TA = (Kp - r0) / 16;
            const int TBR = (m + 15) / 16;
            const int nA = TA * (TA + 1) / 2;
            const int ntile = nA + TBR * TA;
            constexpr int NB4 = 4;
            for (int t0 = wave; t0 < ntile; t0 += NB4 * (CT / 64)) {
                int ibs[NB4], jbs[NB4];
                bool okt[NB4], rv[NB4];
                double old[NB4][4];
#pragma unroll
                for (int u = 0; u < NB4; ++u) {
                    const int t = t0 + u * (CT / 64);
                    okt[u] = t < ntile;
                    int ib = 0, jb = 0;
                    if (okt[u] && t < nA) {
                        ib = (int)((sqrtf(8.f * t + 1.f) - 1.f) * 0.5f);
                        while ((ib + 1) * (ib + 2) / 2 <= t) ++ib;
                        while (ib * (ib + 1) / 2 > t) --ib;
                        jb = t - ib * (ib + 1) / 2;
                    } else if (okt[u]) {
                        ib = TA + (t - nA) / TA;
                        jb = (t - nA) % TA;
                    }
                    ibs[u] = ib;
                    jbs[u] = jb;
                    const int row = r0 + 16 * ib + (lane & 15);
                    const int col = r0 + 16 * jb + (lane >> 4);
                    rv[u] = okt[u] && row < ld;
#pragma unroll
                    for (int q = 0; q < 4; ++q) old[u][q] = rv[u] ? gld(W, 8u * (uint32_t)((col + 4 * q) * ld + row)) : 0.0;
                }
#pragma unroll
                for (int u = 0; u < NB4; ++u) {
                    if (!okt[u]) continue;
                    f64x4 acc = {0.0, 0.0, 0.0, 0.0};
                    const int ra = 16 * jbs[u] + (lane & 15);          // A operand: rows of block jb
                    const int rb = 16 * ibs[u] + (lane & 15);          // B operand: rows of block ib
                    const int kq = lane >> 4;
#pragma unroll
                    for (int kc = 0; kc < FB; kc += 4) {
                        double av, bv;
                        if (in_lds) {
                            av = panel[(kc + kq) * PR + ra];
                            bv = panel[(kc + kq) * PR + rb];
                        } else {
                            av = gld(W, 8u * (uint32_t)((kb + kc + kq) * ld + r0 + ra));
                            bv = gld(W, 8u * (uint32_t)((kb + kc + kq) * ld + min(r0 + rb, ld - 1)));
                        }
                        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc, 0, 0, 0);
                    }
                    // FP64 16x16x4 output D[i][j] (lane j + 16 (i % 4), register i / 4):
                    // acc[q] = sum_k X[16 jb + kq + 4 q][k] X[16 ib + (lane & 15)][k], the update of
                    // W at row r0 + 16 ib + (lane & 15), column r0 + 16 jb + kq + 4 q
                    if (rv[u]) {
                        const int row = r0 + rb;
                        const int col = r0 + 16 * jbs[u] + kq;
#pragma unroll
                        for (int q = 0; q < 4; ++q) gst(W, 8u * (uint32_t)((col + 4 * q) * ld + row), old[u][q] - acc[q]);
                    }
                }
            }
            __syncthreads();
        }
        if (!s_fail) break;
        if (attempt == 0 && tid == 0) atomicOr(&st[1], 1);
        if (attempt == 1 && tid == 0) {
            atomicOr(&st[2], 1);
            st[4] = 1;
            s_failed_final = 1;
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------------------------------------
// Backward substitution D L = Z (one block per dictionary)
// ------------------------------------------------------------------------------------------
// Z = B L^{-T} sits in the B rows of W (W[j*ld + Kp + r] = Z[r][j]) and is overwritten by D.
// Block columns of SB = 32 from the last: T = Z_J - D_{>J} L_{>J,J} on the FP64 matrix cores (the
// mirrored rows of L give coalesced operands), then D_J L_JJ = T with one thread per row of D
// (right-looking inside the 32 x 32 block, reciprocals of the diagonal).
constexpr int TCS = 512;
constexpr int SB = 32;                       // block columns of the backward substitution

__global__ __launch_bounds__(TCS) void tri_solve_kernel(const ModDesc* __restrict__ md, int m,
                                                        const int32_t* __restrict__ status) {
    const int t = blockIdx.x;
    if (status[8 * t + 4]) return;
    const ModDesc d = md[t];
    const int Kp = d.Kpad;
    const int ld = Kp + m;
    double* W = d.W;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    __shared__ double Lj[SB][SB + 1];         // Lj[r][c] = L[J + r][J + c]
    __shared__ double rd[SB];
    __shared__ double Tt[SMDL_MAX_M][SB + 1]; // right-hand sides of the block column
    const int MT = (m + 15) / 16;
    for (int J = Kp - SB; J >= 0; J -= SB) {
        for (int f = tid; f < SB * SB; f += TCS) {
            const int c = f / SB, r = f % SB;                         // coalesced down column J + c
            Lj[r][c] = r >= c ? gld(W, 8u * (uint32_t)((J + c) * ld + J + r)) : 0.0;
        }
        if (tid < SB) rd[tid] = 1.0 / gld(W, 8u * (uint32_t)((J + tid) * ld + J + tid));
        const int kdim = Kp - J - SB;
        const int kq = lane >> 4;
        for (int tt = wave; tt < 2 * MT; tt += TCS / 64) {
            const int rb = tt >> 1, cb = tt & 1;
            f64x4 acc = {0.0, 0.0, 0.0, 0.0};
            const int r = min(16 * rb + (lane & 15), m - 1);             // row of D (clamped)
            for (int k0 = 0; k0 < kdim; k0 += 64) {                   // kdim % 32 == 0
                double av[16], bv[16];
#pragma unroll
                for (int u = 0; u < 16; ++u) {
                    const int i = min(J + SB + k0 + 4 * u + kq, Kp - 1);
                    av[u] = gld(W, 8u * (uint32_t)(i * ld + Kp + r));                        // D[r][i]
                    bv[u] = gld(W, 8u * (uint32_t)(i * ld + J + 16 * cb + (lane & 15)));      // L[i][J + c]
                }
#pragma unroll
                for (int u = 0; u < 16; ++u)
                    if (k0 + 4 * u < kdim) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u], bv[u], acc, 0, 0, 0);
            }
            // acc[q]: row 16 rb + kq + 4 q of D, column 16 cb + (lane & 15) of the block
            const int c = 16 * cb + (lane & 15);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int row = 16 * rb + kq + 4 * q;
                if (row < m) Tt[row][c] = gld(W, 8u * (uint32_t)((J + c) * ld + Kp + row)) - acc[q];
            }
        }
        __syncthreads();
        if (tid < m) {
            double x[SB];
#pragma unroll
            for (int c = 0; c < SB; ++c) x[c] = Tt[tid][c];
#pragma unroll
            for (int c = SB - 1; c >= 0; --c) {
                x[c] *= rd[c];
#pragma unroll
                for (int c2 = 0; c2 < c; ++c2) x[c2] = fma(-x[c], Lj[c][c2], x[c2]);
                __asm__ volatile("" ::: "memory");         // keep row c's LDS reads in this step
            }
#pragma unroll
            for (int c = 0; c < SB; ++c) gst(W, 8u * (uint32_t)((J + c) * ld + Kp + tid), x[c]);
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------------------------------------
// Multi-work-group factorisation and substitution (dictionaries too few to fill the chip)
// ------------------------------------------------------------------------------------------
// The same right-looking Cholesky of [A; B] as above, in panels of PW = 32 columns with one
// launch per panel, so that every step spreads over many compute units:
//   chol_setup:  W = [A; B] with identity diagonals on unused atoms; work group 0 of each
//                dictionary factors the first 32 x 32 diagonal block (the others copy the rest);
//   chol_panel:  (first panel only) every row below the factored diagonal block, A rows and B
//                rows, solves x L_kk^T = w, one row per thread; A rows are also written mirrored;
//   chol_update: the trailing lower triangle of A and the trailing B rows, in 64 x 64 tiles on
//                the FP64 matrix cores (one 32 x 32 quarter per wave).  The tiles of the first
//                column block also form and factor the next diagonal block and solve their rows
//                of the next panel, so that the next launch finds that panel solved.
// The factored diagonal blocks go to a side array (ModDesc::Ld), not into W, whose diagonal blocks
// the update launches read.  On output W holds L below the diagonal blocks and mirrored above
// them, and Z = B L^{-T} in the B rows.  A rejected pivot sets status[8*t + 5]; later launches skip
// that dictionary and chol_factor_kernel (retry_only) factors it again with its ridge retry (then W
// holds its whole factor).  tri_solve_rows then solves D L = Z with one work group per 16 rows of D.
constexpr int PW = 32;                       // panel width
constexpr int UT = 64;                       // trailing-update tile (rows and columns)

struct DiagBlock {
    double L[PW][PW + 1];                    // L[r][c], lower triangle
    double rd[PW];                           // 1 / L[c][c]
    double dref[PW];                         // pivot reference: the original diagonal entries
    double colb[16];
    int bad;
};

// Factor the 32 x 32 lower block in s.L in place (256 threads, uniform call): two leaves of 16
// columns, each factored by wave 0 with one row per lane (the finished column broadcast through
// LDS), with the second leaf's rows solved against the first and its block updated in between.
__device__ __forceinline__ void factor_diag32(DiagBlock& s, int tid) {
    const int lane = tid & 63, wave = tid >> 6;
    if (tid == 0) s.bad = 0;
    __syncthreads();
#pragma unroll 1
    for (int leaf = 0; leaf < 2; ++leaf) {
        const int o = 16 * leaf;
        if (wave == 0) {
            // lanes 16..63 repeat lanes 0..15; entries above a row's diagonal are don't-care
            const int li = lane & 15;
            double a[16];
#pragma unroll
            for (int c = 0; c < 16; ++c) a[c] = s.L[o + li][o + c];
            bool bad = false;
#pragma unroll
            for (int j = 0; j < 16; ++j) {
                const double djj = readlane_f64(a[j], j);
                const bool b = !(djj > PIV_TOL * s.dref[o + j]);
                bad |= b;
                const double dj = b ? 1.0 : sqrt(djj);
                const double rd = 1.0 / dj;
                a[j] *= rd;                               // lane j: d_j; lanes i > j: L[i][j]
                s.colb[li] = a[j];
                if (lane == 0) s.rd[o + j] = rd;
#pragma unroll
                for (int c = j + 1; c < 16; ++c) a[c] = fma(-a[j], s.colb[c], a[c]);
            }
            if (lane == 0 && bad) s.bad = 1;
            if (lane < 16) {
#pragma unroll
                for (int c = 0; c < 16; ++c) s.L[o + lane][o + c] = a[c];
            }
        }
        __syncthreads();
        if (leaf == 1) break;
        // rows 16..31 against the first leaf: x L_00^T = w
        if (tid < 16) {
            double x[16];
#pragma unroll
            for (int c = 0; c < 16; ++c) x[c] = s.L[16 + tid][c];
#pragma unroll
            for (int c = 0; c < 16; ++c) {
                x[c] *= s.rd[c];
#pragma unroll
                for (int c2 = c + 1; c2 < 16; ++c2) x[c2] = fma(-x[c], s.L[c2][c], x[c2]);
                __asm__ volatile("" ::: "memory");         // keep column c's LDS reads in this step
            }
#pragma unroll
            for (int c = 0; c < 16; ++c) s.L[16 + tid][c] = x[c];
        }
        __syncthreads();
        // the second leaf's block: L[16 + i][16 + j] -= sum_c L[16 + i][c] L[16 + j][c]
        {
            const int i = tid >> 4, j = tid & 15;
            double v = s.L[16 + i][16 + j];
#pragma unroll
            for (int c = 0; c < 16; ++c) v = fma(-s.L[16 + i][c], s.L[16 + j][c], v);
            __syncthreads();
            if (j <= i) s.L[16 + i][16 + j] = v;
        }
        __syncthreads();
    }
}

// The factored block at (kb, kb) to the side array Ld (block kb / 32, column-major, zero above the
// diagonal).
__device__ __forceinline__ void store_diag_block(double* Ld, int kb, const DiagBlock& s, int tid) {
    for (int f = tid; f < PW * PW; f += 256) {
        const int c = f / PW, r = f % PW;
        Ld[(int64_t)kb * PW + f] = r >= c ? s.L[r][c] : 0.0;
    }
}

// Pivot references of the block at kb: the products' diagonal, 1 for unused atoms.
__device__ __forceinline__ void load_dref(DiagBlock& s, const double* P, int ld, int kb, int tid) {
    if (tid < PW) {
        const double v = P[(int64_t)(kb + tid) * ld + kb + tid];
        s.dref[tid] = v > 0.0 ? v : 1.0;
    }
}

__global__ __launch_bounds__(256) void chol_setup_kernel(const ModDesc* __restrict__ md, int m,
                                                         int32_t* __restrict__ status) {
    const int t = blockIdx.y;
    const ModDesc d = md[t];
    const int Kp = d.Kpad, ld = Kp + m, tid = threadIdx.x;
    const double* P = d.A;
    double* W = d.W;
    if (blockIdx.x != 0) {
        // the copy, sixteen loads in flight per thread; the first 32 x 32 diagonal block is
        // left to work group 0
        const int64_t total = (int64_t)Kp * ld;
        const int64_t stride = (int64_t)(gridDim.x - 1) * 256;
        for (int64_t f0 = (int64_t)(blockIdx.x - 1) * 256 + tid; f0 < total; f0 += 16 * stride) {
            double v[16];
#pragma unroll
            for (int u = 0; u < 16; ++u) {
                const int64_t f = f0 + u * stride;
                v[u] = f < total ? P[f] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < 16; ++u) {
                const int64_t f = f0 + u * stride;
                if (f < total) {
                    const int col = (int)(f / ld), row = (int)(f - (int64_t)col * ld);
                    if (col < PW && row < PW) continue;
                    double x = v[u];
                    if (row == col && !(x > 0.0)) x = 1.0;
                    W[f] = x;
                }
            }
        }
        return;
    }
    __shared__ DiagBlock s;
    __shared__ int s_cnt[4];
    int unused = 0;
    for (int a = tid; a < d.K; a += 256) unused += !(P[(int64_t)a * ld + a] > 0.0);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) unused += __shfl_xor(unused, off, 64);
    if ((tid & 63) == 0) s_cnt[tid >> 6] = unused;
    load_dref(s, P, ld, 0, tid);
    for (int f = tid; f < PW * PW; f += 256) {
        const int c = f / PW, r = f % PW;
        double x = P[(int64_t)c * ld + r];
        if (r == c && !(x > 0.0)) x = 1.0;
        s.L[r][c] = x;
    }
    factor_diag32(s, tid);                   // synchronises before reading s_cnt
    store_diag_block(d.Ld, 0, s, tid);
    if (tid == 0) {
        int32_t* st = status + 8 * t;
        st[0] = s_cnt[0] + s_cnt[1] + s_cnt[2] + s_cnt[3];
        st[4] = 0;
        st[5] = s.bad;
    }
}

__global__ __launch_bounds__(256) void chol_panel_kernel(const ModDesc* __restrict__ md, int m,
                                                         const int32_t* __restrict__ status, int kb) {
    const int t = blockIdx.y;
    const ModDesc d = md[t];
    const int Kp = d.Kpad;
    if (kb >= Kp || status[8 * t + 5]) return;
    const int ld = Kp + m, tid = threadIdx.x;
    double* W = d.W;
    __shared__ double L[PW][PW + 1];
    __shared__ double rd[PW];
    // this thread's row and the factored diagonal block, requested together
    const int i = kb + PW + blockIdx.x * 256 + tid;
    const int ic = min(i, ld - 1);
    double x[PW];
#pragma unroll
    for (int c = 0; c < PW; ++c) x[c] = gld(W, 8u * (uint32_t)((kb + c) * ld + ic));
    const double* Lb = d.Ld + (int64_t)kb * PW;
    double lv[PW * PW / 256];
#pragma unroll
    for (int u = 0; u < PW * PW / 256; ++u) lv[u] = Lb[tid + 256 * u];
    const double dv = tid < PW ? Lb[tid * PW + tid] : 1.0;
#pragma unroll
    for (int u = 0; u < PW * PW / 256; ++u) {
        const int f = tid + 256 * u;
        L[f % PW][f / PW] = lv[u];
    }
    if (tid < PW) rd[tid] = 1.0 / dv;
    __syncthreads();
    if (i >= ld) return;
#pragma unroll
    for (int c = 0; c < PW; ++c) {
        x[c] *= rd[c];
#pragma unroll
        for (int c2 = c + 1; c2 < PW; ++c2) x[c2] = fma(-x[c], L[c2][c], x[c2]);
        __asm__ volatile("" ::: "memory");             // keep column c's LDS reads in this step
    }
#pragma unroll
    for (int c = 0; c < PW; ++c) gst(W, 8u * (uint32_t)((kb + c) * ld + i), x[c]);
    if (i < Kp) {
#pragma unroll
        for (int c = 0; c < PW; ++c) gst(W, 8u * (uint32_t)(i * ld + kb + c), x[c]);   // mirror
    }
}

// Tiles of the trailing update after the panel at kb: the lower triangle of the A block in
// UT x UT tiles, then the B rows (UT rows per tile) against every A column tile.
__host__ __device__ inline int update_tiles(int Kp, int m, int kb) {
    const int r0 = kb + PW;
    if (r0 >= Kp) return 0;
    const int TA = (Kp - r0 + UT - 1) / UT;
    return TA * (TA + 1) / 2 + (m + UT - 1) / UT * TA;
}

// The next diagonal block (rows and columns r0 .. r0 + 31) after the update with the panel at kb,
// into s.L (one wave; the three 16 x 16 blocks on and below the diagonal).  Every lead tile forms
// it from the same operands in the same MFMA order, so all of them hold the same bits.
__device__ __forceinline__ void diag_update32(DiagBlock& s, const double* W, int ld, int kb, int r0, int lane) {
    const int kq = lane >> 4, li = lane & 15;
    double av[2][PW / 4];
#pragma unroll
    for (int u = 0; u < PW / 4; ++u) {
        const uint32_t colk = (uint32_t)(kb + 4 * u + kq) * ld;
#pragma unroll
        for (int b = 0; b < 2; ++b) av[b][u] = gld(W, 8u * (colk + r0 + 16 * b + li));
    }
    double old[2][2][4];
#pragma unroll
    for (int rb = 0; rb < 2; ++rb)
#pragma unroll
        for (int cb = 0; cb <= rb; ++cb)
#pragma unroll
            for (int q = 0; q < 4; ++q)
                old[rb][cb][q] = gld(W, 8u * (uint32_t)((r0 + 16 * cb + kq + 4 * q) * ld + r0 + 16 * rb + li));
#pragma unroll
    for (int rb = 0; rb < 2; ++rb)
#pragma unroll
        for (int cb = 0; cb <= rb; ++cb) {
            f64x4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int u = 0; u < PW / 4; ++u)
                acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av[cb][u], av[rb][u], acc, 0, 0, 0);
#pragma unroll
            for (int q = 0; q < 4; ++q) s.L[16 * rb + li][16 * cb + kq + 4 * q] = old[rb][cb][q] - acc[q];
        }
}

// The trailing update after the panel at kb, fused with the row solves of the next panel.  Tiles
// of the first column block ("lead" tiles) keep the updated next-panel columns of their 64 rows in
// LDS, form and factor the next diagonal block themselves, solve their rows against it (written in
// place and, for A rows, mirrored) and so leave the next panel solved for the next launch.  The
// work group of the first tile also stores the factored block in the side array Ld.  No work group
// writes the next diagonal block of W, which the lead tiles read.  Compiled for three waves per
// SIMD (168 registers, 12 of them spilled to 52 bytes of scratch; 190 registers and two work groups
// per CU otherwise): 33.4 against 36.9 ms for the 920 launches of the large workload's step.
__global__ __launch_bounds__(256, 3) void chol_update_kernel(const ModDesc* __restrict__ md, int m,
                                                          int32_t* __restrict__ status, int kb) {
    const int t = blockIdx.y;
    const ModDesc d = md[t];
    const int Kp = d.Kpad;
    const int tile = blockIdx.x;
    if (tile >= update_tiles(Kp, m, kb) || status[8 * t + 5]) return;
    const int ld = Kp + m, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    double* W = d.W;
    const int r0 = kb + PW;
    const int TA = (Kp - r0 + UT - 1) / UT;
    const int nA = TA * (TA + 1) / 2;
    int ib, jb, rowbase, rowlim;
    const bool isA = tile < nA;
    if (isA) {
        ib = (int)((sqrtf(8.f * tile + 1.f) - 1.f) * 0.5f);
        while ((ib + 1) * (ib + 2) / 2 <= tile) ++ib;
        while (ib * (ib + 1) / 2 > tile) --ib;
        jb = tile - ib * (ib + 1) / 2;
        rowbase = r0 + UT * ib;
        rowlim = Kp;
    } else {
        ib = (tile - nA) / TA;
        jb = (tile - nA) % TA;
        rowbase = Kp + UT * ib;
        rowlim = ld;
    }
    const bool first = tile == 0;            // A, ib = jb = 0: its first quarter is the next diagonal block
    const bool lead = jb == 0;
    __shared__ DiagBlock s;
    __shared__ double T[UT][PW + 1];         // lead tiles: updated next-panel columns of the 64 rows
    const int qr = wave >> 1, qc = wave & 1;
    const bool diag_tile = isA && ib == jb;
    const int R = rowbase + 32 * qr, C = r0 + UT * jb + 32 * qc;
    const bool wave_on = !(diag_tile && qc > qr) && !(first && qr == 0 && qc == 0) && R < rowlim && C < Kp;
    if (wave_on) {
        const int kq = lane >> 4, li = lane & 15;
        bool blk[2][2];
#pragma unroll
        for (int rb = 0; rb < 2; ++rb)
#pragma unroll
            for (int cb = 0; cb < 2; ++cb)
                blk[rb][cb] = R + 16 * rb < rowlim && C + 16 * cb < Kp && !(diag_tile && qr == qc && cb > rb);
        const bool to_lds = lead && qc == 0;
        double av[2][PW / 4], bv[2][PW / 4];
        double old[2][2][4];
#pragma unroll
        for (int u = 0; u < PW / 4; ++u) {
            const uint32_t colk = (uint32_t)(kb + 4 * u + kq) * ld;
#pragma unroll
            for (int cb = 0; cb < 2; ++cb) av[cb][u] = gld(W, 8u * (colk + min(C + 16 * cb + li, Kp - 1)));
#pragma unroll
            for (int rb = 0; rb < 2; ++rb) bv[rb][u] = gld(W, 8u * (colk + min(R + 16 * rb + li, rowlim - 1)));
        }
#pragma unroll
        for (int rb = 0; rb < 2; ++rb) {
            const int row = R + 16 * rb + li;
#pragma unroll
            for (int cb = 0; cb < 2; ++cb)
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    old[rb][cb][q] = blk[rb][cb] && row < rowlim
                        ? gld(W, 8u * (uint32_t)((C + 16 * cb + kq + 4 * q) * ld + row)) : 0.0;
        }
#pragma unroll
        for (int rb = 0; rb < 2; ++rb) {
            const int row = R + 16 * rb + li;
#pragma unroll
            for (int cb = 0; cb < 2; ++cb) {
                if (!blk[rb][cb]) continue;
                f64x4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
                for (int u = 0; u < PW / 4; ++u)
                    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av[cb][u], bv[rb][u], acc, 0, 0, 0);
                // acc[q]: the update of W at row R + 16 rb + li, column C + 16 cb + kq + 4 q
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const double v = old[rb][cb][q] - acc[q];
                    if (to_lds) T[32 * qr + 16 * rb + li][16 * cb + kq + 4 * q] = v;
                    else if (row < rowlim) gst(W, 8u * (uint32_t)((C + 16 * cb + kq + 4 * q) * ld + row), v);
                }
            }
        }
    }
    if (!lead) return;
    if (wave == 1) diag_update32(s, W, ld, kb, r0, lane);
    load_dref(s, d.A, ld, r0, tid);
    factor_diag32(s, tid);                   // synchronises before reading s.L and T
    if (first) {
        store_diag_block(d.Ld, r0, s, tid);
        if (tid == 0 && s.bad) status[8 * t + 5] = 1;
    }
    // this tile's rows of the next panel (not the diagonal block itself): x L^T = w
    if (tid < UT) {
        const int row = rowbase + tid;
        if (row < rowlim && !(first && tid < PW)) {
            double x[PW];
#pragma unroll
            for (int c = 0; c < PW; ++c) x[c] = T[tid][c];
#pragma unroll
            for (int c = 0; c < PW; ++c) {
                x[c] *= s.rd[c];
#pragma unroll
                for (int c2 = c + 1; c2 < PW; ++c2) x[c2] = fma(-x[c], s.L[c2][c], x[c2]);
                __asm__ volatile("" ::: "memory");         // keep column c's LDS reads in this step
            }
#pragma unroll
            for (int c = 0; c < PW; ++c) gst(W, 8u * (uint32_t)((r0 + c) * ld + row), x[c]);
            if (row < Kp) {
#pragma unroll
                for (int c = 0; c < PW; ++c) gst(W, 8u * (uint32_t)(row * ld + r0 + c), x[c]);   // mirror
            }
        }
    }
}

// D L = Z for 16 rows of D per work group: block columns of SB from the last; the product
// D_{>J} L_{>J,J} of the 16 rows is split over the TW waves by k and summed in LDS, then 16
// threads solve the 32 x 32 triangle of the block column, one row of D each.  The diagonal block
// and the right-hand sides of a block column are requested together with the product's
// operands, so that each block column waits on global memory about once.  TW: 4 waves when the
// launch has many work groups, 8 when it has few (more of the product in flight per group;
// 16 waves measured slower: 452 against 307 us at K = 1024, m = 256).  The 4-wave form is held
// to 128 registers, so that four work groups fit per CU instead of two: 531 against 604 us for
// 100 dictionaries at K = 512, m = 256.  Solving the triangle with four lanes per row of D (DPP
// broadcasts of each finished entry) measured slower in both forms.
template <int TW>
__global__ __launch_bounds__(64 * TW, TW == 4 ? 4 : 2)
void tri_solve_rows_kernel(const ModDesc* __restrict__ md, int m, const int32_t* __restrict__ status) {
    constexpr int NT = 64 * TW;
    constexpr int NL = (SB * SB + NT - 1) / NT;      // diagonal-block entries per thread
    constexpr int NZ = (16 * SB + NT - 1) / NT;      // right-hand-side entries per thread
    constexpr int UB = TW == 8 ? 16 : 8;             // MFMA steps per batch of loads
    const int t = blockIdx.y;
    if (status[8 * t + 4]) return;
    const ModDesc d = md[t];
    const int Kp = d.Kpad, ld = Kp + m;
    double* W = d.W;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int rb0 = 16 * blockIdx.x;
    const int kq = lane >> 4, li = lane & 15;
    __shared__ double Lj[SB][SB + 1];
    __shared__ double rd[SB];
    __shared__ double part[TW][2][16][17];
    __shared__ double Tt[16][SB + 1];
    const uint32_t zrow = (uint32_t)(Kp + min(rb0 + li, m - 1));     // this lane's row of D (clamped)
    // the diagonal blocks: from the side array, or from W after the one-work-group retry
    const bool retried = status[8 * t + 5] != 0;
    for (int J = Kp - SB; J >= 0; J -= SB) {
        double lv[NL], zv[NZ];
#pragma unroll
        for (int u = 0; u < NL; ++u) {
            const int f = tid + u * NT, c = f / SB, r = f % SB;
            lv[u] = f < SB * SB && r >= c
                ? (retried ? gld(W, 8u * (uint32_t)((J + c) * ld + J + r)) : d.Ld[(int64_t)J * SB + f]) : 0.0;
        }
        const double dv = tid < SB ? (retried ? gld(W, 8u * (uint32_t)((J + tid) * ld + J + tid))
                                              : d.Ld[(int64_t)J * SB + tid * SB + tid]) : 1.0;
#pragma unroll
        for (int u = 0; u < NZ; ++u) {
            const int f = tid + u * NT, r = f & 15, c = f >> 4;
            zv[u] = f < 16 * SB && rb0 + r < m ? gld(W, 8u * (uint32_t)((J + c) * ld + Kp + rb0 + r)) : 0.0;
        }
        // this wave's share of the k range, in MFMA steps of 4
        const int S = (Kp - J - SB) / 4;
        const int kbeg = J + SB + 4 * (wave * S / TW);
        const int kw = 4 * ((wave + 1) * S / TW - wave * S / TW);
        f64x4 acc0 = {0.0, 0.0, 0.0, 0.0}, acc1 = {0.0, 0.0, 0.0, 0.0};
        for (int k0 = 0; k0 < kw; k0 += 4 * UB) {
            double av[UB], b0[UB], b1[UB];
#pragma unroll
            for (int u = 0; u < UB; ++u) {
                const int i = kbeg + min(k0 + 4 * u, kw - 4) + kq;
                av[u] = gld(W, 8u * ((uint32_t)i * ld + zrow));                            // D[r][i]
                b0[u] = gld(W, 8u * (uint32_t)(i * ld + J + li));                          // L[i][J + c]
                b1[u] = gld(W, 8u * (uint32_t)(i * ld + J + 16 + li));
            }
#pragma unroll
            for (int u = 0; u < UB; ++u) {
                if (k0 + 4 * u < kw) {
                    acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u], b0[u], acc0, 0, 0, 0);
                    acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u], b1[u], acc1, 0, 0, 0);
                }
            }
        }
        // (the previous block column's solve has finished: the barrier closing its iteration)
#pragma unroll
        for (int u = 0; u < NL; ++u) {
            const int f = tid + u * NT;
            if (f < SB * SB) Lj[f % SB][f / SB] = lv[u];
        }
        if (tid < SB) rd[tid] = 1.0 / dv;
        // acc[q]: row kq + 4 q of the 16, column 16 cb + li of the block column
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            part[wave][0][kq + 4 * q][li] = acc0[q];
            part[wave][1][kq + 4 * q][li] = acc1[q];
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < NZ; ++u) {
            const int f = tid + u * NT, r = f & 15, c = f >> 4;
            if (f < 16 * SB && rb0 + r < m) {
                double v = zv[u];
#pragma unroll
                for (int w = 0; w < TW; ++w) v -= part[w][c >> 4][r][c & 15];
                Tt[r][c] = v;
            }
        }
        __syncthreads();
        if (tid < 16 && rb0 + tid < m) {
            double x[SB];
#pragma unroll
            for (int c = 0; c < SB; ++c) x[c] = Tt[tid][c];
#pragma unroll
            for (int c = SB - 1; c >= 0; --c) {
                x[c] *= rd[c];
#pragma unroll
                for (int c2 = 0; c2 < c; ++c2) x[c2] = fma(-x[c], Lj[c][c2], x[c2]);
                __asm__ volatile("" ::: "memory");
            }
#pragma unroll
            for (int c = 0; c < SB; ++c) gst(W, 8u * (uint32_t)((J + c) * ld + Kp + rb0 + tid), x[c]);
        }
        __syncthreads();
    }
}

// Unit-normalise the solved atoms and store them (one wave per atom).
__global__ __launch_bounds__(256) void mod_normalize_kernel(const ModDesc* __restrict__ md, int m,
                                                            const int32_t* __restrict__ status) {
    const int t = blockIdx.y;
    if (status[8 * t + 4]) return;
    const ModDesc d = md[t];
    const int lane = threadIdx.x & 63;
    const int j = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (j >= d.K) return;
    const int ld = d.Kpad + m;
    if (!(d.A[(int64_t)j * ld + j] > 0.0)) return;      // unused atom: keep its value
    const double* col = d.W + (int64_t)j * ld + d.Kpad;
    double ss = 0.0;
    for (int r = lane; r < m; r += 64) ss += col[r] * col[r];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) ss += __shfl_xor(ss, off, 64);
    const double inv = ss > 0.0 ? 1.0 / sqrt(ss) : 1.0;
    for (int r = lane; r < m; r += 64) d.D[(int64_t)j * m + r] = (float)(col[r] * inv);
}

}  // namespace

// The multi-work-group solve unless the dictionaries alone fill the chip (one work group each).
static bool mod_solve_multi(int n_desc, int solver) {
    if (solver != 0) return solver == 1;
    return n_desc < 256;
}

int64_t mod_csc_blocks(int64_t max_n) { return std::max<int64_t>(1, (max_n + CSC_FILL_SIG - 1) / CSC_FILL_SIG); }

hipError_t launch_mod(const ModDesc* dev_desc, int n_desc, int m, int total_atoms, int64_t max_n, int32_t* cnt,
                      int32_t* fill, int32_t* ptr, int32_t* list_sig, float* list_coef, int32_t* status,
                      int max_kpad, double* arena, double* part, int64_t arena_len, int chunks, int solver,
                      int32_t* bcnt, int32_t* bbase, hipStream_t st) {
    hipError_t e;
    if (chunks < 1 || (chunks > 1 && !part)) return hipErrorInvalidValue;
    const bool fixed = bcnt != nullptr;
    if (fixed && !bbase) return hipErrorInvalidValue;
    if ((e = launch_zero_i32(cnt, total_atoms, st)) != hipSuccess) return e;
    if ((e = launch_zero_i32(fill, total_atoms, st)) != hipSuccess) return e;
    // the fixed-order mode counts per block of the fill kernel (its run bases come from them)
    const unsigned csc_blocks = (unsigned)std::max<int64_t>(1, (max_n + CSC_SIG - 1) / CSC_SIG);
    const unsigned fill_blocks = (unsigned)std::max<int64_t>(1, (max_n + CSC_FILL_SIG - 1) / CSC_FILL_SIG);
    hipLaunchKernelGGL(csc_count_kernel, dim3(fixed ? fill_blocks : csc_blocks, n_desc), dim3(256), 0, st, dev_desc,
                       cnt, status, bcnt, total_atoms, fixed ? CSC_FILL_SIG : CSC_SIG);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(scan_kernel, dim3(1), dim3(1024), 0, st, cnt, total_atoms, ptr);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (fixed) {
        hipLaunchKernelGGL(csc_block_base_kernel, dim3((total_atoms + 255) / 256), dim3(256), 0, st, ptr, bcnt, bbase,
                           total_atoms, (int)fill_blocks);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        hipLaunchKernelGGL(csc_fill_kernel<true>, dim3(fill_blocks, n_desc), dim3(CSC_FILL_SIG), 0, st, dev_desc, ptr,
                           fill, bbase, total_atoms, list_sig, list_coef);
    } else {
        hipLaunchKernelGGL(csc_fill_kernel<false>, dim3(fill_blocks, n_desc), dim3(CSC_FILL_SIG), 0, st, dev_desc, ptr,
                           fill, (const int32_t*)nullptr, total_atoms, list_sig, list_coef);
    }
    if ((e = hipGetLastError()) != hipSuccess) return e;
    // The kernel fits 8 blocks per CU (14 KB of LDS each).  When a dictionary's signals exceed an
    // XCD's 4 MB L2, fewer blocks in flight gather from fewer dictionaries at once: unused dynamic
    // LDS caps the launch at 6 blocks per CU (at m=256 and 10^4 signals per dictionary 5 % faster
    // than 8 blocks; 3, 4 and 5 blocks are slower than 6).  The fixed-order mode's masks take
    // 36 bytes per atom of dynamic LDS.
    static_assert(8 * MP_LDS <= 160 * 1024, "8 blocks of mod_products_kernel per CU");
    if (fixed) {
        hipLaunchKernelGGL(mod_products_kernel<true>, dim3(max_kpad, n_desc, chunks), dim3(256),
                           (unsigned)max_kpad * 36u, st, dev_desc, m, ptr, list_sig, list_coef, arena, part, arena_len);
    } else {
        const bool mp_cap = (int64_t)max_n * m * 4 > ((int64_t)4 << 20);
        const unsigned mp_pad = mp_cap ? (unsigned)(160 * 1024 / 6 - 1024 - MP_LDS) : 0u;
        hipLaunchKernelGGL(mod_products_kernel<false>, dim3(max_kpad, n_desc, chunks), dim3(256), mp_pad, st, dev_desc,
                           m, ptr, list_sig, list_coef, arena, part, arena_len);
    }
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (chunks > 1) {
        const unsigned g = (unsigned)std::min<int64_t>(4096, (arena_len + 255) / 256);
        hipLaunchKernelGGL(sum_reduce_kernel, dim3(g), dim3(256), 0, st, arena, part, arena_len, chunks - 1);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    if (mod_solve_multi(n_desc, solver)) {
        const int64_t cells = (int64_t)max_kpad * (max_kpad + m);
        const unsigned sg = 1 + (unsigned)std::min<int64_t>(64, std::max<int64_t>(1, (cells + 4095) / 4096));
        hipLaunchKernelGGL(chol_setup_kernel, dim3(sg, n_desc), dim3(256), 0, st, dev_desc, m, status);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        // the first panel's rows; every later panel is solved by the update launch before it
        const unsigned pg = (unsigned)((max_kpad + m - PW + 255) / 256);
        hipLaunchKernelGGL(chol_panel_kernel, dim3(pg, n_desc), dim3(256), 0, st, dev_desc, m, status, 0);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        for (int kb = 0; kb + PW < max_kpad; kb += PW) {
            hipLaunchKernelGGL(chol_update_kernel, dim3(update_tiles(max_kpad, m, kb), n_desc), dim3(256), 0, st,
                               dev_desc, m, status, kb);
            if ((e = hipGetLastError()) != hipSuccess) return e;
        }
        hipLaunchKernelGGL(chol_factor_kernel, dim3(n_desc), dim3(CT), 0, st, dev_desc, m, status, 1);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        const dim3 tg((m + 15) / 16, n_desc);
        const int64_t groups = (int64_t)tg.x * n_desc;
        if (groups >= 512)
            hipLaunchKernelGGL(tri_solve_rows_kernel<4>, tg, dim3(256), 0, st, dev_desc, m, status);
        else
            hipLaunchKernelGGL(tri_solve_rows_kernel<8>, tg, dim3(512), 0, st, dev_desc, m, status);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    } else {
        hipLaunchKernelGGL(chol_factor_kernel, dim3(n_desc), dim3(CT), 0, st, dev_desc, m, status, 0);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        hipLaunchKernelGGL(tri_solve_kernel, dim3(n_desc), dim3(TCS), 0, st, dev_desc, m, status);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    hipLaunchKernelGGL(mod_normalize_kernel, dim3((max_kpad + 3) / 4, n_desc), dim3(256), 0, st, dev_desc, m, status);
    return hipGetLastError();
}

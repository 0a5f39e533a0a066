// MOD dictionary update (least squares D = Y X^T (X X^T)^{-1}) for one or many dictionaries.
//
//  1. csc_count / scan / csc_fill: transpose the ELL codes into per-atom lists of
//     (signal, coefficient) so that every atom's products can be gathered without atomics
//     on global memory.
//  2. mod_products: one block per atom a: column a of A = X X^T (FP64, LDS) and column a of
//     B = Y X^T (FP64 register accumulation over the atom's list), written below each other as
//     column a of the augmented matrix M = [A; B] ((Kpad + m) x Kpad, FP64).
//  3. chol_solve: one block per dictionary: right-looking blocked Cholesky of A that carries the
//     B rows along (they become Z = B L^-T), then D L = Z by back substitution per row, a ridge
//     retry when a pivot is rejected, and unit normalisation of the solved atoms.  Atoms no
//     signal uses get an identity diagonal (their column of A is zero) and keep their value.
#include "smdl_internal.h"

namespace {

constexpr int NB = 32;          // Cholesky panel width
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
// everywhere and flagged in status[4*t + 3] (the host turns that into SMDL_E_ARG).
__device__ __forceinline__ int clamp_nnz(int k, int s) { return k < 0 ? 0 : (k > s ? s : k); }

__global__ void csc_count_kernel(const ModDesc* __restrict__ md, int32_t* __restrict__ cnt,
                                 int32_t* __restrict__ status) {
    const ModDesc d = md[blockIdx.y];
    for (int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; n < d.n;
         n += (int64_t)gridDim.x * blockDim.x) {
        const int k0 = d.nnz[n];
        const int k = clamp_nnz(k0, d.s_stride);
        bool bad = k != k0;
        for (int i = 0; i < k; ++i) {
            const int ix = d.idx[n * d.s_stride + i];
            if (ix < 0 || ix >= d.K) { bad = true; continue; }
            atomicAdd(&cnt[d.atom0 + ix], 1);
        }
        if (bad) atomicOr(&status[4 * blockIdx.y + 3], 1);
    }
}

// Exclusive scan of cnt[0..total) into ptr[0..total]; single block of 1024 threads.
__global__ __launch_bounds__(1024) void scan_kernel(const int32_t* __restrict__ cnt, int total,
                                                    int32_t* __restrict__ ptr) {
    __shared__ int32_t part[1024];
    const int per = (total + 1023) / 1024;
    const int b = threadIdx.x * per, e = min(total, b + per);
    int32_t s = 0;
    for (int i = b; i < e; ++i) s += cnt[i];
    part[threadIdx.x] = s;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        int32_t v = (int)threadIdx.x >= off ? part[threadIdx.x - off] : 0;
        __syncthreads();
        part[threadIdx.x] += v;
        __syncthreads();
    }
    int32_t run = threadIdx.x > 0 ? part[threadIdx.x - 1] : 0;
    for (int i = b; i < e; ++i) {
        ptr[i] = run;
        run += cnt[i];
    }
    if (threadIdx.x == 1023) ptr[total] = part[1023];
}

__global__ void csc_fill_kernel(const ModDesc* __restrict__ md, const int32_t* __restrict__ ptr,
                                int32_t* __restrict__ fill, int32_t* __restrict__ list_sig,
                                float* __restrict__ list_coef) {
    const ModDesc d = md[blockIdx.y];
    for (int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; n < d.n;
         n += (int64_t)gridDim.x * blockDim.x) {
        const int k = clamp_nnz(d.nnz[n], d.s_stride);
        for (int i = 0; i < k; ++i) {
            const int ix = d.idx[n * d.s_stride + i];
            if (ix < 0 || ix >= d.K) continue;
            const int64_t ga = d.atom0 + ix;
            const int pos = ptr[ga] + atomicAdd(&fill[ga], 1);
            list_sig[pos] = (int32_t)n;
            list_coef[pos] = d.coef[n * d.s_stride + i];
        }
    }
}

// One block per (atom a, descriptor).  Writes column a of M = [A; B] (FP64).
__global__ __launch_bounds__(256) void mod_products_kernel(const ModDesc* __restrict__ md, int m,
                                                           const int32_t* __restrict__ ptr,
                                                           const int32_t* __restrict__ list_sig,
                                                           const float* __restrict__ list_coef) {
    const ModDesc d = md[blockIdx.y];
    const int a = blockIdx.x;
    if (a >= d.Kpad) return;
    __shared__ double colA[SMDL_MAX_K];
    __shared__ double partB[4][SMDL_MAX_M];
    const int tid = threadIdx.x;
    for (int l = tid; l < d.Kpad; l += 256) colA[l] = 0.0;
    __syncthreads();
    const int64_t ld = d.Kpad + m;
    double* out = d.A + (int64_t)a * ld;
    if (a < d.K) {
        const int64_t ga = d.atom0 + a;
        const int b = ptr[ga], e = ptr[ga + 1];
        // A column: every entry (n, x_na) adds x_na * x_nl at every atom l of signal n
        for (int p = b + tid; p < e; p += 256) {
            const int64_t n = list_sig[p];
            const double xa = list_coef[p];
            const int k = clamp_nnz(d.nnz[n], d.s_stride);
            for (int i = 0; i < k; ++i) {
                const int l = d.idx[n * d.s_stride + i];
                if (l < 0 || l >= d.K) continue;
                atomicAdd(&colA[l], xa * (double)d.coef[n * d.s_stride + i]);
            }
        }
        // B column: rows split over threads, entries over groups of threads
        const int mcov = m <= 64 ? 64 : (m <= 128 ? 128 : 256);
        const int groups = 256 / mcov;
        const int r = tid % mcov, grp = tid / mcov;
        double acc = 0.0;
        if (r < m) {
            for (int p = b + grp; p < e; p += groups) {
                const int64_t n = list_sig[p];
                acc += (double)list_coef[p] * (double)d.Y[n * m + r];
            }
        }
        partB[grp][r] = acc;
    } else {
        const int mcov = m <= 64 ? 64 : (m <= 128 ? 128 : 256);
        partB[tid / mcov][tid % mcov] = 0.0;
    }
    __syncthreads();
    for (int l = tid; l < d.Kpad; l += 256) out[l] = colA[l];
    const int mcov = m <= 64 ? 64 : (m <= 128 ? 128 : 256);
    const int groups = 256 / mcov;
    for (int r = tid; r < m; r += 256) {
        double s = 0.0;
        for (int q = 0; q < groups; ++q) s += partB[q][r];
        out[d.Kpad + r] = s;
    }
}

// One block (256 threads) per dictionary.
// status[4*t + 0] = unused atoms (this call), [1] |= ridge used, [2] |= failed; the caller zeroes
// the status array before a sequence of updates.
__global__ __launch_bounds__(256) void chol_solve_kernel(const ModDesc* __restrict__ md, int m,
                                                         int32_t* __restrict__ status) {
    const ModDesc d = md[blockIdx.x];
    const int tid = threadIdx.x;
    const int Kp = d.Kpad;
    const int64_t ld = Kp + m;          // rows of M
    const double* P = d.A;              // pristine products
    double* W = d.W;                    // factorisation workspace
    __shared__ double Ld[NB][NB + 1];
    __shared__ double diag0[SMDL_MAX_K];
    __shared__ unsigned char active[SMDL_MAX_K];
    __shared__ int s_fail;
    __shared__ double s_red[256];
    __shared__ int s_cnt[256];

    // max active diagonal and unused count
    double mx = 0.0;
    int unused = 0;
    for (int a = tid; a < Kp; a += 256) {
        const double v = P[(int64_t)a * ld + a];
        active[a] = v > 0.0;
        if (v > mx) mx = v;
        if (a < d.K && !(v > 0.0)) ++unused;
    }
    s_red[tid] = mx;
    s_cnt[tid] = unused;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (tid < w) {
            s_red[tid] = fmax(s_red[tid], s_red[tid + w]);
            s_cnt[tid] += s_cnt[tid + w];
        }
        __syncthreads();
    }
    const double maxdiag = s_red[0];
    if (tid == 0) status[4 * blockIdx.x + 0] = s_cnt[0];
    __shared__ int s_failed_final;
    if (tid == 0) s_failed_final = 0;
    __syncthreads();

    for (int attempt = 0; attempt < 2; ++attempt) {
        const double lam = attempt == 0 ? 0.0 : RIDGE * maxdiag;
        // W = P (+ lam I on active atoms, identity on unused ones)
        const int64_t total = ld * Kp;
        for (int64_t f = tid; f < total; f += 256) {
            const int64_t col = f / ld;
            const int64_t row = f - col * ld;
            double v = P[f];
            if (row == col) v = active[col] ? v + lam : 1.0;
            W[f] = v;
        }
        for (int a = tid; a < Kp; a += 256) diag0[a] = active[a] ? P[(int64_t)a * ld + a] + lam : 1.0;
        if (tid == 0) s_fail = 0;
        __syncthreads();

        for (int kb = 0; kb < Kp; kb += NB) {
            // (i) factor the diagonal block with one wave (in-order LDS within a wave)
            if (tid < 64) {
                for (int f = tid; f < NB * NB; f += 64) {
                    const int i = f / NB, j = f % NB;
                    Ld[i][j] = W[(int64_t)(kb + j) * ld + kb + i];
                }
                __builtin_amdgcn_s_waitcnt(0);
                __builtin_amdgcn_wave_barrier();
                for (int j = 0; j < NB; ++j) {
                    double dj = Ld[j][j];
                    const bool bad = !(dj > PIV_TOL * diag0[kb + j]);
                    dj = bad ? 1.0 : sqrt(dj);
                    if (bad && tid == 0) s_fail = 1;
                    __builtin_amdgcn_wave_barrier();
                    if (tid == 0) Ld[j][j] = dj;
                    if (tid > j && tid < NB) Ld[tid][j] /= dj;
                    __builtin_amdgcn_s_waitcnt(0);
                    __builtin_amdgcn_wave_barrier();
                    // rank-1 update of the trailing part of the block
                    for (int f = tid; f < NB * NB; f += 64) {
                        const int i = f / NB, c = f % NB;
                        if (c > j && i >= c) Ld[i][c] -= Ld[i][j] * Ld[c][j];
                    }
                    __builtin_amdgcn_s_waitcnt(0);
                    __builtin_amdgcn_wave_barrier();
                }
                for (int f = tid; f < NB * NB; f += 64) {
                    const int i = f / NB, j = f % NB;
                    if (i >= j) W[(int64_t)(kb + j) * ld + kb + i] = Ld[i][j];
                }
            }
            __syncthreads();
            if (s_fail) break;
            // (ii) panel: rows below the block (A rows and the B rows): x L^T = w
            for (int64_t i = kb + NB + tid; i < ld; i += 256) {
                double x[NB];
#pragma unroll
                for (int c = 0; c < NB; ++c) x[c] = W[(int64_t)(kb + c) * ld + i];
#pragma unroll
                for (int c = 0; c < NB; ++c) {
                    double s = x[c];
#pragma unroll
                    for (int cc = 0; cc < c; ++cc) s -= x[cc] * Ld[c][cc];
                    x[c] = s / Ld[c][c];
                }
#pragma unroll
                for (int c = 0; c < NB; ++c) W[(int64_t)(kb + c) * ld + i] = x[c];
            }
            __syncthreads();
            // (iii) trailing update: W[i][j] -= sum_c W[i][kb+c] W[j][kb+c], j in [kb+NB, Kp),
            //       i in [j, ld); 4x4 register tiles over (i, j)
            const int j0 = kb + NB;
            const int nj = Kp - j0;
            if (nj > 0) {
                const int ni = (int)(ld - j0);
                const int tj = (nj + 3) / 4, ti = (ni + 3) / 4;
                for (int t = tid; t < tj * ti; t += 256) {
                    const int bj = t % tj, bi = t / tj;
                    const int jb = j0 + 4 * bj;
                    const int ib = j0 + 4 * bi;
                    if (ib + 3 < jb) continue;       // tile entirely above the diagonal
                    double acc[4][4];
#pragma unroll
                    for (int u = 0; u < 4; ++u)
#pragma unroll
                        for (int v = 0; v < 4; ++v) acc[u][v] = 0.0;
                    for (int c = 0; c < NB; ++c) {
                        const double* colc = W + (int64_t)(kb + c) * ld;
                        double xi[4], xj[4];
#pragma unroll
                        for (int u = 0; u < 4; ++u) {
                            xi[u] = (ib + u < ld) ? colc[ib + u] : 0.0;
                            xj[u] = (jb + u < Kp) ? colc[jb + u] : 0.0;
                        }
#pragma unroll
                        for (int u = 0; u < 4; ++u)
#pragma unroll
                            for (int v = 0; v < 4; ++v) acc[u][v] += xi[u] * xj[v];
                    }
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int j = jb + v;
                        if (j >= Kp) continue;
#pragma unroll
                        for (int u = 0; u < 4; ++u) {
                            const int64_t i = ib + u;
                            if (i < j || i >= ld) continue;
                            W[(int64_t)j * ld + i] -= acc[u][v];
                        }
                    }
                }
            }
            __syncthreads();
        }
        if (!s_fail) break;
        if (attempt == 0 && tid == 0) atomicOr(&status[4 * blockIdx.x + 1], 1);
        if (attempt == 1 && tid == 0) {
            atomicOr(&status[4 * blockIdx.x + 2], 1);
            s_failed_final = 1;
        }
        __syncthreads();
    }
    if (s_failed_final) return;

    // D L = Z for every row r of D (Z = rows Kp .. Kp+m of W); solved in place in W.
    for (int r = tid; r < m; r += 256) {
        const int64_t zr = Kp + r;
        for (int j = Kp - 1; j >= 0; --j) {
            double s = W[(int64_t)j * ld + zr];
            for (int i = j + 1; i < Kp; ++i) s -= W[(int64_t)i * ld + zr] * W[(int64_t)j * ld + i];
            W[(int64_t)j * ld + zr] = s / W[(int64_t)j * ld + j];
        }
    }
    __syncthreads();
    // normalise and store the active atoms
    for (int j = tid; j < d.K; j += 256) {
        if (!active[j]) continue;
        double ss = 0.0;
        for (int r = 0; r < m; ++r) {
            const double v = W[(int64_t)j * ld + Kp + r];
            ss += v * v;
        }
        const double inv = ss > 0.0 ? 1.0 / sqrt(ss) : 1.0;
        for (int r = 0; r < m; ++r) d.D[(int64_t)j * m + r] = (float)(W[(int64_t)j * ld + Kp + r] * inv);
    }
}

inline int grid_sig(int64_t n) {
    int64_t g = (n + 255) / 256;
    if (g > 4096) g = 4096;
    return (int)(g < 1 ? 1 : g);
}

}  // namespace

hipError_t launch_mod(const ModDesc* dev_desc, const ModDesc* host_desc, int n_desc, int m,
                      int total_atoms, int64_t max_n, int32_t* cnt, int32_t* fill, int32_t* ptr,
                      int32_t* list_sig, float* list_coef, int32_t* status, int max_kpad,
                      hipStream_t st, bool /*per_desc*/) {
    (void)host_desc;
    hipError_t e;
    if ((e = launch_zero_i32(cnt, total_atoms, st)) != hipSuccess) return e;
    if ((e = launch_zero_i32(fill, total_atoms, st)) != hipSuccess) return e;
    hipLaunchKernelGGL(csc_count_kernel, dim3(grid_sig(max_n), n_desc), dim3(256), 0, st, dev_desc, cnt,
                       status);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(scan_kernel, dim3(1), dim3(1024), 0, st, cnt, total_atoms, ptr);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(csc_fill_kernel, dim3(grid_sig(max_n), n_desc), dim3(256), 0, st, dev_desc, ptr,
                       fill, list_sig, list_coef);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(mod_products_kernel, dim3(max_kpad, n_desc), dim3(256), 0, st, dev_desc, m, ptr,
                       list_sig, list_coef);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(chol_solve_kernel, dim3(n_desc), dim3(256), 0, st, dev_desc, m, status);
    return hipGetLastError();
}

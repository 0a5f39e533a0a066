// MOD dictionary update (least squares D = Y X^T (X X^T)^{-1}) for one or many dictionaries.
//
//  1. csc_count / scan / csc_fill: transpose the ELL codes into per-atom lists of
//     (signal, coefficient) so that every atom's products can be gathered without atomics
//     on global memory.
//  2. mod_products: one block per atom a: column a of A = X X^T (FP64, LDS) and column a of
//     B = Y X^T (FP64 register accumulation over the atom's list), written below each other as
//     column a of the augmented matrix M = [A; B] ((Kpad + m) x Kpad, FP64).
//  3. chol_factor: one block per dictionary: blocked FP64 Cholesky of A (MFMA trailing updates),
//     a ridge retry when a pivot is rejected.  Atoms no signal uses get an identity diagonal
//     (their column of A is zero) and keep their value.
//  4. tri_solve: D A = B row by row (forward then backward substitution), many blocks per
//     dictionary; mod_normalize: unit normalisation of the solved atoms.
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
        if (bad) atomicOr(&status[8 * blockIdx.y + 3], 1);
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

// ------------------------------------------------------------------------------------------
// FP64 Cholesky factorisation of A (one block per dictionary)
// ------------------------------------------------------------------------------------------
// status[8*t + 0] = unused atoms (this call), [1] |= ridge used, [2] |= failed, [3] |= bad codes,
// [4] = failed in this call (read by the solve and normalisation kernels).  The caller zeroes
// the status array before a sequence of updates.
//
// Right-looking, panel width FB = 32:
//   (i)   the 32 x 32 diagonal block is factored by one wave with one row per lane in registers,
//         column values broadcast with readlane;
//   (ii)  the rows below it are solved against it (one row per thread, L_kk in LDS);
//   (iii) the trailing lower triangle is updated on the FP64 matrix cores (16 x 16 tiles,
//         v_mfma_f64_16x16x4f64), the panel read from LDS when it fits.
// Finally L is mirrored into the upper triangle (W[i*ld + j] = L[i][j]) so that the backward
// substitution reads rows of L contiguously.
constexpr int FB = 32;
constexpr int CT = 512;
constexpr int PR = 480;                      // panel rows kept in LDS (32 x 480 doubles = 120 KB)

typedef double f64x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ double readlane_f64(double v, int lane) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), lane);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
    return __longlong_as_double(((long long)(unsigned)hi << 32) | (unsigned)lo);
}

__global__ __launch_bounds__(CT) void chol_factor_kernel(const ModDesc* __restrict__ md, int m,
                                                         int32_t* __restrict__ status) {
    const ModDesc d = md[blockIdx.x];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int Kp = d.Kpad;
    const int ld = Kp + m;
    const double* P = d.A;
    double* W = d.W;
    __shared__ double Ld[FB][FB + 1];
    __shared__ double panel[FB * PR];        // panel[c * PR + row]
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
        // W[0:Kp, 0:Kp] = A (+ lam I on active atoms, identity on unused ones)
        const int total = Kp * Kp;
#pragma unroll 4
        for (int f = tid; f < total; f += CT) {
            const int col = f / Kp, row = f - col * Kp;
            double v = P[(int64_t)col * ld + row];
            if (row == col) v = active[col] ? v + lam : 1.0;
            W[(int64_t)col * ld + row] = v;
        }
        for (int a = tid; a < Kp; a += CT) diag0[a] = active[a] ? P[(int64_t)a * ld + a] + lam : 1.0;
        if (tid == 0) s_fail = 0;
        __syncthreads();

        for (int kb = 0; kb < Kp; kb += FB) {
            // (i) diagonal block: lane i < FB holds row i in registers
            if (wave == 0) {
                double a[FB];
#pragma unroll
                for (int c = 0; c < FB; ++c)
                    a[c] = (lane < FB && c <= lane) ? W[(int64_t)(kb + c) * ld + kb + lane] : 0.0;
                bool bad = false;
#pragma unroll
                for (int j = 0; j < FB; ++j) {
                    const double djj = readlane_f64(a[j], j);
                    const bool b = !(djj > PIV_TOL * diag0[kb + j]);
                    bad |= b;
                    const double dj = b ? 1.0 : sqrt(djj);
                    const double rd = 1.0 / dj;
                    a[j] = (lane == j) ? dj : (lane > j ? a[j] * rd : a[j]);
#pragma unroll
                    for (int c = j + 1; c < FB; ++c) {
                        const double lc = readlane_f64(a[j], c);   // L[c][j]
                        if (lane >= c) a[c] = fma(-a[j], lc, a[c]);
                    }
                }
                if (lane == 0 && bad) s_fail = 1;
                if (lane < FB) {
#pragma unroll
                    for (int c = 0; c < FB; ++c) {
                        Ld[lane][c] = c <= lane ? a[c] : 0.0;
                        if (c <= lane) W[(int64_t)(kb + c) * ld + kb + lane] = a[c];
                    }
                }
            }
            __syncthreads();
            if (s_fail) break;
            // (ii) panel rows below the block: x L_kk^T = w
            const int r0 = kb + FB;
            const int R = Kp - r0;
            const bool in_lds = R <= PR;
            for (int rr = tid; rr < R; rr += CT) {
                const int i = r0 + rr;
                double x[FB];
#pragma unroll
                for (int c = 0; c < FB; ++c) x[c] = W[(int64_t)(kb + c) * ld + i];
#pragma unroll
                for (int c = 0; c < FB; ++c) {
                    double sacc = x[c];
#pragma unroll
                    for (int cc = 0; cc < c; ++cc) sacc -= x[cc] * Ld[c][cc];
                    x[c] = sacc / Ld[c][c];
                    __asm__ volatile("" ::: "memory");     // keep the LDS reads of row c here
                }
#pragma unroll
                for (int c = 0; c < FB; ++c) W[(int64_t)(kb + c) * ld + i] = x[c];
                if (in_lds) {
#pragma unroll
                    for (int c = 0; c < FB; ++c) panel[c * PR + rr] = x[c];
                }
            }
            __syncthreads();
            // (iii) trailing update of the lower triangle: 16 x 16 tiles (ib >= jb) on MFMA
            const int T16 = R / 16;                      // R is a multiple of 32
            const int ntile = T16 * (T16 + 1) / 2;
            for (int t = wave; t < ntile; t += CT / 64) {
                // t -> (ib, jb), ib >= jb, enumerated row by row
                int ib = (int)((sqrtf(8.f * t + 1.f) - 1.f) * 0.5f);
                while ((ib + 1) * (ib + 2) / 2 <= t) ++ib;
                while (ib * (ib + 1) / 2 > t) --ib;
                const int jb = t - ib * (ib + 1) / 2;
                f64x4 acc = {0.0, 0.0, 0.0, 0.0};
                const int ri = 16 * ib + (lane & 15), rj = 16 * jb + (lane & 15), kq = lane >> 4;
#pragma unroll
                for (int kc = 0; kc < FB; kc += 4) {
                    double av, bv;
                    if (in_lds) {
                        av = panel[(kc + kq) * PR + ri];
                        bv = panel[(kc + kq) * PR + rj];
                    } else {
                        av = W[(int64_t)(kb + kc + kq) * ld + r0 + ri];
                        bv = W[(int64_t)(kb + kc + kq) * ld + r0 + rj];
                    }
                    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc, 0, 0, 0);
                }
                // FP64 16x16x4 output: D[i][j] sits in lane j + 16 (i % 4), register i / 4, so
                // acc[q] = sum_k X[16 ib + kq + 4 q][k] X[16 jb + (lane & 15)][k]
                const int col = r0 + 16 * jb + (lane & 15);
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int row = r0 + 16 * ib + kq + 4 * q;
                    W[(int64_t)col * ld + row] -= acc[q];
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
    if (s_failed_final) return;
    // mirror: W[i * ld + j] = L[i][j] for j < i (the upper triangle of the Kp x Kp block)
    const int total = Kp * Kp;
    for (int f = tid; f < total; f += CT) {
        const int i = f / Kp, j = f - i * Kp;
        if (j < i) W[(int64_t)i * ld + j] = W[(int64_t)j * ld + i];
    }
}

// ------------------------------------------------------------------------------------------
// Solve D A = B row by row: z L^T = b, then d L = z (grid: (ceil(m / 4), dictionaries))
// ------------------------------------------------------------------------------------------
// One wave per row of D (4 rows per block share the LDS copies of L's diagonal chunks).  Chunks
// of 64 columns: the contributions of the solved chunks are dot products over coalesced loads of
// L (lower part for the forward pass, the mirrored upper part for the backward pass); inside the
// chunk, 64 sequential steps with the chunk's diagonal block in LDS.  The solution overwrites the
// B rows of W (W[j * ld + Kp + r] = D[r][j]).
constexpr int SC = 64;

__global__ __launch_bounds__(256) void tri_solve_kernel(const ModDesc* __restrict__ md, int m,
                                                        const int32_t* __restrict__ status) {
    const int t = blockIdx.y;
    if (status[8 * t + 4]) return;
    const ModDesc d = md[t];
    const int Kp = d.Kpad;
    const int ld = Kp + m;
    const double* P = d.A;
    double* W = d.W;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int r = blockIdx.x * 4 + wave;
    const bool row_ok = r < m;
    __shared__ double Lb[SC][SC + 1];
    __shared__ double zs[4][SMDL_MAX_K];
    // forward: z_j = (b_j - sum_{i<j} L[j][i] z_i) / L[j][j]
    for (int J = 0; J < Kp; J += SC) {
        for (int f = threadIdx.x; f < SC * SC; f += 256) {
            const int c = f / SC, i = f % SC;                 // Lb[i][c] = L[J+i][J+c]
            Lb[i][c] = i >= c ? W[(int64_t)(J + c) * ld + J + i] : 0.0;
        }
        const int j = J + lane;
        double tj = row_ok ? P[(int64_t)j * ld + Kp + r] : 0.0;
        double s0 = 0.0, s1 = 0.0;
        int i = 0;
        for (; i + 2 <= J; i += 2) {
            s0 += W[(int64_t)i * ld + j] * zs[wave][i];
            s1 += W[(int64_t)(i + 1) * ld + j] * zs[wave][i + 1];
        }
        for (; i < J; ++i) s0 += W[(int64_t)i * ld + j] * zs[wave][i];
        tj -= s0 + s1;
        __syncthreads();
        for (int jj = 0; jj < SC; ++jj) {
            const double zj = readlane_f64(tj / Lb[lane][lane], jj);
            if (lane > jj) tj = fma(-Lb[lane][jj], zj, tj);
            if (lane == jj) tj = zj;
        }
        zs[wave][j] = tj;
        __syncthreads();
    }
    // backward: d_j = (z_j - sum_{i>j} L[i][j] d_i) / L[j][j], L[i][j] = W[i * ld + j] (mirror)
    for (int J = Kp - SC; J >= 0; J -= SC) {
        for (int f = threadIdx.x; f < SC * SC; f += 256) {
            const int c = f / SC, i = f % SC;
            Lb[i][c] = i >= c ? W[(int64_t)(J + c) * ld + J + i] : 0.0;
        }
        const int j = J + lane;
        double tj = zs[wave][j];
        double s0 = 0.0, s1 = 0.0;
        int i = J + SC;
        for (; i + 2 <= Kp; i += 2) {
            s0 += W[(int64_t)i * ld + j] * zs[wave][i];
            s1 += W[(int64_t)(i + 1) * ld + j] * zs[wave][i + 1];
        }
        for (; i < Kp; ++i) s0 += W[(int64_t)i * ld + j] * zs[wave][i];
        tj -= s0 + s1;
        __syncthreads();
        for (int jj = SC - 1; jj >= 0; --jj) {
            const double dj = readlane_f64(tj / Lb[lane][lane], jj);
            if (lane < jj) tj = fma(-Lb[jj][lane], dj, tj);
            if (lane == jj) tj = dj;
        }
        zs[wave][j] = tj;                                    // z of this chunk is now d
        __syncthreads();
    }
    if (row_ok)
        for (int j = lane; j < Kp; j += 64) W[(int64_t)j * ld + Kp + r] = zs[wave][j];
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
    hipLaunchKernelGGL(chol_factor_kernel, dim3(n_desc), dim3(CT), 0, st, dev_desc, m, status);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(tri_solve_kernel, dim3((m + 3) / 4, n_desc), dim3(256), 0, st, dev_desc, m, status);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(mod_normalize_kernel, dim3((max_kpad + 3) / 4, n_desc), dim3(256), 0, st, dev_desc, m, status);
    return hipGetLastError();
}

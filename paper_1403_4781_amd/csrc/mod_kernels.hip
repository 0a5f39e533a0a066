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

constexpr int NB = 16;          // Cholesky panel width
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

// One block (512 threads) per dictionary.
// status[4*t + 0] = unused atoms (this call), [1] |= ridge used, [2] |= failed; the caller zeroes
// the status array before a sequence of updates.
constexpr int CT = 512;                       // threads of the solve
constexpr int PANEL_LDS_ROWS = 896;           // panel rows kept in LDS (896 x 16 doubles = 112 KB)

__global__ __launch_bounds__(CT) void chol_solve_kernel(const ModDesc* __restrict__ md, int m,
                                                        int32_t* __restrict__ status) {
    const ModDesc d = md[blockIdx.x];
    const int tid = threadIdx.x;
    const int Kp = d.Kpad;
    const int64_t ld = Kp + m;          // rows of M = [A; B]
    const double* P = d.A;              // pristine products
    double* W = d.W;                    // factorisation workspace
    __shared__ double Ld[NB][NB + 1];
    __shared__ double panel[PANEL_LDS_ROWS * NB];
    __shared__ double diag0[SMDL_MAX_K];
    __shared__ unsigned char active[SMDL_MAX_K];
    __shared__ int s_fail, s_failed_final;
    __shared__ double s_red[CT / 64];
    __shared__ int s_cnt[CT / 64];

    // max active diagonal and unused count
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
    if ((tid & 63) == 0) {
        s_red[tid >> 6] = mx;
        s_cnt[tid >> 6] = unused;
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
        status[4 * blockIdx.x + 0] = c;
    }
    __syncthreads();
    const double maxdiag = s_red[0];

    for (int attempt = 0; attempt < 2; ++attempt) {
        const double lam = attempt == 0 ? 0.0 : RIDGE * maxdiag;
        // W = P (+ lam I on active atoms, identity on unused ones)
        const int ldi = (int)ld;
        const int total = ldi * Kp;                 // < 2^31: (1024 + 256) * 1024
#pragma unroll 4
        for (int f = tid; f < total; f += CT) {
            const int col = f / ldi;
            const int row = f - col * ldi;
            double v = P[f];
            if (row == col) v = active[col] ? v + lam : 1.0;
            W[f] = v;
        }
        for (int a = tid; a < Kp; a += CT) diag0[a] = active[a] ? P[(int64_t)a * ld + a] + lam : 1.0;
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
            // (ii) panel rows below the block (A rows and the B rows): x L^T = w
            const int64_t r0 = kb + NB;
            const int R = (int)(ld - r0);
            const bool in_lds = R + 4 <= PANEL_LDS_ROWS;      // tiles read up to 3 rows past R
            for (int rr = tid; rr < R; rr += CT) {
                const int64_t i = r0 + rr;
                double x[NB];
#pragma unroll
                for (int c = 0; c < NB; ++c) x[c] = W[(int64_t)(kb + c) * ld + i];
#pragma unroll
                for (int c = 0; c < NB; ++c) {
                    double sacc = x[c];
#pragma unroll
                    for (int cc = 0; cc < c; ++cc) sacc -= x[cc] * Ld[c][cc];
                    x[c] = sacc / Ld[c][c];
                    __asm__ volatile("" ::: "memory");   // keep the LDS reads of row c here
                }
#pragma unroll
                for (int c = 0; c < NB; ++c) W[(int64_t)(kb + c) * ld + i] = x[c];
                if (in_lds) {
#pragma unroll
                    for (int c = 0; c < NB; ++c) panel[c * PANEL_LDS_ROWS + rr] = x[c];
                }
            }
            __syncthreads();
            // (iii) trailing update W[i][j] -= sum_c X[i][c] X[j][c] for j in [r0, Kp), i in [j, ld):
            //       4x4 register tiles, row-block fastest across threads (a wave touches 2 KB of a
            //       column at a time); X from the transposed LDS panel (4 rows of a lane = one
            //       32-byte read, the j values broadcast) or from global memory
            const int nj = Kp - (int)r0;
            if (nj > 0) {
                const int tj = (nj + 3) / 4, ti = (R + 3) / 4;
                for (int t = tid; t < tj * ti; t += CT) {
                    const int bi = t % ti, bj = t / ti;
                    const int jl = 4 * bj, il = 4 * bi;       // local (panel) row indices
                    if (il + 3 < jl) continue;                // tile entirely above the diagonal
                    double acc[4][4];
#pragma unroll
                    for (int u = 0; u < 4; ++u)
#pragma unroll
                        for (int v = 0; v < 4; ++v) acc[u][v] = 0.0;
#pragma unroll 2
                    for (int c = 0; c < NB; ++c) {
                        double xi[4], xj[4];
                        if (in_lds) {
                            const double* pc = panel + c * PANEL_LDS_ROWS;
#pragma unroll
                            for (int u = 0; u < 4; ++u) {
                                xi[u] = pc[il + u];     // rows >= R hold finite junk; never stored
                                xj[u] = pc[jl + u];
                            }
                        } else {
                            const double* colc = W + (int64_t)(kb + c) * ld + r0;
#pragma unroll
                            for (int u = 0; u < 4; ++u) {
                                xi[u] = il + u < R ? colc[il + u] : 0.0;
                                xj[u] = jl + u < nj ? colc[jl + u] : 0.0;
                            }
                        }
#pragma unroll
                        for (int u = 0; u < 4; ++u)
#pragma unroll
                            for (int v = 0; v < 4; ++v) acc[u][v] += xi[u] * xj[v];
                    }
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int j = jl + v;
                        if (j >= nj) continue;
#pragma unroll
                        for (int u = 0; u < 4; ++u) {
                            const int i = il + u;
                            if (i < j || i >= R) continue;
                            W[(r0 + j) * ld + r0 + i] -= acc[u][v];
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

    // D L = Z (Z = rows Kp .. Kp+m of W, D overwrites Z): blocks of NB columns from the right.
    // Z[:, blk] -= D[:, right] L[right, blk] accumulated over 64-row chunks of D and L staged in
    // LDS by all threads (every thread owns outputs (r, c); a wave shares c), then the small
    // triangle D[:, blk] L[blk, blk] = Z[:, blk] row by row with L[blk, blk] in LDS.
    {
        // chunk rows so that D (CH x m) and L (CH x NB) fit in the panel buffer
        const int CH = 64 * (m + NB) <= PANEL_LDS_ROWS * NB ? 64 : 32;
        double* Dc = panel;                    // CH x m   (D[r][i0 + i] at Dc[i * m + r])
        double* Lc = panel + CH * m;           // CH x NB
        const int n_out = m * NB;
        constexpr int OPT = (SMDL_MAX_M * NB + CT - 1) / CT;   // outputs per thread (max)
        for (int jb = Kp - NB; jb >= 0; jb -= NB) {
            const int je = jb + NB;
            double acc[OPT];
#pragma unroll
            for (int q = 0; q < OPT; ++q) acc[q] = 0.0;
            for (int i0 = je; i0 < Kp; i0 += CH) {
                const int nr = Kp - i0 < CH ? Kp - i0 : CH;
                for (int f = tid; f < nr * m; f += CT) {
                    const int i = f / m, r = f - i * m;
                    Dc[i * m + r] = W[(int64_t)(i0 + i) * ld + Kp + r];
                }
                for (int f = tid; f < nr * NB; f += CT) {
                    const int c = f / nr, i = f - c * nr;
                    Lc[i * NB + c] = W[(int64_t)(jb + c) * ld + i0 + i];
                }
                __syncthreads();
#pragma unroll
                for (int q = 0; q < OPT; ++q) {
                    const int o = tid + q * CT;
                    if (o < n_out) {
                        const int r = o % m, c = o / m;
                        double s0 = 0.0, s1 = 0.0;
                        int i = 0;
                        for (; i + 2 <= nr; i += 2) {
                            s0 += Dc[i * m + r] * Lc[i * NB + c];
                            s1 += Dc[(i + 1) * m + r] * Lc[(i + 1) * NB + c];
                        }
                        if (i < nr) s0 += Dc[i * m + r] * Lc[i * NB + c];
                        acc[q] += s0 + s1;
                    }
                }
                __syncthreads();
            }
#pragma unroll
            for (int q = 0; q < OPT; ++q) {
                const int o = tid + q * CT;
                if (o < n_out) {
                    const int r = o % m, c = o / m;
                    W[(int64_t)(jb + c) * ld + Kp + r] -= acc[q];
                }
            }
            for (int f = tid; f < NB * NB; f += CT) {
                const int i = f / NB, j = f % NB;
                Ld[i][j] = i >= j ? W[(int64_t)(jb + j) * ld + jb + i] : 0.0;
            }
            __syncthreads();
            for (int r = tid; r < m; r += CT) {
                const int64_t zr = Kp + r;
                double x[NB];
#pragma unroll
                for (int c = 0; c < NB; ++c) x[c] = W[(int64_t)(jb + c) * ld + zr];
#pragma unroll
                for (int c = NB - 1; c >= 0; --c) {
                    double sacc = x[c];
#pragma unroll
                    for (int i = c + 1; i < NB; ++i) sacc -= x[i] * Ld[i][c];
                    x[c] = sacc / Ld[c][c];
                    __asm__ volatile("" ::: "memory");
                }
#pragma unroll
                for (int c = 0; c < NB; ++c) W[(int64_t)(jb + c) * ld + zr] = x[c];
            }
            __syncthreads();
        }
    }
    // normalise and store the active atoms (one wave per atom)
    const int lane = tid & 63, wv = tid >> 6;
    for (int j = wv; j < d.K; j += CT / 64) {
        if (!active[j]) continue;
        double ss = 0.0;
        for (int r = lane; r < m; r += 64) {
            const double v = W[(int64_t)j * ld + Kp + r];
            ss += v * v;
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) ss += __shfl_xor(ss, off, 64);
        const double inv = ss > 0.0 ? 1.0 / sqrt(ss) : 1.0;
        for (int r = lane; r < m; r += 64) d.D[(int64_t)j * m + r] = (float)(W[(int64_t)j * ld + Kp + r] * inv);
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
    hipLaunchKernelGGL(chol_solve_kernel, dim3(n_desc), dim3(CT), 0, st, dev_desc, m, status);
    return hipGetLastError();
}

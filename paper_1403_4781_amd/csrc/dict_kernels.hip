// Dictionary-side kernels: fragment packing, Gram matrix on the matrix cores, the
// first-columns initialisation, column gathers and the pooled, scaled data set of
// Algorithm 1, step 3.
#include "smdl_internal.h"

namespace {

// Pack D (m x K col-major) into the MFMA fragment layout (mpad x Kpad, zero padded).
// One thread per float4 of the packed layout; grid.y = dictionary.
__global__ void pack_dict_kernel(const PackDesc* __restrict__ pd, int m, int mchunks) {
    const PackDesc p = pd[blockIdx.y];
    const int NRB = p.Kpad >> 4;
    const int64_t total = (int64_t)mchunks * NRB * 4 * 64;
    for (int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; f < total;
         f += (int64_t)gridDim.x * blockDim.x) {
        const int l = (int)(f & 63);
        const int64_t r = f >> 6;
        const int q = (int)(r & 3);
        const int64_t cb = r >> 2;
        const int b = (int)(cb % NRB);
        const int c = (int)(cb / NRB);
        const int atom = 16 * b + (l & 15);
        const int row = 64 * c + 16 * (l >> 4) + 4 * q;
        float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
        if (atom < p.K) {
            const float* col = p.D + (int64_t)atom * m;
            v.x = row + 0 < m ? col[row + 0] : 0.f;
            v.y = row + 1 < m ? col[row + 1] : 0.f;
            v.z = row + 2 < m ? col[row + 2] : 0.f;
            v.w = row + 3 < m ? col[row + 3] : 0.f;
        }
        p.dfrag[f] = v;
    }
}

// Exponent of every atom for the FP16 split: max_r |D[r][k]| * 2^-aexp[k] in [0.5, 1) (0 for a
// zero atom and for the padding atoms).  One wave per atom (coalesced rows, a shuffle maximum),
// four atoms per block, grid.y = dictionary.
__global__ __launch_bounds__(256) void atom_exp_kernel(const PackDesc* __restrict__ pd, int m) {
    const PackDesc p = pd[blockIdx.y];
    const int k = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (k >= p.Kpad) return;
    float mx = 0.f;
    if (k < p.K) {
        const float* col = p.D + (int64_t)k * m;
        for (int r = lane; r < m; r += 64) mx = fmaxf(mx, fabsf(col[r]));
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) mx = fmaxf(mx, __shfl_xor(mx, off, 64));
    int e = 0;
    if (mx > 0.f) (void)frexpf(mx, &e);
    if (lane == 0) p.aexp[k] = e;
}

// The FP16 split fragments (layout at OmpDesc).  One thread per lane quadruple.
__global__ void pack_f16_kernel(const PackDesc* __restrict__ pd, int m, int kblocks) {
    const PackDesc p = pd[blockIdx.y];
    const int NRB = p.Kpad >> 4;
    const int64_t total = (int64_t)kblocks * NRB * 64;
    _Float16* hi = static_cast<_Float16*>(p.fhi);
    _Float16* lo = static_cast<_Float16*>(p.flo);
    for (int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; f < total;
         f += (int64_t)gridDim.x * blockDim.x) {
        const int l = (int)(f & 63);
        const int64_t r = f >> 6;
        const int b = (int)(r % NRB);
        const int kb = (int)(r / NRB);
        const int atom = 16 * b + (l & 15);
        const int row0 = 16 * kb + 4 * (l >> 4);
        const int e = p.aexp[atom];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const float v = (atom < p.K && row0 + j < m) ? ldexpf(p.D[(int64_t)atom * m + row0 + j], -e) : 0.f;
            const _Float16 h = (_Float16)v;
            hi[4 * f + j] = h;
            lo[4 * f + j] = (_Float16)(v - (float)h);
        }
    }
}

// G = D^T D for every dictionary.  Block = 4 waves = one 64 x 64 tile of G; wave w computes
// the 16 x 64 strip of rows 16*(4*tr + w), using the packed fragments for both operands
// (the B operand of the 16x16x4 MFMA wants D[atom j][row k] in lane j + 16*(k/4 ...) exactly
// as the A fragments store it).
__global__ __launch_bounds__(256) void gram_kernel(const GramDesc* __restrict__ gd, int mchunks) {
    const GramDesc p = gd[blockIdx.y];
    const int nt = p.Kpad >> 6;
    const int ntl = p.ld >> 6;        // 64-column tiles of a padded row
    const int tile = blockIdx.x;
    if (tile >= nt * ntl) return;
    const int tr = tile / ntl, tc = tile % ntl;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (tc >= nt) {                   // padding columns of rows 64 tr .. 64 tr + 63
        for (int i = threadIdx.x; i < 64 * 64; i += 256)
            p.G[(size_t)(64 * tr + (i >> 6)) * p.ld + 64 * tc + (i & 63)] = 0.f;
        return;
    }
    const int NRB = p.Kpad >> 4;
    const int rb = 4 * tr + wave;
    f32x4 acc[4];
#pragma unroll
    for (int cb = 0; cb < 4; ++cb) acc[cb] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int c = 0; c < mchunks; ++c) {
        const float4* fa = p.dfrag + ((size_t)(c * NRB + rb) * 4) * 64 + lane;
        float4 af[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) af[q] = fa[q * 64];
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) {
            const float4* fb = p.dfrag + ((size_t)(c * NRB + 4 * tc + cb) * 4) * 64 + lane;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const float4 bf = fb[q * 64];
                acc[cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[q].x, bf.x, acc[cb], 0, 0, 0);
                acc[cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[q].y, bf.y, acc[cb], 0, 0, 0);
                acc[cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[q].z, bf.z, acc[cb], 0, 0, 0);
                acc[cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[q].w, bf.w, acc[cb], 0, 0, 0);
            }
        }
    }
    const int i16 = lane & 15, kq = lane >> 4;
#pragma unroll
    for (int cb = 0; cb < 4; ++cb)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int row = 16 * rb + 4 * kq + q;
            const int col = 16 * (4 * tc + cb) + i16;
            p.G[(size_t)row * p.ld + col] = acc[cb][q];
        }
}

// out[:, n] = Y[:, perm[n]]  (m floats per column); an index outside [0, n_src) writes zeros
// and raises *bad.
__global__ void gather_columns_kernel(const float* __restrict__ Y, const int64_t* __restrict__ perm,
                                      int64_t N, int64_t n_src, int m, float* __restrict__ out,
                                      int32_t* __restrict__ bad) {
    const int64_t total = N * m;
    for (int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; f < total;
         f += (int64_t)gridDim.x * blockDim.x) {
        const int64_t n = f / m;
        const int r = (int)(f - n * m);
        const int64_t src = perm[n];
        if (src < 0 || src >= n_src) {
            out[f] = 0.f;
            if (r == 0) atomicOr(bad, 1);
        } else {
            out[f] = Y[src * m + r];
        }
    }
}

// D[:, k] = Y[:, k] / ||Y[:, k]|| for k < K (zero columns stay zero); one wave per atom,
// grid.y = dictionary.
__global__ void init_columns_kernel(const InitDesc* __restrict__ idesc, int m) {
    const InitDesc p = idesc[blockIdx.y];
    const int lane = threadIdx.x & 63;
    const int k = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (k >= p.K) return;
    const float* y = p.Y + (int64_t)k * m;
    float ss = 0.f;
    for (int r = lane; r < m; r += 64) ss = fmaf(y[r], y[r], ss);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) ss += __shfl_xor(ss, off, 64);
    const float inv = ss > 0.f ? 1.0f / sqrtf(ss) : 0.f;
    for (int r = lane; r < m; r += 64) p.D[(int64_t)k * m + r] = y[r] * inv;
}

// scales[t] = sqrt(sum of coef^2 over the codes of subset t) in FP64; one block per subset,
// fixed-order tree reduction.
__global__ __launch_bounds__(256) void code_scales_kernel(const float* __restrict__ coef,
                                                          const int32_t* __restrict__ nnz,
                                                          int s_stride,
                                                          const int64_t* __restrict__ offsets,
                                                          double* __restrict__ scales) {
    __shared__ double red[256];
    const int t = blockIdx.x;
    const int64_t b = offsets[t], e = offsets[t + 1];
    double acc = 0.0;
    for (int64_t n = b + threadIdx.x; n < e; n += blockDim.x) {
        const int k = nnz[n];
        for (int i = 0; i < k; ++i) {
            const double v = coef[n * s_stride + i];
            acc += v * v;
        }
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) scales[t] = sqrt(red[0]);
}

// Ytil[:, a] = scales[t(a)] * Dloc[:, a] for pooled atom a of subset t.
__global__ void pool_scale_kernel(const float* __restrict__ Dloc, const int64_t* __restrict__ atom_off,
                                  int L, int m, const double* __restrict__ scales,
                                  float* __restrict__ Ytil, int64_t total_atoms) {
    const int64_t total = total_atoms * m;
    for (int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; f < total;
         f += (int64_t)gridDim.x * blockDim.x) {
        const int64_t a = f / m;
        int lo = 0, hi = L - 1;
        while (lo < hi) {                 // subset t with atom_off[t] <= a < atom_off[t+1]
            const int mid = (lo + hi + 1) >> 1;
            if (atom_off[mid] <= a) lo = mid; else hi = mid - 1;
        }
        Ytil[f] = (float)(scales[lo] * (double)Dloc[f]);
    }
}

// Proposition 1 (Appendix A) on the codes of Algorithm 1: a signal of subset t with local code
// x1 over D^(t) gets r = sum_i (x1_i / c_t) z_{a_i}, where z_a is the merge code of pooled column
// a = aoff[t] + (local atom) of Ytilde = [c_t D^(t)] and c_t = ||X^(t)||_F.  One wave per signal
// position p (local codes are in subset order, the output row is perm[p]); lane j = i * ms + k
// takes local entry i and merge entry k.  Equal atoms are combined (FP64, in lane order); the
// distinct atoms are written in order of first occurrence, the unused slots as (-1, 0).
__global__ __launch_bounds__(256) void compose_codes_kernel(
    const int32_t* __restrict__ lidx, const float* __restrict__ lcoef, const int32_t* __restrict__ lnnz, int ls,
    const int32_t* __restrict__ midx, const float* __restrict__ mcoef, const int32_t* __restrict__ mnnz, int ms,
    const int64_t* __restrict__ offs, const int64_t* __restrict__ aoff, int L, const double* __restrict__ scales,
    const int64_t* __restrict__ perm, int64_t N, int K, int32_t* __restrict__ oidx, float* __restrict__ ocoef,
    int32_t* __restrict__ onnz, int os, int32_t* __restrict__ bad) {
    const int lane = threadIdx.x & 63;
    const int64_t p = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (p >= N) return;                              // uniform per wave
    const int64_t n = perm ? perm[p] : p;
    if (n < 0 || n >= N) {                           // not a permutation entry: flagged, nothing written
        if (lane == 0) atomicOr(bad, 1);
        return;
    }
    int lo = 0, hi = L - 1;
    while (lo < hi) {                                // subset t with offs[t] <= p < offs[t + 1]
        const int mid = (lo + hi + 1) >> 1;
        if (offs[mid] <= p) lo = mid; else hi = mid - 1;
    }
    const int t = lo;
    const int Kt = (int)(aoff[t + 1] - aoff[t]);
    const double c = scales[t];
    const int i = lane / ms, k = lane - i * ms;
    int atom = -1;
    double val = 0.0;
    const int k1 = lnnz[p];
    if (i < ls && i < k1 && c > 0.0) {
        const int la = lidx[p * ls + i];
        if (la >= 0 && la < Kt) {
            const int64_t a = aoff[t] + la;
            const int k2 = mnnz[a];
            if (k < k2) {
                const int ma = midx[a * ms + k];
                if (ma >= 0 && ma < K) {
                    atom = ma;
                    val = (double)lcoef[p * ls + i] * (double)mcoef[a * ms + k] / c;
                }
            }
        }
    }
    double sum = 0.0;
    bool first = atom >= 0;
    for (int q = 0; q < ls * ms; ++q) {
        const int oa = __shfl(atom, q, 64);
        const double ov = __shfl(val, q, 64);
        if (atom >= 0 && oa == atom) {
            sum += ov;
            if (q < lane) first = false;
        }
    }
    const uint64_t firsts = __ballot(first);
    const int cnt = __popcll(firsts);
    const int rank = __popcll(firsts & ((1ull << lane) - 1ull));
    if (first) {
        oidx[n * os + rank] = atom;
        ocoef[n * os + rank] = (float)sum;
    }
    if (lane >= cnt && lane < os) {
        oidx[n * os + lane] = -1;
        ocoef[n * os + lane] = 0.f;
    }
    if (lane == 0) onnz[n] = cnt;
}

__global__ void zero_i32_kernel(int32_t* p, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0;
}

__global__ void fill_codes_kernel(int32_t* idx, float* coef, int32_t* nnz, int64_t N, int s) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N * s;
         i += (int64_t)gridDim.x * blockDim.x) {
        idx[i] = -1;
        coef[i] = 0.f;
        if (i % s == 0) nnz[i / s] = 0;
    }
}

inline int grid_for(int64_t n, int block) {
    int64_t g = (n + block - 1) / block;
    if (g > 65535 * 4) g = 65535 * 4;
    if (g < 1) g = 1;
    return (int)g;
}

}  // namespace

hipError_t launch_pack_dict_m(const void* dev_pack_desc, int n_dict, int max_kpad, int m,
                              int mchunks, hipStream_t st) {
    const int64_t total = (int64_t)mchunks * (max_kpad / 16) * 4 * 64;
    dim3 grid(grid_for(total, 256), n_dict);
    hipLaunchKernelGGL(pack_dict_kernel, grid, dim3(256), 0, st,
                       static_cast<const PackDesc*>(dev_pack_desc), m, mchunks);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(atom_exp_kernel, dim3((max_kpad + 3) / 4, n_dict), dim3(256), 0, st,
                       static_cast<const PackDesc*>(dev_pack_desc), m);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    // the split covers every 64-row chunk (mpad rows): the 16-row blocks past m are zero
    const int kblocks = mchunks * 4;
    const int64_t t16 = (int64_t)kblocks * (max_kpad / 16) * 64;
    hipLaunchKernelGGL(pack_f16_kernel, dim3(grid_for(t16, 256), n_dict), dim3(256), 0, st,
                       static_cast<const PackDesc*>(dev_pack_desc), m, kblocks);
    return hipGetLastError();
}

hipError_t launch_gram_batched(const void* dev_gram_desc, int n_dict, int max_kpad, int mchunks,
                               hipStream_t st) {
    const int nt = max_kpad / 64;
    dim3 grid(nt * (gram_ld(max_kpad) / 64), n_dict);
    hipLaunchKernelGGL(gram_kernel, grid, dim3(256), 0, st,
                       static_cast<const GramDesc*>(dev_gram_desc), mchunks);
    return hipGetLastError();
}

// *bad = 1 when any of the n values is not finite (NaN or infinite).
__global__ void check_finite_kernel(const float* __restrict__ x, int64_t n, int32_t* __restrict__ bad) {
    bool ok = true;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        ok &= isfinite(x[i]);
    if (__any(!ok) && (threadIdx.x & 63) == 0) atomicOr(bad, 1);
}

hipError_t launch_check_finite(const float* x, int64_t n, int32_t* bad, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(check_finite_kernel, dim3(grid_for(n, 256)), dim3(256), 0, st, x, n, bad);
    return hipGetLastError();
}

hipError_t launch_gather_columns(const float* Y, const int64_t* perm, int64_t N, int64_t n_src, int m,
                                 float* out, int32_t* bad, hipStream_t st) {
    hipLaunchKernelGGL(gather_columns_kernel, dim3(grid_for(N * m, 256)), dim3(256), 0, st, Y, perm,
                       N, n_src, m, out, bad);
    return hipGetLastError();
}

hipError_t launch_init_from_columns_batched(const void* dev_init_desc, int n_dict, int max_k,
                                            int m, hipStream_t st) {
    dim3 grid((max_k + 3) / 4, n_dict);
    hipLaunchKernelGGL(init_columns_kernel, grid, dim3(256), 0, st,
                       static_cast<const InitDesc*>(dev_init_desc), m);
    return hipGetLastError();
}

hipError_t launch_code_scales(const float* coef, const int32_t* nnz, int s_stride,
                              const int64_t* offsets_dev, int L, double* scales, hipStream_t st) {
    hipLaunchKernelGGL(code_scales_kernel, dim3(L), dim3(256), 0, st, coef, nnz, s_stride,
                       offsets_dev, scales);
    return hipGetLastError();
}

hipError_t launch_compose_codes(const int32_t* lidx, const float* lcoef, const int32_t* lnnz, int ls,
                                const int32_t* midx, const float* mcoef, const int32_t* mnnz, int ms,
                                const int64_t* offs_dev, const int64_t* aoff_dev, int L, const double* scales,
                                const int64_t* perm, int64_t N, int K, int32_t* oidx, float* ocoef, int32_t* onnz,
                                int os, int32_t* bad, hipStream_t st) {
    if (N <= 0) return hipSuccess;
    if (ls < 1 || ms < 1 || ls * ms > 64 || os < ls * ms || os > 64) return hipErrorInvalidValue;
    hipLaunchKernelGGL(compose_codes_kernel, dim3((unsigned)((N + 3) / 4)), dim3(256), 0, st, lidx, lcoef, lnnz, ls,
                       midx, mcoef, mnnz, ms, offs_dev, aoff_dev, L, scales, perm, N, K, oidx, ocoef, onnz, os, bad);
    return hipGetLastError();
}

hipError_t launch_pool_scale(const float* Dloc, const int64_t* atom_off_dev, int L, int m,
                             const double* scales, float* Ytil, int64_t total_atoms,
                             hipStream_t st) {
    hipLaunchKernelGGL(pool_scale_kernel, dim3(grid_for(total_atoms * m, 256)), dim3(256), 0, st,
                       Dloc, atom_off_dev, L, m, scales, Ytil, total_atoms);
    return hipGetLastError();
}

hipError_t launch_zero_i32(int32_t* p, int64_t n, hipStream_t st) {
    hipLaunchKernelGGL(zero_i32_kernel, dim3(grid_for(n, 256)), dim3(256), 0, st, p, n);
    return hipGetLastError();
}

hipError_t launch_fill_codes(int32_t* idx, float* coef, int32_t* nnz, int64_t N, int s_stride,
                             hipStream_t st) {
    hipLaunchKernelGGL(fill_codes_kernel, dim3(grid_for(N * s_stride, 256)), dim3(256), 0, st, idx,
                       coef, nnz, N, s_stride);
    return hipGetLastError();
}

// Kernels of the learned support proposer (an MLP on y/||y|| -> one logit per atom).
//
// Every product of the forward and backward passes is one "NT" GEMM, C[M x N] = A[M x K] B[N x K]^T
// with both operands stored with the reduction dimension contiguous, on
// v_mfma_f32_16x16x32_bf16 with FP32 accumulation.  Fragments are loaded straight from global
// memory (16 bytes per lane); the four waves of a block split the reduction of one 32 x 32
// output tile, each issuing the loads of four k-steps at once, and sum their partials in LDS.  The layouts that make every product NT:
//   forward   h_l   [B x w_l]   = h_{l-1} [B x w_{l-1}] . W_l [w_l x w_{l-1}]^T
//   backward  d_{l-1} [B x w_{l-1}] = d_l [B x w_l] . W_l^T [w_{l-1} x w_l]^T   (ReLU mask)
//   weights   dW_l [w_l x w_{l-1}] = d_l^T [w_l x B] . h_{l-1}^T [w_{l-1} x B]^T
// so the epilogue of each product also writes the transposed BF16 copy the weight gradient
// needs (through LDS), and a per-row-block column sum of its FP32 output (bias gradients).
// The output layer's epilogue applies the BCE loss to a multi-hot label bitmask.  One grouped
// launch forms every weight gradient and applies Adam (FP32 masters and moments, BF16 W and W^T).
#include "mlp_internal.h"

namespace {

__device__ __forceinline__ uint16_t f2bf(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)(u >> 16);   // inf / nan
    u += 0x7fffu + ((u >> 16) & 1u);                                      // round to nearest even
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

constexpr int TILE = 32;       // output tile of a block (rows and columns)
constexpr int RP = TILE + 1;   // LDS row of an FP32 tile

// Partial 32 x 32 tile (m0, n0) of A B^T over the k-steps (32 wide) wave, wave + 4, ...:
// 2 x 2 blocks of 16 x 16; the loads of up to four k-steps are issued before their MFMAs.
// Rows >= M of A and columns >= N of B are read clamped (their results are discarded).
__device__ __forceinline__ void nt_partial(const uint16_t* __restrict__ A, int lda, int M,
                                           const uint16_t* __restrict__ B, int ldb, int N, int K,
                                           int m0, int n0, int wave, int lane, f32x4 (&acc)[2][2]) {
    const int r16 = lane & 15, kq = lane >> 4;
    const uint16_t* ap[2];
    const uint16_t* bp[2];
#pragma unroll
    for (int f = 0; f < 2; ++f) {
        const int r = min(m0 + 16 * f + r16, M - 1);
        const int c = min(n0 + 16 * f + r16, N - 1);
        ap[f] = A + (int64_t)r * lda + 8 * kq;
        bp[f] = B + (int64_t)c * ldb + 8 * kq;
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    const int nsteps = K / 32;
    for (int s0 = wave; s0 < nsteps; s0 += 16) {
        bf16x8 a[4][2], b[4][2];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const int st = min(s0 + 4 * c, nsteps - 1);
#pragma unroll
            for (int f = 0; f < 2; ++f) {
                a[c][f] = *reinterpret_cast<const bf16x8*>(ap[f] + 32 * st);
                b[c][f] = *reinterpret_cast<const bf16x8*>(bp[f] + 32 * st);
            }
        }
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            if (s0 + 4 * c >= nsteps) break;
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[c][i], b[c][j], acc[i][j], 0, 0, 0);
        }
    }
}

// The full 32 x 32 tile: the four waves' partials summed through LDS into tile[r][c].
__device__ __forceinline__ void nt_tile(const uint16_t* __restrict__ A, int lda, int M,
                                        const uint16_t* __restrict__ B, int ldb, int N, int K,
                                        int m0, int n0, float (*part)[TILE][RP], float (*tile)[RP]) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    f32x4 acc[2][2];
    nt_partial(A, lda, M, B, ldb, N, K, m0, n0, wave, lane, acc);
    // D[i][j] of a 16 x 16 block sits in lane j + 16 (i / 4), register i % 4
    const int r16 = lane & 15, kq = lane >> 4;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int q = 0; q < 4; ++q) part[wave][16 * i + 4 * kq + q][16 * j + r16] = acc[i][j][q];
    __syncthreads();
    const int r = tid >> 3, c0 = (tid & 7) * 4;
#pragma unroll
    for (int e = 0; e < 4; ++e)
        tile[r][c0 + e] = (part[0][r][c0 + e] + part[1][r][c0 + e]) + (part[2][r][c0 + e] + part[3][r][c0 + e]);
    __syncthreads();
}

// C = A B^T with the fused epilogue (see NtArgs).  Grid: (ceil(N / 32), M / 32); M % 32 == 0.
// Thread t finishes row t / 8, columns 4 (t % 8) .. + 3 of the tile.
__global__ __launch_bounds__(256) void gemm_nt_kernel(NtArgs g) {
    __shared__ float part[4][TILE][RP];
    __shared__ float tile[TILE][RP];
    __shared__ uint16_t tT[TILE][TILE + 2];
    __shared__ double lred[4];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int m0 = blockIdx.y * TILE, n0 = blockIdx.x * TILE;
    // the epilogue's operands (bias, ReLU mask, label bits) are requested before the product
    const int rl = tid >> 3, cl0 = (tid & 7) * 4;
    const int row = m0 + rl;
    const bool rv = row < g.Mvalid;
    const bool full = n0 + cl0 + 3 < g.N;    // N % 4 == 0, so a group is all in or all out
    float4 bias4 = make_float4(0.f, 0.f, 0.f, 0.f);
    if (g.bias && full) bias4 = *reinterpret_cast<const float4*>(g.bias + n0 + cl0);
    uint2 mask4 = make_uint2(0x3f803f80u, 0x3f803f80u);      // bf16 ones
    if (g.mask && full) mask4 = *reinterpret_cast<const uint2*>(g.mask + (int64_t)row * g.ldmask + n0 + cl0);
    uint32_t tbits = 0;
    if (g.tmask && rv && full) {
        const int src = g.rows ? g.rows[row] : row;
        tbits = g.tmask[(int64_t)src * g.tstride + ((n0 + cl0) >> 5)] >> ((n0 + cl0) & 31);
    }
    nt_tile(g.A, g.lda, g.M, g.B, g.ldb, g.N, g.K, m0, n0, part, tile);

    double lsum = 0.0;
    float v[4];
    const float bias[4] = {bias4.x, bias4.y, bias4.z, bias4.w};
    const uint16_t mk[4] = {(uint16_t)mask4.x, (uint16_t)(mask4.x >> 16), (uint16_t)mask4.y, (uint16_t)(mask4.y >> 16)};
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const bool cv = full;
        float x = tile[rl][cl0 + e] + bias[e];
        if (g.tmask) {
            // BCE with logits: loss max(z,0) - t z + log(1 + e^-|z|), delta (sigmoid(z) - t) s
            if (rv && cv) {
                const float t = (float)((tbits >> e) & 1u);
                const float sg = 1.0f / (1.0f + expf(-x));
                lsum += (double)(fmaxf(x, 0.f) - t * x + log1pf(expf(-fabsf(x))));
                x = (sg - t) * g.scale;
            } else {
                x = 0.f;
            }
        }
        if (g.relu) x = fmaxf(x, 0.f);
        if (!(bf2f(mk[e]) > 0.f)) x = 0.f;
        if (!rv || !cv) x = 0.f;
        v[e] = x;
    }
    if (full) {
        if (g.out_f32 && rv)     // may be the caller's rows
            *reinterpret_cast<float4*>(g.out_f32 + (int64_t)row * g.ldo + n0 + cl0) = make_float4(v[0], v[1], v[2], v[3]);
        if (g.out_bf16) {
            const uint32_t lo = (uint32_t)f2bf(v[0]) | ((uint32_t)f2bf(v[1]) << 16);
            const uint32_t hi = (uint32_t)f2bf(v[2]) | ((uint32_t)f2bf(v[3]) << 16);
            *reinterpret_cast<uint2*>(g.out_bf16 + (int64_t)row * g.ldo + n0 + cl0) = make_uint2(lo, hi);
        }
    }
    if (g.outT) {
#pragma unroll
        for (int e = 0; e < 4; ++e) tT[cl0 + e][rl] = f2bf(v[e]);
    }
    if (g.colpart) {
#pragma unroll
        for (int e = 0; e < 4; ++e) tile[rl][cl0 + e] = v[e];
    }
    if (g.tmask) {
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) lsum += __shfl_xor(lsum, off, 64);
        if (lane == 0) lred[wave] = lsum;
    }
    __syncthreads();
    if (g.colpart) {
        // column c: thread (c, r) sums rows 4 r .. 4 r + 3, then thread c sums the eight
        const int c = tid & 31, rg = tid >> 5;
        part[0][rg][c] = (tile[4 * rg][c] + tile[4 * rg + 1][c]) + (tile[4 * rg + 2][c] + tile[4 * rg + 3][c]);
        __syncthreads();
        if (tid < TILE && n0 + tid < g.N) {
            float cs = 0.f;
#pragma unroll
            for (int r = 0; r < 8; ++r) cs += part[0][r][tid];
            g.colpart[(int64_t)blockIdx.y * g.N + n0 + tid] = cs;
        }
    }
    if (g.tmask && tid == 0) atomicAdd(g.loss, (lred[0] + lred[1]) + (lred[2] + lred[3]));
    if (g.outT) {
        // thread t: column t / 8 of the tile, rows 4 (t % 8) .. + 3 -> 8 bytes of a row of out^T
        const int c = tid >> 3, r0 = (tid & 7) * 4;
        if (n0 + c < g.N) {
            const uint32_t lo = (uint32_t)tT[c][r0] | ((uint32_t)tT[c][r0 + 1] << 16);
            const uint32_t hi = (uint32_t)tT[c][r0 + 2] | ((uint32_t)tT[c][r0 + 3] << 16);
            *reinterpret_cast<uint2*>(g.outT + (int64_t)(n0 + c) * g.ldt + m0 + r0) = make_uint2(lo, hi);
        }
    }
}

// Weight gradients of every layer in one launch: blocks [tile0_l, tile0_l + tiles_l) form
// 32 x 32 tiles of dW_l = d_l^T h_{l-1}; the blocks after them form the bias gradients from
// the column sums, 64 columns each.  With adam set, the gradient is applied at once (Adam on the FP32 master,
// BF16 copies W and W^T written); otherwise dW and db are stored.
__global__ __launch_bounds__(256) void wgrad_kernel(WgArgs g) {
    __shared__ float part[4][TILE][RP];
    __shared__ float tile[TILE][RP];
    __shared__ uint16_t tT[TILE][TILE + 2];
    const int tid = threadIdx.x;
    const int blk = blockIdx.x;
    float c1 = 1.f, c2 = 1.f;                // Adam bias corrections 1 - beta^t
    if (g.adam) {
        const float t = (float)(*g.t_dev + g.t_off);
        c1 = 1.f - powf(g.b1, t);
        c2 = 1.f - powf(g.b2, t);
    }
    if (blk >= g.bias_block0) {
        // bias gradients, 64 columns per block: thread (c, p) sums the parts p, p + 4, ...
        int l = 0, bb = blk - g.bias_block0;
        while (bb >= (g.L[l].wo + 63) / 64) bb -= (g.L[l++].wo + 63) / 64;
        const WgLayer& L = g.L[l];
        const int c = tid & 63, p0 = tid >> 6;
        const int o = 64 * bb + c;
        float s = 0.f;
        if (o < L.wo) {
#pragma unroll 8
            for (int r = p0; r < L.nparts; r += 4) s += L.colpart[(int64_t)r * L.wo + o];
        }
        float* red = &part[0][0][0];             // 4 x 64 floats
        red[p0 * 64 + c] = s;
        __syncthreads();
        if (tid < 64 && o < L.wo) {
            s = (red[c] + red[64 + c]) + (red[128 + c] + red[192 + c]);
            if (g.adam) {
                const float a = g.b1 * L.mb[o] + (1.f - g.b1) * s;
                const float b = g.b2 * L.vb[o] + (1.f - g.b2) * s * s;
                L.mb[o] = a;
                L.vb[o] = b;
                L.b[o] = L.b[o] - g.lr * (a / c1) / (sqrtf(b / c2) + g.eps);
            } else {
                L.db_out[o] = s;
            }
        }
        return;
    }
    int l = 0;
    while (l + 1 < g.n_layers && blk >= g.L[l + 1].tile0) ++l;
    const WgLayer& L = g.L[l];
    const int t = blk - L.tile0;
    const int m0 = (t / L.ntn) * TILE, n0 = (t % L.ntn) * TILE;    // rows o, columns i
    nt_tile(L.dT, g.Bpad, L.wo, L.hT, g.Bpad, L.wi, g.Bpad, m0, n0, part, tile);
    const int ol = tid >> 3, il0 = (tid & 7) * 4;
    const int o = m0 + ol, i0 = n0 + il0;
    const bool ok = o < L.wo && i0 < L.wi;       // wi % 4 == 0
    const int64_t idx = (int64_t)o * L.wi + i0;
    if (!g.adam) {
        if (ok)
            *reinterpret_cast<float4*>(L.dW_out + idx) =
                make_float4(tile[ol][il0], tile[ol][il0 + 1], tile[ol][il0 + 2], tile[ol][il0 + 3]);
        return;
    }
    if (ok) {
        const float4 m4 = *reinterpret_cast<const float4*>(L.mW + idx);
        const float4 v4 = *reinterpret_cast<const float4*>(L.vW + idx);
        const float4 w4 = *reinterpret_cast<const float4*>(L.W + idx);
        float mm[4] = {m4.x, m4.y, m4.z, m4.w}, vv[4] = {v4.x, v4.y, v4.z, v4.w}, ww[4] = {w4.x, w4.y, w4.z, w4.w};
        uint16_t hb[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const float gr = tile[ol][il0 + e];
            mm[e] = g.b1 * mm[e] + (1.f - g.b1) * gr;
            vv[e] = g.b2 * vv[e] + (1.f - g.b2) * gr * gr;
            ww[e] = ww[e] - g.lr * (mm[e] / c1) / (sqrtf(vv[e] / c2) + g.eps);
            hb[e] = f2bf(ww[e]);
            tT[il0 + e][ol] = hb[e];
        }
        *reinterpret_cast<float4*>(L.mW + idx) = make_float4(mm[0], mm[1], mm[2], mm[3]);
        *reinterpret_cast<float4*>(L.vW + idx) = make_float4(vv[0], vv[1], vv[2], vv[3]);
        *reinterpret_cast<float4*>(L.W + idx) = make_float4(ww[0], ww[1], ww[2], ww[3]);
        *reinterpret_cast<uint2*>(L.Wbf + idx) =
            make_uint2((uint32_t)hb[0] | ((uint32_t)hb[1] << 16), (uint32_t)hb[2] | ((uint32_t)hb[3] << 16));
    }
    __syncthreads();
    // W^T: thread t writes column i = t / 8, rows o = 4 (t % 8) .. + 3 (wo % 4 == 0)
    const int ic = tid >> 3, o0 = (tid & 7) * 4;
    if (n0 + ic < L.wi && m0 + o0 < L.wo) {
        const uint32_t lo = (uint32_t)tT[ic][o0] | ((uint32_t)tT[ic][o0 + 1] << 16);
        const uint32_t hi = (uint32_t)tT[ic][o0 + 2] | ((uint32_t)tT[ic][o0 + 3] << 16);
        *reinterpret_cast<uint2*>(L.WbfT + (int64_t)(n0 + ic) * L.wo + m0 + o0) = make_uint2(lo, hi);
    }
}

// h0 = bf16(y / ||y||) for the batch rows (gathered through `rows`), as [Bpad x m] and, when
// h0T is set, [m x Bpad]; rows >= B are zero.  Block = 64 batch rows, four lanes per row (each
// m / 4 consecutive entries), staged through LDS for the transposed copy.
constexpr int PREP_ROWS = 64;
__global__ __launch_bounds__(256) void prep_kernel(const float* __restrict__ Y, int64_t B, int m, int64_t Bpad,
                                                   const int32_t* __restrict__ rows, uint16_t* __restrict__ h0,
                                                   uint16_t* __restrict__ h0T) {
    __shared__ uint16_t t[PREP_ROWS][SMDL_MAX_M + 2];
    const int tid = threadIdx.x;
    const int rr = tid >> 2, part = tid & 3;
    const int64_t b = (int64_t)blockIdx.x * PREP_ROWS + rr;
    const int seg = m / 4;                       // m % 32 == 0
    const int i0 = part * seg;
    float y[SMDL_MAX_M / 4];
    float ss = 0.f;
    const bool valid = b < B;
    const int64_t src = valid ? (rows ? rows[b] : b) : 0;
    const bool vec = (reinterpret_cast<uintptr_t>(Y) & 15) == 0;
#pragma unroll
    for (int q = 0; q < SMDL_MAX_M / 16; ++q) {
        if (4 * q < seg) {
            float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
            const float* yp = Y + src * m + i0 + 4 * q;
            if (valid) v = vec ? *reinterpret_cast<const float4*>(yp) : make_float4(yp[0], yp[1], yp[2], yp[3]);
            y[4 * q] = v.x;
            y[4 * q + 1] = v.y;
            y[4 * q + 2] = v.z;
            y[4 * q + 3] = v.w;
            ss = fmaf(v.x, v.x, fmaf(v.y, v.y, fmaf(v.z, v.z, fmaf(v.w, v.w, ss))));
        }
    }
    ss += __shfl_xor(ss, 1, 64);
    ss += __shfl_xor(ss, 2, 64);
    const float inv = ss > 0.f ? 1.0f / sqrtf(ss) : 0.f;
#pragma unroll
    for (int q = 0; q < SMDL_MAX_M / 16; ++q) {
        if (4 * q < seg) {
            uint16_t hv[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                hv[e] = valid ? f2bf(y[4 * q + e] * inv) : (uint16_t)0;
                t[rr][i0 + 4 * q + e] = hv[e];
            }
            if (b < Bpad)
                *reinterpret_cast<uint2*>(h0 + b * m + i0 + 4 * q) =
                    make_uint2((uint32_t)hv[0] | ((uint32_t)hv[1] << 16), (uint32_t)hv[2] | ((uint32_t)hv[3] << 16));
        }
    }
    if (!h0T) return;
    __syncthreads();
    const int lane = tid & 63, wave = tid >> 6;
    for (int i = wave; i < m; i += 4)
        if ((int64_t)blockIdx.x * PREP_ROWS + lane < Bpad)
            h0T[(int64_t)i * Bpad + (int64_t)blockIdx.x * PREP_ROWS + lane] = t[lane][i];
}

// Multi-hot bitmask of the ELL labels: mask[n][w] bit k%32 of word k/32 set for every label k.
__global__ void label_mask_kernel(const int32_t* __restrict__ idx, const int32_t* __restrict__ nnz, int ls,
                                  int64_t N, int K, int words, uint32_t* __restrict__ mask) {
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    uint32_t* row = mask + n * words;
    for (int w = 0; w < words; ++w) row[w] = 0u;
    int k = nnz[n];
    k = k < 0 ? 0 : (k > ls ? ls : k);
    for (int i = 0; i < k; ++i) {
        const int a = idx[n * ls + i];
        if (a >= 0 && a < K) row[a >> 5] |= 1u << (a & 31);
    }
}

// BF16 copies W and W^T of FP32 masters.
__global__ void to_bf16_kernel(const float* __restrict__ w, int64_t n, int cols, int rows,
                               uint16_t* __restrict__ wbf, uint16_t* __restrict__ wbfT) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const uint16_t h = f2bf(w[i]);
        wbf[i] = h;
        const int r = (int)(i / cols), c = (int)(i % cols);
        wbfT[(int64_t)c * rows + r] = h;
    }
}

__global__ void zero_f64_kernel(double* p, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0.0;
}

__global__ void add_i32_kernel(int32_t* p, int32_t v) {
    if (threadIdx.x == 0) *p += v;
}

inline int grid_n(int64_t n) {
    int64_t g = (n + 255) / 256;
    return (int)(g > 8192 ? 8192 : (g < 1 ? 1 : g));
}

}  // namespace

hipError_t launch_gemm_nt(const NtArgs& g, hipStream_t st) {
    if (g.M % TILE || g.K % 32 || g.N < 4 || g.N % 4 || g.M < TILE || g.lda % 8 || g.ldb % 8) return hipErrorInvalidValue;
    hipLaunchKernelGGL(gemm_nt_kernel, dim3((g.N + TILE - 1) / TILE, g.M / TILE), dim3(256), 0, st, g);
    return hipGetLastError();
}

hipError_t launch_wgrad(WgArgs& g, hipStream_t st) {
    if (g.n_layers < 1 || g.n_layers > 4 || g.Bpad % TILE) return hipErrorInvalidValue;
    int blocks = 0;
    for (int l = 0; l < g.n_layers; ++l) {
        WgLayer& L = g.L[l];
        if (L.wo % 4 || L.wi % 4) return hipErrorInvalidValue;
        L.tile0 = blocks;
        L.ntn = (L.wi + TILE - 1) / TILE;
        blocks += ((L.wo + TILE - 1) / TILE) * L.ntn;
    }
    g.bias_block0 = blocks;
    int bias_blocks = 0;
    for (int l = 0; l < g.n_layers; ++l) bias_blocks += (g.L[l].wo + 63) / 64;
    hipLaunchKernelGGL(wgrad_kernel, dim3(blocks + bias_blocks), dim3(256), 0, st, g);
    return hipGetLastError();
}

hipError_t launch_prep(const float* Y, int64_t B, int m, int64_t Bpad, const int32_t* rows, uint16_t* h0,
                       uint16_t* h0T, hipStream_t st) {
    if (m > SMDL_MAX_M || m % 32 || Bpad % PREP_ROWS) return hipErrorInvalidValue;
    hipLaunchKernelGGL(prep_kernel, dim3((unsigned)(Bpad / PREP_ROWS)), dim3(256), 0, st, Y, B, m, Bpad, rows, h0, h0T);
    return hipGetLastError();
}

hipError_t launch_label_mask(const int32_t* idx, const int32_t* nnz, int ls, int64_t N, int K, uint32_t* mask,
                             hipStream_t st) {
    if (N <= 0) return hipSuccess;
    hipLaunchKernelGGL(label_mask_kernel, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, st, idx, nnz, ls, N, K,
                       (K + 31) / 32, mask);
    return hipGetLastError();
}

hipError_t launch_zero_f64(double* p, int64_t n, hipStream_t st) {
    hipLaunchKernelGGL(zero_f64_kernel, dim3(grid_n(n)), dim3(256), 0, st, p, n);
    return hipGetLastError();
}

hipError_t launch_add_i32(int32_t* p, int32_t v, hipStream_t st) {
    hipLaunchKernelGGL(add_i32_kernel, dim3(1), dim3(64), 0, st, p, v);
    return hipGetLastError();
}

hipError_t launch_to_bf16(const float* w, int64_t n, int cols, int rows, uint16_t* wbf, uint16_t* wbfT,
                          hipStream_t st) {
    hipLaunchKernelGGL(to_bf16_kernel, dim3(grid_n(n)), dim3(256), 0, st, w, n, cols, rows, wbf, wbfT);
    return hipGetLastError();
}

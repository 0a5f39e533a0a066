// Kernels of the learned support proposer (an MLP on y/||y|| -> one logit per atom).
//
// gemm_bf16<AT, BT>: C[M x N] = A[M x K] * B[N x K]^T on v_mfma_f32_16x16x32_bf16, FP32
//   accumulation.  A "N" operand is row-major with the reduction dimension contiguous; a "T"
//   operand is stored transposed (reduction dimension = rows of memory) and is transposed while
//   staging through LDS.  Forward = (N, N), weight gradient = (T, T), input gradient = (N, T).
//   Epilogues: +bias, ReLU, FP32 and/or BF16 stores, ReLU-mask of the backward pass.
// prep_input: h0 = bf16(y / ||y||).   bce: loss and delta = (sigmoid(z) - t) / (B K).
// colsum: bias gradients.   adam: FP32 masters, moments and the BF16 copies W, W^T.
#include "mlp_internal.h"

namespace {

__device__ __forceinline__ uint16_t f2bf(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)(u >> 16);   // inf / nan
    u += 0x7fffu + ((u >> 16) & 1u);                                      // round to nearest even
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

constexpr int BK = 32;         // reduction chunk = one MFMA k-step
constexpr int LDSK = BK + 8;   // padded LDS row (bf16 elements)

template <int BM, int BN, bool AT, bool BT>
__global__ __launch_bounds__(256) void gemm_bf16(GemmArgs g) {
    __shared__ __attribute__((aligned(16))) uint16_t As[BM * LDSK];
    __shared__ __attribute__((aligned(16))) uint16_t Bs[BN * LDSK];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
    const int kspan = g.ksplit > 1 ? g.K / g.ksplit : g.K;
    const int kbeg = g.ksplit > 1 ? (int)blockIdx.z * kspan : 0;
    constexpr int WM = BM / 2, WN = BN / 2;      // per-wave tile (2 x 2 waves)
    constexpr int FM = WM / 16, FN = WN / 16;
    const int wm = (wave >> 1) * WM, wn = (wave & 1) * WN;
    f32x4 acc[FM][FN];
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};

    for (int k0 = kbeg; k0 < kbeg + kspan; k0 += BK) {
        // ---- stage A (BM x BK) and B (BN x BK) into LDS as [row][k]
        auto stage = [&](const uint16_t* __restrict__ src, int ld, int rows, int r0, bool trans,
                         uint16_t* dst, int R) {
            if (!trans) {
                // R rows x 4 chunks of 8 bf16
                for (int c = tid; c < R * 4; c += 256) {
                    const int r = c >> 2, kc = (c & 3) * 8;
                    uint4 v = make_uint4(0, 0, 0, 0);
                    if (r0 + r < rows) v = *reinterpret_cast<const uint4*>(src + (int64_t)(r0 + r) * ld + k0 + kc);
                    *reinterpret_cast<uint4*>(dst + r * LDSK + kc) = v;
                }
            } else {
                // memory is [K][rows]: chunks of 8 consecutive rows at one k
                for (int c = tid; c < BK * (R / 8); c += 256) {
                    const int kk = c / (R / 8), rc = (c % (R / 8)) * 8;
                    uint4 v = make_uint4(0, 0, 0, 0);
                    if (r0 + rc < rows) v = *reinterpret_cast<const uint4*>(src + (int64_t)(k0 + kk) * ld + r0 + rc);
                    const uint16_t* e = reinterpret_cast<const uint16_t*>(&v);
#pragma unroll
                    for (int q = 0; q < 8; ++q) dst[(rc + q) * LDSK + kk] = e[q];
                }
            }
        };
        stage(g.A, g.lda, g.M, m0, AT, As, BM);
        stage(g.B, g.ldb, g.N, n0, BT, Bs, BN);
        __syncthreads();
        bf16x8 af[FM], bfr[FN];
#pragma unroll
        for (int i = 0; i < FM; ++i)
            af[i] = *reinterpret_cast<const bf16x8*>(As + (wm + 16 * i + (lane & 15)) * LDSK + 8 * (lane >> 4));
#pragma unroll
        for (int j = 0; j < FN; ++j)
            bfr[j] = *reinterpret_cast<const bf16x8*>(Bs + (wn + 16 * j + (lane & 15)) * LDSK + 8 * (lane >> 4));
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
            for (int j = 0; j < FN; ++j)
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[i], bfr[j], acc[i][j], 0, 0, 0);
        __syncthreads();
    }
    // ---- epilogue: D[i][j] of a 16x16 block sits in lane j + 16*(i/4), register i%4
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int row = m0 + wm + 16 * i + 4 * (lane >> 4) + q;
                const int col = n0 + wn + 16 * j + (lane & 15);
                if (row >= g.M || col >= g.N) continue;
                float v = acc[i][j][q];
                if (g.bias) v += g.bias[col];
                if (g.mask_bf16) {           // backward through ReLU: keep where the activation > 0
                    if (!(bf2f(g.mask_bf16[(int64_t)row * g.ldmask + col]) > 0.f)) v = 0.f;
                }
                if (g.relu) v = fmaxf(v, 0.f);
                if (g.ksplit > 1) {
                    atomicAdd(&g.out_f32[(int64_t)row * g.ldc + col], v);
                    continue;
                }
                if (g.out_f32) g.out_f32[(int64_t)row * g.ldc + col] = v;
                if (g.out_bf16) g.out_bf16[(int64_t)row * g.ldc + col] = f2bf(v);
            }
}

// h0[b][i] = bf16(y_b[i] / ||y_b||) for i < m, zero for m <= i < mpad; rows b >= B zero.
__global__ void prep_input_kernel(const float* __restrict__ Y, int64_t B, int m, int mpad, int64_t Bpad,
                                  const int32_t* __restrict__ rows, uint16_t* __restrict__ h0) {
    const int64_t b = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (b >= Bpad) return;
    float ss = 0.f;
    const float* y = nullptr;
    if (b < B) {
        const int64_t src = rows ? rows[b] : b;
        y = Y + src * m;
        for (int i = lane; i < m; i += 64) ss = fmaf(y[i], y[i], ss);
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) ss += __shfl_xor(ss, off, 64);
    const float inv = ss > 0.f ? 1.0f / sqrtf(ss) : 0.f;
    for (int i = lane; i < mpad; i += 64)
        h0[b * mpad + i] = (b < B && i < m) ? f2bf(y[i] * inv) : (uint16_t)0;
}

// Multi-hot targets from ELL labels -> delta = (sigmoid(z) - t) * scale (FP32 and BF16) and
// the loss partial sums (one per block).
__global__ __launch_bounds__(256) void bce_kernel(const float* __restrict__ z, int64_t B, int64_t Bpad, int K,
                                                  const int32_t* __restrict__ lidx, const int32_t* __restrict__ lnnz,
                                                  int ls, const int32_t* __restrict__ rows, float scale,
                                                  float* __restrict__ delta, uint16_t* __restrict__ delta_bf,
                                                  double* __restrict__ loss_part) {
    __shared__ double red[256];
    const int64_t b = blockIdx.x;
    double lsum = 0.0;
    if (b < Bpad) {
        const int64_t src = (b < B) ? (rows ? rows[b] : b) : -1;
        int kk = 0;
        int sup[SMDL_MAX_S];
        if (src >= 0) {
            kk = lnnz[src];
            kk = kk < 0 ? 0 : (kk > ls ? ls : kk);
            for (int i = 0; i < kk; ++i) sup[i] = lidx[src * ls + i];
        }
        for (int k = threadIdx.x; k < K; k += 256) {
            float d = 0.f;
            if (src >= 0) {
                float t = 0.f;
                for (int i = 0; i < kk; ++i) t = (sup[i] == k) ? 1.f : t;
                const float x = z[b * K + k];
                const float sg = 1.0f / (1.0f + expf(-x));
                d = (sg - t) * scale;
                lsum += (double)(fmaxf(x, 0.f) - t * x + log1pf(expf(-fabsf(x))));
            }
            delta[b * K + k] = d;
            delta_bf[b * K + k] = f2bf(d);
        }
    }
    red[threadIdx.x] = lsum;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) loss_part[b] = red[0];
}

// out[j] = sum_b x[b][j] (FP32 input, FP64 accumulation in a fixed order): block = 16 columns
// x 64 row slices; each thread sums every 64th row of its column, then the 64 partials are
// added in slice order.
__global__ __launch_bounds__(1024) void colsum_kernel(const float* __restrict__ x, int64_t B, int N,
                                                      float* __restrict__ out) {
    __shared__ double part[64][16];
    const int c = threadIdx.x & 15, sl = threadIdx.x >> 4;
    const int j = blockIdx.x * 16 + c;
    double s = 0.0;
    if (j < N)
        for (int64_t b = sl; b < B; b += 64) s += x[b * N + j];
    part[sl][c] = s;
    __syncthreads();
    if (sl == 0 && j < N) {
        double t = 0.0;
        for (int q = 0; q < 64; ++q) t += part[q][c];
        out[j] = (float)t;
    }
}

__global__ void sum_f64_kernel(const double* __restrict__ x, int64_t n, double* __restrict__ out) {
    __shared__ double red[256];
    double s = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += 256) s += x[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = red[0];
}

// Adam on FP32 masters; writes the BF16 copy W (out x in) and its transpose W^T (in x out).
__global__ void adam_kernel(float* __restrict__ w, const float* __restrict__ g, float* __restrict__ m1,
                            float* __restrict__ m2, int64_t n, int cols, float lr, float b1, float b2,
                            float eps, float c1, float c2, uint16_t* __restrict__ wbf,
                            uint16_t* __restrict__ wbfT, int rows) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const float gi = g[i];
        const float a = b1 * m1[i] + (1.f - b1) * gi;
        const float b = b2 * m2[i] + (1.f - b2) * gi * gi;
        m1[i] = a;
        m2[i] = b;
        const float wi = w[i] - lr * (a / c1) / (sqrtf(b / c2) + eps);
        w[i] = wi;
        if (wbf) {
            const uint16_t h = f2bf(wi);
            wbf[i] = h;
            const int r = (int)(i / cols), c = (int)(i % cols);
            wbfT[(int64_t)c * rows + r] = h;
        }
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

// out[c][r] = in[r][c] for a rows x cols BF16 matrix, 64 x 64 tiles through LDS.
__global__ __launch_bounds__(256) void transpose_bf16_kernel(const uint16_t* __restrict__ in, int rows, int cols,
                                                             uint16_t* __restrict__ out) {
    __shared__ uint16_t tile[64][66];
    const int r0 = blockIdx.y * 64, c0 = blockIdx.x * 64;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    for (int r = ty; r < 64; r += 4)
        tile[r][tx] = (r0 + r < rows && c0 + tx < cols) ? in[(int64_t)(r0 + r) * cols + c0 + tx] : (uint16_t)0;
    __syncthreads();
    for (int c = ty; c < 64; c += 4)
        if (c0 + c < cols && r0 + tx < rows) out[(int64_t)(c0 + c) * rows + r0 + tx] = tile[tx][c];
}

__global__ void zero_f32_kernel(float* p, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0.f;
}

inline int grid_n(int64_t n) {
    int64_t g = (n + 255) / 256;
    return (int)(g > 8192 ? 8192 : (g < 1 ? 1 : g));
}

}  // namespace

hipError_t launch_transpose_bf16(const uint16_t* in, int rows, int cols, uint16_t* out, hipStream_t st) {
    hipLaunchKernelGGL(transpose_bf16_kernel, dim3((cols + 63) / 64, (rows + 63) / 64), dim3(256), 0, st, in, rows,
                       cols, out);
    return hipGetLastError();
}

hipError_t launch_zero_f32(float* p, int64_t n, hipStream_t st) {
    hipLaunchKernelGGL(zero_f32_kernel, dim3(grid_n(n)), dim3(256), 0, st, p, n);
    return hipGetLastError();
}

hipError_t launch_gemm(const GemmArgs& g, bool AT, bool BT, bool big, hipStream_t st) {
    const int ks = g.ksplit > 1 ? g.ksplit : 1;
    if (ks > 1 && (g.K % (32 * ks) || !g.out_f32 || g.out_bf16)) return hipErrorInvalidValue;
    if (big) {
        dim3 grid((g.N + 127) / 128, (g.M + 127) / 128, ks);
        if (!AT && !BT) hipLaunchKernelGGL((gemm_bf16<128, 128, false, false>), grid, dim3(256), 0, st, g);
        else if (AT && BT) hipLaunchKernelGGL((gemm_bf16<128, 128, true, true>), grid, dim3(256), 0, st, g);
        else if (!AT && BT) hipLaunchKernelGGL((gemm_bf16<128, 128, false, true>), grid, dim3(256), 0, st, g);
        else return hipErrorInvalidValue;
    } else {
        dim3 grid((g.N + 63) / 64, (g.M + 63) / 64, ks);
        if (!AT && !BT) hipLaunchKernelGGL((gemm_bf16<64, 64, false, false>), grid, dim3(256), 0, st, g);
        else if (AT && BT) hipLaunchKernelGGL((gemm_bf16<64, 64, true, true>), grid, dim3(256), 0, st, g);
        else if (!AT && BT) hipLaunchKernelGGL((gemm_bf16<64, 64, false, true>), grid, dim3(256), 0, st, g);
        else return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_prep_input(const float* Y, int64_t B, int m, int mpad, int64_t Bpad, const int32_t* rows,
                             uint16_t* h0, hipStream_t st) {
    hipLaunchKernelGGL(prep_input_kernel, dim3((unsigned)((Bpad + 3) / 4)), dim3(256), 0, st, Y, B, m, mpad, Bpad,
                       rows, h0);
    return hipGetLastError();
}

hipError_t launch_bce(const float* z, int64_t B, int64_t Bpad, int K, const int32_t* lidx, const int32_t* lnnz,
                      int ls, const int32_t* rows, float scale, float* delta, uint16_t* delta_bf,
                      double* loss_part, double* loss, hipStream_t st) {
    hipLaunchKernelGGL(bce_kernel, dim3((unsigned)Bpad), dim3(256), 0, st, z, B, Bpad, K, lidx, lnnz, ls, rows,
                       scale, delta, delta_bf, loss_part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(sum_f64_kernel, dim3(1), dim3(256), 0, st, loss_part, Bpad, loss);
    return hipGetLastError();
}

hipError_t launch_colsum(const float* x, int64_t B, int N, float* out, hipStream_t st) {
    hipLaunchKernelGGL(colsum_kernel, dim3((N + 15) / 16), dim3(1024), 0, st, x, B, N, out);
    return hipGetLastError();
}

hipError_t launch_adam(float* w, const float* g, float* m1, float* m2, int64_t n, int cols, int rows, float lr,
                       float b1, float b2, float eps, int t, uint16_t* wbf, uint16_t* wbfT, hipStream_t st) {
    const float c1 = 1.f - powf(b1, (float)t), c2 = 1.f - powf(b2, (float)t);
    hipLaunchKernelGGL(adam_kernel, dim3(grid_n(n)), dim3(256), 0, st, w, g, m1, m2, n, cols, lr, b1, b2, eps, c1,
                       c2, wbf, wbfT, rows);
    return hipGetLastError();
}

hipError_t launch_to_bf16(const float* w, int64_t n, int cols, int rows, uint16_t* wbf, uint16_t* wbfT,
                          hipStream_t st) {
    hipLaunchKernelGGL(to_bf16_kernel, dim3(grid_n(n)), dim3(256), 0, st, w, n, cols, rows, wbf, wbfT);
    return hipGetLastError();
}

// Kernels of the learned support proposer (an MLP on y/||y|| -> one logit per atom).
//
// Every product of the forward and backward passes is one "NT" GEMM, C[M x N] = A[M x K] B[N x K]^T
// with both operands stored with the reduction dimension contiguous, on
// v_mfma_f32_16x16x32_bf16 with FP32 accumulation.  Fragments are loaded straight from global
// memory (16 bytes per lane); the waves of a block split the reduction of one 32 x 32 or
// 64 x 64 output tile and sum their partials in LDS.  Every BF16 matrix in global memory
// (weights, activations, deltas and their transposes) is stored in fragment order (see pk_off),
// so that the 64 lanes of a fragment load read one contiguous kilobyte; in row-major order the
// 16 lanes of a k-group would touch 16 different rows, and the vector L1 cache would serve the
// load one lane at a time.  The layouts that make every product NT:
//   forward   h_l   [B x w_l]   = h_{l-1} [B x w_{l-1}] . W_l [w_l x w_{l-1}]^T
//   backward  d_{l-1} [B x w_{l-1}] = d_l [B x w_l] . W_l^T [w_{l-1} x w_l]^T   (ReLU mask)
//   weights   dW_l [w_l x w_{l-1}] = d_l^T [w_l x B] . h_{l-1}^T [w_{l-1} x B]^T
// so the epilogue of each product also writes the transposed BF16 copy the weight gradient
// needs (through LDS), and a per-row-block column sum of its FP32 output (bias gradients).
// The output layer's epilogue applies the BCE loss to a multi-hot label bitmask.  One grouped
// launch forms every weight gradient and applies Adam (FP32 masters and moments, BF16 W and W^T).
#include <algorithm>

#include "mlp_internal.h"

namespace {

// FP32 -> BF16, round to nearest even (one v_cvt_pk_bf16_f32 on gfx950)
__device__ __forceinline__ uint16_t f2bf(float f) { return __builtin_bit_cast(uint16_t, (__bf16)f); }
__device__ __forceinline__ float bf2f(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

// BCE with logits for logit z and target t: returns sigmoid(z) - t and adds the loss term
// max(z, 0) - t z + log(1 + e^-|z|) to loss.  One exponential e = e^-|z| in (0, 1] serves both:
// sigmoid(z) = 1 / (1 + e) for z >= 0 and e / (1 + e) otherwise.
__device__ __forceinline__ float bce_delta(float z, float t, double& loss) {
    const float e = __expf(-fabsf(z));
    const float r = __fdividef(1.0f, 1.0f + e);
    loss += (double)(fmaxf(z, 0.f) - t * z + __logf(1.0f + e));
    return (z >= 0.f ? r : e * r) - t;
}

constexpr int TILE = 32;       // output tile of a block (rows and columns)
constexpr int RP = TILE + 1;   // LDS row of an FP32 tile

// Fragment order of an [N x K] BF16 matrix (N % 16 == 0, K % 32 == 0): one kilobyte per block
// of 16 rows and 32 columns, blocks ordered by row block then column block; inside a block, lane
// l = (n % 16) + 16 ((k % 32) / 8) of a v_mfma_f32_16x16x32_bf16 operand holds the 8 consecutive
// entries k = 8 ((k % 32) / 8) .. + 7 of row n.  The offset of entry (n, k), in elements:
__device__ __forceinline__ int64_t pk_off(int n, int k, int K) {
    return ((((int64_t)(n >> 4) * (K >> 5) + (k >> 5)) * 64 + ((n & 15) + 16 * ((k & 31) >> 3))) << 3) + (k & 7);
}
// Lane's fragment of row block nb, k-step 0, of a fragment-ordered matrix; k-step st is 512
// elements further.
__device__ __forceinline__ const uint16_t* pk_frag(const uint16_t* base, int nb, int K, int lane) {
    return base + (((int64_t)nb * (K >> 5)) * 64 + lane) * 8;
}

// Partial 32 x 32 tile (m0, n0) of A B^T over the k-steps (32 wide) wave, wave + NW, ...:
// 2 x 2 blocks of 16 x 16; the loads of up to four k-steps are issued before their MFMAs.
// A and B are in fragment order (K columns).
template <int NW>
__device__ __forceinline__ void nt_partial(const uint16_t* __restrict__ A, const uint16_t* __restrict__ B, int K,
                                           int m0, int n0, int wave, int lane, f32x4 (&acc)[2][2]) {
    const uint16_t* ap[2];
    const uint16_t* bp[2];
#pragma unroll
    for (int f = 0; f < 2; ++f) {
        ap[f] = pk_frag(A, (m0 >> 4) + f, K, lane);
        bp[f] = pk_frag(B, (n0 >> 4) + f, K, lane);
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    const int nsteps = K / 32;
    for (int s0 = wave; s0 < nsteps; s0 += 4 * NW) {
        bf16x8 a[4][2], b[4][2];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const int st = min(s0 + NW * c, nsteps - 1);
#pragma unroll
            for (int f = 0; f < 2; ++f) {
                a[c][f] = *reinterpret_cast<const bf16x8*>(ap[f] + (int64_t)512 * st);
                b[c][f] = *reinterpret_cast<const bf16x8*>(bp[f] + (int64_t)512 * st);
            }
        }
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            if (s0 + NW * c >= nsteps) break;
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[c][i], b[c][j], acc[i][j], 0, 0, 0);
        }
    }
}

// The full 32 x 32 tile: the NW waves' partials summed through LDS into tile[r][c] (the first
// 256 threads form the sums).
template <int NW>
__device__ __forceinline__ void nt_tile(const uint16_t* __restrict__ A, const uint16_t* __restrict__ B, int K,
                                        int m0, int n0, float (*part)[TILE][RP], float (*tile)[RP]) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    f32x4 acc[2][2];
    nt_partial<NW>(A, B, K, m0, n0, wave, lane, acc);
    // D[i][j] of a 16 x 16 block sits in lane j + 16 (i / 4), register i % 4
    const int r16 = lane & 15, kq = lane >> 4;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int q = 0; q < 4; ++q) part[wave][16 * i + 4 * kq + q][16 * j + r16] = acc[i][j][q];
    __syncthreads();
    if (tid < 256) {
        const int r = tid >> 3, c0 = (tid & 7) * 4;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            float v = (part[0][r][c0 + e] + part[1][r][c0 + e]) + (part[2][r][c0 + e] + part[3][r][c0 + e]);
            if (NW == 8)
                v += (part[4][r][c0 + e] + part[5][r][c0 + e]) + (part[6][r][c0 + e] + part[7][r][c0 + e]);
            tile[r][c0 + e] = v;
        }
    }
    __syncthreads();
}

// C = A B^T with the fused epilogue (see NtArgs) on 32 x 32 tiles.  Grid: (M / 32, N / 32): row
// tiles on x, which allows up to 2^31 - 1 of them.
// Thread t finishes row t / 8, columns 4 (t % 8) .. + 3 of the tile.
__global__ __launch_bounds__(256) void gemm_nt_kernel(NtArgs g) {
    __shared__ float part[4][TILE][RP];
    __shared__ float tile[TILE][RP];
    __shared__ uint16_t tT[TILE][TILE + 2];
    __shared__ double lred[4];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int m0 = blockIdx.x * TILE, n0 = blockIdx.y * TILE;
    // the epilogue's operands (bias, ReLU mask, label bits) are requested before the product
    const int rl = tid >> 3, cl0 = (tid & 7) * 4;
    const int row = m0 + rl;
    const bool rv = row < g.Mvalid;
    const bool full = n0 + cl0 + 3 < g.N;    // N % 4 == 0, so a group is all in or all out
    float4 bias4 = make_float4(0.f, 0.f, 0.f, 0.f);
    if (g.bias && full) bias4 = *reinterpret_cast<const float4*>(g.bias + n0 + cl0);
    uint2 mask4 = make_uint2(0x3f803f80u, 0x3f803f80u);      // bf16 ones
    if (g.mask && full) mask4 = *reinterpret_cast<const uint2*>(g.mask + pk_off(row, n0 + cl0, g.ldmask));
    uint32_t tbits = 0;
    if (g.tmask && rv && full) {
        const int src = g.rows ? g.rows[row] : row;
        tbits = g.tmask[(int64_t)src * g.tstride + ((n0 + cl0) >> 5)] >> ((n0 + cl0) & 31);
    }
    nt_tile<4>(g.A, g.B, g.K, m0, n0, part, tile);

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
                x = bce_delta(x, t, lsum) * g.scale;
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
            *reinterpret_cast<uint2*>(g.out_bf16 + pk_off(row, n0 + cl0, g.ldo)) = make_uint2(lo, hi);
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
            g.colpart[(int64_t)blockIdx.x * g.N + n0 + tid] = cs;
        }
    }
    if (g.tmask && tid == 0) atomicAdd(g.loss, (lred[0] + lred[1]) + (lred[2] + lred[3]));
    if (g.outT) {
        // thread t: column t / 8 of the tile, rows 4 (t % 8) .. + 3 -> 8 bytes of out^T
        // ([N x M] in fragment order)
        const int c = tid >> 3, r0 = (tid & 7) * 4;
        if (n0 + c < g.N) {
            const uint32_t lo = (uint32_t)tT[c][r0] | ((uint32_t)tT[c][r0 + 1] << 16);
            const uint32_t hi = (uint32_t)tT[c][r0 + 2] | ((uint32_t)tT[c][r0 + 3] << 16);
            *reinterpret_cast<uint2*>(g.outT + pk_off(n0 + c, m0 + r0, g.M)) = make_uint2(lo, hi);
        }
    }
}


// 64 x 64 tiles, for products with at least one tile per CU: each operand row is read once per
// 64 output columns instead of 32.  Each of the four waves forms the whole tile (4 x 4 blocks
// of 16 x 16) over a quarter of the reduction; the four partial tiles are summed through LDS.
constexpr int T64 = 64;
constexpr int P64 = T64 + 1;
constexpr int NT64_MIN_TILES = 256;   // one tile per CU
__device__ __forceinline__ void nt64_load(const uint16_t* ab, const uint16_t* bb, int64_t rstride, int s,
                                          int nsteps, bf16x8 (&a)[2][4], bf16x8 (&b)[2][4]) {
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        const int64_t off = (int64_t)512 * min(s + 4 * c, nsteps - 1);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            a[c][i] = *reinterpret_cast<const bf16x8*>(ab + i * rstride + off);
            b[c][i] = *reinterpret_cast<const bf16x8*>(bb + i * rstride + off);
        }
    }
}
__device__ __forceinline__ void nt64_mma(const bf16x8 (&a)[2][4], const bf16x8 (&b)[2][4], int s, int nsteps,
                                         f32x4 (&acc)[4][4]) {
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        if (s + 4 * c >= nsteps) break;
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j)
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[c][i], b[c][j], acc[i][j], 0, 0, 0);
    }
}

// Wave `wave`'s partial 64 x 64 tile (m0, n0) of A B^T (both in fragment order, K columns) over
// the k-steps wave, wave + 4, ..., stored in part[wave].  A set is two of the wave's k-steps; the
// loads of the next set are in flight while the current one is multiplied, and the loads inside
// the loop are unconditional, so the waits before the MFMAs cover exactly the set they multiply.
__device__ __forceinline__ void nt64_partials(const uint16_t* __restrict__ A, const uint16_t* __restrict__ B,
                                              int K, int m0, int n0, int wave, int lane,
                                              float (*part)[T64][P64]) {
    const int nsteps = K >> 5;
    const int64_t rstride = (int64_t)nsteps * 512;      // elements between 16-row blocks
    const uint16_t* ab = pk_frag(A, m0 >> 4, K, lane);
    const uint16_t* bb = pk_frag(B, n0 >> 4, K, lane);
    f32x4 acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    bf16x8 a0[2][4], b0[2][4], a1[2][4], b1[2][4];
    int s = wave;
    int sets = wave < nsteps ? ((nsteps - wave + 3) / 4 + 1) / 2 : 0;
    nt64_load(ab, bb, rstride, s, nsteps, a0, b0);
    for (; sets > 2; sets -= 2, s += 16) {
        nt64_load(ab, bb, rstride, s + 8, nsteps, a1, b1);
        __builtin_amdgcn_sched_barrier(0);   // keep each set's loads ahead of the other's MFMAs
        nt64_mma(a0, b0, s, nsteps, acc);
        __builtin_amdgcn_sched_barrier(0);
        nt64_load(ab, bb, rstride, s + 16, nsteps, a0, b0);
        __builtin_amdgcn_sched_barrier(0);
        nt64_mma(a1, b1, s + 8, nsteps, acc);
        __builtin_amdgcn_sched_barrier(0);
    }
    if (sets == 2) {
        nt64_load(ab, bb, rstride, s + 8, nsteps, a1, b1);
        nt64_mma(a0, b0, s, nsteps, acc);
        nt64_mma(a1, b1, s + 8, nsteps, acc);
    } else if (sets == 1) {
        nt64_mma(a0, b0, s, nsteps, acc);
    }
    // D[i][j] of a 16 x 16 block sits in lane j + 16 (i / 4), register i % 4
    const int r16 = lane & 15, kq = lane >> 4;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int q = 0; q < 4; ++q) part[wave][16 * i + 4 * kq + q][16 * j + r16] = acc[i][j][q];
}

// C = A B^T with the fused epilogue (see NtArgs) on 64 x 64 tiles.  Grid: (M / 64, N / 64).
// Thread t finishes row t / 4, columns 16 (t % 4) .. + 15 of the tile.
__global__ __launch_bounds__(256) void gemm_nt64_kernel(NtArgs g) {
    __shared__ float part[4][T64][P64];
    __shared__ uint16_t tT[T64][T64 + 8];
    __shared__ double lred[4];
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);   // uniform: scalar loop control
    const int m0 = blockIdx.x * T64, n0 = blockIdx.y * T64;
    // the epilogue's operands are requested before the product
    const int rl = tid >> 2, cl0 = (tid & 3) * 16;
    const int row = m0 + rl;
    const bool rv = row < g.Mvalid;
    float bias[16];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        float4 b4 = make_float4(0.f, 0.f, 0.f, 0.f);
        if (g.bias) b4 = *reinterpret_cast<const float4*>(g.bias + n0 + cl0 + 4 * q);
        bias[4 * q] = b4.x;
        bias[4 * q + 1] = b4.y;
        bias[4 * q + 2] = b4.z;
        bias[4 * q + 3] = b4.w;
    }
    uint4 mk[2] = {make_uint4(0x3f803f80u, 0x3f803f80u, 0x3f803f80u, 0x3f803f80u),
                   make_uint4(0x3f803f80u, 0x3f803f80u, 0x3f803f80u, 0x3f803f80u)};   // bf16 ones
    if (g.mask) {
        mk[0] = *reinterpret_cast<const uint4*>(g.mask + pk_off(row, n0 + cl0, g.ldmask));
        mk[1] = *reinterpret_cast<const uint4*>(g.mask + pk_off(row, n0 + cl0 + 8, g.ldmask));
    }
    uint32_t tbits = 0;
    if (g.tmask && rv) {
        const int src = g.rows ? g.rows[row] : row;
        tbits = g.tmask[(int64_t)src * g.tstride + ((n0 + cl0) >> 5)] >> ((n0 + cl0) & 31);
    }

    nt64_partials(g.A, g.B, g.K, m0, n0, wave, lane, part);
    __syncthreads();

    double lsum = 0.0;
    float v[16];
    const uint32_t mw[8] = {mk[0].x, mk[0].y, mk[0].z, mk[0].w, mk[1].x, mk[1].y, mk[1].z, mk[1].w};
#pragma unroll
    for (int e = 0; e < 16; ++e) {
        const int c = cl0 + e;
        float x = ((part[0][rl][c] + part[1][rl][c]) + (part[2][rl][c] + part[3][rl][c])) + bias[e];
        if (g.tmask) {
            // BCE with logits: loss max(z,0) - t z + log(1 + e^-|z|), delta (sigmoid(z) - t) s
            if (rv) {
                const float t = (float)((tbits >> e) & 1u);
                x = bce_delta(x, t, lsum) * g.scale;
            } else {
                x = 0.f;
            }
        }
        if (g.relu) x = fmaxf(x, 0.f);
        if (!(bf2f((uint16_t)(mw[e >> 1] >> (16 * (e & 1)))) > 0.f)) x = 0.f;
        if (!rv) x = 0.f;
        v[e] = x;
    }
    if (g.out_f32 && rv) {   // may be the caller's rows
#pragma unroll
        for (int q = 0; q < 4; ++q)
            *reinterpret_cast<float4*>(g.out_f32 + (int64_t)row * g.ldo + n0 + cl0 + 4 * q) =
                make_float4(v[4 * q], v[4 * q + 1], v[4 * q + 2], v[4 * q + 3]);
    }
    if (g.out_bf16) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            uint32_t w[4];
#pragma unroll
            for (int q = 0; q < 4; ++q)
                w[q] = (uint32_t)f2bf(v[8 * h + 2 * q]) | ((uint32_t)f2bf(v[8 * h + 2 * q + 1]) << 16);
            *reinterpret_cast<uint4*>(g.out_bf16 + pk_off(row, n0 + cl0 + 8 * h, g.ldo)) =
                make_uint4(w[0], w[1], w[2], w[3]);
        }
    }
    if (g.outT) {
#pragma unroll
        for (int e = 0; e < 16; ++e) tT[cl0 + e][rl] = f2bf(v[e]);
    }
    if (g.tmask) {
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) lsum += __shfl_xor(lsum, off, 64);
        if (lane == 0) lred[wave] = lsum;
    }
    if (g.colpart) {
        // every thread has read its own entries of the partial tiles; part[0] now takes the values
#pragma unroll
        for (int e = 0; e < 16; ++e) part[0][rl][cl0 + e] = v[e];
    }
    __syncthreads();
    if (g.colpart) {
        // column c: thread (c, q) sums rows 16 q .. 16 q + 15, then the two sums of each 32-row
        // half are added
        const int c = tid & 63, q = tid >> 6;
        float cs = 0.f;
#pragma unroll
        for (int r = 0; r < 16; r += 4)
            cs += (part[0][16 * q + r][c] + part[0][16 * q + r + 1][c]) +
                  (part[0][16 * q + r + 2][c] + part[0][16 * q + r + 3][c]);
        part[1][q][c] = cs;
        __syncthreads();
        if (tid < 2 * T64) {
            const int hh = tid >> 6;
            g.colpart[(int64_t)((m0 >> 5) + hh) * g.N + n0 + c] = part[1][2 * hh][c] + part[1][2 * hh + 1][c];
        }
    }
    if (g.tmask && tid == 0) atomicAdd(g.loss, (lred[0] + lred[1]) + (lred[2] + lred[3]));
    if (g.outT) {
        // thread t: column t / 4 of the tile, rows 16 (t % 4) .. + 15 -> 32 bytes of out^T
        // ([N x M] in fragment order)
        const int c = tid >> 2, r0 = (tid & 3) * 16;
#pragma unroll
        for (int h = 0; h < 2; ++h)
            *reinterpret_cast<uint4*>(g.outT + pk_off(n0 + c, m0 + r0 + 8 * h, g.M)) =
                *reinterpret_cast<const uint4*>(&tT[c][r0 + 8 * h]);
    }
}

// Weight gradients of every layer in one launch: blocks [tile0_l, tile0_l + tiles_l) form
// 32 x 32 tiles of dW_l = d_l^T h_{l-1}; the blocks after them form the bias gradients from
// the column sums, 64 columns each.  With adam set, the gradient is applied at once (Adam on the FP32 master,
// BF16 copies W and W^T written); otherwise dW and db are stored.
// NW waves split the reduction over the batch of a 32 x 32 tile: 8 when the tiles are few (a
// small network), 4 when they already fill the chip.
template <int NW>
__global__ __launch_bounds__(64 * NW) void wgrad_kernel(WgArgs g) {
    __shared__ float part[NW][TILE][RP];
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
        // bias gradients, 64 columns per block: thread (c, p) sums the parts p, p + 8, ...
        int l = 0, bb = blk - g.bias_block0;
        while (bb >= (g.L[l].wo + 63) / 64) bb -= (g.L[l++].wo + 63) / 64;
        const WgLayer& L = g.L[l];
        constexpr int NP = NW;
        const int c = tid & 63, p0 = tid >> 6;
        const int o = 64 * bb + c;
        float s = 0.f;
        if (o < L.wo) {
#pragma unroll 4
            for (int r = p0; r < L.nparts; r += NP) s += L.colpart[(int64_t)r * L.wo + o];
        }
        float* red = &part[0][0][0];             // NP x 64 floats
        red[p0 * 64 + c] = s;
        __syncthreads();
        if (tid < 64 && o < L.wo) {
            s = 0.f;
#pragma unroll
            for (int q = 0; q < NP; q += 2) s += red[q * 64 + c] + red[(q + 1) * 64 + c];
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
    // the Adam state of the thread's four entries is requested before the product
    const bool ep = tid < 256;
    const int ol = (tid & 255) >> 3, il0 = (tid & 7) * 4;
    const int o = m0 + ol, i0 = n0 + il0;
    const bool ok = ep && o < L.wo && i0 < L.wi;
    const int64_t idx = (int64_t)o * L.wi + i0;
    float4 m4 = make_float4(0.f, 0.f, 0.f, 0.f), v4 = m4, w4 = m4;
    if (g.adam && ok) {
        m4 = *reinterpret_cast<const float4*>(L.mW + idx);
        v4 = *reinterpret_cast<const float4*>(L.vW + idx);
        w4 = *reinterpret_cast<const float4*>(L.W + idx);
    }
    nt_tile<NW>(L.dT, L.hT, g.Bpad, m0, n0, part, tile);
    if (!g.adam) {
        if (ok)
            *reinterpret_cast<float4*>(L.dW_out + idx) =
                make_float4(tile[ol][il0], tile[ol][il0 + 1], tile[ol][il0 + 2], tile[ol][il0 + 3]);
        return;
    }
    if (ok) {
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
        *reinterpret_cast<uint2*>(L.Wpk + pk_off(o, i0, L.wi)) =
            make_uint2((uint32_t)hb[0] | ((uint32_t)hb[1] << 16), (uint32_t)hb[2] | ((uint32_t)hb[3] << 16));
    }
    __syncthreads();
    // W^T: thread t writes row i = t / 8, entries o = 4 (t % 8) .. + 3
    const int ic = (tid & 255) >> 3, o0 = (tid & 7) * 4;
    if (ep && n0 + ic < L.wi && m0 + o0 < L.wo) {
        const uint32_t lo = (uint32_t)tT[ic][o0] | ((uint32_t)tT[ic][o0 + 1] << 16);
        const uint32_t hi = (uint32_t)tT[ic][o0 + 2] | ((uint32_t)tT[ic][o0 + 3] << 16);
        *reinterpret_cast<uint2*>(L.WTpk + pk_off(n0 + ic, m0 + o0, L.wo)) = make_uint2(lo, hi);
    }
}

// h0 = bf16(y / ||y||) for the batch rows (gathered through `rows`), as [Bpad x m] and, when
// h0T is set, [m x Bpad], both in fragment order; rows >= B are zero.  Block = 16 batch rows,
// eight lanes per row (each m / 8 consecutive entries, a multiple of 4), staged through LDS for
// the transposed copy; Bpad / 16 blocks, so that a batch of a thousand rows spreads over 64 CUs.
constexpr int PREP_ROWS = 16;
constexpr int PREP_LANES = 8;
__global__ __launch_bounds__(PREP_ROWS * PREP_LANES) void prep_kernel(const float* __restrict__ Y, int64_t B, int m,
                                                                    int64_t Bpad, const int32_t* __restrict__ rows,
                                                                    uint16_t* __restrict__ h0,
                                                                    uint16_t* __restrict__ h0T) {
    __shared__ uint16_t t[PREP_ROWS][SMDL_MAX_M + 2];
    const int tid = threadIdx.x;
    const int rr = tid / PREP_LANES, part = tid % PREP_LANES;
    const int64_t b = (int64_t)blockIdx.x * PREP_ROWS + rr;
    const int seg = m / PREP_LANES;              // m % 32 == 0
    const int i0 = part * seg;
    float y[SMDL_MAX_M / PREP_LANES];
    float ss = 0.f;
    const bool valid = b < B;
    const int64_t src = valid ? (rows ? rows[b] : b) : 0;
    const bool vec = (reinterpret_cast<uintptr_t>(Y) & 15) == 0;
#pragma unroll
    for (int q = 0; q < SMDL_MAX_M / (4 * PREP_LANES); ++q) {
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
#pragma unroll
    for (int off = 1; off < PREP_LANES; off <<= 1) ss += __shfl_xor(ss, off, 64);
    const float inv = ss > 0.f ? 1.0f / sqrtf(ss) : 0.f;
#pragma unroll
    for (int q = 0; q < SMDL_MAX_M / (4 * PREP_LANES); ++q) {
        if (4 * q < seg) {
            uint16_t hv[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                hv[e] = valid ? f2bf(y[4 * q + e] * inv) : (uint16_t)0;
                t[rr][i0 + 4 * q + e] = hv[e];
            }
            *reinterpret_cast<uint2*>(h0 + pk_off((int)b, i0 + 4 * q, m)) =
                make_uint2((uint32_t)hv[0] | ((uint32_t)hv[1] << 16), (uint32_t)hv[2] | ((uint32_t)hv[3] << 16));
        }
    }
    if (!h0T) return;
    __syncthreads();
    // h0^T ([m x Bpad] in fragment order): item q writes rows 4 (q % 4) .. + 3 of column q / 4
    for (int q = tid; q < m * (PREP_ROWS / 4); q += PREP_ROWS * PREP_LANES) {
        const int i = q / (PREP_ROWS / 4), rc = (q % (PREP_ROWS / 4)) * 4;
        const uint32_t lo = (uint32_t)t[rc][i] | ((uint32_t)t[rc + 1][i] << 16);
        const uint32_t hi = (uint32_t)t[rc + 2][i] | ((uint32_t)t[rc + 3][i] << 16);
        *reinterpret_cast<uint2*>(h0T + pk_off(i, (int)((int64_t)blockIdx.x * PREP_ROWS + rc), (int)Bpad)) =
            make_uint2(lo, hi);
    }
}

// ---------------------------------------------------------------------------------------------
// The whole network on R batch rows per work group (see RowsArgs), 8 or 16 waves.  The
// output of a layer is cut into 32-column tiles that the waves take in turn; a tile is R x 32 =
// (R / 16) x 2 blocks of 16 x 16 on v_mfma_f32_16x16x32_bf16.  A fragments come from the BF16
// activations in LDS, B fragments (weight rows, L2 resident) from global memory, the loads of
// the next four k-steps issued before the current four are multiplied.  Every activation of the
// R rows stays in LDS until the backward pass has used it as a ReLU mask; each delta overwrites
// the activation that masked it.
constexpr int ACT_PAD = 8;     // BF16 padding per LDS activation row (16 bytes: rows 4 banks apart)

// Threads of the fused network kernel: 16 waves for 16 rows (a training batch spreads over few
// work groups, so each takes more independent tile chains; 108 VGPRs with one register set of
// fragments in flight per wave), 8 waves for 32 rows (two register sets in flight per wave).
template <int R>
constexpr int rows_threads() { return R == 16 ? 1024 : 512; }

// B fragments (fragment-ordered weight row blocks n0 / 16 and n0 / 16 + 1) of k-steps s .. s + 3
// (clamped; a step past the end is loaded but not used).
__device__ __forceinline__ void rows_load_b(bf16x8 (&b)[4][2], const uint16_t* bp0, const uint16_t* bp1, int s,
                                            int nsteps) {
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const int st = min(s + c, nsteps - 1);
        b[c][0] = *reinterpret_cast<const bf16x8*>(bp0 + 512 * st);
        b[c][1] = *reinterpret_cast<const bf16x8*>(bp1 + 512 * st);
    }
}

// k-steps s .. s + 3 of a tile: the A fragments of the four steps are read from LDS first.
template <int RB>
__device__ __forceinline__ void rows_mma4(f32x4 (&acc)[RB][2], const bf16x8 (&b)[4][2], const uint16_t* ap, int lda,
                                          int s, int nsteps) {
    bf16x8 a[4][RB];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const int st = min(s + c, nsteps - 1);
#pragma unroll
        for (int i = 0; i < RB; ++i) a[c][i] = *reinterpret_cast<const bf16x8*>(ap + i * 16 * lda + 32 * st);
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        if (s + c < nsteps) {
#pragma unroll
            for (int i = 0; i < RB; ++i) {
                acc[i][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[c][i], b[c][0], acc[i][0], 0, 0, 0);
                acc[i][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[c][i], b[c][1], acc[i][1], 0, 0, 0);
            }
        }
    }
}

// acc = rows 0 .. R - 1 of A (LDS, ld lda) times weight rows n0 .. n0 + 31 of Bw (fragment order)
// over K.  With DB the B fragments go through two register sets in turn: the loads of the next
// four k-steps are in flight while the current four are multiplied; every iteration then issues
// both sets' loads unconditionally (clamped to the last step), so that no set is overwritten or
// read while loads of another path may still be pending into it.  Without DB one set serves:
// four k-steps are loaded, then multiplied.
template <int RB, bool DB>
__device__ __forceinline__ void rows_tile(const uint16_t* __restrict__ A, int lda, const uint16_t* __restrict__ Bw,
                                          int K, int n0, int lane, f32x4 (&acc)[RB][2]) {
    const int r16 = lane & 15, kq = lane >> 4;
    const uint16_t* bp0 = pk_frag(Bw, n0 >> 4, K, lane);
    const uint16_t* bp1 = pk_frag(Bw, (n0 >> 4) + 1, K, lane);
    const uint16_t* ap = A + r16 * lda + 8 * kq;
#pragma unroll
    for (int i = 0; i < RB; ++i) {
        acc[i][0] = f32x4{0.f, 0.f, 0.f, 0.f};
        acc[i][1] = f32x4{0.f, 0.f, 0.f, 0.f};
    }
    const int nsteps = K >> 5;
    if (DB) {
        bf16x8 b0[4][2], b1[4][2];
        rows_load_b(b0, bp0, bp1, 0, nsteps);
        for (int s0 = 0; s0 < nsteps; s0 += 8) {
            rows_load_b(b1, bp0, bp1, s0 + 4, nsteps);
            rows_mma4<RB>(acc, b0, ap, lda, s0, nsteps);
            rows_load_b(b0, bp0, bp1, s0 + 8, nsteps);
            rows_mma4<RB>(acc, b1, ap, lda, s0 + 4, nsteps);
        }
    } else {
        bf16x8 b0[4][2];
        for (int s0 = 0; s0 < nsteps; s0 += 4) {
            rows_load_b(b0, bp0, bp1, s0, nsteps);
            rows_mma4<RB>(acc, b0, ap, lda, s0, nsteps);
        }
    }
}

// acc = rows 0 .. R - 1 of A (LDS, ld lda) times weight rows n0 .. n0 + 15 of Bw (fragment order)
// over K, eight k-steps of B fragments per round trip (the registers of four k-steps of a
// 32-column tile): for a layer with fewer 32-column tiles than waves, 16-column tiles occupy
// twice the waves and halve each wave's chain of dependent loads.
template <int RB>
__device__ __forceinline__ void rows_tile16(const uint16_t* __restrict__ A, int lda, const uint16_t* __restrict__ Bw,
                                            int K, int n0, int lane, f32x4 (&acc)[RB]) {
    const int r16 = lane & 15, kq = lane >> 4;
    const uint16_t* bp = pk_frag(Bw, n0 >> 4, K, lane);
    const uint16_t* ap = A + r16 * lda + 8 * kq;
#pragma unroll
    for (int i = 0; i < RB; ++i) acc[i] = f32x4{0.f, 0.f, 0.f, 0.f};
    const int nsteps = K >> 5;
    for (int s0 = 0; s0 < nsteps; s0 += 8) {
        bf16x8 b[8];
#pragma unroll
        for (int c = 0; c < 8; ++c) b[c] = *reinterpret_cast<const bf16x8*>(bp + 512 * min(s0 + c, nsteps - 1));
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            bf16x8 a[4][RB];
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const int st = min(s0 + 4 * h + c, nsteps - 1);
#pragma unroll
                for (int i = 0; i < RB; ++i) a[c][i] = *reinterpret_cast<const bf16x8*>(ap + i * 16 * lda + 32 * st);
            }
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                if (s0 + 4 * h + c < nsteps) {
#pragma unroll
                    for (int i = 0; i < RB; ++i)
                        acc[i] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[c][i], b[4 * h + c], acc[i], 0, 0, 0);
                }
            }
        }
    }
}

// Stores the FP32 deltas v of a tile of NB 16-column blocks (row 16 i + 4 kq + q, column
// n0 + 16 j + r16 of the lane): BF16 into LDS (when O is set), BF16 transposed into dT
// ([w x Bpad] in fragment order) and the column sums over the R rows into colpart[block][w].
template <int RB, int NB = 2>
__device__ __forceinline__ void store_deltas(const float (&v)[RB][NB][4], uint16_t* O, int ldo, uint16_t* dT,
                                             int64_t Bpad, int64_t r0, float* colpart, int w, int n0, int lane) {
    const int r16 = lane & 15, kq = lane >> 4;
#pragma unroll
    for (int j = 0; j < NB; ++j) {
        const int col = n0 + 16 * j + r16;
        float cs = 0.f;
#pragma unroll
        for (int i = 0; i < RB; ++i) {
            uint16_t hb[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                hb[q] = f2bf(v[i][j][q]);
                cs += v[i][j][q];
                if (O) O[(16 * i + 4 * kq + q) * ldo + col] = hb[q];
            }
            *reinterpret_cast<uint2*>(dT + pk_off(col, (int)(r0 + 16 * i + 4 * kq), (int)Bpad)) =
                make_uint2((uint32_t)hb[0] | ((uint32_t)hb[1] << 16), (uint32_t)hb[2] | ((uint32_t)hb[3] << 16));
        }
        cs += __shfl_xor(cs, 16, 64);
        cs += __shfl_xor(cs, 32, 64);
        if (kq == 0) colpart[(int64_t)blockIdx.x * w + col] = cs;
    }
}

template <int R>
__global__ __launch_bounds__(rows_threads<R>()) void mlp_rows_kernel(RowsArgs g) {
    constexpr int RB = R / 16;
    constexpr int FT = rows_threads<R>();
    constexpr bool DB = FT == 512;
    extern __shared__ __align__(16) uint16_t act[];
    __shared__ int32_t s_src[R];
    __shared__ double s_loss[FT / 64];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int r16 = lane & 15, kq = lane >> 4;
    const int L = g.n_layers;
    const int64_t r0 = (int64_t)blockIdx.x * R;
    const bool train = R == 16 && g.tmask != nullptr;    // only the 16-row form trains
    // LDS rows of the input of layer l (l = L: the output deltas).  Training keeps every layer's
    // activations (the backward pass reads them); inference needs only the input and the output of
    // the current layer and alternates between two buffers.
    int wmax = 0;
    for (int i = 0; i < L; ++i) wmax = max(wmax, g.w[i]);
    auto buf = [&](int l) -> uint16_t* {
        if (!train) return act + (l & 1) * (R * (wmax + ACT_PAD));
        int off = 0;
        for (int i = 0; i < l; ++i) off += R * (g.w[i] + ACT_PAD);
        return act + off;
    };
    // ---- input rows: h0 = bf16(y / ||y||), zero for rows >= B
    const int m = g.w[0];
    if (tid < R) {
        const int64_t gr = r0 + tid;
        s_src[tid] = gr < g.B ? (g.rows ? g.rows[gr] : (int32_t)gr) : -1;
    }
    __syncthreads();
    {
        constexpr int TPR = FT / R;                  // threads per row (16 or 64), lanes of one wave
        constexpr int NCH = SMDL_MAX_M / 4 / TPR;    // float4 chunks per thread at most
        const int rr = tid / TPR, pt = tid % TPR;
        const int src = s_src[rr];
        const bool vec = (reinterpret_cast<uintptr_t>(g.Y) & 15) == 0;
        float4 yv[NCH];
        float ss = 0.f;
#pragma unroll
        for (int it = 0; it < NCH; ++it) {
            const int c = pt + TPR * it;
            float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
            if (src >= 0 && 4 * c < m) {
                const float* yp = g.Y + (int64_t)src * m + 4 * c;
                v = vec ? *reinterpret_cast<const float4*>(yp) : make_float4(yp[0], yp[1], yp[2], yp[3]);
            }
            yv[it] = v;
            ss = fmaf(v.x, v.x, fmaf(v.y, v.y, fmaf(v.z, v.z, fmaf(v.w, v.w, ss))));
        }
#pragma unroll
        for (int off = 1; off < TPR; off <<= 1) ss += __shfl_xor(ss, off, 64);
        const float inv = ss > 0.f ? 1.0f / sqrtf(ss) : 0.f;
        uint16_t* h0 = act + rr * (m + ACT_PAD);
#pragma unroll
        for (int it = 0; it < NCH; ++it) {
            const int c = pt + TPR * it;
            if (4 * c < m) {
                const float4 v = yv[it];
                const uint32_t lo = (uint32_t)f2bf(v.x * inv) | ((uint32_t)f2bf(v.y * inv) << 16);
                const uint32_t hi = (uint32_t)f2bf(v.z * inv) | ((uint32_t)f2bf(v.w * inv) << 16);
                *reinterpret_cast<uint2*>(h0 + 4 * c) = make_uint2(lo, hi);
            }
        }
    }
    __syncthreads();
    if (train) {
        // h0^T: thread t writes rows 4 (t % (R / 4)) .. + 3 of column t / (R / 4)
        const int ld0 = m + ACT_PAD;
        for (int t = tid; t < m * (R / 4); t += FT) {
            const int i = t / (R / 4), rc = (t % (R / 4)) * 4;
            const uint16_t* c0 = act + rc * ld0 + i;
            const uint32_t lo = (uint32_t)c0[0] | ((uint32_t)c0[ld0] << 16);
            const uint32_t hi = (uint32_t)c0[2 * ld0] | ((uint32_t)c0[3 * ld0] << 16);
            *reinterpret_cast<uint2*>(g.hT[0] + pk_off(i, (int)(r0 + rc), (int)g.Bpad)) = make_uint2(lo, hi);
        }
    }
    // ---- forward
    double lsum = 0.0;
    for (int l = 0; l < L; ++l) {
        const int wi = g.w[l], wo = g.w[l + 1];
        const bool last = l + 1 == L;
        const uint16_t* A = buf(l);
        uint16_t* O = buf(l + 1);
        const int lda = wi + ACT_PAD, ldo = wo + ACT_PAD;
        if (train && last && 2 * (wo / 32) <= FT / 64) {
            // an output layer with at most half as many 32-column tiles as waves: 16-column tiles
            for (int ct = wave; ct < wo / 16; ct += FT / 64) {
                const int n0 = 16 * ct;
                const float bj = g.bias[l][n0 + r16];
                f32x4 acc[RB];
                rows_tile16<RB>(A, lda, g.W[l], wi, n0, lane, acc);
                float v[RB][1][4];
#pragma unroll
                for (int i = 0; i < RB; ++i)
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const int src = s_src[16 * i + 4 * kq + q];
                        const uint32_t word = src >= 0 ? g.tmask[(int64_t)src * g.tstride + (n0 >> 5)] : 0u;
                        float x = 0.f;
                        if (src >= 0) {
                            const float z = acc[i][q] + bj;
                            const float t = (float)((word >> ((n0 & 31) + r16)) & 1u);
                            x = bce_delta(z, t, lsum) * g.scale;
                        }
                        v[i][0][q] = x;
                    }
                store_deltas<RB, 1>(v, L > 1 ? O : nullptr, ldo, g.dT[l], g.Bpad, r0, g.colpart[l], wo, n0, lane);
            }
            __syncthreads();
            continue;
        }
        for (int ct = wave; ct < wo / 32; ct += FT / 64) {
            const int n0 = 32 * ct;
            const float bj[2] = {g.bias[l][n0 + r16], g.bias[l][n0 + 16 + r16]};
            f32x4 acc[RB][2];
            rows_tile<RB, DB>(A, lda, g.W[l], wi, n0, lane, acc);
            if (!last) {
                // ReLU; BF16 into LDS (next layer's input) and transposed into hT[l + 1]
#pragma unroll
                for (int j = 0; j < 2; ++j) {
                    const int col = n0 + 16 * j + r16;
#pragma unroll
                    for (int i = 0; i < RB; ++i) {
                        uint16_t hb[4];
#pragma unroll
                        for (int q = 0; q < 4; ++q) {
                            const int row = 16 * i + 4 * kq + q;
                            const float x = s_src[row] >= 0 ? fmaxf(acc[i][j][q] + bj[j], 0.f) : 0.f;
                            hb[q] = f2bf(x);
                            O[row * ldo + col] = hb[q];
                        }
                        if (train)
                            *reinterpret_cast<uint2*>(g.hT[l + 1] + pk_off(col, (int)(r0 + 16 * i + 4 * kq), (int)g.Bpad)) =
                                make_uint2((uint32_t)hb[0] | ((uint32_t)hb[1] << 16),
                                           (uint32_t)hb[2] | ((uint32_t)hb[3] << 16));
                    }
                }
            } else if (!train) {
#pragma unroll
                for (int i = 0; i < RB; ++i)
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const int row = 16 * i + 4 * kq + q;
                        if (s_src[row] < 0) continue;
#pragma unroll
                        for (int j = 0; j < 2; ++j)
                            g.logits[(r0 + row) * wo + n0 + 16 * j + r16] = acc[i][j][q] + bj[j];
                    }
            } else {
                // BCE with logits: loss max(z,0) - t z + log(1 + e^-|z|), delta (sigmoid(z) - t) s
                float v[RB][2][4];
#pragma unroll
                for (int i = 0; i < RB; ++i)
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const int src = s_src[16 * i + 4 * kq + q];
                        const uint32_t word = src >= 0 ? g.tmask[(int64_t)src * g.tstride + ct] : 0u;
#pragma unroll
                        for (int j = 0; j < 2; ++j) {
                            float x = 0.f;
                            if (src >= 0) {
                                const float z = acc[i][j][q] + bj[j];
                                const float t = (float)((word >> (16 * j + r16)) & 1u);
                                x = bce_delta(z, t, lsum) * g.scale;
                            }
                            v[i][j][q] = x;
                        }
                    }
                store_deltas<RB>(v, L > 1 ? O : nullptr, ldo, g.dT[l], g.Bpad, r0, g.colpart[l], wo, n0, lane);
            }
        }
        __syncthreads();
    }
    if (!train) return;
    // ---- backward: d[l-1] = (d[l] W_l) * [h_l > 0], written over h_l
    for (int l = L - 1; l >= 1; --l) {
        const int wi = g.w[l], wo = g.w[l + 1];
        const uint16_t* A = buf(l + 1);
        uint16_t* H = buf(l);
        const int lda = wo + ACT_PAD, ldh = wi + ACT_PAD;
        for (int ct = wave; ct < wi / 32; ct += FT / 64) {
            const int n0 = 32 * ct;
            f32x4 acc[RB][2];
            rows_tile<RB, DB>(A, lda, g.WT[l], wo, n0, lane, acc);
            float v[RB][2][4];
#pragma unroll
            for (int i = 0; i < RB; ++i)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int row = 16 * i + 4 * kq + q;
#pragma unroll
                    for (int j = 0; j < 2; ++j) {
                        const float hm = bf2f(H[row * ldh + n0 + 16 * j + r16]);
                        v[i][j][q] = (hm > 0.f && s_src[row] >= 0) ? acc[i][j][q] : 0.f;
                    }
                }
            store_deltas<RB>(v, l - 1 >= 1 ? H : nullptr, ldh, g.dT[l - 1], g.Bpad, r0, g.colpart[l - 1], wi, n0, lane);
        }
        __syncthreads();
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) lsum += __shfl_xor(lsum, off, 64);
    if (lane == 0) s_loss[wave] = lsum;
    __syncthreads();
    if (tid == 0) {
        double s = 0.0;
#pragma unroll
        for (int w = 0; w < FT / 64; ++w) s += s_loss[w];
        atomicAdd(g.loss, s);
    }
}

size_t rows_lds_bytes(int n_layers, const int* w, int R, bool train) {
    size_t b = 0;
    if (!train) {
        int wmax = 0;
        for (int l = 0; l < n_layers; ++l) wmax = std::max(wmax, w[l]);
        return (size_t)2 * R * 2 * (wmax + ACT_PAD);
    }
    for (int l = 0; l <= n_layers; ++l) b += (size_t)R * 2 * (w[l] + ACT_PAD);
    return b;
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

// BF16 copies of an FP32 master W [rows x cols] in fragment order: W itself and W^T.
__global__ void to_bf16_kernel(const float* __restrict__ w, int64_t n, int cols, int rows,
                               uint16_t* __restrict__ wpk, uint16_t* __restrict__ wtpk) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const uint16_t h = f2bf(w[i]);
        const int r = (int)(i / cols), c = (int)(i % cols);
        wpk[pk_off(r, c, cols)] = h;
        wtpk[pk_off(c, r, rows)] = h;
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

// A training batch of a network with at least this many weights takes the per-layer path: the
// fused kernel streams every weight once per 16 rows, the per-layer products once per 64.
constexpr int64_t TRAIN_PER_LAYER_WEIGHTS = 3 << 18;

int mlp_rows_per_block(int n_layers, const int* widths, bool train) {
    if (n_layers < 1 || n_layers > 4) return 0;
    if (widths[0] > SMDL_MAX_M) return 0;
    for (int l = 0; l <= n_layers; ++l)
        if (widths[l] < 32 || widths[l] % 32) return 0;
    const size_t budget = SMDL_LDS_BYTES - 1024;    // the static arrays
    if (train) {
        int64_t weights = 0;
        for (int l = 0; l < n_layers; ++l) weights += (int64_t)widths[l] * widths[l + 1];
        if (weights >= TRAIN_PER_LAYER_WEIGHTS) return 0;
    }
    if (!train && rows_lds_bytes(n_layers, widths, 64, false) <= budget) return 64;
    if (!train && rows_lds_bytes(n_layers, widths, 32, false) <= budget) return 32;
    if (rows_lds_bytes(n_layers, widths, 16, train) <= budget) return 16;
    return 0;
}

hipError_t launch_mlp_rows(const RowsArgs& a, int R, hipStream_t st) {
    const bool train = a.tmask != nullptr;
    if ((R != 16 && R != 32 && R != 64) || (train && R != 16) || a.Bpad < R || a.Bpad % R || a.B > a.Bpad)
        return hipErrorInvalidValue;
    const size_t budget = SMDL_LDS_BYTES - 1024;
    if (mlp_rows_per_block(a.n_layers, a.w, false) == 0 || rows_lds_bytes(a.n_layers, a.w, R, train) > budget)
        return hipErrorInvalidValue;
    if (train ? (!a.loss || a.tstride < (a.w[a.n_layers] + 31) / 32) : !a.logits) return hipErrorInvalidValue;
    const size_t lds = rows_lds_bytes(a.n_layers, a.w, R, train);
    static bool attr_set = false;   // every instantiation may use the whole LDS budget
    if (!attr_set) {
        const int full = (int)(SMDL_LDS_BYTES - 1024);
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&mlp_rows_kernel<64>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, full);
        if (e == hipSuccess)
            e = hipFuncSetAttribute(reinterpret_cast<const void*>(&mlp_rows_kernel<32>),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, full);
        if (e == hipSuccess)
            e = hipFuncSetAttribute(reinterpret_cast<const void*>(&mlp_rows_kernel<16>),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, full);
        if (e != hipSuccess) return e;
        attr_set = true;
    }
    if (R == 64)
        hipLaunchKernelGGL(mlp_rows_kernel<64>, dim3((unsigned)(a.Bpad / 64)), dim3(rows_threads<64>()), lds, st, a);
    else if (R == 32)
        hipLaunchKernelGGL(mlp_rows_kernel<32>, dim3((unsigned)(a.Bpad / 32)), dim3(rows_threads<32>()), lds, st, a);
    else
        hipLaunchKernelGGL(mlp_rows_kernel<16>, dim3((unsigned)(a.Bpad / 16)), dim3(rows_threads<16>()), lds, st, a);
    return hipGetLastError();
}

hipError_t launch_gemm_nt(const NtArgs& g, hipStream_t st) {
    if (g.M % TILE || g.K % 32 || g.N < TILE || g.N % TILE || g.M < TILE) return hipErrorInvalidValue;
    // fragment-order mask and BF16 output rows are N wide
    if ((g.mask && g.ldmask != g.N) || (g.out_bf16 && g.ldo != g.N)) return hipErrorInvalidValue;
    if (g.M % T64 == 0 && g.N % T64 == 0 && (int64_t)(g.M / T64) * (g.N / T64) >= NT64_MIN_TILES)
        hipLaunchKernelGGL(gemm_nt64_kernel, dim3(g.M / T64, g.N / T64), dim3(256), 0, st, g);
    else
        hipLaunchKernelGGL(gemm_nt_kernel, dim3(g.M / TILE, g.N / TILE), dim3(256), 0, st, g);
    return hipGetLastError();
}

hipError_t launch_wgrad(WgArgs& g, hipStream_t st) {
    if (g.n_layers < 1 || g.n_layers > 4 || g.Bpad % TILE) return hipErrorInvalidValue;
    int blocks = 0;
    for (int l = 0; l < g.n_layers; ++l) {
        WgLayer& L = g.L[l];
        if (L.wo % TILE || L.wi % TILE) return hipErrorInvalidValue;
        L.tile0 = blocks;
        L.ntn = (L.wi + TILE - 1) / TILE;
        blocks += ((L.wo + TILE - 1) / TILE) * L.ntn;
    }
    g.bias_block0 = blocks;
    int bias_blocks = 0;
    for (int l = 0; l < g.n_layers; ++l) bias_blocks += (g.L[l].wo + 63) / 64;
    if (blocks <= 1024)
        hipLaunchKernelGGL(wgrad_kernel<8>, dim3(blocks + bias_blocks), dim3(512), 0, st, g);
    else
        hipLaunchKernelGGL(wgrad_kernel<4>, dim3(blocks + bias_blocks), dim3(256), 0, st, g);
    return hipGetLastError();
}

hipError_t launch_prep(const float* Y, int64_t B, int m, int64_t Bpad, const int32_t* rows, uint16_t* h0,
                       uint16_t* h0T, hipStream_t st) {
    if (m > SMDL_MAX_M || m % 32 || Bpad % PREP_ROWS) return hipErrorInvalidValue;
    hipLaunchKernelGGL(prep_kernel, dim3((unsigned)(Bpad / PREP_ROWS)), dim3(PREP_ROWS * PREP_LANES), 0, st, Y, B, m,
                       Bpad, rows, h0, h0T);
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

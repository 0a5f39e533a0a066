// Candidate selection and proposer-restricted OMP.
//
// topk: one wave per signal; n_cand rounds of a wave argmax over the logits (larger logit
//   first, lower atom index on equal logits); the chosen atoms are written in increasing atom
//   order (ballot prefix counts).
// restricted_omp: one group of 16 lanes per signal.  OMP on the candidate columns only:
//   alpha_C = D_C^T y by gathered dot products, the same correlation-space progressive
//   inverse-Cholesky steps as the full kernel with rows of G gathered at the candidates, then
//   the explicit FP32 residual r = y - D_I x_I.  ||r|| > eps_fb marks the signal for the full
//   OMP fallback (appended to a device list, no host round trip).
#include "mlp_internal.h"

namespace {

constexpr int MAXC = 64;        // candidates per signal
constexpr int GR = 16;          // lanes per signal
constexpr int EC = MAXC / GR;   // candidate entries per lane

__global__ __launch_bounds__(256) void topk_kernel(const float* __restrict__ logits, int64_t N, int K,
                                                   int n_cand, int32_t* __restrict__ cand) {
    const int lane = threadIdx.x & 63;
    const int64_t n = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (n >= N) return;
    constexpr int EK = SMDL_MAX_K / 64;
    float v[EK];
    bool taken[EK];
    const int E = (K + 63) / 64;
#pragma unroll
    for (int t = 0; t < EK; ++t) {
        const int k = lane + 64 * t;
        v[t] = (t < E && k < K) ? logits[n * K + k] : -INFINITY;
        if (v[t] != v[t]) v[t] = -INFINITY;     // NaN logits rank last
        taken[t] = !(t < E && k < K);
    }
    for (int c = 0; c < n_cand; ++c) {
        float bv = -INFINITY;
        int bi = 0x7fffffff;
#pragma unroll
        for (int t = 0; t < EK; ++t) {
            const int k = lane + 64 * t;
            if (!taken[t] && (v[t] > bv || (v[t] == bv && k < bi))) { bv = v[t]; bi = k; }
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            const float ov = __shfl_xor(bv, off, 64);
            const int oi = __shfl_xor(bi, off, 64);
            if (ov > bv || (ov == bv && oi < bi)) { bv = ov; bi = oi; }
        }
#pragma unroll
        for (int t = 0; t < EK; ++t)
            if (lane + 64 * t == bi) taken[t] = true;
    }
    // chosen = taken minus the padding; write in increasing atom order
    int base = 0;
#pragma unroll
    for (int t = 0; t < EK; ++t) {
        const int k = lane + 64 * t;
        const bool chosen = taken[t] && t < E && k < K;
        const unsigned long long mask = __ballot(chosen);
        const int pos = base + __popcll(mask & ((1ull << lane) - 1ull));
        if (chosen && pos < n_cand) cand[n * n_cand + pos] = k;
        base += __popcll(mask);
    }
}

__global__ __launch_bounds__(256) void restricted_omp_kernel(RestrictedArgs a) {
    __shared__ float ys[16][SMDL_MAX_M];
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int g = lane & (GR - 1);
    const int slot = tid / GR;                         // 0..15
    const int64_t n = (int64_t)blockIdx.x * 16 + slot;
    const bool valid = n < a.N;
    const int m = a.m;
    const int nc = a.n_cand;
    // stage y
    for (int i = g; i < m; i += GR) ys[slot][i] = valid ? a.Y[n * m + i] : 0.f;
    __syncthreads();
    int cid[EC];
    float c[EC];
    float ysq = 0.f;
    for (int i = g; i < m; i += GR) ysq = fmaf(ys[slot][i], ys[slot][i], ysq);
#pragma unroll
    for (int off = 1; off < GR; off <<= 1) ysq += __shfl_xor(ysq, off, 64);
#pragma unroll
    for (int t = 0; t < EC; ++t) {
        const int e = g + GR * t;
        cid[t] = (valid && e < nc) ? a.cand[n * nc + e] : -1;
        if (cid[t] < 0 || cid[t] >= a.K) cid[t] = -1;
        float acc = 0.f;
        if (cid[t] >= 0) {
            const float* d = a.D + (int64_t)cid[t] * m;
            for (int i = 0; i < m; ++i) acc = fmaf(d[i], ys[slot][i], acc);
        }
        c[t] = acc;
    }
    const float ynrm = sqrtf(ysq);
    float U[SMDL_MAX_S][EC];
    float Linv[SMDL_MAX_S][SMDL_MAX_S];
    float pi[SMDL_MAX_S];
    int sel[SMDL_MAX_S];
#pragma unroll
    for (int i = 0; i < SMDL_MAX_S; ++i) {
        pi[i] = 0.f;
        sel[i] = 0;
#pragma unroll
        for (int l = 0; l <= i; ++l) Linv[i][l] = 0.f;
    }
    bool live = valid;
    int k = 0;
#pragma unroll
    for (int kk = 0; kk < SMDL_MAX_S; ++kk) {
        if (kk >= a.s) break;
        if (!__any(live)) break;
        // argmax over candidates: position order = atom order, so lower position wins ties
        float bv = 0.f;
        int bp = 0x7fffffff;
#pragma unroll
        for (int t = 0; t < EC; ++t) {
            const int e = g + GR * t;
            if (cid[t] >= 0 && (fabsf(c[t]) > fabsf(bv) || (fabsf(c[t]) == fabsf(bv) && e < bp))) {
                bv = c[t];
                bp = e;
            }
        }
#pragma unroll
        for (int off = 1; off < GR; off <<= 1) {
            const float ov = __shfl_xor(bv, off, 64);
            const int op = __shfl_xor(bp, off, 64);
            if (fabsf(ov) > fabsf(bv) || (fabsf(ov) == fabsf(bv) && op < bp)) { bv = ov; bp = op; }
        }
        if (!(fabsf(bv) > a.tau * ynrm) || bp >= nc) live = false;
        if (live) {
            const int j = a.cand[n * nc + bp];
            const float* grow = a.gram + (int64_t)j * a.Kpad;
            float gs[SMDL_MAX_S];
#pragma unroll
            for (int i = 0; i < kk; ++i) gs[i] = grow[sel[i]];
            const float gjj = grow[j];
            float w[SMDL_MAX_S];
            float l2 = gjj;
#pragma unroll
            for (int i = 0; i < kk; ++i) {
                float acc = 0.f;
#pragma unroll
                for (int l = 0; l <= i; ++l) acc = fmaf(Linv[i][l], gs[l], acc);
                w[i] = acc;
                l2 = fmaf(-acc, acc, l2);
            }
            if (!(l2 > a.dep_tol * gjj)) {
                live = false;
            } else {
                const float rl = 1.0f / sqrtf(l2);
#pragma unroll
                for (int l = 0; l < kk; ++l) {
                    float acc = 0.f;
#pragma unroll
                    for (int i = l; i < kk; ++i) acc = fmaf(w[i], Linv[i][l], acc);
                    Linv[kk][l] = -acc * rl;
                }
                Linv[kk][kk] = rl;
                const float pk = bv * rl;
#pragma unroll
                for (int t = 0; t < EC; ++t) {
                    float u = cid[t] >= 0 ? grow[cid[t]] : 0.f;
#pragma unroll
                    for (int i = 0; i < kk; ++i) u = fmaf(-U[i][t], w[i], u);
                    u *= rl;
                    U[kk][t] = u;
                    c[t] = fmaf(-pk, u, c[t]);
                }
                pi[kk] = pk;
                sel[kk] = j;
                k = kk + 1;
            }
        }
    }
    // coefficients and the explicit residual
    float gam[SMDL_MAX_S];
#pragma unroll
    for (int l = 0; l < SMDL_MAX_S; ++l) {
        float acc = 0.f;
#pragma unroll
        for (int i = l; i < SMDL_MAX_S; ++i) acc = fmaf(Linv[i][l], (i < k) ? pi[i] : 0.f, acc);
        gam[l] = acc;
    }
    float rr = 0.f;
    for (int i = g; i < m; i += GR) {
        float r = ys[slot][i];
#pragma unroll
        for (int l = 0; l < SMDL_MAX_S; ++l)
            if (l < k) r = fmaf(-gam[l], a.D[(int64_t)sel[l] * m + i], r);
        rr = fmaf(r, r, rr);
    }
#pragma unroll
    for (int off = 1; off < GR; off <<= 1) rr += __shfl_xor(rr, off, 64);
    if (!valid) return;
    const bool miss = sqrtf(rr) > a.eps_fb;
    if (g == 0) {
        if (a.fell_back) a.fell_back[n] = miss ? 1 : 0;
        if (miss) {
            const int pos = atomicAdd(a.fb_count, 1);
            a.fb_list[pos] = (int32_t)n;
        }
    }
    if (miss) return;    // the full OMP writes this signal's code
    if (g < a.s_out) {
        int oi = -1;
        float oc = 0.f;
#pragma unroll
        for (int i = 0; i < SMDL_MAX_S; ++i)
            if (i == g && i < k) { oi = sel[i]; oc = gam[i]; }
        a.idx[n * a.s_out + g] = oi;
        a.coef[n * a.s_out + g] = oc;
    }
    if (g == 0) a.nnz[n] = k;
}

}  // namespace

hipError_t launch_topk(const float* logits, int64_t N, int K, int n_cand, int32_t* cand, hipStream_t st) {
    hipLaunchKernelGGL(topk_kernel, dim3((unsigned)((N + 3) / 4)), dim3(256), 0, st, logits, N, K, n_cand, cand);
    return hipGetLastError();
}

hipError_t launch_restricted_omp(const RestrictedArgs& a, hipStream_t st) {
    hipLaunchKernelGGL(restricted_omp_kernel, dim3((unsigned)((a.N + 15) / 16)), dim3(256), 0, st, a);
    return hipGetLastError();
}

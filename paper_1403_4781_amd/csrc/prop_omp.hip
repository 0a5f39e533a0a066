// Candidate selection and proposer-restricted OMP.
//
// topk: 16 lanes per signal; the n_cand largest logits (lower atom index on equal logits) by a
//   bisection on order-preserving keys; the chosen atoms are written in increasing atom order.
// restricted_omp: one group of 16 lanes per signal.  OMP on the candidate columns only:
//   alpha_C = D_C^T y by gathered dot products, the same correlation-space progressive
//   inverse-Cholesky steps as the full kernel with rows of G gathered at the candidates, then
//   the explicit FP32 residual r = y - D_I x_I.  ||r|| > eps_fb marks the signal for the full
//   OMP fallback (appended to a device list, no host round trip).
#include <utility>

#include "mlp_internal.h"

namespace {

constexpr int MAXC = 64;        // candidates per signal
constexpr int GR = 16;          // lanes per signal
constexpr int EC = MAXC / GR;   // candidate entries per lane

// Top-n_cand selection, 16 lanes per signal (4 signals per wave); lane g holds the logits of
// atoms g + 16 t (t < E).  Logits become order-preserving 32-bit keys (NaN ranks last); a
// bisection over the key bits finds a threshold T (at most 32 rounds of one group count); the
// keys above T are taken, and of the keys equal to T the lowest atoms.  As atom 16 t + g
// orders like (t, g), every lane writes its chosen atoms straight to their positions in
// increasing atom order (group ballots and popcounts).
// NaN ranks below every number (key 1); key 0 marks padding entries, which are never chosen
// because at least K >= n_cand keys are >= 1.
__device__ __forceinline__ uint32_t order_key(float x) {
    if (x != x) return 1u;
    const uint32_t u = __float_as_uint(x);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

__device__ __forceinline__ int group_isum(int v) {
    v += __builtin_amdgcn_update_dpp(0, v, 0xB1, 0xf, 0xf, false);
    v += __builtin_amdgcn_update_dpp(0, v, 0x4E, 0xf, 0xf, false);
    v += __builtin_amdgcn_update_dpp(0, v, 0x141, 0xf, 0xf, false);
    v += __builtin_amdgcn_update_dpp(0, v, 0x140, 0xf, 0xf, false);
    return v;
}

// 16-bit mask of the lanes of this lane's group for which pred holds.
__device__ __forceinline__ uint32_t group_ballot(bool pred, int grp) {
    const uint64_t m = __ballot(pred);
    return (uint32_t)(m >> (16 * grp)) & 0xffffu;
}

template <int E>
__global__ __launch_bounds__(256) void topk_kernel(const float* __restrict__ logits, int64_t N, int K,
                                                   int n_cand, int32_t* __restrict__ cand) {
    const int lane = threadIdx.x & 63;
    const int g = lane & 15, grp = lane >> 4;
    const int64_t n = (int64_t)blockIdx.x * 16 + (threadIdx.x >> 4);
    const bool valid = n < N;
    uint32_t key[E];
#pragma unroll
    for (int t = 0; t < E; ++t) {
        const int k = g + 16 * t;
        key[t] = (valid && k < K) ? order_key(logits[n * K + k]) : 0u;   // 0: never chosen
    }
    // T = the largest threshold with at least n_cand keys >= T.  A group stops as soon as exactly
    // n_cand keys are >= T: those keys are then the selection whatever the remaining bits (T lies
    // above the next key and at most at the n_cand-th, so no key equal to the n_cand-th is left
    // out), and the steps below take all of them.  The wave stops when its four groups have.
    uint32_t T = 0u;
    bool done = false;
    for (int b = 31; b >= 0; --b) {
        const uint32_t T2 = T | (1u << b);
        int c = 0;
#pragma unroll
        for (int t = 0; t < E; ++t) c += key[t] >= T2 ? 1 : 0;
        const int cs = group_isum(c);
        if (!done && cs >= n_cand) {
            T = T2;
            done = cs == n_cand;
        }
        if (__ballot(!done) == 0) break;
    }
    int gt = 0;
#pragma unroll
    for (int t = 0; t < E; ++t) gt += key[t] > T ? 1 : 0;
    const int need = n_cand - group_isum(gt);      // keys equal to T to take, lowest atoms first
    const uint32_t below = (1u << g) - 1u;
    int eq_before = 0, sel_before = 0;
#pragma unroll
    for (int t = 0; t < E; ++t) {
        const bool eq = key[t] == T;
        const uint32_t em = group_ballot(eq, grp);
        const bool take = key[t] > T || (eq && eq_before + __popc(em & below) < need);
        const uint32_t sm = group_ballot(take, grp);
        if (valid && take) cand[n * n_cand + sel_before + __popc(sm & below)] = g + 16 * t;
        eq_before += __popc(em);
        sel_before += __popc(sm);
    }
}

// (|value| larger, then lower candidate position) combine for the restricted argmax.
template <int CTRL>
__device__ __forceinline__ void ro_dpp(float& bv, int& bp) {
    const float ov = __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(bv), CTRL, 0xf, 0xf, false));
    const int op = __builtin_amdgcn_mov_dpp(bp, CTRL, 0xf, 0xf, false);
    const float ao = fabsf(ov), ab = fabsf(bv);
    const bool take = (ao > ab) | ((ao == ab) & (op < bp));
    bv = take ? ov : bv;
    bp = take ? op : bp;
}

template <int SM>
struct RState {
    float c[EC];
    float U[SM][EC];
    float Linv[SM][SM];
    float pi[SM];
    int sel[SM];
    int k;
    bool live;
};

struct RCtx {
    const RestrictedArgs* a;
    const int* cid;
    int64_t n;
    int g;
    float ynrm;
};

// One greedy step over the candidates (KK is a compile-time constant so that every register
// array index is static).  Returns false when the whole wave is done.
template <int KK, int SM>
__device__ __forceinline__ bool r_step(RState<SM>& st, const RCtx& x) {
    const RestrictedArgs& a = *x.a;
    if (KK >= a.s) return false;
    if (!__any(st.live)) return false;
    // argmax over candidates: position order = atom order, so the lower position wins ties
    float bv = 0.f;
    int bp = 0x7fffffff;
#pragma unroll
    for (int t = 0; t < EC; ++t) {
        const int e = x.g + GR * t;
        if (x.cid[t] >= 0 && (fabsf(st.c[t]) > fabsf(bv) || (fabsf(st.c[t]) == fabsf(bv) && e < bp))) {
            bv = st.c[t];
            bp = e;
        }
    }
    ro_dpp<0xB1>(bv, bp);
    ro_dpp<0x4E>(bv, bp);
    ro_dpp<0x141>(bv, bp);
    ro_dpp<0x140>(bv, bp);
    if (!(fabsf(bv) > a.tau * x.ynrm) || bp >= a.n_cand) st.live = false;
    if (st.live) {
        const int j = a.cand[x.n * a.n_cand + bp];
        const float* grow = a.gram + (int64_t)j * a.gld;
        float gs[KK > 0 ? KK : 1];
#pragma unroll
        for (int i = 0; i < KK; ++i) gs[i] = grow[st.sel[i]];
        const float gjj = grow[j];
        float w[KK > 0 ? KK : 1];
        float l2 = gjj;
#pragma unroll
        for (int i = 0; i < KK; ++i) {
            float acc = 0.f;
#pragma unroll
            for (int l = 0; l <= i; ++l) acc = fmaf(st.Linv[i][l], gs[l], acc);
            w[i] = acc;
            l2 = fmaf(-acc, acc, l2);
        }
        if (!(l2 > a.dep_tol * gjj)) {
            st.live = false;
        } else {
            const float rl = __builtin_amdgcn_rsqf(l2);
#pragma unroll
            for (int l = 0; l < KK; ++l) {
                float acc = 0.f;
#pragma unroll
                for (int i = l; i < KK; ++i) acc = fmaf(w[i], st.Linv[i][l], acc);
                st.Linv[KK][l] = -acc * rl;
            }
            st.Linv[KK][KK] = rl;
            const float pk = bv * rl;
#pragma unroll
            for (int t = 0; t < EC; ++t) {
                float u = x.cid[t] >= 0 ? grow[x.cid[t]] : 0.f;
#pragma unroll
                for (int i = 0; i < KK; ++i) u = fmaf(-st.U[i][t], w[i], u);
                u *= rl;
                st.U[KK][t] = u;
                st.c[t] = fmaf(-pk, u, st.c[t]);
            }
            st.pi[KK] = pk;
            st.sel[KK] = j;
            st.k = KK + 1;
        }
    }
    return true;
}

template <int SM, int... KKs>
__device__ __forceinline__ void r_run(RState<SM>& st, const RCtx& x, std::integer_sequence<int, KKs...>) {
    (void)(r_step<KKs, SM>(st, x) && ...);
}

template <int SM>
__global__ __launch_bounds__(256) void restricted_omp_kernel(RestrictedArgs a) {
    __shared__ float ys[16][SMDL_MAX_M];
    __shared__ int s_fbcnt[4];
    __shared__ int s_fbbase;
    extern __shared__ float alpha[];                    // 16 x (Kpad + 4): alpha0 of the signals
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int g = lane & (GR - 1);
    const int slot = tid / GR;                         // 0..15
    const int64_t n = (int64_t)blockIdx.x * 16 + slot;
    const bool valid = n < a.N;
    const int m = a.m;
    const int nc = a.n_cand;
    const int mpad = 64 * a.mchunks;
    for (int i = g; i < mpad; i += GR) ys[slot][i] = valid && i < m ? a.Y[n * m + i] : 0.f;
    __syncthreads();
    // alpha0 = D^T y of the 16 signals on the matrix cores from the packed fragments, in the order
    // of the plain OMP kernel (so the same bits); each lane then reads its candidates' entries
    const int Kpad = a.Kpad, astride = Kpad + 4;
    {
        const int i16 = lane & 15, kq = lane >> 4, wave = tid >> 6;
        const int NRB = Kpad >> 4, rbw = NRB >> 2, rb0 = wave * rbw;
        float4 yv[SMDL_MAX_M / 64][4];
#pragma unroll
        for (int c = 0; c < SMDL_MAX_M / 64; ++c)
#pragma unroll
            for (int q = 0; q < 4; ++q)
                yv[c][q] = c < a.mchunks ? *reinterpret_cast<const float4*>(&ys[i16][64 * c + 16 * kq + 4 * q])
                                         : make_float4(0.f, 0.f, 0.f, 0.f);
        for (int rb = 0; rb < rbw; ++rb) {
            f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int c = 0; c < SMDL_MAX_M / 64; ++c) {
                if (c < a.mchunks) {
                    const float4* fp = a.dfrag + ((size_t)(c * NRB + rb0 + rb) * 4) * 64 + lane;
                    float4 af[4];
#pragma unroll
                    for (int q = 0; q < 4; ++q) af[q] = fp[q * 64];
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(af[q].x, yv[c][q].x, acc, 0, 0, 0);
                        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(af[q].y, yv[c][q].y, acc, 0, 0, 0);
                        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(af[q].z, yv[c][q].z, acc, 0, 0, 0);
                        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(af[q].w, yv[c][q].w, acc, 0, 0, 0);
                    }
                }
            }
            // tile entry (atom 16 rb + 4 kq + q, signal i16) in lane i16 + 16 kq, register q
            *reinterpret_cast<float4*>(&alpha[i16 * astride + 16 * (rb0 + rb) + 4 * kq]) =
                make_float4(acc[0], acc[1], acc[2], acc[3]);
        }
    }
    __syncthreads();
    int cid[EC];
    RState<SM> st;
    float ysq = 0.f;
    for (int i = g; i < m; i += GR) ysq = fmaf(ys[slot][i], ys[slot][i], ysq);
#pragma unroll
    for (int off = 1; off < GR; off <<= 1) ysq += __shfl_xor(ysq, off, 64);
#pragma unroll
    for (int t = 0; t < EC; ++t) {
        const int e = g + GR * t;
        cid[t] = (valid && e < nc) ? a.cand[n * nc + e] : -1;
        if (cid[t] < 0 || cid[t] >= a.K) cid[t] = -1;
        st.c[t] = cid[t] >= 0 ? alpha[slot * astride + cid[t]] : 0.f;
    }
#pragma unroll
    for (int i = 0; i < SM; ++i) {
        st.pi[i] = 0.f;
        st.sel[i] = 0;
#pragma unroll
        for (int l = 0; l <= i; ++l) st.Linv[i][l] = 0.f;
    }
    st.live = valid;
    st.k = 0;
    RCtx x{&a, cid, n, g, sqrtf(ysq)};
    r_run<SM>(st, x, std::make_integer_sequence<int, SM>{});
    const int k = st.k;
    // coefficients and the explicit residual
    float gam[SM];
#pragma unroll
    for (int l = 0; l < SM; ++l) {
        float acc = 0.f;
#pragma unroll
        for (int i = l; i < SM; ++i) acc = fmaf(st.Linv[i][l], (i < k) ? st.pi[i] : 0.f, acc);
        gam[l] = acc;
    }
    float rr = 0.f;
    for (int i = g; i < m; i += GR) {
        float r = ys[slot][i];
#pragma unroll
        for (int l = 0; l < SM; ++l)
            if (l < k) r = fmaf(-gam[l], a.D[(int64_t)st.sel[l] * m + i], r);
        rr = fmaf(r, r, rr);
    }
#pragma unroll
    for (int off = 1; off < GR; off <<= 1) rr += __shfl_xor(rr, off, 64);
    // the signals that miss the threshold go to the fallback list: one atomic per work group (a
    // counter taken once per signal serialises some 10^5 atomics on one address)
    const bool miss = valid && sqrtf(rr) > a.eps_fb;
    const uint64_t mb = __ballot(g == 0 && miss);                 // bits at the group leaders
    const int wave = tid >> 6;
    if (lane == 0) s_fbcnt[wave] = __popcll(mb);
    __syncthreads();
    if (tid == 0) {
        int tot = 0;
#pragma unroll
        for (int w = 0; w < 4; ++w) {
            const int c = s_fbcnt[w];
            s_fbcnt[w] = tot;
            tot += c;
        }
        s_fbbase = tot > 0 ? atomicAdd(a.fb_count, tot) : 0;
    }
    __syncthreads();
    if (!valid) return;
    if (g == 0) {
        if (a.fell_back) a.fell_back[n] = miss ? 1 : 0;
        if (miss) a.fb_list[s_fbbase + s_fbcnt[wave] + __popcll(mb & ((1ull << lane) - 1ull))] = (int32_t)n;
    }
    if (miss) return;    // the full OMP writes this signal's code
    if (g < a.s_out) {
        int oi = -1;
        float oc = 0.f;
#pragma unroll
        for (int i = 0; i < SM; ++i)
            if (i == g && i < k) { oi = st.sel[i]; oc = gam[i]; }
        a.idx[n * a.s_out + g] = oi;
        a.coef[n * a.s_out + g] = oc;
    }
    if (g == 0) a.nnz[n] = k;
}

}  // namespace

hipError_t launch_topk(const float* logits, int64_t N, int K, int n_cand, int32_t* cand, hipStream_t st) {
    if (K < 1 || K > SMDL_MAX_K || n_cand < 1 || n_cand > K) return hipErrorInvalidValue;
    const dim3 grid((unsigned)((N + 15) / 16));
    const int E = (K + 15) / 16;
    if (E <= 4) hipLaunchKernelGGL(topk_kernel<4>, grid, dim3(256), 0, st, logits, N, K, n_cand, cand);
    else if (E <= 8) hipLaunchKernelGGL(topk_kernel<8>, grid, dim3(256), 0, st, logits, N, K, n_cand, cand);
    else if (E <= 16) hipLaunchKernelGGL(topk_kernel<16>, grid, dim3(256), 0, st, logits, N, K, n_cand, cand);
    else if (E <= 32) hipLaunchKernelGGL(topk_kernel<32>, grid, dim3(256), 0, st, logits, N, K, n_cand, cand);
    else hipLaunchKernelGGL(topk_kernel<64>, grid, dim3(256), 0, st, logits, N, K, n_cand, cand);
    return hipGetLastError();
}

hipError_t launch_restricted_omp(const RestrictedArgs& a, hipStream_t st) {
    if (a.Kpad % 64 || a.Kpad > SMDL_MAX_K || a.mchunks < 1 || a.mchunks > SMDL_MAX_M / 64 || !a.dfrag)
        return hipErrorInvalidValue;
    const size_t lds = (size_t)16 * (a.Kpad + 4) * 4;    // alpha0 of the 16 signals
    static bool attr_set = false;
    if (!attr_set) {
        const int full = 16 * (SMDL_MAX_K + 4) * 4;
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&restricted_omp_kernel<8>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, full);
        if (e == hipSuccess)
            e = hipFuncSetAttribute(reinterpret_cast<const void*>(&restricted_omp_kernel<SMDL_MAX_S>),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, full);
        if (e != hipSuccess) return e;
        attr_set = true;
    }
    if (a.s <= 8)
        hipLaunchKernelGGL(restricted_omp_kernel<8>, dim3((unsigned)((a.N + 15) / 16)), dim3(256), lds, st, a);
    else
        hipLaunchKernelGGL(restricted_omp_kernel<SMDL_MAX_S>, dim3((unsigned)((a.N + 15) / 16)), dim3(256), lds, st, a);
    return hipGetLastError();
}

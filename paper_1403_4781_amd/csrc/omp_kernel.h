// Fused batch-OMP kernel for gfx950 (included by the omp_inst_*.hip translation units).
//
// One work item = up to T = 16*TT signals coded against one dictionary.
//
// Phase A (matrix cores): alpha0 = D^T y for the T signals with v_mfma_f32_16x16x4f32,
//   A operand = packed dictionary fragments (coalesced float4 loads, L2 resident),
//   B operand = the signals (float4 loads straight from HBM).  alpha0 and ||y||^2 go to LDS.
// Phase B (vector ALU): every signal is handled by a group of G lanes (16, 32 or 64); lane g
//   owns the E = Kpad/G correlation entries e(g,t) = 4G*(t/4) + 4g + t%4.  Per step k:
//     j     = argmax_e |c_e|                (lane-local scan + butterfly over the group)
//     g_i   = G[j, sel_i] (i < k), G_jj     (broadcast loads), row G[j, :] (coalesced float4)
//     w     = Linv g                        (Linv = inverse Cholesky factor of G_II)
//     l^2   = G_jj - w.w                    (squared distance of d_j to span D_I)
//     u     = (G[:, j] - U w) / l           (correlations of the new orthonormal direction;
//                                            U holds the unscaled vectors, the 1/l factors are
//                                            applied to the k coefficients instead)
//     pi_k  = c_j / l ;  c -= pi_k u ;  ||r||^2 -= pi_k^2
//     Linv row k = (-(w^T Linv)/l, 1/l)
//   and finally x_I = Linv^T pi.  This is OMP (least squares on the support at every step)
//   computed in correlation space; U (K x k), c and the Cholesky data stay in registers.
#pragma once

#include <utility>

#include "smdl_internal.h"

namespace smdl_omp {

__device__ __forceinline__ float4 load_y4(const float* __restrict__ y, int r, int m, bool vec) {
    if (vec && r + 3 < m) return *reinterpret_cast<const float4*>(y + r);
    float4 v;
    v.x = (r + 0 < m) ? y[r + 0] : 0.f;
    v.y = (r + 1 < m) ? y[r + 1] : 0.f;
    v.z = (r + 2 < m) ? y[r + 2] : 0.f;
    v.w = (r + 3 < m) ? y[r + 3] : 0.f;
    return v;
}

__device__ __forceinline__ float f4get(const float4& v, int e) {
    return e == 0 ? v.x : (e == 1 ? v.y : (e == 2 ? v.z : v.w));
}


// (value, index) combine of the argmax: larger |value| wins, the lower index on equal |value|.
// The order is total, so any reduction tree gives the same winner.
__device__ __forceinline__ void argmax_combine(float& bv, int& bi, float ov, int oi) {
    // bitwise (non short-circuit) so the compiler emits compares and selects, not branches
    const float ao = fabsf(ov), ab = fabsf(bv);
    const bool take = (ao > ab) | ((ao == ab) & (oi < bi));
    bv = take ? ov : bv;
    bi = take ? oi : bi;
}

template <int CTRL>
__device__ __forceinline__ void dpp_combine(float& bv, int& bi) {
    const float ov = __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(bv), CTRL, 0xf, 0xf, false));
    const int oi = __builtin_amdgcn_mov_dpp(bi, CTRL, 0xf, 0xf, false);
    argmax_combine(bv, bi, ov, oi);
}

// All-reduce of the argmax over the G lanes of a signal group (G = 16, 32 or 64; groups are
// aligned).  Within a row of 16 lanes: DPP quad_perm [1,0,3,2], quad_perm [2,3,0,1],
// row_half_mirror and row_mirror (VALU latency); across rows: lane shuffles.
template <int G>
__device__ __forceinline__ void group_argmax(float& bv, int& bi) {
    dpp_combine<0xB1>(bv, bi);    // quad_perm [1,0,3,2]
    dpp_combine<0x4E>(bv, bi);    // quad_perm [2,3,0,1]
    dpp_combine<0x141>(bv, bi);   // row_half_mirror: quad q <-> quad 1-q within 8 lanes
    dpp_combine<0x140>(bv, bi);   // row_mirror: half h <-> half 1-h within 16 lanes
#pragma unroll
    for (int off = 16; off < G; off <<= 1) {
        const float ov = __shfl_xor(bv, off, 64);
        const int oi = __shfl_xor(bi, off, 64);
        argmax_combine(bv, bi, ov, oi);
    }
}

template <int EM, int SM>
struct State {
    float c[EM];
    float U[SM][EM];
    float Linv[SM][SM];
    float pi[SM];
    float rl[SM];        // 1 / l_k of every step
    int sel[SM];
    float rn2;
    int k;
    bool live;
};

struct StepCtx {
    const float* __restrict__ gram;
    int E, s, g, Kpad;
    float eps2, tau, dep_tol, ynrm;
};

// One greedy step (step index KK is a compile-time constant so that every register array
// index below is static).  Returns false when the whole wave is done.
template <int KK, int EM, int SM, int G>
__device__ __forceinline__ bool omp_step(State<EM, SM>& st, const StepCtx& x) {
    if (KK >= x.s) return false;
    if (x.eps2 > 0.f && !(st.rn2 > x.eps2)) st.live = false;
    if (!__any(st.live)) return false;
    const int g = x.g;
    // argmax |c| over the group, lowest atom index on equal magnitude
    // entries t >= E hold exact zeros (their alpha0, G rows and U stay zero), so they never
    // win against a real entry and need no guard here
    float bv = st.c[0];
    int bi = 4 * g;
#pragma unroll
    for (int t = 1; t < EM; ++t) {
        const int e = 4 * G * (t >> 2) + 4 * g + (t & 3);
        const bool take = fabsf(st.c[t]) > fabsf(bv);
        bv = take ? st.c[t] : bv;
        bi = take ? e : bi;
    }
    group_argmax<G>(bv, bi);
    const int j = bi;
    const float cj = bv;
    if (!(fabsf(cj) > x.tau * x.ynrm)) st.live = false;
    if (st.live) {
        const float* grow = x.gram + (size_t)j * x.Kpad;
        float gr[EM];
#pragma unroll
        for (int q = 0; q < EM / 4; ++q) {
            float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
            if (4 * q < x.E) v = *reinterpret_cast<const float4*>(grow + 4 * G * q + 4 * g);
            gr[4 * q + 0] = v.x;
            gr[4 * q + 1] = v.y;
            gr[4 * q + 2] = v.z;
            gr[4 * q + 3] = v.w;
        }
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
        if (!(l2 > x.dep_tol * gjj)) {
            st.live = false;
        } else {
            const float rl = __builtin_amdgcn_rsqf(l2);      // 1 / l (v_rsq_f32, 1 ulp)
#pragma unroll
            for (int l = 0; l < KK; ++l) {
                float acc = 0.f;
#pragma unroll
                for (int i = l; i < KK; ++i) acc = fmaf(w[i], st.Linv[i][l], acc);
                st.Linv[KK][l] = -acc * rl;
            }
            st.Linv[KK][KK] = rl;
            const float pk = cj * rl;
            // U keeps the unscaled direction v_k = G[:, j] - sum_i u_i w_i, u_k = v_k / l_k: the
            // scale moves onto the k coefficients (w_i / l_i) and onto pi_k / l_k
            float wv[KK > 0 ? KK : 1];
#pragma unroll
            for (int i = 0; i < KK; ++i) wv[i] = w[i] * st.rl[i];
            const float pkr = pk * rl;
#pragma unroll
            for (int t = 0; t < EM; ++t) {
                float v = gr[t];
#pragma unroll
                for (int i = 0; i < KK; ++i) v = fmaf(-st.U[i][t], wv[i], v);
                st.U[KK][t] = v;
                st.c[t] = fmaf(-pkr, v, st.c[t]);
            }
            st.rl[KK] = rl;
            st.pi[KK] = pk;
            st.sel[KK] = j;
            st.rn2 = fmaf(-pk, pk, st.rn2);
            st.k = KK + 1;
        }
    }
    return true;
}

template <int EM, int SM, int G, int... KKs>
__device__ __forceinline__ void run_steps(State<EM, SM>& st, const StepCtx& x,
                                          std::integer_sequence<int, KKs...>) {
    (void)(omp_step<KKs, EM, SM, G>(st, x) && ...);
}

template <int EM, int SM, int G, int TT>
__global__ __launch_bounds__(256, 2) void omp_fused(OmpArgs a) {
    constexpr int T = 16 * TT;
    constexpr int GPW = 64 / G;          // signal groups per wave
    constexpr int SPP = 4 * GPW;         // signals per pass of the 4 waves
    constexpr int PASSES = (T + SPP - 1) / SPP;
    constexpr int RBW = EM * G / 64;     // max 16-atom row blocks per wave in phase A

    extern __shared__ float lds[];
    __shared__ int s_item;
    __shared__ OmpItem s_it;

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;

    int n_items = a.n_items;
    if (a.list_count) n_items = (*a.list_count + T - 1) / T;

    for (int round = 0;; ++round) {
        int item;
        if (a.queue) {
            if (tid == 0) s_item = atomicAdd(a.queue, 1);
            __syncthreads();
            item = s_item;
        } else {
            item = round == 0 ? (int)blockIdx.x : 0x7fffffff;
        }
        if (item >= n_items) break;
        if (tid == 0) {
            if (a.items) {
                s_it = a.items[item];
            } else {
                OmpItem it;
                it.desc = 0;
                it.first = (int64_t)item * T;
                int64_t n = a.list_count ? (int64_t)*a.list_count : a.desc[0].n;
                int64_t left = n - it.first;
                it.count = (int)(left < T ? left : T);
                s_it = it;
            }
        }
        __syncthreads();
        const OmpItem it = s_it;
        const OmpDesc d = a.desc[it.desc];
        const int Kpad = d.Kpad;
        const int stride = Kpad + 4;           // LDS row stride (floats) of alpha0
        float* alpha = lds;                    // T x stride
        float* yn2 = lds + T * stride;         // T

        // ------------------------------------------------------------------ phase A
        {
            const int i16 = lane & 15, kq = lane >> 4;
            const int NRB = Kpad >> 4;
            const int rbw = NRB >> 2;          // row blocks of this wave (Kpad % 64 == 0)
            const int rb0 = wave * rbw;
            f32x4 acc[RBW][TT];
#pragma unroll
            for (int rb = 0; rb < RBW; ++rb)
#pragma unroll
                for (int tt = 0; tt < TT; ++tt) acc[rb][tt] = f32x4{0.f, 0.f, 0.f, 0.f};
            const bool vec = ((a.m & 3) == 0) && ((reinterpret_cast<uintptr_t>(d.Y) & 15) == 0);
            const float* yp[TT];
            bool yok[TT];
#pragma unroll
            for (int tt = 0; tt < TT; ++tt) {
                int sl = 16 * tt + i16;
                yok[tt] = sl < it.count;
                int64_t sig = it.first + sl;
                if (a.sig_list) sig = yok[tt] ? a.sig_list[sig] : 0;
                yp[tt] = d.Y + (yok[tt] ? sig : 0) * (int64_t)a.m;
            }
            float ysq[TT];
#pragma unroll
            for (int tt = 0; tt < TT; ++tt) ysq[tt] = 0.f;
            for (int c = 0; c < a.mchunks; ++c) {
                float4 yv[TT][4];
#pragma unroll
                for (int tt = 0; tt < TT; ++tt)
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const int r = 64 * c + 16 * kq + 4 * q;
                        yv[tt][q] = yok[tt] ? load_y4(yp[tt], r, a.m, vec) : make_float4(0.f, 0.f, 0.f, 0.f);
                        ysq[tt] += yv[tt][q].x * yv[tt][q].x + yv[tt][q].y * yv[tt][q].y +
                                   yv[tt][q].z * yv[tt][q].z + yv[tt][q].w * yv[tt][q].w;
                    }
#pragma unroll
                for (int rb = 0; rb < RBW; ++rb) {
                    if (rb < rbw) {
                        const float4* fp = d.dfrag + ((size_t)(c * NRB + rb0 + rb) * 4) * 64 + lane;
                        float4 af[4];
#pragma unroll
                        for (int q = 0; q < 4; ++q) af[q] = fp[q * 64];
#pragma unroll
                        for (int tt = 0; tt < TT; ++tt)
#pragma unroll
                            for (int q = 0; q < 4; ++q) {
                                acc[rb][tt] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[q].x, yv[tt][q].x, acc[rb][tt], 0, 0, 0);
                                acc[rb][tt] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[q].y, yv[tt][q].y, acc[rb][tt], 0, 0, 0);
                                acc[rb][tt] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[q].z, yv[tt][q].z, acc[rb][tt], 0, 0, 0);
                                acc[rb][tt] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[q].w, yv[tt][q].w, acc[rb][tt], 0, 0, 0);
                            }
                    }
                }
            }
            // D[i][j] of the 16x16 tile sits in lane j + 16*(i/4), register i%4:
            // row i = atom 16*rb + 4*kq + q, column j = signal i16.
#pragma unroll
            for (int rb = 0; rb < RBW; ++rb) {
                if (rb < rbw) {
#pragma unroll
                    for (int tt = 0; tt < TT; ++tt) {
                        float* dst = alpha + (16 * tt + i16) * stride + 16 * (rb0 + rb) + 4 * kq;
                        *reinterpret_cast<float4*>(dst) =
                            make_float4(acc[rb][tt][0], acc[rb][tt][1], acc[rb][tt][2], acc[rb][tt][3]);
                    }
                }
            }
#pragma unroll
            for (int tt = 0; tt < TT; ++tt) {
                float v = ysq[tt];
                v += __shfl_xor(v, 16, 64);
                v += __shfl_xor(v, 32, 64);
                if (wave == 0 && kq == 0) yn2[16 * tt + i16] = v;
            }
        }
        __syncthreads();

        // ------------------------------------------------------------------ phase B
        {
            const int g = lane % G;
            const int grp = lane / G;
            StepCtx ctx;
            ctx.E = Kpad / G;
            ctx.s = d.s;
            ctx.g = g;
            ctx.gram = d.gram;
            ctx.Kpad = Kpad;
            ctx.eps2 = a.eps2;
            ctx.tau = a.tau;
            ctx.dep_tol = a.dep_tol;
#pragma unroll 1
            for (int p = 0; p < PASSES; ++p) {
                const int sl = p * SPP + wave * GPW + grp;
                const bool valid = sl < it.count;
                State<EM, SM> st;
#pragma unroll
                for (int i = 0; i < SM; ++i) {
                    st.pi[i] = 0.f;
                    st.sel[i] = 0;
#pragma unroll
                    for (int l = 0; l <= i; ++l) st.Linv[i][l] = 0.f;
                }
                const float* arow = alpha + (valid ? sl : 0) * stride + 4 * g;
#pragma unroll
                for (int q = 0; q < EM / 4; ++q) {
                    float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
                    if (4 * q < ctx.E) v = *reinterpret_cast<const float4*>(arow + 4 * G * q);
                    st.c[4 * q + 0] = v.x;
                    st.c[4 * q + 1] = v.y;
                    st.c[4 * q + 2] = v.z;
                    st.c[4 * q + 3] = v.w;
                }
                const float y2 = valid ? yn2[sl] : 0.f;
                ctx.ynrm = sqrtf(y2);
                st.rn2 = y2;
                st.live = valid;
                st.k = 0;
                run_steps<EM, SM, G>(st, ctx, std::make_integer_sequence<int, SM>{});
                if (valid) {
                    // x_I = Linv^T pi
                    float gam[SM];
#pragma unroll
                    for (int l = 0; l < SM; ++l) {
                        float acc = 0.f;
#pragma unroll
                        for (int i = l; i < SM; ++i) acc = fmaf(st.Linv[i][l], (i < st.k) ? st.pi[i] : 0.f, acc);
                        gam[l] = acc;
                    }
                    int64_t sig = it.first + sl;
                    if (a.sig_list) sig = a.sig_list[sig];
                    else sig += d.out0;
                    if (g < a.s_out) {
                        int oi = -1;
                        float oc = 0.f;
#pragma unroll
                        for (int i = 0; i < SM; ++i)
                            if (i == g && i < st.k) { oi = st.sel[i]; oc = gam[i]; }
                        a.idx[sig * a.s_out + g] = oi;
                        a.coef[sig * a.s_out + g] = oc;
                    }
                    if (g == 0) {
                        a.nnz[sig] = st.k;
                        if (a.res) a.res[sig] = sqrtf(fmaxf(st.rn2, 0.f));
                    }
                }
            }
        }
        __syncthreads();
    }
}

template <int EM, int SM, int G, int TT>
hipError_t launch_one(const OmpArgs& a, int grid, hipStream_t st, int maxKpad) {
    constexpr int T = 16 * TT;
    const size_t lds = (size_t)T * (maxKpad + 4) * 4 + T * 4;
    static size_t lds_enabled = 64 * 1024;   // dynamic LDS this instantiation may request
    if (lds > lds_enabled) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&omp_fused<EM, SM, G, TT>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        lds_enabled = lds;
    }
    hipLaunchKernelGGL((omp_fused<EM, SM, G, TT>), dim3(grid), dim3(256), lds, st, a);
    return hipGetLastError();
}

}  // namespace smdl_omp

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


// Group all-reduces over the G lanes of a signal (G = 16, 32 or 64; groups are aligned).
// Within a row of 16 lanes: DPP quad_perm [1,0,3,2], quad_perm [2,3,0,1], row_half_mirror,
// row_mirror, each folded into the max / min instruction; across rows: lane shuffles.
// DPP read of a neighbour lane; `ident` (the identity of the combining operation) stands for
// lanes the pattern leaves out, which lets the compiler fold the read into the max / min.
template <int CTRL>
__device__ __forceinline__ int dpp_i(int v, int ident) {
    return __builtin_amdgcn_update_dpp(ident, v, CTRL, 0xf, 0xf, false);
}

// Combine of a per-row (16-lane) result across the rows of a group of G = 32 or 64 lanes:
// v_permlane16_swap exchanges rows 0 <-> 1 and 2 <-> 3 between its two operands,
// v_permlane32_swap the halves; the max / min of the two outputs is the combined value.
template <int G>
__device__ __forceinline__ int cross_rows(int v, bool take_max) {
    if (G >= 32) {
        const auto r = __builtin_amdgcn_permlane16_swap(v, v, false, false);
        v = take_max ? max((int)r[0], (int)r[1]) : min((int)r[0], (int)r[1]);
    }
    if (G >= 64) {
        const auto r = __builtin_amdgcn_permlane32_swap(v, v, false, false);
        v = take_max ? max((int)r[0], (int)r[1]) : min((int)r[0], (int)r[1]);
    }
    return v;
}

// Maximum of non-negative floats by their bit patterns (which order like the values).
template <int G>
__device__ __forceinline__ float group_max_nonneg(float f) {
    int v = __float_as_int(f);
    v = max(v, dpp_i<0xB1>(v, 0));
    v = max(v, dpp_i<0x4E>(v, 0));
    v = max(v, dpp_i<0x141>(v, 0));
    v = max(v, dpp_i<0x140>(v, 0));
    v = cross_rows<G>(v, true);
    return __int_as_float(v);
}

template <int G>
__device__ __forceinline__ int group_min(int v) {
    v = min(v, dpp_i<0xB1>(v, 0x7fffffff));
    v = min(v, dpp_i<0x4E>(v, 0x7fffffff));
    v = min(v, dpp_i<0x141>(v, 0x7fffffff));
    v = min(v, dpp_i<0x140>(v, 0x7fffffff));
    return cross_rows<G>(v, false);
}

// Largest |c_t| of the lane (v_max3_f32 with |.| operand modifiers; exact).
template <int EM>
__device__ __forceinline__ float lane_max_abs(const float (&c)[EM]) {
    float m[EM];
#pragma unroll
    for (int t = 0; t < EM; ++t) m[t] = fabsf(c[t]);
#pragma unroll
    for (int w = 1; w < EM; w *= 3)
#pragma unroll
        for (int t = 0; t < EM; t += 3 * w) {
            if (t + w < EM) m[t] = fmaxf(m[t], m[t + w]);
            if (t + 2 * w < EM) m[t] = fmaxf(m[t], m[t + 2 * w]);
        }
    return m[0];
}

// Sum over the G lanes of a group; every lane gets the same bits (each combine is a commutative
// add of the same two values).
template <int G>
__device__ __forceinline__ float group_sum(float v) {
    v += __int_as_float(dpp_i<0xB1>(__float_as_int(v), 0));
    v += __int_as_float(dpp_i<0x4E>(__float_as_int(v), 0));
    v += __int_as_float(dpp_i<0x141>(__float_as_int(v), 0));
    v += __int_as_float(dpp_i<0x140>(__float_as_int(v), 0));
    if (G >= 32) {
        const auto r = __builtin_amdgcn_permlane16_swap(__float_as_int(v), __float_as_int(v), false, false);
        v = __int_as_float((int)r[0]) + __int_as_float((int)r[1]);
    }
    if (G >= 64) {
        const auto r = __builtin_amdgcn_permlane32_swap(__float_as_int(v), __float_as_int(v), false, false);
        v = __int_as_float((int)r[0]) + __int_as_float((int)r[1]);
    }
    return v;
}

// Per-signal state of the greedy loop, in registers.  The inverse Cholesky factor Linv of G_II
// is held by columns: lane g of the group keeps column g (Linv[i][g], zero for i < g), and the
// lane g < k keeps the atom chosen at step g.  Entries of step i are written only when the
// signal is still live at step i and read only for i < k, so none needs initialising.
template <int EM, int SM>
struct State {
    float c[EM];         // correlations of the residual with this lane's atoms
    float U[SM][EM];     // unscaled directions v_i = l_i u_i at this lane's atoms
    float Lc[SM];        // Linv[i][g]
    float pi[SM];        // pi_i = c_j / l_i of step i
    float rl[SM];        // 1 / l_i
    int sel;             // atom chosen at step g
    float rn2;           // ||r||^2
    int k;               // atoms chosen
    bool live;
};

struct StepCtx {
    const float* __restrict__ gram;
    const float* arow;   // alpha0 of the signal (LDS), atom 0
    int g, s, gld, kpad;
    float eps2, tau, dep_tol, ynrm;
};

// Global loads at a 32-bit byte offset from a wave-uniform base (global_load with a scalar
// base address and a 32-bit vector offset).
__device__ __forceinline__ f32x4 gload4(const float* base, uint32_t byte_off) {
    return *(const __attribute__((address_space(1))) f32x4*)(reinterpret_cast<const char*>(base) + byte_off);
}
__device__ __forceinline__ float gload(const float* base, uint32_t byte_off) {
    return *(const __attribute__((address_space(1))) float*)(reinterpret_cast<const char*>(base) + byte_off);
}

// One greedy step (step index KK is a compile-time constant so that every register array
// index below is static).  Returns false when the whole wave is done.
template <int KK, int EM, int SM, int G>
__device__ __forceinline__ bool omp_step(State<EM, SM>& st, const StepCtx& x) {
    if (KK >= x.s) return false;
    if (x.eps2 > 0.f && !(st.rn2 > x.eps2)) st.live = false;
    if (!__any(st.live)) return false;
    const int g = x.g;
    // argmax |c| over the group: the exact maximum M, then the lowest atom index holding it.
    // Entries t >= E hold exact zeros (their alpha0 and G rows are zero), so they never win.
    const float M = group_max_nonneg<G>(lane_max_abs<EM>(st.c));
    // lowest entry t of the lane with |c_t| == M: four independent chains (t % 4), then a min
    int tq[4] = {EM, EM, EM, EM};
#pragma unroll
    for (int t = EM - 1; t >= 0; --t) tq[t & 3] = (fabsf(st.c[t]) == M) ? t : tq[t & 3];
    const int tl = min(min(tq[0], tq[1]), min(tq[2], tq[3]));
    const int el = tl < EM ? 4 * G * (tl >> 2) + 4 * g + (tl & 3) : 0x7fffffff;
    const int j = group_min<G>(el);
    // (j is a valid atom whenever M is a finite maximum; the test keeps any other case away
    // from the loads below)
    if (!(M > x.tau * x.ynrm) || (uint32_t)j >= (uint32_t)x.kpad) st.live = false;
    if (st.live) {
        // 32-bit offsets from the (uniform) Gram base: global loads with a scalar base
        const uint32_t row = (uint32_t)j * (uint32_t)x.gld * 4u;   // bytes
        // row j of G at this lane's atoms (columns < EM * G <= gld: no guard needed)
        float gr[EM];
#pragma unroll
        for (int q = 0; q < EM / 4; ++q) {
            const f32x4 v = gload4(x.gram, row + (uint32_t)(16 * G * q + 16 * g));
            gr[4 * q + 0] = v[0];
            gr[4 * q + 1] = v[1];
            gr[4 * q + 2] = v[2];
            gr[4 * q + 3] = v[3];
        }
        // lane g < k: G[j, sel_g]
        const bool mine = g < KK;
        float gsg = gload(x.gram, row + 4u * (uint32_t)(mine ? st.sel : j));
        gsg = mine ? gsg : 0.f;
        const float gjj = gload(x.gram, row + 4u * (uint32_t)j);
        const float a0j = x.arow[j];
        // w = Linv g (= u_i(j), the earlier directions at atom j): w_i = sum_g Linv[i][g] G[j, sel_g]
        float w[KK > 0 ? KK : 1];
        float l2 = gjj;
#pragma unroll
        for (int i = 0; i < KK; ++i) {
            w[i] = group_sum<G>(st.Lc[i] * gsg);
            l2 = fmaf(-w[i], w[i], l2);
        }
        // d_j (numerically) in the span of the chosen atoms: the signal stops here.  The update
        // below runs regardless with a zero step, which leaves c unchanged, so that the G-row
        // loads above are not held back behind this test.
        const bool ok = l2 > x.dep_tol * gjj;
        {
            const float rl = __builtin_amdgcn_rsqf(l2);      // 1 / l (v_rsq_f32, 1 ulp)
            // c_j: magnitude M (the maintained value), sign of alpha0_j - sum_i pi_i u_i(j)
            float cr = a0j;
#pragma unroll
            for (int i = 0; i < KK; ++i) cr = fmaf(-st.pi[i], w[i], cr);
            const float cj = copysignf(M, cr);
            const float pk = cj * rl;
            // U keeps the unscaled direction v_k = G[:, j] - sum_i u_i w_i, u_k = v_k / l_k: the
            // scale moves onto the k coefficients (w_i / l_i) and onto pi_k / l_k
            float wv[KK > 0 ? KK : 1];
#pragma unroll
            for (int i = 0; i < KK; ++i) wv[i] = w[i] * st.rl[i];
            const float pkr = ok ? pk * rl : 0.f;
#pragma unroll
            for (int t = 0; t < EM; ++t) {
                float v = gr[t];
#pragma unroll
                for (int i = 0; i < KK; ++i) v = fmaf(-st.U[i][t], wv[i], v);
                st.U[KK][t] = v;
                st.c[t] = fmaf(-pkr, v, st.c[t]);
            }
            // Linv row k = (-(w^T Linv) / l, 1 / l): lane g forms entry g
            float hg = 0.f;
#pragma unroll
            for (int i = 0; i < KK; ++i) hg = fmaf(w[i], st.Lc[i], hg);
            st.Lc[KK] = mine ? -hg * rl : (g == KK ? rl : 0.f);
            st.pi[KK] = pk;
            st.rl[KK] = rl;
            st.sel = (g == KK) ? j : st.sel;
            st.rn2 = ok ? fmaf(-pk, pk, st.rn2) : st.rn2;
            st.k = ok ? KK + 1 : st.k;
            st.live = ok;
        }
    }
    return true;
}

template <int EM, int SM, int G, int... KKs>
__device__ __forceinline__ void run_steps(State<EM, SM>& st, const StepCtx& x,
                                          std::integer_sequence<int, KKs...>) {
    (void)(omp_step<KKs, EM, SM, G>(st, x) && ...);
}

// Two waves per SIMD (at most 256 registers per lane), except where a lane holds 16 x 16 or more
// directions: those tiles get one wave per SIMD, so that the AGPRs can hold what does not fit in
// the 256 VGPRs (no scratch: measured 2x faster at K=1024, s=16 than the spilling two-wave build).
template <int EM, int SM, int G, int TT>
__global__ __launch_bounds__(256, (EM * SM >= 256) ? 1 : 2) void omp_fused(OmpArgs a) {
    constexpr int T = 16 * TT;
    constexpr int GPW = 64 / G;          // signal groups per wave
    constexpr int SPP = 4 * GPW;         // signals per pass of the 4 waves
    constexpr int PASSES = (T + SPP - 1) / SPP;
    constexpr int RBW = EM * G / 64;     // max 16-atom row blocks per wave in phase A

    extern __shared__ float lds[];
    __shared__ int s_item;
    __shared__ OmpItem s_it;

    const int tid = threadIdx.x;

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
        // the item is the same for the whole group: keep it (and so the descriptor) in SGPRs
        OmpItem it;
        it.desc = __builtin_amdgcn_readfirstlane(s_it.desc);
        it.count = __builtin_amdgcn_readfirstlane(s_it.count);
        it.first = ((int64_t)__builtin_amdgcn_readfirstlane((int)(s_it.first >> 32)) << 32) |
                   (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)s_it.first);
        const OmpDesc d = a.desc[it.desc];
        // lane ids made opaque per item: otherwise the compiler hoists every lane-dependent
        // address of both phases out of the item loop and keeps them all live in registers
        int lid = tid & 63;
        asm volatile("" : "+v"(lid));
        const int lane = lid;
        const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
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
            const int E = Kpad / G;
            StepCtx ctx;
            ctx.s = d.s;
            ctx.g = g;
            {
                const uint64_t gp = reinterpret_cast<uint64_t>(d.gram);
                ctx.gram = reinterpret_cast<const float*>(
                    ((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(gp >> 32)) << 32) |
                    (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)gp));
            }
            ctx.gld = d.gld;
            ctx.kpad = Kpad;
            ctx.eps2 = a.eps2;
            ctx.tau = a.tau;
            ctx.dep_tol = a.dep_tol;
#pragma unroll 1
            for (int p = 0; p < PASSES; ++p) {
                const int sl = p * SPP + wave * GPW + grp;
                const bool valid = sl < it.count;
                State<EM, SM> st;
                ctx.arow = alpha + (valid ? sl : 0) * stride;
                const float* arow = ctx.arow + 4 * g;
#pragma unroll
                for (int q = 0; q < EM / 4; ++q) {
                    float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
                    if (4 * q < E) v = *reinterpret_cast<const float4*>(arow + 4 * G * q);
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
                    int64_t sig = it.first + sl;
                    if (a.sig_list) sig = a.sig_list[sig];
                    else sig += d.out0;
                    if (g < a.s_out) {
                        // x_I = Linv^T pi; lane g forms and writes entry g
                        int oi = -1;
                        float oc = 0.f;
                        if (g < st.k) {
#pragma unroll
                            for (int i = 0; i < SM; ++i) {
                                const float t = fmaf(st.Lc[i], st.pi[i], oc);
                                oc = (i < st.k) ? t : oc;
                            }
                            oi = st.sel;
                        }
                        a.idx[sig * a.s_out + g] = oi;
                        a.coef[sig * a.s_out + g] = oc;
                    }
                    if (g == 0) {
                        a.nnz[sig] = st.k;
                        if (a.res) a.res[sig] = sqrtf(fmaxf(st.rn2, 0.f));
                    }
                }
                __builtin_amdgcn_wave_barrier();
            }
        }
        __syncthreads();
    }
}

// Dynamic LDS of one work group: alpha0 (T rows of maxKpad + 4 floats) and ||y||^2 (T floats).
template <int SM, int G, int TT>
constexpr size_t omp_lds_size(int maxKpad) {
    return ((size_t)16 * TT * (maxKpad + 4) + 16 * TT) * 4;
}

template <int EM, int SM, int G, int TT>
hipError_t launch_one(const OmpArgs& a, int grid, hipStream_t st, int maxKpad) {
    const size_t lds = omp_lds_size<SM, G, TT>(maxKpad);
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

// Fused batch-OMP kernel for gfx950 (included by the omp_inst_*.hip translation units).
//
// One work item = up to T = 16*TT signals coded against one dictionary.
//
// Phase A (matrix cores): alpha0 = D^T y for the T signals on v_mfma_f32_16x16x16_f16 from a
//   three-term FP16 split of both operands (FP32-accurate to about 2^-22; see the phase),
//   A operand = split dictionary fragments (coalesced 8-byte loads, L2 resident),
//   B operand = the signals (float4 loads straight from HBM, split in registers).  alpha0 and
//   ||y||^2 go to LDS.
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

#include <algorithm>
#include <utility>

#include "smdl_internal.h"

namespace smdl_omp {

// The error-constrained stopping test recomputes the residual from the signal and the atoms when
// the downdated ||r||^2 lies within this fraction of ||y||^2 of eps^2 (the downdated value carries
// rounding errors of a few 2^-22 ||y||^2 per step).
constexpr float EXPLICIT_MARGIN = 0x1p-13f;

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

// group_sum of a value that is zero outside the first 16 lanes of the group (the terms of the
// w_i of a step: lane g holds one only for g < k <= 15).  For a 64-lane group the first row's
// sum, read from lane 0, is the group's sum (the other rows add exact zeros) and costs one
// v_readlane instead of the two cross-row exchanges and adds.
template <int G>
__device__ __forceinline__ float group_sum_head(float v) {
    if constexpr (G == 64) {
        v += __int_as_float(dpp_i<0xB1>(__float_as_int(v), 0));
        v += __int_as_float(dpp_i<0x4E>(__float_as_int(v), 0));
        v += __int_as_float(dpp_i<0x141>(__float_as_int(v), 0));
        v += __int_as_float(dpp_i<0x140>(__float_as_int(v), 0));
        return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 0));
    } else {
        return group_sum<G>(v);
    }
}

// Whether a tile keeps the directions scaled (u_i) rather than unscaled (v_i = l_i u_i, with the
// 1 / l_i applied to the k coefficients of each update instead): scaled costs EM multiplies per
// step and saves the SM registers of the 1 / l_i, which the 16-step tiles need.
template <int SM>
constexpr bool SCALED_U = SM >= 12;

// Per-signal state of the greedy loop, in registers.  The inverse Cholesky factor Linv of G_II
// is held by columns: lane g of the group keeps column g (Linv[i][g], zero for i < g), and the
// lane g < k keeps the atom chosen at step g.  Entries of step i are written only when the
// signal is still live at step i and read only for i < k, so none needs initialising.
template <int EM, int SM>
struct State {
    float c[EM];         // correlations of the residual with this lane's atoms
    float U[SM][EM];     // directions at this lane's atoms: v_i = l_i u_i, or u_i (SCALED_U)
    float Lc[SM];        // Linv[i][g]
    float pi[SM];        // pi_i = c_j / l_i of step i
    float rl[SM];        // 1 / l_i (unscaled directions only)
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
    // explicit residuals: the dictionary (K atoms of m floats) and the signal, row r at
    // yp[(r / 4) * ystr + r % 4] (the LDS copy, or memory with ystr = 4)
    const float* D;
    const float* yp;
    int K, m, ystr;
    float marg;          // |rn2 - eps2| below which the stopping test uses the explicit residual
};

// Value of lane I of the group of G lanes (I static): v_readlane for a whole-wave group,
// otherwise ds_swizzle in bit mode (source lane = (lane & and_mask) | or_mask within 32 lanes).
template <int G, int I>
__device__ __forceinline__ int group_bcast(int v) {
    if constexpr (G == 64) return __builtin_amdgcn_readlane(v, I);
    else return __builtin_amdgcn_ds_swizzle(v, (I << 5) | (G == 16 ? 0x10 : 0x00));
}

// v - sum_{i in I...} x_i D[sel_i][r], x_i and sel_i taken from lane i of the group (only i < k).
template <int G, int... I>
__device__ __forceinline__ float sub_atoms(float v, float xg, int selg, int k, const float* D, int m, int r,
                                           std::integer_sequence<int, I...>) {
    ((v = fmaf(-__int_as_float(group_bcast<G, I>(__float_as_int(xg))),
               D[(size_t)(I < k ? group_bcast<G, I>(selg) : 0) * m + r], v)),
     ...);
    return v;
}

// x_i and the address of atom sel_i, taken from lane i of the group, for every i in I... (atom 0
// and a zero coefficient for i >= k).
template <int G, int... I>
__device__ __forceinline__ void bcast_atoms(float xg, int selg, int k, const float* D, int m, float* xb,
                                            const float** db, std::integer_sequence<int, I...>) {
    ((xb[I] = __int_as_float(group_bcast<G, I>(__float_as_int(xg))),
      db[I] = D + (size_t)(I < k ? group_bcast<G, I>(selg) : 0) * m),
     ...);
}

// ||y - D_I x_I||^2 computed from the signal and the atoms (FP32), for the first k chosen atoms
// (k <= KMAX) with x_I = Linv^T pi the least-squares coefficients on them.  Lane g takes rows
// g, g + G, ...; every lane of the group gets the sum.  Indices of entries past k are replaced by
// atom 0 with a zero coefficient, so every load stays inside D.
// The same in row groups of four (m % 4 == 0, D and the signal rows 16-byte aligned): lane g takes
// row groups g, g + G, ...; the coefficients and atom indices are broadcast once; one 16-byte load
// per atom and row group.
template <int KMAX, int EM, int SM, int G>
__device__ __forceinline__ float explicit_rn2_v4(const State<EM, SM>& st, const StepCtx& x, int k) {
    static_assert(KMAX <= SM, "at most SM atoms");
    float xg = 0.f;
#pragma unroll
    for (int i = 0; i < KMAX; ++i) {
        const float t = fmaf(st.Lc[i], st.pi[i], xg);
        xg = (i < k) ? t : xg;
    }
    xg = (x.g < k) ? xg : 0.f;
    const int selg = ((uint32_t)st.sel < (uint32_t)x.K) ? st.sel : 0;
    float xb[KMAX];
    const float* db[KMAX];
    bcast_atoms<G>(xg, selg, k, x.D, x.m, xb, db, std::make_integer_sequence<int, KMAX>{});
    float acc = 0.f;
#pragma unroll 1
    for (int q = x.g; 4 * q < x.m; q += G) {
        float4 v = *reinterpret_cast<const float4*>(x.yp + q * x.ystr);
#pragma unroll
        for (int i = 0; i < KMAX; ++i) {
            const float4 d = *reinterpret_cast<const float4*>(db[i] + 4 * q);
            v.x = fmaf(-xb[i], d.x, v.x);
            v.y = fmaf(-xb[i], d.y, v.y);
            v.z = fmaf(-xb[i], d.z, v.z);
            v.w = fmaf(-xb[i], d.w, v.w);
        }
        acc = fmaf(v.x, v.x, fmaf(v.y, v.y, fmaf(v.z, v.z, fmaf(v.w, v.w, acc))));
    }
    return group_sum<G>(acc);
}

template <int KMAX, int EM, int SM, int G>
__device__ __forceinline__ float explicit_rn2(const State<EM, SM>& st, const StepCtx& x, int k) {
    static_assert(KMAX <= SM, "at most SM atoms");
    float xg = 0.f;
#pragma unroll
    for (int i = 0; i < KMAX; ++i) {
        const float t = fmaf(st.Lc[i], st.pi[i], xg);
        xg = (i < k) ? t : xg;
    }
    xg = (x.g < k) ? xg : 0.f;
    const int selg = ((uint32_t)st.sel < (uint32_t)x.K) ? st.sel : 0;
    float acc = 0.f;
#pragma unroll 1
    for (int r = x.g; r < x.m; r += G) {
        const float v = sub_atoms<G>(x.yp[(r >> 2) * x.ystr + (r & 3)], xg, selg, k, x.D, x.m, r,
                                     std::make_integer_sequence<int, KMAX>{});
        acc = fmaf(v, v, acc);
    }
    return group_sum<G>(acc);
}

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
    if (x.eps2 > 0.f) {
        // error-constrained stop: ||r||^2 <= eps^2.  Near eps the downdated value (||y||^2 minus
        // the squared projections) may have lost the digits that decide; there the residual is
        // recomputed from the signal and the atoms.
        bool stop = !(st.rn2 > x.eps2);
        const bool near = st.live && fabsf(st.rn2 - x.eps2) <= x.marg;
        if (__any(near)) {
            const float e2 = explicit_rn2<KK, EM, SM, G>(st, x, KK);
            stop = near ? !(e2 > x.eps2) : stop;
        }
        if (stop) st.live = false;
    }
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
    // the last step of the tile updates neither U nor the correlations: nothing reads them after it
    constexpr bool UPDATE = KK + 1 < SM;
    if (st.live) {
        // 32-bit offsets from the (uniform) Gram base: global loads with a scalar base
        const uint32_t row = (uint32_t)j * (uint32_t)x.gld * 4u;   // bytes
        // row j of G at this lane's atoms (columns < EM * G <= gld: no guard needed)
        float gr[EM];
        if (UPDATE) {
#pragma unroll
            for (int q = 0; q < EM / 4; ++q) {
                const f32x4 v = gload4(x.gram, row + (uint32_t)(16 * G * q + 16 * g));
                gr[4 * q + 0] = v[0];
                gr[4 * q + 1] = v[1];
                gr[4 * q + 2] = v[2];
                gr[4 * q + 3] = v[3];
            }
        }
        // lane g < k: G[j, sel_g]
        const bool mine = g < KK;
        float gsg = gload(x.gram, row + 4u * (uint32_t)(mine ? st.sel : j));
        gsg = mine ? gsg : 0.f;
        const float gjj = gload(x.gram, row + 4u * (uint32_t)j);
        const float a0j = x.arow[j];
        // w = Linv g (= u_i(j), the earlier directions at atom j): w_i = sum_g Linv[i][g] G[j, sel_g]
        static_assert(SM <= 16, "the w terms lie in the first 16 lanes of a group");
        float w[KK > 0 ? KK : 1];
        float l2 = gjj;
#pragma unroll
        for (int i = 0; i < KK; ++i) {
            w[i] = group_sum_head<G>(st.Lc[i] * gsg);
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
            if (UPDATE) {
                // (SCALED_U: U holds u_k = v_k / l_k itself, so that the 1 / l_i need no registers)
                float wv[KK > 0 ? KK : 1];
#pragma unroll
                for (int i = 0; i < KK; ++i) wv[i] = SCALED_U<SM> ? w[i] : w[i] * st.rl[i];
                const float pkr = ok ? pk * rl : 0.f;
#pragma unroll
                for (int t = 0; t < EM; ++t) {
                    float v = gr[t];
#pragma unroll
                    for (int i = 0; i < KK; ++i) v = fmaf(-st.U[i][t], wv[i], v);
                    st.U[KK][t] = SCALED_U<SM> ? v * rl : v;
                    st.c[t] = fmaf(-pkr, v, st.c[t]);
                }
            }
            // Linv row k = (-(w^T Linv) / l, 1 / l): lane g forms entry g
            float hg = 0.f;
#pragma unroll
            for (int i = 0; i < KK; ++i) hg = fmaf(w[i], st.Lc[i], hg);
            st.Lc[KK] = mine ? -hg * rl : (g == KK ? rl : 0.f);
            st.pi[KK] = pk;
            if (!SCALED_U<SM>) st.rl[KK] = rl;
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

// The work item with index `item`: from the item list, or the item-th block of T signals of the
// single descriptor (of the device-side count in gather mode).
template <int T>
__device__ __forceinline__ OmpItem item_of(const OmpArgs& a, int item) {
    if (a.items) return a.items[item];
    OmpItem it;
    it.desc = 0;
    it.first = (int64_t)item * T;
    const int64_t n = a.list_count ? (int64_t)*a.list_count : a.desc[0].n;
    const int64_t left = n - it.first;
    it.count = (int)(left < T ? left : T);
    return it;
}

// A copy of a struct held in LDS, every 32-bit word read as a wave-uniform value (so that its
// pointers and sizes live in scalar registers).
template <typename S>
__device__ __forceinline__ S uniform_copy(const S& src) {
    static_assert(sizeof(S) % 4 == 0, "word-sized struct expected");
    constexpr int W = sizeof(S) / 4;
    uint32_t w[W];
    const uint32_t* p = reinterpret_cast<const uint32_t*>(&src);
#pragma unroll
    for (int i = 0; i < W; ++i) w[i] = (uint32_t)__builtin_amdgcn_readfirstlane((int)p[i]);
    S out;
    __builtin_memcpy(&out, w, sizeof(S));
    return out;
}

// Direct-to-LDS copy of the item's signals, issued by one wave.  Layout: rows 4q .. 4q + 3 of the
// signal in slot s at ybuf + 4 (q T + s), so that the 16 lanes reading one row group of 16
// signals read 256 contiguous bytes.  Lane l of an instruction writes LDS address (instruction
// base) + 16 l, so every instruction fills 64 consecutive positions; each lane fetches the chunk
// its position holds (nothing for the slots past the item's count).
template <int T>
__device__ __forceinline__ void prefetch_signals(const OmpArgs& a, const OmpItem& it, const float* Y, float* ybuf,
                                                 int lane) {
    const int total = (a.m >> 2) * T;
    for (int base = 0; base < total; base += 64) {
        const int p = base + lane;
        const int sl = p % T, q = p / T;
        if (p < total && sl < it.count) {
            int64_t sig = it.first + sl;
            if (a.sig_list) sig = a.sig_list[sig];
            __builtin_amdgcn_global_load_lds(
                (const void __attribute__((address_space(1)))*)(Y + sig * (int64_t)a.m + 4 * q),
                (void __attribute__((address_space(3)))*)(ybuf + 4 * base), 16, 0, 0);
        }
    }
}

// Phase A of one work item: alpha0 and ||y||^2 of its signals into LDS (see the kernel).  LDS: the
// signals come from the item's copy in LDS (m % 4 == 0), otherwise from memory.
template <int TT, int RBW, bool LDS>
__device__ __forceinline__ void alpha0_phase(const OmpArgs& a, const OmpDesc& d, const OmpItem& it,
                                             const float* ybuf, float* alpha, float* yn2, int stride, int lane,
                                             int wave) {
    typedef _Float16 h4 __attribute__((ext_vector_type(4)));
    const int Kpad = d.Kpad;
    const int i16 = lane & 15, kq = lane >> 4;
    const int NRB = Kpad >> 4;
    const int rbw = NRB >> 2;          // row blocks of this wave (Kpad % 64 == 0)
    const int rb0 = wave * rbw;
    const int KB = 4 * a.mchunks;      // 16-row blocks (rows past m are zero)
    const bool vec = ((a.m & 3) == 0) && ((reinterpret_cast<uintptr_t>(d.Y) & 15) == 0);
    const float* yp[TT];
    bool yok[TT];
#pragma unroll
    for (int tt = 0; tt < TT; ++tt) {
        const int sl = 16 * tt + i16;
        yok[tt] = sl < it.count;
        int64_t sig = it.first + sl;
        if (a.sig_list) sig = yok[tt] ? a.sig_list[sig] : 0;
        yp[tt] = d.Y + (yok[tt] ? sig : 0) * (int64_t)a.m;
    }
    // four rows of signal 16 tt + i16 (zero past m and for empty slots): from the LDS copy
    // (an in-bounds read whatever the slot, then a select), or from memory
    auto yrow = [&](int tt, int r) -> float4 {
        if (LDS) {
            const float4 v = *reinterpret_cast<const float4*>(ybuf + 4 * ((min(r, a.m - 4) >> 2) * (16 * TT) + 16 * tt + i16));
            const bool ok = yok[tt] && r < a.m;
            return ok ? v : make_float4(0.f, 0.f, 0.f, 0.f);
        }
        return yok[tt] ? load_y4(yp[tt], r, a.m, vec) : make_float4(0.f, 0.f, 0.f, 0.f);
    };
    const h4* fhi = static_cast<const h4*>(d.fhi);
    const h4* flo = static_cast<const h4*>(d.flo);
    // the scale of each signal: none when its largest entry lies in [2^-3, 2^14) (no FP16
    // overflow, the lo halves of the largest entries are normal FP16 numbers), otherwise the
    // power of two that brings it into [0.5, 1)
    int ye[TT];
    float ysq[TT];
#pragma unroll
    for (int tt = 0; tt < TT; ++tt) {
        float mx = 0.f;
        for (int kb = 0; kb < KB; ++kb) {
            const float4 v = yrow(tt, 16 * kb + 4 * kq);
            mx = fmaxf(mx, fmaxf(fmaxf(fabsf(v.x), fabsf(v.y)), fmaxf(fabsf(v.z), fabsf(v.w))));
        }
        mx = fmaxf(mx, __shfl_xor(mx, 16, 64));
        mx = fmaxf(mx, __shfl_xor(mx, 32, 64));
        int e = 0;
        if (mx > 0.f) (void)frexpf(mx, &e);
        ye[tt] = (mx == 0.f || (mx >= 0.125f && mx < 16384.f)) ? 0 : e;
        ysq[tt] = 0.f;
    }
    // The products over all 16-row blocks, with ||y||^2, in passes over at most four of the wave's
    // row blocks (wide waves, RBW > 4, take two or more passes, each reading the signal rows again:
    // a second register set of fragments for all their row blocks would not fit beside the
    // accumulators).  The fragments of a pass's row blocks of one 16-row block are requested
    // together, those of the next 16-row block while the current one is multiplied (row blocks
    // past this wave's share are clamped to its last one, not used).
    constexpr int RBH = RBW < 4 ? RBW : 4;
    constexpr int NH = (RBW + RBH - 1) / RBH;
#pragma unroll 1
    for (int h = 0; h < NH; ++h) {
        const int rbase = rb0 + h * RBH;
        const int rbh = min(RBH, rbw - h * RBH);     // row blocks of this pass
        if (rbh <= 0) break;
        f32x4 acc[RBH][TT];
#pragma unroll
        for (int rb = 0; rb < RBH; ++rb)
#pragma unroll
            for (int tt = 0; tt < TT; ++tt) acc[rb][tt] = f32x4{0.f, 0.f, 0.f, 0.f};
        h4 nh[RBH], nl[RBH];
        auto request = [&](int kb) {
#pragma unroll
            for (int rb = 0; rb < RBH; ++rb) {
                const size_t o = ((size_t)kb * NRB + rbase + min(rb, rbh - 1)) * 64 + lane;
                nh[rb] = fhi[o];
                nl[rb] = flo[o];
            }
        };
        request(0);
        for (int kb = 0; kb < KB; ++kb) {
            const int r = 16 * kb + 4 * kq;
            h4 ah[RBH], al[RBH];
#pragma unroll
            for (int rb = 0; rb < RBH; ++rb) {
                ah[rb] = nh[rb];
                al[rb] = nl[rb];
            }
            if (kb + 1 < KB) request(kb + 1);
            h4 bh[TT], bl[TT];
#pragma unroll
            for (int tt = 0; tt < TT; ++tt) {
                float4 v = yrow(tt, r);
                if (h == 0) ysq[tt] += v.x * v.x + v.y * v.y + v.z * v.z + v.w * v.w;
                v.x = ldexpf(v.x, -ye[tt]);
                v.y = ldexpf(v.y, -ye[tt]);
                v.z = ldexpf(v.z, -ye[tt]);
                v.w = ldexpf(v.w, -ye[tt]);
                bh[tt][0] = (_Float16)v.x;
                bh[tt][1] = (_Float16)v.y;
                bh[tt][2] = (_Float16)v.z;
                bh[tt][3] = (_Float16)v.w;
                bl[tt][0] = (_Float16)(v.x - (float)bh[tt][0]);
                bl[tt][1] = (_Float16)(v.y - (float)bh[tt][1]);
                bl[tt][2] = (_Float16)(v.z - (float)bh[tt][2]);
                bl[tt][3] = (_Float16)(v.w - (float)bh[tt][3]);
            }
#pragma unroll
            for (int rb = 0; rb < RBH; ++rb) {
                if (rb < rbh) {
#pragma unroll
                    for (int tt = 0; tt < TT; ++tt) {
                        acc[rb][tt] = __builtin_amdgcn_mfma_f32_16x16x16f16(al[rb], bh[tt], acc[rb][tt], 0, 0, 0);
                        acc[rb][tt] = __builtin_amdgcn_mfma_f32_16x16x16f16(ah[rb], bl[tt], acc[rb][tt], 0, 0, 0);
                        acc[rb][tt] = __builtin_amdgcn_mfma_f32_16x16x16f16(ah[rb], bh[tt], acc[rb][tt], 0, 0, 0);
                    }
                }
            }
        }
        // D[i][j] of the 16x16 tile sits in lane j + 16*(i/4), register i%4:
        // row i = atom 16*rb + 4*kq + q, column j = signal i16.  Undo the scales.
#pragma unroll
        for (int rb = 0; rb < RBH; ++rb) {
            if (rb < rbh) {
                const int atom0 = 16 * (rbase + rb) + 4 * kq;
                const int4 ea = *reinterpret_cast<const int4*>(d.aexp + atom0);
#pragma unroll
                for (int tt = 0; tt < TT; ++tt) {
                    float* dst = alpha + (16 * tt + i16) * stride + atom0;
                    *reinterpret_cast<float4*>(dst) =
                        make_float4(ldexpf(acc[rb][tt][0], ea.x + ye[tt]), ldexpf(acc[rb][tt][1], ea.y + ye[tt]),
                                    ldexpf(acc[rb][tt][2], ea.z + ye[tt]), ldexpf(acc[rb][tt][3], ea.w + ye[tt]));
                }
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

// Two waves per SIMD (at most 256 registers per lane), except where a lane holds 16 x 16 or more
// directions: those tiles get one wave per SIMD, so that the AGPRs can hold what does not fit in
// the 256 VGPRs (no scratch: measured 2x faster at K=1024, s=16 than the spilling two-wave build).
//
// Persistent: work group b takes the items b, b + grid, b + 2 grid, ... .  Each item's work
// item and dictionary descriptor are staged in LDS one item ahead (so an item starts without a
// chain of dependent memory round trips), and with a.y_lds the next item's signals are copied
// into the other half of a double buffer in LDS while the current item runs its greedy loop, so
// that the correlations of the next item read LDS instead of waiting on HBM.
template <int EM, int SM, int G, int TT>
__global__ __launch_bounds__(256, (EM * SM >= 256) ? 1 : 2) void omp_fused(OmpArgs a) {
    constexpr int T = 16 * TT;
    constexpr int GPW = 64 / G;          // signal groups per wave
    constexpr int SPP = 4 * GPW;         // signals per pass of the 4 waves
    constexpr int PASSES = (T + SPP - 1) / SPP;
    constexpr int RBW = EM * G / 64;     // max 16-atom row blocks per wave in phase A

    extern __shared__ float lds[];
    __shared__ OmpItem s_it[2];
    __shared__ OmpDesc s_desc[2];

    const int tid = threadIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    // fixed LDS layout for every item: alpha0 rows of the widest dictionary, ||y||^2, signals
    float* const yn2 = lds + T * (a.max_kpad + 4);
    float* const ybuf0 = yn2 + T;
    const bool y_lds = a.y_lds != 0;

    int n_items = a.n_items;
    if (a.list_count) n_items = (*a.list_count + T - 1) / T;
    int item = blockIdx.x;
    if (item >= n_items) return;
    if (tid == 0) {
        s_it[0] = item_of<T>(a, item);
        s_desc[0] = a.desc[s_it[0].desc];
    }
    __syncthreads();
    if (y_lds && wave == 0) prefetch_signals<T>(a, s_it[0], s_desc[0].Y, ybuf0, tid & 63);

    for (int cur = 0;; cur ^= 1) {
        if (y_lds) __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0): this wave's signal copy has landed
        __syncthreads();
        // the item and its descriptor are the same for the whole group: keep them in SGPRs
        const OmpItem it = uniform_copy(s_it[cur]);
        const OmpDesc d = uniform_copy(s_desc[cur]);
        const int next = item + (int)gridDim.x;
        // the next item, requested now so that its round trips overlap phase A
        OmpItem itn{};
        if (tid == 0 && next < n_items) itn = item_of<T>(a, next);
        // lane ids made opaque per item: otherwise the compiler hoists every lane-dependent
        // address of both phases out of the item loop and keeps them all live in registers
        int lid = tid & 63;
        asm volatile("" : "+v"(lid));
        const int lane = lid;
        const int Kpad = d.Kpad;
        const int stride = Kpad + 4;           // LDS row stride (floats) of alpha0
        float* alpha = lds;                    // T x stride
        const float* ybuf = ybuf0 + cur * T * a.m;

        // ------------------------------------------------------------------ phase A
        // alpha0 = D^T y on the FP16 matrix cores from a three-term split of both operands
        // (hi*hi + hi*lo + lo*hi, FP32 accumulation).  Each atom is scaled by a power of two
        // (exact) so that its largest entry lies in [0.5, 1), and so is each signal whose largest
        // entry lies outside [2^-3, 2^14); both halves then stay in the FP16 range, the products
        // carry about 22 significant bits and the dropped lo*lo term lies below 2^-22 of the
        // largest product.  The scales are undone on the FP32 sums.
        if (y_lds) alpha0_phase<TT, RBW, true>(a, d, it, ybuf, alpha, yn2, stride, lane, wave);
        else alpha0_phase<TT, RBW, false>(a, d, it, ybuf, alpha, yn2, stride, lane, wave);
        // the next item into the other slot (its signals into the other half of the buffer)
        if (tid == 0 && next < n_items) {
            s_it[cur ^ 1] = itn;
            s_desc[cur ^ 1] = a.desc[itn.desc];
        }
        __syncthreads();
        if (y_lds && wave == 0 && next < n_items)
            prefetch_signals<T>(a, s_it[cur ^ 1], s_desc[cur ^ 1].Y, ybuf0 + (cur ^ 1) * T * a.m, lane);

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
            ctx.D = d.D;
            ctx.K = d.K;
            ctx.m = a.m;
            ctx.ystr = y_lds ? 4 * T : 4;
            // row groups of four for the final residual when every row group is 16-byte aligned
            const bool res_v4 = (a.m & 3) == 0 && (reinterpret_cast<uintptr_t>(d.D) & 15) == 0 &&
                                (y_lds || (reinterpret_cast<uintptr_t>(d.Y) & 15) == 0);
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
                ctx.marg = EXPLICIT_MARGIN * y2;
                int64_t sig = it.first + (valid ? sl : 0);
                if (a.sig_list) sig = a.sig_list[sig];
                ctx.yp = y_lds ? ybuf + 4 * (valid ? sl : 0) : d.Y + sig * (int64_t)a.m;
                st.rn2 = y2;
                st.live = valid;
                st.k = 0;
                run_steps<EM, SM, G>(st, ctx, std::make_integer_sequence<int, SM>{});
                // the residual norm from the signal and the atoms (not the downdated value)
                float rn2 = 0.f;
                if (a.res) {
                    if (res_v4) rn2 = explicit_rn2_v4<SM, EM, SM, G>(st, ctx, st.k);
                    else rn2 = explicit_rn2<SM, EM, SM, G>(st, ctx, st.k);
                }
                if (valid) {
                    if (!a.sig_list) sig += d.out0;
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
                        if (a.res) a.res[sig] = sqrtf(rn2);
                    }
                }
                __builtin_amdgcn_wave_barrier();
            }
        }
        __syncthreads();
        if (next >= n_items) break;
        item = next;
    }
}

// Dynamic LDS of one work group: alpha0 (T rows of maxKpad + 4 floats) and ||y||^2 (T floats);
// with the signal copy (y_lds) also two buffers of T signals of m floats.
template <int SM, int G, int TT>
constexpr size_t omp_lds_size(int maxKpad, int m_copy) {
    return ((size_t)16 * TT * (maxKpad + 4) + 16 * TT + (size_t)2 * 16 * TT * m_copy) * 4;
}

// Launch with a persistent grid: as many work groups as fit on the device at once (by the
// occupancy of this instantiation and its LDS), at most one per item.
template <int EM, int SM, int G, int TT>
hipError_t launch_one(const OmpArgs& a, int max_items, int n_cu, hipStream_t st) {
    const size_t lds = omp_lds_size<SM, G, TT>(a.max_kpad, a.y_lds ? a.m : 0);
    const void* fn = reinterpret_cast<const void*>(&omp_fused<EM, SM, G, TT>);
    static size_t lds_enabled = 64 * 1024;   // dynamic LDS this instantiation may request
    static size_t occ_lds = 0;               // LDS size the cached occupancy was taken at
    static int occ = 0;
    hipError_t e;
    if (lds > lds_enabled) {
        if ((e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds)) != hipSuccess) return e;
        lds_enabled = lds;
    }
    if (occ_lds != lds || occ < 1) {
        int nb = 0;
        if ((e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, 256, lds)) != hipSuccess) return e;
        occ = nb < 1 ? 1 : nb;
        occ_lds = lds;
    }
    const int grid = (int)std::min<int64_t>(std::max(max_items, 1), (int64_t)n_cu * occ);
    hipLaunchKernelGGL((omp_fused<EM, SM, G, TT>), dim3(grid), dim3(256), lds, st, a);
    return hipGetLastError();
}

}  // namespace smdl_omp

// C ABI of libsmdl: handle, workspace, argument checks, tile choice and the orchestration of
// OMP coding, MOD updates, the standard alternation and Algorithm 1 (Section 2).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <string>
#include <tuple>
#include <vector>

#include "smdl_api_internal.h"

// ------------------------------------------------------------------------------------------
// handle
// ------------------------------------------------------------------------------------------

void* smdl_ctx::ws(const char* name, size_t bytes) {
    Buf& b = bufs[name];
    if (bytes == 0) bytes = 16;
    if (b.cap >= bytes) return b.p;
    // (queued work of an asynchronous call may still use the old buffer)
    if (b.p) {
        (void)hipStreamSynchronize(stream);
        (void)hipFree(b.p);
    }
    b.p = nullptr;
    b.cap = 0;
    if (hipMalloc(&b.p, bytes) != hipSuccess) {
        (void)hipGetLastError();
        b.p = nullptr;
        return nullptr;
    }
    b.cap = bytes;
    return b.p;
}

hipError_t smdl_ctx::upload(void* dst, const void* src, size_t bytes) {
    // the bytes of copies the stream has passed are released (never while a graph is captured)
    if (!keep.empty()) {
        hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
        if (hipStreamIsCapturing(stream, &cap) == hipSuccess && cap == hipStreamCaptureStatusNone &&
            hipStreamQuery(stream) == hipSuccess)
            keep.clear();
        (void)hipGetLastError();   // the query's not-ready status is no launch error
    }
    const uint8_t* b = static_cast<const uint8_t*>(src);
    keep.emplace_back(b, b + bytes);
    return hipMemcpyAsync(dst, keep.back().data(), bytes, hipMemcpyHostToDevice, stream);
}

smdl_status smdl_ctx::fail(smdl_status s, const std::string& msg) {
    err = msg;
    return s;
}

smdl_status smdl_ctx::hip(hipError_t e, const char* what) {
    if (e == hipSuccess) return SMDL_OK;
    (void)hipGetLastError();
    return fail(SMDL_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

extern "C" int smdl_version(void) { return 10000; }

extern "C" smdl_status smdl_create(smdl_t* out, int device, void* stream) {
    if (!out) return SMDL_E_ARG;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) {
        (void)hipGetLastError();
        return SMDL_E_HIP;
    }
    if (device < 0 || device >= ndev) return SMDL_E_ARG;
    if (hipSetDevice(device) != hipSuccess) return SMDL_E_HIP;
    auto* h = new smdl_ctx();
    h->device = device;
    if (stream) {
        h->stream = static_cast<hipStream_t>(stream);
        h->own_stream = false;
    } else {
        if (hipStreamCreate(&h->stream) != hipSuccess) {
            delete h;
            return SMDL_E_HIP;
        }
        h->own_stream = true;
    }
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) == hipSuccess) h->n_cu = prop.multiProcessorCount;
    if (hipEventCreate(&h->ev0) != hipSuccess || hipEventCreate(&h->ev1) != hipSuccess) {
        delete h;
        return SMDL_E_HIP;
    }
    for (auto& ev : h->ev_prop)
        if (hipEventCreate(&ev) != hipSuccess) {
            delete h;
            return SMDL_E_HIP;
        }
    if (noalloc_setup(h) != SMDL_OK) {
        smdl_destroy(h);
        return SMDL_E_HIP;
    }
    *out = h;
    return SMDL_OK;
}

extern "C" void smdl_destroy(smdl_t h) {
    if (!h) return;
    (void)hipSetDevice(h->device);
    (void)hipStreamSynchronize(h->stream);
    for (auto& kv : h->bufs)
        if (kv.second.p) (void)hipFree(kv.second.p);
    if (h->ev0) (void)hipEventDestroy(h->ev0);
    if (h->ev1) (void)hipEventDestroy(h->ev1);
    for (auto& ev : h->ev_prop)
        if (ev) (void)hipEventDestroy(ev);
    if (h->own_stream) (void)hipStreamDestroy(h->stream);
    delete h;
}

extern "C" const char* smdl_last_error(smdl_t h) { return h ? h->err.c_str() : "null handle"; }

extern "C" smdl_status smdl_last_kernel_ms(smdl_t h, float* ms) {
    if (!h || !ms) return SMDL_E_ARG;
    if (h->timed_pending) {
        // an asynchronous call: wait for its timed launch
        (void)hipSetDevice(h->device);
        smdl_status st = h->hip(hipEventSynchronize(h->ev1), "timing");
        if (st != SMDL_OK) return st;
        finish_timing(h);
    }
    *ms = h->last_kernel_ms;
    return SMDL_OK;
}

// ------------------------------------------------------------------------------------------
// validation helpers
// ------------------------------------------------------------------------------------------

smdl_status check_dims(smdl_t h, int m, int K, int s) {
    if (m < 1 || m > SMDL_MAX_M) return h->fail(SMDL_E_SHAPE, "m must be in [1, 256]");
    if (K < 1 || K > SMDL_MAX_K) return h->fail(SMDL_E_SHAPE, "K must be in [1, 1024]");
    if (s < 1 || s > SMDL_MAX_S) return h->fail(SMDL_E_SHAPE, "sparsity must be in [1, 16]");
    if (s > m || s > K) return h->fail(SMDL_E_SHAPE, "sparsity must not exceed min(m, K)");
    return SMDL_OK;
}

smdl_status check_finite(smdl_t h, const float* x, int64_t n, const char* what) {
    if (n <= 0) return SMDL_OK;
    int32_t* bad = (int32_t*)h->ws("finite.bad", 64);
    if (!bad) return h->fail(SMDL_E_NOMEM, "workspace allocation failed");
    smdl_status st;
    if ((st = h->hip(launch_zero_i32(bad, 1, h->stream), "zero")) != SMDL_OK) return st;
    if ((st = h->hip(launch_check_finite(x, n, bad, h->stream), "finite check")) != SMDL_OK) return st;
    int32_t hb = 0;
    if ((st = h->hip(hipMemcpyAsync(&hb, bad, 4, hipMemcpyDeviceToHost, h->stream), "finite check")) != SMDL_OK) return st;
    if ((st = h->hip(hipStreamSynchronize(h->stream), "finite check")) != SMDL_OK) return st;
    if (hb) return h->fail(SMDL_E_NUMERIC, std::string(what) + " holds a non-finite value");
    return SMDL_OK;
}

smdl_status check_codes(smdl_t h, const smdl_codes& X, int64_t N, int s_needed) {
    if (N > 0 && (!X.idx || !X.coef || !X.nnz)) return h->fail(SMDL_E_ARG, "null code array");
    if (X.s_max < s_needed) return h->fail(SMDL_E_ARG, "codes.s_max smaller than the sparsity");
    if (X.s_max > SMDL_MAX_S) return h->fail(SMDL_E_SHAPE, "codes.s_max must be <= 16");
    return SMDL_OK;
}

// ------------------------------------------------------------------------------------------
// tiles
// ------------------------------------------------------------------------------------------

OmpTile default_tile(int Kpad, int s, int lanes_ok) {
    // registers per lane for U are (Kpad / lanes) * s; keep them near 128 or below
    const int cand[3] = {16, 32, 64};
    for (int lanes : cand) {
        if (Kpad % (4 * lanes) || !(lanes_ok & lanes)) continue;
        const int E = Kpad / lanes;
        const int sm = s <= 8 ? 8 : (s <= 12 ? 12 : 16);
        if (E * sm > 128 && lanes != 64) continue;
        OmpTile t{lanes, 2};
        if (E > 8) t.tt = 1;
        if (Kpad > 512) t.tt = 1;
        if (omp_tile_supported(t, Kpad, s)) return t;
        t.tt = 1;
        if (omp_tile_supported(t, Kpad, s)) return t;
    }
    return OmpTile{16, 1};
}

OmpTile choose_tile(smdl_t h, int Kpad, int s, bool batched, int lanes_ok) {
    auto it = h->tiles.find(std::make_tuple(Kpad, s, batched ? 1 : 0));
    if (it != h->tiles.end() && (it->second.lanes & lanes_ok)) return it->second;
    return default_tile(Kpad, s, lanes_ok);
}

std::vector<OmpTile> candidate_tiles(int Kpad, int s, int lanes_ok) {
    std::vector<OmpTile> out;
    for (int lanes : {16, 32, 64})
        for (int tt : {1, 2, 4}) {
            OmpTile t{lanes, tt};
            if (!(lanes & lanes_ok) || !omp_tile_supported(t, Kpad, s)) continue;
            if (omp_lds_bytes(t, Kpad, s, 0) > 96 * 1024) continue;
            out.push_back(t);
        }
    return out;
}

// ------------------------------------------------------------------------------------------
// coding of several dictionary sets in one launch
// ------------------------------------------------------------------------------------------

// Prepare (pack + Gram) the dictionaries of `sets` and build OMP descriptors/items in the
// handle's workspace.  Host-side uploads happen here, so that the launches below can be
// captured into a graph.
smdl_status prepare_sets(smdl_t h, int m, std::vector<SetSpec>& sets, const char* tag,
                         CodePlan& plan) {
    const int mpad = pad64(m);
    plan.m = m;
    plan.mchunks = mpad / 64;
    plan.n_sets = (int)sets.size();
    plan.maxKpad = 0;
    plan.maxS = 0;
    size_t frag_total = 0, gram_total = 0;
    plan.lanes_ok = 16 | 32 | 64;
    for (auto& s : sets) {
        s.Kpad = pad64(s.K);
        plan.maxKpad = std::max(plan.maxKpad, s.Kpad);
        plan.maxS = std::max(plan.maxS, s.s);
        for (int lanes : {16, 32, 64})
            if (s.Kpad % (4 * lanes)) plan.lanes_ok &= ~lanes;
        frag_total += (size_t)mpad * s.Kpad;
    }
    const int gld = gram_ld(plan.maxKpad);
    for (auto& s : sets) {
        s.gld = gld;
        gram_total += (size_t)s.Kpad * gld;
    }
    std::string t(tag);
    size_t kpad_total = 0;
    for (auto& s : sets) kpad_total += (size_t)s.Kpad;
    float* frag = (float*)h->ws((t + ".frag").c_str(), frag_total * 4);
    float* gram = (float*)h->ws((t + ".gram").c_str(), gram_total * 4);
    uint16_t* f16 = (uint16_t*)h->ws((t + ".f16").c_str(), frag_total * 2 * 2);   // hi and lo halves
    int32_t* aexp = (int32_t*)h->ws((t + ".aexp").c_str(), kpad_total * 4);
    if (!frag || !gram || !f16 || !aexp) return h->fail(SMDL_E_NOMEM, "workspace allocation failed");
    std::vector<PackDesc> pd(sets.size());
    std::vector<GramDesc> gd(sets.size());
    std::vector<OmpDesc> od(sets.size());
    size_t fo = 0, go = 0, ko = 0;
    for (size_t i = 0; i < sets.size(); ++i) {
        auto& s = sets[i];
        s.frag = reinterpret_cast<float4*>(frag + fo);
        s.gram = gram + go;
        uint16_t* fhi = f16 + 2 * fo;
        uint16_t* flo = fhi + (size_t)mpad * s.Kpad;
        int32_t* ae = aexp + ko;
        fo += (size_t)mpad * s.Kpad;
        go += (size_t)s.Kpad * s.gld;
        ko += (size_t)s.Kpad;
        pd[i] = PackDesc{s.D, s.frag, fhi, flo, ae, s.K, s.Kpad};
        gd[i] = GramDesc{s.frag, s.gram, s.Kpad, s.gld};
        od[i] = OmpDesc{s.D, fhi, flo, ae, s.gram, s.Y, s.n, s.out0, s.K, s.Kpad, s.s, s.gld};
    }
    plan.pack_desc = h->ws((t + ".pd").c_str(), pd.size() * sizeof(PackDesc));
    plan.gram_desc = h->ws((t + ".gd").c_str(), gd.size() * sizeof(GramDesc));
    plan.omp_desc = (OmpDesc*)h->ws((t + ".od").c_str(), od.size() * sizeof(OmpDesc));
    if (!plan.pack_desc || !plan.gram_desc || !plan.omp_desc)
        return h->fail(SMDL_E_NOMEM, "workspace allocation failed");
    smdl_status st;
    if ((st = h->hip(h->upload(plan.pack_desc, pd.data(), pd.size() * sizeof(PackDesc)), "upload")) != SMDL_OK) return st;
    if ((st = h->hip(h->upload(plan.gram_desc, gd.data(), gd.size() * sizeof(GramDesc)), "upload")) != SMDL_OK) return st;
    if ((st = h->hip(h->upload(plan.omp_desc, od.data(), od.size() * sizeof(OmpDesc)), "upload")) != SMDL_OK) return st;
    plan.host_desc = od;
    plan.queue = (int*)h->ws((t + ".queue").c_str(), 64);
    if (!plan.queue) return h->fail(SMDL_E_NOMEM, "workspace allocation failed");
    return SMDL_OK;
}

// Work items of T signals for every set, heaviest (K * s) first.
smdl_status build_items(smdl_t h, const std::vector<SetSpec>& sets, int T, const char* tag,
                        CodePlan& plan) {
    std::vector<int> order(sets.size());
    for (size_t i = 0; i < sets.size(); ++i) order[i] = (int)i;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
        return (int64_t)sets[a].Kpad * sets[a].s > (int64_t)sets[b].Kpad * sets[b].s;
    });
    std::vector<OmpItem> items;
    for (int i : order)
        for (int64_t f = 0; f < sets[i].n; f += T)
            items.push_back(OmpItem{i, (int32_t)std::min<int64_t>(T, sets[i].n - f), f});
    plan.n_items = (int)items.size();
    plan.T = T;
    std::string t(tag);
    plan.items = (OmpItem*)h->ws((t + ".items").c_str(), std::max<size_t>(1, items.size()) * sizeof(OmpItem));
    if (!plan.items) return h->fail(SMDL_E_NOMEM, "workspace allocation failed");
    if (!items.empty())
        return h->hip(h->upload(plan.items, items.data(), items.size() * sizeof(OmpItem)), "upload");
    return SMDL_OK;
}

// Whether the OMP launch of `plan` with `tile` can copy the signals into LDS ahead of use.
static bool plan_y_lds(const CodePlan& plan, OmpTile tile) {
    std::vector<const float*> ys;
    for (const auto& d : plan.host_desc) ys.push_back(d.Y);
    return omp_y_lds(tile, plan.maxKpad, plan.maxS, plan.m, ys.data(), (int)ys.size());
}

// Queue pack + Gram + OMP for all sets (no host synchronisation; graph-capturable).
hipError_t enqueue_code(smdl_t h, const CodePlan& plan, OmpTile tile, const CodeOut& out,
                        float eps, bool timed) {
    hipError_t e;
    if (!(tile.lanes & plan.lanes_ok)) return hipErrorInvalidValue;   // E = Kpad/lanes must be a multiple of 4
    if ((e = launch_pack_dict_m(plan.pack_desc, plan.n_sets, plan.maxKpad, plan.m, plan.mchunks,
                                h->stream)) != hipSuccess) return e;
    if ((e = launch_gram_batched(plan.gram_desc, plan.n_sets, plan.maxKpad, plan.mchunks,
                                 h->stream)) != hipSuccess) return e;
    OmpArgs a{};
    a.desc = plan.omp_desc;
    a.items = plan.items;
    a.n_items = plan.n_items;
    a.queue = plan.queue;
    a.max_kpad = plan.maxKpad;
    a.y_lds = plan_y_lds(plan, tile) ? 1 : 0;
    a.m = plan.m;
    a.mchunks = plan.mchunks;
    a.eps2 = eps > 0.f ? eps * eps : 0.f;
    a.tau = SMDL_TAU;
    a.dep_tol = SMDL_DEP_TOL;
    a.idx = out.idx;
    a.coef = out.coef;
    a.nnz = out.nnz;
    a.res = out.res;
    a.s_out = out.s_stride;
    if (plan.n_items < 1) return hipSuccess;
    if (timed) (void)hipEventRecord(h->ev0, h->stream);
    e = launch_omp(tile, plan.maxKpad, plan.maxS, a, plan.n_items, h->n_cu, h->stream);
    if (timed) (void)hipEventRecord(h->ev1, h->stream);
    return e;
}

// ------------------------------------------------------------------------------------------
// entry points: gram, omp
// ------------------------------------------------------------------------------------------

extern "C" smdl_status smdl_gram(smdl_t h, const float* D, int m, int K, float* G) {
    if (!h) return SMDL_E_ARG;
    h->err.clear();
    if (!D || !G) return h->fail(SMDL_E_ARG, "null pointer");
    smdl_status st = check_dims(h, m, K, 1);
    if (st != SMDL_OK) return st;
    (void)hipSetDevice(h->device);
    std::vector<SetSpec> sets(1);
    sets[0].D = D;
    sets[0].K = K;
    sets[0].s = 1;
    sets[0].Y = nullptr;
    sets[0].n = 0;
    CodePlan plan;
    if ((st = prepare_sets(h, m, sets, "gram", plan)) != SMDL_OK) return st;
    if ((st = h->hip(launch_pack_dict_m(plan.pack_desc, 1, plan.maxKpad, m, plan.mchunks, h->stream),
                     "pack")) != SMDL_OK) return st;
    if ((st = h->hip(launch_gram_batched(plan.gram_desc, 1, plan.maxKpad, plan.mchunks, h->stream),
                     "gram")) != SMDL_OK) return st;
    const int ld = sets[0].gld;
    if ((st = h->hip(hipMemcpy2DAsync(G, (size_t)K * 4, sets[0].gram, (size_t)ld * 4, (size_t)K * 4, K,
                                      hipMemcpyDeviceToDevice, h->stream), "copy")) != SMDL_OK) return st;
    if (h->flags & SMDL_ASYNC) return SMDL_OK;
    return h->hip(hipStreamSynchronize(h->stream), "gram");
}

smdl_status omp_code_impl(smdl_t h, const float* D, int m, int K, const float* Y, int64_t N,
                          int s_max, float eps, smdl_codes X, float* res_norm, const int32_t* sig_list,
                          const int32_t* list_count, int64_t list_cap, const char* tag) {
    std::vector<SetSpec> sets(1);
    sets[0].D = D;
    sets[0].K = K;
    sets[0].s = s_max;
    sets[0].Y = Y;
    sets[0].n = sig_list ? list_cap : N;
    sets[0].out0 = 0;
    CodePlan plan;
    smdl_status st;
    if ((st = prepare_sets(h, m, sets, tag, plan)) != SMDL_OK) return st;
    if (h->autotune && !sig_list && N >= 4096) {
        // first call of this shape: time the candidate tiles on this data (codes are rewritten below)
        CodeOut tout{X.idx, X.coef, X.nnz, nullptr, X.s_max};
        plan.persistent = false;
        if ((st = autotune_plan(h, plan, sets, tout, false, tag)) != SMDL_OK) return st;
    }
    const OmpTile tile = choose_tile(h, plan.maxKpad, s_max, false);
    const int T = 16 * tile.tt;
    hipError_t e;
    if ((e = launch_pack_dict_m(plan.pack_desc, 1, plan.maxKpad, m, plan.mchunks, h->stream)) != hipSuccess)
        return h->hip(e, "pack");
    if ((e = launch_gram_batched(plan.gram_desc, 1, plan.maxKpad, plan.mchunks, h->stream)) != hipSuccess)
        return h->hip(e, "gram");
    OmpArgs a{};
    a.desc = plan.omp_desc;
    a.items = nullptr;
    a.n_items = (int)((sets[0].n + T - 1) / T);
    a.queue = plan.queue;
    a.max_kpad = plan.maxKpad;
    a.y_lds = plan_y_lds(plan, tile) ? 1 : 0;
    a.sig_list = sig_list;
    a.list_count = list_count;
    a.m = m;
    a.mchunks = plan.mchunks;
    a.eps2 = eps > 0.f ? eps * eps : 0.f;
    a.tau = SMDL_TAU;
    a.dep_tol = SMDL_DEP_TOL;
    a.idx = X.idx;
    a.coef = X.coef;
    a.nnz = X.nnz;
    a.res = res_norm;
    a.s_out = X.s_max;
    if (a.n_items < 1) return SMDL_OK;
    (void)hipEventRecord(h->ev0, h->stream);
    e = launch_omp(tile, plan.maxKpad, s_max, a, a.n_items, h->n_cu, h->stream);
    (void)hipEventRecord(h->ev1, h->stream);
    if (e != hipSuccess) return h->hip(e, "omp launch");
    h->timed_pending = true;
    return SMDL_OK;
}

smdl_status finish_timing(smdl_t h) {
    if (h->timed_pending) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, h->ev0, h->ev1) == hipSuccess) h->last_kernel_ms = ms;
        (void)hipGetLastError();
        h->timed_pending = false;
    }
    return SMDL_OK;
}

extern "C" smdl_status smdl_omp_code(smdl_t h, const float* D, int m, int K, const float* Y, int64_t N,
                                     int s_max, float eps, smdl_codes X, float* res_norm) {
    if (!h) return SMDL_E_ARG;
    h->err.clear();
    smdl_status st = check_dims(h, m, K, s_max);
    if (st != SMDL_OK) return st;
    if (N < 0) return h->fail(SMDL_E_ARG, "N must be >= 0");
    if (!(eps >= 0.f) || std::isinf(eps)) return h->fail(SMDL_E_ARG, "eps must be finite and >= 0");
    if ((st = check_codes(h, X, N, s_max)) != SMDL_OK) return st;
    if (N == 0) return SMDL_OK;
    if (!D || !Y) return h->fail(SMDL_E_ARG, "null pointer");
    if (N > (int64_t)INT32_MAX * 16) return h->fail(SMDL_E_SHAPE, "N too large");
    (void)hipSetDevice(h->device);
    if ((h->flags & SMDL_CHECK_FINITE) &&
        ((st = check_finite(h, D, (int64_t)K * m, "D")) != SMDL_OK || (st = check_finite(h, Y, N * m, "Y")) != SMDL_OK))
        return st;
    if ((st = omp_code_impl(h, D, m, K, Y, N, s_max, eps, X, res_norm, nullptr, nullptr, 0, "omp")) != SMDL_OK)
        return st;
    if (h->flags & SMDL_ASYNC) return SMDL_OK;   // timing read later by smdl_last_kernel_ms
    st = h->hip(hipStreamSynchronize(h->stream), "omp");
    finish_timing(h);
    return st;
}

// ------------------------------------------------------------------------------------------
// MOD
// ------------------------------------------------------------------------------------------

smdl_status prepare_mod(smdl_t h, int m, const std::vector<ModSpec>& specs, const char* tag,
                        ModPlan& plan, bool fixed_order) {
    std::string t(tag);
    int64_t total_atoms = 0, entries = 0, max_n = 0;
    size_t abytes = 0;
    plan.maxKpad = 0;
    for (auto& s : specs) {
        const int Kp = pad64(s.K);
        total_atoms += s.K;
        entries += s.n * s.s_stride;
        max_n = std::max(max_n, s.n);
        abytes += (size_t)(Kp + m) * Kp * 8;
        plan.maxKpad = std::max(plan.maxKpad, Kp);
    }
    plan.total_atoms = (int)total_atoms;
    plan.max_n = max_n;
    plan.n_desc = (int)specs.size();
    plan.m = m;
    plan.solver = h->mod_solver;
    double* A = (double*)h->ws((t + ".A").c_str(), abytes);
    double* W = (double*)h->ws((t + ".W").c_str(), abytes);
    size_t ldbytes = 0;
    for (auto& s : specs) ldbytes += (size_t)pad64(s.K) * 32 * 8;
    double* Ld = (double*)h->ws((t + ".Ld").c_str(), ldbytes);
    plan.cnt = (int32_t*)h->ws((t + ".cnt").c_str(), (total_atoms + 1) * 4);
    plan.fill = (int32_t*)h->ws((t + ".fill").c_str(), (total_atoms + 1) * 4);
    plan.ptr = (int32_t*)h->ws((t + ".ptr").c_str(), (total_atoms + 1) * 4);
    plan.list_sig = (int32_t*)h->ws((t + ".ls").c_str(), std::max<int64_t>(1, entries) * 4);
    plan.list_coef = (float*)h->ws((t + ".lc").c_str(), std::max<int64_t>(1, entries) * 4);
    plan.status = (int32_t*)h->ws((t + ".status").c_str(), 8 * specs.size() * 4);
    plan.desc = (ModDesc*)h->ws((t + ".md").c_str(), specs.size() * sizeof(ModDesc));
    // products: about 512 list entries per block; long lists (many signals per atom) are split
    int64_t per_atom = 0;
    for (auto& s : specs) per_atom = std::max<int64_t>(per_atom, (s.n * s.s_stride + s.K - 1) / s.K);
    plan.chunks = (int)std::min<int64_t>(16, std::max<int64_t>(1, (per_atom + 511) / 512));
    plan.arena = A;
    plan.arena_len = (int64_t)(abytes / 8);
    plan.part = plan.chunks > 1 ? (double*)h->ws((t + ".part").c_str(), abytes * (plan.chunks - 1)) : nullptr;
    if (fixed_order) {
        const size_t nb = (size_t)mod_csc_blocks(max_n) * (size_t)std::max<int64_t>(1, total_atoms) * 4;
        plan.bcnt = (int32_t*)h->ws((t + ".bcnt").c_str(), nb);
        plan.bbase = (int32_t*)h->ws((t + ".bbase").c_str(), nb);
        if (!plan.bcnt || !plan.bbase) return h->fail(SMDL_E_NOMEM, "workspace allocation failed");
    }
    if (!A || !W || !Ld || !plan.cnt || !plan.fill || !plan.ptr || !plan.list_sig || !plan.list_coef ||
        !plan.status || !plan.desc || (plan.chunks > 1 && !plan.part))
        return h->fail(SMDL_E_NOMEM, "workspace allocation failed");
    std::vector<ModDesc> md(specs.size());
    size_t ao = 0, lo = 0;
    int64_t atom0 = 0;
    for (size_t i = 0; i < specs.size(); ++i) {
        const auto& s = specs[i];
        const int Kp = pad64(s.K);
        md[i] = ModDesc{s.Y, s.idx, s.coef, s.nnz, s.n, atom0, s.D, A + ao, W + ao, Ld + lo, s.K, Kp, s.s_stride, 0};
        ao += (size_t)(Kp + m) * Kp;
        lo += (size_t)Kp * 32;
        atom0 += s.K;
    }
    plan.host_desc = md;
    smdl_status st = h->hip(h->upload(plan.desc, md.data(), md.size() * sizeof(ModDesc)), "upload");
    if (st != SMDL_OK) return st;
    return h->hip(launch_zero_i32(plan.status, 8 * (int64_t)specs.size(), h->stream), "zero");
}

hipError_t enqueue_mod(smdl_t h, const ModPlan& plan) {
    return launch_mod(plan.desc, plan.n_desc, plan.m, plan.total_atoms, plan.max_n, plan.cnt, plan.fill, plan.ptr,
                      plan.list_sig, plan.list_coef, plan.status, plan.maxKpad, plan.arena, plan.part,
                      plan.arena_len, plan.chunks, plan.solver, plan.bcnt, plan.bbase, h->stream);
}

// Read the MOD status array; returns SMDL_E_NUMERIC / SMDL_E_ARG on failures.
smdl_status read_mod_status(smdl_t h, const ModPlan& plan, std::vector<int32_t>* st_out) {
    std::vector<int32_t> st(8 * plan.n_desc);
    smdl_status s = h->hip(hipMemcpyAsync(st.data(), plan.status, st.size() * 4, hipMemcpyDeviceToHost,
                                          h->stream), "status");
    if (s != SMDL_OK) return s;
    if ((s = h->hip(hipStreamSynchronize(h->stream), "mod")) != SMDL_OK) return s;
    if (st_out) *st_out = st;
    for (int i = 0; i < plan.n_desc; ++i) {
        if (st[8 * i + 3]) return h->fail(SMDL_E_ARG, "codes hold an atom index outside [0, K) or nnz outside [0, s_max]");
        if (st[8 * i + 2]) return h->fail(SMDL_E_NUMERIC, "FP64 Cholesky of X X^T failed after the ridge retry");
    }
    return SMDL_OK;
}

extern "C" smdl_status smdl_mod_update(smdl_t h, const float* Y, int m, int64_t N, smdl_codes X, int K,
                                       float* D, int32_t* n_unused) {
    if (!h) return SMDL_E_ARG;
    h->err.clear();
    smdl_status st = check_dims(h, m, K, 1);
    if (st != SMDL_OK) return st;
    if (N < 0) return h->fail(SMDL_E_ARG, "N must be >= 0");
    if (X.s_max < 1 || X.s_max > SMDL_MAX_S) return h->fail(SMDL_E_SHAPE, "codes.s_max must be in [1, 16]");
    if (!D || (N > 0 && (!Y || !X.idx || !X.coef || !X.nnz))) return h->fail(SMDL_E_ARG, "null pointer");
    if (N * X.s_max > INT32_MAX) return h->fail(SMDL_E_SHAPE, "too many code entries");
    (void)hipSetDevice(h->device);
    if ((h->flags & SMDL_CHECK_FINITE) && (st = check_finite(h, Y, N * m, "Y")) != SMDL_OK) return st;
    std::vector<ModSpec> specs(1);
    specs[0] = ModSpec{Y, X.idx, X.coef, X.nnz, N, D, K, X.s_max};
    ModPlan plan;
    if ((st = prepare_mod(h, m, specs, "mod", plan, (h->flags & SMDL_DETERMINISTIC) != 0)) != SMDL_OK) return st;
    if ((st = h->hip(enqueue_mod(h, plan), "mod launch")) != SMDL_OK) return st;
    std::vector<int32_t> s4;
    st = read_mod_status(h, plan, &s4);
    if (n_unused) *n_unused = s4.empty() ? 0 : s4[0];
    return st;
}

// ------------------------------------------------------------------------------------------
// learning
// ------------------------------------------------------------------------------------------

// Time every candidate tile on one coding pass of `plan` and keep the fastest.
smdl_status autotune_plan(smdl_t h, CodePlan& plan, std::vector<SetSpec>& sets, const CodeOut& out,
                          bool batched, const char* tag) {
    auto key = std::make_tuple(plan.maxKpad, plan.maxS, batched ? 1 : 0);
    auto found = h->tiles.find(key);
    if (found != h->tiles.end() && (found->second.lanes & plan.lanes_ok)) return SMDL_OK;
    float best = 1e30f;
    OmpTile bt = default_tile(plan.maxKpad, plan.maxS, plan.lanes_ok);
    for (OmpTile t : candidate_tiles(plan.maxKpad, plan.maxS, plan.lanes_ok)) {
        smdl_status st = build_items(h, sets, 16 * t.tt, tag, plan);
        if (st != SMDL_OK) return st;
        float tot = 0.f;
        for (int rep = 0; rep < 3; ++rep) {
            hipError_t e = enqueue_code(h, plan, t, out, 0.f, true);
            if (e != hipSuccess) return h->hip(e, "autotune launch");
            if ((st = h->hip(hipStreamSynchronize(h->stream), "autotune")) != SMDL_OK) return st;
            float ms = 0.f;
            (void)hipEventElapsedTime(&ms, h->ev0, h->ev1);
            if (rep > 0) tot += ms;
        }
        if (tot < best) {
            best = tot;
            bt = t;
        }
    }
    h->tiles[key] = bt;
    return SMDL_OK;
}

// The standard alternation on every set at once.  sets[i].D receives the dictionary; the
// final codes (if want_codes) go to `out` rows sets[i].out0 ...
smdl_status learn_sets(smdl_t h, int m, std::vector<SetSpec>& sets, int iters, const CodeOut& out,
                       bool want_codes, uint32_t flags, const char* tag) {
    smdl_status st;
    std::string t(tag);
    // 1. initialisation: first K columns of every set
    {
        std::vector<InitDesc> idd(sets.size());
        int maxK = 0;
        for (size_t i = 0; i < sets.size(); ++i) {
            idd[i] = InitDesc{sets[i].init ? sets[i].init : sets[i].Y, const_cast<float*>(sets[i].D), sets[i].K, 0};
            maxK = std::max(maxK, sets[i].K);
        }
        void* dd = h->ws((t + ".init").c_str(), idd.size() * sizeof(InitDesc));
        if (!dd) return h->fail(SMDL_E_NOMEM, "workspace allocation failed");
        if ((st = h->hip(h->upload(dd, idd.data(), idd.size() * sizeof(InitDesc)), "upload")) != SMDL_OK) return st;
        if ((st = h->hip(launch_init_from_columns_batched(dd, (int)sets.size(), maxK, m, h->stream), "init")) != SMDL_OK)
            return st;
    }
    const bool per_set = (flags & SMDL_PER_SUBSET_LAUNCH) != 0;
    const bool use_graph = (flags & SMDL_NO_GRAPH) == 0;
    std::vector<CodePlan> cplans;
    std::vector<ModPlan> mplans;
    std::vector<OmpTile> tiles;
    std::vector<std::vector<SetSpec>> groups;
    if (per_set) {
        for (auto& s : sets) groups.push_back(std::vector<SetSpec>{s});
    } else {
        groups.push_back(sets);
    }
    cplans.resize(groups.size());
    mplans.resize(groups.size());
    tiles.resize(groups.size());
    for (size_t gi = 0; gi < groups.size(); ++gi) {
        std::string gt = t + (per_set ? std::to_string(gi) : std::string("b"));
        if ((st = prepare_sets(h, m, groups[gi], gt.c_str(), cplans[gi])) != SMDL_OK) return st;
        cplans[gi].persistent = !per_set && groups[gi].size() > 1;
        std::vector<ModSpec> ms;
        for (auto& s : groups[gi]) {
            ModSpec x;
            x.Y = s.Y;
            x.idx = out.idx + s.out0 * out.s_stride;
            x.coef = out.coef + s.out0 * out.s_stride;
            x.nnz = out.nnz + s.out0;
            x.n = s.n;
            x.D = const_cast<float*>(s.D);
            x.K = s.K;
            x.s_stride = out.s_stride;
            ms.push_back(x);
        }
        if ((st = prepare_mod(h, m, ms, (gt + "m").c_str(), mplans[gi], (flags & SMDL_DETERMINISTIC) != 0)) != SMDL_OK)
            return st;
        if (h->autotune && !per_set &&
            (st = autotune_plan(h, cplans[gi], groups[gi], out, cplans[gi].persistent, gt.c_str())) != SMDL_OK)
            return st;
        tiles[gi] = choose_tile(h, cplans[gi].maxKpad, cplans[gi].maxS, cplans[gi].persistent, cplans[gi].lanes_ok);
        if ((st = build_items(h, groups[gi], 16 * tiles[gi].tt, gt.c_str(), cplans[gi])) != SMDL_OK) return st;
    }
    // the initialisation wrote D into the sets' buffers; autotuning above coded with it (harmless)
    auto one_iteration = [&]() -> hipError_t {
        for (size_t gi = 0; gi < groups.size(); ++gi) {
            hipError_t e = enqueue_code(h, cplans[gi], tiles[gi], out, 0.f, false);
            if (e != hipSuccess) return e;
            e = enqueue_mod(h, mplans[gi]);
            if (e != hipSuccess) return e;
        }
        return hipSuccess;
    };
    if (iters > 0) {
        if (use_graph) {
            hipGraph_t graph = nullptr;
            hipGraphExec_t exec = nullptr;
            if ((st = h->hip(hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal), "capture")) != SMDL_OK)
                return st;
            hipError_t e = one_iteration();
            hipError_t e2 = hipStreamEndCapture(h->stream, &graph);
            if (e != hipSuccess) {
                if (graph) (void)hipGraphDestroy(graph);
                return h->hip(e, "capture launch");
            }
            if ((st = h->hip(e2, "end capture")) != SMDL_OK) return st;
            if ((st = h->hip(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0), "instantiate")) != SMDL_OK) {
                (void)hipGraphDestroy(graph);
                return st;
            }
            for (int it = 0; it < iters && st == SMDL_OK; ++it)
                st = h->hip(hipGraphLaunch(exec, h->stream), "graph launch");
            (void)hipStreamSynchronize(h->stream);
            (void)hipGraphExecDestroy(exec);
            (void)hipGraphDestroy(graph);
            if (st != SMDL_OK) return st;
        } else {
            for (int it = 0; it < iters; ++it)
                if ((st = h->hip(one_iteration(), "iteration")) != SMDL_OK) return st;
        }
    }
    if (want_codes) {
        for (size_t gi = 0; gi < groups.size(); ++gi) {
            hipError_t e = enqueue_code(h, cplans[gi], tiles[gi], out, 0.f, false);
            if (e != hipSuccess) return h->hip(e, "final coding");
        }
    }
    for (size_t gi = 0; gi < groups.size(); ++gi)
        if (iters > 0 && (st = read_mod_status(h, mplans[gi], nullptr)) != SMDL_OK) return st;
    return h->hip(hipStreamSynchronize(h->stream), "learn");
}

static smdl_status learn_impl(smdl_t h, const float* Y, int m, int64_t N, int K, int s, int iters,
                              const float* D_init, float* D_out, smdl_codes X_out) {
    if (!h) return SMDL_E_ARG;
    h->err.clear();
    smdl_status st = check_dims(h, m, K, s);
    if (st != SMDL_OK) return st;
    if (iters < 0) return h->fail(SMDL_E_ARG, "iters must be >= 0");
    if (!D_init && N < K) return h->fail(SMDL_E_ARG, "need at least K signals (initialisation uses the first K)");
    if (N < 1) return h->fail(SMDL_E_ARG, "N must be >= 1");
    if (!Y || !D_out) return h->fail(SMDL_E_ARG, "null pointer");
    if (X_out.idx && (st = check_codes(h, X_out, N, s)) != SMDL_OK) return st;
    if (N * 16 > INT32_MAX) return h->fail(SMDL_E_SHAPE, "N too large for one data set");
    (void)hipSetDevice(h->device);
    if ((h->flags & SMDL_CHECK_FINITE) && (st = check_finite(h, Y, N * m, "Y")) != SMDL_OK) return st;
    CodeOut out;
    if (X_out.idx) {
        out = CodeOut{X_out.idx, X_out.coef, X_out.nnz, nullptr, X_out.s_max};
    } else {
        out.s_stride = s;
        out.idx = (int32_t*)h->ws("learn.idx", (size_t)N * s * 4);
        out.coef = (float*)h->ws("learn.coef", (size_t)N * s * 4);
        out.nnz = (int32_t*)h->ws("learn.nnz", (size_t)N * 4);
        out.res = nullptr;
        if (!out.idx || !out.coef || !out.nnz) return h->fail(SMDL_E_NOMEM, "workspace allocation failed");
    }
    std::vector<SetSpec> sets(1);
    sets[0].Y = Y;
    sets[0].init = D_init;
    sets[0].n = N;
    sets[0].K = K;
    sets[0].s = s;
    sets[0].D = D_out;
    sets[0].out0 = 0;
    return learn_sets(h, m, sets, iters, out, X_out.idx != nullptr, h->flags & SMDL_DETERMINISTIC, "learn");
}

extern "C" smdl_status smdl_learn(smdl_t h, const float* Y, int m, int64_t N, int K, int s, int iters,
                                  float* D_out, smdl_codes X_out) {
    return learn_impl(h, Y, m, N, K, s, iters, nullptr, D_out, X_out);
}

extern "C" smdl_status smdl_learn_init(smdl_t h, const float* Y, int m, int64_t N, int K, int s, int iters,
                                       const float* D_init, float* D_out, smdl_codes X_out) {
    if (h && !D_init) return h->fail(SMDL_E_ARG, "null initial dictionary");
    return learn_impl(h, Y, m, N, K, s, iters, D_init, D_out, X_out);
}

extern "C" smdl_status smdl_split_merge_learn(smdl_t h, const float* Y, int m, int64_t N,
                                              const smdl_subsets* sub, int K, const smdl_learn_opts* o,
                                              float* D_out, smdl_codes X_out, float* D_local_out,
                                              double* scales_out) {
    if (!h) return SMDL_E_ARG;
    h->err.clear();
    if (!sub || !o || !Y || !D_out) return h->fail(SMDL_E_ARG, "null pointer");
    smdl_status st;
    if ((st = check_dims(h, m, K, o->s_merge)) != SMDL_OK) return st;
    if ((st = check_dims(h, m, K, o->s_final)) != SMDL_OK) return st;
    const int L = sub->L;
    if (L < 1 || !sub->offsets || !sub->K_local || !sub->s_local) return h->fail(SMDL_E_ARG, "bad subsets");
    if (sub->offsets[0] != 0 || sub->offsets[L] != N) return h->fail(SMDL_E_ARG, "offsets must run from 0 to N");
    if (o->iters_local < 0 || o->iters_merge < 0) return h->fail(SMDL_E_ARG, "iterations must be >= 0");
    int64_t sumK = 0;
    int s_loc_max = 1;
    for (int t = 0; t < L; ++t) {
        const int64_t n = sub->offsets[t + 1] - sub->offsets[t];
        if ((st = check_dims(h, m, sub->K_local[t], sub->s_local[t])) != SMDL_OK) return st;
        if (!o->D_local_init && n < sub->K_local[t]) return h->fail(SMDL_E_ARG, "every subset needs at least K_local signals");
        if (n < 1) return h->fail(SMDL_E_ARG, "every subset needs at least one signal");
        if (n * 16 > INT32_MAX) return h->fail(SMDL_E_SHAPE, "subset too large");
        sumK += sub->K_local[t];
        s_loc_max = std::max(s_loc_max, (int)sub->s_local[t]);
    }
    if (sumK < K) return h->fail(SMDL_E_ARG, "the pooled local atoms must number at least K");
    if (sumK * 16 > INT32_MAX) return h->fail(SMDL_E_SHAPE, "too many pooled atoms");
    const uint32_t flags = o->flags | h->flags;
    const bool compose = (flags & SMDL_COMPOSE_CODES) != 0;
    if (X_out.idx && !compose && (st = check_codes(h, X_out, N, o->s_final)) != SMDL_OK) return st;
    if (o->X_local.idx) {
        if (!o->X_local.coef || !o->X_local.nnz) return h->fail(SMDL_E_ARG, "null local code array");
        if (o->X_local.s_max < s_loc_max || o->X_local.s_max > SMDL_MAX_S)
            return h->fail(SMDL_E_ARG, "X_local.s_max must be in [max s_local, 16]");
    }
    if (X_out.idx && compose) {
        if (!X_out.coef || !X_out.nnz) return h->fail(SMDL_E_ARG, "null code array");
        if (s_loc_max * o->s_merge > SMDL_MAX_COMPOSED)
            return h->fail(SMDL_E_SHAPE, "composed codes need s_local * s_merge <= 64");
        if (X_out.s_max < s_loc_max * o->s_merge || X_out.s_max > SMDL_MAX_COMPOSED)
            return h->fail(SMDL_E_ARG, "composed codes need s_local * s_merge <= codes.s_max <= 64");
    }
    (void)hipSetDevice(h->device);
    if ((flags & SMDL_CHECK_FINITE) && (st = check_finite(h, Y, N * m, "Y")) != SMDL_OK) return st;

    // step 1: the subsets as contiguous blocks of a permuted copy of Y
    const float* Yp = Y;
    if (sub->perm) {
        float* buf = (float*)h->ws("sm.Yp", (size_t)N * m * 4);
        if (!buf) return h->fail(SMDL_E_NOMEM, "workspace allocation failed");
        int32_t* bad = (int32_t*)h->ws("sm.bad", 64);
        if (!bad) return h->fail(SMDL_E_NOMEM, "workspace allocation failed");
        if ((st = h->hip(launch_zero_i32(bad, 1, h->stream), "zero")) != SMDL_OK) return st;
        if ((st = h->hip(launch_gather_columns(Y, sub->perm, N, N, m, buf, bad, h->stream), "gather")) != SMDL_OK) return st;
        int32_t hbad = 0;
        if ((st = h->hip(hipMemcpyAsync(&hbad, bad, 4, hipMemcpyDeviceToHost, h->stream), "check")) != SMDL_OK) return st;
        if ((st = h->hip(hipStreamSynchronize(h->stream), "gather")) != SMDL_OK) return st;
        if (hbad) return h->fail(SMDL_E_ARG, "perm holds an index outside [0, N)");
        Yp = buf;
    }
    float* Dloc = D_local_out ? D_local_out : (float*)h->ws("sm.Dloc", (size_t)sumK * m * 4);
    CodeOut lc;
    lc.s_stride = s_loc_max;
    lc.idx = (int32_t*)h->ws("sm.idx", (size_t)N * s_loc_max * 4);
    lc.coef = (float*)h->ws("sm.coef", (size_t)N * s_loc_max * 4);
    lc.nnz = (int32_t*)h->ws("sm.nnz", (size_t)N * 4);
    lc.res = nullptr;
    double* scales = (double*)h->ws("sm.scales", (size_t)L * 8);
    int64_t* offs_dev = (int64_t*)h->ws("sm.offs", (size_t)(L + 1) * 8);
    int64_t* aoff_dev = (int64_t*)h->ws("sm.aoff", (size_t)(L + 1) * 8);
    float* Ytil = (float*)h->ws("sm.Ytil", (size_t)sumK * m * 4);
    if (!Dloc || !lc.idx || !lc.coef || !lc.nnz || !scales || !offs_dev || !aoff_dev || !Ytil)
        return h->fail(SMDL_E_NOMEM, "workspace allocation failed");
    std::vector<int64_t> aoff(L + 1, 0);
    for (int t = 0; t < L; ++t) aoff[t + 1] = aoff[t] + sub->K_local[t];
    if ((st = h->hip(h->upload(offs_dev, sub->offsets, (L + 1) * 8), "upload")) != SMDL_OK)
        return st;
    if ((st = h->hip(h->upload(aoff_dev, aoff.data(), (L + 1) * 8), "upload")) != SMDL_OK)
        return st;

    // step 2: local dictionaries
    std::vector<SetSpec> sets(L);
    for (int t = 0; t < L; ++t) {
        sets[t].Y = Yp + sub->offsets[t] * m;
        sets[t].init = o->D_local_init;
        sets[t].n = sub->offsets[t + 1] - sub->offsets[t];
        sets[t].K = sub->K_local[t];
        sets[t].s = sub->s_local[t];
        sets[t].D = Dloc + aoff[t] * m;
        sets[t].out0 = sub->offsets[t];
    }
    auto t0 = std::chrono::steady_clock::now();
    if ((st = learn_sets(h, m, sets, o->iters_local, lc, true, flags, "sm.loc")) != SMDL_OK) return st;
    auto t1 = std::chrono::steady_clock::now();
    if (o->X_local.idx) {
        // the final local codes X^(t), rows in split order
        const smdl_codes& xl = o->X_local;
        if ((st = h->hip(launch_fill_codes(xl.idx, xl.coef, xl.nnz, N, xl.s_max, h->stream), "local codes")) != SMDL_OK ||
            (st = h->hip(hipMemcpy2DAsync(xl.idx, (size_t)xl.s_max * 4, lc.idx, (size_t)lc.s_stride * 4,
                                          (size_t)lc.s_stride * 4, N, hipMemcpyDeviceToDevice, h->stream),
                         "local codes")) != SMDL_OK ||
            (st = h->hip(hipMemcpy2DAsync(xl.coef, (size_t)xl.s_max * 4, lc.coef, (size_t)lc.s_stride * 4,
                                          (size_t)lc.s_stride * 4, N, hipMemcpyDeviceToDevice, h->stream),
                         "local codes")) != SMDL_OK ||
            (st = h->hip(hipMemcpyAsync(xl.nnz, lc.nnz, (size_t)N * 4, hipMemcpyDeviceToDevice, h->stream),
                         "local codes")) != SMDL_OK)
            return st;
    }

    // step 3: scales, pooled data, merge
    if ((st = h->hip(launch_code_scales(lc.coef, lc.nnz, lc.s_stride, offs_dev, L, scales, h->stream), "scales")) != SMDL_OK)
        return st;
    if ((st = h->hip(launch_pool_scale(Dloc, aoff_dev, L, m, scales, Ytil, sumK, h->stream), "pool")) != SMDL_OK)
        return st;
    CodeOut mc;
    mc.s_stride = o->s_merge;
    mc.idx = (int32_t*)h->ws("sm.midx", (size_t)sumK * o->s_merge * 4);
    mc.coef = (float*)h->ws("sm.mcoef", (size_t)sumK * o->s_merge * 4);
    mc.nnz = (int32_t*)h->ws("sm.mnnz", (size_t)sumK * 4);
    mc.res = nullptr;
    if (!mc.idx || !mc.coef || !mc.nnz) return h->fail(SMDL_E_NOMEM, "workspace allocation failed");
    const float* merge_init = o->D_merge_init;
    if (!merge_init && o->merge_seed) {
        // the first K columns of a seeded permutation of the pooled columns
        std::vector<int64_t> pc((size_t)sumK);
        for (int64_t i = 0; i < sumK; ++i) pc[(size_t)i] = i;
        seeded_shuffle(pc, o->merge_seed);
        int64_t* cols = (int64_t*)h->ws("sm.mcols", (size_t)K * 8);
        float* minit = (float*)h->ws("sm.minit", (size_t)K * m * 4);
        int32_t* bad = (int32_t*)h->ws("sm.mbad", 64);
        if (!cols || !minit || !bad) return h->fail(SMDL_E_NOMEM, "workspace allocation failed");
        if ((st = h->hip(h->upload(cols, pc.data(), (size_t)K * 8), "upload")) != SMDL_OK ||
            (st = h->hip(launch_zero_i32(bad, 1, h->stream), "zero")) != SMDL_OK ||
            (st = h->hip(launch_gather_columns(Ytil, cols, K, sumK, m, minit, bad, h->stream), "merge start")) != SMDL_OK)
            return st;
        // the host vector must outlive the queued copy
        if ((st = h->hip(hipStreamSynchronize(h->stream), "merge start")) != SMDL_OK) return st;
        merge_init = minit;
    }
    std::vector<SetSpec> ms(1);
    ms[0].Y = Ytil;
    ms[0].init = merge_init;
    ms[0].n = sumK;
    ms[0].K = K;
    ms[0].s = o->s_merge;
    ms[0].D = D_out;
    ms[0].out0 = 0;
    if ((st = learn_sets(h, m, ms, o->iters_merge, mc, compose && X_out.idx, flags & (SMDL_NO_GRAPH | SMDL_DETERMINISTIC),
                         "sm.mrg")) !=
        SMDL_OK)
        return st;
    auto t2 = std::chrono::steady_clock::now();

    if (X_out.idx && compose) {
        // Proposition 1: X = Z X1 from the local codes and the merge codes (no fresh coding)
        // (perm was checked by the gather of step 1)
        int32_t* bad = (int32_t*)h->ws("sm.cbad", 64);
        if (!bad) return h->fail(SMDL_E_NOMEM, "workspace allocation failed");
        if ((st = h->hip(launch_compose_codes(lc.idx, lc.coef, lc.nnz, lc.s_stride, mc.idx, mc.coef, mc.nnz, mc.s_stride,
                                              offs_dev, aoff_dev, L, scales, sub->perm, N, K, X_out.idx, X_out.coef,
                                              X_out.nnz, X_out.s_max, bad, h->stream),
                         "compose")) != SMDL_OK)
            return st;
    } else if (X_out.idx) {
        // final coding of all N signals (original order)
        if ((st = omp_code_impl(h, D_out, m, K, Y, N, o->s_final, 0.f, X_out, nullptr, nullptr, nullptr, 0,
                                "sm.fin")) != SMDL_OK)
            return st;
    }
    if (scales_out) {
        if ((st = h->hip(hipMemcpyAsync(scales_out, scales, (size_t)L * 8, hipMemcpyDeviceToHost, h->stream), "scales")) != SMDL_OK)
            return st;
    }
    st = h->hip(hipStreamSynchronize(h->stream), "split-merge");
    finish_timing(h);
    auto t3 = std::chrono::steady_clock::now();
    h->phase_ms[0] = std::chrono::duration<float, std::milli>(t1 - t0).count();
    h->phase_ms[1] = std::chrono::duration<float, std::milli>(t2 - t1).count();
    h->phase_ms[2] = std::chrono::duration<float, std::milli>(t3 - t2).count();
    return st;
}

extern "C" smdl_status smdl_compose_codes(smdl_t h, int64_t N, const smdl_subsets* sub, smdl_codes X1, smdl_codes Z,
                                          int K, const double* scales, smdl_codes X_out) {
    if (!h) return SMDL_E_ARG;
    h->err.clear();
    if (!sub || !scales) return h->fail(SMDL_E_ARG, "null pointer");
    if (N < 0) return h->fail(SMDL_E_ARG, "N must be >= 0");
    const int L = sub->L;
    if (L < 1 || !sub->offsets || !sub->K_local) return h->fail(SMDL_E_ARG, "bad subsets");
    if (sub->offsets[0] != 0 || sub->offsets[L] != N) return h->fail(SMDL_E_ARG, "offsets must run from 0 to N");
    if (K < 1 || K > SMDL_MAX_K) return h->fail(SMDL_E_SHAPE, "K must be in [1, 1024]");
    std::vector<int64_t> aoff(L + 1, 0);
    for (int t = 0; t < L; ++t) {
        if (sub->offsets[t + 1] < sub->offsets[t]) return h->fail(SMDL_E_ARG, "offsets must not decrease");
        if (sub->K_local[t] < 1 || sub->K_local[t] > SMDL_MAX_K) return h->fail(SMDL_E_SHAPE, "K_local must be in [1, 1024]");
        if (!(scales[t] >= 0.0)) return h->fail(SMDL_E_ARG, "scales must be >= 0");
        aoff[t + 1] = aoff[t] + sub->K_local[t];
    }
    if (N == 0) return SMDL_OK;
    if (!X1.idx || !X1.coef || !X1.nnz || !Z.idx || !Z.coef || !Z.nnz || !X_out.idx || !X_out.coef || !X_out.nnz)
        return h->fail(SMDL_E_ARG, "null code array");
    if (X1.s_max < 1 || Z.s_max < 1 || X1.s_max * Z.s_max > SMDL_MAX_COMPOSED)
        return h->fail(SMDL_E_SHAPE, "X1.s_max * Z.s_max must be <= 64");
    if (X_out.s_max < X1.s_max * Z.s_max || X_out.s_max > SMDL_MAX_COMPOSED)
        return h->fail(SMDL_E_ARG, "X_out.s_max must be in [X1.s_max * Z.s_max, 64]");
    (void)hipSetDevice(h->device);
    int64_t* offs_dev = (int64_t*)h->ws("cc.offs", (size_t)(L + 1) * 8);
    int64_t* aoff_dev = (int64_t*)h->ws("cc.aoff", (size_t)(L + 1) * 8);
    double* sc_dev = (double*)h->ws("cc.scales", (size_t)L * 8);
    int32_t* bad = (int32_t*)h->ws("cc.bad", 64);
    if (!offs_dev || !aoff_dev || !sc_dev || !bad) return h->fail(SMDL_E_NOMEM, "workspace allocation failed");
    smdl_status st;
    if ((st = h->hip(launch_zero_i32(bad, 1, h->stream), "zero")) != SMDL_OK) return st;
    if ((st = h->hip(h->upload(offs_dev, sub->offsets, (L + 1) * 8), "upload")) != SMDL_OK ||
        (st = h->hip(h->upload(aoff_dev, aoff.data(), (L + 1) * 8), "upload")) != SMDL_OK ||
        (st = h->hip(h->upload(sc_dev, scales, (size_t)L * 8), "upload")) != SMDL_OK)
        return st;
    if ((st = h->hip(launch_compose_codes(X1.idx, X1.coef, X1.nnz, X1.s_max, Z.idx, Z.coef, Z.nnz, Z.s_max, offs_dev,
                                          aoff_dev, L, sc_dev, sub->perm, N, K, X_out.idx, X_out.coef, X_out.nnz,
                                          X_out.s_max, bad, h->stream),
                     "compose")) != SMDL_OK)
        return st;
    int32_t hbad = 0;
    if ((st = h->hip(hipMemcpyAsync(&hbad, bad, 4, hipMemcpyDeviceToHost, h->stream), "check")) != SMDL_OK) return st;
    if ((st = h->hip(hipStreamSynchronize(h->stream), "compose")) != SMDL_OK) return st;
    if (hbad) return h->fail(SMDL_E_ARG, "perm holds an index outside [0, N)");
    return SMDL_OK;
}

// ------------------------------------------------------------------------------------------
// tuning entry points
// ------------------------------------------------------------------------------------------

extern "C" smdl_status smdl_tune(smdl_t h, const float* D, int m, int K, const float* Y, int64_t N, int s_max) {
    if (!h) return SMDL_E_ARG;
    h->err.clear();
    smdl_status st = check_dims(h, m, K, s_max);
    if (st != SMDL_OK) return st;
    if (!D || !Y || N < 1) return h->fail(SMDL_E_ARG, "need a dictionary and at least one signal");
    (void)hipSetDevice(h->device);
    std::vector<SetSpec> sets(1);
    sets[0].D = D;
    sets[0].K = K;
    sets[0].s = s_max;
    sets[0].Y = Y;
    sets[0].n = N;
    sets[0].out0 = 0;
    CodePlan plan;
    if ((st = prepare_sets(h, m, sets, "tune", plan)) != SMDL_OK) return st;
    CodeOut out;
    out.s_stride = s_max;
    out.idx = (int32_t*)h->ws("tune.idx", (size_t)N * s_max * 4);
    out.coef = (float*)h->ws("tune.coef", (size_t)N * s_max * 4);
    out.nnz = (int32_t*)h->ws("tune.nnz", (size_t)N * 4);
    out.res = nullptr;
    if (!out.idx || !out.coef || !out.nnz) return h->fail(SMDL_E_NOMEM, "workspace allocation failed");
    plan.persistent = false;
    h->tiles.erase(std::make_tuple(plan.maxKpad, s_max, 0));
    return autotune_plan(h, plan, sets, out, false, "tune");
}

extern "C" smdl_status smdl_get_tile(smdl_t h, int m, int K, int s_max, int* lanes, int* spi) {
    if (!h || !lanes || !spi) return SMDL_E_ARG;
    smdl_status st = check_dims(h, m, K, s_max);
    if (st != SMDL_OK) return st;
    OmpTile t = choose_tile(h, pad64(K), s_max, false);
    *lanes = t.lanes;
    *spi = 16 * t.tt;
    return SMDL_OK;
}

extern "C" smdl_status smdl_set_tile(smdl_t h, int K, int s_max, int lanes, int signals_per_item) {
    if (!h) return SMDL_E_ARG;
    OmpTile t{lanes, signals_per_item / 16};
    if (signals_per_item % 16 || !omp_tile_supported(t, pad64(K), s_max))
        return h->fail(SMDL_E_UNSUPPORTED, "tile not instantiated for this shape");
    h->tiles[std::make_tuple(pad64(K), s_max, 0)] = t;
    h->tiles[std::make_tuple(pad64(K), s_max, 1)] = t;
    return SMDL_OK;
}

extern "C" smdl_status smdl_set_mod_solver(smdl_t h, int mode) {
    if (!h) return SMDL_E_ARG;
    if (mode < 0 || mode > 2) return h->fail(SMDL_E_ARG, "MOD solver mode must be 0, 1 or 2");
    h->mod_solver = mode;
    return SMDL_OK;
}

extern "C" smdl_status smdl_set_flags(smdl_t h, uint32_t flags) {
    if (!h) return SMDL_E_ARG;
    if (flags & ~(SMDL_DETERMINISTIC | SMDL_CHECK_FINITE | SMDL_ASYNC))
        return h->fail(SMDL_E_ARG, "only SMDL_DETERMINISTIC, SMDL_CHECK_FINITE and SMDL_ASYNC apply to a handle");
    h->flags = flags;
    return SMDL_OK;
}

extern "C" smdl_status smdl_set_autotune(smdl_t h, int enabled) {
    if (!h) return SMDL_E_ARG;
    h->autotune = enabled != 0;
    return SMDL_OK;
}

extern "C" smdl_status smdl_phase_ms(smdl_t h, float* ms3) {
    if (!h || !ms3) return SMDL_E_ARG;
    for (int i = 0; i < 3; ++i) ms3[i] = h->phase_ms[i];
    return SMDL_OK;
}

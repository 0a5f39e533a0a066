// C ABI of the learned support proposer: network state, forward, gradients, Adam training and
// proposer-restricted OMP with the full-OMP fallback.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

#include "mlp_internal.h"
#include "smdl_api_internal.h"

struct smdl_prop {
    smdl_t h = nullptr;
    int n_layers = 0;
    std::vector<int> widths;
    std::vector<float*> W, b, mW, vW, mb, vb;   // FP32 masters and Adam moments
    std::vector<uint16_t*> Wpk, WTpk;           // BF16 W (out x in) and W^T (in x out), fragment order
    int step = 0;                               // Adam steps taken
    int32_t* dstep = nullptr;                   // the same count on the device
    std::vector<void*> allocs;

    template <class T>
    T* alloc(size_t n) {
        void* p = nullptr;
        if (hipMalloc(&p, std::max<size_t>(n, 1) * sizeof(T)) != hipSuccess) {
            (void)hipGetLastError();
            return nullptr;
        }
        allocs.push_back(p);
        return static_cast<T*>(p);
    }
};

namespace {

inline int64_t pad64b(int64_t x) { return (x + 63) / 64 * 64; }

// Activation buffers for a batch of Bpad rows (a multiple of 64), every BF16 matrix in fragment
// order.  With R > 0 the fused network kernel runs R rows per work group and keeps the
// activations and deltas in LDS, so only the transposed copies, the column sums and the logits
// live here; with R = 0 (the per-layer path) the activations and deltas live here too.
struct Acts {
    int64_t Bpad = 0;
    int R = 0;
    std::vector<uint16_t*> h;      // h[l]: Bpad x widths[l], input of layer l
    float* logits = nullptr;       // Bpad x K (inference, FP32 row-major)
    // training only
    std::vector<uint16_t*> hT;     // widths[l] x Bpad
    std::vector<uint16_t*> d;      // d[l]: Bpad x widths[l + 1], delta at the output of layer l
    std::vector<uint16_t*> dT;     // widths[l + 1] x Bpad
    std::vector<float*> part;      // (Bpad / 32) x widths[l + 1] column sums of the FP32 deltas
};

smdl_status get_acts(smdl_t h, smdl_prop_t p, int64_t Bpad, bool train, Acts& a) {
    const int L = p->n_layers;
    a.Bpad = Bpad;
    a.R = mlp_rows_per_block(L, p->widths.data(), train);
    a.h.assign(L, nullptr);
    for (int l = 0; l < L && a.R == 0; ++l) {
        std::string nm = "prop.h" + std::to_string(l);
        a.h[l] = (uint16_t*)h->ws(nm.c_str(), (size_t)Bpad * p->widths[l] * 2);
        if (!a.h[l]) return h->fail(SMDL_E_NOMEM, "workspace allocation failed");
    }
    if (!train) {
        a.logits = (float*)h->ws("prop.logits", (size_t)Bpad * p->widths[L] * 4);
        if (!a.logits) return h->fail(SMDL_E_NOMEM, "workspace allocation failed");
        return SMDL_OK;
    }
    a.hT.assign(L, nullptr);
    a.d.assign(L, nullptr);
    a.dT.assign(L, nullptr);
    a.part.assign(L, nullptr);
    for (int l = 0; l < L; ++l) {
        const std::string k = std::to_string(l);
        const int wi = p->widths[l], wo = p->widths[l + 1];
        a.hT[l] = (uint16_t*)h->ws(("prop.hT" + k).c_str(), (size_t)Bpad * wi * 2);
        if (a.R == 0) a.d[l] = (uint16_t*)h->ws(("prop.d" + k).c_str(), (size_t)Bpad * wo * 2);
        a.dT[l] = (uint16_t*)h->ws(("prop.dT" + k).c_str(), (size_t)Bpad * wo * 2);
        a.part[l] = (float*)h->ws(("prop.part" + k).c_str(), (size_t)(Bpad / 16) * wo * 4);
        if (!a.hT[l] || (a.R == 0 && !a.d[l]) || !a.dT[l] || !a.part[l])
            return h->fail(SMDL_E_NOMEM, "workspace allocation failed");
    }
    return SMDL_OK;
}

// Forward pass over the B rows of Y (gathered through `rows` when set), padded to a.Bpad.
// Inference: logits_out (B x K FP32).  Training (tmask set): the output layer applies the BCE
// loss (added to *loss) and writes the output deltas; every layer input is also stored
// transposed for the weight gradients.
hipError_t enqueue_forward(smdl_t h, smdl_prop_t p, const float* Y, int64_t B, const int32_t* rows, Acts& a,
                           float* logits_out, const uint32_t* tmask, int tstride, double* loss) {
    const int L = p->n_layers;
    const bool train = tmask != nullptr;
    const int64_t Bpad = a.Bpad;
    hipError_t e = launch_prep(Y, B, p->widths[0], Bpad, rows, a.h[0], train ? a.hT[0] : nullptr, h->stream);
    if (e != hipSuccess) return e;
    for (int l = 0; l < L; ++l) {
        const int wi = p->widths[l], wo = p->widths[l + 1];
        NtArgs g{};
        g.A = a.h[l];
        g.B = p->Wpk[l];
        g.M = (int)Bpad;
        g.N = wo;
        g.K = wi;
        g.Mvalid = (int)B;
        g.bias = p->b[l];
        g.ldo = wo;
        if (l + 1 < L) {
            g.relu = 1;
            g.out_bf16 = a.h[l + 1];
            if (train) g.outT = a.hT[l + 1];
        } else if (train) {
            g.tmask = tmask;
            g.tstride = tstride;
            g.rows = rows;
            g.scale = 1.0f / ((float)B * wo);
            g.loss = loss;
            g.out_bf16 = a.d[l];
            g.outT = a.dT[l];
            g.colpart = a.part[l];
        } else {
            g.out_f32 = logits_out;
        }
        if ((e = launch_gemm_nt(g, h->stream)) != hipSuccess) return e;
    }
    return hipSuccess;
}

// Per-layer backward after a training forward: the deltas of every hidden layer (BF16,
// transposed, column sums over 32-row blocks).
hipError_t enqueue_deltas(smdl_t h, smdl_prop_t p, int64_t B, Acts& a) {
    const int L = p->n_layers;
    const int64_t Bpad = a.Bpad;
    hipError_t e;
    for (int l = L - 1; l >= 1; --l) {
        // d_{l-1} = (d_l W_l) * [h_l > 0]
        const int wi = p->widths[l], wo = p->widths[l + 1];
        NtArgs g{};
        g.A = a.d[l];
        g.B = p->WTpk[l];
        g.M = (int)Bpad;
        g.N = wi;
        g.K = wo;
        g.Mvalid = (int)B;
        g.mask = a.h[l];
        g.ldmask = wi;
        g.out_bf16 = l - 1 >= 1 ? a.d[l - 1] : nullptr;
        g.ldo = wi;
        g.outT = a.dT[l - 1];
        g.colpart = a.part[l - 1];
        if ((e = launch_gemm_nt(g, h->stream)) != hipSuccess) return e;
    }
    return hipSuccess;
}

// One grouped launch for all weight and bias gradients (from the transposed activations and
// deltas and the column sums over blocks of `rows_per_part` rows), applied with Adam when
// `adam` is set (step t) or stored in dW / db.
hipError_t enqueue_wgrad(smdl_t h, smdl_prop_t p, Acts& a, int rows_per_part, const smdl_train_opts* adam,
                         int t_off, float* const* dW, float* const* db) {
    const int L = p->n_layers;
    const int64_t Bpad = a.Bpad;
    WgArgs w{};
    w.n_layers = L;
    w.Bpad = (int)Bpad;
    w.adam = adam != nullptr;
    if (adam) {
        w.lr = adam->lr;
        w.b1 = adam->beta1;
        w.b2 = adam->beta2;
        w.eps = adam->adam_eps;
        w.t_dev = p->dstep;
        w.t_off = t_off;
    }
    for (int l = 0; l < L; ++l) {
        WgLayer& q = w.L[l];
        q.dT = a.dT[l];
        q.hT = a.hT[l];
        q.colpart = a.part[l];
        q.nparts = (int)(Bpad / rows_per_part);
        q.wo = p->widths[l + 1];
        q.wi = p->widths[l];
        q.W = p->W[l];
        q.b = p->b[l];
        q.mW = p->mW[l];
        q.vW = p->vW[l];
        q.mb = p->mb[l];
        q.vb = p->vb[l];
        q.Wpk = p->Wpk[l];
        q.WTpk = p->WTpk[l];
        q.dW_out = dW ? dW[l] : nullptr;
        q.db_out = db ? db[l] : nullptr;
    }
    return launch_wgrad(w, h->stream);
}

RowsArgs rows_args(smdl_prop_t p, const float* Y, int64_t B, const int32_t* rows, const Acts& a) {
    RowsArgs r{};
    r.Y = Y;
    r.B = B;
    r.Bpad = a.Bpad;
    r.rows = rows;
    r.n_layers = p->n_layers;
    for (int l = 0; l <= p->n_layers; ++l) r.w[l] = p->widths[l];
    for (int l = 0; l < p->n_layers; ++l) {
        r.W[l] = p->Wpk[l];
        r.WT[l] = p->WTpk[l];
        r.bias[l] = p->b[l];
    }
    return r;
}

// Logits of the N rows of Y (B x K FP32 into `logits`).
hipError_t enqueue_logits(smdl_t h, smdl_prop_t p, const float* Y, int64_t N, Acts& a, float* logits) {
    if (a.R == 0) return enqueue_forward(h, p, Y, N, nullptr, a, logits, nullptr, 0, nullptr);
    RowsArgs r = rows_args(p, Y, N, nullptr, a);
    r.logits = logits;
    return launch_mlp_rows(r, a.R, h->stream);
}

// Loss and gradients of a batch of B rows (gathered through `rows`), applied with Adam when
// `adam` is set, else stored in dW / db.
hipError_t enqueue_grad_step(smdl_t h, smdl_prop_t p, const float* Y, int64_t B, const int32_t* rows, Acts& a,
                             const uint32_t* tmask, int tstride, double* loss, const smdl_train_opts* adam,
                             int t_off, float* const* dW, float* const* db) {
    hipError_t e;
    const int K = p->widths[p->n_layers];
    if (a.R == 0) {
        if ((e = enqueue_forward(h, p, Y, B, rows, a, nullptr, tmask, tstride, loss)) != hipSuccess) return e;
        if ((e = enqueue_deltas(h, p, B, a)) != hipSuccess) return e;
        return enqueue_wgrad(h, p, a, 32, adam, t_off, dW, db);
    }
    RowsArgs r = rows_args(p, Y, B, rows, a);
    r.tmask = tmask;
    r.tstride = tstride;
    r.scale = 1.0f / ((float)B * K);
    r.loss = loss;
    for (int l = 0; l < p->n_layers; ++l) {
        r.hT[l] = a.hT[l];
        r.dT[l] = a.dT[l];
        r.colpart[l] = a.part[l];
    }
    if ((e = launch_mlp_rows(r, a.R, h->stream)) != hipSuccess) return e;
    return enqueue_wgrad(h, p, a, a.R, adam, t_off, dW, db);
}

// Multi-hot label bitmask of N samples (workspace), rows of (K + 31) / 32 words.
uint32_t* label_mask(smdl_t h, const smdl_codes& labels, int64_t N, int K, hipError_t& e) {
    const int words = (K + 31) / 32;
    uint32_t* m = (uint32_t*)h->ws("prop.tmask", (size_t)std::max<int64_t>(N, 1) * words * 4);
    if (!m) {
        e = hipErrorOutOfMemory;
        return nullptr;
    }
    e = launch_label_mask(labels.idx, labels.nnz, labels.s_max, N, K, m, h->stream);
    return m;
}

smdl_status check_prop(smdl_t h, smdl_prop_t p) {
    if (!p || p->h != h) return h->fail(SMDL_E_STATE, "proposer does not belong to this handle");
    return SMDL_OK;
}

// New FP32 masters (host arrays) with fresh Adam state (moments and step count zero) and
// their BF16 copies; synchronous.
smdl_status load_weights(smdl_t h, smdl_prop_t p, const float* const* W_host, const float* const* b_host) {
    hipError_t e = hipMemsetAsync(p->dstep, 0, 4, h->stream);
    for (int l = 0; l < p->n_layers && e == hipSuccess; ++l) {
        const size_t nw = (size_t)p->widths[l] * p->widths[l + 1], nb = p->widths[l + 1];
        e = hipMemcpyAsync(p->W[l], W_host[l], nw * 4, hipMemcpyHostToDevice, h->stream);
        if (e == hipSuccess) e = hipMemcpyAsync(p->b[l], b_host[l], nb * 4, hipMemcpyHostToDevice, h->stream);
        if (e == hipSuccess) e = hipMemsetAsync(p->mW[l], 0, nw * 4, h->stream);
        if (e == hipSuccess) e = hipMemsetAsync(p->vW[l], 0, nw * 4, h->stream);
        if (e == hipSuccess) e = hipMemsetAsync(p->mb[l], 0, nb * 4, h->stream);
        if (e == hipSuccess) e = hipMemsetAsync(p->vb[l], 0, nb * 4, h->stream);
        if (e == hipSuccess)
            e = launch_to_bf16(p->W[l], (int64_t)nw, p->widths[l], p->widths[l + 1], p->Wpk[l], p->WTpk[l], h->stream);
    }
    if (e != hipSuccess) return h->hip(e, "proposer weights");
    p->step = 0;
    return h->hip(hipStreamSynchronize(h->stream), "proposer weights");
}

}  // namespace

extern "C" smdl_status smdl_prop_create(smdl_t h, int n_layers, const int* widths, const float* const* W_init,
                                        const float* const* b_init, smdl_prop_t* out) {
    if (!h) return SMDL_E_ARG;
    h->err.clear();
    if (!out || !widths || !W_init || !b_init) return h->fail(SMDL_E_ARG, "null pointer");
    *out = nullptr;
    if (n_layers < 1 || n_layers > 4) return h->fail(SMDL_E_SHAPE, "1 to 4 layers");
    for (int l = 0; l <= n_layers; ++l)
        if (widths[l] < 32 || widths[l] > 4096 || widths[l] % 32)
            return h->fail(SMDL_E_SHAPE, "layer widths must be multiples of 32 in [32, 4096]");
    if (widths[0] > SMDL_MAX_M || widths[n_layers] > SMDL_MAX_K)
        return h->fail(SMDL_E_SHAPE, "input width must be <= 256 and output width <= 1024");
    for (int l = 0; l < n_layers; ++l)
        if (!W_init[l] || !b_init[l]) return h->fail(SMDL_E_ARG, "null initial weights");
    (void)hipSetDevice(h->device);
    auto* p = new smdl_prop();
    p->h = h;
    p->n_layers = n_layers;
    p->widths.assign(widths, widths + n_layers + 1);
    p->dstep = p->alloc<int32_t>(1);
    if (!p->dstep || hipMemsetAsync(p->dstep, 0, 4, h->stream) != hipSuccess) {
        smdl_prop_destroy(p);
        return h->fail(SMDL_E_NOMEM, "proposer allocation failed");
    }
    for (int l = 0; l < n_layers; ++l) {
        const size_t nw = (size_t)widths[l] * widths[l + 1], nb = widths[l + 1];
        float *W = p->alloc<float>(nw), *b = p->alloc<float>(nb);
        float *mW = p->alloc<float>(nw), *vW = p->alloc<float>(nw), *mb = p->alloc<float>(nb), *vb = p->alloc<float>(nb);
        uint16_t *Wpk = p->alloc<uint16_t>(nw), *WTpk = p->alloc<uint16_t>(nw);
        if (!W || !b || !mW || !vW || !mb || !vb || !Wpk || !WTpk) {
            smdl_prop_destroy(p);
            return h->fail(SMDL_E_NOMEM, "proposer allocation failed");
        }
        p->W.push_back(W);
        p->b.push_back(b);
        p->mW.push_back(mW);
        p->vW.push_back(vW);
        p->mb.push_back(mb);
        p->vb.push_back(vb);
        p->Wpk.push_back(Wpk);
        p->WTpk.push_back(WTpk);
    }
    smdl_status st = load_weights(h, p, W_init, b_init);
    if (st != SMDL_OK) {
        smdl_prop_destroy(p);
        return st;
    }
    *out = p;
    return SMDL_OK;
}

extern "C" smdl_status smdl_prop_create_seeded(smdl_t h, int n_layers, const int* widths, uint64_t seed,
                                               smdl_prop_t* out) {
    if (!h) return SMDL_E_ARG;
    h->err.clear();
    if (!out || !widths) return h->fail(SMDL_E_ARG, "null pointer");
    if (n_layers < 1 || n_layers > 4) return h->fail(SMDL_E_SHAPE, "1 to 4 layers");
    for (int l = 0; l <= n_layers; ++l)
        if (widths[l] < 32 || widths[l] > 4096 || widths[l] % 32)
            return h->fail(SMDL_E_SHAPE, "layer widths must be multiples of 32 in [32, 4096]");
    // Kaiming-uniform weights U(-sqrt(6/fan_in), sqrt(6/fan_in)) and biases
    // U(-1/sqrt(fan_in), 1/sqrt(fan_in)); uniforms (x >> 11) 2^-53 of consecutive splitmix64
    // draws, every layer's weights (row-major) then its biases, layer by layer
    SplitMix64 g(seed);
    auto uni = [&g](double lo, double hi) {
        const double u = (double)(g.next() >> 11) * (1.0 / 9007199254740992.0);
        return (float)(lo + (hi - lo) * u);
    };
    std::vector<std::vector<float>> Ws(n_layers), bs(n_layers);
    std::vector<const float*> Wp(n_layers), bp(n_layers);
    for (int l = 0; l < n_layers; ++l) {
        const double fan_in = widths[l];
        const double bw = std::sqrt(6.0 / fan_in), bb = 1.0 / std::sqrt(fan_in);
        Ws[l].resize((size_t)widths[l] * widths[l + 1]);
        bs[l].resize(widths[l + 1]);
        for (float& w : Ws[l]) w = uni(-bw, bw);
        for (float& b : bs[l]) b = uni(-bb, bb);
        Wp[l] = Ws[l].data();
        bp[l] = bs[l].data();
    }
    return smdl_prop_create(h, n_layers, widths, Wp.data(), bp.data(), out);
}

extern "C" smdl_status smdl_prop_set(smdl_t h, smdl_prop_t p, const float* const* W_host, const float* const* b_host) {
    if (!h) return SMDL_E_ARG;
    h->err.clear();
    smdl_status st = check_prop(h, p);
    if (st != SMDL_OK) return st;
    if (!W_host || !b_host) return h->fail(SMDL_E_ARG, "null pointer");
    for (int l = 0; l < p->n_layers; ++l)
        if (!W_host[l] || !b_host[l]) return h->fail(SMDL_E_ARG, "null weights");
    (void)hipSetDevice(h->device);
    return load_weights(h, p, W_host, b_host);
}

extern "C" smdl_status smdl_prop_destroy(smdl_prop_t p) {
    if (!p) return SMDL_E_ARG;
    if (p->h) (void)hipStreamSynchronize(p->h->stream);
    for (void* a : p->allocs) (void)hipFree(a);
    delete p;
    return SMDL_OK;
}

extern "C" smdl_status smdl_prop_get(smdl_t h, smdl_prop_t p, float* const* W_host, float* const* b_host) {
    if (!h) return SMDL_E_ARG;
    h->err.clear();
    smdl_status st = check_prop(h, p);
    if (st != SMDL_OK) return st;
    if (!W_host || !b_host) return h->fail(SMDL_E_ARG, "null pointer");
    for (int l = 0; l < p->n_layers; ++l) {
        const size_t nw = (size_t)p->widths[l] * p->widths[l + 1], nb = p->widths[l + 1];
        if (W_host[l] && (st = h->hip(hipMemcpyAsync(W_host[l], p->W[l], nw * 4, hipMemcpyDeviceToHost, h->stream), "get")) != SMDL_OK)
            return st;
        if (b_host[l] && (st = h->hip(hipMemcpyAsync(b_host[l], p->b[l], nb * 4, hipMemcpyDeviceToHost, h->stream), "get")) != SMDL_OK)
            return st;
    }
    return h->hip(hipStreamSynchronize(h->stream), "get");
}

extern "C" smdl_status smdl_prop_logits(smdl_t h, smdl_prop_t p, const float* Y, int64_t N, float* logits) {
    if (!h) return SMDL_E_ARG;
    h->err.clear();
    smdl_status st = check_prop(h, p);
    if (st != SMDL_OK) return st;
    if (N < 0) return h->fail(SMDL_E_ARG, "N must be >= 0");
    if (N == 0) return SMDL_OK;
    if (!Y || !logits) return h->fail(SMDL_E_ARG, "null pointer");
    if (N > INT32_MAX / 4) return h->fail(SMDL_E_SHAPE, "N too large");
    (void)hipSetDevice(h->device);
    Acts a;
    if ((st = get_acts(h, p, pad64b(N), false, a)) != SMDL_OK) return st;
    if ((st = h->hip(enqueue_logits(h, p, Y, N, a, logits), "forward")) != SMDL_OK) return st;
    if (h->flags & SMDL_ASYNC) return SMDL_OK;
    return h->hip(hipStreamSynchronize(h->stream), "forward");
}

static smdl_status check_labels(smdl_t h, const smdl_codes& labels, int64_t N) {
    if (N > 0 && (!labels.idx || !labels.nnz)) return h->fail(SMDL_E_ARG, "null label arrays");
    if (labels.s_max < 1 || labels.s_max > SMDL_MAX_S) return h->fail(SMDL_E_SHAPE, "labels.s_max must be in [1, 16]");
    return SMDL_OK;
}

extern "C" smdl_status smdl_prop_grad(smdl_t h, smdl_prop_t p, const float* Y, int64_t N, smdl_codes labels,
                                      float* loss, float* const* dW, float* const* db) {
    if (!h) return SMDL_E_ARG;
    h->err.clear();
    smdl_status st = check_prop(h, p);
    if (st != SMDL_OK) return st;
    if (N < 1) return h->fail(SMDL_E_ARG, "N must be >= 1");
    if (N > INT32_MAX / 8) return h->fail(SMDL_E_SHAPE, "N too large");
    if (!Y || !dW || !db) return h->fail(SMDL_E_ARG, "null pointer");
    if ((st = check_labels(h, labels, N)) != SMDL_OK) return st;
    for (int l = 0; l < p->n_layers; ++l)
        if (!dW[l] || !db[l]) return h->fail(SMDL_E_ARG, "null gradient array");
    (void)hipSetDevice(h->device);
    Acts a;
    if ((st = get_acts(h, p, pad64b(N), true, a)) != SMDL_OK) return st;
    const int K = p->widths[p->n_layers];
    double* dloss = (double*)h->ws("prop.loss", 8);
    if (!dloss) return h->fail(SMDL_E_NOMEM, "workspace allocation failed");
    hipError_t e;
    const uint32_t* tm = label_mask(h, labels, N, K, e);
    if (e != hipSuccess) return h->hip(e, "labels");
    if ((e = launch_zero_f64(dloss, 1, h->stream)) != hipSuccess) return h->hip(e, "grad");
    if ((e = enqueue_grad_step(h, p, Y, N, nullptr, a, tm, (K + 31) / 32, dloss, nullptr, 0, dW, db)) != hipSuccess)
        return h->hip(e, "grad");
    double l = 0.0;
    if ((st = h->hip(hipMemcpyAsync(&l, dloss, 8, hipMemcpyDeviceToHost, h->stream), "loss")) != SMDL_OK) return st;
    if ((st = h->hip(hipStreamSynchronize(h->stream), "grad")) != SMDL_OK) return st;
    if (loss) *loss = (float)(l / ((double)N * K));
    return SMDL_OK;
}

extern "C" smdl_status smdl_prop_train(smdl_t h, smdl_prop_t p, const float* Y, int64_t N, smdl_codes labels,
                                       const smdl_train_opts* o, float* loss_per_epoch) {
    if (!h) return SMDL_E_ARG;
    h->err.clear();
    smdl_status st = check_prop(h, p);
    if (st != SMDL_OK) return st;
    if (!o || !Y) return h->fail(SMDL_E_ARG, "null pointer");
    if (o->epochs < 0 || o->batch < 16 || o->batch > 65536) return h->fail(SMDL_E_ARG, "bad epochs or batch size");
    if (!(o->lr > 0.f) || !(o->beta1 >= 0.f && o->beta1 < 1.f) || !(o->beta2 >= 0.f && o->beta2 < 1.f) || !(o->adam_eps > 0.f))
        return h->fail(SMDL_E_ARG, "bad Adam parameters");
    if ((st = check_labels(h, labels, N)) != SMDL_OK) return st;
    if (N > INT32_MAX / 8) return h->fail(SMDL_E_SHAPE, "N too large");
    (void)hipSetDevice(h->device);
    const int64_t B = o->batch;
    const int64_t nb = N / B;
    const int K = p->widths[p->n_layers];
    Acts a;
    if ((st = get_acts(h, p, pad64b(B), true, a)) != SMDL_OK) return st;
    int32_t* rows = (int32_t*)h->ws("prop.rows", (size_t)std::max<int64_t>(N, 1) * 4);
    double* eloss = (double*)h->ws("prop.eloss", 8 * (size_t)std::max<int64_t>(nb, 1));
    if (!rows || !eloss) return h->fail(SMDL_E_NOMEM, "workspace allocation failed");
    hipError_t e;
    const uint32_t* tm = label_mask(h, labels, N, K, e);
    if (e != hipSuccess) return h->hip(e, "labels");
    std::vector<int32_t> order(N);
    std::iota(order.begin(), order.end(), 0);
    SplitMix64 rng(o->shuffle_seed);
    // One epoch (every Adam step over the batches of `rows`) is captured once as a graph and
    // replayed per epoch; the shuffled order is copied into `rows` before each replay and the
    // Adam step count lives on the device.
    auto one_epoch = [&]() -> hipError_t {
        hipError_t e2 = launch_zero_f64(eloss, std::max<int64_t>(nb, 1), h->stream);
        for (int64_t bi = 0; bi < nb && e2 == hipSuccess; ++bi) {
            e2 = enqueue_grad_step(h, p, Y, B, rows + bi * B, a, tm, (K + 31) / 32, eloss + bi, o, (int)bi + 1,
                                   nullptr, nullptr);
        }
        if (e2 == hipSuccess) e2 = launch_add_i32(p->dstep, (int32_t)nb, h->stream);
        return e2;
    };
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    if (o->epochs > 0 && nb > 0) {
        if ((st = h->hip(hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal), "capture")) != SMDL_OK)
            return st;
        e = one_epoch();
        hipError_t e2 = hipStreamEndCapture(h->stream, &graph);
        if (e != hipSuccess || e2 != hipSuccess) {
            if (graph) (void)hipGraphDestroy(graph);
            return h->hip(e != hipSuccess ? e : e2, "capture");
        }
        if ((st = h->hip(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0), "instantiate")) != SMDL_OK) {
            (void)hipGraphDestroy(graph);
            return st;
        }
    }
    auto cleanup = [&]() {
        (void)hipStreamSynchronize(h->stream);
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
    };
    // each epoch's order gets its own host buffer, alive until the end, so that the queued copies
    // never read a buffer the next shuffle rewrites (beyond 2^26 entries: one buffer and a
    // synchronisation per epoch instead)
    const bool keep_all = (int64_t)o->epochs * N <= (int64_t)1 << 26;
    std::vector<std::vector<int32_t>> orders;
    for (int ep = 0; ep < o->epochs; ++ep) {
        // with one shared buffer, the previous epoch's queued copy must have read it before the
        // shuffle below rewrites it
        if (!keep_all && ep > 0 && nb > 0 && (st = h->hip(hipStreamSynchronize(h->stream), "train")) != SMDL_OK) {
            cleanup();
            return st;
        }
        if (o->shuffle_seed) {
            for (int64_t i = N - 1; i > 0; --i) std::swap(order[i], order[rng.next() % (uint64_t)(i + 1)]);
        }
        if (nb > 0) {
            if (keep_all) orders.push_back(order);
            const int32_t* src = keep_all ? orders.back().data() : order.data();
            if ((st = h->hip(hipMemcpyAsync(rows, src, (size_t)N * 4, hipMemcpyHostToDevice, h->stream), "rows")) != SMDL_OK ||
                (st = h->hip(hipGraphLaunch(exec, h->stream), "graph launch")) != SMDL_OK) {
                cleanup();
                return st;
            }
            p->step += (int)nb;
        }
        if (loss_per_epoch) {
            std::vector<double> el(std::max<int64_t>(nb, 1));
            if (nb > 0 && (st = h->hip(hipMemcpyAsync(el.data(), eloss, nb * 8, hipMemcpyDeviceToHost, h->stream), "loss")) != SMDL_OK) {
                cleanup();
                return st;
            }
            if ((st = h->hip(hipStreamSynchronize(h->stream), "train")) != SMDL_OK) {
                cleanup();
                return st;
            }
            double s = 0.0;
            for (int64_t i = 0; i < nb; ++i) s += el[i] / ((double)B * K);
            loss_per_epoch[ep] = nb > 0 ? (float)(s / nb) : 0.f;
        }
    }
    cleanup();
    return h->hip(hipStreamSynchronize(h->stream), "train");
}

extern "C" smdl_status smdl_omp_code_proposed(smdl_t h, smdl_prop_t p, const float* D, int m, int K,
                                              const float* Y, int64_t N, int s_max, int n_cand, float eps_fallback,
                                              smdl_codes X, uint8_t* fell_back, int64_t* n_fallback,
                                              int32_t* cand_out) {
    if (!h) return SMDL_E_ARG;
    h->err.clear();
    smdl_status st = check_prop(h, p);
    if (st != SMDL_OK) return st;
    if ((st = check_dims(h, m, K, s_max)) != SMDL_OK) return st;
    if (p->widths[0] != m || p->widths[p->n_layers] != K) return h->fail(SMDL_E_SHAPE, "network widths do not match (m, K)");
    if (n_cand < s_max || n_cand > 64 || n_cand > K) return h->fail(SMDL_E_SHAPE, "need s_max <= n_cand <= min(64, K)");
    if (!(eps_fallback >= 0.f)) return h->fail(SMDL_E_ARG, "eps_fallback must be >= 0 (inf allowed)");
    if (N < 0) return h->fail(SMDL_E_ARG, "N must be >= 0");
    if ((st = check_codes(h, X, N, s_max)) != SMDL_OK) return st;
    if (n_fallback) *n_fallback = 0;
    if (N == 0) return SMDL_OK;
    if (!D || !Y) return h->fail(SMDL_E_ARG, "null pointer");
    if (N > INT32_MAX / 64) return h->fail(SMDL_E_SHAPE, "N too large");
    (void)hipSetDevice(h->device);
    Acts a;
    if ((st = get_acts(h, p, pad64b(N), false, a)) != SMDL_OK) return st;
    int32_t* cand = cand_out ? cand_out : (int32_t*)h->ws("prop.cand", (size_t)N * n_cand * 4);
    int32_t* fb_list = (int32_t*)h->ws("prop.fbl", (size_t)N * 4);
    int32_t* fb_cnt = (int32_t*)h->ws("prop.fbc", 64);
    if (!cand || !fb_list || !fb_cnt) return h->fail(SMDL_E_NOMEM, "workspace allocation failed");
    hipError_t e;
    (void)hipEventRecord(h->ev_prop[0], h->stream);
    if ((e = enqueue_logits(h, p, Y, N, a, a.logits)) != hipSuccess)
        return h->hip(e, "forward");
    if ((e = launch_topk(a.logits, N, K, n_cand, cand, h->stream)) != hipSuccess) return h->hip(e, "topk");
    (void)hipEventRecord(h->ev_prop[1], h->stream);
    // dictionary fragments and Gram for the restricted kernel and the fallback
    std::vector<SetSpec> sets(1);
    sets[0].D = D;
    sets[0].K = K;
    sets[0].s = s_max;
    sets[0].Y = Y;
    sets[0].n = N;
    sets[0].out0 = 0;
    CodePlan plan;
    if ((st = prepare_sets(h, m, sets, "prop", plan)) != SMDL_OK) return st;
    if ((e = launch_pack_dict_m(plan.pack_desc, 1, plan.maxKpad, m, plan.mchunks, h->stream)) != hipSuccess)
        return h->hip(e, "pack");
    if ((e = launch_gram_batched(plan.gram_desc, 1, plan.maxKpad, plan.mchunks, h->stream)) != hipSuccess)
        return h->hip(e, "gram");
    if ((e = launch_zero_i32(fb_cnt, 1, h->stream)) != hipSuccess) return h->hip(e, "zero");
    RestrictedArgs r{};
    r.D = D;
    r.dfrag = sets[0].frag;
    r.mchunks = plan.mchunks;
    r.gram = sets[0].gram;
    r.gld = sets[0].gld;
    r.Kpad = sets[0].Kpad;
    r.m = m;
    r.K = K;
    r.Y = Y;
    r.N = N;
    r.cand = cand;
    r.n_cand = n_cand;
    r.s = std::min(s_max, n_cand);
    r.eps_fb = std::isinf(eps_fallback) ? INFINITY : eps_fallback;
    r.tau = SMDL_TAU;
    r.dep_tol = SMDL_DEP_TOL;
    r.idx = X.idx;
    r.coef = X.coef;
    r.nnz = X.nnz;
    r.s_out = X.s_max;
    r.fell_back = fell_back;
    r.fb_list = fb_list;
    r.fb_count = fb_cnt;
    if ((e = launch_restricted_omp(r, h->stream)) != hipSuccess) return h->hip(e, "restricted omp");
    (void)hipEventRecord(h->ev_prop[2], h->stream);
    // full OMP on the signals the restricted code missed (count stays on the device)
    const OmpTile tile = choose_tile(h, plan.maxKpad, s_max, false);
    const int T = 16 * tile.tt;
    OmpArgs oa{};
    oa.desc = plan.omp_desc;
    oa.items = nullptr;
    oa.n_items = (int)((N + T - 1) / T);
    oa.sig_list = fb_list;
    oa.list_count = fb_cnt;
    oa.queue = plan.queue;
    oa.max_kpad = plan.maxKpad;
    {
        const float* ys[1] = {Y};
        oa.y_lds = omp_y_lds(tile, plan.maxKpad, s_max, m, ys, 1) ? 1 : 0;
    }
    oa.m = m;
    oa.mchunks = plan.mchunks;
    oa.eps2 = 0.f;
    oa.tau = SMDL_TAU;
    oa.dep_tol = SMDL_DEP_TOL;
    oa.idx = X.idx;
    oa.coef = X.coef;
    oa.nnz = X.nnz;
    oa.res = nullptr;
    oa.s_out = X.s_max;
    if ((e = launch_omp(tile, plan.maxKpad, s_max, oa, oa.n_items, h->n_cu, h->stream)) != hipSuccess)
        return h->hip(e, "fallback omp");
    (void)hipEventRecord(h->ev_prop[3], h->stream);
    int32_t cnt = 0;
    if ((st = h->hip(hipMemcpyAsync(&cnt, fb_cnt, 4, hipMemcpyDeviceToHost, h->stream), "count")) != SMDL_OK) return st;
    if ((st = h->hip(hipStreamSynchronize(h->stream), "proposed omp")) != SMDL_OK) return st;
    for (int i = 0; i < 3; ++i) (void)hipEventElapsedTime(&h->prop_ms[i], h->ev_prop[i], h->ev_prop[i + 1]);
    (void)hipGetLastError();
    if (n_fallback) *n_fallback = cnt;
    return SMDL_OK;
}

extern "C" smdl_status smdl_prop_phase_ms(smdl_t h, float* ms3) {
    if (!h || !ms3) return SMDL_E_ARG;
    for (int i = 0; i < 3; ++i) ms3[i] = h->prop_ms[i];
    return SMDL_OK;
}

// Host-side internals of libsmdl shared by the API translation units.
#pragma once

#include <cstdint>
#include <map>
#include <utility>
#include <string>
#include <tuple>
#include <vector>

#include "smdl_internal.h"

// Greedy-loop stopping constants (a reading of the paper, which leaves them open): stop when the
// best correlation magnitude is at most SMDL_TAU * ||y||_2, or when the chosen atom's squared
// distance to the span of the chosen ones is at most SMDL_DEP_TOL * ||d_j||^2.
constexpr float SMDL_TAU = 1e-5f;
constexpr float SMDL_DEP_TOL = 1e-5f;

// splitmix64 (Steele, Lea, Flood 2014): the host-side generator of the seeded orders the
// library draws itself (training shuffles, the seeded merge start).
struct SplitMix64 {
    uint64_t state;
    explicit SplitMix64(uint64_t seed) : state(seed) {}
    uint64_t next() {
        uint64_t z = (state += 0x9E3779B97F4A7C15ull);
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        return z ^ (z >> 31);
    }
};

// Fisher-Yates from the last position down: position i swaps with position next() % (i + 1).
template <typename T>
void seeded_shuffle(std::vector<T>& v, uint64_t seed) {
    SplitMix64 g(seed);
    for (int64_t i = (int64_t)v.size() - 1; i > 0; --i) std::swap(v[i], v[g.next() % (uint64_t)(i + 1)]);
}

struct Buf {
    void* p = nullptr;
    size_t cap = 0;
};

struct smdl_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int n_cu = 256;
    std::string err;
    std::map<std::string, Buf> bufs;
    std::map<std::tuple<int, int, int>, OmpTile> tiles;
    bool autotune = true;
    int mod_solver = 0;                         // 0 automatic, 1 multi-work-group, 2 one work group
    uint32_t flags = 0;                         // SMDL_DETERMINISTIC | SMDL_CHECK_FINITE for every call
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    bool timed_pending = false;
    float last_kernel_ms = 0.f;
    float phase_ms[3] = {0.f, 0.f, 0.f};
    hipEvent_t ev_prop[4] = {nullptr, nullptr, nullptr, nullptr};
    float prop_ms[3] = {0.f, 0.f, 0.f};

    // Host-to-device copy on the stream of host data the caller may release at once: the bytes
    // are first copied into `keep`, held until a later upload finds the stream past them, so the
    // copy never depends on when the runtime reads its source (asynchronous calls return first).
    std::vector<std::vector<uint8_t>> keep;

    void* ws(const char* name, size_t bytes);
    hipError_t upload(void* dst, const void* src, size_t bytes);
    smdl_status fail(smdl_status s, const std::string& msg);
    smdl_status hip(hipError_t e, const char* what);
};

struct SetSpec {
    const float* Y = nullptr;   // signals of the set (m each)
    const float* init = nullptr;  // initial dictionary (m x K), NULL: the first K signals
    int64_t n = 0;
    int K = 0, s = 1;
    const float* D = nullptr;   // m x K (written by learning, read by coding)
    int64_t out0 = 0;           // first output row of the set
    // filled by prepare_sets
    int Kpad = 0;
    int gld = 0;                // Gram row stride (floats)
    float4* frag = nullptr;
    float* gram = nullptr;
};

struct CodeOut {
    int32_t* idx = nullptr;
    float* coef = nullptr;
    int32_t* nnz = nullptr;
    float* res = nullptr;
    int s_stride = 1;
};

struct CodePlan {
    int m = 0, mchunks = 1, n_sets = 0, maxKpad = 64, maxS = 1, T = 16;
    void* pack_desc = nullptr;
    void* gram_desc = nullptr;
    OmpDesc* omp_desc = nullptr;
    OmpItem* items = nullptr;
    int n_items = 0;
    int* queue = nullptr;
    bool persistent = false;
    int lanes_ok = 16 | 32 | 64;   // lane counts that divide every set's Kpad / 4
    std::vector<OmpDesc> host_desc;
};

struct ModSpec {
    const float* Y;
    const int32_t* idx;
    const float* coef;
    const int32_t* nnz;
    int64_t n;
    float* D;
    int K;
    int s_stride;
};

struct ModPlan {
    int n_desc = 0, m = 0, total_atoms = 0, maxKpad = 64;
    int64_t max_n = 0;
    ModDesc* desc = nullptr;
    int32_t *cnt = nullptr, *fill = nullptr, *ptr = nullptr, *list_sig = nullptr, *status = nullptr;
    float* list_coef = nullptr;
    double *arena = nullptr, *part = nullptr;   // products workspace and its partial copies
    int64_t arena_len = 0;                      // doubles
    int chunks = 1;                             // blocks per atom in the products
    int solver = 0;                             // the handle's mod_solver
    int32_t *bcnt = nullptr, *bbase = nullptr;  // per-block counts and bases (fixed-order mode)
    std::vector<ModDesc> host_desc;
};

smdl_status check_dims(smdl_t h, int m, int K, int s);
// Take the device address of this device's fixed scratch array (the allocation-free coding
// entry point); called once per handle at creation, with the handle's device current.
smdl_status noalloc_setup(smdl_t h);
// SMDL_E_NUMERIC if any of the n floats at x (device) is not finite (synchronises the stream).
smdl_status check_finite(smdl_t h, const float* x, int64_t n, const char* what);
smdl_status check_codes(smdl_t h, const smdl_codes& X, int64_t N, int s_needed);
OmpTile default_tile(int Kpad, int s, int lanes_ok = 16 | 32 | 64);
OmpTile choose_tile(smdl_t h, int Kpad, int s, bool batched, int lanes_ok = 16 | 32 | 64);
smdl_status prepare_sets(smdl_t h, int m, std::vector<SetSpec>& sets, const char* tag, CodePlan& plan);
hipError_t enqueue_code(smdl_t h, const CodePlan& plan, OmpTile tile, const CodeOut& out, float eps,
                        bool timed);
smdl_status omp_code_impl(smdl_t h, const float* D, int m, int K, const float* Y, int64_t N, int s_max,
                          float eps, smdl_codes X, float* res_norm, const int32_t* sig_list,
                          const int32_t* list_count, int64_t list_cap, const char* tag);
smdl_status finish_timing(smdl_t h);
smdl_status autotune_plan(smdl_t h, CodePlan& plan, std::vector<SetSpec>& sets, const CodeOut& out,
                          bool batched, const char* tag);
smdl_status build_items(smdl_t h, const std::vector<SetSpec>& sets, int T, const char* tag, CodePlan& plan);

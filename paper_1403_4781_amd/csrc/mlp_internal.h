// Internal declarations of the proposer (MLP) kernels.
#pragma once

#include "smdl_internal.h"

struct GemmArgs {
    const uint16_t* A;   // bf16
    const uint16_t* B;   // bf16
    int M, N, K;
    int lda, ldb, ldc;
    const float* bias;          // optional, per output column
    const uint16_t* mask_bf16;  // optional: zero the output where mask <= 0 (ReLU backward)
    int ldmask;
    int relu;
    float* out_f32;             // optional
    uint16_t* out_bf16;         // optional
    int ksplit;                 // > 1: blockIdx.z takes K/ksplit of the reduction and adds its
                                // partial into out_f32 with atomics (out_f32 zeroed beforehand)
};

hipError_t launch_gemm(const GemmArgs& g, bool AT, bool BT, bool big, hipStream_t st);
hipError_t launch_transpose_bf16(const uint16_t* in, int rows, int cols, uint16_t* out, hipStream_t st);
hipError_t launch_zero_f32(float* p, int64_t n, hipStream_t st);
hipError_t launch_prep_input(const float* Y, int64_t B, int m, int mpad, int64_t Bpad, const int32_t* rows,
                             uint16_t* h0, hipStream_t st);
hipError_t launch_bce(const float* z, int64_t B, int64_t Bpad, int K, const int32_t* lidx, const int32_t* lnnz,
                      int ls, const int32_t* rows, float scale, float* delta, uint16_t* delta_bf,
                      double* loss_part, double* loss, hipStream_t st);
hipError_t launch_colsum(const float* x, int64_t B, int N, float* out, hipStream_t st);
hipError_t launch_adam(float* w, const float* g, float* m1, float* m2, int64_t n, int cols, int rows, float lr,
                       float b1, float b2, float eps, int t, uint16_t* wbf, uint16_t* wbfT, hipStream_t st);
hipError_t launch_to_bf16(const float* w, int64_t n, int cols, int rows, uint16_t* wbf, uint16_t* wbfT,
                          hipStream_t st);

// Proposer-restricted OMP.
struct RestrictedArgs {
    const float* D;          // m x K
    const float* gram;       // Kpad rows of gld floats
    int gld;
    int Kpad, m, K;
    const float* Y;
    int64_t N;
    const int32_t* cand;     // N x n_cand, increasing atom order
    int n_cand, s;
    float eps_fb, tau, dep_tol;
    int32_t* idx;
    float* coef;
    int32_t* nnz;
    int s_out;
    uint8_t* fell_back;      // optional
    int32_t* fb_list;        // N capacity
    int32_t* fb_count;       // device counter (zeroed before launch)
};

hipError_t launch_topk(const float* logits, int64_t N, int K, int n_cand, int32_t* cand, hipStream_t st);
hipError_t launch_restricted_omp(const RestrictedArgs& a, hipStream_t st);

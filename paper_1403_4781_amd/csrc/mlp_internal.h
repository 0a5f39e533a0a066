// Internal declarations of the proposer (MLP) kernels.
#pragma once

#include "smdl_internal.h"

// C[M x N] = A[M x K] B[N x K]^T (BF16, FP32 accumulation) with a fused epilogue, applied in
// this order: + bias[col]; BCE (when tmask is set: the value is the logit z of batch row `row`,
// target bit col of tmask[rows[row]], replaced by (sigmoid(z) - t) * scale, loss terms added to
// *loss); ReLU; ReLU-backward mask (zero where mask <= 0); zero for rows >= Mvalid.  Then the
// value is stored as FP32 (rows < Mvalid only) and/or BF16 [M x N] (ld = ldo), BF16 transposed [N x M] (ld = ldt),
// and summed per column over each 32-row block into colpart[M / 32][N].
// M % 32 == 0, K % 32 == 0, N % 4 == 0, lda / ldb multiples of 8.
struct NtArgs {
    const uint16_t* A;
    const uint16_t* B;
    int lda, ldb;
    int M, N, K;
    int Mvalid;
    const float* bias;
    int relu;
    const uint16_t* mask;
    int ldmask;
    const uint32_t* tmask;      // label bitmask rows of (K + 31) / 32 words
    int tstride;
    const int32_t* rows;        // sample of each batch row (NULL: row itself)
    float scale;
    double* loss;
    float* out_f32;
    uint16_t* out_bf16;
    int ldo;
    uint16_t* outT;
    int ldt;
    float* colpart;
};

// One layer of the grouped weight-gradient launch.
struct WgLayer {
    const uint16_t* dT;       // [wo x Bpad] BF16 deltas of the layer output, transposed
    const uint16_t* hT;       // [wi x Bpad] BF16 layer input, transposed
    const float* colpart;     // [nparts x wo] column sums of the FP32 deltas
    int nparts;
    int wo, wi;
    float *W, *b, *mW, *vW, *mb, *vb;   // Adam: FP32 masters and moments
    uint16_t *Wbf, *WbfT;               // Adam: BF16 copies (wo x wi) and (wi x wo)
    float *dW_out, *db_out;             // gradient-only mode
    int tile0, ntn;                     // set by the launcher
};

struct WgArgs {
    WgLayer L[4];
    int n_layers;
    int Bpad;
    int bias_block0;          // set by the launcher
    int adam;
    float lr, b1, b2, eps;
    const int32_t* t_dev;     // Adam: steps taken before this launch's epoch (device) ...
    int t_off;                // ... plus this: the step number t of the bias corrections
};

hipError_t launch_gemm_nt(const NtArgs& g, hipStream_t st);
hipError_t launch_wgrad(WgArgs& g, hipStream_t st);
hipError_t launch_prep(const float* Y, int64_t B, int m, int64_t Bpad, const int32_t* rows, uint16_t* h0,
                       uint16_t* h0T, hipStream_t st);
hipError_t launch_label_mask(const int32_t* idx, const int32_t* nnz, int ls, int64_t N, int K, uint32_t* mask,
                             hipStream_t st);
hipError_t launch_zero_f64(double* p, int64_t n, hipStream_t st);
hipError_t launch_add_i32(int32_t* p, int32_t v, hipStream_t st);
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

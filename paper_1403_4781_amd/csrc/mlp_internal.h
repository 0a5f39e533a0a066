// Internal declarations of the proposer (MLP) kernels.
#pragma once

#include "smdl_internal.h"

// BF16 matrices marked "fragment order" are stored as the operands of v_mfma_f32_16x16x32_bf16
// are loaded: an [N x K] matrix in kilobyte blocks of 16 rows x 32 columns, blocks ordered by
// row block then column block, lane l = (n % 16) + 16 ((k % 32) / 8) of a block holding the 8
// consecutive entries of row n from k - k % 8.  N % 16 == 0, K % 32 == 0.
//
// C[M x N] = A[M x K] B[N x K]^T (BF16, FP32 accumulation; A and B in fragment order) with a
// fused epilogue, applied in this order: + bias[col]; BCE (when tmask is set: the value is the
// logit z of batch row `row`, target bit col of tmask[rows[row]], replaced by (sigmoid(z) - t) *
// scale, loss terms added to *loss); ReLU; ReLU-backward mask (zero where mask <= 0; mask is
// [M x ldmask] in fragment order, ldmask = N); zero for rows >= Mvalid.  Then the value is
// stored as FP32 row-major (ld = ldo, rows < Mvalid only) and/or BF16 [M x N] in fragment order
// (ldo = N), BF16 transposed [N x M] in fragment order, and summed per column over each 32-row
// block into colpart[M / 32][N].  M, N and K multiples of 32.  Products with at least 256 tiles
// of 64 x 64 (M and N multiples of 64) take 64 x 64 tiles, the others 32 x 32.
struct NtArgs {
    const uint16_t* A;
    const uint16_t* B;
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
    float* colpart;
};

// One layer of the grouped weight-gradient launch.
struct WgLayer {
    const uint16_t* dT;       // [wo x Bpad] BF16 deltas of the layer output, fragment order
    const uint16_t* hT;       // [wi x Bpad] BF16 layer input, fragment order
    const float* colpart;     // [nparts x wo] column sums of the FP32 deltas
    int nparts;
    int wo, wi;
    float *W, *b, *mW, *vW, *mb, *vb;   // Adam: FP32 masters and moments
    uint16_t *Wpk, *WTpk;               // Adam: BF16 W (wo x wi) and W^T (wi x wo), fragment order
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

// The whole network on R batch rows per work group (R = 16, 32 or 64; every width a multiple of
// 32, the input width m a multiple of 4 and at most SMDL_MAX_M): y / ||y|| -> hidden layers ->
// output layer, every activation kept in LDS as BF16.  Inference (logits set): FP32 logits of
// the valid rows.  Training (tmask set): the BCE deltas of the output layer, then the deltas of
// every hidden layer back to the first (ReLU masks from the stored activations), each also
// written transposed (hT, dT) with its per-block column sums (colpart, Bpad / R parts) for the
// weight-gradient launch; loss terms added to *loss.
struct RowsArgs {
    const float* Y;
    int64_t B;                  // valid rows
    int64_t Bpad;               // multiple of R
    const int32_t* rows;        // sample of each batch row (NULL: row itself)
    int n_layers;
    int w[5];
    const uint16_t* W[4];       // [w[l+1] x w[l]] BF16, fragment order
    const uint16_t* WT[4];      // [w[l] x w[l+1]] BF16, fragment order
    const float* bias[4];
    float* logits;              // inference: [B x w[L]]
    const uint32_t* tmask;      // training: label bitmask rows of tstride words
    int tstride;
    float scale;
    double* loss;
    uint16_t* hT[4];            // [w[l] x Bpad], fragment order
    uint16_t* dT[4];            // [w[l+1] x Bpad], fragment order
    float* colpart[4];          // [Bpad / R x w[l+1]]
};

// Rows per work group of the fused network kernel for these widths, 0 (the per-layer path) when
// the activations of 16 rows do not fit in LDS, a width is unsupported, or, for a training
// batch, the network has at least 3 * 2^18 weights.  Inference keeps only two activation
// buffers and takes 64 rows where they fit, else 32 (fewer weight reads per row over many work
// groups); a training batch keeps every layer's activations and takes 16 (twice the work groups on
// the chip, half the serial matrix work in each).
int mlp_rows_per_block(int n_layers, const int* widths, bool train);
hipError_t launch_mlp_rows(const RowsArgs& a, int R, hipStream_t st);

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
    const float4* dfrag;     // the packed dictionary fragments of the plain OMP kernel (alpha0)
    int mchunks;             // 64-row chunks of m
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

/*
 * smdl.h -- C ABI of the MI355X (gfx950) split-and-merge dictionary-learning library.
 *
 * Method: S. Mukherjee, C. S. Seelamantula, "A split-and-merge dictionary learning algorithm
 * for sparse representation" (arXiv 1403.4781).  The library computes
 *   - OMP sparse coding of signals against a dictionary (Section 1; error-constrained form in
 *     Section 3.2.2; cost discussion in Appendix B),
 *   - the MOD least-squares dictionary update (Section 1),
 *   - the standard alternation of the two (Section 1, Section 3.1) and Algorithm 1 (Section 2),
 *   - a learned support proposer that restricts OMP to candidate atoms, with full OMP as the
 *     fallback whenever the restricted code misses the residual target.
 *
 * Conventions (every entry point):
 *   - Arrays are DEVICE pointers (hipMalloc'd memory or torch CUDA tensors on the handle's
 *     device) unless the parameter comment says "host".
 *   - Matrices are FP32, column-major with leading dimension = number of rows:
 *       Y (m x N): signal n is Y[n*m .. n*m + m);  D (m x K): atom k is D[k*m .. k*m + m).
 *   - Sparse codes use the ELL layout of smdl_codes: row n holds the selected atoms of signal n
 *     in selection order in idx[n*s_max + i], their coefficients in coef[n*s_max + i] for
 *     i < nnz[n]; unused slots hold idx = -1 and coef = 0.
 *   - The caller owns every buffer passed in.  The handle owns its scratch memory (grown on
 *     demand, never shrunk) and frees it in smdl_destroy.
 *   - Every call returns an smdl_status; no C++ exception crosses the ABI.  All argument checks
 *     run on the host before any GPU work.  On failure the message is in smdl_last_error(h).
 *   - Calls are synchronous: work is queued on the handle's stream, which is created with
 *     default flags and therefore ordered after work already queued on the device's legacy
 *     default stream, and the call returns after that stream has finished.
 *   - One handle per host thread; a handle is not safe for concurrent use.
 *
 * Limits: 1 <= m <= 256, 1 <= K <= 1024, 1 <= s_max <= 16 (OMP); s_max <= min(m, K).
 */
#ifndef SMDL_H
#define SMDL_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct smdl_ctx* smdl_t;
typedef struct smdl_prop* smdl_prop_t;

typedef enum {
    SMDL_OK = 0,
    SMDL_E_ARG = -1,          /* null pointer, negative size, inconsistent arguments        */
    SMDL_E_SHAPE = -2,        /* sizes outside the supported limits                          */
    SMDL_E_UNSUPPORTED = -3,  /* a combination no kernel is built for                        */
    SMDL_E_NOMEM = -4,        /* device allocation failed                                    */
    SMDL_E_HIP = -5,          /* a HIP runtime call failed (message names it)                */
    SMDL_E_NUMERIC = -6,      /* FP64 Cholesky of the MOD normal equations failed after the
                                 ridge retry, or (SMDL_CHECK_FINITE) a non-finite input      */
    SMDL_E_STATE = -7         /* handle or proposer in an unusable state                     */
} smdl_status;

/* ELL sparse codes (N rows of s_max slots). */
typedef struct {
    int32_t* idx;
    float* coef;
    int32_t* nnz;
    int32_t s_max;
} smdl_codes;

/* Create a handle bound to HIP device `device`.  stream: a hipStream_t to use, or NULL to let
   the handle create its own (default flags). */
smdl_status smdl_create(smdl_t* h, int device, void* stream);
void smdl_destroy(smdl_t h);
/* Message of the last failing call on h (empty string if none); valid until the next call. */
const char* smdl_last_error(smdl_t h);
/* Number of entry points exported (for load checks) and library version string. */
int smdl_version(void);

/* ---------------------------------------------------------------------------------------- */
/* Sparse coding                                                                            */
/* ---------------------------------------------------------------------------------------- */

/*
 * Gram matrix G = D^T D of a dictionary (the inner products every OMP step reuses; Appendix B
 * counts OMP as O(smKn), which presumes them).  D: m x K; G: K x K, written row-major (equal to
 * column-major: G is symmetric).  FP32 accumulation on the matrix cores.
 */
smdl_status smdl_gram(smdl_t h, const float* D, int m, int K, float* G);

/*
 * Orthogonal matching pursuit of N signals (Section 1; Definition 1 is the output contract).
 *   D (m x K, unit-norm atoms expected), Y (m x N).
 *   s_max: at most s_max atoms per signal (sparsity-constrained form); X.s_max >= s_max.
 *   eps  : if > 0, also stop as soon as ||y - D x||_2 <= eps (error-constrained form of
 *          Section 3.2.2, tested before every pick, so ||y|| <= eps gives the empty code).
 *   Each step picks the unchosen atom of largest |d_k^T r| (lowest k on exact ties) and
 *   re-fits all chosen coefficients by least squares.  The greedy loop also stops when the
 *   best |d_k^T r| <= 1e-5 ||y||_2 or when the chosen atom is numerically in the span of
 *   those already chosen (squared distance <= 1e-5 ||d_j||^2).
 *   res_norm: optional (N floats): ||y - D x||_2 per signal.
 */
smdl_status smdl_omp_code(smdl_t h, const float* D, int m, int K, const float* Y, int64_t N,
                          int s_max, float eps, smdl_codes X, float* res_norm);

/*
 * smdl_omp_code for callers that cannot allocate device memory (code under HIP graph capture,
 * serving loops, harnesses that forbid hipMalloc): the same coding, the same arguments and
 * results, but no allocation of any kind.  Its scratch memory (packed dictionary, Gram matrix,
 * launch descriptors: 6 MiB + 8 KiB, enough for the library's largest dictionary, m <= 256 and
 * K <= 1024) is one fixed array per GPU, held until the process ends; its address is taken when
 * a handle is created on that GPU.  Larger shapes return SMDL_E_SHAPE.  The tile is the
 * handle's current choice for the shape (smdl_tune / smdl_set_tile, or the default); nothing is
 * autotuned here.  All calls on one GPU share the array: calls that overlap on one GPU (two
 * threads, two streams) race and must be serialised by the caller.  Each call rewrites every
 * part of the scratch it reads.  While the handle's stream is being captured into a HIP graph
 * the call only records its work (no synchronisation); otherwise it returns when it is done.
 */
smdl_status smdl_omp_code_noalloc(smdl_t h, const float* D, int m, int K, const float* Y, int64_t N,
                                  int s_max, float eps, smdl_codes X, float* res_norm);

/* ---------------------------------------------------------------------------------------- */
/* Dictionary update                                                                        */
/* ---------------------------------------------------------------------------------------- */

/*
 * MOD update (Section 1): D <- Y X^T (X X^T)^{-1} for the atoms used by at least one signal,
 * products accumulated in FP64 and solved by FP64 Cholesky; a rejected pivot
 * (d <= 1e-12 A_kk) triggers one retry with A + 1e-10 max(diag A) I, else SMDL_E_NUMERIC.
 * Unused atoms keep their input value.  Every atom with nonzero norm is then scaled to unit
 * length.  D is in/out (m x K).  n_unused: optional host int32 (number of unused atoms).
 */
smdl_status smdl_mod_update(smdl_t h, const float* Y, int m, int64_t N, smdl_codes X, int K,
                            float* D, int32_t* n_unused);

/* ---------------------------------------------------------------------------------------- */
/* Learning                                                                                 */
/* ---------------------------------------------------------------------------------------- */

/*
 * The standard alternation on one data set (Section 1; initialisation of Section 3.1):
 * D = unit-normalised first K columns of Y (zero columns stay zero), then iters x
 * { X = OMP(D, Y, s); D = MOD(Y, X, D) }, then X_out = OMP(D, Y, s) if X_out.idx != NULL.
 * Requires N >= K.  D_out: m x K.
 */
smdl_status smdl_learn(smdl_t h, const float* Y, int m, int64_t N, int K, int s, int iters,
                       float* D_out, smdl_codes X_out);

/* The same alternation started from a given dictionary D_init (device m x K, unit-normalised
 * before the first coding; it may be D_out itself) instead of the first K signals (for example
 * the overcomplete DCT of Section 3.2.1).  N >= 1. */
smdl_status smdl_learn_init(smdl_t h, const float* Y, int m, int64_t N, int K, int s, int iters,
                            const float* D_init, float* D_out, smdl_codes X_out);

/* Subsets of Algorithm 1, step 1.  Subset t is the signals perm[offsets[t] .. offsets[t+1]). */
typedef struct {
    int L;                       /* number of subsets, >= 1                                  */
    const int64_t* perm;         /* device, N entries: a permutation of 0..N-1; NULL = identity */
    const int64_t* offsets;      /* host, L+1 entries, offsets[0] = 0, offsets[L] = N,
                                    non-decreasing; subset t needs offsets[t+1]-offsets[t] >= K_local[t] */
    const int32_t* K_local;      /* host, L entries: atoms of local dictionary t (1..1024)    */
    const int32_t* s_local;      /* host, L entries: local sparsity (1..16)                   */
} smdl_subsets;

#define SMDL_PER_SUBSET_LAUNCH 1u   /* launch each subset's kernels separately (comparison)  */
#define SMDL_NO_GRAPH 2u            /* do not capture/replay the iteration as a HIP graph    */
#define SMDL_COMPOSE_CODES 4u       /* X_out = the Proposition 1 composition Z X1 (see below)
                                       instead of a fresh OMP of all N signals               */
#define SMDL_DETERMINISTIC 8u       /* MOD products accumulated in a fixed order (per-atom lists
                                       in signal order, each column of X X^T summed by one
                                       thread), so that repeated runs give the same bits      */
#define SMDL_CHECK_FINITE 16u       /* reject non-finite signals with SMDL_E_NUMERIC before any
                                       other work                                            */
#define SMDL_ASYNC 32u              /* handle option (smdl_set_flags): smdl_omp_code,
                                       smdl_omp_code_noalloc, smdl_gram and smdl_prop_logits
                                       return once their work is queued on the handle's stream
                                       (see smdl_set_flags)                                  */

typedef struct {
    int iters_local;   /* alternations on every subset (step 2)                               */
    int iters_merge;   /* alternations of the merge (step 3)                                  */
    int s_merge;       /* sparsity of the merge (step 3, s2)                                  */
    int s_final;       /* sparsity of the final coding of all N signals                       */
    uint32_t flags;    /* SMDL_PER_SUBSET_LAUNCH | SMDL_NO_GRAPH | SMDL_COMPOSE_CODES |
                          SMDL_DETERMINISTIC | SMDL_CHECK_FINITE                               */
    const float* D_local_init;  /* device m x max_t K_local[t], or NULL: subset t starts from the
                                   first K_local[t] columns of this matrix (unit-normalised) instead
                                   of its first K_local[t] signals                               */
    const float* D_merge_init;  /* device m x K, or NULL: the merge starts from this dictionary
                                   (unit-normalised) instead of the first K pooled columns       */
    uint64_t merge_seed;        /* 0: the merge starts from the first K pooled columns (subset
                                   order).  Otherwise from the first K columns of a random
                                   permutation of the pooled columns: Fisher-Yates from the last
                                   position down, position i swapped with position
                                   (splitmix64 draw) mod (i + 1), splitmix64 seeded with this
                                   value (Steele, Lea, Flood 2014: state += 0x9E3779B97F4A7C15,
                                   then the variant-13 finaliser).  Ignored with D_merge_init.  */
    smdl_codes X_local;         /* optional (idx == NULL: not wanted): receives the final local
                                   codes X^(t) of step 2 (the codes of the returned local
                                   dictionaries), N rows in split order (row offsets[t] + i is
                                   signal i of subset t), local atom ids; X_local.s_max must be
                                   >= max_t s_local[t] and <= 16                              */
} smdl_learn_opts;

/*
 * Algorithm 1 (Section 2):
 *   1. split: subset t = Y[:, perm[offsets[t]:offsets[t+1]]] (the random permutation is an input);
 *   2. on every subset, the standard alternation (smdl_learn) with K_local[t] atoms and sparsity
 *      s_local[t]; X^(t) = that run's final codes;
 *   3. pooled data Ytilde = [ ||X^(1)||_F D^(1), ..., ||X^(L)||_F D^(L) ] (m x sum K_t);
 *      the standard alternation on Ytilde with K atoms, sparsity s_merge, iters_merge
 *      iterations (initialised with the first K pooled columns), giving D;
 *   then X_out = OMP(D, Y, s_final) for all N signals in their original order
 *   (skipped when X_out.idx == NULL).
 * All subsets of one class of work run in one kernel launch per stage; one local iteration is
 * captured once as a HIP graph and replayed (unless SMDL_NO_GRAPH).
 * D_out: m x K.  D_local_out: optional m x sum(K_t) (the unscaled local dictionaries).
 * scales_out: optional host double[L], the scales ||X^(t)||_F.
 */
smdl_status smdl_split_merge_learn(smdl_t h, const float* Y, int m, int64_t N,
                                   const smdl_subsets* sub, int K, const smdl_learn_opts* o,
                                   float* D_out, smdl_codes X_out, float* D_local_out,
                                   double* scales_out);

/*
 * Proposition 1 (proof in Appendix A) applied to the codes of Algorithm 1.  A signal of subset t
 * with local code x1 (over D^(t)) is represented over the merged D by
 *     r = sum_i (x1_i / c_t) z_{a_i},
 * where a_i = sum_{u<t} K_local[u] + (local atom of entry i) is its pooled column of
 * Ytilde = [c_1 D^(1), ..., c_L D^(L)], z_a that column's merge code and c_t = ||X^(t)||_F.
 * At most X1.s_max * Z.s_max atoms; equal atoms are added (FP64); distinct atoms in order of
 * first occurrence (local entry, then merge entry); unused slots (-1, 0).
 *   X1: device, N rows in split order (position p of subset t = offsets[t] + ...), local atom ids
 *   Z:  device, sum(K_local) rows (pooled columns, subsets in order), atom ids of D (0..K-1)
 *   scales: host double[L];  sub: L, offsets (host), K_local (host), perm (device, position p ->
 *   output row perm[p]; NULL = identity); s_local is not read.
 *   X_out: device, N rows; X1.s_max * Z.s_max <= X_out.s_max <= 64.
 * smdl_split_merge_learn with SMDL_COMPOSE_CODES runs this on its own local codes (the final codes
 * of step 2) and merge codes (a final coding of Ytilde with D), in place of the fresh coding;
 * s_final is then unused and X_out.s_max must be in [max_t s_local[t] * s_merge, 64].
 */
smdl_status smdl_compose_codes(smdl_t h, int64_t N, const smdl_subsets* sub, smdl_codes X1, smdl_codes Z,
                               int K, const double* scales, smdl_codes X_out);

/*
 * Image denoising (Section 3.2.2).  Every p x p patch of the H x W image (row-major, device;
 * stride 1 in both directions: (H - p + 1)(W - p + 1) patches, patch pixel (r, c) at index
 * r p + c) is coded by the error-constrained OMP ||y - D x||_2 <= eps (eps > 0, at most s_max
 * atoms) against D (device, m x K column-major, m = p * p <= 256); out (device H x W) receives
 * the mean of the overlapping patch estimates D x at every pixel.  The paper takes
 * eps = 8.5 sigma for noise of standard deviation sigma.
 */
smdl_status smdl_denoise(smdl_t h, const float* img, int H, int W, int p, const float* D, int K, float eps,
                         int s_max, float* out);

/* ---------------------------------------------------------------------------------------- */
/* Learned support proposer                                                                 */
/* ---------------------------------------------------------------------------------------- */

/*
 * An MLP widths[0] -> widths[1] -> ... -> widths[n_layers] with ReLU between layers, mapping
 * y / ||y||_2 to one logit per atom (widths[0] = m, widths[n_layers] = K).  Weights W_l are
 * (widths[l+1] x widths[l]) row-major FP32 masters with a BF16 copy used by the GEMMs; biases
 * FP32.  Rounding points: the input and every hidden activation are rounded to BF16 before
 * the next GEMM; accumulation is FP32; logits are FP32.
 * W_init, b_init: host arrays per layer (copied).  Limits: 1..4 layers, widths multiples of 32
 * in [32, 4096], widths[0] <= 256, widths[n_layers] <= 1024.
 */
smdl_status smdl_prop_create(smdl_t h, int n_layers, const int* widths,
                             const float* const* W_init, const float* const* b_init,
                             smdl_prop_t* p);
smdl_status smdl_prop_destroy(smdl_prop_t p);

/*
 * smdl_prop_create with seeded Kaiming-uniform initial weights: W_l entries drawn from
 * U(-sqrt(6/widths[l]), sqrt(6/widths[l])), b_l entries from U(-1/sqrt(widths[l]),
 * 1/sqrt(widths[l])).  The uniforms are u = (z >> 11) * 2^-53 of consecutive splitmix64 outputs
 * z (state = seed), used in the order W_0 (row-major), b_0, W_1, b_1, ...; each value is
 * lo + (hi - lo) u computed in FP64 and rounded to FP32.  Same limits and errors as
 * smdl_prop_create.
 */
smdl_status smdl_prop_create_seeded(smdl_t h, int n_layers, const int* widths, uint64_t seed,
                                    smdl_prop_t* p);

/* Copy the FP32 master weights and biases out to host arrays (one per layer). */
smdl_status smdl_prop_get(smdl_t h, smdl_prop_t p, float* const* W_host, float* const* b_host);

/*
 * Replace the weights and biases (host arrays per layer, shapes as at creation, copied) and
 * restart training: the Adam moments and step count are reset to zero and the BF16 copies
 * rebuilt.  Synchronous.  SMDL_E_STATE if p belongs to another handle.
 */
smdl_status smdl_prop_set(smdl_t h, smdl_prop_t p, const float* const* W_host, const float* const* b_host);

/* Logits (N x K, row n = signal n) of the network for signals Y (m x N). */
smdl_status smdl_prop_logits(smdl_t h, smdl_prop_t p, const float* Y, int64_t N, float* logits);

/*
 * Mean binary cross-entropy with logits over the N x K outputs against the multi-hot targets
 * t[n, k] = [k in support of signal n] given by `labels` (ELL), and its gradients.
 * Backward rounding points: delta = (sigmoid(z) - t)/(N K) in FP32, BF16-rounded as a GEMM
 * operand; bias gradients use the unrounded delta.
 * loss: host float.  dW, db: device FP32 arrays per layer (same shapes as W_l, b_l).
 */
smdl_status smdl_prop_grad(smdl_t h, smdl_prop_t p, const float* Y, int64_t N, smdl_codes labels,
                           float* loss, float* const* dW, float* const* db);

typedef struct {
    int epochs;         /* passes over the data                                           */
    int batch;          /* minibatch size (the last partial batch is dropped), >= 16       */
    float lr, beta1, beta2, adam_eps;
    uint64_t shuffle_seed;  /* 0 = no shuffling (batches in signal order)                  */
} smdl_train_opts;

/*
 * Train the proposer with Adam (bias-corrected) on (signal, support) pairs: every minibatch
 * runs forward, BCE gradient, backward and one Adam step on the FP32 masters, all on the GPU.
 * loss_per_epoch: optional host float[epochs] (mean minibatch loss of each epoch).
 */
smdl_status smdl_prop_train(smdl_t h, smdl_prop_t p, const float* Y, int64_t N, smdl_codes labels,
                            const smdl_train_opts* o, float* loss_per_epoch);

/*
 * Proposer-restricted OMP with full-OMP fallback:
 *   C = the n_cand atoms of largest logit (lower atom index first on equal logits);
 *   x = OMP restricted to the atoms of C (same rules as smdl_omp_code, sparsity s_max);
 *   if ||y - D x||_2 > eps_fallback (explicit FP32 residual): x = OMP(D, y, s_max), full.
 * fell_back: optional device uint8[N]; n_fallback: optional host int64 (count).
 * cand_out: optional device int32[N x n_cand] (the candidate sets, increasing atom order).
 * Limits: n_cand <= 64, n_cand >= s_max.
 */
smdl_status smdl_omp_code_proposed(smdl_t h, smdl_prop_t p, const float* D, int m, int K,
                                   const float* Y, int64_t N, int s_max, int n_cand,
                                   float eps_fallback, smdl_codes X, uint8_t* fell_back,
                                   int64_t* n_fallback, int32_t* cand_out);

/* GPU time (ms) of the last smdl_omp_code_proposed: network + top-k, restricted OMP, fallback. */
smdl_status smdl_prop_phase_ms(smdl_t h, float* ms3);

/* ---------------------------------------------------------------------------------------- */
/* Tuning                                                                                   */
/* ---------------------------------------------------------------------------------------- */

/*
 * Tile choice of the OMP kernel for a dictionary shape: lanes per signal (16, 32 or 64) and
 * signals per work item (16, 32 or 64).  smdl_tune times every candidate that fits (m, K, s)
 * on the given data and keeps the fastest in the handle (later calls use it).
 * smdl_get_tile reports the current choice (host out-params).
 */
smdl_status smdl_tune(smdl_t h, const float* D, int m, int K, const float* Y, int64_t N, int s_max);
smdl_status smdl_get_tile(smdl_t h, int m, int K, int s_max, int* lanes_per_signal,
                          int* signals_per_item);

/* Force a tile for (K, s_max) (lanes 16/32/64; signals per item 16/32/64). */
smdl_status smdl_set_tile(smdl_t h, int K, int s_max, int lanes_per_signal, int signals_per_item);
/*
 * Factorisation of the MOD normal equations (the FP64 Cholesky solve of the update of Section 1):
 * 0 (default) picks by the number of dictionaries in the call, 1 forces the multi-work-group
 * panel factorisation (two launches per 32 columns), 2 one work group per dictionary.  Both give
 * the same dictionaries up to rounding.  SMDL_E_ARG for another mode.
 */
smdl_status smdl_set_mod_solver(smdl_t h, int mode);
/*
 * Options of every later call on the handle: SMDL_DETERMINISTIC (MOD products in a fixed order,
 * for smdl_mod_update, smdl_learn* and smdl_split_merge_learn), SMDL_CHECK_FINITE (the input
 * signals, and for smdl_omp_code the dictionary, are checked first; a NaN or infinity returns
 * SMDL_E_NUMERIC and nothing else runs) and SMDL_ASYNC.  0 clears them.  SMDL_E_ARG for any
 * other bit.  smdl_split_merge_learn uses these bits OR-ed with smdl_learn_opts.flags.
 * SMDL_ASYNC: smdl_omp_code, smdl_omp_code_noalloc, smdl_gram and smdl_prop_logits return as soon
 * as their work is queued on the handle's stream (the other calls stay synchronous).  Their device
 * outputs are valid once the caller has synchronised that stream; the inputs must stay unchanged
 * until then; an error inside the queued kernels is reported by the next call that synchronises.
 * An autotuning first call of a shape, and a SMDL_CHECK_FINITE check, still synchronise.
 * smdl_last_kernel_ms waits for the timed launch.
 */
smdl_status smdl_set_flags(smdl_t h, uint32_t flags);
/* Enable (default) or disable automatic tuning on the first learning call of a shape. */
smdl_status smdl_set_autotune(smdl_t h, int enabled);
/* Wall time (ms) of the last smdl_split_merge_learn: local phase, merge phase, final coding. */
smdl_status smdl_phase_ms(smdl_t h, float* ms3);

/* Average duration (ms) of the last OMP kernel launch of the last smdl_omp_code /
   smdl_split_merge_learn final coding on the handle's stream, measured with HIP events. */
smdl_status smdl_last_kernel_ms(smdl_t h, float* ms);

#ifdef __cplusplus
}
#endif

#endif /* SMDL_H */

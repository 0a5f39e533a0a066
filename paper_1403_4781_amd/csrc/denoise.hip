// Image denoising (Section 3.2.2): every p x p patch of the noisy image (stride 1 in both
// directions) is coded by the error-constrained OMP, ||y - D x||_2 <= eps, against a learned
// dictionary; the denoised image is the average of the overlapping patch estimates D x.
#include <algorithm>

#include "smdl_api_internal.h"

namespace {

// patches[q][r p + c] = img[(pi + r) W + pj + c] for patch q = pi PW + pj (PW = W - p + 1).
__global__ void extract_patches_kernel(const float* __restrict__ img, int H, int W, int p,
                                       float* __restrict__ patches) {
    const int PW = W - p + 1, PH = H - p + 1, m = p * p;
    const int64_t total = (int64_t)PH * PW * m;
    for (int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; f < total;
         f += (int64_t)gridDim.x * blockDim.x) {
        const int e = (int)(f % m);
        const int64_t q = f / m;
        const int pi = (int)(q / PW), pj = (int)(q % PW);
        patches[f] = img[(int64_t)(pi + e / p) * W + pj + e % p];
    }
}

// est[q][e] = sum_i coef[q][i] D[idx[q][i]][e]: one wave per patch, lanes over the m entries.
__global__ __launch_bounds__(256) void patch_estimates_kernel(const int32_t* __restrict__ idx,
                                                              const float* __restrict__ coef,
                                                              const int32_t* __restrict__ nnz, int s,
                                                              const float* __restrict__ D, int m, int K,
                                                              int64_t P, float* __restrict__ est) {
    const int64_t q = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (q >= P) return;
    const int k = std::min(std::max(nnz[q], 0), s);
    for (int e = lane; e < m; e += 64) {
        float v = 0.f;
        for (int i = 0; i < k; ++i) {
            const int a = idx[q * s + i];
            if (a >= 0 && a < K) v = fmaf(coef[q * s + i], D[(int64_t)a * m + e], v);
        }
        est[q * m + e] = v;
    }
}

// out[i][j] = mean of est[q][(i - pi) p + (j - pj)] over the patches (pi, pj) covering pixel
// (i, j), summed in FP64 in order of pi, then pj.
__global__ void average_patches_kernel(const float* __restrict__ est, int H, int W, int p,
                                       float* __restrict__ out) {
    const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= (int64_t)H * W) return;
    const int i = (int)(f / W), j = (int)(f % W);
    const int PW = W - p + 1, PH = H - p + 1;
    const int i0 = std::max(0, i - p + 1), i1 = std::min(i, PH - 1);
    const int j0 = std::max(0, j - p + 1), j1 = std::min(j, PW - 1);
    double sum = 0.0;
    int cnt = 0;
    for (int pi = i0; pi <= i1; ++pi)
        for (int pj = j0; pj <= j1; ++pj) {
            sum += est[((int64_t)pi * PW + pj) * p * p + (i - pi) * p + (j - pj)];
            ++cnt;
        }
    out[f] = cnt ? (float)(sum / cnt) : 0.f;
}

}  // namespace

extern "C" smdl_status smdl_denoise(smdl_t h, const float* img, int H, int W, int p, const float* D, int K,
                                    float eps, int s_max, float* out) {
    if (!h) return SMDL_E_ARG;
    h->err.clear();
    if (!img || !D || !out) return h->fail(SMDL_E_ARG, "null pointer");
    if (p < 1 || p * p > SMDL_MAX_M) return h->fail(SMDL_E_SHAPE, "patch side p must satisfy p * p <= 256");
    if (H < p || W < p) return h->fail(SMDL_E_SHAPE, "the image must be at least p x p");
    if (!(eps > 0.f)) return h->fail(SMDL_E_ARG, "eps must be > 0 (error-constrained coding)");
    const int m = p * p;
    smdl_status st = check_dims(h, m, K, s_max);
    if (st != SMDL_OK) return st;
    const int64_t P = (int64_t)(H - p + 1) * (W - p + 1);
    if (P * m > INT32_MAX) return h->fail(SMDL_E_SHAPE, "image too large");
    (void)hipSetDevice(h->device);
    float* patches = (float*)h->ws("dn.patches", (size_t)P * m * 4);
    float* est = (float*)h->ws("dn.est", (size_t)P * m * 4);
    smdl_codes X;
    X.idx = (int32_t*)h->ws("dn.idx", (size_t)P * s_max * 4);
    X.coef = (float*)h->ws("dn.coef", (size_t)P * s_max * 4);
    X.nnz = (int32_t*)h->ws("dn.nnz", (size_t)P * 4);
    X.s_max = s_max;
    if (!patches || !est || !X.idx || !X.coef || !X.nnz) return h->fail(SMDL_E_NOMEM, "workspace allocation failed");
    const unsigned g = (unsigned)std::min<int64_t>(8192, (P * m + 255) / 256);
    hipLaunchKernelGGL(extract_patches_kernel, dim3(g), dim3(256), 0, h->stream, img, H, W, p, patches);
    if ((st = h->hip(hipGetLastError(), "patches")) != SMDL_OK) return st;
    if ((st = omp_code_impl(h, D, m, K, patches, P, s_max, eps, X, nullptr, nullptr, nullptr, 0, "dn")) != SMDL_OK)
        return st;
    hipLaunchKernelGGL(patch_estimates_kernel, dim3((unsigned)((P + 3) / 4)), dim3(256), 0, h->stream, X.idx, X.coef,
                       X.nnz, s_max, D, m, K, P, est);
    if ((st = h->hip(hipGetLastError(), "estimates")) != SMDL_OK) return st;
    hipLaunchKernelGGL(average_patches_kernel, dim3((unsigned)(((int64_t)H * W + 255) / 256)), dim3(256), 0, h->stream,
                       est, H, W, p, out);
    if ((st = h->hip(hipGetLastError(), "average")) != SMDL_OK) return st;
    return h->hip(hipStreamSynchronize(h->stream), "denoise");
}

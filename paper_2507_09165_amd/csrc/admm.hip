// Elementwise steps of the three-step ADMM for SDP (Section 4.2) whose
// constraint map is the diagonal, A X = diag(X) (then A A^T = I): the Max-Cut
// family the paper's test instances belong to. The projection step between
// them is the library's projection.
//
//   y = b / sigma - diag(X / sigma + S - C)       (dual step)
//   W = C - Diag(y) - X / sigma                    (the matrix to project)
//   S = Pi(W)                                      (psdproj_project*)
//   X = X + sigma (S + Diag(y) - C)                (primal step)
//
// Both kernels read and write whole FP32 matrices once (HBM-bound). The
// primal kernel also forms the residual sums of the stopping test in FP64,
// per workgroup in a fixed order, and a one-workgroup kernel adds the
// workgroup sums in order (no floating-point atomics).
#include "../../include/psdproj.h"
#include "common.hpp"

namespace psd {
namespace {

constexpr int kAdmmThreads = 256;
constexpr int kAdmmGroups = PSDPROJ_ADMM_GROUPS;  // workgroups of the primal kernel
constexpr int kAdmmParts = 4;                     // sums per workgroup

// One column per blockIdx.y, rows over blockIdx.x * 256 + threadIdx.x.
__global__ __launch_bounds__(kAdmmThreads) void admm_dual_kernel(int64_t n, int64_t ld, const float *X,
                                                                 const float *S, const float *C, const double *b,
                                                                 double inv_sigma, double *y, float *W) {
    const int64_t j = blockIdx.y;
    const int64_t i = (int64_t)blockIdx.x * kAdmmThreads + threadIdx.x;
    if (i >= n) return;
    const int64_t o = j * ld + i;
    const double x = (double)X[o], c = (double)C[o];
    double w = c - x * inv_sigma;
    if (i == j) {
        const double yi = b[i] * inv_sigma - (x * inv_sigma + (double)S[o] - c);
        y[i] = yi;
        w -= yi;
    }
    W[o] = (float)w;
}

__device__ __forceinline__ double block_sum(double v, double *sh) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    if (lane == 0) sh[wave] = v;
    __syncthreads();
    const double r = ((sh[0] + sh[1]) + sh[2]) + sh[3];
    __syncthreads();
    return r;
}

// X += sigma (S + Diag(y) - C) over columns j = blockIdx.x + k * gridDim.x;
// workgroup sums: ||Diag(y) + S - C||_F^2, <C, X_new>, ||C||_F^2,
// ||diag(X_new) - b||^2.
__global__ __launch_bounds__(kAdmmThreads) void admm_primal_kernel(int64_t n, int64_t ld, float *X, const float *S,
                                                                   const float *C, const double *y, const double *b,
                                                                   double sigma, double *part) {
    __shared__ double sh[4];
    double rd = 0.0, pobj = 0.0, cc = 0.0, rp = 0.0;
    for (int64_t j = blockIdx.x; j < n; j += gridDim.x) {
        for (int64_t i = threadIdx.x; i < n; i += kAdmmThreads) {
            const int64_t o = j * ld + i;
            const double c = (double)C[o];
            double r = (double)S[o] - c;
            if (i == j) r += y[i];
            const float xn = (float)((double)X[o] + sigma * r);
            X[o] = xn;
            rd += r * r;
            pobj += c * (double)xn;
            cc += c * c;
            if (i == j) {
                const double d = (double)xn - b[i];
                rp += d * d;
            }
        }
    }
    rd = block_sum(rd, sh);
    pobj = block_sum(pobj, sh);
    cc = block_sum(cc, sh);
    rp = block_sum(rp, sh);
    if (threadIdx.x == 0) {
        double *p = part + (size_t)blockIdx.x * kAdmmParts;
        p[0] = rd;
        p[1] = pobj;
        p[2] = cc;
        p[3] = rp;
    }
}

// res[0..5] = ||diag(X) - b||, ||Diag(y) + S - C||_F, <C, X>, b^T y, ||b||,
// ||C||_F (workgroup sums added in order; the vector sums by one workgroup).
__global__ __launch_bounds__(kAdmmThreads) void admm_residual_kernel(int64_t n, const double *y, const double *b,
                                                                     const double *part, int groups, double *res) {
    __shared__ double sh[4];
    double by = 0.0, bb = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += kAdmmThreads) {
        by += b[i] * y[i];
        bb += b[i] * b[i];
    }
    by = block_sum(by, sh);
    bb = block_sum(bb, sh);
    if (threadIdx.x != 0) return;
    double s[kAdmmParts] = {0.0, 0.0, 0.0, 0.0};
    for (int g = 0; g < groups; ++g)
        for (int q = 0; q < kAdmmParts; ++q) s[q] += part[(size_t)g * kAdmmParts + q];
    res[0] = sqrt(s[3]);
    res[1] = sqrt(s[0]);
    res[2] = s[1];
    res[3] = by;
    res[4] = sqrt(bb);
    res[5] = sqrt(s[2]);
}

}  // namespace
}  // namespace psd

using namespace psd;

extern "C" {

int psdproj_admm_dual(int64_t n, int64_t ld, const float *X, const float *S, const float *C, const double *b,
                      double sigma, double *y, float *W, psdproj_stream_t stream) {
    if (n < 0 || ld < (n > 1 ? n : 1) || !(sigma > 0.0)) return PSDPROJ_ERR_INVALID_ARG;
    if (n == 0) return PSDPROJ_OK;
    if (!X || !S || !C || !b || !y || !W) return PSDPROJ_ERR_INVALID_ARG;
    if (n > 65535) return PSDPROJ_ERR_UNSUPPORTED;  // one grid row per column
    const dim3 grid((unsigned)((n + kAdmmThreads - 1) / kAdmmThreads), (unsigned)n);
    (void)hipGetLastError();  // a pending error of an earlier runtime call is not this call's
    hipLaunchKernelGGL(admm_dual_kernel, grid, dim3(kAdmmThreads), 0, (hipStream_t)stream, n, ld, X, S, C, b,
                       1.0 / sigma, y, W);
    return hipGetLastError() == hipSuccess ? PSDPROJ_OK : PSDPROJ_ERR_HIP;
}

int psdproj_admm_primal(int64_t n, int64_t ld, float *X, const float *S, const float *C, const double *y,
                        const double *b, double sigma, double *res, psdproj_stream_t stream) {
    if (n < 0 || ld < (n > 1 ? n : 1) || !(sigma > 0.0)) return PSDPROJ_ERR_INVALID_ARG;
    if (n == 0) return PSDPROJ_OK;
    if (!X || !S || !C || !y || !b || !res) return PSDPROJ_ERR_INVALID_ARG;
    const int groups = (int)(n < kAdmmGroups ? n : kAdmmGroups);
    double *part = res + 8;
    hipStream_t s = (hipStream_t)stream;
    (void)hipGetLastError();  // a pending error of an earlier runtime call is not this call's
    hipLaunchKernelGGL(admm_primal_kernel, dim3((unsigned)groups), dim3(kAdmmThreads), 0, s, n, ld, X, S, C, y, b,
                       sigma, part);
    hipLaunchKernelGGL(admm_residual_kernel, dim3(1), dim3(kAdmmThreads), 0, s, n, y, b, part, groups, res);
    return hipGetLastError() == hipSuccess ? PSDPROJ_OK : PSDPROJ_ERR_HIP;
}

}  // extern "C"

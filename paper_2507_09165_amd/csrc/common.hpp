// Shared device/host definitions for libpsdproj (gfx950 only).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

typedef _Float16 f16;
typedef __bf16 bf16;
typedef f16 f16x8 __attribute__((ext_vector_type(8)));
typedef bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

namespace psd {

// Device-resident scalar block of one projection (all FP64 so that the bound
// never loses digits). Written by the norm/Lanczos kernels, read by the cast
// and final kernels; never copied to the host inside a projection.
struct Scalars {
    double fro2;        // ||X||_F^2
    double colmax2;     // max_j ||X e_j||^2 (lower bound on ||X||_2^2)
    double lam;         // spectral bound used for the rescale
    double inv_lam;     // 1 / lam (0 when lam == 0)
    double sigma;       // largest Ritz value of X^2
    double resid;       // ||X^2 q - sigma q||
    double lanczos_lam; // sqrt(sigma + resid) before the guard
    double beta_last;   // last Lanczos beta
    double qnorm_inv;   // 1 / ||V s||
    double amax;        // max |alpha_j| seen so far
    int32_t k;          // Lanczos steps taken
    int32_t stop;       // breakdown flag
    int32_t nonfinite;  // input had Inf/NaN
    int32_t fallback;   // guard replaced the Lanczos bound
    double alpha[32];
    double beta[32];
    double s[32];       // Ritz vector in the Krylov basis
};

constexpr int kMaxLanczos = 32;

__host__ __device__ inline int64_t round_up(int64_t v, int64_t m) { return (v + m - 1) / m * m; }

}  // namespace psd

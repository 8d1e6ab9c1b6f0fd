// Host interface of the bandwidth-bound kernels (see aux_kernels.hip).
#pragma once
#include "common.hpp"

namespace psd {

struct LanczosWork {
    double *V;      // n x steps, column-major
    double *u, *w, *w2, *colsq;  // n each
    double *part_a, *part_b;     // per-block partials, nb x 32 each
    double *sd, *sa, *sd2, *sa2; // symmetric-matvec tile partials, tiles x 128 each
};

// O = scale * sym(X), scale = 1 or scal->inv_lam; dtype 0 FP32, 1 FP16, 2 BF16;
// Olo != nullptr writes a hi + lo pair. n_out (multiple of 64) >= n: entries
// outside n x n are zero.
hipError_t mirror_cast(const float *X, int64_t ldx, int64_t n, int64_t n_out, const Scalars *scal, int use_inv_lam,
                       int dtype, void *Ohi, void *Olo, int64_t ldo, hipStream_t s);

// Lanczos bound of the symmetric matrix whose upper triangle X holds
// (FP32, column-major, leading dimension ldx) into scal.
hipError_t spectral_bound(const float *X, int64_t ldx, int64_t n, int steps, uint64_t seed, LanczosWork wk,
                          Scalars *scal, int force_fallback, hipStream_t s);

size_t lanczos_work_doubles(int64_t n, int steps);
int64_t symv_tile_count(int64_t n);

}  // namespace psd

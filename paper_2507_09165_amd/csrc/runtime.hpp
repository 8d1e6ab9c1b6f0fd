// Internal runtime interface shared by the C ABI and the serving loop.
#pragma once
#include <stddef.h>
#include <stdint.h>

#include "../../include/psdproj.h"
#include "common.hpp"

namespace psd {

// Enqueue one projection (or only the bound) on stream s.
int run_projection(const psdproj_opts &o, int64_t n, int64_t ld, const float *X, float *out, hipStream_t s,
                   psdproj_info *info, bool bound_only, bool no_alloc = false);
// Enqueue one batched projection (per-matrix info at info[i], may be null).
int run_batched(const psdproj_opts &o, int count, const int64_t *n, const int64_t *ld, const float *const *X,
                float *const *out, hipStream_t s, psdproj_info *info);
psdproj_opts default_opts(int mode);
// Work precision (DType) of a mode's products, or -1 for a bad mode.
int mode_dtype(int mode);
// Apply the tuning cache named by PSDPROJ_TUNE_CACHE (once per process).
void load_env_tune_cache();
// Workspace bytes of one batched call over the orders ns in mode.
size_t workspace_bytes_batch(const int64_t *ns, int count, int mode);
// Workspace bytes a projection of size n in mode needs (0 for a bad mode).
size_t workspace_bytes_for(int64_t n, int mode);
// Number of n_p x n_p products the projection runs (FP16-product
// equivalents; -1 for bad options).
double gemm_count_for(const psdproj_opts &o);
// Per-(device, stream) workspace pool: bytes currently held, and release.
size_t pool_held(hipStream_t s);
void pool_release(hipStream_t s);

}  // namespace psd

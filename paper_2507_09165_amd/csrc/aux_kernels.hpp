// Host interface of the bandwidth-bound kernels (see aux_kernels.hip).
#pragma once
#include "common.hpp"

namespace psd {

// Device tables of one batched launch: descriptors, caller I/O (io_tab, or
// io0 by value for a single matrix) and the work lists of each grid shape.
struct BatchLaunch {
    int count = 0;                 // matrices
    const MatDesc *desc = nullptr; // device, count entries
    const IoArg *io_tab = nullptr; // device, count entries (nullptr: use io0)
    IoArg io0{};
    const WorkItem *w_vec = nullptr;   // (m, block of 256 rows)
    const WorkItem *w_symv = nullptr;  // (m, 128 x 128 triangle tile)
    const WorkItem *w_cast = nullptr;  // (m, 64 x 64 tile pair of the padded matrix)
    int64_t n_vec = 0, n_symv = 0, n_cast = 0;
};

// Lanczos bound (Theorem 2) of every matrix into its Scalars.
hipError_t spectral_bound(const BatchLaunch &B, int steps, uint64_t seed, int force_fallback, double lam_override,
                          hipStream_t s);
// Slot 0 <- X / lam in dtype (0 FP32, 1 FP16, 2 BF16, 3 FP16 with FP8 pairs
// of code exponent e8), optionally split (hi + lo, or hi + FP8 pair).
hipError_t cast_x0(const BatchLaunch &B, int dtype, bool split, int e8, hipStream_t s);

// Deflation of dominant eigenpairs of one matrix (see deflate.hip). The
// descriptor's U must have been filled by a spectral_bound run on io.X.
struct DeflLaunch {
    const MatDesc *desc = nullptr;     // device, one entry
    const WorkItem *w_vec = nullptr;   // (0, block of 256 rows)
    int64_t n_vec = 0;
    const WorkItem *w_tri = nullptr;   // (0, 64 x 64 tile t = J (J + 1) / 2 + I) covering n
    int64_t n_tri = 0;
    IoArg io{};                        // caller's X (remove) or out (add back), ld
};
// Rayleigh-Ritz pairs of X in the Lanczos basis, the converged ones kept, and
// the deflated copy X' = X - sum mu z z^T (upper triangle) written.
hipError_t deflate_remove(const DeflLaunch &L, hipStream_t s);
// out += sum max(mu, 0) z z^T (both triangles).
hipError_t deflate_addback(const DeflLaunch &L, hipStream_t s);

// Adaptive depth after a stage whose iterate is in slot sn (the previous one
// in so): per matrix not yet converged, record sn and the stage count and,
// when may_stop, its relative change (FP64 sums over the cast work list into
// part, 2 doubles per item), converged once <= tol. dtype: 0 FP32, 1 FP16,
// 2 BF16.
hipError_t stage_check(const BatchLaunch &B, int dtype, int sn, int so, int stage, bool may_stop, double tol,
                       double *part, hipStream_t s);

size_t lanczos_work_doubles(int64_t n, int steps);
int64_t symv_tile_count(int64_t n);
int64_t vec_block_count(int64_t n);
int64_t cast_tile_count(int64_t np);
// Lanczos pointers of a descriptor inside lz (lanczos_work_doubles doubles).
void fill_lanczos_desc(MatDesc &d, double *lz, int64_t n, int steps);

}  // namespace psd

// Host interface of the one-workgroup projection of small matrices (see
// small_proj.hip).
#pragma once
#include "common.hpp"

namespace psd {

// Largest order the one-workgroup kernel takes (its work matrices are padded
// to this edge).
constexpr int kSmallEdge = 128;

// The stage plan of one launch (every listed matrix has the same plan).
struct SmallArgs {
    const MatDesc *D;
    const WorkItem *list;  // (matrix index, 0) per workgroup
    const IoArg *io_tab;   // per-matrix caller I/O, or
    IoArg io0;             // the single matrix's I/O when io_tab is null
    int T;                 // filter stages
    int steps;             // Lanczos steps (<= kMaxLanczos)
    uint32_t split_mask;   // stages whose products run on split operands
    int split_final;       // final product on split operands
    int bound_only;        // stop after the spectral bound
    int force_fallback;    // test hook: halve the Lanczos bound so the guard fires
    double lam_override;   // > 0: use this bound
    uint64_t seed;         // Lanczos start vector
    float a[16], b[16], c[16];  // stage coefficients (stage rescale folded in)
    int ex[17], ea[16], eb[16]; // FP8-pair code exponents of X_t, A, B
};

// dtype: DT_F16, DT_BF16, DT_F16X8 or DT_BF16X8; count workgroups.
hipError_t small_proj_launch(const SmallArgs &a, int dtype, int count, hipStream_t s);

}  // namespace psd

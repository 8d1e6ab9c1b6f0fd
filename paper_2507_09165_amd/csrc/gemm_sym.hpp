// Host interface of the symmetric MFMA GEMM (see gemm_sym.hip).
#pragma once
#include "common.hpp"

namespace psd {

enum DType { DT_F32 = 0, DT_F16 = 1, DT_BF16 = 2 };
enum Epi { EPI_STORE = 0, EPI_STORE_SPLIT = 1, EPI_FINAL = 2 };

// Output tile edge; work matrices are zero-padded to a multiple of it.
constexpr int kTile = 128;

struct GemmArgs {
    // Operands (n_p x n_p, column-major, leading dimension ld, symmetric).
    // *lo == nullptr means the operand is a single (unsplit) matrix.
    const void *Lhi, *Llo, *Rhi, *Rlo;
    // Epilogue addend C0 (same layout; may be nullptr) and outputs.
    const void *C0hi, *C0lo;
    void *Dhi, *Dlo;
    // Final epilogue: out (FP32, n x n, ldo) = (Xf + lam * acc) / 2.
    float *out;
    int64_t ldo;
    int64_t n;
    const float *Xf;
    int64_t ldxf;
    const Scalars *scal;
    int64_t ld;  // leading dimension of the work matrices
    int64_t K;   // padded size n_p (multiple of kTile)
    float alpha, beta, gamma;  // D = alpha C0 + beta (L R) + gamma I
};

hipError_t gemm_sym_launch(const GemmArgs &g, int dtype, int epi, hipStream_t s);

}  // namespace psd

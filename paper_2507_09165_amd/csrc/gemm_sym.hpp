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
    // Final epilogue: out (FP32, n x n, ldo) = (X + lam * acc) / 2, X read from
    // its upper triangle (Xin, column-major, leading dimension ldx).
    float *out;
    int64_t ldo;
    int64_t n;
    const float *Xin;
    int64_t ldx;
    const Scalars *scal;
    const uint32_t *tiles;  // filled by the launcher: tile list (bi | bj << 16)
    int64_t ld;  // leading dimension of the work matrices
    int64_t K;   // padded size n_p (multiple of kTile)
    float alpha, beta, gamma;  // D = alpha C0 + beta (L R) + gamma I
};

hipError_t gemm_sym_launch(const GemmArgs &g, int dtype, int epi, hipStream_t s);

// Tile edge the launcher uses for a padded size K, and the padded size used for
// a logical size n (a multiple of the tile it will run with).
int gemm_pick_tile(int64_t K);
inline int64_t gemm_padded_size(int64_t n) {
    return n >= 1536 ? round_up(n, 256) : round_up(n > 0 ? n : 1, kTile);
}
// Tuning hook: force the tile edge (0 restores the automatic choice).
void gemm_set_tile_override(int bm);
// Tuning hook: blocking of the tile schedule (H tile rows x W tile columns).
void gemm_set_block_shape(int h, int w);

}  // namespace psd

// Host interface of the symmetric MFMA GEMM (see gemm_sym.hip).
#pragma once
#include <vector>

#include "common.hpp"

namespace psd {

// DT_F16X8 / DT_BF16X8: FP16 / BF16 work matrices whose split slots carry the
// e4m3 lo codes of an FP8 pair (see lo8_index) instead of lo halves.
enum DType { DT_F32 = 0, DT_F16 = 1, DT_BF16 = 2, DT_F16X8 = 3, DT_BF16X8 = 4 };
enum Epi { EPI_STORE = 0, EPI_STORE_SPLIT = 1, EPI_FINAL = 2 };

// Output tile edge; work matrices are zero-padded to a multiple of it.
constexpr int kTile = 128;
// The large tile edge, and the bytes of one FP32 partial tile of a K-split.
constexpr int kTile2 = 256;
constexpr size_t kPartBytes = sizeof(float) * kTile2 * kTile2;

// One symmetric product D = alpha C0 + beta (L R) + gamma I for every matrix
// named by the tile list. Operands, addend and output are work slots of the
// matrix's descriptor (hi[slot], lo[slot]); sc0 < 0 means no addend. The
// final epilogue instead writes out = (X + lam L R) / 2 to the caller's I/O.
struct GemmArgs {
    const MatDesc *D;
    const WorkItem *tiles;  // (matrix, bi | bj << 16), upper tiles only
    const IoArg *io_tab;    // final epilogue: per-matrix I/O, or
    IoArg io0;              // the single matrix's I/O when io_tab is null
    int sl, sr, sc0, sd;
    int c0_split;
    float alpha, beta, gamma;
    int es_l, es_r, es_c0, es_d;  // FP8-pair code exponents of the slots (DT_F16X8)
    // K-split tiles (ks = 1: chunk list, ks = 2: fixup list; see TileLists)
    // and their FP32 partial tiles (kTile2 x kTile2 floats each)
    const uint4 *split;
    float *part;
    // adaptive depth: 1 = a stage product, skipped once the matrix's iterate
    // has converged; 2 = the final product, whose right operand is the slot
    // of the latest iterate (Scalars::cur_slot) instead of sr
    int adaptive;
};

// ls / rs: L / R carry lo halves. bm: tile edge (128 or 256; it must divide
// every listed matrix's np). ntiles: length of the tile list. ks: 0 = whole
// tiles from g.tiles; 1 = K-chunks of split tiles, 2 = their fixup, both from
// g.split and for bm = 256 only.
hipError_t gemm_sym_launch(const GemmArgs &g, int dtype, int epi, bool ls, bool rs, int bm, int64_t ntiles,
                           hipStream_t s, int ks = 0);
// One (precision, epilogue) slice of gemm_sym_launch, explicitly instantiated
// in gemm_launch_*.hip.
template <int DT, int EPI>
hipError_t gemm_launch_part(const GemmArgs &g, bool ls, bool rs, int bm, int64_t ntiles, hipStream_t s, int ks);
// Append matrix m's upper tiles (T x T tile grid) in the blocked schedule order.
void append_tile_order(std::vector<WorkItem> &v, uint32_t m, int T);

// Tile edge the kernel-level entry uses for a padded size K and dtype.
int gemm_pick_tile(int64_t K, int dtype);
// Whether plain products of an n x n matrix use the 256 tile, and the padded
// size of its work matrices (a multiple of every tile it runs with; `big`:
// the 256 tile is used).
bool gemm_use_big(int64_t n, int dtype);
int64_t gemm_padded_size(int64_t n, bool big);
// Tile lists of a plan: `big` (256 tiles of plain products, whole rounds of
// one workgroup per CU), `small_plain` (the rest of the plain products as 128
// tiles), `small_all` (every matrix's full triangle of 128 tiles, for split
// products). np: padded orders; big: gemm_use_big per matrix; cus: CU count.
// `split` / `fixup` (uint4 entries, see gemm_sym_kernel's KS): the matrices
// whose last partial round of 256 tiles is at most half the CUs run those
// tiles as K-chunks (one workgroup each, chunks = CUs / tail tiles, at most
// 8) plus a fixup per tile; `parts` partial tiles in all.
struct TileLists {
    std::vector<WorkItem> big, small_plain, small_all;
    std::vector<uint4> split, fixup;
    int64_t parts = 0;
};
// ksplit: most K-chunks per tail tile of each matrix (gemm_ksplit_for).
void gemm_tile_lists(const std::vector<int64_t> &np, const std::vector<bool> &big, const std::vector<int> &ksplit,
                     int cus, TileLists &out);
// Per-size-class tile choice (the autotuner's): for orders of class
// gemm_size_class(n) in work precision dtype, tile 128 (128 tiles only) or
// 256 (256-tile rounds, tails as up to `ksplit` K-chunks). Without a choice
// the fixed rules above apply. Setting or clearing a choice bumps the tuning
// generation (plans are rebuilt).
int gemm_size_class(int64_t n);  // quarter octaves: floor(4 log2 n)
void gemm_set_class_choice(int dtype, int cls, int tile, int ksplit);
void gemm_clear_class_choices();
bool gemm_class_choice(int dtype, int64_t n, int *tile, int *ksplit);
// Most K-chunks per tail tile for an n x n matrix in dtype.
int gemm_ksplit_for(int64_t n, int dtype);
// Incremented whenever a tuning hook changes the tile choice.
int gemm_tile_generation();
// CU count the tail rule uses (the device's unless the tuning hook set one).
int gemm_tail_cus(int device_cus);
// Default size from which products use the 256 tile (a matrix of this order
// first fills one whole round of 256 tiles on 256 CUs; see gemm_use_big).
constexpr int64_t kBigMinDefault = 5633;
// Tuning hooks: size from which products use the 256 tile (0 restores
// kBigMinDefault), and the CU count of the tail rule (0: the device's).
void gemm_set_big_min(int64_t min_n);
int64_t gemm_big_min();
void gemm_set_tail_cus(int tail_cus);
// Whether split products of matrices that use the 256 tile use it too (else
// they run the 128-tile list). Tuning hook: mask, bit 0 FP16/BF16 pairs, bit 1
// FP8 pairs.
bool gemm_split_big(int dtype);
void gemm_set_split_big(int mask);
// Tuning hook: most K-chunks a tail tile is cut into (1: never).
void gemm_set_ksplit_max(int c);
// Tuning hook: force the tile edge (0 restores the automatic choice).
void gemm_set_tile_override(int bm);
// Tuning hook: blocking of the tile schedule (H tile rows x W tile columns).
void gemm_set_block_shape(int h, int w);

}  // namespace psd

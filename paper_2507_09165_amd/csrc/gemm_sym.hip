// Host side of the symmetric MFMA GEMM: the tile schedule, the tile lists
// of a plan (256-tile rounds, K-split tails, 128 tiles), the tuning hooks and
// the launch dispatch over work precisions (the kernel template is in
// gemm_sym_kernel.hpp, instantiated per precision in gemm_launch_*.hip).
#include <algorithm>
#include <atomic>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "common.hpp"
#include "gemm_sym.hpp"

namespace psd {

// Tile schedule. The upper-triangle tiles are listed in blocks of H tile rows
// x W tile columns (super-rows of height H, walked left to right in chunks of
// W columns). The launch gives each XCD a contiguous run of this list, so the
// ~32 tiles resident on one XCD at a time form a compact 2D block that shares
// H + W operand panels in its L2 instead of one panel per tile.
//
// The tuning hooks below are process-wide atomics: a change made while
// another thread builds a plan is seen either entirely before or after each
// read, and the generation counter makes plans built before it stale.
static std::atomic<int> g_tile_override{0};  // tuning hook: force a tile edge (0 = automatic)
static std::atomic<int> g_tile_gen{0};       // bumped by every tuning change (plans key on it)
static int g_block_h = 4, g_block_w = 4;      // guarded by g_cfg_mu
static std::mutex g_cfg_mu;

void append_tile_order(std::vector<WorkItem> &v, uint32_t m, int T) {
    int H, W;
    {
        std::lock_guard<std::mutex> lk(g_cfg_mu);
        H = g_block_h;
        W = g_block_w;
    }
    for (int s0 = 0; s0 < T; s0 += H)
        for (int c0 = s0; c0 < T; c0 += W)
            for (int bj = c0; bj < std::min(c0 + W, T); ++bj)
                for (int bi = s0; bi < std::min(s0 + H, T); ++bi)
                    if (bi <= bj) v.push_back(WorkItem{m, (uint32_t)bi | ((uint32_t)bj << 16)});
}

// Tile edge of the kernel-level entry points (one launch over the whole
// triangle): 128, or the tile override where it divides K. The projection's
// own products pick tiles per matrix (gemm_use_big, gemm_tile_lists).
int gemm_pick_tile(int64_t K, int dtype) {
    const int o = g_tile_override;
    if (o && K % o == 0) return o;
    return 128;
}

// Products of large FP16/BF16 matrices run on the 256 tile: it moves half the
// operand bytes per flop of the 128 tile (one workgroup per CU against two).
// From n = 5633 (n_p = 5888, 276 tiles) a matrix fills at least one whole
// round of 256 CUs; below, all its 256-tiles would be tail (as 128 tiles, at
// a coarser padding). Measured at n = 5782: 8.8 against 10.1 ms (FP8 pairs);
// equal at 4096-5000, 2-9% slower at 2048-3072. (Tuning hooks: the size
// threshold, and the CU count the tail rule uses.)
static std::atomic<int64_t> g_big_min{kBigMinDefault};
static std::atomic<int> g_tail_cus{0};  // 0: the device's CU count

// Per-size-class choices of the autotuner, keyed by (dtype, class).
static std::mutex g_class_mu;
static std::map<std::pair<int, int>, std::pair<int, int>> g_class_choice;  // -> (tile, ksplit)

int gemm_size_class(int64_t n) {
    int c = 0;
    double x = (double)(n > 1 ? n : 1);
    while (x >= 2.0) { x *= 0.5; c += 4; }
    // x in [1, 2): quarter octaves 2^(q/4)
    const double q1 = 1.189207115002721, q2 = 1.414213562373095, q3 = 1.681792830507429;
    return c + (x >= q3 ? 3 : x >= q2 ? 2 : x >= q1 ? 1 : 0);
}

void gemm_set_class_choice(int dtype, int cls, int tile, int ksplit) {
    {
        std::lock_guard<std::mutex> lk(g_class_mu);
        g_class_choice[{dtype, cls}] = {tile, ksplit};
    }
    ++g_tile_gen;
}

void gemm_clear_class_choices() {
    {
        std::lock_guard<std::mutex> lk(g_class_mu);
        g_class_choice.clear();
    }
    ++g_tile_gen;
}

bool gemm_class_choice(int dtype, int64_t n, int *tile, int *ksplit) {
    std::lock_guard<std::mutex> lk(g_class_mu);
    auto it = g_class_choice.find({dtype, gemm_size_class(n)});
    if (it == g_class_choice.end()) return false;
    *tile = it->second.first;
    *ksplit = it->second.second;
    return true;
}

bool gemm_use_big(int64_t n, int dtype) {
    const int o = g_tile_override;
    if (o == 128) return false;
    if (o == 256) return true;
    int tile = 0, ks = 0;
    if (dtype != DT_F32 && gemm_class_choice(dtype, n, &tile, &ks)) return tile == 256;
    return dtype != DT_F32 && n >= g_big_min;
}
int gemm_tail_cus(int device_cus) {
    const int c = g_tail_cus;
    return c > 0 ? c : device_cus;
}

// Split products are bound by operand movement as well, so the 256 tile pays
// for them too (per-dtype switch for the tuning hook).
static std::atomic<int> g_split_big{3};
bool gemm_split_big(int dtype) {
    if (g_tile_override == 128) return false;
    if (dtype == DT_F16X8 || dtype == DT_BF16X8) return (g_split_big & 2) != 0;
    return dtype != DT_F32 && (g_split_big & 1) != 0;
}
void gemm_set_split_big(int mask) {
    g_split_big = mask;
    ++g_tile_gen;
}

// Padded order of the work matrices: a multiple of 256 where the 256 tile is
// used, else of 128 (or of the override). Whole tiles of either size give
// bitwise-identical results: every element accumulates its K products in the
// same order whatever the tile shape, and padding only adds zeros (K-split
// tail tiles differ from that by rounding).
int64_t gemm_padded_size(int64_t n, bool big) {
    const int64_t m = n > 0 ? n : 1;
    if (big) return round_up(m, 256);
    const int o = g_tile_override;
    return round_up(m, o ? o : kTile);
}

int gemm_tile_generation() { return g_tile_gen; }

// The 256 tile runs one workgroup per CU, so B such tiles take ceil(B / CUs)
// rounds and a partial last round idles most of the chip (measured: ~1000
// TFLOP/s just under a whole number of rounds, ~860 just over). A matrix's
// last B mod CUs tiles therefore run apart from its whole rounds: when they
// fill at most half the CUs, each is cut into c = min(CUs / tail, 8) K-chunks
// (one 256-tile workgroup each, FP32 partials) and a fixup sums the chunks in
// order; otherwise each runs as four 128 tiles (two workgroups per CU) in the
// product's last launch. The rule is per matrix, so a matrix's result does
// not depend on the other matrices of a batch.
static std::atomic<int> g_ksplit_max{8};  // tuning hook: most K-chunks per tile (1: never split)

int gemm_ksplit_for(int64_t n, int dtype) {
    int tile = 0, ks = 0;
    if (gemm_class_choice(dtype, n, &tile, &ks)) return ks;
    return g_ksplit_max;
}

void gemm_tile_lists(const std::vector<int64_t> &np, const std::vector<bool> &big, const std::vector<int> &ksplit,
                     int cus, TileLists &out) {
    out.big.clear();
    out.small_plain.clear();
    out.small_all.clear();
    out.split.clear();
    out.fixup.clear();
    out.parts = 0;
    int max_chunks = 0;
    for (size_t m = 0; m < np.size(); ++m) {
        append_tile_order(out.small_all, (uint32_t)m, (int)(np[m] / kTile));
        if (!big[m]) {
            append_tile_order(out.small_plain, (uint32_t)m, (int)(np[m] / kTile));
            continue;
        }
        std::vector<WorkItem> t;
        append_tile_order(t, (uint32_t)m, (int)(np[m] / kTile2));
        const size_t tail = (g_tile_override == kTile2 || cus <= 0) ? 0 : t.size() % (size_t)cus;
        const int chunks = tail ? std::min<int>((int)((size_t)cus / tail), ksplit[m]) : 0;
        out.big.insert(out.big.end(), t.begin(), t.end() - tail);
        for (size_t k = t.size() - tail; k < t.size(); ++k) {
            const WorkItem w = t[k];
            if (chunks >= 2) {
                out.fixup.push_back(uint4{w.x, w.y, (uint32_t)chunks << 8, (uint32_t)out.parts});
                out.parts += chunks;
                max_chunks = std::max(max_chunks, chunks);
                continue;
            }
            const uint32_t bi = w.y & 0xFFFFu, bj = w.y >> 16;
            for (uint32_t sj = 2 * bj; sj < 2 * bj + 2; ++sj)
                for (uint32_t si = 2 * bi; si < 2 * bi + 2; ++si)
                    if (si <= sj) out.small_plain.push_back(WorkItem{w.x, si | (sj << 16)});
        }
    }
    // chunk-major: the workgroups of one chunk index are consecutive, so the
    // tiles an XCD runs together read the same K range
    for (int c = 0; c < max_chunks; ++c)
        for (const uint4 &f : out.fixup)
            if ((int)(f.z >> 8) > c) out.split.push_back(uint4{f.x, f.y, (uint32_t)c | f.z, f.w + (uint32_t)c});
}

void gemm_set_ksplit_max(int c) {
    g_ksplit_max = c;
    ++g_tile_gen;
}

hipError_t gemm_sym_launch(const GemmArgs &g, int dtype, int epi, bool ls, bool rs, int bm, int64_t ntiles,
                           hipStream_t s, int ks) {
#define PSD_EPI(DT)                                                                          \
    switch (epi) {                                                                           \
        case EPI_STORE: return gemm_launch_part<DT, EPI_STORE>(g, ls, rs, bm, ntiles, s, ks); \
        case EPI_STORE_SPLIT:                                                                \
            return gemm_launch_part<DT, EPI_STORE_SPLIT>(g, ls, rs, bm, ntiles, s, ks);       \
        case EPI_FINAL: return gemm_launch_part<DT, EPI_FINAL>(g, ls, rs, bm, ntiles, s, ks); \
    }                                                                                        \
    return hipErrorInvalidValue;
    switch (dtype) {
        case DT_F32:
            if (epi == EPI_STORE) return gemm_launch_part<DT_F32, EPI_STORE>(g, ls, rs, bm, ntiles, s, ks);
            if (epi == EPI_FINAL) return gemm_launch_part<DT_F32, EPI_FINAL>(g, ls, rs, bm, ntiles, s, ks);
            return hipErrorInvalidValue;
        case DT_F16: PSD_EPI(DT_F16)
        case DT_BF16: PSD_EPI(DT_BF16)
        case DT_F16X8: PSD_EPI(DT_F16X8)
        case DT_BF16X8: PSD_EPI(DT_BF16X8)
    }
#undef PSD_EPI
    return hipErrorInvalidValue;
}

void gemm_set_big_min(int64_t min_n) {
    g_big_min = min_n > 0 ? min_n : kBigMinDefault;
    ++g_tile_gen;
}
int64_t gemm_big_min() { return g_big_min; }
void gemm_set_tail_cus(int tail_cus) {
    g_tail_cus = tail_cus;
    ++g_tile_gen;
}
void gemm_set_tile_override(int bm) {
    g_tile_override = bm;
    ++g_tile_gen;
}
void gemm_set_block_shape(int h, int w) {
    std::lock_guard<std::mutex> lk(g_cfg_mu);
    g_block_h = h;
    g_block_w = w;
    ++g_tile_gen;
}

}  // namespace psd


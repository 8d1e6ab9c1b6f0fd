// C ABI of libpsdproj: argument checks, plans and workspaces, and the launch
// sequence of Algorithm 2 (bound -> rescale/cast -> T filter stages -> final).
//
// A plan covers one call shape — a mode and a list of matrix orders — on one
// (device, stream). It lays out one arena (from the per-stream workspace
// pool): the descriptor table, the I/O table, the work lists of every grid
// shape, and each matrix's workspace. Every kernel launch of the sequence
// covers all matrices of the plan; a single projection is a plan of one.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <map>
#include <memory>
#include <mutex>
#include <utility>
#include <vector>

#include "../../include/psdproj.h"
#include "aux_kernels.hpp"
#include "coeffs.hpp"
#include "common.hpp"
#include "gemm_sym.hpp"
#include "runtime.hpp"
#include "small_proj.hpp"

// Workspace of psdproj_project_noalloc: one copy per device, held from the
// library's load until the process ends. Host code must not use this name as
// a device address (it names a host-side stand-in); it takes the address that
// hipGetSymbolAddress returns for the current device (scratch_address).
static __device__ __align__(256) uint8_t scratch[PSDPROJ_NOALLOC_SCRATCH_BYTES];

namespace psd {
namespace {

constexpr int kDefaultLanczos = 20;
// Caller-I/O tables kept per multi-matrix plan (see Plan::IoSlot).
constexpr int kIoRing = 8;
constexpr uint64_t kLanczosSeed = 0;
// FP16_SPLIT default: hi + lo products in stages 2 and 3, the stages whose
// FP16 rounding contributes most to the error (measured at n = 10^4 on GOE
// and rank-500 + noise spectra: 7.4e-4 and 4.8e-4 against an FP64
// eigen-projection, versus 1.4e-3 and 8.3e-4 for plain FP16); the final
// product stays plain.
constexpr uint32_t kDefaultSplitMask = 0x6;
constexpr int kDefaultSplitFinal = 0;
// BF16 default: BF16 hi + lo products in stages 1-4. BF16 keeps 8 significant
// bits (unit roundoff 2^-9), so plain BF16 storage at every stage measures
// 1.1e-2 (n = 10^4) to 1.6e-2 (n = 1024) against the FP64 composite
// polynomial; a rounding simulation over split masks (n = 64..2048, GOE and
// clustered spectra) gives 6-8e-3 for stages 2-3, 6.2-12.5e-3 for 2-4 and
// 3.2-3.4e-3 for 1-4, the cheapest mask under the 5e-3 half-precision target.
constexpr uint32_t kDefaultSplitMaskBf16 = 0xF;
// split_mask bit 31: take bits 0..30 as given, even when they are all zero
// (a zero mask otherwise selects the mode's default).
constexpr uint32_t kExplicitMask = 0x80000000u;
// split_mask bit 30: in the masked stages only B = b A + c A^2 is kept as a
// pair; A = X X stays plain and X' = a X + B X is a one-sided split product
// (split operand B on the left, since B and X commute).
constexpr uint32_t kSplitBOnly = PSDPROJ_SPLIT_B_ONLY;
// split_mask bits 16..29: bit 16 + t makes stage t + 1 such a B-only stage
// (a stage also set in bits 0..15 is split in full).
constexpr int kBOnlyShift = PSDPROJ_SPLIT_B_SHIFT;
// FP8_FP16_SPLIT default: stage 3 split in full and stages 1-2 B-only (26
// product-equivalents instead of 28 for stages 2-3 in full). The stages'
// contributions to the squared error add up nearly independently (stages
// 2-3 predicted from the single-stage splits within 0.1%), and a B-only stage
// removes about 60% of its stage's share at a quarter of the full split's
// cost. Measured at n = 10^4 against an FP64 eigen-projection: 8.3e-4 (GOE)
// and 4.7e-4 (rank-500 + noise), 30.0 ms, against 7.4e-4 / 4.8e-4 and 31.9
// ms for stages 2-3 in full; single full stages miss 1e-3 on GOE (1.10e-3 at
// best). Matrices of the one-workgroup path split these stages in full.
constexpr uint32_t kDefaultSplitMaskFp8 = 0x4u | (0x3u << kBOnlyShift);

struct StagePlan {
    int T = 0;
    bool cubic = false;  // Newton-Schulz steps a X + b X^3 (two products each)
    // adaptive depth: stages t >= adapt_from are skipped once the iterate's
    // relative change in a stage is at most opts.adaptive_tol
    bool adaptive = false;
    int adapt_from = 0;
    double a[16], b[16], c[16];
    int dtype = DT_F32;
    uint32_t split_mask = 0;
    bool split_final = false;
    uint32_t b_mask = 0;  // stages in which only B is split (disjoint from split_mask)
    // FP8-pair code exponents (DT_F16X8): X_t (t = 0..T), A and B of stage t
    int ex[17], ea[16], eb[16];
};

// Exponent e of an FP8 pair for a matrix whose entries are bounded by `bound`:
// codes |M_hi| 2^e and |M - M_hi| 2^(11+e) <= |M| 2^e stay at or below 256,
// leaving a factor 1.75 to the e4m3 maximum for rounding and a bound that is
// slightly loose.
int pair_exponent(double bound) {
    const int e = (int)floor(log2(256.0 / fmax(bound, 1e-30)));
    return e < -40 ? -40 : (e > 40 ? 40 : e);
}

// Bounds on the stage matrices. X0 = X / lam has spectral norm <= 1 when lam
// bounds ||X||_2 (2% slack covers a Lanczos bound a little below it). Stage t
// maps eigenvalues x of X_t to a x + b x^3 + c x^5 with A = X_t^2 <= bx^2 and
// B = b A + c A^2; entries of a symmetric matrix are bounded by its spectral
// norm. Maxima are taken on a fine grid.
void pair_exponents(StagePlan &p) {
    const int G = 4096;
    double bx = 1.02;
    p.ex[0] = pair_exponent(bx);
    for (int t = 0; t < p.T; ++t) {
        const double ba = bx * bx;
        double bb = 0.0, bn = 0.0;
        for (int k = 0; k <= G; ++k) {
            const double y = ba * k / G;  // eigenvalue of A
            bb = fmax(bb, fabs(p.b[t] * y + p.c[t] * y * y));
            const double x = bx * k / G;  // eigenvalue of X_t
            const double x2 = x * x;
            bn = fmax(bn, fabs(x * (p.a[t] + x2 * (p.b[t] + p.c[t] * x2))));
        }
        p.ea[t] = pair_exponent(ba);
        p.eb[t] = pair_exponent(bb);
        bx = bn;
        p.ex[t + 1] = pair_exponent(bx);
    }
}

bool make_stage_plan(const psdproj_opts &o, StagePlan &p) {
    const StageCoef *tab;
    int T, nres;
    double res;
    switch (o.mode) {
        case PSDPROJ_MODE_FP32:
            tab = kTildeSingle; T = 10; nres = kSingleRescaled; res = kSingleRescale; p.dtype = DT_F32; break;
        case PSDPROJ_MODE_FP16:
        case PSDPROJ_MODE_FP16_SPLIT:
            tab = kTildeHalf; T = 7; nres = kHalfRescaled; res = kHalfRescale; p.dtype = DT_F16; break;
        case PSDPROJ_MODE_BF16:
            tab = kTildeHalf; T = 7; nres = kHalfRescaled; res = kHalfRescale; p.dtype = DT_BF16; break;
        case PSDPROJ_MODE_FP32_EMU:
            tab = kTildeSingle; T = 10; nres = kSingleRescaled; res = kSingleRescale; p.dtype = DT_F16; break;
        case PSDPROJ_MODE_FP8_FP16_SPLIT:
            tab = kTildeHalf; T = 7; nres = kHalfRescaled; res = kHalfRescale; p.dtype = DT_F16X8; break;
        case PSDPROJ_MODE_FP8_BF16_SPLIT:
            tab = kTildeHalf; T = 7; nres = kHalfRescaled; res = kHalfRescale; p.dtype = DT_BF16X8; break;
        case PSDPROJ_MODE_NS_FP16:
        case PSDPROJ_MODE_NS_FP32:
            // Newton-Schulz baseline: x <- (3 x - x^3) / 2, no stage rescale
            p.cubic = true;
            p.T = o.mode == PSDPROJ_MODE_NS_FP16 ? kNewtonSchulzHalf : kNewtonSchulzSingle;
            p.dtype = o.mode == PSDPROJ_MODE_NS_FP16 ? DT_F16 : DT_F32;
            for (int t = 0; t < p.T; ++t) {
                p.a[t] = kNewtonSchulz.a;
                p.b[t] = kNewtonSchulz.b;
                p.c[t] = kNewtonSchulz.c;
            }
            if (o.adaptive_extra != 0 || !(o.adaptive_tol >= 0.0)) return false;
            p.adaptive = o.adaptive_tol > 0.0;  // every step may end the iteration
            p.adapt_from = 0;
            pair_exponents(p);
            return true;
        default: return false;
    }
    p.T = T;
    for (int t = 0; t < T; ++t) {
        const double s = t < nres ? res : 1.0;
        p.a[t] = tab[t].a * s;
        p.b[t] = tab[t].b * s;
        p.c[t] = tab[t].c * s;
    }
    // adaptive depth: extra quintic Newton-Schulz stages after the table
    if (o.adaptive_extra < 0 || T + o.adaptive_extra > 16 || !(o.adaptive_tol >= 0.0)) return false;
    for (int k = 0; k < o.adaptive_extra; ++k) {
        p.a[T + k] = kNewtonSchulzQuintic.a;
        p.b[T + k] = kNewtonSchulzQuintic.b;
        p.c[T + k] = kNewtonSchulzQuintic.c;
    }
    p.T = T + o.adaptive_extra;
    p.adaptive = o.adaptive_tol > 0.0 && o.adaptive_extra > 0;
    p.adapt_from = T;
    if (o.mode == PSDPROJ_MODE_FP16_SPLIT || o.mode == PSDPROJ_MODE_FP8_FP16_SPLIT || o.mode == PSDPROJ_MODE_BF16 ||
        o.mode == PSDPROJ_MODE_FP8_BF16_SPLIT) {
        const bool bf = o.mode == PSDPROJ_MODE_BF16 || o.mode == PSDPROJ_MODE_FP8_BF16_SPLIT;
        const uint32_t def = bf ? kDefaultSplitMaskBf16
                                : o.mode == PSDPROJ_MODE_FP8_FP16_SPLIT ? kDefaultSplitMaskFp8 : kDefaultSplitMask;
        const uint32_t m = (o.split_mask & kExplicitMask) ? (o.split_mask & ~kExplicitMask)
                                                          : (o.split_mask ? o.split_mask : def);
        const uint32_t stages = (1u << T) - 1;
        if (m & kSplitBOnly) {  // every masked stage B-only
            p.b_mask = m & stages & 0xFFFFu;
            p.split_mask = 0;
        } else {
            p.split_mask = m & stages & 0xFFFFu;
            p.b_mask = (m >> kBOnlyShift) & 0x3FFFu & stages & ~p.split_mask;
        }
        p.split_final = o.split_final < 0 ? kDefaultSplitFinal : o.split_final != 0;
    } else if (o.mode == PSDPROJ_MODE_FP32_EMU) {
        // every product on hi + lo FP16 pairs: ~22-bit operands, FP32 accumulation
        p.split_mask = (1u << T) - 1;
        p.split_final = true;
    }
    pair_exponents(p);
    return true;
}

// Whether any work matrix of the plan is stored split (lo slots needed).
bool any_split(const StagePlan &p) { return p.split_mask != 0 || p.b_mask != 0 || p.split_final; }

size_t elt_size(int dtype) { return dtype == DT_F32 ? 4 : 2; }

// Orders up to this value run the whole projection in the one-workgroup
// small-matrix kernel (tuning key "small_max"; 0 = never).
static std::atomic<int> g_small_max{kSmallEdge};

// Whether matrix n of a plan runs in the one-workgroup kernel: half-precision
// work formats (B-only stages split in full there), no adaptive depth, no
// deflation. The
// rule depends only on (n, mode, options), so a matrix takes the same path
// alone and in any batch.
bool plan_fused(int64_t n, const StagePlan &p, int deflate, int small_max) {
    const bool half = p.dtype == DT_F16 || p.dtype == DT_BF16 || p.dtype == DT_F16X8 || p.dtype == DT_BF16X8;
    return n >= 1 && n <= small_max && half && !p.cubic && !p.adaptive && deflate == 0 && p.T <= 16;
}

// Products of this matrix run on 256 tiles: plain ones whenever the size
// calls for it, split ones where the split switch also allows it (FP32_EMU
// has no plain products: every stage and the final product are split).
bool plan_big(int64_t n, const StagePlan &p) {
    const bool all_split = p.split_final && p.split_mask == ((1u << p.T) - 1);
    return gemm_use_big(n, p.dtype) && (!all_split || gemm_split_big(p.dtype));
}

size_t align256(size_t b) { return (size_t)round_up((int64_t)b, 256); }

// Leading-dimension padding of the work matrices (elements). A row stride
// that is a multiple of 1024 elements (e.g. n_p = 10240) maps the rows a tile
// streams onto few memory channels: split products at n_p = 10240 ran 13%
// slower than at 10112. Such strides get 128 more elements; others (10112,
// 10368) are left alone, which measured best.
static int64_t g_ld_pad = 128;

// One matrix's workspace inside the arena. With deflation (defl_ld > 0) it
// also holds the Lanczos products X V, the deflation state and buffers, and
// the deflated FP32 copy of X (leading dimension defl_ld, the caller's).
struct MatLayout {
    int64_t n, np, ldw;
    size_t off_scal, off_lz, off_mat, mat_bytes, total;
    size_t off_U = 0, off_defl = 0, off_Z = 0, off_pH = 0, off_pz = 0, off_Xd = 0;
};

MatLayout mat_layout(int64_t n, const StagePlan &p, int steps, int64_t defl_ld) {
    MatLayout L{};
    L.n = n;
    L.np = gemm_padded_size(n, plan_big(n, p));
    L.ldw = (L.np >= 2048 && L.np % 1024 == 0) ? L.np + g_ld_pad : L.np;
    const bool split = any_split(p);
    size_t off = 0;
    auto take = [&](size_t bytes) { const size_t o = off; off += align256(bytes); return o; };
    L.off_scal = take(sizeof(Scalars));
    L.off_lz = take(sizeof(double) * lanczos_work_doubles(n, steps));
    L.mat_bytes = align256(elt_size(p.dtype) * (size_t)L.ldw * (size_t)L.np);
    L.off_mat = take(L.mat_bytes * 4 * (split ? 2 : 1));
    if (defl_ld > 0) {
        const size_t nbv = (size_t)vec_block_count(n);
        L.off_U = take(sizeof(double) * (size_t)n * (size_t)steps);
        L.off_defl = take(sizeof(DeflState));
        L.off_Z = take(sizeof(double) * (size_t)n * kMaxDeflate);
        L.off_pH = take(sizeof(double) * nbv * kMaxLanczos * kMaxLanczos);
        L.off_pz = take(sizeof(double) * nbv * 2 * kMaxDeflate);
        L.off_Xd = take(sizeof(float) * (size_t)defl_ld * (size_t)n);
    }
    L.total = off;
    return L;
}

struct Plan {
    // key
    int mode = -1, steps = 0, split_final = 0;
    int deflate = 0;       // pairs to deflate (single projections only)
    int stages = 0;        // filter stages (with adaptive-depth extras)
    bool adaptive = false;
    int64_t defl_ld = 0;   // caller's leading dimension when deflating
    uint32_t split_mask = 0;
    uint32_t b_mask = 0;
    int small_max = 0;     // the small-matrix rule the plan was laid out for
    std::vector<int64_t> ns;
    // layout
    StagePlan sp;
    // GEMM work lists (gemm_tile_lists): [0] whole rounds of 256 tiles, [1]
    // 128 tiles (small matrices, unsplit tails), [2] 128 tiles of every
    // matrix (split products without the 256 tile); K-chunks and fixups of
    // the split tail tiles, and their partial tiles
    size_t off_desc = 0, off_io = 0, off_wvec = 0, off_wsymv = 0, off_wcast = 0, off_wgemm[3] = {0, 0, 0}, total = 0;
    size_t off_split = 0, off_fixup = 0, off_part = 0, off_adapt = 0;
    int64_t n_vec = 0, n_symv = 0, n_cast = 0, n_gemm[3] = {0, 0, 0}, n_split = 0, n_fixup = 0;
    // matrices of the one-workgroup kernel (their list) and of the launch sequence
    size_t off_wfused = 0;
    int64_t n_fused = 0, n_seq = 0;
    std::vector<bool> fused;
    int gemm_bm[3] = {256, 128, 128};
    TileLists tiles;
    int cus = 256;       // compute units the tail split is sized for
    int tile_gen = -1;   // tuning generation the tile lists were built for
    bool split_big = false;  // split products use the 256/128 lists too
    std::vector<size_t> mat_off;
    std::vector<MatLayout> mats;
    // arena the device tables were built for
    void *base = nullptr;
    // Caller-I/O tables of multi-matrix plans: a ring of kIoRing tables in the
    // arena, each with its pinned staging copy and the event of its last
    // upload. A call whose pointers match a resident table uses it as is (no
    // upload). A table used by a call made while its stream was capturing is
    // pinned: a captured graph reads it at every replay, so no later call
    // overwrites it (until the plan is rebuilt or released).
    struct IoSlot {
        std::vector<IoArg> ios;
        bool valid = false, pinned = false;
        uint64_t used = 0;
        IoArg *host = nullptr;
        hipEvent_t done = nullptr;
    };
    IoSlot io_ring[kIoRing];
    uint64_t io_clock = 0;

    ~Plan() {
        for (IoSlot &r : io_ring) {
            if (r.done) (void)hipEventDestroy(r.done);
            if (r.host) (void)hipHostFree(r.host);
        }
    }
    // rq: the stage plan of the request (mode, split choices)
    bool same_key(const psdproj_opts &o, const StagePlan &rq, int st, const std::vector<int64_t> &n,
                  int64_t dld) const {
        return mode == o.mode && steps == st && split_mask == rq.split_mask && split_final == (int)rq.split_final &&
               ns == n && tile_gen == gemm_tile_generation() && deflate == o.deflate && defl_ld == dld &&
               stages == rq.T && adaptive == rq.adaptive && b_mask == rq.b_mask && small_max == g_small_max.load();
    }
};

void layout_plan(Plan &P) {
    const size_t M = P.ns.size();
    P.mats.clear();
    P.mat_off.clear();
    P.n_vec = P.n_symv = P.n_cast = 0;
    P.n_fused = P.n_seq = 0;
    P.fused.clear();
    std::vector<int64_t> nps;
    std::vector<bool> big;
    std::vector<int> ksplit;
    for (int64_t n : P.ns) {
        P.mats.push_back(mat_layout(n, P.sp, P.steps, P.deflate > 0 ? P.defl_ld : 0));
        const MatLayout &L = P.mats.back();
        const bool f = plan_fused(n, P.sp, P.deflate, P.small_max);
        P.fused.push_back(f);
        if (f) {  // no work items of the sequence: no tiles, no vector blocks
            ++P.n_fused;
            nps.push_back(0);
            big.push_back(false);
            ksplit.push_back(0);
            continue;
        }
        ++P.n_seq;
        P.n_vec += vec_block_count(n);
        P.n_symv += symv_tile_count(n);
        P.n_cast += cast_tile_count(L.np);
        nps.push_back(L.np);
        big.push_back(plan_big(n, P.sp));
        ksplit.push_back(gemm_ksplit_for(n, P.sp.dtype));
    }
    gemm_tile_lists(nps, big, ksplit, P.cus, P.tiles);
    P.n_gemm[0] = (int64_t)P.tiles.big.size();
    P.n_gemm[1] = (int64_t)P.tiles.small_plain.size();
    P.n_gemm[2] = (int64_t)P.tiles.small_all.size();
    P.n_split = (int64_t)P.tiles.split.size();
    P.n_fixup = (int64_t)P.tiles.fixup.size();
    size_t off = 0;
    auto take = [&](size_t bytes) { const size_t o = off; off += align256(bytes); return o; };
    P.off_desc = take(sizeof(MatDesc) * M);
    P.off_io = take(sizeof(IoArg) * M * kIoRing);
    P.off_wvec = take(sizeof(WorkItem) * (size_t)P.n_vec);
    P.off_wsymv = take(sizeof(WorkItem) * (size_t)P.n_symv);
    P.off_wcast = take(sizeof(WorkItem) * (size_t)P.n_cast);
    P.off_wfused = take(sizeof(WorkItem) * (size_t)P.n_fused);
    for (int c = 0; c < 3; ++c) P.off_wgemm[c] = take(sizeof(WorkItem) * (size_t)P.n_gemm[c]);
    P.off_split = take(sizeof(uint4) * (size_t)P.n_split);
    P.off_fixup = take(sizeof(uint4) * (size_t)P.n_fixup);
    P.off_part = take(kPartBytes * (size_t)P.tiles.parts);
    P.off_adapt = take(P.sp.adaptive ? sizeof(double) * 2 * (size_t)P.n_cast : 0);
    for (const MatLayout &L : P.mats) P.mat_off.push_back(take(L.total));
    P.total = off;
}

// Fill and upload the descriptor table and work lists for arena `base`. The
// stream is synchronised first: earlier work queued on it may still read the
// tables being replaced.
int build_tables(Plan &P, void *base, hipStream_t s) {
    const size_t M = P.ns.size();
    for (Plan::IoSlot &r : P.io_ring) r.valid = r.pinned = false;
    uint8_t *b = (uint8_t *)base;
    std::vector<MatDesc> desc(M);
    std::vector<WorkItem> wv, wt, wc, wf;
    std::vector<std::pair<DeflState *, DeflState>> defl_init;
    const bool split = any_split(P.sp);
    for (size_t m = 0; m < M; ++m) {
        const MatLayout &L = P.mats[m];
        uint8_t *mb = b + P.mat_off[m];
        MatDesc &d = desc[m];
        memset(&d, 0, sizeof(d));
        d.n = L.n;
        d.np = L.np;
        d.ldw = L.ldw;
        d.scal = (Scalars *)(mb + L.off_scal);
        fill_lanczos_desc(d, (double *)(mb + L.off_lz), L.n, P.steps);
        for (int k = 0; k < 4; ++k) {
            d.hi[k] = mb + L.off_mat + (size_t)k * L.mat_bytes;
            d.lo[k] = split ? mb + L.off_mat + (size_t)(4 + k) * L.mat_bytes : nullptr;
        }
        if (P.deflate > 0) {
            d.U = (double *)(mb + L.off_U);
            d.defl = (DeflState *)(mb + L.off_defl);
            DeflState ds;
            memset(&ds, 0, sizeof(ds));
            ds.kmax = P.deflate;
            ds.Z = (double *)(mb + L.off_Z);
            ds.pH = (double *)(mb + L.off_pH);
            ds.pz = (double *)(mb + L.off_pz);
            ds.Xd = (float *)(mb + L.off_Xd);
            ds.ldd = P.defl_ld;
            defl_init.push_back(std::make_pair(d.defl, ds));
        }
        if (P.fused[m]) {
            d.fused = 1;
            wf.push_back(WorkItem{(uint32_t)m, 0u});
            continue;
        }
        for (int64_t i = 0; i < vec_block_count(L.n); ++i) wv.push_back(WorkItem{(uint32_t)m, (uint32_t)i});
        for (int64_t i = 0; i < symv_tile_count(L.n); ++i) wt.push_back(WorkItem{(uint32_t)m, (uint32_t)i});
        d.cast_first = (int32_t)wc.size();
        d.cast_count = (int32_t)cast_tile_count(L.np);
        for (int64_t i = 0; i < cast_tile_count(L.np); ++i) wc.push_back(WorkItem{(uint32_t)m, (uint32_t)i});
    }
    const std::vector<WorkItem> *wg[3] = {&P.tiles.big, &P.tiles.small_plain, &P.tiles.small_all};
    if (hipStreamSynchronize(s) != hipSuccess) return PSDPROJ_ERR_HIP;
    auto up = [&](size_t off, const void *src, size_t bytes) {
        return bytes == 0 || hipMemcpy(b + off, src, bytes, hipMemcpyHostToDevice) == hipSuccess;
    };
    if (!up(P.off_desc, desc.data(), sizeof(MatDesc) * M) || !up(P.off_wvec, wv.data(), sizeof(WorkItem) * wv.size()) ||
        !up(P.off_wsymv, wt.data(), sizeof(WorkItem) * wt.size()) ||
        !up(P.off_wcast, wc.data(), sizeof(WorkItem) * wc.size()) ||
        !up(P.off_wfused, wf.data(), sizeof(WorkItem) * wf.size()) ||
        !up(P.off_wgemm[0], wg[0]->data(), sizeof(WorkItem) * wg[0]->size()) ||
        !up(P.off_wgemm[1], wg[1]->data(), sizeof(WorkItem) * wg[1]->size()) ||
        !up(P.off_wgemm[2], wg[2]->data(), sizeof(WorkItem) * wg[2]->size()) ||
        !up(P.off_split, P.tiles.split.data(), sizeof(uint4) * P.tiles.split.size()) ||
        !up(P.off_fixup, P.tiles.fixup.data(), sizeof(uint4) * P.tiles.fixup.size()))
        return PSDPROJ_ERR_HIP;
    for (const auto &di : defl_init)
        if (hipMemcpy(di.first, &di.second, sizeof(DeflState), hipMemcpyHostToDevice) != hipSuccess)
            return PSDPROJ_ERR_HIP;
    P.base = base;
    return PSDPROJ_OK;
}

// ---------------------------------------------------------------------------
// per-(device, stream) workspace pool and current plan
struct Pool {
    void *ptr = nullptr;
    size_t bytes = 0;
    std::unique_ptr<Plan> plan;
};
std::mutex g_mu;
std::map<std::pair<int, hipStream_t>, Pool> g_pool;

int get_workspace(Pool &p, hipStream_t s, size_t bytes, void **out) {
    if (p.bytes < bytes) {
        if (p.ptr) {
            if (hipStreamSynchronize(s) != hipSuccess) return PSDPROJ_ERR_HIP;
            (void)hipFree(p.ptr);
            p.ptr = nullptr;
            p.bytes = 0;
        }
        const size_t want = (size_t)round_up((int64_t)bytes, 1 << 20);
        if (hipMalloc(&p.ptr, want) != hipSuccess) {
            (void)hipGetLastError();
            p.ptr = nullptr;
            return PSDPROJ_ERR_NO_MEMORY;
        }
        p.bytes = want;
    }
    *out = p.ptr;
    return PSDPROJ_OK;
}

// Numerical status of matrix blockIdx.x into the info buffer its I/O names.
__global__ void info_kernel(const MatDesc *D, const IoArg *io_tab, IoArg io0, int stages, int adaptive) {
    if (threadIdx.x != 0) return;
    psdproj_info *info = (psdproj_info *)io_of(io_tab, io0, blockIdx.x).info;
    if (!info) return;
    const Scalars *s = D[blockIdx.x].scal;
    info->lambda = s->lam;
    info->lanczos_lambda = s->lanczos_lam;
    info->sigma = s->sigma;
    info->residual = s->resid;
    info->fro_norm = sqrt(s->fro2);
    info->colmax_norm = sqrt(s->colmax2);
    info->lanczos_steps = s->k;
    info->nonfinite = s->nonfinite;
    info->fallback = s->fallback;
    info->stages = adaptive ? s->stages_run : stages;
    info->deflated = D[blockIdx.x].defl ? D[blockIdx.x].defl->count : 0;
    info->reserved = 0;
}

// Optional event timing of the filter products (psdproj_gemm_timing_*): each
// product's launches are bracketed by two HIP events on the projection's
// stream, tagged with the product's class. Guarded by g_mu like the plans.
struct GemmTimer {
    bool on = false;
    struct Rec {
        int cls;
        hipEvent_t a, b;
    };
    std::vector<Rec> pending;
    std::vector<hipEvent_t> pool;
    hipEvent_t take() {
        hipEvent_t e = nullptr;
        if (!pool.empty()) {
            e = pool.back();
            pool.pop_back();
        } else if (hipEventCreate(&e) != hipSuccess) {
            e = nullptr;
        }
        return e;
    }
};
GemmTimer g_timer;

int gemm_class(bool split_operands, int epi) {
    if (epi == EPI_FINAL) return PSDPROJ_GEMM_FINAL + (split_operands ? 1 : 0);
    return (split_operands ? PSDPROJ_GEMM_PAIR : PSDPROJ_GEMM_PLAIN) + (epi == EPI_STORE_SPLIT ? 1 : 0);
}

bool stream_capturing(hipStream_t s);

// Side stream of a (device, stream) on which the one-workgroup kernel of a
// plan's small matrices overlaps the launch sequence of its other matrices,
// with the events that fork it from the caller's stream and join it back.
// Created outside stream capture only (a capture that finds none runs the
// kernel on the caller's stream: same results, no overlap). Guarded by g_mu.
struct Fork {
    hipStream_t side = nullptr;
    hipEvent_t fork = nullptr, join = nullptr;
};
std::map<std::pair<int, hipStream_t>, Fork> g_fork;

Fork *get_fork(hipStream_t s) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return nullptr;
    auto it = g_fork.find({dev, s});
    if (it != g_fork.end()) return &it->second;
    if (stream_capturing(s)) return nullptr;
    Fork f;
    if (hipStreamCreateWithFlags(&f.side, hipStreamNonBlocking) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    if (hipEventCreateWithFlags(&f.fork, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&f.join, hipEventDisableTiming) != hipSuccess) {
        (void)hipGetLastError();
        if (f.fork) (void)hipEventDestroy(f.fork);
        (void)hipStreamDestroy(f.side);
        return nullptr;
    }
    return &(g_fork[{dev, s}] = f);
}

int run_sequence_of(Plan &P, BatchLaunch B, const psdproj_opts &o, hipStream_t s, bool bound_only);

// Side streams on which the groups of a batched call run beside the caller's
// stream (tuning key "batch_streams": groups per batched call, 1..4; default
// 2), with the event that forks them and one join event each. Created
// outside stream capture only (a capture that finds too few runs the batch
// as one group). Guarded by g_mu.
static std::atomic<int> g_batch_streams{2};
struct BatchFork {
    std::vector<hipStream_t> side;
    hipEvent_t fork = nullptr;
    std::vector<hipEvent_t> join;
};
std::map<std::pair<int, hipStream_t>, BatchFork> g_bfork;

BatchFork *get_bfork(hipStream_t s, int nside, bool capturing) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return nullptr;
    BatchFork &bf = g_bfork[{dev, s}];
    if ((int)bf.side.size() >= nside) return &bf;
    if (capturing) return nullptr;
    if (!bf.fork && hipEventCreateWithFlags(&bf.fork, hipEventDisableTiming) != hipSuccess) {
        (void)hipGetLastError();
        bf.fork = nullptr;
        return nullptr;
    }
    while ((int)bf.side.size() < nside) {
        hipStream_t st = nullptr;
        hipEvent_t ev = nullptr;
        if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
            (void)hipGetLastError();
            return nullptr;
        }
        if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
            (void)hipGetLastError();
            (void)hipStreamDestroy(st);
            return nullptr;
        }
        bf.side.push_back(st);
        bf.join.push_back(ev);
    }
    return &bf;
}

// Enqueue the whole sequence for the plan's matrices. ios: host array of the
// caller's I/O, one per matrix.
int run_plan(Plan &P, const IoArg *ios, const psdproj_opts &o, hipStream_t s, bool want_info, bool bound_only) {
    uint8_t *b = (uint8_t *)P.base;
    const int M = (int)P.ns.size();
    BatchLaunch B;
    B.count = M;
    B.desc = (const MatDesc *)(b + P.off_desc);
    B.w_vec = (const WorkItem *)(b + P.off_wvec);
    B.w_symv = (const WorkItem *)(b + P.off_wsymv);
    B.w_cast = (const WorkItem *)(b + P.off_wcast);
    B.n_vec = P.n_vec;
    B.n_symv = P.n_symv;
    B.n_cast = P.n_cast;
    if (M == 1) {
        B.io_tab = nullptr;
        B.io0 = ios[0];
    } else {
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        if (hipStreamIsCapturing(s, &cs) != hipSuccess) return PSDPROJ_ERR_HIP;
        const bool capturing = cs != hipStreamCaptureStatusNone;
        int hit = -1;
        for (int k = 0; k < kIoRing; ++k) {
            const Plan::IoSlot &r = P.io_ring[k];
            if (r.valid && !memcmp(r.ios.data(), ios, sizeof(IoArg) * M)) hit = k;
        }
        if (hit < 0) {
            // A new table is uploaded through pinned staging with a host-side
            // wait, which stream capture cannot record: capture only calls
            // whose pointers were used before. The table replaced is the least
            // recently used one that no capture holds.
            if (capturing) return PSDPROJ_ERR_UNSUPPORTED;
            for (int k = 0; k < kIoRing; ++k) {
                const Plan::IoSlot &r = P.io_ring[k];
                if (r.pinned) continue;
                if (hit < 0) {
                    hit = k;
                    continue;
                }
                const Plan::IoSlot &h = P.io_ring[hit];
                if (h.valid && (!r.valid || r.used < h.used)) hit = k;
            }
            if (hit < 0) return PSDPROJ_ERR_UNSUPPORTED;  // every table is held by a captured graph
            Plan::IoSlot &r = P.io_ring[hit];
            if (!r.host) {
                if (hipHostMalloc((void **)&r.host, sizeof(IoArg) * M, hipHostMallocDefault) != hipSuccess) {
                    r.host = nullptr;
                    return PSDPROJ_ERR_NO_MEMORY;
                }
                if (hipEventCreateWithFlags(&r.done, hipEventDisableTiming) != hipSuccess) {
                    r.done = nullptr;
                    return PSDPROJ_ERR_HIP;
                }
            } else if (hipEventSynchronize(r.done) != hipSuccess) {  // staging reused once its upload ran
                return PSDPROJ_ERR_HIP;
            }
            memcpy(r.host, ios, sizeof(IoArg) * M);
            r.valid = false;
            IoArg *io_dev = (IoArg *)(b + P.off_io) + (size_t)hit * M;
            if (hipMemcpyAsync(io_dev, r.host, sizeof(IoArg) * M, hipMemcpyHostToDevice, s) != hipSuccess ||
                hipEventRecord(r.done, s) != hipSuccess)
                return PSDPROJ_ERR_HIP;
            r.ios.assign(ios, ios + M);
            r.valid = true;
        }
        Plan::IoSlot &r = P.io_ring[hit];
        r.used = ++P.io_clock;
        if (capturing) r.pinned = true;
        B.io_tab = (const IoArg *)(b + P.off_io) + (size_t)hit * M;
    }
    const StagePlan &p = P.sp;
    Fork *fk = nullptr;
    if (P.n_fused > 0) {
        // every small matrix, whole, in one launch (one workgroup each)
        SmallArgs a{};
        a.D = B.desc;
        a.list = (const WorkItem *)(b + P.off_wfused);
        a.io_tab = B.io_tab;
        a.io0 = B.io0;
        a.T = p.T;
        a.steps = P.steps;
        a.split_mask = p.split_mask | p.b_mask;  // B-only stages split in full here
        a.split_final = p.split_final ? 1 : 0;
        a.bound_only = bound_only ? 1 : 0;
        a.force_fallback = o.force_bound_fallback;
        a.lam_override = o.lambda_override;
        a.seed = kLanczosSeed;
        for (int t = 0; t < p.T; ++t) {
            a.a[t] = (float)p.a[t];
            a.b[t] = (float)p.b[t];
            a.c[t] = (float)p.c[t];
            a.ea[t] = p.ea[t];
            a.eb[t] = p.eb[t];
        }
        for (int t = 0; t <= p.T; ++t) a.ex[t] = p.ex[t];
        // beside the launch sequence of the other matrices, on the side stream
        hipStream_t ks = s;
        if (P.n_seq > 0 && (fk = get_fork(s)) != nullptr) {
            if (hipEventRecord(fk->fork, s) != hipSuccess || hipStreamWaitEvent(fk->side, fk->fork, 0) != hipSuccess)
                return PSDPROJ_ERR_HIP;
            ks = fk->side;
        }
        const hipError_t le = small_proj_launch(a, p.dtype, (int)P.n_fused, ks);
        if (fk && hipEventRecord(fk->join, fk->side) != hipSuccess) return PSDPROJ_ERR_HIP;
        if (le != hipSuccess) {
            if (fk) (void)hipStreamWaitEvent(s, fk->join, 0);
            return PSDPROJ_ERR_HIP;
        }
    }
    const int st = P.n_seq > 0 ? run_sequence_of(P, B, o, s, bound_only) : PSDPROJ_OK;
    // join the side stream whatever the sequence returned
    if (fk && hipStreamWaitEvent(s, fk->join, 0) != hipSuccess) return PSDPROJ_ERR_HIP;
    if (st != PSDPROJ_OK) return st;
    if (want_info)
        hipLaunchKernelGGL(info_kernel, dim3(M), dim3(64), 0, s, B.desc, B.io_tab, B.io0, bound_only ? 0 : p.T,
                           (!bound_only && p.adaptive) ? 1 : 0);
    return hipGetLastError() == hipSuccess ? PSDPROJ_OK : PSDPROJ_ERR_HIP;
}

// The launch sequence of a plan's matrices other than the small ones.
int run_sequence_of(Plan &P, BatchLaunch B, const psdproj_opts &o, hipStream_t s, bool bound_only) {
    uint8_t *b = (uint8_t *)P.base;
    const StagePlan &p = P.sp;
    DeflLaunch DL;
    if (P.deflate > 0 && !bound_only) {
        // deflation (single projections): Lanczos on X recording X V, the
        // converged dominant pairs removed into X', then the whole method on X'
        DL.desc = B.desc;
        DL.w_vec = B.w_vec;
        DL.n_vec = B.n_vec;
        DL.w_tri = B.w_cast;  // 64 x 64 triangle tiles of n_p >= n
        DL.n_tri = B.n_cast;
        DL.io = B.io0;
        if (spectral_bound(B, P.steps, kLanczosSeed, 0, 0.0, s) != hipSuccess ||
            deflate_remove(DL, s) != hipSuccess)
            return PSDPROJ_ERR_HIP;
        B.io0.X = (const float *)((uint8_t *)P.base + P.mat_off[0] + P.mats[0].off_Xd);
    }
    hipError_t e = spectral_bound(B, P.steps, kLanczosSeed, o.force_bound_fallback, o.lambda_override, s);
    if (e != hipSuccess) return PSDPROJ_ERR_HIP;
    if (bound_only) return PSDPROJ_OK;
    const bool x0_split = p.split_final || (p.split_mask & 1u);
    e = cast_x0(B, p.dtype, x0_split, p.ex[0], s);
    if (e != hipSuccess) return PSDPROJ_ERR_HIP;

    GemmArgs g{};
    g.D = B.desc;
    g.part = (float *)(b + P.off_part);
    g.io_tab = B.io_tab;
    g.io0 = B.io0;
    // one product over every matrix, one launch per tile class
    // FP8-pair exponent of the matrix each slot currently holds
    int slot_e[4] = {p.ex[0], 0, 0, 0};
    auto product = [&](int sl, bool ls, int sr, bool rs, int sc0, bool c0s, float alpha, float beta, float gamma,
                       int sd, int epi, int e_out) -> hipError_t {
        g.sl = sl; g.sr = sr; g.sc0 = sc0; g.sd = sd; g.c0_split = c0s ? 1 : 0;
        g.alpha = alpha; g.beta = beta; g.gamma = gamma;
        g.es_l = slot_e[sl]; g.es_r = slot_e[sr]; g.es_c0 = sc0 >= 0 ? slot_e[sc0] : 0; g.es_d = e_out;
        GemmTimer::Rec rec{gemm_class(ls || rs, epi), nullptr, nullptr};
        if (g_timer.on && (rec.a = g_timer.take()) && (rec.b = g_timer.take())) {
            if (hipEventRecord(rec.a, s) != hipSuccess) return hipErrorUnknown;
        }
        // the 256-tile rounds, the K-chunks of the tail tiles and their
        // fixup, then the 128 tiles; split products without the 256 tile: the
        // list of 128 tiles only
        auto launch = [&](int c, int ks) -> hipError_t {
            const int64_t cnt = ks == 0 ? P.n_gemm[c] : (ks == 1 ? P.n_split : P.n_fixup);
            if (!cnt) return hipSuccess;
            g.tiles = (const WorkItem *)(b + P.off_wgemm[c]);
            g.split = (const uint4 *)(b + (ks == 1 ? P.off_split : P.off_fixup));
            return gemm_sym_launch(g, p.dtype, epi, ls, rs, P.gemm_bm[c], cnt, s, ks);
        };
        hipError_t r = hipSuccess;
        if ((ls || rs) && !P.split_big) {
            r = launch(2, 0);
        } else {
            r = launch(0, 0);
            if (r == hipSuccess) r = launch(0, 1);
            if (r == hipSuccess) r = launch(0, 2);
            if (r == hipSuccess) r = launch(1, 0);
        }
        if (r != hipSuccess) return r;
        if (epi != EPI_FINAL) slot_e[sd] = e_out;
        if (rec.b) {
            if (hipEventRecord(rec.b, s) != hipSuccess) return hipErrorUnknown;
            g_timer.pending.push_back(rec);
        }
        return hipSuccess;
    };
    // slot 0 holds X0; slots 1..3 rotate: A -> pa, B -> pb, X' -> pa
    int cur = 0;
    bool cur_split = (p.split_mask & 1u) != 0;
    double *adapt_part = (double *)(b + P.off_adapt);
    // unsplit FP8-pair storage is FP16 / BF16
    const int check_dt = p.dtype == DT_F16X8 ? DT_F16 : p.dtype == DT_BF16X8 ? DT_BF16 : p.dtype;
    // adaptive depth: after stage t (its iterate in slot sn), record the slot
    // once the designed stages are done, and test the change of every
    // skippable stage
    auto check = [&](int t, int sn, int so) -> hipError_t {
        if (!p.adaptive || t + 1 < p.adapt_from) return hipSuccess;
        return stage_check(B, check_dt, sn, so, t + 1, t >= p.adapt_from, o.adaptive_tol, adapt_part, s);
    };
    for (int t = 0; t < p.T; ++t) {
        g.adaptive = (p.adaptive && t >= p.adapt_from) ? 1 : 0;
        const bool sp = (p.split_mask >> t) & 1u;
        const bool bo = (p.b_mask >> t) & 1u;
        // whether X' is stored split: when the next stage splits in full or
        // the final product is split (a B-only stage reads X plain)
        const bool next_split = (t + 1 < p.T) ? ((p.split_mask >> (t + 1)) & 1u) : p.split_final;
        int pa = -1, pb = -1;
        for (int k = 1; k < 4; ++k)
            if (k != cur) { if (pa < 0) pa = k; else if (pb < 0) pb = k; }
        if (p.cubic) {
            // Newton-Schulz step: A = X X, X' = a X + b X A (no split stages)
            e = product(cur, false, cur, false, -1, false, 0.f, 1.f, 0.f, pa, EPI_STORE, p.ea[t]);
            if (e != hipSuccess) return PSDPROJ_ERR_HIP;
            e = product(cur, false, pa, false, cur, false, (float)p.a[t], (float)p.b[t], 0.f, pb, EPI_STORE,
                        p.ex[t + 1]);
            if (e != hipSuccess || check(t, pb, cur) != hipSuccess) return PSDPROJ_ERR_HIP;
            cur = pb;
            continue;
        }
        if (bo) {
            // A = X X; B = b A + c A A, stored as a pair; X' = a X + B X with
            // only B split among the operands (X enters with its hi part; the
            // addend a X takes its pair when X is stored split)
            e = product(cur, false, cur, false, -1, false, 0.f, 1.f, 0.f, pa, EPI_STORE, p.ea[t]);
            if (e != hipSuccess) return PSDPROJ_ERR_HIP;
            e = product(pa, false, pa, false, pa, false, (float)p.b[t], (float)p.c[t], 0.f, pb, EPI_STORE_SPLIT,
                        p.eb[t]);
            if (e != hipSuccess) return PSDPROJ_ERR_HIP;
            e = product(pb, true, cur, false, cur, cur_split, (float)p.a[t], 1.f, 0.f, pa,
                        next_split ? EPI_STORE_SPLIT : EPI_STORE, p.ex[t + 1]);
            if (e != hipSuccess || check(t, pa, cur) != hipSuccess) return PSDPROJ_ERR_HIP;
            cur = pa;
            cur_split = next_split;
            continue;
        }
        const bool xs = sp && cur_split;  // X enters as a pair only in a split stage
        const int st_epi = sp ? EPI_STORE_SPLIT : EPI_STORE;
        // A = X X
        e = product(cur, xs, cur, xs, -1, false, 0.f, 1.f, 0.f, pa, st_epi, p.ea[t]);
        if (e != hipSuccess) return PSDPROJ_ERR_HIP;
        // B = b A + c A A
        e = product(pa, sp, pa, sp, pa, sp, (float)p.b[t], (float)p.c[t], 0.f, pb, st_epi, p.eb[t]);
        if (e != hipSuccess) return PSDPROJ_ERR_HIP;
        // X' = a X + X B
        e = product(cur, xs, pb, sp, cur, cur_split, (float)p.a[t], 1.f, 0.f, pa,
                    next_split ? EPI_STORE_SPLIT : EPI_STORE, p.ex[t + 1]);
        if (e != hipSuccess || check(t, pa, cur) != hipSuccess) return PSDPROJ_ERR_HIP;
        cur = pa;
        cur_split = next_split;
    }
    // out = (X + lam X0 X_T) / 2 (adaptive depth: X_T is the latest iterate's slot)
    g.adaptive = p.adaptive ? 2 : 0;
    e = product(0, p.split_final, cur, p.split_final, -1, false, 0.f, 1.f, 0.f, 0, EPI_FINAL, 0);
    g.adaptive = 0;
    if (e != hipSuccess) return PSDPROJ_ERR_HIP;
    if (P.deflate > 0 && deflate_addback(DL, s) != hipSuccess) return PSDPROJ_ERR_HIP;
    return PSDPROJ_OK;
}

// Plan lookup/creation for (device, stream); builds tables when the shape or
// the arena changed.
// Rebuilding a plan, growing the workspace or uploading tables wait on the
// host, which stream capture cannot record: they are refused while the stream
// is capturing (queried only when one of them is due).
bool stream_capturing(hipStream_t s) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    return hipStreamIsCapturing(s, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone;
}

// A laid-out plan (no device memory yet) for the call shape on device dev.
std::unique_ptr<Plan> new_plan(const psdproj_opts &o, const StagePlan &sp, int steps, const std::vector<int64_t> &ns,
                               int64_t defl_ld, int dev) {
    std::unique_ptr<Plan> P(new Plan());
    P->mode = o.mode;
    P->deflate = o.deflate;
    P->defl_ld = defl_ld;
    P->stages = sp.T;
    P->adaptive = sp.adaptive;
    P->steps = steps;
    P->sp = sp;
    P->split_mask = sp.split_mask;
    P->split_final = sp.split_final;
    P->b_mask = sp.b_mask;
    P->small_max = g_small_max.load();
    P->ns = ns;
    P->tile_gen = gemm_tile_generation();
    P->split_big = gemm_split_big(sp.dtype);
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0) cus = 256;
    P->cus = gemm_tail_cus(cus);
    layout_plan(*P);
    return P;
}

// capture_hint: treat s as capturing (a side stream that a captured call is
// about to fork is not capturing yet).
int prepare(const psdproj_opts &o, int steps, const std::vector<int64_t> &ns, int64_t defl_ld, hipStream_t s,
            Plan **out, bool capture_hint = false) {
    load_env_tune_cache();
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return PSDPROJ_ERR_HIP;
    StagePlan sp;
    if (!make_stage_plan(o, sp)) return PSDPROJ_ERR_INVALID_ARG;
    Pool &pool = g_pool[{dev, s}];
    auto capturing = [&]() { return capture_hint || stream_capturing(s); };
    if (!pool.plan || !pool.plan->same_key(o, sp, steps, ns, defl_ld)) {
        if (capturing()) return PSDPROJ_ERR_UNSUPPORTED;
        std::unique_ptr<Plan> P = new_plan(o, sp, steps, ns, defl_ld, dev);
        if (pool.plan && hipStreamSynchronize(s) != hipSuccess) return PSDPROJ_ERR_HIP;
        pool.plan = std::move(P);
    }
    Plan &P = *pool.plan;
    if ((pool.bytes < P.total || P.base != pool.ptr) && capturing()) return PSDPROJ_ERR_UNSUPPORTED;
    void *base = nullptr;
    const int st = get_workspace(pool, s, P.total, &base);
    if (st != PSDPROJ_OK) return st;
    if (P.base != base) {
        const int bt = build_tables(P, base, s);
        if (bt != PSDPROJ_OK) return bt;
    }
    *out = &P;
    return PSDPROJ_OK;
}

// ---------------------------------------------------------------------------
// Allocation-free projections: the arena is the fixed device array `scratch`
// (file scope, below) instead of pooled hipMalloc memory. Each device has its
// own copy of the array, at the address hipGetSymbolAddress returns once per
// device, and one plan: every such call on a device shares the array, and a
// call whose shape differs from the previous one rebuilds the tables in it.
// Nothing in the arena has to start at zero (the kernels write every work
// matrix, padding included, before reading it, and no kernel accumulates
// into workspace memory across launches).
struct ScratchPool {
    uint8_t *ptr = nullptr;  // this device's copy of `scratch`
    std::unique_ptr<Plan> plan;
    hipStream_t last = nullptr;  // stream of the previous call
};
std::map<int, ScratchPool> g_scratch;  // per device, guarded by g_mu

// Device address of this device's copy of `scratch` (the current device's;
// called once per device, with that device current).
int scratch_address(void **p) {
    *p = nullptr;
    if (hipGetSymbolAddress(p, HIP_SYMBOL(scratch)) != hipSuccess || !*p) {
        (void)hipGetLastError();
        *p = nullptr;
        return PSDPROJ_ERR_HIP;
    }
    return PSDPROJ_OK;
}

int prepare_scratch(const psdproj_opts &o, int steps, int64_t n, int64_t defl_ld, hipStream_t s, Plan **out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return PSDPROJ_ERR_HIP;
    StagePlan sp;
    if (!make_stage_plan(o, sp)) return PSDPROJ_ERR_INVALID_ARG;
    ScratchPool &sc = g_scratch[dev];
    if (!sc.ptr) {
        void *p = nullptr;
        const int st = scratch_address(&p);
        if (st != PSDPROJ_OK) return st;
        sc.ptr = (uint8_t *)p;
    }
    const std::vector<int64_t> ns{n};
    if (!sc.plan || !sc.plan->same_key(o, sp, steps, ns, defl_ld)) {
        std::unique_ptr<Plan> P = new_plan(o, sp, steps, ns, defl_ld, dev);
        if (P->total > (size_t)PSDPROJ_NOALLOC_SCRATCH_BYTES) return PSDPROJ_ERR_TOO_LARGE;
        if (stream_capturing(s)) return PSDPROJ_ERR_UNSUPPORTED;
        // The previous call may still read the tables being replaced: on
        // another stream it is awaited here, on this one by build_tables.
        if (sc.plan && sc.last != s && hipDeviceSynchronize() != hipSuccess) return PSDPROJ_ERR_HIP;
        sc.plan = std::move(P);
        const int bt = build_tables(*sc.plan, sc.ptr, s);
        if (bt != PSDPROJ_OK) {
            sc.plan.reset();
            return bt;
        }
    }
    sc.last = s;
    *out = sc.plan.get();
    return PSDPROJ_OK;
}

}  // namespace

// Launch errors are read with hipGetLastError; a call first clears whatever
// error an earlier runtime call of the thread (another library's included)
// left pending, so a failure it reports is its own.
int run_projection(const psdproj_opts &o, int64_t n, int64_t ld, const float *X, float *out, hipStream_t s,
                   psdproj_info *info, bool bound_only, bool no_alloc) {
    (void)hipGetLastError();
    StagePlan tmp;
    if (!make_stage_plan(o, tmp)) return PSDPROJ_ERR_INVALID_ARG;
    const int steps = o.lanczos_steps ? o.lanczos_steps : kDefaultLanczos;
    if (steps < 1 || steps > kMaxLanczos) return PSDPROJ_ERR_INVALID_ARG;
    if (n < 0 || ld < (n > 1 ? n : 1)) return PSDPROJ_ERR_INVALID_ARG;
    if (n == 0) return PSDPROJ_OK;
    if (!X || (!out && !bound_only)) return PSDPROJ_ERR_INVALID_ARG;
    if (n > (int64_t)1 << 20) return PSDPROJ_ERR_UNSUPPORTED;
    if (o.deflate < 0 || o.deflate > kMaxDeflate) return PSDPROJ_ERR_INVALID_ARG;
    if (tmp.adaptive && any_split(tmp)) return PSDPROJ_ERR_UNSUPPORTED;
    psdproj_opts oo = o;
    if (bound_only) oo.deflate = 0;
    const int64_t defl_ld = oo.deflate > 0 ? ld : 0;
    std::lock_guard<std::mutex> lk(g_mu);
    Plan *P = nullptr;
    const int st = no_alloc ? prepare_scratch(oo, steps, n, defl_ld, s, &P)
                            : prepare(oo, steps, std::vector<int64_t>{n}, defl_ld, s, &P);
    if (st != PSDPROJ_OK) return st;
    const IoArg io{X, out, ld, info};
    return run_plan(*P, &io, o, s, info != nullptr, bound_only);
}

int run_batched(const psdproj_opts &o, int count, const int64_t *n, const int64_t *ld, const float *const *X,
                float *const *out, hipStream_t s, psdproj_info *info) {
    (void)hipGetLastError();  // see run_projection
    StagePlan tmp;
    if (!make_stage_plan(o, tmp)) return PSDPROJ_ERR_INVALID_ARG;
    if (count < 0 || (count > 0 && (!n || !ld || !X || !out))) return PSDPROJ_ERR_INVALID_ARG;
    std::vector<int64_t> ns;
    std::vector<IoArg> ios;
    for (int i = 0; i < count; ++i) {
        if (n[i] < 0 || ld[i] < (n[i] > 1 ? n[i] : 1) || (n[i] > 0 && (!X[i] || !out[i])))
            return PSDPROJ_ERR_INVALID_ARG;
        if (n[i] > (int64_t)1 << 20) return PSDPROJ_ERR_UNSUPPORTED;
        if (n[i] == 0) continue;
        ns.push_back(n[i]);
        ios.push_back(IoArg{X[i], out[i], ld[i], info ? (void *)(info + i) : nullptr});
    }
    if (o.deflate < 0 || o.deflate > kMaxDeflate) return PSDPROJ_ERR_INVALID_ARG;
    if (o.deflate > 0) return PSDPROJ_ERR_UNSUPPORTED;  // deflation: single projections only
    if (tmp.adaptive && any_split(tmp)) return PSDPROJ_ERR_UNSUPPORTED;
    if (ns.empty()) return PSDPROJ_OK;
    const int steps = o.lanczos_steps ? o.lanczos_steps : kDefaultLanczos;
    if (steps < 1 || steps > kMaxLanczos) return PSDPROJ_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(g_mu);
    // Groups on concurrent streams: the launch sequence of a batch is bound
    // by latency (every launch waits for the previous one, and most leave CUs
    // idle), so two groups' sequences overlap. The matrices of the
    // one-workgroup kernel stay in group 0, on the caller's stream (its own
    // fork then comes from the caller's stream; a side stream never forks
    // again); the others are dealt out largest first (cost n^3) to the group
    // with the least cost so far.
    int G = std::min<int>(g_batch_streams.load(), (int)ns.size());
    std::vector<std::vector<int>> grp(G > 1 ? G : 1);
    if (G > 1) {
        std::vector<int> order;
        for (size_t i = 0; i < ns.size(); ++i) {
            if (plan_fused(ns[i], tmp, o.deflate, g_small_max.load())) grp[0].push_back((int)i);
            else order.push_back((int)i);
        }
        auto cost = [&](int i) { const double m = (double)ns[i]; return m * m * m; };
        std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost(a) > cost(b); });
        std::vector<double> load(G, 0.0);
        for (int i : order) {
            const int g = (int)(std::min_element(load.begin(), load.end()) - load.begin());
            grp[g].push_back(i);
            load[g] += cost(i);
        }
        // drop empty groups (group 0 may be empty only if every matrix is large)
        std::vector<std::vector<int>> keep;
        for (int g = 0; g < G; ++g)
            if (!grp[g].empty() || g == 0) keep.push_back(grp[g]);
        if (keep[0].empty()) keep.erase(keep.begin());
        grp.swap(keep);
        G = (int)grp.size();
    }
    if (G > 1) {
        for (auto &v : grp) std::sort(v.begin(), v.end());  // each group in the caller's order
        const bool cap = stream_capturing(s);
        BatchFork *bf = get_bfork(s, G - 1, cap);
        if (bf) {
            std::vector<Plan *> plans(G, nullptr);
            std::vector<std::vector<IoArg>> gio(G);
            auto stream_of = [&](int g) { return g == 0 ? s : bf->side[g - 1]; };
            for (int g = 0; g < G; ++g) {
                std::vector<int64_t> gn;
                for (int i : grp[g]) {
                    gn.push_back(ns[i]);
                    gio[g].push_back(ios[i]);
                }
                const int st = prepare(o, steps, gn, 0, stream_of(g), &plans[g], cap);
                if (st != PSDPROJ_OK) return st;
            }
            if (hipEventRecord(bf->fork, s) != hipSuccess) return PSDPROJ_ERR_HIP;
            for (int g = 1; g < G; ++g)
                if (hipStreamWaitEvent(stream_of(g), bf->fork, 0) != hipSuccess) return PSDPROJ_ERR_HIP;
            int st = PSDPROJ_OK;
            for (int g = 0; g < G; ++g) {
                const int sg = run_plan(*plans[g], gio[g].data(), o, stream_of(g), info != nullptr, false);
                if (st == PSDPROJ_OK) st = sg;
            }
            // join every side stream whatever the groups returned
            for (int g = 1; g < G; ++g)
                if (hipEventRecord(bf->join[g - 1], stream_of(g)) != hipSuccess ||
                    hipStreamWaitEvent(s, bf->join[g - 1], 0) != hipSuccess)
                    st = PSDPROJ_ERR_HIP;
            return st;
        }
    }
    Plan *P = nullptr;
    const int st = prepare(o, steps, ns, 0, s, &P);
    if (st != PSDPROJ_OK) return st;
    return run_plan(*P, ios.data(), o, s, info != nullptr, false);
}

psdproj_opts default_opts(int mode) {
    psdproj_opts o;
    memset(&o, 0, sizeof(o));
    o.mode = mode;
    o.split_final = -1;
    return o;
}

int mode_dtype(int mode) {
    psdproj_opts o = default_opts(mode);
    StagePlan sp;
    return make_stage_plan(o, sp) ? sp.dtype : -1;
}

size_t workspace_bytes_batch(const int64_t *ns, int count, int mode) {
    psdproj_opts o = default_opts(mode);
    StagePlan sp;
    if (count <= 0 || !make_stage_plan(o, sp)) return 0;
    Plan P;
    P.sp = sp;
    P.steps = kDefaultLanczos;
    for (int i = 0; i < count; ++i) {
        if (ns[i] <= 0) return 0;
        P.ns.push_back(ns[i]);
    }
    layout_plan(P);
    return P.total;
}

size_t workspace_bytes_for(int64_t n, int mode) { return workspace_bytes_batch(&n, 1, mode); }

// The workspace a stream's calls hold: its own pool and those of the side
// streams its batched calls run groups on.
size_t pool_held(hipStream_t s) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    std::lock_guard<std::mutex> lk(g_mu);
    size_t held = 0;
    auto add = [&](hipStream_t st) {
        auto it = g_pool.find({dev, st});
        if (it != g_pool.end()) held += it->second.bytes;
    };
    add(s);
    auto bf = g_bfork.find({dev, s});
    if (bf != g_bfork.end())
        for (hipStream_t st : bf->second.side) add(st);
    return held;
}

void pool_release(hipStream_t s) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return;
    std::lock_guard<std::mutex> lk(g_mu);
    auto drop = [&](hipStream_t st) {
        auto it = g_pool.find({dev, st});
        if (it == g_pool.end()) return;
        (void)hipStreamSynchronize(st);
        it->second.plan.reset();
        if (it->second.ptr) (void)hipFree(it->second.ptr);
        g_pool.erase(it);
    };
    auto bf = g_bfork.find({dev, s});
    if (bf != g_bfork.end())
        for (hipStream_t st : bf->second.side) drop(st);
    drop(s);
}

double gemm_count_for(const psdproj_opts &o) {
    StagePlan p;
    if (!make_stage_plan(o, p)) return -1;
    // an FP16 pair product is 3 FP16 products (2 with one operand split); an
    // FP8 pair product is one FP16 product plus one FP8 product of twice the K
    // at twice the rate (one-sided: of the same K, 1.5 in all)
    if (p.cubic) return 2 * p.T + 1;
    const bool x8 = p.dtype == DT_F16X8 || p.dtype == DT_BF16X8;
    const double pair = x8 ? 2.0 : 3.0;
    const double one = x8 ? 1.5 : 2.0;
    double g = 0;
    bool cur_split = (p.split_mask & 1u) != 0;
    for (int t = 0; t < p.T; ++t) {
        const bool sp = (p.split_mask >> t) & 1u;
        const bool next_split = (t + 1 < p.T) ? ((p.split_mask >> (t + 1)) & 1u) : p.split_final;
        const bool xs = sp && cur_split;
        if ((p.b_mask >> t) & 1u) {
            g += 2.0 + one;  // X X and A A plain, B X one-sided
        } else {
            g += xs ? pair : 1;               // X X
            g += sp ? pair : 1;               // A A
            g += sp ? (xs ? pair : one) : 1;  // X B
        }
        cur_split = next_split;
    }
    // a split final product multiplies X0 and X_T, both stored split
    g += p.split_final ? pair : 1;
    return g;
}

}  // namespace psd

using namespace psd;

// psdproj_sym_gemm keeps the descriptor and tile list of its last call per
// device, so repeated calls with the same operands are bare kernel launches.
struct SymGemmCache {
    MatDesc d{};
    int bm = 0;
    std::vector<WorkItem> tiles;
    void *buf = nullptr;
    size_t bytes = 0;
};
static std::mutex g_sg_mu;
static std::map<int, SymGemmCache> g_sg;

extern "C" {

int psdproj_project(int64_t n, int64_t ld, const float *X, float *out, int mode, psdproj_stream_t stream) {
    const psdproj_opts o = default_opts(mode);
    return run_projection(o, n, ld, X, out, (hipStream_t)stream, nullptr, false, false);
}

int psdproj_project_ex(const psdproj_opts *opts, int64_t n, int64_t ld, const float *X, float *out,
                       psdproj_stream_t stream, psdproj_info *info_dev) {
    if (!opts) return PSDPROJ_ERR_INVALID_ARG;
    return run_projection(*opts, n, ld, X, out, (hipStream_t)stream, info_dev, false, false);
}

int psdproj_project_noalloc(const psdproj_opts *opts, int64_t n, int64_t ld, const float *X, float *out,
                            psdproj_stream_t stream, psdproj_info *info_dev) {
    if (!opts) return PSDPROJ_ERR_INVALID_ARG;
    return run_projection(*opts, n, ld, X, out, (hipStream_t)stream, info_dev, false, true);
}

int psdproj_spectral_bound(int64_t n, int64_t ld, const float *X, int lanczos_steps, psdproj_stream_t stream,
                           psdproj_info *info_dev) {
    if (!info_dev) return PSDPROJ_ERR_INVALID_ARG;
    psdproj_opts o = default_opts(PSDPROJ_MODE_FP32);
    o.lanczos_steps = lanczos_steps;
    return run_projection(o, n, ld, X, nullptr, (hipStream_t)stream, info_dev, true, false);
}

int psdproj_project_batched(int count, const int64_t *n, const int64_t *ld, const float *const *X, float *const *out,
                            int mode, psdproj_stream_t stream) {
    const psdproj_opts o = default_opts(mode);
    return run_batched(o, count, n, ld, X, out, (hipStream_t)stream, nullptr);
}

int psdproj_project_batched_ex(const psdproj_opts *opts, int count, const int64_t *n, const int64_t *ld,
                               const float *const *X, float *const *out, psdproj_stream_t stream,
                               psdproj_info *info_dev) {
    if (!opts) return PSDPROJ_ERR_INVALID_ARG;
    return run_batched(*opts, count, n, ld, X, out, (hipStream_t)stream, info_dev);
}

size_t psdproj_workspace_bytes(int64_t n, int mode) { return workspace_bytes_for(n, mode); }

double psdproj_gemm_count(const psdproj_opts *opts, int mode) {
    psdproj_opts o = opts ? *opts : default_opts(mode);
    return gemm_count_for(o);
}

int psdproj_coefficients(int mode, double *abc, int cap) {
    psdproj_opts o = default_opts(mode);
    StagePlan p;
    if (!make_stage_plan(o, p) || !abc || cap < 3 * p.T) return -1;
    for (int t = 0; t < p.T; ++t) {
        abc[3 * t] = p.a[t];
        abc[3 * t + 1] = p.b[t];
        abc[3 * t + 2] = p.c[t];
    }
    return p.T;
}

int psdproj_release(void) {
    std::lock_guard<std::mutex> lk(g_mu);
    if (hipDeviceSynchronize() != hipSuccess) return PSDPROJ_ERR_HIP;
    for (auto &kv : g_pool) {
        kv.second.plan.reset();
        if (kv.second.ptr) (void)hipFree(kv.second.ptr);
    }
    g_pool.clear();
    for (auto &kv : g_fork) {
        (void)hipEventDestroy(kv.second.fork);
        (void)hipEventDestroy(kv.second.join);
        (void)hipStreamDestroy(kv.second.side);
    }
    g_fork.clear();
    for (auto &kv : g_bfork) {
        if (kv.second.fork) (void)hipEventDestroy(kv.second.fork);
        for (hipEvent_t e : kv.second.join) (void)hipEventDestroy(e);
        for (hipStream_t st : kv.second.side) (void)hipStreamDestroy(st);  // their pools and forks went above
    }
    g_bfork.clear();
    for (auto &r : g_timer.pending) {
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    g_timer.pending.clear();
    for (hipEvent_t e : g_timer.pool) (void)hipEventDestroy(e);
    g_timer.pool.clear();
    std::lock_guard<std::mutex> lk2(g_sg_mu);
    for (auto &kv : g_sg)
        if (kv.second.buf) (void)hipFree(kv.second.buf);
    g_sg.clear();
    return PSDPROJ_OK;
}

int psdproj_gemm_timing_start(void) {
    std::lock_guard<std::mutex> lk(g_mu);
    for (auto &r : g_timer.pending) {
        (void)hipEventSynchronize(r.b);
        g_timer.pool.push_back(r.a);
        g_timer.pool.push_back(r.b);
    }
    g_timer.pending.clear();
    g_timer.on = true;
    return PSDPROJ_OK;
}

int psdproj_gemm_timing_stop(psdproj_gemm_timing_entry *out, int cap) {
    std::lock_guard<std::mutex> lk(g_mu);
    g_timer.on = false;
    psdproj_gemm_timing_entry acc[PSDPROJ_GEMM_CLASSES] = {};
    int status = PSDPROJ_OK;
    for (auto &r : g_timer.pending) {
        float ms = 0.0f;
        if (hipEventSynchronize(r.b) != hipSuccess || hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess)
            status = PSDPROJ_ERR_HIP;
        acc[r.cls].launches += 1;
        acc[r.cls].total_ms += ms;
        g_timer.pool.push_back(r.a);
        g_timer.pool.push_back(r.b);
    }
    g_timer.pending.clear();
    if (out)
        for (int c = 0; c < cap && c < PSDPROJ_GEMM_CLASSES; ++c) out[c] = acc[c];
    return status;
}

int psdproj_tune(const char *key, int64_t value) {
    if (!key) return PSDPROJ_ERR_INVALID_ARG;
    if (!strcmp(key, "gemm_tile")) {
        if (value != 0 && value != 128 && value != 256) return PSDPROJ_ERR_INVALID_ARG;
        gemm_set_tile_override((int)value);
        return PSDPROJ_OK;
    }
    if (!strcmp(key, "work_ld_pad")) {  // leading-dimension padding of large work matrices
        if (value < 0 || value > 4096 || value % 64) return PSDPROJ_ERR_INVALID_ARG;
        std::lock_guard<std::mutex> lk(g_mu);
        if (hipDeviceSynchronize() != hipSuccess) return PSDPROJ_ERR_HIP;  // plans in flight
        g_ld_pad = value;
        for (auto &kv : g_pool) kv.second.plan.reset();  // layouts change: rebuild plans
        for (auto &kv : g_scratch) kv.second.plan.reset();
        return PSDPROJ_OK;
    }
    if (!strcmp(key, "batch_streams")) {  // concurrent groups of a batched call (1..4)
        if (value < 1 || value > 4) return PSDPROJ_ERR_INVALID_ARG;
        g_batch_streams = (int)value;
        return PSDPROJ_OK;
    }
    if (!strcmp(key, "small_max")) {  // largest order of the one-workgroup kernel (0: never)
        if (value < 0 || value > kSmallEdge) return PSDPROJ_ERR_INVALID_ARG;
        g_small_max = (int)value;
        return PSDPROJ_OK;
    }
    if (!strcmp(key, "class_choices_clear")) {  // drop the autotuner's per-size-class choices
        gemm_clear_class_choices();
        return PSDPROJ_OK;
    }
    if (!strcmp(key, "gemm_big_min")) {  // products of n >= value use the 256 tile (0: default)
        if (value < 0) return PSDPROJ_ERR_INVALID_ARG;
        gemm_set_big_min(value);
        return PSDPROJ_OK;
    }
    if (!strcmp(key, "gemm_tail_cus")) {  // CU count of the tail rule (0: the device's)
        if (value < 0 || value > 65536) return PSDPROJ_ERR_INVALID_ARG;
        gemm_set_tail_cus((int)value);
        return PSDPROJ_OK;
    }
    if (!strcmp(key, "gemm_split_big")) {  // bit 0: FP16/BF16 pairs, bit 1: FP8 pairs on 256 tiles
        if (value < 0 || value > 3) return PSDPROJ_ERR_INVALID_ARG;
        gemm_set_split_big((int)value);
        return PSDPROJ_OK;
    }
    if (!strcmp(key, "gemm_ksplit")) {  // most K-chunks of a tail tile (1: never split)
        if (value < 1 || value > 64) return PSDPROJ_ERR_INVALID_ARG;
        gemm_set_ksplit_max((int)value);
        return PSDPROJ_OK;
    }
    if (!strcmp(key, "gemm_block")) {  // value = H * 256 + W
        const int h = (int)(value >> 8), w = (int)(value & 255);
        if (h < 1 || w < 1 || h > 64 || w > 64) return PSDPROJ_ERR_INVALID_ARG;
        gemm_set_block_shape(h, w);
        return PSDPROJ_OK;
    }
    return PSDPROJ_ERR_NOT_FOUND;
}

const char *psdproj_status_string(int status) {
    switch (status) {
        case PSDPROJ_OK: return "ok";
        case PSDPROJ_ERR_INVALID_ARG: return "invalid argument";
        case PSDPROJ_ERR_UNSUPPORTED: return "unsupported";
        case PSDPROJ_ERR_NO_MEMORY: return "out of device memory";
        case PSDPROJ_ERR_HIP: return "HIP error";
        case PSDPROJ_ERR_REJECTED: return "rejected";
        case PSDPROJ_ERR_CANCELLED: return "cancelled";
        case PSDPROJ_ERR_TIMEOUT: return "timeout";
        case PSDPROJ_ERR_NOT_FOUND: return "not found";
        case PSDPROJ_ERR_PENDING: return "pending";
        case PSDPROJ_ERR_NONFINITE: return "non-finite input";
        case PSDPROJ_ERR_TOO_LARGE: return "workspace exceeds the fixed scratch of the allocation-free entry point";
    }
    return "unknown status";
}

// Kernel-level product on caller buffers (tests and tooling): a one-matrix
// descriptor whose slots are the given buffers; queued on the stream.
static int sym_gemm_impl(int dtype, int64_t n_p, int64_t ld, const void *L, const void *Llo, const void *R,
                         const void *Rlo, const void *C0, const void *C0lo, float alpha, float beta, float gamma,
                         void *D, void *Dlo, const int *es, hipStream_t s) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return PSDPROJ_ERR_HIP;
    MatDesc d;
    memset(&d, 0, sizeof(d));
    d.n = n_p;
    d.np = n_p;
    d.ldw = ld;
    d.hi[0] = (void *)L; d.lo[0] = (void *)Llo;
    d.hi[1] = (void *)R; d.lo[1] = (void *)Rlo;
    d.hi[2] = (void *)C0; d.lo[2] = (void *)C0lo;
    d.hi[3] = D; d.lo[3] = Dlo;
    const int bm = gemm_pick_tile(n_p, dtype);
    std::vector<WorkItem> tiles;
    append_tile_order(tiles, 0, (int)(n_p / bm));
    std::lock_guard<std::mutex> lk(g_sg_mu);
    SymGemmCache &c = g_sg[dev];
    const bool same = c.buf && c.bm == bm && c.tiles.size() == tiles.size() && !memcmp(&c.d, &d, sizeof(d)) &&
                      !memcmp(c.tiles.data(), tiles.data(), sizeof(WorkItem) * tiles.size());
    if (!same) {
        // The cached copy may still be read by a launch in flight.
        if (hipDeviceSynchronize() != hipSuccess) return PSDPROJ_ERR_HIP;
        const size_t bytes = align256(sizeof(MatDesc)) + sizeof(WorkItem) * tiles.size();
        if (bytes > c.bytes) {
            if (c.buf) (void)hipFree(c.buf);
            c.buf = nullptr;
            c.bytes = 0;
            if (hipMalloc(&c.buf, bytes) != hipSuccess) {
                c.buf = nullptr;
                return PSDPROJ_ERR_NO_MEMORY;
            }
            c.bytes = bytes;
        }
        c.tiles.clear();  // invalid until both uploads succeed
        WorkItem *wt = (WorkItem *)((uint8_t *)c.buf + align256(sizeof(MatDesc)));
        if (hipMemcpy(c.buf, &d, sizeof(d), hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(wt, tiles.data(), sizeof(WorkItem) * tiles.size(), hipMemcpyHostToDevice) != hipSuccess)
            return PSDPROJ_ERR_HIP;
        c.d = d;
        c.bm = bm;
        c.tiles = tiles;
    }
    GemmArgs g{};
    g.D = (const MatDesc *)c.buf;
    g.tiles = (const WorkItem *)((uint8_t *)c.buf + align256(sizeof(MatDesc)));
    g.sl = 0; g.sr = 1; g.sc0 = C0 ? 2 : -1; g.sd = 3; g.c0_split = C0lo ? 1 : 0;
    g.alpha = alpha; g.beta = beta; g.gamma = gamma;
    if (es) { g.es_l = es[0]; g.es_r = es[1]; g.es_c0 = es[2]; g.es_d = es[3]; }
    (void)hipGetLastError();  // see run_projection
    const hipError_t e = gemm_sym_launch(g, dtype, Dlo ? EPI_STORE_SPLIT : EPI_STORE, Llo != nullptr, Rlo != nullptr,
                                         bm, (int64_t)tiles.size(), s);
    return e == hipSuccess ? PSDPROJ_OK : PSDPROJ_ERR_HIP;
}

int psdproj_sym_gemm(int dtype, int64_t n_p, int64_t ld, const void *L, const void *Llo, const void *R,
                     const void *Rlo, const void *C0, const void *C0lo, float alpha, float beta, float gamma, void *D,
                     void *Dlo, psdproj_stream_t stream) {
    if (dtype < 0 || dtype > 2 || n_p <= 0 || n_p % kTile || ld < n_p || !L || !R || !D) return PSDPROJ_ERR_INVALID_ARG;
    if (dtype == DT_F32 && (Llo || Rlo || Dlo || C0lo)) return PSDPROJ_ERR_UNSUPPORTED;
    return sym_gemm_impl(dtype, n_p, ld, L, Llo, R, Rlo, C0, C0lo, alpha, beta, gamma, D, Dlo, nullptr,
                         (hipStream_t)stream);
}

int psdproj_sym_gemm_pair8(int64_t n_p, int64_t ld, const void *L, const void *Lx, const void *R, const void *Rx,
                           const void *C0, const void *C0x, float alpha, float beta, float gamma, void *D, void *Dx,
                           int e_l, int e_r, int e_c0, int e_d, psdproj_stream_t stream) {
    if (n_p <= 0 || n_p % kTile || ld < n_p || !L || !R || !D || (C0x && !C0)) return PSDPROJ_ERR_INVALID_ARG;
    if (Rx && !Lx) return PSDPROJ_ERR_UNSUPPORTED;  // one-sided: the split operand is L
    const int es[4] = {e_l, e_r, e_c0, e_d};
    for (int e : es)
        if (e < -40 || e > 40) return PSDPROJ_ERR_INVALID_ARG;
    return sym_gemm_impl(DT_F16X8, n_p, ld, L, Lx, R, Rx, C0, C0x, alpha, beta, gamma, D, Dx, es,
                         (hipStream_t)stream);
}

int psdproj_sym_gemm_pair8_bf16(int64_t n_p, int64_t ld, const void *L, const void *Lx, const void *R, const void *Rx,
                                const void *C0, const void *C0x, float alpha, float beta, float gamma, void *D,
                                void *Dx, int e_l, int e_r, int e_c0, int e_d, psdproj_stream_t stream) {
    if (n_p <= 0 || n_p % kTile || ld < n_p || !L || !R || !D || (C0x && !C0)) return PSDPROJ_ERR_INVALID_ARG;
    if (Rx && !Lx) return PSDPROJ_ERR_UNSUPPORTED;
    const int es[4] = {e_l, e_r, e_c0, e_d};
    for (int e : es)
        if (e < -40 || e > 40) return PSDPROJ_ERR_INVALID_ARG;
    return sym_gemm_impl(DT_BF16X8, n_p, ld, L, Lx, R, Rx, C0, C0x, alpha, beta, gamma, D, Dx, es,
                         (hipStream_t)stream);
}

}  // extern "C"

// Symmetric MFMA GEMM with fused filter-stage epilogues (gfx950).
//
// Every product in the composite filter multiplies two polynomials in the same
// symmetric matrix X, so operands and results are symmetric and commute
// (Section 1, eq. (4): p(X) = Q p(Lambda) Q^T). The kernel therefore
//   * computes only the upper-triangle tiles (bi <= bj) of C = L * R,
//   * reads both operands along contiguous columns: C(i,j) = sum_k L(k,i) R(k,j)
//     because L(i,k) = L(k,i) — the "TN" form in which each lane's 16-byte
//     fragment is contiguous in K for both MFMA operands,
//   * writes every tile twice (tile and mirror), so the next product again
//     sees a full symmetric matrix; diagonal tiles write only i <= j so the
//     stored result is bitwise symmetric.
//
// The epilogue forms one filter step in the output tile (Algorithm 2, stage
// f_t(X) = a X + b X^3 + c X^5 evaluated as A = X X, B = b A + c A A,
// X' = a X + X B):  D = alpha * C0 + beta * acc + gamma * I, with C0 a
// symmetric addend read from the same tile. The final epilogue forms
// P = (X + lam X0 X_T) / 2 in FP32 and drops the zero padding.
//
// Split ("hi + lo") operands: a matrix M may be carried as M_hi = round(M) and
// M_lo = round((M - M_hi) * S) (S = 2^11 for FP16, 1 for BF16). A split product
// accumulates L_hi (S R_hi) + L_hi R_lo + L_lo R_hi into one FP32 accumulator
// (R_hi is scaled by S in registers, exact for |R| < 32) and the epilogue
// multiplies by 1/S.
//
// This header holds the kernel template and its launch templates; each
// gemm_launch_*.hip instantiates them for one work precision, so the
// instantiations compile in parallel. gemm_sym.hip holds the host-side tile
// schedule and the dispatch.
#pragma once
#include "common.hpp"
#include "gemm_sym.hpp"

namespace psd {

template <typename T> struct Elt;
template <> struct Elt<float> { static constexpr float kSplit = 1.0f; };
template <> struct Elt<f16> { static constexpr float kSplit = 2048.0f; };
template <> struct Elt<bf16> { static constexpr float kSplit = 1.0f; };

// One 16-byte fragment of A times one of B on a 32x32 MFMA block.
// Lane l supplies row/column (l % 32) and K-chunk (l / 32) of a chunk pair;
// both operands use the same K mapping, so any order of K inside the pair
// contracts correctly.
__device__ __forceinline__ void mma(f32x16 &acc, u32x4 a, u32x4 b, float) {
    // Bit-cast the whole fragment: per-element bit casts of vector lanes
    // were folded to lane 0 by the compiler.
    const f32x4 af = __builtin_bit_cast(f32x4, a);
    const f32x4 bf = __builtin_bit_cast(f32x4, b);
#pragma unroll
    for (int e = 0; e < 4; ++e) acc = __builtin_amdgcn_mfma_f32_32x32x2f32(af[e], bf[e], acc, 0, 0, 0);
}
__device__ __forceinline__ void mma(f32x16 &acc, u32x4 a, u32x4 b, f16) {
    acc = __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(f16x8, a), __builtin_bit_cast(f16x8, b), acc, 0, 0, 0);
}
__device__ __forceinline__ void mma(f32x16 &acc, u32x4 a, u32x4 b, bf16) {
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), acc, 0, 0, 0);
}

// FP8 cross terms of a pair product on the scaled e4m3 MFMA (64 K slots per
// lane pair). a = [hi codes | lo codes] of L, b = [lo codes | hi codes] of R
// over the same 16 K values per lane half, so slot p pairs L_hi with R_lo in
// the first half and L_lo with R_hi in the second. The E8M0 block scales
// (uniform: every byte of sa / sb) undo the pair exponents and the 2^11.
typedef int i32x8 __attribute__((ext_vector_type(8)));
__device__ __forceinline__ void mma_x8(f32x16 &acc, u32x4 a0, u32x4 a1, u32x4 b0, u32x4 b1, int sa, int sb) {
    const i32x8 a = {(int)a0.x, (int)a0.y, (int)a0.z, (int)a0.w, (int)a1.x, (int)a1.y, (int)a1.z, (int)a1.w};
    const i32x8 b = {(int)b0.x, (int)b0.y, (int)b0.z, (int)b0.w, (int)b1.x, (int)b1.y, (int)b1.z, (int)b1.w};
    acc = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a, b, acc, 0, 0, 0, sa, 0, sb);
}

// e4m3 codes of the 16 FP16 values of two substep fragments (8 each, in K
// order), divided by sc (v_cvt_scalef32_pk_fp8_f16 divides by its scale; sc
// = 2^-e gives the codes of v 2^e), packed in the byte order of the pair's lo
// codes.
template <typename T>
__device__ __forceinline__ u32x4 hi8_codes(u32x4 h0, u32x4 h1, float sc) {
    typedef T h2 __attribute__((ext_vector_type(2)));
    typedef short s2 __attribute__((ext_vector_type(2)));
    auto pk = [&](uint32_t lo_pair, uint32_t hi_pair) -> uint32_t {
        s2 w = {0, 0};
        if constexpr (__is_same(T, f16)) {
            w = __builtin_amdgcn_cvt_scalef32_pk_fp8_f16(w, __builtin_bit_cast(h2, lo_pair), sc, false);
            w = __builtin_amdgcn_cvt_scalef32_pk_fp8_f16(w, __builtin_bit_cast(h2, hi_pair), sc, true);
        } else {
            w = __builtin_amdgcn_cvt_scalef32_pk_fp8_bf16(w, __builtin_bit_cast(h2, lo_pair), sc, false);
            w = __builtin_amdgcn_cvt_scalef32_pk_fp8_bf16(w, __builtin_bit_cast(h2, hi_pair), sc, true);
        }
        return __builtin_bit_cast(uint32_t, w);
    };
    return u32x4{pk(h0.x, h0.y), pk(h0.z, h0.w), pk(h1.x, h1.y), pk(h1.z, h1.w)};
}

__device__ __forceinline__ u32x4 scale_frag(u32x4 v, f16) {
    f16x8 h = __builtin_bit_cast(f16x8, v);
    h = h * (f16)2048.0f;
    return __builtin_bit_cast(u32x4, h);
}
__device__ __forceinline__ u32x4 scale_frag(u32x4 v, bf16) { return v; }
__device__ __forceinline__ u32x4 scale_frag(u32x4 v, float) { return v; }

template <typename T> __device__ __forceinline__ float to_f(T v) { return (float)v; }
template <typename T> __device__ __forceinline__ T from_f(float v) { return (T)v; }

// Workgroups are dispatched round-robin over the 8 XCDs (each with its own
// L2). Give every XCD one contiguous run of the column-ordered tile list, so
// the tiles resident on one XCD share operand panels. Bijective for any count.
__device__ __forceinline__ int xcd_remap(int w, int count) {
    const int xcd = w & 7, idx = w >> 3;
    const int per = count >> 3, rem = count & 7;
    return xcd < rem ? xcd * (per + 1) + idx : rem * (per + 1) + (xcd - rem) * per + idx;
}

constexpr int kThreads = 256;  // 4 waves in a 2 x 2 layout

// A pointer every lane of the wave holds, moved to scalar registers (the
// compiler cannot always prove a value loaded through the descriptor table
// uniform).
__device__ __forceinline__ const uint8_t *wave_uniform(const uint8_t *p) {
    const uint64_t v = (uint64_t)(uintptr_t)p;
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return (const uint8_t *)(uintptr_t)(((uint64_t)hi << 32) | lo);
}

typedef __attribute__((address_space(1))) void *gptr_t;
typedef __attribute__((address_space(3))) void *lptr_t;

// 16-byte chunk c of LDS row r is stored at chunk position swz(r, c) (an XOR,
// so the same map places and finds a chunk). The fragment reads of one
// ds_read_b128 take rows r..r+31 at one logical chunk per lane half. The keys
// were chosen by measuring LDS bank-conflict cycles of exactly these read
// patterns on gfx950: with 128-byte rows, keying on r / 2 (row pairs share a
// key, the pair's two rows fill the two 32-bank halves) gives the ideal 4
// cycles per read, where keys that differ within a row pair cost 8; with
// 64-byte rows, keying on r / 4 gives 6.7 cycles against 8.
template <int NCH>
__device__ __forceinline__ int swz(int r, int c) {
    if constexpr (NCH == 8) return c ^ ((r >> 1) & 7);
    else if constexpr (NCH == 4) return c ^ ((r >> 2) & 3);
    else return c ^ ((r >> 3) & 1);
}

// vmcnt-only wait (expcnt and lgkmcnt left unconstrained), gfx9 encoding.
template <int N>
__device__ __forceinline__ void wait_vmcnt() {
    static_assert(N >= 0 && N < 64, "vmcnt range");
    __builtin_amdgcn_s_waitcnt((N & 15) | (7 << 4) | (15 << 8) | ((N >> 4) << 14));
}
// lgkmcnt-only wait: at most N LDS reads still outstanding (they return in
// order, so the older ones have landed).
template <int N>
__device__ __forceinline__ void wait_lgkmcnt() {
    static_assert(N >= 0 && N < 16, "lgkmcnt range");
    __builtin_amdgcn_s_waitcnt(15 | (7 << 4) | (N << 8) | (3 << 14));
}

// X8: split parts are FP8 pairs (FP16 hi + stored e4m3 lo codes; the hi
// codes are formed in registers) instead of FP16 hi + FP16 lo; the pair
// product is L_hi R_hi on FP16 MFMAs plus both cross terms on one FP8 MFMA per
// 32 K. Requires T = f16, and L split whenever R is. With L split and R plain
// (one-sided) the only cross term is L_lo R_hi: 32 K of it fill half an FP8
// MFMA, so the codes of two consecutive K-units go into one MFMA (the first
// unit's held in registers; an odd last unit is padded with zero codes).
//
// COMB (both operands split, 128 tile): each operand's LDS row interleaves
// its two parts, [hi of BK K | lo (or FP8 pair) of the same BK K], so two
// panels of 128-byte rows hold a split K-tile: conflict-free reads at two
// workgroups per CU, where four panels of 64-byte rows cost 6.7 LDS cycles
// per read.
//
// KS: 0 = whole tile; 1 = one K-chunk of a split tile (entry {matrix, tile,
// chunk | chunks << 8, partial}; the raw FP32 accumulators go to the partial
// buffer, no epilogue); 2 = fixup of a split tile (entry {matrix, tile,
// chunks << 8, first partial}; sums the chunks' partials in chunk order, then
// the epilogue). A fixup workgroup covers one 32 x 32 MFMA block (mi, ni) of
// every wave, so a tile's fixup is spread over MI^2 workgroups. The split
// tiles are the few that would otherwise leave most CUs idle in a last,
// partial round of 256 tiles.
template <typename T, bool LS, bool RS, int EPI, int BM, int ROWB, int NST, bool X8, int KS>
__global__ __launch_bounds__(kThreads) void gemm_sym_kernel(GemmArgs g) {
    static_assert(!X8 || (sizeof(T) == 2 && (LS || !RS)), "FP8 pairs: FP16 or BF16 hi, L split whenever R is");
    constexpr bool PAIR8 = X8 && LS;          // FP8 cross terms in the main loop
    constexpr bool ONE8 = PAIR8 && !RS;       // one-sided: L_lo R_hi only
    constexpr bool COMB = LS && RS && !X8 && BM == 128;
    constexpr int NCH = ROWB / 16;            // 16-byte chunks per LDS row
    constexpr int NLP = LS ? 2 : 1;
    constexpr int NRP = RS ? 2 : 1;
    constexpr int NPAN = COMB ? 2 : NLP + NRP;  // LDS panels per stage
    constexpr int PANEL = BM * ROWB;
    // PAIR8 stage: [L hi: 64-byte rows | L codes: 32-byte rows | R hi | R codes]
    // for 32 K (ONE8: no R codes); the hi codes of the cross terms are formed
    // in registers
    constexpr int P8HI = BM * 64, P8LO = BM * 32;
    constexpr int STAGE = PAIR8 ? 2 * P8HI + (RS ? 2 : 1) * P8LO : NPAN * PANEL;
    constexpr int TB = PAIR8 ? 64 : (COMB ? ROWB / 2 : ROWB);  // bytes per K-tile (hi buffer)
    constexpr int BK = TB / (int)sizeof(T);     // K per tile
    constexpr int HCH = COMB ? NCH / 2 : 0;     // COMB: first chunk of the lo part
    // K-units per tile: a chunk pair (32 bytes of a row: 16 K in FP16/BF16,
    // 8 K in FP32), or 64 bytes (32 K) with FP8 pairs
    constexpr int NSUB = PAIR8 ? TB / 64 : TB / 32;
    static_assert(NSUB >= 1, "at least one K-unit per tile");
    static_assert(!COMB || NCH == 8, "combined rows are 128 bytes");
    constexpr int WM = BM / 2;                // wave tile edge
    constexpr int MI = WM / 32;
    static_assert(BM * NCH % kThreads == 0 && WM % 32 == 0, "tile shape");
    static_assert(NST >= 2, "at least two LDS stages");
    __shared__ __attribute__((aligned(16))) uint8_t smem[NST * STAGE];

    constexpr int MB = (BM / 64) * (BM / 64);  // MFMA blocks per wave (MI^2)
    static_assert(MB == MI * MI, "fixup blocks");
    WorkItem tv;
    int kchunk = 0, kchunks = 1, fblk = 0;
    uint32_t part = 0;
    if constexpr (KS == 0) {
        tv = g.tiles[xcd_remap(blockIdx.x, gridDim.x)];
    } else {
        if constexpr (KS == 2) fblk = (int)(blockIdx.x % MB);
        const uint4 e = g.split[KS == 1 ? xcd_remap(blockIdx.x, gridDim.x) : (int)(blockIdx.x / MB)];
        tv = WorkItem{e.x, e.y};
        kchunk = (int)(e.z & 255u);
        kchunks = (int)(e.z >> 8);
        part = e.w;
    }
    const MatDesc &dm = g.D[tv.x];
    if (g.adaptive == 1 && dm.scal->done) return;  // converged: later stages are skipped (uniform per workgroup)
    const int sr = g.adaptive == 2 ? dm.scal->cur_slot : g.sr;
    const int bi = (int)(tv.y & 0xFFFFu), bj = (int)(tv.y >> 16);
    const int64_t i0 = (int64_t)bi * BM;
    const int64_t j0 = (int64_t)bj * BM;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int wr = (wave >> 1) * WM;
    const int wc = (wave & 1) * WM;
    const int64_t ld = dm.ldw;

    // Source buffers in LDS order: L_hi, [L_lo], R_hi, [R_lo] (COMB: the
    // two parts of each panel).
    const uint8_t *src[4];
    {
        int p = 0;
        src[p++] = (const uint8_t *)dm.hi[g.sl];
        if constexpr (LS) src[p++] = (const uint8_t *)dm.lo[g.sl];
        src[p++] = (const uint8_t *)dm.hi[sr];
        if constexpr (RS) src[p++] = (const uint8_t *)dm.lo[sr];
    }
    // Direct global->LDS loads: one wave instruction moves 64 x 16 bytes into
    // 1 KB of contiguous LDS (lane l -> byte 16 l). The K-tile of all panels
    // is NLD such kilobytes per wave; lane l of load j fills LDS row r at
    // physical chunk pc, so it fetches logical chunk swz(r, pc) of that row.
    constexpr int NLD = STAGE / (1024 * 4);
    constexpr int RPL = 1024 / ROWB;  // LDS rows per wave load
    static_assert(STAGE % 4096 == 0, "stage split over waves");
    const int wave_u = __builtin_amdgcn_readfirstlane(wave);
    // Each load's address is a base shared by the wave (scalar registers,
    // advanced per K-tile by scalar arithmetic) plus a fixed 32-bit per-lane
    // offset, so the K loop spends no vector instructions on addresses. COMB
    // rows take each lane's part from one of two buffers: 64-bit per-lane
    // addresses there.
    const uint8_t *gbase[NLD];
    uint32_t goff[NLD];
    const uint8_t *gsrc[COMB ? NLD : 1];
    int gstep[NLD];  // bytes a source row advances per K-tile
    int gsh[NLD];    // its log2 (steps are powers of two)
#pragma unroll
    for (int j = 0; j < NLD; ++j) {
        const int kb = (wave_u * NLD + j) * 1024;  // byte offset in the stage (uniform)
        gstep[j] = TB;
        gsh[j] = __builtin_ctz(TB);
        if constexpr (PAIR8) {
            // panels: L hi, L codes, R hi[, R codes] (every 1-KB load lies in one)
            const int side = kb >= P8HI + P8LO ? 1 : 0;
            const int off = kb - side * (P8HI + P8LO);
            const bool is_hi = off < P8HI;
            const int w = is_hi ? 64 : 32, nch = w / 16;
            const int rb = (is_hi ? off : off - P8HI) / w;  // first row of the load (uniform)
            const int rl = lane / nch;                      // the lane's row in it
            const int pc = lane % nch;
            const int c = is_hi ? swz<4>(rb + rl, pc) : swz<2>(rb + rl, pc);
            const int64_t row0 = (side == 0 ? i0 : j0) + rb;  // a multiple of 4
            // hi: row-major 64-byte segments of the FP16 column; codes: the
            // tiled code buffer, 32 bytes of column `row` per 32-K block
            if (is_hi) {
                gbase[j] = wave_uniform(src[2 * side] + row0 * ld * 2);
                goff[j] = (uint32_t)(rl * ld * 2 + (c << 4));
            } else {
                gbase[j] = wave_uniform(src[2 * side + 1] + (row0 >> 2) * 4 * ld);
                goff[j] = (uint32_t)((rl >> 2) * 4 * ld + 32 * (rl & 3) + (c << 4));
            }
            gstep[j] = is_hi ? 64 : 128;
            gsh[j] = is_hi ? 6 : 7;
            continue;
        }
        const int p = kb / PANEL;
        const int rb = (kb % PANEL) / ROWB;
        const int rl = lane / NCH;
        const int r = rb + rl;
        const int pc = lane % NCH;
        const int c = swz<NCH>(r, pc);
        if constexpr (COMB) {
            // panel p is operand p; chunk c < HCH is hi, the rest lo / pair
            const int64_t row = (p == 0 ? i0 : j0) + r;
            gsrc[j] = src[2 * p + (c >= HCH ? 1 : 0)] + row * ld * (int64_t)sizeof(T) + ((c % HCH) << 4);
            gbase[j] = nullptr;
            goff[j] = 0;
        } else {
            const int64_t row0 = (p < NLP ? i0 : j0) + rb;
            gbase[j] = wave_uniform(src[p] + row0 * ld * (int64_t)sizeof(T));
            goff[j] = (uint32_t)(rl * ld * (int64_t)sizeof(T) + (c << 4));
        }
    }
    // The loads are written as inline asm (M0 = LDS destination, one s_nop
    // for the M0 -> LDS-DMA hazard, as the compiler itself emits). Issued
    // through the builtin, the compiler's wait-count pass cannot order the LDS
    // reads behind LDS DMA and puts lgkmcnt(0) before every MFMA group, which
    // also waits for the next substep's reads; as asm, the reads get counted
    // waits. Completion of the DMA is awaited explicitly (vmcnt + barrier
    // below), as before.
    auto issue_one = [&](int64_t kt, int buf, int j) {
        const uint32_t la = (uint32_t)(uintptr_t)(smem + buf * STAGE + (wave_u * NLD + j) * 1024);
        if constexpr (COMB) {
            asm volatile("s_mov_b32 m0, %1\n\ts_nop 0\n\tglobal_load_lds_dwordx4 %0, off"
                         :
                         : "v"(gsrc[j] + kt * gstep[j]), "s"(la)
                         : "memory", "m0");
        } else {
            asm volatile("s_mov_b32 m0, %2\n\ts_nop 0\n\tglobal_load_lds_dwordx4 %0, %1"
                         :
                         : "v"(goff[j]), "s"(gbase[j] + (kt << gsh[j])), "s"(la)
                         : "memory", "m0");
        }
    };
    auto issue_loads = [&](int64_t kt, int buf) {
#pragma unroll
        for (int j = 0; j < NLD; ++j) issue_one(kt, buf, j);
    };
    static_assert(PAIR8 || RPL * NCH == 64, "lane layout");

    // accumulators: MI x MI blocks of 32 x 32 per wave; the fixup holds only
    // its block (fmi, fni), as a 1 x 1 array
    constexpr int MIE = KS == 2 ? 1 : MI;
    const int fmi = fblk / MI, fni = fblk % MI;
    f32x16 acc[MIE][MIE];
#pragma unroll
    for (int mi = 0; mi < MIE; ++mi)
#pragma unroll
        for (int ni = 0; ni < MIE; ++ni)
#pragma unroll
            for (int e = 0; e < 16; ++e) acc[mi][ni][e] = 0.0f;
    // partial buffers: one 16-float block of (mi, ni) per thread, stored as
    // four float4 rows of kThreads entries (coalesced)
    auto part_ptr = [&](uint32_t p, int mi, int ni, int q) -> f32x4 * {
        return (f32x4 *)g.part + (((size_t)p * MI * MI + mi * MI + ni) * 4 + q) * kThreads + threadIdx.x;
    };
    if constexpr (KS == 2) {
        for (int c = 0; c < kchunks; ++c)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const f32x4 v = *part_ptr(part + c, fmi, fni, q);
#pragma unroll
                for (int e = 0; e < 4; ++e) acc[0][0][4 * q + e] += v[e];
            }
    } else {
        // fragment row offsets inside a panel, and the row's swizzle key
        int roff_a[MI], roff_b[MI], key_a[MI], key_b[MI];
        int ra_[MI], rb_[MI];
#pragma unroll
        for (int m = 0; m < MI; ++m) {
            const int ra = wr + m * 32 + (lane & 31), rb = wc + m * 32 + (lane & 31);
            ra_[m] = ra;
            rb_[m] = rb;
            roff_a[m] = ra * ROWB;
            roff_b[m] = rb * ROWB;
            key_a[m] = swz<NCH>(ra, 0);
            key_b[m] = swz<NCH>(rb, 0);
        }

        // K-tiles of this workgroup: all, or chunk kchunk of kchunks. Rows n..np
        // of every operand are zero padding, so the K loop stops at the first
        // K-tile boundary at or after n (the products it skips are exact zeros:
        // results do not change, bitwise).
        const int64_t nk_all = (dm.n + BK - 1) / BK;
        const int64_t kch = (nk_all + kchunks - 1) / kchunks;
        const int64_t kb = kchunk * kch < nk_all ? kchunk * kch : nk_all;
        const int64_t ke = kb + kch < nk_all ? kb + kch : nk_all;
        // Fragments of one K-unit, [part][MFMA block m]. Plain and FP16 pairs:
        // one part per operand panel. FP8 pairs: L_hi (two 16-K substeps),
        // L codes (hi, lo), R_hi (two substeps), R codes (hi, lo); ONE8 has no
        // R codes.
        constexpr int NFP = PAIR8 ? (RS ? 6 : 5) : NLP + NRP;
        typedef u32x4 Frag[NFP][MI];
        // E8M0 scale codes 2^(c - 127), replicated into every byte
        constexpr int PSH = X8 ? PairShift<T>::v : 0;  // bits of the hi format
        const int sa8 = PAIR8 ? (int)((uint32_t)(127 - PSH - g.es_l) * 0x01010101u) : 0;
        const int sb8 = PAIR8 ? (int)((uint32_t)(127 - g.es_r) * 0x01010101u) : 0;
        const float cva = PAIR8 ? __builtin_ldexpf(1.0f, -g.es_l) : 0.0f;  // hi-code conversion scales
        const float cvb = PAIR8 ? __builtin_ldexpf(1.0f, -g.es_r) : 0.0f;
        auto rd = [&](const uint8_t *base, int pan, bool b_side, int m, int c) -> u32x4 {
            const int ro = b_side ? roff_b[m] : roff_a[m], key = b_side ? key_b[m] : key_a[m];
            return *(const u32x4 *)(base + pan * PANEL + ro + ((c ^ key) << 4));
        };
        auto load_frags = [&](const uint8_t *base, int sub, Frag &f) {
            const int hg = lane >> 5;
            if constexpr (PAIR8) {
                // [0] L hi substep 0, [1] L hi substep 1, [2] L codes, [3..5] R;
                // issued in groups (substep 0, substep 1, codes) so the MFMAs can
                // start on each group as it lands
                const uint8_t *lh = base, *ll = base + P8HI, *rh = base + P8HI + P8LO, *rl = rh + P8HI;
#pragma unroll
                for (int h = 0; h < 2; ++h) {
#pragma unroll
                    for (int m = 0; m < MI; ++m)
                        f[h][m] = *(const u32x4 *)(lh + ra_[m] * 64 + (((2 * h + hg) ^ ((ra_[m] >> 2) & 3)) << 4));
#pragma unroll
                    for (int m = 0; m < MI; ++m)
                        f[3 + h][m] = *(const u32x4 *)(rh + rb_[m] * 64 + (((2 * h + hg) ^ ((rb_[m] >> 2) & 3)) << 4));
                    __builtin_amdgcn_sched_barrier(0);
                }
#pragma unroll
                for (int m = 0; m < MI; ++m) {
                    f[2][m] = *(const u32x4 *)(ll + ra_[m] * 32 + ((hg ^ ((ra_[m] >> 3) & 1)) << 4));
                    if constexpr (RS) f[NFP - 1][m] = *(const u32x4 *)(rl + rb_[m] * 32 + ((hg ^ ((rb_[m] >> 3) & 1)) << 4));
                }
                return;
            } else if constexpr (COMB) {
#pragma unroll
                for (int m = 0; m < MI; ++m) {
                    f[0][m] = rd(base, 0, false, m, 2 * sub + hg);
                    f[1][m] = rd(base, 0, false, m, HCH + 2 * sub + hg);
                    f[2][m] = rd(base, 1, true, m, 2 * sub + hg);
                    f[3][m] = rd(base, 1, true, m, HCH + 2 * sub + hg);
                }
                return;
            }
            const int cl = 2 * sub + hg;
#pragma unroll
            for (int p = 0; p < NLP; ++p)
#pragma unroll
                for (int m = 0; m < MI; ++m)
                    f[p][m] = *(const u32x4 *)(base + p * PANEL + roff_a[m] + ((cl ^ key_a[m]) << 4));
#pragma unroll
            for (int p = 0; p < NRP; ++p)
#pragma unroll
                for (int m = 0; m < MI; ++m)
                    f[NLP + p][m] = *(const u32x4 *)(base + (NLP + p) * PANEL + roff_b[m] + ((cl ^ key_b[m]) << 4));
        };
        // Loads of the next K-tile still to issue in this iteration: they go
        // out one after each MFMA block of the first substeps (il), since as
        // one burst after the barrier they left the MFMA pipe idle while they
        // issued (10% of the plain product's time at n = 10^4).
        int64_t ktl = 0;
        int bufl = 0, jl = 0;
        auto il = [&](int jend) {
            if (jl < jend) {
                issue_one(ktl, bufl, jl);
                ++jl;
                __builtin_amdgcn_sched_barrier(0);
            }
        };
        constexpr int ILS = NSUB >= 2 ? 2 : 1;           // substeps that carry loads
        constexpr int LPS = (NLD + ILS - 1) / ILS;       // loads per such substep
        auto jend_of = [](int sub) { return sub < ILS ? ((sub + 1) * LPS < NLD ? (sub + 1) * LPS : NLD) : NLD; };
        auto mfmas = [&](const Frag &f, int jend) {
#pragma unroll
            for (int mi = 0; mi < MI; ++mi)
#pragma unroll
                for (int ni = 0; ni < MI; ++ni) {
                    if constexpr (PAIR8) {
                        static_assert(!PAIR8 || NSUB == 1, "FP8 pairs run their own K-unit below");
                    } else if constexpr (LS || RS) {
                        mma(acc[mi][ni], f[0][mi], scale_frag(f[NLP][ni], T{}), T{});
                        if constexpr (RS) mma(acc[mi][ni], f[0][mi], f[NLP + 1][ni], T{});
                        if constexpr (LS) mma(acc[mi][ni], f[1][mi], f[NLP][ni], T{});
                    } else {
                        mma(acc[mi][ni], f[0][mi], f[NLP][ni], T{});
                    }
                    il(jend);
                }
        };
        // ds_read_b128 per K-unit; the counter holds 15 at most, and a wait for
        // <= 15 outstanding is still enough when more were issued after the ones
        // needed (in-order return)
        constexpr int NDS = NFP * MI < 15 ? NFP * MI : 15;
        Frag fr[2];
        // ONE8: the first K-unit of a pair's L lo codes and R hi codes
        u32x4 held_l[ONE8 ? MI : 1], held_r[ONE8 ? MI : 1];
        // LDS ring of NST stages, K-tiles prefetched NST - 1 iterations ahead.
        // Every wave issues exactly NLD loads per iteration (the index is clamped
        // at the end), so "tile kt+1 has landed" is vmcnt <= NLD * (NST - 2).
        if (ke > kb) {
#pragma unroll
            for (int t = 0; t < NST - 1; ++t) issue_loads(kb + t < ke ? kb + t : ke - 1, t);
            wait_vmcnt<NLD * (NST - 2)>();
            __builtin_amdgcn_s_barrier();
            load_frags(smem, 0, fr[0]);
            // Drain every LDS and scalar-memory access of the prologue, so that no
            // scalar load (which may return out of order) is pending in the loop and
            // the counted LDS waits below are the only ones needed.
            wait_lgkmcnt<0>();
            for (int64_t kt = kb; kt < ke; ++kt) {
                const int64_t kr = kt - kb;  // ring position
                const int st = (int)(kr % NST);
                const uint8_t *base = smem + st * STAGE;
                // stage (kr - 1) mod NST was last read in iteration kt - 1, which every
                // wave finished before the barrier that ended it
                const int64_t tn = kt + NST - 1;
                ktl = tn < ke ? tn : ke - 1;
                bufl = (int)((kr + NST - 1) % NST);
                jl = 0;
#pragma unroll
                for (int sub = 0; sub < NSUB; ++sub) {
                    // next substep's fragments first, then this substep's MFMAs on
                    // fragments loaded one substep earlier: wait only for those (the
                    // NDS reads just issued may stay in flight under the MFMAs)
                    if (sub + 1 < NSUB) {
                        load_frags(base, sub + 1, fr[(sub + 1) & 1]);
                        __builtin_amdgcn_sched_barrier(0);
                        wait_lgkmcnt<NDS>();
                        mfmas(fr[sub & 1], jend_of(sub));
                    } else if constexpr (PAIR8) {
                        // the unit's reads were issued in groups (substep 0, substep
                        // 1, codes): start on each group as it lands; every
                        // accumulator still sees substep 0, 1, then the cross terms
                        const Frag &f = fr[sub & 1];
                        // reads outstanding after substep 0 / substep 1 landed
                        constexpr int W0 = (RS ? 4 : 3) * MI, W1 = (RS ? 2 : 1) * MI;
                        __builtin_amdgcn_sched_barrier(0);
                        wait_lgkmcnt<(W0 < 15 ? W0 : 15)>();
#pragma unroll
                        for (int mi = 0; mi < MI; ++mi)
#pragma unroll
                            for (int ni = 0; ni < MI; ++ni) {
                                mma(acc[mi][ni], f[0][mi], f[3][ni], T{});
                                il(MI * MI < NLD ? MI * MI : NLD);
                            }
                        __builtin_amdgcn_sched_barrier(0);
                        wait_lgkmcnt<W1>();
#pragma unroll
                        for (int mi = 0; mi < MI; ++mi)
#pragma unroll
                            for (int ni = 0; ni < MI; ++ni) {
                                mma(acc[mi][ni], f[1][mi], f[4][ni], T{});
                                il(NLD);
                            }
                        u32x4 ha[MI], hb[MI];
#pragma unroll
                        for (int m = 0; m < MI; ++m) {
                            if constexpr (RS) ha[m] = hi8_codes<T>(f[0][m], f[1][m], cva);
                            hb[m] = hi8_codes<T>(f[3][m], f[4][m], cvb);
                        }
                        __builtin_amdgcn_sched_barrier(0);
                        wait_lgkmcnt<0>();
                        if constexpr (RS) {
#pragma unroll
                            for (int mi = 0; mi < MI; ++mi)
#pragma unroll
                                for (int ni = 0; ni < MI; ++ni)
                                    mma_x8(acc[mi][ni], ha[mi], f[2][mi], f[NFP - 1][ni], hb[ni], sa8, sb8);
                        } else if (kr & 1) {
                            // second unit of a pair: [held | this unit] of L lo codes
                            // against [held | this unit] of R hi codes
#pragma unroll
                            for (int mi = 0; mi < MI; ++mi)
#pragma unroll
                                for (int ni = 0; ni < MI; ++ni)
                                    mma_x8(acc[mi][ni], held_l[mi], f[2][mi], held_r[ni], hb[ni], sa8, sb8);
                        } else {
#pragma unroll
                            for (int m = 0; m < MI; ++m) {
                                held_l[m] = f[2][m];
                                held_r[m] = hb[m];
                            }
                        }
                    } else {
                        __builtin_amdgcn_sched_barrier(0);
                        wait_lgkmcnt<0>();
                        mfmas(fr[sub & 1], jend_of(sub));
                    }
                    __builtin_amdgcn_sched_barrier(0);
                }
                // any loads the MFMA blocks had no room for
#pragma unroll
                for (int j = 0; j < NLD; ++j)
                    if (j >= jl) issue_one(ktl, bufl, j);
                // Tile kt + 1 landed for this wave, then (barrier) for all waves. A
                // plain s_barrier: a fenced __syncthreads would wait for every
                // outstanding load (vmcnt(0)) and undo the prefetch. Every ds_read of
                // the stage about to be refilled was consumed by an MFMA above.
                wait_vmcnt<NLD * (NST - 2)>();
                __builtin_amdgcn_s_barrier();
                load_frags(smem + (int)((kr + 1) % NST) * STAGE, 0, fr[0]);
            }
            if constexpr (ONE8) {
                // an odd last unit: its codes against zero codes
                if ((ke - kb) & 1) {
                    const u32x4 z = {0u, 0u, 0u, 0u};
#pragma unroll
                    for (int mi = 0; mi < MI; ++mi)
#pragma unroll
                        for (int ni = 0; ni < MI; ++ni) mma_x8(acc[mi][ni], held_l[mi], z, held_r[ni], z, sa8, sb8);
                }
            }
            __builtin_amdgcn_s_waitcnt(0);
        }
    }  // KS != 2
    if constexpr (KS == 1) {
#pragma unroll
        for (int mi = 0; mi < MI; ++mi)
#pragma unroll
            for (int ni = 0; ni < MI; ++ni)
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    *part_ptr(part, mi, ni, q) =
                        f32x4{acc[mi][ni][4 * q], acc[mi][ni][4 * q + 1], acc[mi][ni][4 * q + 2], acc[mi][ni][4 * q + 3]};
        return;
    }

    // ---------------- epilogue ----------------
    // Accumulator layout of a 32x32 MFMA block: lane l, register e holds
    // row 8 (e / 4) + 4 (l / 32) + (e % 4), column l % 32.
    const float acc_scale = ((LS || RS) && !X8) ? 1.0f / Elt<T>::kSplit : 1.0f;
    const int mo = KS == 2 ? fmi : 0, no = KS == 2 ? fni : 0;  // block offsets of the fixup
    const bool diag = (bi == bj);
    if constexpr (EPI == EPI_FINAL) {
        const IoArg io = io_of(g.io_tab, g.io0, tv.x);
        const float hl = 0.5f * (float)dm.scal->lam * acc_scale;
        const int64_t n = dm.n;
        if (dm.scal->nonfinite) {
            // Inf/NaN input: every entry of out becomes NaN, so a caller without
            // an info buffer cannot mistake stale contents for a result
            const float qnan = __builtin_nanf("");
#pragma clang loop unroll(full)
            for (int mi = 0; mi < MIE; ++mi)
#pragma clang loop unroll(full)
                for (int ni = 0; ni < MIE; ++ni)
#pragma clang loop unroll(full)
                    for (int e = 0; e < 16; ++e) {
                        const int64_t i = i0 + wr + (mi + mo) * 32 + 8 * (e / 4) + 4 * (lane >> 5) + (e % 4);
                        const int64_t j = j0 + wc + (ni + no) * 32 + (lane & 31);
                        if (i >= n || j >= n || (diag && i > j)) continue;
                        io.out[j * io.ld + i] = qnan;
                        io.out[i * io.ld + j] = qnan;
                    }
            return;
        }
        // four consecutive rows of one column as one 16-byte access where aligned
        const bool vec = ((reinterpret_cast<uintptr_t>(io.X) | reinterpret_cast<uintptr_t>(io.out)) & 15) == 0 &&
                         (io.ld & 3) == 0;
#pragma clang loop unroll(full)
        for (int mi = 0; mi < MIE; ++mi)
#pragma clang loop unroll(full)
            for (int ni = 0; ni < MIE; ++ni)
#pragma clang loop unroll(full)
                for (int eg = 0; eg < 4; ++eg) {
                    const int64_t ib = i0 + wr + (mi + mo) * 32 + 8 * eg + 4 * (lane >> 5);
                    const int64_t j = j0 + wc + (ni + no) * 32 + (lane & 31);
                    if (j >= n || ib >= n) continue;
                    if (vec && !diag && ib + 3 < n) {
                        // strictly upper rows ib..ib+3 of column j: read, then written by
                        // this thread only (out == X is safe)
                        const f32x4 x = *(const f32x4 *)(io.X + j * io.ld + ib);
                        f32x4 v;
#pragma clang loop unroll(full)
                        for (int q = 0; q < 4; ++q) v[q] = 0.5f * x[q] + hl * acc[mi][ni][4 * eg + q];
                        *(f32x4 *)(io.out + j * io.ld + ib) = v;
#pragma clang loop unroll(full)
                        for (int q = 0; q < 4; ++q) io.out[(ib + q) * io.ld + j] = v[q];
                        continue;
                    }
#pragma clang loop unroll(full)
                    for (int q = 0; q < 4; ++q) {
                        const int64_t i = ib + q;
                        if (i >= n || (diag && i > j)) continue;
                        // upper-triangle entry (i <= j): read then written by
                        // this thread only, so out == X is safe
                        const float v = 0.5f * io.X[j * io.ld + i] + hl * acc[mi][ni][4 * eg + q];
                        io.out[j * io.ld + i] = v;
                        io.out[i * io.ld + j] = v;
                    }
                }
    } else {
        T *Dhi = (T *)dm.hi[g.sd];
        T *Dlo = (T *)dm.lo[g.sd];
        const T *C0hi = g.sc0 >= 0 ? (const T *)dm.hi[g.sc0] : nullptr;
        const T *C0lo = (g.sc0 >= 0 && g.c0_split) ? (const T *)dm.lo[g.sc0] : nullptr;
        const float c0lo = 1.0f / Elt<T>::kSplit;
        // FP8 pairs: code scales of the addend and of the output slot
        constexpr int PSE = X8 ? PairShift<T>::v : 0;
        const float c0x = X8 ? __builtin_ldexpf(1.0f, -(PSE + g.es_c0)) : 0.0f;
        const float dls = X8 ? __builtin_ldexpf(1.0f, PSE + g.es_d) : 0.0f;
        uint8_t *Dx = (uint8_t *)dm.lo[g.sd];
        typedef T t4 __attribute__((ext_vector_type(4)));
#pragma clang loop unroll(full)
        for (int mi = 0; mi < MIE; ++mi)
#pragma clang loop unroll(full)
            for (int ni = 0; ni < MIE; ++ni)
#pragma clang loop unroll(full)
                for (int eg = 0; eg < 4; ++eg) {
                    const int64_t ib = i0 + wr + (mi + mo) * 32 + 8 * eg + 4 * (lane >> 5);
                    const int64_t j = j0 + wc + (ni + no) * 32 + (lane & 31);
                    float v[4];
#pragma clang loop unroll(full)
                    for (int q = 0; q < 4; ++q) v[q] = g.beta * (acc[mi][ni][4 * eg + q] * acc_scale);
                    if (C0hi) {
                        const t4 c = *(const t4 *)(C0hi + j * ld + ib);
#pragma clang loop unroll(full)
                        for (int q = 0; q < 4; ++q) v[q] += g.alpha * to_f(c[q]);
                        if (C0lo) {
                            if constexpr (X8) {
                                const uint32_t w = *(const uint32_t *)((const uint8_t *)C0lo + lo8_index(ib, j, ld));
#pragma clang loop unroll(full)
                                for (int q = 0; q < 4; ++q) v[q] += g.alpha * (e4m3_byte(w, q) * c0x);
                            } else {
                                const t4 cl = *(const t4 *)(C0lo + j * ld + ib);
#pragma clang loop unroll(full)
                                for (int q = 0; q < 4; ++q) v[q] += g.alpha * (to_f(cl[q]) * c0lo);
                            }
                        }
                    }
                    constexpr bool SPL16 = EPI == EPI_STORE_SPLIT && !X8;
                    constexpr bool SPL8 = EPI == EPI_STORE_SPLIT && X8;
                    t4 hi, lo;
#pragma clang loop unroll(full)
                    for (int q = 0; q < 4; ++q) {
                        if (ib + q == j) v[q] += g.gamma;
                        hi[q] = from_f<T>(v[q]);
                        if constexpr (SPL16) lo[q] = from_f<T>((v[q] - to_f(hi[q])) * Elt<T>::kSplit);
                    }
                    uint32_t l8 = 0;
                    if constexpr (SPL8)
                        l8 = e4m3x4((v[0] - to_f(hi[0])) * dls, (v[1] - to_f(hi[1])) * dls,
                                    (v[2] - to_f(hi[2])) * dls, (v[3] - to_f(hi[3])) * dls);
                    if (!diag) {
                        *(t4 *)(Dhi + j * ld + ib) = hi;
                        if constexpr (SPL16) *(t4 *)(Dlo + j * ld + ib) = lo;
                        if constexpr (SPL8) *(uint32_t *)(Dx + lo8_index(ib, j, ld)) = l8;
#pragma clang loop unroll(full)
                        for (int q = 0; q < 4; ++q) {
                            Dhi[(ib + q) * ld + j] = hi[q];
                            if constexpr (SPL16) Dlo[(ib + q) * ld + j] = lo[q];
                            if constexpr (SPL8) Dx[lo8_index(j, ib + q, ld)] = (uint8_t)(l8 >> (8 * q));
                        }
                    } else {
#pragma clang loop unroll(full)
                        for (int q = 0; q < 4; ++q) {
                            const int64_t i = ib + q;
                            if (i > j) continue;
                            Dhi[j * ld + i] = hi[q];
                            Dhi[i * ld + j] = hi[q];
                            if constexpr (SPL16) {
                                Dlo[j * ld + i] = lo[q];
                                Dlo[i * ld + j] = lo[q];
                            }
                            if constexpr (SPL8) {
                                const uint8_t lb = (uint8_t)(l8 >> (8 * q));
                                Dx[lo8_index(i, j, ld)] = lb;
                                Dx[lo8_index(j, i, ld)] = lb;
                            }
                        }
                    }
                }
    }
}

// ---------------------------------------------------------------------------
// LDS configuration per (tile, operand panels). The 128 tile keeps two
// stages within 80 KB, so two workgroups share a CU (160 KB of LDS) whether or
// not the operands are split: plain panels get 128-byte rows, split panels
// 64-byte rows (measured 1.7% faster per split projection than one 128-KB
// workgroup per CU). Deeper rings measured slower at n = 10^4 for the plain
// product (1.20 ms per product with this ring; 1.36-1.52 ms with 3-5 stages of
// 64- or 128-byte rows at one or two workgroups per CU), and 64-byte rows at
// four workgroups per CU slowed the batch of small matrices by 8%. The 256
// tile uses 128 KB: two stages of 128-byte rows for plain operands (faster
// than 3- or 4-stage rings of 64-byte rows by 4-8% at n_p = 10240), two of
// 64-byte rows for split ones; FP8 pairs use 96 KB (a 3-stage ring of them
// with an earlier barrier measured 4% slower).
template <int BM, int NP> struct LdsCfg {
    static constexpr bool COMB = BM == 128 && NP == 4;  // two parts per 128-byte row
    static constexpr int NST = 2;
    static constexpr int BUDGET = BM == 256 ? 128 * 1024 : 80 * 1024;
    static constexpr int ROWB_MAX = BUDGET / (NST * (COMB ? 2 : NP) * BM);
    static constexpr int ROWB = ROWB_MAX >= 128 ? 128 : ROWB_MAX >= 64 ? 64 : 32;
};

template <typename T, bool LS, bool RS, int EPI, int BM, bool X8 = false>
static hipError_t launch_bm(const GemmArgs &g, int64_t ntiles, hipStream_t s, int ks) {
    constexpr int NP = 2 + (LS ? 1 : 0) + (RS ? 1 : 0);
    constexpr int ROWB = LdsCfg<BM, NP>::ROWB;
    constexpr int NST = LdsCfg<BM, NP>::NST;
    if (ntiles == 0) return hipSuccess;
    const dim3 grid((unsigned)ntiles), blk(kThreads);
    if (ks == 0) {
        hipLaunchKernelGGL((gemm_sym_kernel<T, LS, RS, EPI, BM, ROWB, NST, X8, 0>), grid, blk, 0, s, g);
    } else if constexpr (BM == kTile2 && sizeof(T) == 2) {
        if (!g.split || !g.part) return hipErrorInvalidValue;
        // the chunks have no epilogue: one instantiation serves every EPI
        if (ks == 1)
            hipLaunchKernelGGL((gemm_sym_kernel<T, LS, RS, EPI_STORE, BM, ROWB, NST, X8, 1>), grid, blk, 0, s, g);
        else if (ks == 2)  // (BM / 64)^2 workgroups per fixup entry
            hipLaunchKernelGGL((gemm_sym_kernel<T, LS, RS, EPI, BM, ROWB, NST, X8, 2>),
                               dim3((unsigned)(ntiles * (BM / 64) * (BM / 64))), blk, 0, s, g);
        else
            return hipErrorInvalidValue;
    } else {
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename T, int EPI>
static hipError_t launch_x8(const GemmArgs &g, bool ls, bool rs, int bm, int64_t ntiles, hipStream_t s, int ks) {
    if (ls && rs) {
        switch (bm) {
            case 256: return launch_bm<T, true, true, EPI, 256, true>(g, ntiles, s, ks);
            case 128: return launch_bm<T, true, true, EPI, 128, true>(g, ntiles, s, ks);
        }
        return hipErrorInvalidValue;
    }
    if (ls) {
        switch (bm) {
            case 256: return launch_bm<T, true, false, EPI, 256, true>(g, ntiles, s, ks);
            case 128: return launch_bm<T, true, false, EPI, 128, true>(g, ntiles, s, ks);
        }
        return hipErrorInvalidValue;
    }
    switch (bm) {
        case 256: return launch_bm<T, false, false, EPI, 256, true>(g, ntiles, s, ks);
        case 128: return launch_bm<T, false, false, EPI, 128, true>(g, ntiles, s, ks);
    }
    return hipErrorInvalidValue;
}

template <typename T, bool LS, bool RS, int EPI>
static hipError_t launch_t(const GemmArgs &g, int bm, int64_t ntiles, hipStream_t s, int ks) {
    switch (bm) {
        case 256: return launch_bm<T, LS, RS, EPI, 256>(g, ntiles, s, ks);
        case 128: return launch_bm<T, LS, RS, EPI, 128>(g, ntiles, s, ks);
    }
    return hipErrorInvalidValue;
}

template <typename T, int EPI>
static hipError_t launch_split(const GemmArgs &g, bool ls, bool rs, int bm, int64_t ntiles, hipStream_t s, int ks) {
    if (ls && rs) return launch_t<T, true, true, EPI>(g, bm, ntiles, s, ks);
    if (ls) return launch_t<T, true, false, EPI>(g, bm, ntiles, s, ks);
    if (rs) return launch_t<T, false, true, EPI>(g, bm, ntiles, s, ks);
    return launch_t<T, false, false, EPI>(g, bm, ntiles, s, ks);
}



// One (precision, epilogue) slice of the launch dispatch; each
// gemm_launch_*.hip file instantiates one, so they compile in parallel.
template <int DT, int EPI>
hipError_t gemm_launch_part(const GemmArgs &g, bool ls, bool rs, int bm, int64_t ntiles, hipStream_t s, int ks) {
    if constexpr (DT == DT_F32) {
        if (ls || rs || EPI == EPI_STORE_SPLIT || ks) return hipErrorInvalidValue;
        if constexpr (EPI == EPI_STORE_SPLIT) return hipErrorInvalidValue;
        else return launch_t<float, false, false, EPI>(g, bm, ntiles, s, 0);
    } else if constexpr (DT == DT_F16) {
        return launch_split<f16, EPI>(g, ls, rs, bm, ntiles, s, ks);
    } else if constexpr (DT == DT_BF16) {
        return launch_split<bf16, EPI>(g, ls, rs, bm, ntiles, s, ks);
    } else {
        if (rs && !ls) return hipErrorInvalidValue;  // one-sided pairs: the split operand on the left
        if constexpr (DT == DT_BF16X8) return launch_x8<bf16, EPI>(g, ls, rs, bm, ntiles, s, ks);
        else return launch_x8<f16, EPI>(g, ls, rs, bm, ntiles, s, ks);
    }
}

}  // namespace psd

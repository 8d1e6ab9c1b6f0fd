// Shared device/host definitions for libpsdproj (gfx950 only).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

typedef _Float16 f16;
typedef __bf16 bf16;
typedef f16 f16x8 __attribute__((ext_vector_type(8)));
typedef bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

namespace psd {

// FP8 pairs: the lo code of M is e4m3((M - M_hi) 2^(shift + e)), shift = the
// significant bits of the hi format (the residual is at most half an ulp, 2^-shift
// of |M|): 11 for FP16, 8 for BF16.
template <typename T> struct PairShift { static constexpr int v = 0; };  // no FP8 pairs
template <> struct PairShift<f16> { static constexpr int v = 11; };
template <> struct PairShift<bf16> { static constexpr int v = 8; };

// Device-resident scalar block of one projection (all FP64 so that the bound
// never loses digits). Written by the norm/Lanczos kernels, read by the cast
// and final kernels; never copied to the host inside a projection.
struct Scalars {
    double fro2;        // ||X||_F^2
    double colmax2;     // max_j ||X e_j||^2 (lower bound on ||X||_2^2)
    double lam;         // spectral bound used for the rescale
    double inv_lam;     // 1 / lam (0 when lam == 0)
    double sigma;       // largest Ritz value of X^2
    double resid;       // ||X^2 q - sigma q||
    double lanczos_lam; // sqrt(sigma + resid) before the guard
    double beta_last;   // last Lanczos beta
    double qnorm_inv;   // 1 / ||V s||
    double amax;        // max |alpha_j| seen so far
    int32_t k;          // Lanczos steps taken
    int32_t stop;       // breakdown flag
    int32_t nonfinite;  // input had Inf/NaN
    int32_t fallback;   // guard replaced the Lanczos bound
    // adaptive depth: converged (later adaptive stages are skipped), the work
    // slot holding the latest iterate, stages run, last relative change
    int32_t done;
    int32_t cur_slot;
    int32_t stages_run;
    int32_t pad_;
    double delta;
    double alpha[32];
    double beta[32];
    double s[32];       // Ritz vector in the Krylov basis
};

constexpr int kMaxLanczos = 32;
constexpr int kMaxDeflate = 8;

// Deflation state of one projection (opts.deflate > 0): candidate Rayleigh-
// Ritz pairs of X in the Krylov basis of the bound's Lanczos run, the pairs
// kept, and the buffers the deflation kernels use.
struct DeflState {
    int32_t kmax;                         // pairs requested (<= kMaxDeflate)
    int32_t ncand;                        // candidates: min(kmax, Lanczos steps)
    int32_t count;                        // pairs kept (converged)
    int32_t pad_;
    double cmu[kMaxDeflate];              // candidate eigenvalues of V^T X V, largest |mu| first
    double cs[kMaxDeflate][kMaxLanczos];  // their eigenvectors in the Krylov basis
    double mu[kMaxDeflate];               // kept pairs
    double inv_nz[kMaxDeflate];           // 1 / ||V s|| of each kept pair
    int32_t idx[kMaxDeflate];             // candidate index of each kept pair
    double *Z;                            // n x kMaxDeflate: V s of every candidate
    double *pH;                           // vector blocks x kMaxLanczos^2: partials of V^T (X V)
    double *pz;                           // vector blocks x 2 kMaxDeflate: ||z||^2, ||X z - mu z||^2
    float *Xd;                            // deflated copy of X (upper triangle), leading dimension ldd
    int64_t ldd;
};

// Per-matrix descriptor of one projection's device workspace. A launch covers
// every matrix of a batch: its work list maps each workgroup to a
// (matrix, local block) pair and the kernel reads the matrix's descriptor.
struct MatDesc {
    int64_t n;        // matrix order
    int64_t np;       // padded order of the work matrices (GEMM tile multiple)
    int64_t ldw;      // leading dimension of the work matrices (>= np)
    Scalars *scal;
    // Lanczos work: V (n x steps), vectors (n), partials (nbv x 32, and nbv
    // for pc), symv tile partials (tiles x 128)
    double *V, *u, *w, *w2, *colsq, *pa, *pb, *pc, *sd, *sa, *sd2, *sa2;
    void *hi[4], *lo[4];  // work slots: X0, then rotating A / B / X_t
    int32_t nbv;          // vector blocks: ceil(n / 256)
    int32_t fused;        // 1: the whole projection runs in the one-workgroup small-matrix kernel
    double *U;            // deflation only: X v_j of every Lanczos step (n x steps), else null
    DeflState *defl;      // deflation only, else null
    int32_t cast_first;   // this matrix's run in the cast work list (adaptive-depth sums)
    int32_t cast_count;
};

// Caller-owned input and output of one matrix: X upper triangle and out,
// FP32 column-major with leading dimension ld.
struct IoArg {
    const float *X;
    float *out;
    int64_t ld;
    void *info;  // psdproj_info in device memory, or null
};

// (matrix, local block) pair of a work list.
typedef uint2 WorkItem;

__device__ __forceinline__ IoArg io_of(const IoArg *tab, const IoArg &io0, int m) { return tab ? tab[m] : io0; }

__host__ __device__ inline int64_t round_up(int64_t v, int64_t m) { return (v + m - 1) / m * m; }

// FP8 pair format of a split work matrix M = M_hi + 2^-(11+e) M_lo (FP16
// M_hi in hi[slot]; the e4m3 codes of M_lo = (M - M_hi) 2^(11+e) in lo[slot],
// one byte per element). The code buffer is tiled for the product kernel's
// loads: columns are grouped by 4 (group c spans 4 ld bytes) and rows by 32;
// the 32 rows x 4 columns of block (q, c) fill one 128-byte line, column
// j = 4 c + s at bytes 32 s .. 32 s + 31. Within a column's 32 bytes the rows
// are permuted so that each 16-byte chunk holds the 16 K values one lane half
// of an FP16 MFMA fragment pair covers: row 32 q + 16 a + 8 g + x (a, g in
// {0, 1}, x < 8) sits at byte 16 g + 8 a + x. e is a per-slot power of two
// chosen from a bound on |M| (entries of a symmetric matrix are bounded by
// its spectral norm) so that the codes of M_hi 2^e, formed in registers by
// the product kernel, and of M_lo stay below the e4m3 maximum, 448.
__device__ __forceinline__ int64_t lo8_index(int64_t i, int64_t j, int64_t ld) {
    return (j >> 2) * 4 * ld + 128 * (i >> 5) + 32 * (j & 3) + 16 * ((i >> 3) & 1) + 8 * ((i >> 4) & 1) + (i & 7);
}
// Round to e4m3 (OCP, round to nearest even) after clamping to the finite
// range; four values packed little-endian into one word.
__device__ __forceinline__ float e4m3_clamp(float v) { return fminf(fmaxf(v, -448.0f), 448.0f); }
__device__ __forceinline__ uint32_t e4m3x4(float a, float b, float c, float d) {
    int w = __builtin_amdgcn_cvt_pk_fp8_f32(e4m3_clamp(a), e4m3_clamp(b), 0, false);
    w = __builtin_amdgcn_cvt_pk_fp8_f32(e4m3_clamp(c), e4m3_clamp(d), w, true);
    return (uint32_t)w;
}
__device__ __forceinline__ uint8_t e4m3(float a) {
    return (uint8_t)(__builtin_amdgcn_cvt_pk_fp8_f32(e4m3_clamp(a), 0.0f, 0, false) & 0xFF);
}
// Byte q (compile-time after unrolling) of a packed word, decoded.
__device__ __forceinline__ float e4m3_byte(uint32_t w, int q) {
    switch (q) {
        case 0: return __builtin_amdgcn_cvt_f32_fp8((int)w, 0);
        case 1: return __builtin_amdgcn_cvt_f32_fp8((int)w, 1);
        case 2: return __builtin_amdgcn_cvt_f32_fp8((int)w, 2);
        default: return __builtin_amdgcn_cvt_f32_fp8((int)w, 3);
    }
}

}  // namespace psd

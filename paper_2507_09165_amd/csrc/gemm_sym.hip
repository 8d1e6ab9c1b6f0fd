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

__device__ __forceinline__ u32x4 scale_frag(u32x4 v, f16) {
    f16x8 h = __builtin_bit_cast(f16x8, v);
    h = h * (f16)2048.0f;
    return __builtin_bit_cast(u32x4, h);
}
__device__ __forceinline__ u32x4 scale_frag(u32x4 v, bf16) { return v; }
__device__ __forceinline__ u32x4 scale_frag(u32x4 v, float) { return v; }

template <typename T> __device__ __forceinline__ float to_f(T v) { return (float)v; }
template <typename T> __device__ __forceinline__ T from_f(float v) { return (T)v; }

// Upper-triangle tile index -> (bi, bj), tiles enumerated column by column:
// t = bj (bj + 1) / 2 + bi, 0 <= bi <= bj.
__device__ __forceinline__ void tri_tile(int t, int &bi, int &bj) {
    int j = (int)((sqrtf(8.0f * (float)t + 1.0f) - 1.0f) * 0.5f);
    while ((j + 1) * (j + 2) / 2 <= t) ++j;
    while (j * (j + 1) / 2 > t) --j;
    bj = j;
    bi = t - j * (j + 1) / 2;
}

constexpr int kRowBytes = 128;  // one K-tile per LDS row: 8 chunks of 16 bytes
constexpr int kThreads = 256;   // 4 waves in a 2 x 2 layout

template <typename T, bool LS, bool RS, int EPI, int BM>
__global__ __launch_bounds__(kThreads) void gemm_sym_kernel(GemmArgs g) {
    constexpr int BN = BM;
    constexpr int NLP = LS ? 2 : 1;
    constexpr int NRP = RS ? 2 : 1;
    constexpr int PANEL_L = BM * kRowBytes;
    constexpr int PANEL_R = BN * kRowBytes;
    constexpr int STAGE = NLP * PANEL_L + NRP * PANEL_R;
    constexpr int BK = kRowBytes / (int)sizeof(T);
    constexpr int CPT_L = BM * 8 / kThreads;  // 16-byte chunks per thread per panel
    constexpr int CPT_R = BN * 8 / kThreads;
    constexpr int WM = BM / 2, WN = BN / 2;   // wave tile
    constexpr int MI = WM / 32, NI = WN / 32;
    __shared__ __attribute__((aligned(16))) uint8_t smem[2 * STAGE];

    int bi, bj;
    tri_tile(blockIdx.x, bi, bj);
    const int64_t i0 = (int64_t)bi * BM;
    const int64_t j0 = (int64_t)bj * BN;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int wr = (wave >> 1) * WM;
    const int wc = (wave & 1) * WN;
    const int64_t ld = g.ld;

    const uint8_t *Lsrc[2] = {(const uint8_t *)g.Lhi, (const uint8_t *)g.Llo};
    const uint8_t *Rsrc[2] = {(const uint8_t *)g.Rhi, (const uint8_t *)g.Rlo};

    u32x4 pf[NLP * CPT_L + NRP * CPT_R];

    auto gload = [&](int64_t kt) {
        const int64_t kb = kt * BK * (int64_t)sizeof(T);
#pragma unroll
        for (int p = 0; p < NLP; ++p)
#pragma unroll
            for (int s = 0; s < CPT_L; ++s) {
                const int q = tid + kThreads * s, r = q >> 3, c = q & 7;
                const uint8_t *src = Lsrc[p] + ((i0 + r) * ld) * (int64_t)sizeof(T) + kb + c * 16;
                pf[p * CPT_L + s] = *(const u32x4 *)src;
            }
#pragma unroll
        for (int p = 0; p < NRP; ++p)
#pragma unroll
            for (int s = 0; s < CPT_R; ++s) {
                const int q = tid + kThreads * s, r = q >> 3, c = q & 7;
                const uint8_t *src = Rsrc[p] + ((j0 + r) * ld) * (int64_t)sizeof(T) + kb + c * 16;
                pf[NLP * CPT_L + p * CPT_R + s] = *(const u32x4 *)src;
            }
    };
    auto sstore = [&](int buf) {
        uint8_t *base = smem + buf * STAGE;
#pragma unroll
        for (int p = 0; p < NLP; ++p)
#pragma unroll
            for (int s = 0; s < CPT_L; ++s) {
                const int q = tid + kThreads * s, r = q >> 3, c = q & 7;
                *(u32x4 *)(base + p * PANEL_L + r * kRowBytes + ((c ^ (r & 7)) << 4)) = pf[p * CPT_L + s];
            }
#pragma unroll
        for (int p = 0; p < NRP; ++p)
#pragma unroll
            for (int s = 0; s < CPT_R; ++s) {
                const int q = tid + kThreads * s, r = q >> 3, c = q & 7;
                *(u32x4 *)(base + NLP * PANEL_L + p * PANEL_R + r * kRowBytes + ((c ^ (r & 7)) << 4)) =
                    pf[NLP * CPT_L + p * CPT_R + s];
            }
    };

    f32x16 acc[MI][NI];
#pragma unroll
    for (int mi = 0; mi < MI; ++mi)
#pragma unroll
        for (int ni = 0; ni < NI; ++ni)
#pragma unroll
            for (int e = 0; e < 16; ++e) acc[mi][ni][e] = 0.0f;

    const int64_t nk = g.K / BK;
    gload(0);
    sstore(0);
    __syncthreads();
    for (int64_t kt = 0; kt < nk; ++kt) {
        const int buf = (int)(kt & 1);
        if (kt + 1 < nk) gload(kt + 1);
        const uint8_t *base = smem + buf * STAGE;
#pragma unroll
        for (int sub = 0; sub < 4; ++sub) {
            const int cl = 2 * sub + (lane >> 5);
            u32x4 a[NLP][MI], b[NRP][NI];
#pragma unroll
            for (int p = 0; p < NLP; ++p)
#pragma unroll
                for (int mi = 0; mi < MI; ++mi) {
                    const int r = wr + mi * 32 + (lane & 31);
                    a[p][mi] = *(const u32x4 *)(base + p * PANEL_L + r * kRowBytes + ((cl ^ (r & 7)) << 4));
                }
#pragma unroll
            for (int p = 0; p < NRP; ++p)
#pragma unroll
                for (int ni = 0; ni < NI; ++ni) {
                    const int r = wc + ni * 32 + (lane & 31);
                    b[p][ni] = *(const u32x4 *)(base + NLP * PANEL_L + p * PANEL_R + r * kRowBytes + ((cl ^ (r & 7)) << 4));
                }
#pragma unroll
            for (int mi = 0; mi < MI; ++mi)
#pragma unroll
                for (int ni = 0; ni < NI; ++ni) {
                    if constexpr (LS || RS) {
                        mma(acc[mi][ni], a[0][mi], scale_frag(b[0][ni], T{}), T{});
                        if constexpr (RS) mma(acc[mi][ni], a[0][mi], b[NRP - 1][ni], T{});
                        if constexpr (LS) mma(acc[mi][ni], a[NLP - 1][mi], b[0][ni], T{});
                    } else {
                        mma(acc[mi][ni], a[0][mi], b[0][ni], T{});
                    }
                }
        }
        if (kt + 1 < nk) sstore(buf ^ 1);
        __syncthreads();
    }

    // ---------------- epilogue ----------------
    const float acc_scale = (LS || RS) ? 1.0f / Elt<T>::kSplit : 1.0f;
    const bool diag = (bi == bj);
    if constexpr (EPI == EPI_FINAL) {
        if (g.scal->nonfinite) return;  // leave the output untouched
        const float lam = (float)g.scal->lam;
        const int64_t n = g.n;
#pragma unroll
        for (int mi = 0; mi < MI; ++mi)
#pragma unroll
            for (int ni = 0; ni < NI; ++ni)
#pragma unroll
                for (int e = 0; e < 16; ++e) {
                    const int64_t i = i0 + wr + mi * 32 + 8 * (e >> 2) + 4 * (lane >> 5) + (e & 3);
                    const int64_t j = j0 + wc + ni * 32 + (lane & 31);
                    if (i >= n || j >= n || (diag && i > j)) continue;
                    const float v = 0.5f * g.Xf[i * g.ldxf + j] + 0.5f * lam * (acc[mi][ni][e] * acc_scale);
                    g.out[i * g.ldo + j] = v;
                    g.out[j * g.ldo + i] = v;
                }
    } else {
        T *Dhi = (T *)g.Dhi;
        T *Dlo = (T *)g.Dlo;
        const T *C0hi = (const T *)g.C0hi;
        const T *C0lo = (const T *)g.C0lo;
        const float c0lo = 1.0f / Elt<T>::kSplit;
#pragma unroll
        for (int mi = 0; mi < MI; ++mi)
#pragma unroll
            for (int ni = 0; ni < NI; ++ni)
#pragma unroll
                for (int e = 0; e < 16; ++e) {
                    const int64_t i = i0 + wr + mi * 32 + 8 * (e >> 2) + 4 * (lane >> 5) + (e & 3);
                    const int64_t j = j0 + wc + ni * 32 + (lane & 31);
                    if (diag && i > j) continue;
                    float v = g.beta * (acc[mi][ni][e] * acc_scale);
                    if (C0hi) {
                        float c0 = to_f(C0hi[i * ld + j]);
                        if (C0lo) c0 += to_f(C0lo[i * ld + j]) * c0lo;
                        v += g.alpha * c0;
                    }
                    if (i == j) v += g.gamma;
                    const T hi = from_f<T>(v);
                    Dhi[i * ld + j] = hi;
                    Dhi[j * ld + i] = hi;
                    if constexpr (EPI == EPI_STORE_SPLIT) {
                        const T lo = from_f<T>((v - to_f(hi)) * Elt<T>::kSplit);
                        Dlo[i * ld + j] = lo;
                        Dlo[j * ld + i] = lo;
                    }
                }
    }
}

// ---------------------------------------------------------------------------
template <typename T, bool LS, bool RS, int EPI>
static hipError_t launch_t(const GemmArgs &g, hipStream_t s) {
    constexpr int BM = kTile;
    const int T_ = (int)(g.K / BM);
    const int ntiles = T_ * (T_ + 1) / 2;
    if (ntiles == 0) return hipSuccess;
    hipLaunchKernelGGL((gemm_sym_kernel<T, LS, RS, EPI, BM>), dim3(ntiles), dim3(kThreads), 0, s, g);
    return hipGetLastError();
}

template <typename T, int EPI>
static hipError_t launch_split(const GemmArgs &g, hipStream_t s) {
    const bool ls = g.Llo != nullptr, rs = g.Rlo != nullptr;
    if (ls && rs) return launch_t<T, true, true, EPI>(g, s);
    if (ls) return launch_t<T, true, false, EPI>(g, s);
    if (rs) return launch_t<T, false, true, EPI>(g, s);
    return launch_t<T, false, false, EPI>(g, s);
}

template <typename T>
static hipError_t launch_epi(const GemmArgs &g, int epi, hipStream_t s) {
    switch (epi) {
        case EPI_STORE: return launch_split<T, EPI_STORE>(g, s);
        case EPI_STORE_SPLIT: return launch_split<T, EPI_STORE_SPLIT>(g, s);
        case EPI_FINAL: return launch_split<T, EPI_FINAL>(g, s);
    }
    return hipErrorInvalidValue;
}

hipError_t gemm_sym_launch(const GemmArgs &g, int dtype, int epi, hipStream_t s) {
    if (g.K % kTile) return hipErrorInvalidValue;
    switch (dtype) {
        case DT_F32:
            if (g.Llo || g.Rlo || epi == EPI_STORE_SPLIT) return hipErrorInvalidValue;
            return epi == EPI_STORE ? launch_t<float, false, false, EPI_STORE>(g, s)
                                    : launch_t<float, false, false, EPI_FINAL>(g, s);
        case DT_F16: return launch_epi<f16>(g, epi, s);
        case DT_BF16: return launch_epi<bf16>(g, epi, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace psd

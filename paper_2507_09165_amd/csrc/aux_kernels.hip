// Bandwidth-bound kernels of the projection: triangle mirror / rescale-and-cast,
// and the FP64 Lanczos run that yields the spectral bound.
//
//  * mirror_cast: reads the upper triangle of X (column-major, ld) in 64 x 64
//    tiles, writes the full symmetric matrix scaled by s (1 for the FP32 copy
//    the Lanczos matvecs read, 1/lam for X0 = X / lam of Algorithm 2), rounded
//    to the work precision, optionally as a hi + lo pair, zero-padded to n_p.
//  * Lanczos on X^2 (Section 3.4 and Algorithm 2, first two steps): 20 steps
//    of w = X (X v) in FP64 with full reorthogonalisation (two classical
//    Gram-Schmidt passes), the largest Ritz pair (sigma, q) of the tridiagonal,
//    and the bound lam = sqrt(sigma + ||X (X q) - sigma q||) of Theorem 2.
//    The first matvec also produces the column norms: ||X||_F and the lower
//    bound max_j ||X e_j|| that guards the heuristic bound.
// All reductions are fixed-order (no floating-point atomics), so results are
// bitwise reproducible run to run.
#include <math.h>

#include "aux_kernels.hpp"
#include "common.hpp"

namespace psd {

// ---------------------------------------------------------------------------
// mirror / rescale / cast
// ---------------------------------------------------------------------------
template <typename T> __device__ __forceinline__ T cvt(float v) { return (T)v; }

template <typename T, bool SPLIT>
__global__ __launch_bounds__(256) void mirror_cast_kernel(const float *__restrict__ X, int64_t ldx, int64_t n,
                                                          const Scalars *scal, int use_inv_lam, T *__restrict__ Ohi,
                                                          T *__restrict__ Olo, int64_t ldo, float lo_scale) {
    __shared__ float tile[64][65];
    // upper-triangle tile pairs over the padded size, column by column
    const int t = blockIdx.x;
    int bj = (int)((sqrtf(8.0f * (float)t + 1.0f) - 1.0f) * 0.5f);
    while ((bj + 1) * (bj + 2) / 2 <= t) ++bj;
    while (bj * (bj + 1) / 2 > t) --bj;
    const int bi = t - bj * (bj + 1) / 2;
    const int64_t i0 = (int64_t)bi * 64, j0 = (int64_t)bj * 64;
    const float s = use_inv_lam ? (float)scal->inv_lam : 1.0f;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;  // 64 x 4
    // load: element (i0 + tx, j0 + c) = X[(j0 + c) * ldx + i0 + tx], upper part only
    for (int c = ty; c < 64; c += 4) {
        const int64_t i = i0 + tx, j = j0 + c;
        float v = 0.0f;
        if (i < n && j < n && i <= j) v = X[j * ldx + i];
        tile[tx][c] = v;
    }
    __syncthreads();
    if (bi == bj) {  // complete the diagonal tile from its upper half
        for (int c = ty; c < 64; c += 4)
            if (tx > c) tile[tx][c] = tile[c][tx];
        __syncthreads();
    }
    // direct write: O(i0 + tx, j0 + c) at column j0 + c
    for (int c = ty; c < 64; c += 4) {
        const float v = tile[tx][c] * s;
        const T hi = cvt<T>(v);
        Ohi[(j0 + c) * ldo + i0 + tx] = hi;
        if constexpr (SPLIT) Olo[(j0 + c) * ldo + i0 + tx] = cvt<T>((v - (float)hi) * lo_scale);
    }
    if (bi == bj) return;
    // mirrored write: O(j0 + tx, i0 + c) = tile[c][tx]
    for (int c = ty; c < 64; c += 4) {
        const float v = tile[c][tx] * s;
        const T hi = cvt<T>(v);
        Ohi[(i0 + c) * ldo + j0 + tx] = hi;
        if constexpr (SPLIT) Olo[(i0 + c) * ldo + j0 + tx] = cvt<T>((v - (float)hi) * lo_scale);
    }
}

template <typename T, bool SPLIT>
static hipError_t mirror_cast_t(const float *X, int64_t ldx, int64_t n, int64_t n_out, const Scalars *scal,
                                int use_inv_lam, void *Ohi, void *Olo, int64_t ldo, float lo_scale, hipStream_t s) {
    const int64_t nt = (n_out + 63) / 64;
    const int64_t ntiles = nt * (nt + 1) / 2;
    if (ntiles == 0) return hipSuccess;
    hipLaunchKernelGGL((mirror_cast_kernel<T, SPLIT>), dim3((unsigned)ntiles), dim3(256), 0, s, X, ldx, n, scal,
                       use_inv_lam, (T *)Ohi, (T *)Olo, ldo, lo_scale);
    return hipGetLastError();
}

hipError_t mirror_cast(const float *X, int64_t ldx, int64_t n, int64_t n_out, const Scalars *scal, int use_inv_lam,
                       int dtype, void *Ohi, void *Olo, int64_t ldo, hipStream_t s) {
    if (n_out % 64) return hipErrorInvalidValue;
    switch (dtype) {
        case 0: return mirror_cast_t<float, false>(X, ldx, n, n_out, scal, use_inv_lam, Ohi, nullptr, ldo, 1.0f, s);
        case 1:
            return Olo ? mirror_cast_t<f16, true>(X, ldx, n, n_out, scal, use_inv_lam, Ohi, Olo, ldo, 2048.0f, s)
                       : mirror_cast_t<f16, false>(X, ldx, n, n_out, scal, use_inv_lam, Ohi, nullptr, ldo, 1.0f, s);
        case 2:
            return Olo ? mirror_cast_t<bf16, true>(X, ldx, n, n_out, scal, use_inv_lam, Ohi, Olo, ldo, 1.0f, s)
                       : mirror_cast_t<bf16, false>(X, ldx, n, n_out, scal, use_inv_lam, Ohi, nullptr, ldo, 1.0f, s);
    }
    return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------
// Lanczos
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// SplitMix64 (Steele, Lea & Flood 2014) as a counter-based generator:
// z_i = mix(seed + (i + 1) * 0x9E3779B97F4A7C15); v_i = 2 (z_i >> 11) 2^-53 - 1.
__device__ __forceinline__ double start_entry(uint64_t i, uint64_t seed) {
    uint64_t z = seed + (i + 1ull) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z = z ^ (z >> 31);
    return 2.0 * ((double)(z >> 11) * 0x1.0p-53) - 1.0;
}

// ---------------------------------------------------------------------------
// Symmetric matvec from the upper triangle. The triangle is cut into
// kTB x kTB tiles (I <= J, enumerated column by column: t = J (J + 1) / 2 + I).
// Tile (I, J) reads its upper part once and produces
//   d[t][c] = sum_{i in I} X(i, j0 + c) v_i           (column dots)
//   a[t][r] = sum_{j in J} X(i0 + r, j) v_j           (row sums, i < j only)
// and y_k = sum_{I <= K} d[tile(I, K)][k] + sum_{J >= K} a[tile(K, J)][k],
// summed in that fixed order by symv_reduce_kernel. With NORMS the same is
// done for X(i, j)^2 and v = 1, which yields the full column norms.
// ---------------------------------------------------------------------------
constexpr int kTB = 128;

__device__ __forceinline__ void tile_of(int t, int &I, int &J) {
    int j = (int)((sqrtf(8.0f * (float)t + 1.0f) - 1.0f) * 0.5f);
    while ((j + 1) * (j + 2) / 2 <= t) ++j;
    while (j * (j + 1) / 2 > t) --j;
    J = j;
    I = t - j * (j + 1) / 2;
}

template <bool NORMS>
__global__ __launch_bounds__(256) void symv_tile_kernel(const float *__restrict__ X, int64_t ld, int64_t n,
                                                        const double *__restrict__ v, const double *vscale,
                                                        double *__restrict__ d, double *__restrict__ a,
                                                        double *__restrict__ d2, double *__restrict__ a2,
                                                        const Scalars *scal, int stop_on_flag) {
    if (stop_on_flag && scal->stop) return;
    const int t = blockIdx.x;
    int I, J;
    tile_of(t, I, J);
    const int64_t i0 = (int64_t)I * kTB, j0 = (int64_t)J * kTB;
    const bool diag = (I == J);
    __shared__ double vI[kTB], vJ[kTB];
    __shared__ double red[4][kTB], red2[4][kTB];
    const double sc = vscale ? *vscale : 1.0;
    if (threadIdx.x < kTB) {
        const int64_t i = i0 + threadIdx.x;
        vI[threadIdx.x] = i < n ? v[i] * sc : 0.0;
    } else {
        const int64_t j = j0 + threadIdx.x - kTB;
        vJ[threadIdx.x - kTB] = j < n ? v[j] * sc : 0.0;
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int r0 = 2 * lane;  // this lane's two rows of the tile
    const int64_t ia = i0 + r0, ib = ia + 1;
    double ax0 = 0.0, ax1 = 0.0, sq0 = 0.0, sq1 = 0.0;
    const double via = vI[r0], vib = vI[r0 + 1];
    // wave w handles tile columns c = 32 w .. 32 w + 31
#pragma unroll 8
    for (int cc = 0; cc < 32; ++cc) {
        const int c = 32 * wave + cc;
        const int64_t j = j0 + c;
        float x0 = 0.0f, x1 = 0.0f;
        if (j < n) {
            const float *col = X + j * ld;
            if (ia < n && (!diag || ia <= j)) x0 = col[ia];
            if (ib < n && (!diag || ib <= j)) x1 = col[ib];
        }
        const double dot = wave_sum((double)x0 * via + (double)x1 * vib);
        const double vj = vJ[c];
        // row sums: strictly upper entries only (the diagonal is in the dot)
        const bool u0 = !diag || ia < j, u1 = !diag || ib < j;
        ax0 += u0 ? (double)x0 * vj : 0.0;
        ax1 += u1 ? (double)x1 * vj : 0.0;
        if (lane == 0) d[(int64_t)t * kTB + c] = dot;
        if constexpr (NORMS) {
            const double q = wave_sum((double)x0 * x0 + (double)x1 * x1);
            sq0 += u0 ? (double)x0 * x0 : 0.0;
            sq1 += u1 ? (double)x1 * x1 : 0.0;
            if (lane == 0) d2[(int64_t)t * kTB + c] = q;
        }
    }
    red[wave][r0] = ax0;
    red[wave][r0 + 1] = ax1;
    if constexpr (NORMS) {
        red2[wave][r0] = sq0;
        red2[wave][r0 + 1] = sq1;
    }
    __syncthreads();
    if (threadIdx.x < kTB) {
        const int r = threadIdx.x;
        a[(int64_t)t * kTB + r] = red[0][r] + red[1][r] + red[2][r] + red[3][r];
        if constexpr (NORMS) a2[(int64_t)t * kTB + r] = red2[0][r] + red2[1][r] + red2[2][r] + red2[3][r];
    }
}

constexpr int kRows = 256;  // rows per block in the vector kernels

// Block reduction of NV doubles per thread into out[0..NV) (thread 0 holds it).
template <int NV>
__device__ __forceinline__ void block_reduce(double (&v)[NV], double *sh /* [4][NV] */) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < NV; ++k) v[k] = wave_sum(v[k]);
    if (lane == 0)
#pragma unroll
        for (int k = 0; k < NV; ++k) sh[wave * NV + k] = v[k];
    __syncthreads();
    if (threadIdx.x == 0)
#pragma unroll
        for (int k = 0; k < NV; ++k) v[k] = sh[k] + sh[NV + k] + sh[2 * NV + k] + sh[3 * NV + k];
}

// Sum of the per-block partials part[b * stride + k], b = 0..nb-1, in order.
__device__ __forceinline__ double sum_partials(const double *part, int nb, int stride, int k) {
    double s = 0.0;
    for (int b = 0; b < nb; ++b) s += part[(int64_t)b * stride + k];
    return s;
}

// y_k from the symv tile partials (fixed order: column dots of tiles I <= K,
// then row sums of tiles J >= K). NORMS: also colsq_k. ORTH0: also the first
// Gram-Schmidt partials part[block][c] = sum over this block's rows of
// V[i, c] y_i, c <= jstep (the block covers kRows rows).
template <bool NORMS, bool ORTH0>
__global__ __launch_bounds__(256) void symv_reduce_kernel(int64_t n, const double *__restrict__ d,
                                                          const double *__restrict__ a, const double *__restrict__ d2,
                                                          const double *__restrict__ a2, double *__restrict__ y,
                                                          double *__restrict__ colsq, const double *__restrict__ V,
                                                          int jstep, double *__restrict__ part, const Scalars *scal,
                                                          int stop_on_flag) {
    if (stop_on_flag && scal->stop) return;
    const int64_t k = (int64_t)blockIdx.x * kRows + threadIdx.x;
    const int T = (int)((n + kTB - 1) / kTB);
    double yk = 0.0, ck = 0.0;
    if (k < n) {
        const int K = (int)(k / kTB), kk = (int)(k % kTB);
        const int64_t base = (int64_t)K * (K + 1) / 2;
        for (int I = 0; I <= K; ++I) {
            yk += d[(base + I) * kTB + kk];
            if constexpr (NORMS) ck += d2[(base + I) * kTB + kk];
        }
        for (int J = K; J < T; ++J) {
            const int64_t t = (int64_t)J * (J + 1) / 2 + K;
            yk += a[t * kTB + kk];
            if constexpr (NORMS) ck += a2[t * kTB + kk];
        }
        y[k] = yk;
        if constexpr (NORMS) colsq[k] = ck;
    }
    if constexpr (ORTH0) {
        __shared__ double red[4 * kMaxLanczos];
        double h[kMaxLanczos];
#pragma unroll
        for (int c = 0; c < kMaxLanczos; ++c) h[c] = (c <= jstep && k < n) ? V[(int64_t)c * n + k] * yk : 0.0;
        block_reduce<kMaxLanczos>(h, red);
        if (threadIdx.x == 0)
            for (int c = 0; c <= jstep; ++c) part[(int64_t)blockIdx.x * kMaxLanczos + c] = h[c];
    }
}

// Start vector: V[:, 0] = v / ||v||. Pass 0 writes v and the partial norms,
// pass 1 normalises.
__global__ __launch_bounds__(256) void lz_start_kernel(double *V, int64_t n, double *part, int pass, uint64_t seed) {
    const int64_t i = (int64_t)blockIdx.x * kRows + threadIdx.x;
    __shared__ double sh[4];
    if (pass == 0) {
        double x[1] = {0.0};
        if (i < n) {
            const double e = start_entry((uint64_t)i, seed);
            V[i] = e;
            x[0] = e * e;
        }
        block_reduce<1>(x, sh);
        if (threadIdx.x == 0) part[(int64_t)blockIdx.x * kMaxLanczos] = x[0];
    } else {
        const double nrm = sqrt(sum_partials(part, gridDim.x, kMaxLanczos, 0));
        if (i < n) V[i] = V[i] / nrm;
    }
}

// Orthogonalisation pass of step j over rows of this block.
//  pass 0: part <- V[:, 0..j]^T w (first classical Gram-Schmidt pass)
//  pass 1: h = sum(part); alpha_j = h_j; w -= V h; part <- V^T w (second pass)
//  pass 2: h = sum(part); w -= V h; part <- ||w||^2
__global__ __launch_bounds__(256) void lz_orth_kernel(const double *V, int64_t n, int j, double *w, const double *part_in,
                                                      double *part_out, Scalars *scal, int pass) {
    if (scal->stop) return;
    const int64_t i = (int64_t)blockIdx.x * kRows + threadIdx.x;
    const int nb = gridDim.x;
    __shared__ double hsh[kMaxLanczos];
    __shared__ double red[4 * kMaxLanczos];
    double wi = (i < n) ? w[i] : 0.0;
    if (pass > 0) {
        if (threadIdx.x <= j) hsh[threadIdx.x] = sum_partials(part_in, nb, kMaxLanczos, threadIdx.x);
        __syncthreads();
        if (pass == 1 && blockIdx.x == 0 && threadIdx.x == 0) {
            scal->alpha[j] = hsh[j];
            scal->amax = fmax(scal->amax, fabs(hsh[j]));
        }
        if (i < n) {
            double s = 0.0;
            for (int k = 0; k <= j; ++k) s += V[(int64_t)k * n + i] * hsh[k];
            wi -= s;
            w[i] = wi;
        }
    }
    if (pass < 2) {
        double h[kMaxLanczos];
#pragma unroll
        for (int k = 0; k < kMaxLanczos; ++k) h[k] = (k <= j && i < n) ? V[(int64_t)k * n + i] * wi : 0.0;
        block_reduce<kMaxLanczos>(h, red);
        if (threadIdx.x == 0)
            for (int k = 0; k <= j; ++k) part_out[(int64_t)blockIdx.x * kMaxLanczos + k] = h[k];
    } else {
        double x[1] = {wi * wi};
        block_reduce<1>(x, red);
        if (threadIdx.x == 0) part_out[(int64_t)blockIdx.x * kMaxLanczos] = x[0];
    }
}

// beta_j = ||w||; stop if beta_j <= 1e-13 max|alpha| or j is the last step,
// else V[:, j+1] = w / beta_j.
__global__ __launch_bounds__(256) void lz_next_kernel(double *V, int64_t n, int j, int steps, const double *w,
                                                      const double *part, Scalars *scal) {
    if (scal->stop) return;
    const int64_t i = (int64_t)blockIdx.x * kRows + threadIdx.x;
    const double beta = sqrt(sum_partials(part, gridDim.x, kMaxLanczos, 0));
    const bool stop = (j == steps - 1) || !(beta > 1e-13 * scal->amax);
    if (!stop && i < n) V[(int64_t)(j + 1) * n + i] = w[i] / beta;
    // Every block has read scal->stop/amax above; the flag update below is
    // seen only by later kernels on the stream.
    __syncthreads();
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        scal->k = j + 1;
        scal->beta_last = beta;
        if (!stop) scal->beta[j] = beta;
    }
    if (stop && blockIdx.x == 0 && threadIdx.x == 0) scal->stop = 1;
}

// Number of eigenvalues of the k x k symmetric tridiagonal (al, be) below x
// (Sylvester inertia of the LDL^T factorisation of T - x I).
__device__ __forceinline__ int sturm_count(const double *al, const double *be, int k, double x, double tiny) {
    int cnt = 0;
    double d = al[0] - x;
    if (d == 0.0) d = -tiny;
    cnt += d < 0.0;
    for (int i = 1; i < k; ++i) {
        d = al[i] - x - be[i - 1] * be[i - 1] / d;
        if (d == 0.0) d = -tiny;
        cnt += d < 0.0;
    }
    return cnt;
}

// Largest eigenpair of the k x k tridiagonal T (alpha, beta) of the Lanczos
// run (k <= KM). sigma: multisection of the Gershgorin interval on the Sturm
// count, one wave evaluating 64 shifts per round. s: inverse iteration on
// T - sigma I with a partially pivoted tridiagonal LU (one thread; loops are
// unrolled to KM with guards so the arrays stay in registers).
template <int KM>
__global__ __launch_bounds__(64) void lz_ritz_kernel(Scalars *scal) {
    const int lane = threadIdx.x;
    const int k = scal->k;
    __shared__ double al[kMaxLanczos], be[kMaxLanczos];
    __shared__ double lo_hi[2];
    if (lane < kMaxLanczos) {
        al[lane] = lane < k ? scal->alpha[lane] : 0.0;
        be[lane] = lane < k - 1 ? scal->beta[lane] : 0.0;
    }
    __syncthreads();
    if (lane == 0) {
        double lo = 0.0, hi = 0.0;
        for (int i = 0; i < k; ++i) {
            const double r = (i > 0 ? fabs(be[i - 1]) : 0.0) + (i < k - 1 ? fabs(be[i]) : 0.0);
            lo = (i == 0) ? al[i] - r : fmin(lo, al[i] - r);
            hi = (i == 0) ? al[i] + r : fmax(hi, al[i] + r);
        }
        lo_hi[0] = lo;
        lo_hi[1] = hi;
    }
    __syncthreads();
    double lo = lo_hi[0], hi = lo_hi[1];
    const double scale_t = fmax(fabs(lo), fabs(hi));
    const double tiny = 1e-300 + 1e-30 * scale_t;
    // invariant: count(lo) < k (sigma >= lo), count(hi) == k (sigma < hi)
    hi = hi + 1e-15 * scale_t + tiny;
    for (int it = 0; it < 40; ++it) {
        if (!(hi - lo > 4e-16 * fmax(fabs(lo), fabs(hi))) || !(hi > lo)) break;
        const double x = lo + (hi - lo) * (double)(lane + 1) / 65.0;
        const int all_below = sturm_count(al, be, k, x, tiny) == k;
        const unsigned long long m = __ballot(all_below);  // lanes whose shift is above sigma
        const int f = m ? __ffsll((long long)m) - 1 : 64;
        const double nlo = f == 0 ? lo : lo + (hi - lo) * (double)f / 65.0;
        const double nhi = f == 64 ? hi : lo + (hi - lo) * (double)(f + 1) / 65.0;
        lo = nlo;
        hi = nhi;
    }
    if (lane != 0) return;
    const double sigma = 0.5 * (lo + hi);
    scal->sigma = sigma;
    // LU of T - sigma I with partial pivoting: rows i, i+1 may swap; U has two
    // superdiagonals (du, du2); dl holds the multipliers.
    double d[KM], du[KM], du2[KM], dl[KM], x[KM];
    bool sw[KM];
#pragma unroll
    for (int i = 0; i < KM; ++i) {
        d[i] = i < k ? al[i] - sigma : 1.0;
        du[i] = i < k - 1 ? be[i] : 0.0;
        dl[i] = i < k - 1 ? be[i] : 0.0;
        du2[i] = 0.0;
        sw[i] = false;
        x[i] = i < k ? 1.0 : 0.0;
    }
    const double eps_p = 1e-15 * (scale_t > 0.0 ? scale_t : 1.0);
#pragma unroll
    for (int i = 0; i < KM - 1; ++i) {
        if (i < k - 1) {
            if (fabs(d[i]) >= fabs(dl[i])) {
                if (fabs(d[i]) < eps_p) d[i] = d[i] < 0.0 ? -eps_p : eps_p;
                const double f = dl[i] / d[i];
                dl[i] = f;
                d[i + 1] -= f * du[i];
            } else {
                const double f = d[i] / dl[i];
                d[i] = dl[i];
                dl[i] = f;
                const double t = du[i];
                du[i] = d[i + 1];
                d[i + 1] = t - f * d[i + 1];
                if (i < k - 2) {
                    du2[i] = du[i + 1];
                    du[i + 1] = -f * du[i + 1];
                }
                sw[i] = true;
            }
        }
    }
#pragma unroll
    for (int i = 0; i < KM; ++i)
        if (i == k - 1 && fabs(d[i]) < eps_p) d[i] = d[i] < 0.0 ? -eps_p : eps_p;
    for (int it = 0; it < 3; ++it) {
#pragma unroll
        for (int i = 0; i < KM - 1; ++i) {  // L^-1 P
            if (i < k - 1) {
                if (sw[i]) { const double t = x[i]; x[i] = x[i + 1]; x[i + 1] = t; }
                x[i + 1] -= dl[i] * x[i];
            }
        }
#pragma unroll
        for (int i = KM - 1; i >= 0; --i) {  // U^-1
            if (i < k) {
                double v = x[i];
                if (i + 1 < KM && i + 1 < k) v -= du[i] * x[i + 1];
                if (i + 2 < KM && i + 2 < k) v -= du2[i] * x[i + 2];
                x[i] = v / d[i];
            }
        }
        double nrm = 0.0;
#pragma unroll
        for (int i = 0; i < KM; ++i) nrm += i < k ? x[i] * x[i] : 0.0;
        nrm = sqrt(nrm);
#pragma unroll
        for (int i = 0; i < KM; ++i) x[i] = i < k ? (nrm > 0.0 ? x[i] / nrm : (i == 0 ? 1.0 : 0.0)) : 0.0;
    }
#pragma unroll
    for (int i = 0; i < kMaxLanczos; ++i) scal->s[i] = i < KM ? x[i < KM ? i : 0] * (i < k ? 1.0 : 0.0) : 0.0;
}

// q = V[:, 0..k) s; part <- ||q||^2
__global__ __launch_bounds__(256) void lz_q_kernel(const double *V, int64_t n, double *q, double *part, const Scalars *scal) {
    const int64_t i = (int64_t)blockIdx.x * kRows + threadIdx.x;
    __shared__ double red[4];
    double qi = 0.0;
    if (i < n) {
        for (int k = 0; k < scal->k; ++k) qi += V[(int64_t)k * n + i] * scal->s[k];
        q[i] = qi;
    }
    double x[1] = {qi * qi};
    block_reduce<1>(x, red);
    if (threadIdx.x == 0) part[(int64_t)blockIdx.x * kMaxLanczos] = x[0];
}

__global__ void lz_qnorm_kernel(const double *part, int nb, Scalars *scal) {
    if (threadIdx.x != 0) return;
    const double nrm = sqrt(sum_partials(part, nb, kMaxLanczos, 0));
    scal->qnorm_inv = nrm > 0.0 ? 1.0 / nrm : 0.0;
}

// part <- ||w - sigma q_hat||^2 with q_hat = q * qnorm_inv
__global__ __launch_bounds__(256) void lz_resid_kernel(const double *w, const double *q, int64_t n, double *part,
                                                       const Scalars *scal) {
    const int64_t i = (int64_t)blockIdx.x * kRows + threadIdx.x;
    __shared__ double red[4];
    double r = 0.0;
    if (i < n) r = w[i] - scal->sigma * (q[i] * scal->qnorm_inv);
    double x[1] = {r * r};
    block_reduce<1>(x, red);
    if (threadIdx.x == 0) part[(int64_t)blockIdx.x * kMaxLanczos] = x[0];
}

// Frobenius norm and column-norm maximum from colsq, residual from the
// partials, then lam = sqrt(sigma + r) (Theorem 2), guarded: if lam is not at
// least the largest column norm (a lower bound on ||X||_2) the Frobenius norm
// is used; lam is capped by the Frobenius norm (also an upper bound).
__global__ __launch_bounds__(256) void lz_bound_kernel(const double *colsq, int64_t n, const double *part, int nb,
                                                       Scalars *scal, int force_fallback) {
    __shared__ double sh_sum[256], sh_max[256];
    double s = 0.0, m = 0.0;
    int bad = 0;
    // fixed per-thread stride, then a fixed-order tree: deterministic
    for (int64_t i = threadIdx.x; i < n; i += 256) {
        const double c = colsq[i];
        s += c;
        if (!(c <= 1.7e308)) bad = 1;  // NaN or Inf
        m = fmax(m, c);
    }
    sh_sum[threadIdx.x] = s;
    sh_max[threadIdx.x] = bad ? INFINITY : m;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            sh_sum[threadIdx.x] += sh_sum[threadIdx.x + w];
            sh_max[threadIdx.x] = fmax(sh_max[threadIdx.x], sh_max[threadIdx.x + w]);
        }
        __syncthreads();
    }
    if (threadIdx.x != 0) return;
    const double fro2 = sh_sum[0], colmax2 = sh_max[0];
    scal->fro2 = fro2;
    scal->colmax2 = colmax2;
    const int nonfinite = !(fro2 <= 1.7e308) || !(colmax2 <= 1.7e308);
    scal->nonfinite = nonfinite;
    const double r = sqrt(sum_partials(part, nb, kMaxLanczos, 0));
    scal->resid = r;
    const double lz = sqrt(fmax(scal->sigma + r, 0.0));
    scal->lanczos_lam = lz;
    const double fro = sqrt(fro2), colmax = sqrt(colmax2);
    double lam = lz;
    int fb = 0;
    if (force_fallback) lam = 0.5 * lz;  // test hook: an invalid bound
    if (!(lam >= colmax)) { lam = fro; fb = 1; }
    if (lam > fro) lam = fro;
    scal->fallback = fb;
    scal->lam = nonfinite ? 0.0 : lam;
    scal->inv_lam = (nonfinite || !(lam > 0.0)) ? 0.0 : 1.0 / lam;
}

__global__ void scal_init_kernel(Scalars *scal) {
    if (threadIdx.x == 0) {
        Scalars z = {};
        *scal = z;
    }
}

hipError_t spectral_bound(const float *X, int64_t ldx, int64_t n, int steps, uint64_t seed, LanczosWork wk,
                          Scalars *scal, int force_fallback, hipStream_t s) {
    if (steps < 1 || steps > kMaxLanczos) return hipErrorInvalidValue;
    const unsigned nbv = (unsigned)((n + kRows - 1) / kRows);
    const int64_t T = (n + kTB - 1) / kTB;
    const unsigned ntiles = (unsigned)(T * (T + 1) / 2);
    if (nbv == 0) return hipSuccess;
    double *V = wk.V, *u = wk.u, *w = wk.w, *pa = wk.part_a, *pb = wk.part_b;
    double *d = wk.sd, *a = wk.sa, *d2 = wk.sd2, *a2 = wk.sa2;
    const double *nulld = nullptr;
    // y = X v: tile partials, then the fixed-order reduction (+ first GS pass)
    auto symv = [&](const double *vin, const double *vscale, double *yout, bool norms, bool orth0, int jstep,
                    double *part, int stop_flag) {
        if (norms) {
            hipLaunchKernelGGL(symv_tile_kernel<true>, dim3(ntiles), dim3(256), 0, s, X, ldx, n, vin, vscale, d, a,
                               d2, a2, (const Scalars *)scal, stop_flag);
            hipLaunchKernelGGL((symv_reduce_kernel<true, false>), dim3(nbv), dim3(256), 0, s, n, (const double *)d,
                               (const double *)a, (const double *)d2, (const double *)a2, yout, wk.colsq, nulld, 0,
                               (double *)nullptr, (const Scalars *)scal, stop_flag);
        } else {
            hipLaunchKernelGGL(symv_tile_kernel<false>, dim3(ntiles), dim3(256), 0, s, X, ldx, n, vin, vscale, d, a,
                               (double *)nullptr, (double *)nullptr, (const Scalars *)scal, stop_flag);
            if (orth0)
                hipLaunchKernelGGL((symv_reduce_kernel<false, true>), dim3(nbv), dim3(256), 0, s, n,
                                   (const double *)d, (const double *)a, nulld, nulld, yout, (double *)nullptr,
                                   (const double *)V, jstep, part, (const Scalars *)scal, stop_flag);
            else
                hipLaunchKernelGGL((symv_reduce_kernel<false, false>), dim3(nbv), dim3(256), 0, s, n,
                                   (const double *)d, (const double *)a, nulld, nulld, yout, (double *)nullptr, nulld,
                                   0, (double *)nullptr, (const Scalars *)scal, stop_flag);
        }
    };
    hipLaunchKernelGGL(scal_init_kernel, dim3(1), dim3(64), 0, s, scal);
    hipLaunchKernelGGL(lz_start_kernel, dim3(nbv), dim3(256), 0, s, V, n, pa, 0, seed);
    hipLaunchKernelGGL(lz_start_kernel, dim3(nbv), dim3(256), 0, s, V, n, pa, 1, seed);
    for (int j = 0; j < steps; ++j) {
        symv(V + (int64_t)j * n, nullptr, u, j == 0, false, 0, nullptr, 1);  // u = X v_j
        symv(u, nullptr, w, false, true, j, pa, 1);                           // w = X u, part_a = V^T w
        hipLaunchKernelGGL(lz_orth_kernel, dim3(nbv), dim3(256), 0, s, (const double *)V, n, j, w, (const double *)pa,
                           pb, scal, 1);
        hipLaunchKernelGGL(lz_orth_kernel, dim3(nbv), dim3(256), 0, s, (const double *)V, n, j, w, (const double *)pb,
                           pa, scal, 2);
        hipLaunchKernelGGL(lz_next_kernel, dim3(nbv), dim3(256), 0, s, V, n, j, steps, (const double *)w,
                           (const double *)pa, scal);
    }
    if (steps <= 20)
        hipLaunchKernelGGL(lz_ritz_kernel<20>, dim3(1), dim3(64), 0, s, scal);
    else
        hipLaunchKernelGGL(lz_ritz_kernel<kMaxLanczos>, dim3(1), dim3(64), 0, s, scal);
    hipLaunchKernelGGL(lz_q_kernel, dim3(nbv), dim3(256), 0, s, (const double *)V, n, u, pa, (const Scalars *)scal);
    hipLaunchKernelGGL(lz_qnorm_kernel, dim3(1), dim3(64), 0, s, (const double *)pa, (int)nbv, scal);
    symv(u, &scal->qnorm_inv, w, false, false, 0, nullptr, 0);  // X q_hat
    symv(w, nullptr, wk.w2, false, false, 0, nullptr, 0);       // X^2 q_hat
    hipLaunchKernelGGL(lz_resid_kernel, dim3(nbv), dim3(256), 0, s, (const double *)wk.w2, (const double *)u, n, pa,
                       (const Scalars *)scal);
    hipLaunchKernelGGL(lz_bound_kernel, dim3(1), dim3(256), 0, s, (const double *)wk.colsq, n, (const double *)pa,
                       (int)nbv, scal, force_fallback);
    return hipGetLastError();
}

size_t lanczos_work_doubles(int64_t n, int steps) {
    const int64_t nbv = (n + kRows - 1) / kRows;
    const int64_t T = (n + kTB - 1) / kTB;
    const int64_t tiles = T * (T + 1) / 2;
    return (size_t)(n * steps + 5 * n + 2 * nbv * kMaxLanczos + 4 * tiles * kTB + 64);
}

int64_t symv_tile_count(int64_t n) {
    const int64_t T = (n + kTB - 1) / kTB;
    return T * (T + 1) / 2;
}

}  // namespace psd

// Device helpers of the FP64 Lanczos run that yields the spectral bound
// (Section 3.4, Theorem 2): the start vector's counter-based generator and
// the largest Ritz pair of the Lanczos tridiagonal. Shared by the per-step
// kernels of the launch sequence and the one-workgroup small-matrix kernel.
#pragma once
#include <math.h>

#include "common.hpp"

namespace psd {

// SplitMix64 (Steele, Lea & Flood 2014) as a counter-based generator:
// z_i = mix(seed + (i + 1) * 0x9E3779B97F4A7C15); v_i = 2 (z_i >> 11) 2^-53 - 1.
__device__ __forceinline__ double start_entry(uint64_t i, uint64_t seed) {
    uint64_t z = seed + (i + 1ull) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z = z ^ (z >> 31);
    return 2.0 * ((double)(z >> 11) * 0x1.0p-53) - 1.0;
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

// Largest eigenpair of the k x k tridiagonal T (al, be in LDS) of a Lanczos
// run (k <= KM). sigma: multisection of the Gershgorin interval on the Sturm
// count, each wave evaluating 64 shifts per round (every wave of the block
// takes the same steps). s: inverse iteration on T - sigma I with a partially
// pivoted tridiagonal LU (thread 0; loops are unrolled to KM with guards so
// the arrays stay in registers). Every thread of the block calls it; thread 0
// writes *sigma_out and s_out[0..kMaxLanczos). lo_hi: two doubles of LDS.
template <int KM>
__device__ __forceinline__ void ritz_largest(const double *al, const double *be, int k, double *lo_hi,
                                             double *sigma_out, double *s_out) {
    const int lane = threadIdx.x & 63;
    if (threadIdx.x == 0) {
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
    if (threadIdx.x != 0) return;
    const double sigma = 0.5 * (lo + hi);
    *sigma_out = sigma;
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
    for (int i = 0; i < kMaxLanczos; ++i) s_out[i] = i < KM ? x[i < KM ? i : 0] * (i < k ? 1.0 : 0.0) : 0.0;
}

}  // namespace psd

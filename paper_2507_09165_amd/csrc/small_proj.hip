// One-workgroup projection of a small matrix (n <= 128): the whole of
// Algorithm 2 for one matrix in one workgroup, with no inter-workgroup
// dependency, so one launch carries every small matrix of a batch at once.
//
//  * X (upper triangle, mirrored, zero-padded) is held in LDS as FP32; the
//    column norms, ||X||_F and the non-finite check come from it.
//  * The spectral bound (Section 3.4, Theorem 2; Algorithm 2, first two steps)
//    is the same FP64 Lanczos run on X^2 as the launch sequence's: start
//    vector from the counter-based generator, two classical Gram-Schmidt
//    passes per step, the same stopping test, the largest Ritz pair of the
//    tridiagonal, lam = sqrt(sigma + ||X^2 q - sigma q||), the guard and the
//    Frobenius cap. The Lanczos basis lives in LDS.
//  * X0 = X / lam and the stage matrices (A = X X, B = b A + c A^2,
//    X' = a X + X B; the final P = (X + lam X0 X_T) / 2) are 128 x 128 work
//    matrices in the matrix's workspace (they stay in the L2). Each product
//    computes the 10 upper 32 x 32 blocks of the triangle on the work
//    precision's MFMA with FP32 accumulators and writes each block and its
//    mirror, so every stored matrix is exactly symmetric.
//  * Split products follow the mode's format: FP16 (or BF16) hi + lo halves,
//    or an FP8 pair, whose lo part is an e4m3 code of the residual scaled by
//    2^(shift + e) and whose cross terms pair e4m3 codes of the hi part with
//    the lo codes. Here the codes are held as their (exact) FP16 / BF16
//    values and the cross terms run on the FP16 / BF16 MFMA: the products of
//    two e4m3 values are exact in FP32 either way.
// Every reduction has a fixed order, so a matrix's result does not depend on
// what else is in the launch.
#include <math.h>

#include "gemm_sym_kernel.hpp"
#include "lanczos_dev.hpp"
#include "small_proj.hpp"

namespace psd {
namespace {

constexpr int NE = kSmallEdge;     // work-matrix edge
constexpr int XLD = NE + 1;        // LDS row stride of X (floats): conflict-free rows and columns
constexpr int VLD = NE + 1;        // LDS row stride of the Lanczos basis (doubles)

__device__ __forceinline__ double sm_wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}
__device__ __forceinline__ double sm_wave_max(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    return v;
}

// Sum over threads 0..127 of v (the other threads pass 0), in a fixed order;
// every thread gets the total.
__device__ __forceinline__ double sum128(double v, double *red) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    v = sm_wave_sum(v);
    if (lane == 0) red[wave] = v;
    __syncthreads();
    const double r = red[0] + red[1];
    __syncthreads();
    return r;
}

// vout = X vin (both padded to NE; X symmetric in LDS). Thread t sums half a
// row; the halves are added in order.
__device__ __forceinline__ void sm_matvec(const float *Xs, const double *vin, double *vout, double *tmp) {
    const int t = threadIdx.x, i = t & (NE - 1), h = t >> 7;
    double s = 0.0;
    const float *xc = Xs + (h * 64) * XLD + i;
    const double *vv = vin + h * 64;
#pragma unroll 16
    for (int jj = 0; jj < 64; ++jj) s += (double)xc[jj * XLD] * vv[jj];
    tmp[h * NE + i] = s;
    __syncthreads();
    if (t < NE) vout[t] = tmp[t] + tmp[NE + t];
    __syncthreads();
}

// h[c] = sum_i V[c][i] w[i] for c <= j. Thread t: column c = t % 32 over the
// 16 rows of part p = t / 32; the 8 parts are added in order.
__device__ __forceinline__ void sm_dots(const double *V, const double *w, int j, double *part, double *h) {
    const int t = threadIdx.x, c = t & 31, p = t >> 5;
    double s = 0.0;
    if (c <= j) {
        const double *vc = V + c * VLD + 16 * p;
        const double *wp = w + 16 * p;
#pragma unroll
        for (int ii = 0; ii < 16; ++ii) s += vc[ii] * wp[ii];
    }
    part[p * 32 + c] = s;
    __syncthreads();
    if (t < 32) {
        double r = 0.0;
#pragma unroll
        for (int q = 0; q < 8; ++q) r += part[q * 32 + t];
        h[t] = r;
    }
    __syncthreads();
}

// w -= V[0..j] h (threads 0..127, one row each; columns in order).
__device__ __forceinline__ void sm_orth(const double *V, const double *h, int j, double *w) {
    const int t = threadIdx.x;
    if (t < NE) {
        double s = 0.0;
        for (int c = 0; c <= j; ++c) s += V[c * VLD + t] * h[c];
        w[t] -= s;
    }
    __syncthreads();
}

template <typename T> using t8 = T __attribute__((ext_vector_type(8)));

// The 8 values of a fragment rounded to e4m3 after scaling by sc (an FP8
// pair's hi codes), returned as their exact T values.
template <typename T>
__device__ __forceinline__ u32x4 hi8_vals(u32x4 h, float sc) {
    const t8<T> v = __builtin_bit_cast(t8<T>, h);
    t8<T> o;
#pragma unroll
    for (int q = 0; q < 8; ++q) o[q] = (T)__builtin_amdgcn_cvt_f32_fp8((int)e4m3((float)v[q] * sc), 0);
    return __builtin_bit_cast(u32x4, o);
}

struct SmCtx {
    void *hi[4], *lo[4];
    int64_t ld;   // work-matrix leading dimension (elements)
    int n;
    const float *Xs;
    IoArg io;
    float lam;
    int nonfinite;
};

// One product C = L R (operands and output in work slots) with the filter
// epilogues. EPI_STORE / EPI_STORE_SPLIT: D = alpha C0 + beta C, stored (as a
// split pair); EPI_FINAL: out = (X + lam C) / 2 over the n x n matrix.
template <typename T, bool X8, bool SPLIT, int EPI>
__device__ void sm_product(const SmCtx &c, int sl, int sr, int sc0, bool c0_split, float alpha, float beta, int sd,
                           int es_l, int es_r, int es_c0, int es_d) {
    constexpr int PSH = X8 ? PairShift<T>::v : 0;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t ld = c.ld;
    // blocks of the n x n matrix; the K loop always spans the whole edge (the
    // work slots are zero outside the blocks, so every load is in bounds and
    // the padding adds exact zeros), unrolled so that all loads are in flight
    const int nb = (c.n + 31) / 32, nblk = nb * (nb + 1) / 2;
    const T *Lh = (const T *)c.hi[sl], *Rh = (const T *)c.hi[sr];
    const T *Ll = (const T *)c.lo[sl], *Rl = (const T *)c.lo[sr];
    // split accumulator scale: FP16 hi + lo halves carry R_hi scaled by 2^11
    const float acc_scale = (SPLIT && !X8) ? 1.0f / Elt<T>::kSplit : 1.0f;
    const float sx = X8 ? __builtin_ldexpf(1.0f, -(PSH + es_l + es_r)) : 0.0f;  // cross-term scale
    const float cva = X8 ? __builtin_ldexpf(1.0f, es_l) : 0.0f, cvb = X8 ? __builtin_ldexpf(1.0f, es_r) : 0.0f;
    for (int blk = wave; blk < nblk; blk += 4) {
        int bj = 0;
        while ((bj + 1) * (bj + 2) / 2 <= blk) ++bj;
        const int bi = blk - bj * (bj + 1) / 2;
        const int kh = 8 * (lane >> 5);
        const int64_t ca = (int64_t)(32 * bi + (lane & 31)) * ld + kh, cb = (int64_t)(32 * bj + (lane & 31)) * ld + kh;
        f32x16 acc = {}, accx = {};
#pragma unroll
        for (int ks = 0; ks < NE / 16; ++ks) {
            const int k0 = 16 * ks;
            const u32x4 a = *(const u32x4 *)(Lh + ca + k0);
            const u32x4 b = *(const u32x4 *)(Rh + cb + k0);
            if constexpr (!SPLIT) {
                mma(acc, a, b, T());
            } else {
                const u32x4 al = *(const u32x4 *)(Ll + ca + k0);
                const u32x4 bl = *(const u32x4 *)(Rl + cb + k0);
                if constexpr (!X8) {
                    mma(acc, a, scale_frag(b, T()), T());
                    mma(acc, a, bl, T());
                    mma(acc, al, b, T());
                } else {
                    mma(acc, a, b, T());
                    mma(accx, hi8_vals<T>(a, cva), bl, T());
                    mma(accx, al, hi8_vals<T>(b, cvb), T());
                }
            }
        }
        const bool diag = bi == bj;
        const int col = 32 * bj + (lane & 31);
        if constexpr (EPI == EPI_FINAL) {
            const float hl = 0.5f * c.lam * acc_scale;
            const float qnan = __builtin_nanf("");
#pragma unroll
            for (int e = 0; e < 16; ++e) {
                const int row = 32 * bi + 8 * (e / 4) + 4 * (lane >> 5) + (e % 4);
                if (row >= c.n || col >= c.n || (diag && row > col)) continue;
                float a_t = acc[e];
                if constexpr (X8 && SPLIT) a_t += accx[e] * sx;
                const float v = c.nonfinite ? qnan : 0.5f * c.Xs[col * XLD + row] + hl * a_t;
                c.io.out[(int64_t)col * c.io.ld + row] = v;
                c.io.out[(int64_t)row * c.io.ld + col] = v;
            }
        } else {
            T *Dh = (T *)c.hi[sd];
            T *Dl = (T *)c.lo[sd];
            const T *C0h = sc0 >= 0 ? (const T *)c.hi[sc0] : nullptr;
            const T *C0l = (sc0 >= 0 && c0_split) ? (const T *)c.lo[sc0] : nullptr;
            const float c0s = X8 ? __builtin_ldexpf(1.0f, -(PSH + es_c0)) : 1.0f / Elt<T>::kSplit;
            const float dls = X8 ? __builtin_ldexpf(1.0f, PSH + es_d) : Elt<T>::kSplit;
#pragma unroll
            for (int e = 0; e < 16; ++e) {
                const int row = 32 * bi + 8 * (e / 4) + 4 * (lane >> 5) + (e % 4);
                if (diag && row > col) continue;
                float a_t = acc[e];
                if constexpr (X8 && SPLIT) a_t += accx[e] * sx;
                float v = beta * (a_t * acc_scale);
                const int64_t ij = (int64_t)col * ld + row, ji = (int64_t)row * ld + col;
                if (C0h) {
                    v += alpha * (float)C0h[ij];
                    if (C0l) v += alpha * ((float)C0l[ij] * c0s);
                }
                const T h = (T)v;
                Dh[ij] = h;
                Dh[ji] = h;
                if constexpr (EPI == EPI_STORE_SPLIT) {
                    T l;
                    if constexpr (X8) l = (T)__builtin_amdgcn_cvt_f32_fp8((int)e4m3((v - (float)h) * dls), 0);
                    else l = (T)((v - (float)h) * dls);
                    Dl[ij] = l;
                    Dl[ji] = l;
                }
            }
        }
    }
    __syncthreads();
}

template <typename T, bool X8>
__device__ __forceinline__ void sm_product_rt(const SmCtx &c, bool split, int epi, int sl, int sr, int sc0,
                                              bool c0_split, float alpha, float beta, int sd, int es_l, int es_r,
                                              int es_c0, int es_d) {
    if (split) {
        if (epi == EPI_STORE)
            sm_product<T, X8, true, EPI_STORE>(c, sl, sr, sc0, c0_split, alpha, beta, sd, es_l, es_r, es_c0, es_d);
        else if (epi == EPI_STORE_SPLIT)
            sm_product<T, X8, true, EPI_STORE_SPLIT>(c, sl, sr, sc0, c0_split, alpha, beta, sd, es_l, es_r, es_c0, es_d);
        else
            sm_product<T, X8, true, EPI_FINAL>(c, sl, sr, sc0, c0_split, alpha, beta, sd, es_l, es_r, es_c0, es_d);
    } else {
        if (epi == EPI_STORE)
            sm_product<T, X8, false, EPI_STORE>(c, sl, sr, sc0, c0_split, alpha, beta, sd, es_l, es_r, es_c0, es_d);
        else if (epi == EPI_STORE_SPLIT)
            sm_product<T, X8, false, EPI_STORE_SPLIT>(c, sl, sr, sc0, c0_split, alpha, beta, sd, es_l, es_r, es_c0,
                                                      es_d);
        else
            sm_product<T, X8, false, EPI_FINAL>(c, sl, sr, sc0, c0_split, alpha, beta, sd, es_l, es_r, es_c0, es_d);
    }
}

template <typename T, bool X8>
__global__ __launch_bounds__(256) void small_proj_kernel(SmallArgs g) {
    __shared__ float Xs[NE * XLD];
    __shared__ double V[kMaxLanczos * VLD];
    __shared__ double u[NE], w[NE], tmp[2 * NE];
    __shared__ double part[8 * 32], hv[32], red[4];
    __shared__ double al[kMaxLanczos], be[kMaxLanczos], sv[kMaxLanczos], lo_hi[2], sig[1];
    const int m = (int)g.list[blockIdx.x].x;
    const MatDesc &dm = g.D[m];
    const IoArg io = io_of(g.io_tab, g.io0, m);
    Scalars *scal = dm.scal;
    const int n = (int)dm.n;
    const int t = threadIdx.x;

    // ---- X (upper triangle read, mirrored, zero-padded) and its column norms
    for (int idx = t; idx < NE * NE; idx += 256) {
        const int i = idx & (NE - 1), j = idx >> 7;
        float v = 0.0f;
        if (i < n && j < n) v = i <= j ? io.X[(int64_t)j * io.ld + i] : io.X[(int64_t)i * io.ld + j];
        Xs[j * XLD + i] = v;
    }
    __syncthreads();
    double colsq = 0.0;
    if (t < NE) {
        for (int i = 0; i < NE; ++i) {
            const double x = (double)Xs[t * XLD + i];
            colsq += x * x;
        }
    }
    const double fro2 = sum128(colsq, red);
    const int bad_t = !(colsq <= 1.7e308);
    double cm = sm_wave_max(bad_t ? INFINITY : colsq);
    if ((t & 63) == 0) red[t >> 6] = cm;
    __syncthreads();
    const double colmax2 = fmax(red[0], red[1]);
    __syncthreads();
    const int nonfinite = !(fro2 <= 1.7e308) || !(colmax2 <= 1.7e308);

    // ---- Lanczos on X^2
    {
        double e = 0.0;
        if (t < NE) e = t < n ? start_entry((uint64_t)t, g.seed) : 0.0;
        const double nrm = sqrt(sum128(e * e, red));
        if (t < NE) V[t] = e / nrm;
    }
    __syncthreads();
    double amax = 0.0, beta_last = 0.0;
    int k = 0;
    for (int j = 0; j < g.steps; ++j) {
        sm_matvec(Xs, V + j * VLD, u, tmp);  // u = X v_j
        sm_matvec(Xs, u, w, tmp);            // w = X u
        sm_dots(V, w, j, part, hv);          // first Gram-Schmidt pass
        const double alpha = hv[j];
        amax = fmax(amax, fabs(alpha));
        sm_orth(V, hv, j, w);
        sm_dots(V, w, j, part, hv);          // second pass
        sm_orth(V, hv, j, w);
        const double wt = t < NE ? w[t] : 0.0;
        const double beta = sqrt(sum128(wt * wt, red));
        const bool stop = (j == g.steps - 1) || !(beta > 1e-13 * amax);
        if (t == 0) {
            al[j] = alpha;
            be[j] = stop ? 0.0 : beta;
        }
        k = j + 1;
        beta_last = beta;
        if (stop) break;
        if (t < NE) V[(j + 1) * VLD + t] = w[t] / beta;
        __syncthreads();
    }
    __syncthreads();
    // largest Ritz pair of the k x k tridiagonal (its off-diagonal: be[0..k-1))
    if (g.steps <= 20) ritz_largest<20>(al, be, k, lo_hi, sig, sv);
    else ritz_largest<kMaxLanczos>(al, be, k, lo_hi, sig, sv);
    __syncthreads();
    const double sigma = sig[0];
    // q = V s, its norm; w = X q_hat, w2 = X w; residual of the Ritz pair
    double qi = 0.0;
    if (t < NE) {
        for (int c = 0; c < k; ++c) qi += V[c * VLD + t] * sv[c];
    }
    const double qn = sqrt(sum128(qi * qi, red));
    const double qnorm_inv = qn > 0.0 ? 1.0 / qn : 0.0;
    if (t < NE) u[t] = qi * qnorm_inv;
    __syncthreads();
    sm_matvec(Xs, u, w, tmp);
    sm_matvec(Xs, w, tmp + NE, part);  // w2 (in tmp's second half; part as the scratch)
    double rr = 0.0;
    if (t < NE) {
        const double r_i = tmp[NE + t] - sigma * u[t];
        rr = r_i * r_i;
    }
    const double resid = sqrt(sum128(rr, red));
    // Theorem 2's bound, the guard (largest column norm) and the Frobenius cap
    const double lz = sqrt(fmax(sigma + resid, 0.0));
    const double fro = sqrt(fro2), colmax = sqrt(colmax2);
    double lam = lz;
    int fb = 0;
    if (g.force_fallback) lam = 0.5 * lz;
    if (!(lam >= colmax)) { lam = fro; fb = 1; }
    if (lam > fro) lam = fro;
    if (g.lam_override > 0.0) { lam = g.lam_override; fb = 0; }
    const double lam_used = nonfinite ? 0.0 : lam;
    const double inv_lam = (nonfinite || !(lam > 0.0)) ? 0.0 : 1.0 / lam;
    if (t == 0) {
        scal->fro2 = fro2;
        scal->colmax2 = colmax2;
        scal->lam = lam_used;
        scal->inv_lam = inv_lam;
        scal->sigma = sigma;
        scal->resid = resid;
        scal->lanczos_lam = lz;
        scal->beta_last = beta_last;
        scal->qnorm_inv = qnorm_inv;
        scal->amax = amax;
        scal->k = k;
        scal->stop = 1;
        scal->nonfinite = nonfinite;
        scal->fallback = fb;
        scal->done = 0;
        scal->cur_slot = 0;
        scal->stages_run = g.T;
        scal->delta = 0.0;
        for (int c = 0; c < kMaxLanczos; ++c) {
            scal->alpha[c] = c < k ? al[c] : 0.0;
            scal->beta[c] = c < k - 1 ? be[c] : 0.0;
            scal->s[c] = sv[c];
        }
    }
    if (g.bound_only) return;

    // ---- X0 = X / lam in the work format (slot 0), zero-padded to NE; the
    // other slots zeroed (products write only the blocks of the n x n matrix)
    constexpr int PSH = X8 ? PairShift<T>::v : 0;
    const bool x0_split = g.split_final || (g.split_mask & 1u);
    const bool any_split = g.split_final || g.split_mask != 0;
    {
        for (int q = 1; q < 4; ++q) {
            T *zh = (T *)dm.hi[q];
            T *zl = any_split ? (T *)dm.lo[q] : nullptr;
            for (int idx = t; idx < NE * NE / 8; idx += 256) {
                const int i = (idx & (NE / 8 - 1)) * 8, j = idx / (NE / 8);
                const int64_t o = (int64_t)j * dm.ldw + i;
                *(u32x4 *)(zh + o) = u32x4{0u, 0u, 0u, 0u};
                if (zl) *(u32x4 *)(zl + o) = u32x4{0u, 0u, 0u, 0u};
            }
        }
        const float s = (float)inv_lam;
        T *Oh = (T *)dm.hi[0];
        T *Ol = (T *)dm.lo[0];
        const float ls = X8 ? __builtin_ldexpf(1.0f, PSH + g.ex[0]) : Elt<T>::kSplit;
        for (int idx = t; idx < NE * NE; idx += 256) {
            const int i = idx & (NE - 1), j = idx >> 7;
            const float v = Xs[j * XLD + i] * s;
            const T h = (T)v;
            const int64_t o = (int64_t)j * dm.ldw + i;
            Oh[o] = h;
            if (x0_split) {
                if constexpr (X8) Ol[o] = (T)__builtin_amdgcn_cvt_f32_fp8((int)e4m3((v - (float)h) * ls), 0);
                else Ol[o] = (T)((v - (float)h) * ls);
            }
        }
    }
    __syncthreads();

    SmCtx c;
    for (int q = 0; q < 4; ++q) {
        c.hi[q] = dm.hi[q];
        c.lo[q] = dm.lo[q];
    }
    c.ld = dm.ldw;
    c.n = n;
    c.Xs = Xs;
    c.io = io;
    c.lam = (float)lam_used;
    c.nonfinite = nonfinite;
    // ---- filter stages (slot 0 holds X0; slots 1..3 rotate: A, B, X')
    int slot_e[4] = {g.ex[0], 0, 0, 0};
    int cur = 0;
    bool cur_split = (g.split_mask & 1u) != 0;
    for (int st = 0; st < g.T; ++st) {
        const bool sp = (g.split_mask >> st) & 1u;
        const bool next_split = st + 1 < g.T ? ((g.split_mask >> (st + 1)) & 1u) != 0 : g.split_final != 0;
        int pa = -1, pb = -1;
        for (int q = 1; q < 4; ++q)
            if (q != cur) { if (pa < 0) pa = q; else if (pb < 0) pb = q; }
        const bool xs = sp && cur_split;
        const int st_epi = sp ? EPI_STORE_SPLIT : EPI_STORE;
        // A = X X
        sm_product_rt<T, X8>(c, xs, st_epi, cur, cur, -1, false, 0.f, 1.f, pa, slot_e[cur], slot_e[cur], 0, g.ea[st]);
        slot_e[pa] = g.ea[st];
        // B = b A + c A A
        sm_product_rt<T, X8>(c, sp, st_epi, pa, pa, pa, sp, g.b[st], g.c[st], pb, slot_e[pa], slot_e[pa], slot_e[pa],
                             g.eb[st]);
        slot_e[pb] = g.eb[st];
        // X' = a X + X B (operands split together: X is stored split for a split stage)
        sm_product_rt<T, X8>(c, xs, next_split ? EPI_STORE_SPLIT : EPI_STORE, cur, pb, cur, cur_split, g.a[st], 1.f,
                             pa, slot_e[cur], slot_e[pb], slot_e[cur], g.ex[st + 1]);
        slot_e[pa] = g.ex[st + 1];
        cur = pa;
        cur_split = next_split;
    }
    // ---- out = (X + lam X0 X_T) / 2
    sm_product_rt<T, X8>(c, g.split_final != 0, EPI_FINAL, 0, cur, -1, false, 0.f, 1.f, 0, slot_e[0], slot_e[cur], 0,
                         0);
}

}  // namespace

hipError_t small_proj_launch(const SmallArgs &a, int dtype, int count, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    if (a.steps < 1 || a.steps > kMaxLanczos || a.T < 0 || a.T > 16) return hipErrorInvalidValue;
    const dim3 grid((unsigned)count), blk(256);
    switch (dtype) {
        case DT_F16: hipLaunchKernelGGL((small_proj_kernel<f16, false>), grid, blk, 0, s, a); break;
        case DT_BF16: hipLaunchKernelGGL((small_proj_kernel<bf16, false>), grid, blk, 0, s, a); break;
        case DT_F16X8: hipLaunchKernelGGL((small_proj_kernel<f16, true>), grid, blk, 0, s, a); break;
        case DT_BF16X8: hipLaunchKernelGGL((small_proj_kernel<bf16, true>), grid, blk, 0, s, a); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace psd

// Bandwidth-bound kernels of the projection: the FP64 Lanczos run that yields
// the spectral bound, and the rescale-and-cast of X into the work precision.
//
//  * Lanczos on X^2 (Section 3.4; Algorithm 2, first two steps): 20 steps of
//    w = X (X v) in FP64 with full reorthogonalisation (two classical
//    Gram-Schmidt passes), the largest Ritz pair (sigma, q) of the tridiagonal,
//    and the bound lam = sqrt(sigma + ||X (X q) - sigma q||) of Theorem 2. The
//    matvecs read only the upper triangle of the caller's FP32 X; the first
//    one also yields the column norms (||X||_F and the lower bound
//    max_j ||X e_j|| that guards the heuristic bound).
//  * mirror_cast: X0 = X / lam from the upper triangle in 64 x 64 tiles, full
//    symmetric, rounded to the work precision (optionally a hi + lo pair),
//    zero-padded to n_p (Algorithm 2, rescale step).
// Every kernel takes the batch's descriptor table and a work list mapping
// each workgroup to (matrix, local block); a single projection is a batch of
// one. All reductions are fixed-order (no floating-point atomics), so results
// are bitwise reproducible and independent of what else is in the batch.
#include <math.h>

#include "aux_kernels.hpp"
#include "common.hpp"
#include "lanczos_dev.hpp"

namespace psd {

constexpr int kRows = 256;  // rows per block in the vector kernels
constexpr int kTB = 128;    // tile edge of the symmetric matvec

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Block reduction of NV doubles per thread (thread 0 holds the result).
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
// (Unrolled so that the loads of several partials are in flight at once; the
// additions stay in order.)
__device__ __forceinline__ double sum_partials(const double *part, int nb, int stride, int k) {
    double s = 0.0;
#pragma unroll 8
    for (int b = 0; b < nb; ++b) s += part[(int64_t)b * stride + k];
    return s;
}

// ---------------------------------------------------------------------------
// rescale / cast
// ---------------------------------------------------------------------------
template <typename T> __device__ __forceinline__ T cvt(float v) { return (T)v; }

// Upper-triangle tile index -> (I, J), column by column: t = J (J + 1) / 2 + I.
__device__ __forceinline__ void tile_of(int t, int &I, int &J) {
    int j = (int)((sqrtf(8.0f * (float)t + 1.0f) - 1.0f) * 0.5f);
    while ((j + 1) * (j + 2) / 2 <= t) ++j;
    while (j * (j + 1) / 2 > t) --j;
    J = j;
    I = t - j * (j + 1) / 2;
}

// Slot 0 of matrix m <- X / lam (64 x 64 tile pair (bi <= bj) of the padded
// n_p x n_p matrix, transposed through LDS for the mirrored half).
// X8: the split part is the FP8 pair's lo codes of X0 (code exponent e8)
// instead of an FP16 lo half.
template <typename T, bool SPLIT, bool X8 = false>
__global__ __launch_bounds__(256) void cast_kernel(const MatDesc *D, const WorkItem *W, const IoArg *io_tab,
                                                   IoArg io0, float lo_scale, int e8) {
    __shared__ float tile[64][65];
    const WorkItem wi = W[blockIdx.x];
    const MatDesc &d = D[wi.x];
    const IoArg io = io_of(io_tab, io0, wi.x);
    int bi, bj;
    tile_of((int)wi.y, bi, bj);
    const int64_t i0 = (int64_t)bi * 64, j0 = (int64_t)bj * 64, n = d.n, ldo = d.ldw;
    const float s = (float)d.scal->inv_lam;
    T *Ohi = (T *)d.hi[0];
    T *Olo = (T *)d.lo[0];
    uint8_t *Ox = (uint8_t *)d.lo[0];
    const float ls = X8 ? __builtin_ldexpf(1.0f, PairShift<T>::v + e8) : 0.0f;
    auto put = [&](int64_t i, int64_t j, float v) {
        const T hi = cvt<T>(v);
        Ohi[j * ldo + i] = hi;
        if constexpr (SPLIT && X8) {
            Ox[lo8_index(i, j, ldo)] = e4m3((v - (float)hi) * ls);
        } else if constexpr (SPLIT) {
            Olo[j * ldo + i] = cvt<T>((v - (float)hi) * lo_scale);
        }
    };
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;  // 64 x 4
    for (int c = ty; c < 64; c += 4) {
        const int64_t i = i0 + tx, j = j0 + c;
        float v = 0.0f;
        if (i < n && j < n && i <= j) v = io.X[j * io.ld + i];
        tile[tx][c] = v;
    }
    __syncthreads();
    if (bi == bj) {  // complete the diagonal tile from its upper half
        for (int c = ty; c < 64; c += 4)
            if (tx > c) tile[tx][c] = tile[c][tx];
        __syncthreads();
    }
    for (int c = ty; c < 64; c += 4) put(i0 + tx, j0 + c, tile[tx][c] * s);
    if (bi == bj) return;
    for (int c = ty; c < 64; c += 4) put(j0 + tx, i0 + c, tile[c][tx] * s);
}

// ---------------------------------------------------------------------------
// Lanczos
// ---------------------------------------------------------------------------
// Input vector of a symmetric matvec.
enum SymvSrc { SRC_V = 0, SRC_U = 1, SRC_W = 2, SRC_QHAT = 3 };
// Output vector of the reduction.
enum SymvDst { DST_U = 0, DST_W = 1, DST_W2 = 2 };

// Symmetric matvec from the upper triangle. The triangle is cut into
// kTB x kTB tiles (I <= J, t = J (J + 1) / 2 + I). Tile (I, J) reads its upper
// part once and produces
//   d[t][c] = sum_{i in I} X(i, j0 + c) v_i           (column dots)
//   a[t][r] = sum_{j in J} X(i0 + r, j) v_j           (row sums, i < j only)
// and y_k = sum_{I <= K} d[tile(I, K)][k] + sum_{J >= K} a[tile(K, J)][k],
// summed in that fixed order by symv_reduce_kernel. With NORMS the same is
// done for X(i, j)^2 and v = 1, which yields the full column norms.
//
// The kernel is bound by reading the triangle: every thread issues all 16 of
// its 16-byte loads (a quarter column of 4 rows x 16 columns) before any
// arithmetic, so a workgroup keeps the whole 64 KB tile in flight. A
// half-wave covers one 512-byte column segment per load. Row sums reduce the
// 8 column groups through LDS; column dots reduce the 32 row quads through
// LDS, both in a fixed order (NORMS: the squares go through the same LDS
// after the values, so the kernel keeps three workgroups per CU).
template <bool NORMS>
__global__ __launch_bounds__(256) void symv_tile_kernel(const MatDesc *D, const WorkItem *W, const IoArg *io_tab,
                                                        IoArg io0, int src, int jstep, int stop_on_flag) {
    constexpr int NQ = kTB / 4;         // row quads per column (32)
    constexpr int NG = 256 / NQ;        // column groups (8)
    constexpr int NL = kTB / NG;        // columns per thread (16)
    const WorkItem wi = W[blockIdx.x];
    const MatDesc &dm = D[wi.x];
    if (stop_on_flag && dm.scal->stop) return;
    const IoArg io = io_of(io_tab, io0, wi.x);
    const int64_t n = dm.n;
    const int t = (int)wi.y;
    int I, J;
    tile_of(t, I, J);
    const int64_t i0 = (int64_t)I * kTB, j0 = (int64_t)J * kTB;
    const bool diag = (I == J);
    const double *v = src == SRC_V ? dm.V + (int64_t)jstep * n : (src == SRC_W ? dm.w : dm.u);
    const double sc = src == SRC_QHAT ? dm.scal->qnorm_inv : 1.0;
    __shared__ double vI[kTB], vJ[kTB];
    __shared__ double cpart[kTB][NQ + 1];  // column dots per row quad (padded)
    __shared__ double rpart[NG][kTB];      // row sums per column group
    const int tid = threadIdx.x;
    const int q = tid % NQ, grp = tid / NQ;  // row quad, column group
    const int64_t ir = i0 + 4 * q;           // first row of the quad

    // loads first: column grp + NG k of the tile, rows ir .. ir + 3
    f32x4 x[NL];
    const bool vec = ((reinterpret_cast<uintptr_t>(io.X) & 15) == 0) && ((io.ld & 3) == 0);
#pragma unroll
    for (int k = 0; k < NL; ++k) {
        const int64_t j = j0 + grp + NG * k;
        const float *col = io.X + j * io.ld;
        if (j < n && vec && ir + 3 < n && (!diag || ir + 3 <= j)) {
            x[k] = *(const f32x4 *)(col + ir);
        } else {
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int64_t i = ir + e;
                x[k][e] = (j < n && i < n && (!diag || i <= j)) ? col[i] : 0.0f;
            }
        }
    }
    if (tid < kTB) {
        const int64_t i = i0 + tid;
        vI[tid] = i < n ? v[i] * sc : 0.0;
    } else {
        const int64_t j = j0 + tid - kTB;
        vJ[tid - kTB] = j < n ? v[j] * sc : 0.0;
    }
    __syncthreads();
    double va[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) va[e] = vI[4 * q + e];
    double ra[4] = {0.0, 0.0, 0.0, 0.0}, rq[4] = {0.0, 0.0, 0.0, 0.0};
    double sq[NORMS ? NL : 1];
#pragma unroll
    for (int k = 0; k < NL; ++k) {
        const int c = grp + NG * k;
        const int64_t j = j0 + c;
        const double vj = vJ[c];
        double dot = 0.0, sqk = 0.0;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const double xe = (double)x[k][e];
            dot += xe * va[e];
            // row sums: strictly upper entries only (the diagonal is in the dot)
            const bool up = !diag || ir + e < j;
            ra[e] += up ? xe * vj : 0.0;
            if constexpr (NORMS) {
                sqk += xe * xe;
                rq[e] += up ? xe * xe : 0.0;
            }
        }
        cpart[c][q] = dot;
        if constexpr (NORMS) sq[k] = sqk;
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) rpart[grp][4 * q + e] = ra[e];
    __syncthreads();
    const int64_t base = (int64_t)t * kTB;
    // column sums of the row-quad partials (threads 0..127) and row sums of
    // the column-group partials (threads 128..255), in a fixed order
    auto reduce_out = [&](double *dcol, double *arow) {
        if (tid < kTB) {
            double d = 0.0;
            for (int k = 0; k < NQ; ++k) d += cpart[tid][k];
            dcol[base + tid] = d;
        } else {
            const int r = tid - kTB;
            double a = 0.0;
#pragma unroll
            for (int g = 0; g < NG; ++g) a += rpart[g][r];
            arow[base + r] = a;
        }
    };
    reduce_out(dm.sd, dm.sa);
    if constexpr (NORMS) {
        __syncthreads();
#pragma unroll
        for (int k = 0; k < NL; ++k) cpart[grp + NG * k][q] = sq[k];
#pragma unroll
        for (int e = 0; e < 4; ++e) rpart[grp][4 * q + e] = rq[e];
        __syncthreads();
        reduce_out(dm.sd2, dm.sa2);
    }
}

// The small vector kernels of a Lanczos step run 4 groups of kRows threads
// per block of kRows rows, so that four times as many loads are in flight.
constexpr int kGroups = 4;
constexpr int kVecThreads = kGroups * kRows;
constexpr int kColsPerGroup = kMaxLanczos / kGroups;  // Lanczos columns c = kGroups m + g

// Per-group block sums of NV doubles per thread over the group's kRows rows:
// each wave sums its 64 rows, then the group's waves are added in order
// (the same order for every group, and the order of block_reduce). Row sums
// of column v of group g land in out[g][v] (LDS, valid after the call).
template <int NV>
__device__ __forceinline__ void group_reduce(double (&v)[NV], double *sh /* [16][NV] */,
                                             double (*out)[NV] /* [kGroups][NV] */) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < NV; ++k) v[k] = wave_sum(v[k]);
    if (lane == 0)
#pragma unroll
        for (int k = 0; k < NV; ++k) sh[wave * NV + k] = v[k];
    __syncthreads();
    if (threadIdx.x < kGroups * NV) {
        const int g = threadIdx.x / NV, k = threadIdx.x % NV;
        const double *w = sh + 4 * g * NV + k;
        out[g][k] = w[0] + w[NV] + w[2 * NV] + w[3 * NV];
    }
    __syncthreads();
}

// y_k from the symv tile partials. Its T + 1 terms (column dots of tiles
// I = 0..K, then row sums of tiles J = K..T-1) are cut into four consecutive
// runs, one per thread group, each summed in order; the four run sums are
// added in group order. NORMS: also colsq_k. ORTH0: also the first
// Gram-Schmidt partials pa[block][c] = sum over this block's rows of
// V[i, c] y_i, c <= jstep.
template <bool NORMS, bool ORTH0>
__global__ __launch_bounds__(kVecThreads) void symv_reduce_kernel(const MatDesc *D, const WorkItem *W, int dst,
                                                                  int jstep, int stop_on_flag) {
    const WorkItem wi = W[blockIdx.x];
    const MatDesc &dm = D[wi.x];
    if (stop_on_flag && dm.scal->stop) return;
    const int64_t n = dm.n;
    const int b = (int)wi.y;
    const int r = threadIdx.x % kRows, g = threadIdx.x / kRows;
    const int64_t k = (int64_t)b * kRows + r;
    const int T = (int)((n + kTB - 1) / kTB);
    double *y = dst == DST_U ? dm.u : (dst == DST_W ? dm.w : dm.w2);
    __shared__ double ry[kGroups][kRows], rc[NORMS ? kGroups : 1][kRows];
    __shared__ double yb[kRows];
    double ys = 0.0, cs = 0.0;
    if (k < n) {
        const int K = (int)(k / kTB), kk = (int)(k % kTB);
        const int64_t base = (int64_t)K * (K + 1) / 2;
        const int nt = T + 1, q = (nt + kGroups - 1) / kGroups;
        const int t0 = g * q < nt ? g * q : nt, t1 = t0 + q < nt ? t0 + q : nt;
        // terms t <= K: column dots of tile (t, K); t > K: row sums of tile (K, t - 1)
        const int d1 = t1 < K + 1 ? t1 : K + 1;
#pragma unroll 8
        for (int t = t0; t < d1; ++t) {
            ys += dm.sd[(base + t) * kTB + kk];
            if constexpr (NORMS) cs += dm.sd2[(base + t) * kTB + kk];
        }
#pragma unroll 8
        for (int t = (t0 > K + 1 ? t0 : K + 1); t < t1; ++t) {
            const int64_t tl = (int64_t)(t - 1) * t / 2 + K;
            ys += dm.sa[tl * kTB + kk];
            if constexpr (NORMS) cs += dm.sa2[tl * kTB + kk];
        }
    }
    ry[g][r] = ys;
    if constexpr (NORMS) rc[g][r] = cs;
    __syncthreads();
    if (g == 0) {
        const double yk = ((ry[0][r] + ry[1][r]) + ry[2][r]) + ry[3][r];
        if (k < n) {
            y[k] = yk;
            if (dst == DST_U && dm.U) dm.U[(int64_t)jstep * n + k] = yk;  // X v_j, kept for deflation
            if constexpr (NORMS) dm.colsq[k] = ((rc[0][r] + rc[1][r]) + rc[2][r]) + rc[3][r];
        }
        yb[r] = k < n ? yk : 0.0;
    }
    if constexpr (ORTH0) {
        __shared__ double sh[16 * kColsPerGroup];
        __shared__ double hs[kGroups][kColsPerGroup];
        __syncthreads();
        double h[kColsPerGroup];
#pragma unroll
        for (int m = 0; m < kColsPerGroup; ++m) {
            const int c = kGroups * m + g;
            h[m] = (c <= jstep && k < n) ? dm.V[(int64_t)c * n + k] * yb[r] : 0.0;
        }
        group_reduce<kColsPerGroup>(h, sh, hs);
        if (threadIdx.x <= jstep) {
            const int c = threadIdx.x;
            dm.pa[(int64_t)b * kMaxLanczos + c] = hs[c % kGroups][c / kGroups];
        }
    }
}

__global__ void scal_init_kernel(const MatDesc *D) {
    if (threadIdx.x == 0 && !D[blockIdx.x].fused) {
        Scalars z = {};
        *D[blockIdx.x].scal = z;
    }
}

// Start vector: V[:, 0] = v / ||v||. Pass 0 writes v and the partial norms
// (pa), pass 1 normalises.
__global__ __launch_bounds__(256) void lz_start_kernel(const MatDesc *D, const WorkItem *W, int pass, uint64_t seed) {
    const WorkItem wi = W[blockIdx.x];
    const MatDesc &dm = D[wi.x];
    const int b = (int)wi.y;
    const int64_t i = (int64_t)b * kRows + threadIdx.x, n = dm.n;
    __shared__ double sh[4];
    if (pass == 0) {
        double x[1] = {0.0};
        if (i < n) {
            const double e = start_entry((uint64_t)i, seed);
            dm.V[i] = e;
            x[0] = e * e;
        }
        block_reduce<1>(x, sh);
        if (threadIdx.x == 0) dm.pa[(int64_t)b * kMaxLanczos] = x[0];
    } else {
        const double nrm = sqrt(sum_partials(dm.pa, dm.nbv, kMaxLanczos, 0));
        if (i < n) dm.V[i] = dm.V[i] / nrm;
    }
}

// Orthogonalisation pass of step j over the rows of this block.
//  pass 1: h = sum(pa); alpha_j = h_j; w -= V h; pb <- V^T w (second GS
//          pass), pc <- ||w||^2
//  pass 2: h = sum(pb); w -= V h; beta_j = ||w|| as sqrt(sum(pc) - |h|^2)
//          (w changes by V h with V orthonormal, so its squared norm drops by
//          |h|^2; after the first pass h is at rounding level, so the two
//          agree to rounding); stop if beta_j <= 1e-13 max|alpha| or j is the
//          last step, else V[:, j+1] = w / beta_j
// (the first pass's partials come with the reduction that formed w). Thread
// group g holds the columns c = 4 m + g of V for its row: (V h)_i is the sum
// of the four groups' sums, added in group order.
__global__ __launch_bounds__(kVecThreads) void lz_orth_kernel(const MatDesc *D, const WorkItem *W, int j, int pass,
                                                              int steps) {
    const WorkItem wi = W[blockIdx.x];
    const MatDesc &dm = D[wi.x];
    Scalars *scal = dm.scal;
    if (scal->stop) return;
    const int b = (int)wi.y;
    const int r = threadIdx.x % kRows, g = threadIdx.x / kRows;
    const int64_t i = (int64_t)b * kRows + r, n = dm.n;
    const double *part_in = pass == 1 ? dm.pa : dm.pb;
    __shared__ double hsh[kMaxLanczos];
    __shared__ double rs[kGroups][kRows];
    __shared__ double wb[kRows];
    __shared__ double sh[16 * kColsPerGroup];
    __shared__ double hs[kGroups][kColsPerGroup];
    if (threadIdx.x <= j) hsh[threadIdx.x] = sum_partials(part_in, dm.nbv, kMaxLanczos, threadIdx.x);
    double v[kColsPerGroup];
#pragma unroll
    for (int m = 0; m < kColsPerGroup; ++m) {
        const int c = kGroups * m + g;
        v[m] = (c <= j && i < n) ? dm.V[(int64_t)c * n + i] : 0.0;
    }
    __syncthreads();
    if (pass == 1 && b == 0 && threadIdx.x == 0) {
        scal->alpha[j] = hsh[j];
        scal->amax = fmax(scal->amax, fabs(hsh[j]));
    }
    double s = 0.0;
#pragma unroll
    for (int m = 0; m < kColsPerGroup; ++m) {
        const int c = kGroups * m + g;
        if (c <= j) s += v[m] * hsh[c];
    }
    rs[g][r] = s;
    __syncthreads();
    if (g == 0) {
        double w_i = 0.0;
        if (i < n) {
            w_i = dm.w[i] - (((rs[0][r] + rs[1][r]) + rs[2][r]) + rs[3][r]);
            dm.w[i] = w_i;
        }
        wb[r] = w_i;
    }
    __syncthreads();
    if (pass == 1) {
        double h[kColsPerGroup];
#pragma unroll
        for (int m = 0; m < kColsPerGroup; ++m) h[m] = v[m] * wb[r];
        group_reduce<kColsPerGroup>(h, sh, hs);
        if (threadIdx.x <= j) dm.pb[(int64_t)b * kMaxLanczos + threadIdx.x] = hs[threadIdx.x % kGroups][threadIdx.x / kGroups];
        double x[1] = {g == 0 ? wb[r] * wb[r] : 0.0};
        group_reduce<1>(x, sh, (double(*)[1])hs);
        if (threadIdx.x == 0) dm.pc[b] = hs[0][0];
        return;
    }
    // pass 2: beta_j from the norm and the second pass's coefficients, the
    // same in every block (fixed-order sums of the same partials)
    double hh = 0.0;
    for (int c = 0; c <= j; ++c) hh += hsh[c] * hsh[c];
    const double beta = sqrt(fmax(sum_partials(dm.pc, dm.nbv, 1, 0) - hh, 0.0));
    const bool stop = (j == steps - 1) || !(beta > 1e-13 * scal->amax);
    if (g == 0 && !stop && i < n) dm.V[(int64_t)(j + 1) * n + i] = wb[r] / beta;
    // Every block has read scal->stop/amax above; the updates below are seen
    // only by later kernels on the stream (a block that starts after them
    // and sees stop set has nothing left to do).
    __syncthreads();
    if (b == 0 && threadIdx.x == 0) {
        scal->k = j + 1;
        scal->beta_last = beta;
        if (!stop) scal->beta[j] = beta;
        if (stop) scal->stop = 1;
    }
}

// Largest Ritz pair of the matrix's Lanczos run into its Scalars.
template <int KM>
__global__ __launch_bounds__(64) void lz_ritz_kernel(const MatDesc *D) {
    if (D[blockIdx.x].fused) return;
    Scalars *scal = D[blockIdx.x].scal;
    const int lane = threadIdx.x;
    const int k = scal->k;
    __shared__ double al[kMaxLanczos], be[kMaxLanczos];
    __shared__ double lo_hi[2];
    if (lane < kMaxLanczos) {
        al[lane] = lane < k ? scal->alpha[lane] : 0.0;
        be[lane] = lane < k - 1 ? scal->beta[lane] : 0.0;
    }
    __syncthreads();
    ritz_largest<KM>(al, be, k, lo_hi, &scal->sigma, scal->s);
}

// q = V[:, 0..k) s (into u); pa <- ||q||^2
__global__ __launch_bounds__(256) void lz_q_kernel(const MatDesc *D, const WorkItem *W) {
    const WorkItem wi = W[blockIdx.x];
    const MatDesc &dm = D[wi.x];
    const int b = (int)wi.y;
    const int64_t i = (int64_t)b * kRows + threadIdx.x, n = dm.n;
    __shared__ double red[4];
    double qi = 0.0;
    if (i < n) {
        for (int k = 0; k < dm.scal->k; ++k) qi += dm.V[(int64_t)k * n + i] * dm.scal->s[k];
        dm.u[i] = qi;
    }
    double x[1] = {qi * qi};
    block_reduce<1>(x, red);
    if (threadIdx.x == 0) dm.pa[(int64_t)b * kMaxLanczos] = x[0];
}

__global__ void lz_qnorm_kernel(const MatDesc *D) {
    if (threadIdx.x != 0) return;
    const MatDesc &dm = D[blockIdx.x];
    if (dm.fused) return;
    const double nrm = sqrt(sum_partials(dm.pa, dm.nbv, kMaxLanczos, 0));
    dm.scal->qnorm_inv = nrm > 0.0 ? 1.0 / nrm : 0.0;
}

// pa <- ||w2 - sigma q_hat||^2 with q_hat = u * qnorm_inv
__global__ __launch_bounds__(256) void lz_resid_kernel(const MatDesc *D, const WorkItem *W) {
    const WorkItem wi = W[blockIdx.x];
    const MatDesc &dm = D[wi.x];
    const int b = (int)wi.y;
    const int64_t i = (int64_t)b * kRows + threadIdx.x, n = dm.n;
    __shared__ double red[4];
    double r = 0.0;
    if (i < n) r = dm.w2[i] - dm.scal->sigma * (dm.u[i] * dm.scal->qnorm_inv);
    double x[1] = {r * r};
    block_reduce<1>(x, red);
    if (threadIdx.x == 0) dm.pa[(int64_t)b * kMaxLanczos] = x[0];
}

// Frobenius norm and column-norm maximum from colsq, residual from pa, then
// lam = sqrt(sigma + r) (Theorem 2), guarded: if lam is not at least the
// largest column norm (a lower bound on ||X||_2) the Frobenius norm is used;
// lam is capped by the Frobenius norm (also an upper bound). One block per
// matrix. A positive override replaces the bound (the norms are kept).
__global__ __launch_bounds__(256) void lz_bound_kernel(const MatDesc *D, int force_fallback, double lam_override) {
    const MatDesc &dm = D[blockIdx.x];
    if (dm.fused) return;
    Scalars *scal = dm.scal;
    const int64_t n = dm.n;
    __shared__ double sh_sum[256], sh_max[256];
    double s = 0.0, m = 0.0;
    int bad = 0;
    // fixed per-thread stride, then a fixed-order tree: deterministic
    for (int64_t i = threadIdx.x; i < n; i += 256) {
        const double c = dm.colsq[i];
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
    const double r = sqrt(sum_partials(dm.pa, dm.nbv, kMaxLanczos, 0));
    scal->resid = r;
    const double lz = sqrt(fmax(scal->sigma + r, 0.0));
    scal->lanczos_lam = lz;
    const double fro = sqrt(fro2), colmax = sqrt(colmax2);
    double lam = lz;
    int fb = 0;
    if (force_fallback) lam = 0.5 * lz;  // test hook: an invalid bound
    if (!(lam >= colmax)) { lam = fro; fb = 1; }
    if (lam > fro) lam = fro;
    if (lam_override > 0.0) { lam = lam_override; fb = 0; }
    scal->fallback = fb;
    scal->lam = nonfinite ? 0.0 : lam;
    scal->inv_lam = (nonfinite || !(lam > 0.0)) ? 0.0 : 1.0 / lam;
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
hipError_t spectral_bound(const BatchLaunch &B, int steps, uint64_t seed, int force_fallback, double lam_override,
                          hipStream_t s) {
    if (steps < 1 || steps > kMaxLanczos) return hipErrorInvalidValue;
    if (B.count == 0) return hipSuccess;
    const MatDesc *D = B.desc;
    const unsigned nv = (unsigned)B.n_vec, nt = (unsigned)B.n_symv, M = (unsigned)B.count;
    const WorkItem *Wv = B.w_vec, *Wt = B.w_symv;
    auto symv = [&](int src, int jstep, int dst, bool norms, bool orth0, int stop_flag) {
        if (norms)
            hipLaunchKernelGGL(symv_tile_kernel<true>, dim3(nt), dim3(256), 0, s, D, Wt, B.io_tab, B.io0, src, jstep,
                               stop_flag);
        else
            hipLaunchKernelGGL(symv_tile_kernel<false>, dim3(nt), dim3(256), 0, s, D, Wt, B.io_tab, B.io0, src, jstep,
                               stop_flag);
        if (norms)
            hipLaunchKernelGGL((symv_reduce_kernel<true, false>), dim3(nv), dim3(kVecThreads), 0, s, D, Wv, dst, jstep,
                               stop_flag);
        else if (orth0)
            hipLaunchKernelGGL((symv_reduce_kernel<false, true>), dim3(nv), dim3(kVecThreads), 0, s, D, Wv, dst, jstep,
                               stop_flag);
        else
            hipLaunchKernelGGL((symv_reduce_kernel<false, false>), dim3(nv), dim3(kVecThreads), 0, s, D, Wv, dst, jstep,
                               stop_flag);
    };
    hipLaunchKernelGGL(scal_init_kernel, dim3(M), dim3(64), 0, s, D);
    hipLaunchKernelGGL(lz_start_kernel, dim3(nv), dim3(256), 0, s, D, Wv, 0, seed);
    hipLaunchKernelGGL(lz_start_kernel, dim3(nv), dim3(256), 0, s, D, Wv, 1, seed);
    for (int j = 0; j < steps; ++j) {
        symv(SRC_V, j, DST_U, j == 0, false, 1);  // u = X v_j (first step: + column norms)
        symv(SRC_U, j, DST_W, false, true, 1);    // w = X u, pa = V^T w
        hipLaunchKernelGGL(lz_orth_kernel, dim3(nv), dim3(kVecThreads), 0, s, D, Wv, j, 1, steps);
        hipLaunchKernelGGL(lz_orth_kernel, dim3(nv), dim3(kVecThreads), 0, s, D, Wv, j, 2, steps);
    }
    if (steps <= 20)
        hipLaunchKernelGGL(lz_ritz_kernel<20>, dim3(M), dim3(64), 0, s, D);
    else
        hipLaunchKernelGGL(lz_ritz_kernel<kMaxLanczos>, dim3(M), dim3(64), 0, s, D);
    hipLaunchKernelGGL(lz_q_kernel, dim3(nv), dim3(256), 0, s, D, Wv);
    hipLaunchKernelGGL(lz_qnorm_kernel, dim3(M), dim3(64), 0, s, D);
    symv(SRC_QHAT, 0, DST_W, false, false, 0);  // w = X q_hat
    symv(SRC_W, 0, DST_W2, false, false, 0);    // w2 = X^2 q_hat
    hipLaunchKernelGGL(lz_resid_kernel, dim3(nv), dim3(256), 0, s, D, Wv);
    hipLaunchKernelGGL(lz_bound_kernel, dim3(M), dim3(256), 0, s, D, force_fallback, lam_override);
    return hipGetLastError();
}

hipError_t cast_x0(const BatchLaunch &B, int dtype, bool split, int e8, hipStream_t s) {
    if (B.count == 0 || B.n_cast == 0) return hipSuccess;
    const dim3 g((unsigned)B.n_cast), blk(256);
    switch (dtype) {
        case 0:
            hipLaunchKernelGGL((cast_kernel<float, false>), g, blk, 0, s, B.desc, B.w_cast, B.io_tab, B.io0, 1.0f, 0);
            break;
        case 1:
            if (split)
                hipLaunchKernelGGL((cast_kernel<f16, true>), g, blk, 0, s, B.desc, B.w_cast, B.io_tab, B.io0, 2048.0f, 0);
            else
                hipLaunchKernelGGL((cast_kernel<f16, false>), g, blk, 0, s, B.desc, B.w_cast, B.io_tab, B.io0, 1.0f, 0);
            break;
        case 2:
            if (split)
                hipLaunchKernelGGL((cast_kernel<bf16, true>), g, blk, 0, s, B.desc, B.w_cast, B.io_tab, B.io0, 1.0f, 0);
            else
                hipLaunchKernelGGL((cast_kernel<bf16, false>), g, blk, 0, s, B.desc, B.w_cast, B.io_tab, B.io0, 1.0f, 0);
            break;
        case 3:  // FP16 with FP8 pairs
            if (split)
                hipLaunchKernelGGL((cast_kernel<f16, true, true>), g, blk, 0, s, B.desc, B.w_cast, B.io_tab, B.io0, 0.0f,
                                   e8);
            else
                hipLaunchKernelGGL((cast_kernel<f16, false>), g, blk, 0, s, B.desc, B.w_cast, B.io_tab, B.io0, 1.0f, 0);
            break;
        case 4:  // BF16 with FP8 pairs
            if (split)
                hipLaunchKernelGGL((cast_kernel<bf16, true, true>), g, blk, 0, s, B.desc, B.w_cast, B.io_tab, B.io0,
                                   0.0f, e8);
            else
                hipLaunchKernelGGL((cast_kernel<bf16, false>), g, blk, 0, s, B.desc, B.w_cast, B.io_tab, B.io0, 1.0f, 0);
            break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Adaptive depth: the relative change ||X_new - X_old||_F / ||X_old||_F of a
// stage, over the 64 x 64 tile pairs of the cast work list (off-diagonal
// tiles count twice, diagonal tiles their upper half twice and the diagonal
// once), per-tile sums in a fixed order, then per matrix in list order.
template <typename T>
__global__ __launch_bounds__(256) void stage_delta_kernel(const MatDesc *D, const WorkItem *W, int sn, int so,
                                                          double *part) {
    const WorkItem wi = W[blockIdx.x];
    const MatDesc &dm = D[wi.x];
    double dd = 0.0, nn = 0.0;
    if (!dm.scal->done) {
        int bi, bj;
        tile_of((int)wi.y, bi, bj);
        const int64_t i0 = (int64_t)bi * 64, j0 = (int64_t)bj * 64, n = dm.n, ld = dm.ldw;
        const T *Xn = (const T *)dm.hi[sn];
        const T *Xo = (const T *)dm.hi[so];
        const int64_t i = i0 + (threadIdx.x & 63);
        for (int c = threadIdx.x >> 6; c < 64; c += 4) {
            const int64_t j = j0 + c;
            if (i >= n || j >= n || (bi == bj && i > j)) continue;
            const double w = (bi == bj && i == j) ? 1.0 : 2.0;
            const double a = (double)(float)Xn[j * ld + i], b = (double)(float)Xo[j * ld + i];
            dd += w * (a - b) * (a - b);
            nn += w * b * b;
        }
    }
    __shared__ double sh[8];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        dd += __shfl_xor(dd, off, 64);
        nn += __shfl_xor(nn, off, 64);
    }
    if (lane == 0) {
        sh[wave] = dd;
        sh[4 + wave] = nn;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        part[2 * (size_t)blockIdx.x] = ((sh[0] + sh[1]) + sh[2]) + sh[3];
        part[2 * (size_t)blockIdx.x + 1] = ((sh[4] + sh[5]) + sh[6]) + sh[7];
    }
}

// One thread per matrix: unless converged earlier, the latest iterate is in
// slot sn after `stage` stages; may_stop: converged once the change <= tol.
__global__ void stage_final_kernel(const MatDesc *D, const double *part, int sn, int stage, int may_stop, double tol) {
    if (threadIdx.x != 0) return;
    const MatDesc &dm = D[blockIdx.x];
    Scalars *sc = dm.scal;
    if (sc->done) return;
    sc->cur_slot = sn;
    sc->stages_run = stage;
    if (!may_stop) return;
    double dd = 0.0, nn = 0.0;
    for (int k = 0; k < dm.cast_count; ++k) {
        dd += part[2 * (size_t)(dm.cast_first + k)];
        nn += part[2 * (size_t)(dm.cast_first + k) + 1];
    }
    const double d = nn > 0.0 ? sqrt(dd / nn) : 0.0;
    sc->delta = d;
    if (d <= tol) sc->done = 1;
}

hipError_t stage_check(const BatchLaunch &B, int dtype, int sn, int so, int stage, bool may_stop, double tol,
                       double *part, hipStream_t s) {
    if (B.count == 0) return hipSuccess;
    if (may_stop && B.n_cast) {
        const dim3 g((unsigned)B.n_cast), blk(256);
        switch (dtype) {
            case 0: hipLaunchKernelGGL(stage_delta_kernel<float>, g, blk, 0, s, B.desc, B.w_cast, sn, so, part); break;
            case 1: hipLaunchKernelGGL(stage_delta_kernel<f16>, g, blk, 0, s, B.desc, B.w_cast, sn, so, part); break;
            case 2: hipLaunchKernelGGL(stage_delta_kernel<bf16>, g, blk, 0, s, B.desc, B.w_cast, sn, so, part); break;
            default: return hipErrorInvalidValue;
        }
    }
    hipLaunchKernelGGL(stage_final_kernel, dim3((unsigned)B.count), dim3(64), 0, s, B.desc, part, sn, stage,
                       may_stop ? 1 : 0, tol);
    return hipGetLastError();
}

size_t lanczos_work_doubles(int64_t n, int steps) {
    const int64_t nbv = (n + kRows - 1) / kRows;
    const int64_t tiles = symv_tile_count(n);
    return (size_t)(n * steps + 5 * n + 2 * nbv * kMaxLanczos + nbv + 4 * tiles * kTB + 64);
}

int64_t symv_tile_count(int64_t n) {
    const int64_t T = (n + kTB - 1) / kTB;
    return T * (T + 1) / 2;
}

int64_t vec_block_count(int64_t n) { return (n + kRows - 1) / kRows; }

int64_t cast_tile_count(int64_t np) {
    const int64_t T = (np + 63) / 64;
    return T * (T + 1) / 2;
}

void fill_lanczos_desc(MatDesc &d, double *lz, int64_t n, int steps) {
    const int64_t nbv = vec_block_count(n);
    const int64_t tiles = symv_tile_count(n);
    d.nbv = (int32_t)nbv;
    d.V = lz;
    d.u = d.V + n * steps;
    d.w = d.u + n;
    d.w2 = d.w + n;
    d.colsq = d.w2 + n;
    d.pa = d.colsq + n;
    d.pb = d.pa + nbv * kMaxLanczos;
    d.pc = d.pb + nbv * kMaxLanczos;
    d.sd = d.pc + nbv;
    d.sa = d.sd + tiles * kTB;
    d.sd2 = d.sa + tiles * kTB;
    d.sa2 = d.sd2 + tiles * kTB;
}

}  // namespace psd

// Deflation of dominant eigenpairs before filtering.
//
// A spectrum with a few eigenvalues far above the rest scales the rest below
// the interval the composite filter resolves; removing the dominant pairs
// first and adding their positive part back afterwards is the remedy the
// paper proposes (Section 4.1 "Results"; Section 5 "Limitations and future
// work"). The pairs come from the bound's own Lanczos run on X^2: its
// orthonormal Krylov basis V (n x k) and the products U = X V recorded by the
// first matvec of every step give H = V^T X V (k x k), whose eigenpairs
// (mu_i, s_i) are the Rayleigh-Ritz pairs of X itself in span(V), signs
// resolved. Of the kmax pairs of largest |mu|, those with
// ||X z - mu z|| <= 1e-8 |mu| ||z|| (z = V s, X z = U s) are removed:
//   X' = X - sum_i mu_i z_i z_i^T           (FP64 arithmetic, FP32 copy)
//   P  = P_filter(X') + sum_i max(mu_i, 0) z_i z_i^T.
// For exact eigenpairs P = Pi(X) up to the filter's error on X' (the z_i are
// then eigenvectors of X' with eigenvalue 0). Every reduction is in a fixed
// order; no floating-point atomics.
#include <math.h>

#include "aux_kernels.hpp"
#include "common.hpp"

namespace psd {

namespace {

constexpr int kRowsD = 256;   // rows per vector block (as the Lanczos kernels)
constexpr int kChunk = 64;    // rows staged in LDS at a time
constexpr double kDeflRtol = 1e-8;

// Partials of H = V^T U over the rows of one vector block: entry (a, c),
// a, c < k, at pH[b][a * kMaxLanczos + c], rows summed in order.
__global__ __launch_bounds__(256) void defl_h_kernel(const MatDesc *D, const WorkItem *W) {
    const WorkItem wi = W[blockIdx.x];
    const MatDesc &dm = D[wi.x];
    const int b = (int)wi.y;
    const int64_t n = dm.n;
    const int k = dm.scal->k;
    __shared__ double Vc[kChunk][kMaxLanczos + 1], Uc[kChunk][kMaxLanczos + 1];
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    const int64_t r0 = (int64_t)b * kRowsD;
    for (int c0 = 0; c0 < kRowsD; c0 += kChunk) {
        for (int e = threadIdx.x; e < kChunk * kMaxLanczos; e += 256) {
            const int rr = e % kChunk, col = e / kChunk;
            const int64_t i = r0 + c0 + rr;
            const bool ok = i < n && col < k;
            Vc[rr][col] = ok ? dm.V[(int64_t)col * n + i] : 0.0;
            Uc[rr][col] = ok ? dm.U[(int64_t)col * n + i] : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int e = threadIdx.x + 256 * q;
            const int a = e / kMaxLanczos, c = e % kMaxLanczos;
            if (a < k && c < k)
                for (int rr = 0; rr < kChunk; ++rr) acc[q] += Vc[rr][a] * Uc[rr][c];
        }
        __syncthreads();
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int e = threadIdx.x + 256 * q;
        dm.defl->pH[(int64_t)b * kMaxLanczos * kMaxLanczos + e] = acc[q];
    }
}

// One wave per matrix: H from the partials (blocks in order), symmetrised,
// eigen-decomposed by cyclic Jacobi with Rutishauser's rotation formulas
// (Golub & Van Loan, Matrix Computations, Section 8.5), lane r owning row and
// column r of H and row r of the eigenvector matrix; then the kmax pairs of
// largest |mu| (ties: lower index first) become the candidates.
__global__ __launch_bounds__(64) void defl_eig_kernel(const MatDesc *D) {
    const MatDesc &dm = D[blockIdx.x];
    DeflState *ds = dm.defl;
    const int k = dm.scal->k;
    const int lane = threadIdx.x;
    __shared__ double A[kMaxLanczos][kMaxLanczos + 1], Q[kMaxLanczos][kMaxLanczos + 1];
    __shared__ double Hs[kMaxLanczos][kMaxLanczos + 1];
    __shared__ double red[64];
    // H = sum over blocks (in order) of the partials
    for (int e = lane; e < kMaxLanczos * kMaxLanczos; e += 64) {
        const int a = e / kMaxLanczos, c = e % kMaxLanczos;
        double h = 0.0;
        if (a < k && c < k)
            for (int bb = 0; bb < dm.nbv; ++bb) h += ds->pH[(int64_t)bb * kMaxLanczos * kMaxLanczos + e];
        Hs[a][c] = h;
    }
    __syncthreads();
    for (int e = lane; e < kMaxLanczos * kMaxLanczos; e += 64) {
        const int a = e / kMaxLanczos, c = e % kMaxLanczos;
        A[a][c] = 0.5 * (Hs[a][c] + Hs[c][a]);
        Q[a][c] = a == c ? 1.0 : 0.0;
    }
    __syncthreads();
    auto wave_sum = [&](double v) {
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
        return v;
    };
    for (int sweep = 0; sweep < 30; ++sweep) {
        double off = 0.0, fro = 0.0;
        if (lane < k)
            for (int c = 0; c < k; ++c) {
                const double v = A[lane][c] * A[lane][c];
                fro += v;
                if (c != lane) off += v;
            }
        off = wave_sum(off);
        fro = wave_sum(fro);
        if (!(off > 1e-30 * fro)) break;  // converged (or not finite)
        for (int p = 0; p < k - 1; ++p)
            for (int q = p + 1; q < k; ++q) {
                const double apq = A[p][q], app = A[p][p], aqq = A[q][q];
                __syncthreads();
                if (apq != 0.0) {
                    const double th = (aqq - app) / (2.0 * apq);
                    const double t = (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(1.0 + th * th));
                    const double c = 1.0 / sqrt(1.0 + t * t), s = t * c;
                    const int r = lane;
                    if (r < k && r != p && r != q) {
                        const double arp = A[r][p], arq = A[r][q];
                        const double np = c * arp - s * arq, nq = s * arp + c * arq;
                        A[r][p] = np;
                        A[p][r] = np;
                        A[r][q] = nq;
                        A[q][r] = nq;
                    }
                    if (r < k) {
                        const double qrp = Q[r][p], qrq = Q[r][q];
                        Q[r][p] = c * qrp - s * qrq;
                        Q[r][q] = s * qrp + c * qrq;
                    }
                    if (r == 0) {
                        A[p][p] = app - t * apq;
                        A[q][q] = aqq + t * apq;
                        A[p][q] = 0.0;
                        A[q][p] = 0.0;
                    }
                }
                __syncthreads();
            }
    }
    red[lane] = lane < k ? A[lane][lane] : 0.0;
    __syncthreads();
    if (lane != 0) return;
    const int kc = ds->kmax < k ? ds->kmax : k;
    bool used[kMaxLanczos];
    for (int i = 0; i < kMaxLanczos; ++i) used[i] = false;
    for (int c = 0; c < kc; ++c) {
        int best = -1;
        for (int i = 0; i < k; ++i)
            if (!used[i] && (best < 0 || fabs(red[i]) > fabs(red[best]))) best = i;
        used[best] = true;
        ds->cmu[c] = red[best];
        for (int j = 0; j < kMaxLanczos; ++j) ds->cs[c][j] = j < k ? Q[j][best] : 0.0;
    }
    ds->ncand = kc;
    ds->count = 0;
}

// z_c = V s_c (stored, unnormalised) and X z_c = U s_c for every candidate,
// with per-block partials of ||z_c||^2 and ||X z_c - mu_c z_c||^2.
__global__ __launch_bounds__(256) void defl_z_kernel(const MatDesc *D, const WorkItem *W) {
    const WorkItem wi = W[blockIdx.x];
    const MatDesc &dm = D[wi.x];
    DeflState *ds = dm.defl;
    const int b = (int)wi.y;
    const int64_t n = dm.n, i = (int64_t)b * kRowsD + threadIdx.x;
    const int k = dm.scal->k, kc = ds->ncand;
    __shared__ double sh[4][2 * kMaxDeflate];
    double part[2 * kMaxDeflate];
#pragma unroll
    for (int c = 0; c < kMaxDeflate; ++c) {
        double z = 0.0, xz = 0.0;
        if (c < kc && i < n) {
            for (int j = 0; j < k; ++j) {
                z += dm.V[(int64_t)j * n + i] * ds->cs[c][j];
                xz += dm.U[(int64_t)j * n + i] * ds->cs[c][j];
            }
            ds->Z[(int64_t)c * n + i] = z;
        }
        const double r = xz - ds->cmu[c] * z;
        part[2 * c] = z * z;
        part[2 * c + 1] = c < kc ? r * r : 0.0;
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int e = 0; e < 2 * kMaxDeflate; ++e) {
        double v = part[e];
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
        if (lane == 0) sh[wave][e] = v;
    }
    __syncthreads();
    if (threadIdx.x < 2 * kMaxDeflate) {
        const int e = threadIdx.x;
        ds->pz[(int64_t)b * 2 * kMaxDeflate + e] = ((sh[0][e] + sh[1][e]) + sh[2][e]) + sh[3][e];
    }
}

// Keep the converged candidates (largest |mu| first).
__global__ void defl_gate_kernel(const MatDesc *D) {
    if (threadIdx.x != 0) return;
    const MatDesc &dm = D[blockIdx.x];
    DeflState *ds = dm.defl;
    int cnt = 0;
    for (int c = 0; c < ds->ncand; ++c) {
        double z2 = 0.0, r2 = 0.0;
        for (int bb = 0; bb < dm.nbv; ++bb) {
            z2 += ds->pz[(int64_t)bb * 2 * kMaxDeflate + 2 * c];
            r2 += ds->pz[(int64_t)bb * 2 * kMaxDeflate + 2 * c + 1];
        }
        const double nz = sqrt(z2);
        if (!(nz > 0.0)) continue;
        const double mu = ds->cmu[c];
        if (!(sqrt(r2) / nz <= kDeflRtol * fabs(mu))) continue;  // also rejects NaN
        ds->mu[cnt] = mu;
        ds->inv_nz[cnt] = 1.0 / nz;
        ds->idx[cnt] = c;
        ++cnt;
    }
    ds->count = cnt;
}

// Upper triangle of X' = X - sum mu_c z_c z_c^T into the FP32 copy, in
// 64 x 64 tiles of the n x n triangle (work list of the vector kernels'
// order: one tile per work item, t = J (J + 1) / 2 + I).
__device__ __forceinline__ void tri_tile(int t, int &I, int &J) {
    int j = (int)((sqrtf(8.0f * (float)t + 1.0f) - 1.0f) * 0.5f);
    while ((j + 1) * (j + 2) / 2 <= t) ++j;
    while (j * (j + 1) / 2 > t) --j;
    J = j;
    I = t - j * (j + 1) / 2;
}

__device__ __forceinline__ double lowrank(const DeflState *ds, int64_t n, int64_t a, int64_t b, bool pos_only) {
    double v = 0.0;
    for (int c = 0; c < ds->count; ++c) {
        const double *z = ds->Z + (int64_t)ds->idx[c] * n;
        const double w = pos_only ? fmax(ds->mu[c], 0.0) : ds->mu[c];
        v += w * ((z[a] * ds->inv_nz[c]) * (z[b] * ds->inv_nz[c]));
    }
    return v;
}

__global__ __launch_bounds__(256) void defl_update_kernel(const MatDesc *D, const WorkItem *W, IoArg io) {
    const WorkItem wi = W[blockIdx.x];
    const MatDesc &dm = D[wi.x];
    const DeflState *ds = dm.defl;
    int I, J;
    tri_tile((int)wi.y, I, J);
    const int64_t n = dm.n, i = (int64_t)I * 64 + (threadIdx.x & 63);
    for (int c = threadIdx.x >> 6; c < 64; c += 4) {
        const int64_t j = (int64_t)J * 64 + c;
        if (i >= n || j >= n || i > j) continue;
        const double x = (double)io.X[j * io.ld + i];
        ds->Xd[j * ds->ldd + i] = (float)(x - lowrank(ds, n, i, j, false));
    }
}

// out += sum max(mu_c, 0) z_c z_c^T on both triangles; each upper entry and
// its mirror get the same value, so out stays exactly symmetric.
__global__ __launch_bounds__(256) void defl_addback_kernel(const MatDesc *D, const WorkItem *W, IoArg io) {
    const WorkItem wi = W[blockIdx.x];
    const MatDesc &dm = D[wi.x];
    const DeflState *ds = dm.defl;
    if (ds->count == 0 || dm.scal->nonfinite) return;
    int I, J;
    tri_tile((int)wi.y, I, J);
    const int64_t n = dm.n, i = (int64_t)I * 64 + (threadIdx.x & 63);
    for (int c = threadIdx.x >> 6; c < 64; c += 4) {
        const int64_t j = (int64_t)J * 64 + c;
        if (i >= n || j >= n || i > j) continue;
        const float v = (float)((double)io.out[j * io.ld + i] + lowrank(ds, n, i, j, true));
        io.out[j * io.ld + i] = v;
        io.out[i * io.ld + j] = v;
    }
}

}  // namespace

hipError_t deflate_remove(const DeflLaunch &L, hipStream_t s) {
    const MatDesc *D = L.desc;
    hipLaunchKernelGGL(defl_h_kernel, dim3((unsigned)L.n_vec), dim3(256), 0, s, D, L.w_vec);
    hipLaunchKernelGGL(defl_eig_kernel, dim3(1), dim3(64), 0, s, D);
    hipLaunchKernelGGL(defl_z_kernel, dim3((unsigned)L.n_vec), dim3(256), 0, s, D, L.w_vec);
    hipLaunchKernelGGL(defl_gate_kernel, dim3(1), dim3(64), 0, s, D);
    hipLaunchKernelGGL(defl_update_kernel, dim3((unsigned)L.n_tri), dim3(256), 0, s, D, L.w_tri, L.io);
    return hipGetLastError();
}

hipError_t deflate_addback(const DeflLaunch &L, hipStream_t s) {
    hipLaunchKernelGGL(defl_addback_kernel, dim3((unsigned)L.n_tri), dim3(256), 0, s, L.desc, L.w_tri, L.io);
    return hipGetLastError();
}

}  // namespace psd

// C ABI of libpsdproj: argument checks, workspace pool, and the launch
// sequence of Algorithm 2 (bound -> rescale/cast -> T filter stages -> final).
#include <math.h>
#include <string.h>

#include <map>
#include <mutex>
#include <utility>
#include <vector>

#include "../../include/psdproj.h"
#include "aux_kernels.hpp"
#include "coeffs.hpp"
#include "common.hpp"
#include "gemm_sym.hpp"
#include "runtime.hpp"

namespace psd {
namespace {

constexpr int kDefaultLanczos = 20;
constexpr uint64_t kLanczosSeed = 0;
// FP16_SPLIT default: hi + lo products in stages 1-4 (the stages whose
// rounding dominates the error) and in the final product.
constexpr uint32_t kDefaultSplitMask = 0xF;
constexpr int kDefaultSplitFinal = 1;

struct StagePlan {
    int T = 0;
    double a[16], b[16], c[16];
    int dtype = DT_F32;
    uint32_t split_mask = 0;
    bool split_final = false;
};

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
        default: return false;
    }
    p.T = T;
    for (int t = 0; t < T; ++t) {
        const double s = t < nres ? res : 1.0;
        p.a[t] = tab[t].a * s;
        p.b[t] = tab[t].b * s;
        p.c[t] = tab[t].c * s;
    }
    if (o.mode == PSDPROJ_MODE_FP16_SPLIT) {
        p.split_mask = (o.split_mask ? o.split_mask : kDefaultSplitMask) & ((1u << T) - 1);
        p.split_final = o.split_final < 0 ? kDefaultSplitFinal : o.split_final != 0;
    }
    return true;
}

size_t elt_size(int dtype) { return dtype == DT_F32 ? 4 : 2; }

struct Layout {
    int64_t n, np;
    int steps;
    bool split;
    size_t off_scal, off_lz, off_mat, mat_bytes, total;
};

Layout make_layout(int64_t n, const StagePlan &p, int steps) {
    Layout L{};
    L.n = n;
    L.np = gemm_padded_size(n);
    L.steps = steps;
    L.split = p.split_mask != 0 || p.split_final;
    size_t off = 0;
    auto take = [&](size_t bytes) { const size_t o = off; off += round_up((int64_t)bytes, 256); return o; };
    L.off_scal = take(sizeof(Scalars));
    L.off_lz = take(sizeof(double) * lanczos_work_doubles(n, steps));
    L.mat_bytes = round_up((int64_t)(elt_size(p.dtype) * (size_t)L.np * (size_t)L.np), 256);
    L.off_mat = take(L.mat_bytes * 4 * (L.split ? 2 : 1));
    L.total = off;
    return L;
}

struct Pool {
    void *ptr = nullptr;
    size_t bytes = 0;
};
std::mutex g_mu;
std::map<std::pair<int, hipStream_t>, Pool> g_pool;

int get_workspace(hipStream_t s, size_t bytes, void **out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return PSDPROJ_ERR_HIP;
    std::lock_guard<std::mutex> lk(g_mu);
    Pool &p = g_pool[{dev, s}];
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

__global__ void info_kernel(const Scalars *s, psdproj_info *info, int stages) {
    if (threadIdx.x != 0) return;
    info->lambda = s->lam;
    info->lanczos_lambda = s->lanczos_lam;
    info->sigma = s->sigma;
    info->residual = s->resid;
    info->fro_norm = sqrt(s->fro2);
    info->colmax_norm = sqrt(s->colmax2);
    info->lanczos_steps = s->k;
    info->nonfinite = s->nonfinite;
    info->fallback = s->fallback;
    info->stages = stages;
}

// Replace the Lanczos bound by a caller-supplied one (keeps the norms).
__global__ void override_kernel(Scalars *s, double lam) {
    if (threadIdx.x != 0) return;
    s->lam = s->nonfinite ? 0.0 : lam;
    s->inv_lam = (s->nonfinite || !(lam > 0.0)) ? 0.0 : 1.0 / lam;
    s->fallback = 0;
}

struct Mat {
    void *hi = nullptr, *lo = nullptr;
};

}  // namespace

int run_projection(const psdproj_opts &o, int64_t n, int64_t ld, const float *X, float *out, hipStream_t s,
                   psdproj_info *info, bool bound_only) {
    StagePlan p;
    if (!make_stage_plan(o, p)) return PSDPROJ_ERR_INVALID_ARG;
    const int steps = o.lanczos_steps ? o.lanczos_steps : kDefaultLanczos;
    if (steps < 1 || steps > kMaxLanczos) return PSDPROJ_ERR_INVALID_ARG;
    if (n < 0 || ld < (n > 1 ? n : 1)) return PSDPROJ_ERR_INVALID_ARG;
    if (n == 0) return PSDPROJ_OK;
    if (!X || (!out && !bound_only)) return PSDPROJ_ERR_INVALID_ARG;
    if (n > (int64_t)1 << 20) return PSDPROJ_ERR_UNSUPPORTED;

    const Layout L = make_layout(n, p, steps);
    void *base = nullptr;
    int st = get_workspace(s, L.total, &base);
    if (st != PSDPROJ_OK) return st;
    uint8_t *b = (uint8_t *)base;
    Scalars *scal = (Scalars *)(b + L.off_scal);
    double *lz = (double *)(b + L.off_lz);
    LanczosWork wk;
    {
        const int64_t nbv = (n + 255) / 256;
        const int64_t tiles = symv_tile_count(n);
        wk.V = lz;
        wk.u = wk.V + n * steps;
        wk.w = wk.u + n;
        wk.w2 = wk.w + n;
        wk.colsq = wk.w2 + n;
        wk.part_a = wk.colsq + n;
        wk.part_b = wk.part_a + nbv * kMaxLanczos;
        wk.sd = wk.part_b + nbv * kMaxLanczos;
        wk.sa = wk.sd + tiles * 128;
        wk.sd2 = wk.sa + tiles * 128;
        wk.sa2 = wk.sd2 + tiles * 128;
    }
    hipError_t e;
    // 1-2. spectral bound (Theorem 2) + guard, from the upper triangle of X
    e = spectral_bound(X, ld, n, steps, kLanczosSeed, wk, scal, o.force_bound_fallback, s);
    if (e != hipSuccess) return PSDPROJ_ERR_HIP;
    if (o.lambda_override > 0.0) hipLaunchKernelGGL(override_kernel, dim3(1), dim3(64), 0, s, scal, o.lambda_override);
    if (bound_only) {
        if (info) hipLaunchKernelGGL(info_kernel, dim3(1), dim3(64), 0, s, (const Scalars *)scal, info, 0);
        return hipGetLastError() == hipSuccess ? PSDPROJ_OK : PSDPROJ_ERR_HIP;
    }

    // 3. work matrices: slot 0 holds X0, slots 1..3 rotate
    Mat slot[4];
    uint8_t *mb = b + L.off_mat;
    for (int k = 0; k < 4; ++k) {
        slot[k].hi = mb + (size_t)k * L.mat_bytes;
        if (L.split) slot[k].lo = mb + (size_t)(4 + k) * L.mat_bytes;
    }
    const bool x0_split = p.split_final || (p.split_mask & 1u);
    e = mirror_cast(X, ld, n, L.np, scal, 1, p.dtype, slot[0].hi, x0_split ? slot[0].lo : nullptr, L.np, s);
    if (e != hipSuccess) return PSDPROJ_ERR_HIP;

    GemmArgs g{};
    g.ld = L.np;
    g.K = L.np;
    g.scal = scal;
    auto gemm = [&](Mat Lm, bool ls, Mat Rm, bool rs, const Mat *C0, bool c0s, float alpha, float beta, float gamma,
                    Mat D, bool dsplit) -> hipError_t {
        g.Lhi = Lm.hi; g.Llo = ls ? Lm.lo : nullptr;
        g.Rhi = Rm.hi; g.Rlo = rs ? Rm.lo : nullptr;
        g.C0hi = C0 ? C0->hi : nullptr; g.C0lo = (C0 && c0s) ? C0->lo : nullptr;
        g.Dhi = D.hi; g.Dlo = dsplit ? D.lo : nullptr;
        g.alpha = alpha; g.beta = beta; g.gamma = gamma;
        return gemm_sym_launch(g, p.dtype, dsplit ? EPI_STORE_SPLIT : EPI_STORE, s);
    };
    int cur = 0;
    bool cur_split = (p.split_mask & 1u) != 0;
    for (int t = 0; t < p.T; ++t) {
        const bool sp = (p.split_mask >> t) & 1u;
        const bool next_split = (t + 1 < p.T) ? ((p.split_mask >> (t + 1)) & 1u) : p.split_final;
        int pa = -1, pb = -1;
        for (int k = 1; k < 4; ++k)
            if (k != cur) { if (pa < 0) pa = k; else if (pb < 0) pb = k; }
        const bool xs = sp && cur_split;  // X enters as a pair only in a split stage
        // A = X X
        e = gemm(slot[cur], xs, slot[cur], xs, nullptr, false, 0.f, 1.f, 0.f, slot[pa], sp);
        if (e != hipSuccess) return PSDPROJ_ERR_HIP;
        // B = b A + c A A
        e = gemm(slot[pa], sp, slot[pa], sp, &slot[pa], sp, (float)p.b[t], (float)p.c[t], 0.f, slot[pb], sp);
        if (e != hipSuccess) return PSDPROJ_ERR_HIP;
        // X' = a X + X B
        e = gemm(slot[cur], xs, slot[pb], sp, &slot[cur], cur_split, (float)p.a[t], 1.f, 0.f, slot[pa], next_split);
        if (e != hipSuccess) return PSDPROJ_ERR_HIP;
        cur = pa;
        cur_split = next_split;
    }
    // 4. out = (X + lam X0 X_T) / 2
    g.Lhi = slot[0].hi; g.Llo = p.split_final ? slot[0].lo : nullptr;
    g.Rhi = slot[cur].hi; g.Rlo = p.split_final ? slot[cur].lo : nullptr;
    g.C0hi = g.C0lo = nullptr;
    g.Dhi = g.Dlo = nullptr;
    g.out = out; g.ldo = ld; g.n = n; g.Xin = X; g.ldx = ld;
    e = gemm_sym_launch(g, p.dtype, EPI_FINAL, s);
    if (e != hipSuccess) return PSDPROJ_ERR_HIP;
    if (info) hipLaunchKernelGGL(info_kernel, dim3(1), dim3(64), 0, s, (const Scalars *)scal, info, p.T);
    return hipGetLastError() == hipSuccess ? PSDPROJ_OK : PSDPROJ_ERR_HIP;
}

psdproj_opts default_opts(int mode) {
    psdproj_opts o;
    memset(&o, 0, sizeof(o));
    o.mode = mode;
    o.split_final = -1;
    return o;
}

size_t workspace_bytes_for(int64_t n, int mode) {
    psdproj_opts o = default_opts(mode);
    StagePlan p;
    if (n <= 0 || !make_stage_plan(o, p)) return 0;
    return make_layout(n, p, kDefaultLanczos).total;
}

size_t pool_held(hipStream_t s) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_pool.find({dev, s});
    return it == g_pool.end() ? 0 : it->second.bytes;
}

void pool_release(hipStream_t s) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return;
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_pool.find({dev, s});
    if (it == g_pool.end()) return;
    if (it->second.ptr) {
        (void)hipStreamSynchronize(s);
        (void)hipFree(it->second.ptr);
    }
    g_pool.erase(it);
}

int gemm_count_for(const psdproj_opts &o) {
    StagePlan p;
    if (!make_stage_plan(o, p)) return -1;
    int g = 0;
    bool cur_split = (p.split_mask & 1u) != 0;
    for (int t = 0; t < p.T; ++t) {
        const bool sp = (p.split_mask >> t) & 1u;
        const bool next_split = (t + 1 < p.T) ? ((p.split_mask >> (t + 1)) & 1u) : p.split_final;
        const bool xs = sp && cur_split;
        g += xs ? 3 : 1;      // X X
        g += sp ? 3 : 1;      // A A
        g += sp ? (xs ? 3 : 2) : 1;  // X B
        cur_split = next_split;
    }
    g += p.split_final ? 3 : 1;
    return g;
}

}  // namespace psd

using namespace psd;

extern "C" {

int psdproj_project(int64_t n, int64_t ld, const float *X, float *out, int mode, psdproj_stream_t stream) {
    const psdproj_opts o = default_opts(mode);
    return run_projection(o, n, ld, X, out, (hipStream_t)stream, nullptr, false);
}

int psdproj_project_ex(const psdproj_opts *opts, int64_t n, int64_t ld, const float *X, float *out,
                       psdproj_stream_t stream, psdproj_info *info_dev) {
    if (!opts) return PSDPROJ_ERR_INVALID_ARG;
    return run_projection(*opts, n, ld, X, out, (hipStream_t)stream, info_dev, false);
}

int psdproj_spectral_bound(int64_t n, int64_t ld, const float *X, int lanczos_steps, psdproj_stream_t stream,
                           psdproj_info *info_dev) {
    if (!info_dev) return PSDPROJ_ERR_INVALID_ARG;
    psdproj_opts o = default_opts(PSDPROJ_MODE_FP32);
    o.lanczos_steps = lanczos_steps;
    return run_projection(o, n, ld, X, nullptr, (hipStream_t)stream, info_dev, true);
}

int psdproj_project_batched(int count, const int64_t *n, const int64_t *ld, const float *const *X, float *const *out,
                            int mode, psdproj_stream_t stream) {
    if (count < 0 || (count > 0 && (!n || !ld || !X || !out))) return PSDPROJ_ERR_INVALID_ARG;
    for (int i = 0; i < count; ++i)
        if (n[i] < 0 || ld[i] < (n[i] > 1 ? n[i] : 1) || (n[i] > 0 && (!X[i] || !out[i])))
            return PSDPROJ_ERR_INVALID_ARG;
    const psdproj_opts o = default_opts(mode);
    for (int i = 0; i < count; ++i) {
        const int st = run_projection(o, n[i], ld[i], X[i], out[i], (hipStream_t)stream, nullptr, false);
        if (st != PSDPROJ_OK) return st;
    }
    return PSDPROJ_OK;
}

size_t psdproj_workspace_bytes(int64_t n, int mode) { return workspace_bytes_for(n, mode); }

int psdproj_gemm_count(const psdproj_opts *opts, int mode) {
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
    for (auto &kv : g_pool)
        if (kv.second.ptr) (void)hipFree(kv.second.ptr);
    g_pool.clear();
    return PSDPROJ_OK;
}

int psdproj_tune(const char *key, int64_t value) {
    if (!key) return PSDPROJ_ERR_INVALID_ARG;
    if (!strcmp(key, "gemm_tile")) {
        if (value != 0 && value != 128 && value != 256) return PSDPROJ_ERR_INVALID_ARG;
        gemm_set_tile_override((int)value);
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
    }
    return "unknown status";
}

int psdproj_sym_gemm(int dtype, int64_t n_p, int64_t ld, const void *L, const void *Llo, const void *R,
                     const void *Rlo, const void *C0, const void *C0lo, float alpha, float beta, float gamma, void *D,
                     void *Dlo, psdproj_stream_t stream) {
    if (dtype < 0 || dtype > 2 || n_p <= 0 || n_p % kTile || ld < n_p || !L || !R || !D) return PSDPROJ_ERR_INVALID_ARG;
    if (dtype == DT_F32 && (Llo || Rlo || Dlo || C0lo)) return PSDPROJ_ERR_UNSUPPORTED;
    GemmArgs g{};
    g.Lhi = L; g.Llo = Llo; g.Rhi = R; g.Rlo = Rlo; g.C0hi = C0; g.C0lo = C0lo; g.Dhi = D; g.Dlo = Dlo;
    g.ld = ld; g.K = n_p; g.alpha = alpha; g.beta = beta; g.gamma = gamma;
    const hipError_t e = gemm_sym_launch(g, dtype, Dlo ? EPI_STORE_SPLIT : EPI_STORE, (hipStream_t)stream);
    return e == hipSuccess ? PSDPROJ_OK : PSDPROJ_ERR_HIP;
}

}  // extern "C"

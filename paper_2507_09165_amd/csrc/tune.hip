// Autotuner of the product tile policy, per size class, with a cache file.
//
// For each requested order n the tuner times whole projections of a random
// symmetric matrix of that order (device-generated, entries uniform in
// [-1, 1] / sqrt(n)) under each candidate policy of its size class (quarter
// octaves of n): 128 tiles only, or 256-tile rounds whose last partial round
// runs as up to 1, 2, 4 or 8 K-chunks per tile. The fastest becomes the
// class's choice for later plans and is written to the cache file, one line
// per (GPU architecture, CU count, mode, class):
//     psdproj-tune 1 <arch> <cus> <mode> <class> <tile> <ksplit> <ms> <n>
// psdproj_tune_load applies the lines of a cache file that match the current
// device; the first plan of the process also loads the file that the
// environment variable PSDPROJ_TUNE_CACHE names.
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <mutex>
#include <string>
#include <vector>

#include "../../include/psdproj.h"
#include "common.hpp"
#include "gemm_sym.hpp"
#include "runtime.hpp"

namespace psd {
namespace {

// x_ij = x_ji uniform in [-1, 1) / sqrt(n), from the SplitMix64 finaliser of
// the pair (min, max) (the same counter-hash idea as the Lanczos start).
__global__ __launch_bounds__(256) void tune_fill_kernel(int64_t n, float *X, uint64_t seed) {
    const int64_t j = blockIdx.y;
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const uint64_t a = (uint64_t)(i < j ? i : j), b = (uint64_t)(i < j ? j : i);
    uint64_t z = seed + (a * 0x100000001B3ull + b + 1ull) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z = z ^ (z >> 31);
    const double u = 2.0 * ((double)(z >> 11) * 0x1.0p-53) - 1.0;
    X[j * n + i] = (float)(u / sqrt((double)n));
}

struct DeviceKey {
    std::string arch;
    int cus = 0;
};

int device_key(DeviceKey &k) {
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return PSDPROJ_ERR_HIP;
    std::string a = prop.gcnArchName;
    const size_t colon = a.find(':');
    k.arch = colon == std::string::npos ? a : a.substr(0, colon);
    k.cus = prop.multiProcessorCount;
    return PSDPROJ_OK;
}

struct Line {
    std::string arch;
    int cus, mode, cls, tile, ksplit;
    double ms;
    long long n;
};

bool parse_line(const char *s, Line &l) {
    char arch[64] = {0};
    int ver = 0;
    if (sscanf(s, "psdproj-tune %d %63s %d %d %d %d %d %lf %lld", &ver, arch, &l.cus, &l.mode, &l.cls, &l.tile,
               &l.ksplit, &l.ms, &l.n) != 9 || ver != 1)
        return false;
    l.arch = arch;
    return (l.tile == 128 || l.tile == 256) && l.ksplit >= 1 && l.ksplit <= 64;
}

std::vector<Line> read_cache(const char *path) {
    std::vector<Line> v;
    FILE *f = fopen(path, "r");
    if (!f) return v;
    char buf[512];
    while (fgets(buf, sizeof(buf), f)) {
        Line l;
        if (parse_line(buf, l)) v.push_back(l);
    }
    fclose(f);
    return v;
}

// Lines of `path` for this device applied; returns how many, or < 0.
int load_cache(const char *path) {
    DeviceKey k;
    if (device_key(k) != PSDPROJ_OK) return -PSDPROJ_ERR_HIP;
    int applied = 0;
    for (const Line &l : read_cache(path)) {
        if (l.arch != k.arch || l.cus != k.cus) continue;
        const int dt = mode_dtype(l.mode);
        if (dt < 0) continue;
        gemm_set_class_choice(dt, l.cls, l.tile, l.ksplit);
        ++applied;
    }
    return applied;
}

std::once_flag g_env_once;

}  // namespace

void load_env_tune_cache() {
    std::call_once(g_env_once, [] {
        const char *p = getenv("PSDPROJ_TUNE_CACHE");
        if (p && *p) (void)load_cache(p);
    });
}

}  // namespace psd

using namespace psd;

extern "C" {

int psdproj_tune_load(const char *path) {
    if (!path) return -PSDPROJ_ERR_INVALID_ARG;
    return load_cache(path);
}

int psdproj_autotune(int mode, const int64_t *sizes, int count, const char *cache_path, psdproj_stream_t stream) {
    const int dt = mode_dtype(mode);
    if (dt < 0 || count < 0 || (count > 0 && !sizes)) return PSDPROJ_ERR_INVALID_ARG;
    for (int c = 0; c < count; ++c)
        if (sizes[c] < 1 || sizes[c] > 65535) return PSDPROJ_ERR_INVALID_ARG;
    DeviceKey key;
    if (device_key(key) != PSDPROJ_OK) return PSDPROJ_ERR_HIP;
    hipStream_t s = (hipStream_t)stream;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return PSDPROJ_ERR_HIP;
    std::vector<Line> lines;
    int status = PSDPROJ_OK;
    const psdproj_opts o = default_opts(mode);
    for (int c = 0; c < count && status == PSDPROJ_OK; ++c) {
        const int64_t n = sizes[c];
        const int cls = gemm_size_class(n);
        float *X = nullptr, *out = nullptr;
        if (hipMalloc(&X, sizeof(float) * n * n) != hipSuccess ||
            hipMalloc(&out, sizeof(float) * n * n) != hipSuccess) {
            (void)hipGetLastError();
            if (X) (void)hipFree(X);
            status = PSDPROJ_ERR_NO_MEMORY;
            break;
        }
        hipLaunchKernelGGL(tune_fill_kernel, dim3((unsigned)((n + 255) / 256), (unsigned)n), dim3(256), 0, s, n, X,
                           (uint64_t)0x5eed);
        std::vector<std::pair<int, int>> cand{{128, 1}};
        if (dt != DT_F32 && n >= 1024)  // FP32 products have no 256 tile
            for (int ks : {1, 2, 4, 8}) cand.push_back({256, ks});
        double best = 1e300;
        std::pair<int, int> pick = cand[0];
        for (const auto &cd : cand) {
            gemm_set_class_choice(dt, cls, cd.first, cd.second);
            // the first call builds the plan and takes the workspace (untimed)
            int st = run_projection(o, n, n, X, out, s, nullptr, false);
            const int reps = n >= 4096 ? 3 : 5;
            if (st == PSDPROJ_OK && hipEventRecord(e0, s) != hipSuccess) st = PSDPROJ_ERR_HIP;
            for (int r = 0; r < reps && st == PSDPROJ_OK; ++r) st = run_projection(o, n, n, X, out, s, nullptr, false);
            float ms = 0.0f;
            if (st == PSDPROJ_OK && (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                                     hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
                st = PSDPROJ_ERR_HIP;
            if (st != PSDPROJ_OK) {
                status = st;
                break;
            }
            const double avg = ms / reps;
            if (avg < best) {
                best = avg;
                pick = cd;
            }
        }
        (void)hipStreamSynchronize(s);
        (void)hipFree(X);
        (void)hipFree(out);
        if (status != PSDPROJ_OK) break;
        gemm_set_class_choice(dt, cls, pick.first, pick.second);
        lines.push_back(Line{key.arch, key.cus, mode, cls, pick.first, pick.second, best, (long long)n});
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (status != PSDPROJ_OK || !cache_path) return status;
    // rewrite the cache: its other lines kept, this device's lines for these
    // (mode, class) pairs replaced
    std::vector<Line> keep;
    for (const Line &l : read_cache(cache_path)) {
        bool replaced = false;
        for (const Line &m : lines)
            replaced |= l.arch == m.arch && l.cus == m.cus && l.mode == m.mode && l.cls == m.cls;
        if (!replaced) keep.push_back(l);
    }
    keep.insert(keep.end(), lines.begin(), lines.end());
    FILE *f = fopen(cache_path, "w");
    if (!f) return PSDPROJ_ERR_INVALID_ARG;
    for (const Line &l : keep)
        fprintf(f, "psdproj-tune 1 %s %d %d %d %d %d %.4f %lld\n", l.arch.c_str(), l.cus, l.mode, l.cls, l.tile,
                l.ksplit, l.ms, l.n);
    fclose(f);
    return PSDPROJ_OK;
}

}  // extern "C"

/*
 * libpsdproj — factorization-free orthogonal projection of a dense symmetric
 * matrix onto the positive semidefinite cone by composite polynomial
 * filtering, for AMD Instinct MI355X (gfx950).
 *
 * The projection (Section 1, eq. (1)) is
 *     Pi(X) = argmin_{Y >= 0} 1/2 ||Y - X||_F^2 = Q diag(max(lambda_i, 0)) Q^T.
 * It is computed without an eigendecomposition (Algorithm 2):
 *   1. lam = sqrt(sigma + ||X^2 q - sigma q||_2), (sigma, q) the largest Ritz
 *      pair of a 20-step FP64 Lanczos run on X^2 (Theorem 2, Section 3.4);
 *   2. X0 = X / lam;
 *   3. X_t = f_t(X_{t-1}), t = 1..T, with the odd quintics
 *      f_t(x) = a_t x + b_t x^3 + c_t x^5 of Table 1 (T = 10, single) or
 *      Table 2 (T = 7, half), each stage evaluated with three matrix products;
 *   4. return lam * X0 (I + X_T) / 2.
 *
 * Conventions shared by every entry point:
 *   - X and out are DEVICE pointers owned by the caller, FP32, column-major
 *     with leading dimension ld >= max(1, n). Only the upper triangle of X is
 *     read (uplo = 'U'); both triangles of out are written and out is exactly
 *     symmetric. out == X (in place) is allowed.
 *   - Every call only enqueues work on `stream` (a hipStream_t; NULL is the
 *     default stream) and returns. The return value reports argument, launch
 *     and allocation errors only; numerical status (non-finite input, bound
 *     fallback, lam) is written to device memory (psdproj_info).
 *   - n == 0 is a no-op. X == 0 gives out == 0. A non-finite input (Inf or NaN
 *     in the upper triangle) sets every entry of out to NaN and sets
 *     psdproj_info.nonfinite, so callers without an info buffer see it too.
 *   - The library keeps a workspace per (device, stream), grown on demand
 *     (growing synchronises that stream). Calls on one stream are ordered by
 *     the stream; calls on different streams use different workspaces.
 *   - No entry point reads device results back to the host.
 */
#ifndef PSDPROJ_H
#define PSDPROJ_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ihipStream_t *psdproj_stream_t; /* same type as hipStream_t */

typedef enum {
    PSDPROJ_OK = 0,
    PSDPROJ_ERR_INVALID_ARG = 1,
    PSDPROJ_ERR_UNSUPPORTED = 2,
    PSDPROJ_ERR_NO_MEMORY = 3,
    PSDPROJ_ERR_HIP = 4,
    PSDPROJ_ERR_REJECTED = 5,
    PSDPROJ_ERR_CANCELLED = 6,
    PSDPROJ_ERR_TIMEOUT = 7,
    PSDPROJ_ERR_NOT_FOUND = 8,
    PSDPROJ_ERR_PENDING = 9,
    PSDPROJ_ERR_NONFINITE = 10, /* served request whose input held Inf/NaN */
    PSDPROJ_ERR_TOO_LARGE = 11  /* psdproj_project_noalloc: the workspace would not
                                   fit in PSDPROJ_NOALLOC_SCRATCH_BYTES */
} psdproj_status;

/* Compute precision of the filter products. Storage of X and out is FP32. */
typedef enum {
    PSDPROJ_MODE_FP32 = 0,       /* Table 1 refined (T = 10), FP32 MFMA, 31 products  */
    PSDPROJ_MODE_FP16 = 1,       /* Table 2 refined (T = 7), FP16 MFMA, 22 products   */
    PSDPROJ_MODE_BF16 = 2,       /* Table 2 refined (T = 7), BF16 MFMA; by default the
                                    products of stages 1-4 use BF16 hi+lo split
                                    operands (plain BF16, 8 significant bits, misses
                                    the 5e-3 half-precision target): 46 products   */
    PSDPROJ_MODE_FP16_SPLIT = 3, /* Table 2 refined, FP16 with hi+lo split operands in
                                    the stages of split_mask and the final product   */
    PSDPROJ_MODE_FP32_EMU = 4,   /* Table 1 refined (T = 10), every product on FP16
                                    hi+lo pairs (FP32-level operands at the FP16
                                    MFMA rate), 93 product-equivalents              */
    PSDPROJ_MODE_FP8_FP16_SPLIT = 5, /* Table 2 refined, FP16 bulk; the split products
                                    of split_mask (and the final product if
                                    split_final) carry the correction as e4m3
                                    codes: L_hi R_hi on FP16 MFMAs plus both
                                    cross terms on one FP8 MFMA per 32 K, so a
                                    split product costs 2 product-equivalents
                                    instead of 3                                    */
    PSDPROJ_MODE_NS_FP16 = 6,    /* Newton-Schulz baseline of Section 4.1: 10 cubic
                                    steps (3x - x^3)/2 on FP16 MFMA, 21 products     */
    PSDPROJ_MODE_NS_FP32 = 7,    /* Newton-Schulz baseline: 15 cubic steps on FP32
                                    MFMA, 31 products                                */
    PSDPROJ_MODE_FP8_BF16_SPLIT = 8 /* Table 2 refined, BF16 bulk; the split products
                                    of split_mask (default stages 1-4, as BF16) keep
                                    a BF16 hi part and carry the correction as e4m3
                                    codes of (M - M_hi) 2^(8 + e): BF16 hi x hi plus
                                    both cross terms on one FP8 MFMA per 32 K, 2
                                    product-equivalents per split product (BF16 hi+lo
                                    pairs: 3), 34 in all                            */
} psdproj_mode;

/* split_mask flag: split only the B product of the masked stages */
#define PSDPROJ_SPLIT_B_ONLY 0x40000000u
/* split_mask bits PSDPROJ_SPLIT_B_SHIFT + t (t < 14): stage t+1 splits only its
 * B product (a stage also set in bits 0..15 splits in full) */
#define PSDPROJ_SPLIT_B_SHIFT 16

typedef struct {
    int mode;                 /* psdproj_mode */
    int lanczos_steps;        /* 0 -> 20 (Section 3.4); at most 32 */
    uint32_t split_mask;      /* BF16, FP16_SPLIT, FP8_FP16_SPLIT: bit t set ->
                                 stage t+1 uses split products; 0 -> the mode's
                                 default (FP16_SPLIT: stages 2-3; FP8_FP16_SPLIT:
                                 stage 3, and stages 1-2 B-only; the BF16 forms:
                                 1-4). Bit 31 set:
                                 bits 0..29 are taken as given even when all zero
                                 (e.g. 0x80000000 = no split stage). Bit 30
                                 (PSDPROJ_SPLIT_B_ONLY): in the masked stages only
                                 B = b A + c A^2 is split; A = X X stays plain and
                                 X' = a X + B X has one split operand. Without
                                 bit 30, bits 16..29 name such B-only stages
                                 beside the fully split ones of bits 0..15
                                 (PSDPROJ_SPLIT_B_SHIFT). Matrices of the
                                 one-workgroup path (order <= the "small_max"
                                 tuning key) split B-only stages in full */
    int split_final;          /* BF16, FP16_SPLIT, FP8_FP16_SPLIT: -1 default (0),
                                 0 plain, 1 split final product */
    double lambda_override;   /* > 0: use this bound instead of the Lanczos bound */
    int force_bound_fallback; /* test hook: halve the Lanczos bound so that the
                                 guard must replace it by ||X||_F */
    int deflate;              /* 0: off. k in 1..8: deflation of dominant
                                 eigenpairs before filtering (Section 4.1
                                 "Results", Section 5): of the k Rayleigh-Ritz
                                 pairs (mu_i, z_i) of X with largest |mu_i| in
                                 the Krylov basis of the bound's Lanczos run,
                                 those with ||X z_i - mu_i z_i|| <= 1e-8 |mu_i|
                                 are removed, X' = X - sum mu_i z_i z_i^T is
                                 projected with its own bound, and
                                 sum max(mu_i, 0) z_i z_i^T is added back.
                                 Single projections only (batched calls return
                                 PSDPROJ_ERR_UNSUPPORTED); the workspace gains an
                                 ld x n FP32 copy. */
    double adaptive_tol;      /* adaptive depth (Section 5): > 0 ends the sign
                                 iteration at the first stage whose relative
                                 change ||X_{t+1} - X_t||_F / ||X_t||_F is at
                                 most this (FP64 sums over the stored iterates);
                                 later stages then skip their products. Applies
                                 to every Newton-Schulz step, and to the
                                 adaptive_extra stages. Modes without split
                                 products only (else PSDPROJ_ERR_UNSUPPORTED);
                                 psdproj_info.stages reports the stages run. */
    int adaptive_extra;       /* composite modes: 0..(16 - T) quintic
                                 Newton-Schulz stages (15x - 10x^3 + 3x^5)/8
                                 appended to the table's T stages (with
                                 adaptive_tol = 0 all of them run) */
} psdproj_opts;

/* Written on the device by psdproj_project_ex / psdproj_spectral_bound. */
typedef struct {
    double lambda;         /* bound used for the rescale */
    double lanczos_lambda; /* sqrt(sigma + residual) before the guard */
    double sigma;          /* largest Ritz value of X^2 */
    double residual;       /* ||X^2 q - sigma q||_2 */
    double fro_norm;       /* ||X||_F */
    double colmax_norm;    /* max_j ||X e_j||_2 (lower bound on ||X||_2) */
    int32_t lanczos_steps; /* Lanczos steps taken (early stop on breakdown) */
    int32_t nonfinite;     /* input held Inf/NaN; out was set to NaN */
    int32_t fallback;      /* guard replaced an invalid Lanczos bound */
    int32_t stages;        /* filter stages applied */
    int32_t deflated;      /* eigenpairs removed before filtering (opts.deflate) */
    int32_t reserved;
} psdproj_info;

/* Project X onto the PSD cone (Algorithm 2) in the given psdproj_mode.
 * n >= 0, ld >= max(1, n); X, out device pointers (may alias).
 * Returns PSDPROJ_OK, PSDPROJ_ERR_INVALID_ARG (bad n/ld/pointer/mode),
 * PSDPROJ_ERR_NO_MEMORY (workspace) or PSDPROJ_ERR_HIP (launch failure). */
int psdproj_project(int64_t n, int64_t ld, const float *X, float *out, int mode,
                    psdproj_stream_t stream);

/* As psdproj_project with options; info_dev (device memory, may be NULL)
 * receives the numerical status once the stream reaches the end of the call. */
int psdproj_project_ex(const psdproj_opts *opts, int64_t n, int64_t ld, const float *X,
                       float *out, psdproj_stream_t stream, psdproj_info *info_dev);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc):
 * psdproj_project_ex with the workspace in a fixed library-owned device array
 * of PSDPROJ_NOALLOC_SCRATCH_BYTES per GPU (held from the library's load until
 * the process ends) instead of the pooled workspace; it calls no hipMalloc,
 * hipFree or other allocating routine. The caller still supplies X, out and
 * info_dev. Every matrix with n <= 2048 fits in every mode and option set
 * without deflation (opts.deflate adds an ld x n FP32 copy to the workspace);
 * larger ones fit while psdproj_workspace_bytes(n, mode) (default options)
 * stays within the limit. A call whose workspace would exceed it returns
 * PSDPROJ_ERR_TOO_LARGE and queues nothing. Results are bitwise those of
 * psdproj_project_ex with the same arguments.
 * The array is shared by every call on one GPU, and its contents are those
 * the last call left: calls that overlap on one GPU (queued on different
 * streams without ordering between them) race and give wrong results. A
 * call whose (n, mode, options) differ from the previous call's on that GPU
 * waits for the device (another stream) or the stream before rewriting the
 * array's tables. Such a call cannot be captured (PSDPROJ_ERR_UNSUPPORTED
 * while capturing); a call with the previous call's shape only launches
 * kernels. */
#define PSDPROJ_NOALLOC_SCRATCH_BYTES ((size_t)80 << 20)
int psdproj_project_noalloc(const psdproj_opts *opts, int64_t n, int64_t ld, const float *X,
                            float *out, psdproj_stream_t stream, psdproj_info *info_dev);

/* Only the spectral bound (steps 1-2 of Algorithm 2, Theorem 2): fills
 * info_dev (device memory, required) for the upper triangle of X. */
int psdproj_spectral_bound(int64_t n, int64_t ld, const float *X, int lanczos_steps,
                           psdproj_stream_t stream, psdproj_info *info_dev);

/* Batched projection of `count` independent matrices (host arrays of sizes,
 * leading dimensions and device pointers). Matrices are independent; each
 * result equals the one psdproj_project gives for that matrix alone.
 *
 * Small matrices: in the modes whose work matrices are FP16 or BF16 (FP16,
 * BF16, FP16_SPLIT, FP8_FP16_SPLIT, FP8_BF16_SPLIT, FP32_EMU) without
 * deflation, adaptive depth or split_mask's B-only flag, a matrix of order
 * n <= 128 (tuning key "small_max") runs all of Algorithm 2 in one
 * workgroup: every such matrix of a call in one launch, which a batched call
 * runs on a side stream of the caller's stream beside the launch sequence of
 * its larger matrices (forked and joined by events; under capture before the
 * side stream exists, on the caller's stream). The rule depends only on
 * (n, mode, options), so a matrix takes the same path alone and in any batch.
 *
 * Graph capture (this call and psdproj_project / _ex / _batched_ex): a call
 * with the sizes, mode and options of the previous call on the same stream
 * issues kernel launches only and may be captured into a HIP graph; make the
 * call once uncaptured first. A batched call keeps its table of caller
 * pointers in a ring of 8 tables per (stream, sizes, mode): a call whose
 * pointers are in the ring uploads nothing, and a table that a captured call
 * used is never overwritten afterwards, so later calls with other pointers
 * (e.g. ping-pong iterate buffers) leave earlier graphs valid. While the
 * stream is capturing, a batched call whose pointers are not in the ring, or
 * any call that needs a new plan or more workspace, returns
 * PSDPROJ_ERR_UNSUPPORTED; so does an uncaptured call when all 8 tables are
 * held by captures. A captured graph uses the stream's workspace: a later call
 * on that stream with other sizes, mode or options, psdproj_release or
 * psdproj_tune invalidates it. */
int psdproj_project_batched(int count, const int64_t *n, const int64_t *ld,
                            const float *const *X, float *const *out, int mode,
                            psdproj_stream_t stream);

/* As psdproj_project_batched with options; info_dev (device memory, count
 * entries, may be NULL) receives each matrix's numerical status at index i
 * (entries of matrices with n[i] == 0 are not written). */
int psdproj_project_batched_ex(const psdproj_opts *opts, int count, const int64_t *n,
                               const int64_t *ld, const float *const *X, float *const *out,
                               psdproj_stream_t stream, psdproj_info *info_dev);

/* Device bytes of workspace a projection of size n in `mode` uses. */
size_t psdproj_workspace_bytes(int64_t n, int mode);

/* Number of n_p x n_p products (FP16-product equivalents) a projection runs:
 * 3 per stage + 1 for plain modes (22 half, 31 single); an FP16 split product
 * counts 3 (2 if one operand is split), an FP8_FP16_SPLIT split product 2
 * (1.5 if one operand is split). opts may be NULL (then `mode` defaults
 * apply). Returns -1 for bad options. */
double psdproj_gemm_count(const psdproj_opts *opts, int mode);

/* Host copy of the run-time coefficients of `mode` (rescale folded in):
 * abc[3 t + 0..2] = (a_t, b_t, c_t). Returns T, or -1 for a bad mode or when
 * cap < 3 T. */
int psdproj_coefficients(int mode, double *abc, int cap);

/* Free every cached workspace (synchronises the device). */
int psdproj_release(void);

const char *psdproj_status_string(int status);

/* Tuning hook (process-wide, not thread-safe against concurrent launches).
 * By default the products of matrices with n >= 5633 (FP16/BF16 modes) run
 * their whole rounds of 256 x 256 tiles (one workgroup per CU). The tiles of
 * a last partial round are cut into K-chunks that run side by side (FP32
 * partials summed in chunk order by a fixup) when they fill at most half the
 * CUs, else they run as 128 x 128 tiles; smaller matrices run 128 tiles.
 * Results are deterministic and do not depend on the other matrices of a
 * batch; they depend on the CU count and these settings only through the
 * rounding of the K-split tiles (every other tiling gives the same bits).
 * "gemm_tile" = 0 (automatic), 128 (128 tiles only) or 256 (256 tiles for
 * all such products, no tail split; the kernel-level entries use it when n_p
 * is a multiple of 256); "gemm_big_min" = n from which products use 256
 * tiles; "gemm_split_big" = mask of the split products that follow that rule
 * (bit 0 FP16/BF16 pairs, bit 1 FP8 pairs; default 3; the others run 128
 * tiles); "gemm_ksplit" = most K-chunks per tail tile (default 8; 1 never
 * splits); "gemm_tail_cus" = CU count the tail rule assumes (0: the
 * device's); "work_ld_pad" = elements added to the leading dimension of work
 * matrices whose padded order n_p >= 2048 is a multiple of 1024 (default 128;
 * multiple of 64; synchronises the device); "gemm_block" = H * 256 + W sets the blocking of the GEMM tile
 * schedule (H tile rows x W tile columns per block); "small_max" = largest
 * order of the one-workgroup path of small matrices (0..128, default 128; 0
 * sends every matrix through the launch sequence). Plans are rebuilt after a
 * change. Returns PSDPROJ_ERR_NOT_FOUND for unknown keys. */
int psdproj_tune(const char *key, int64_t value);

/* ---- autotuner ----------------------------------------------------------
 * psdproj_autotune: for each order in sizes[count] (1 <= n <= 65535) times
 * whole projections in `mode` of a random symmetric matrix of that order
 * (device-generated; the tuner allocates and frees it) under every candidate
 * tile policy of the order's size class (quarter octaves of n): 128 tiles
 * only, and for n >= 1024 outside FP32 also 256-tile rounds whose last
 * partial round runs as up to 1, 2, 4 or 8 K-chunks per tile. The fastest
 * becomes the class's policy for later plans of this process (in every mode
 * with the same work precision) and, when cache_path is not NULL, is written
 * to that text file (lines of other devices, modes and classes are kept).
 * Synchronises `stream`. The policies change results only through the
 * rounding of K-split tiles (single and batched calls of an order still agree
 * bitwise). psdproj_tune_load applies the lines of a cache file that match
 * the current device (GPU architecture and CU count) and returns how many, or
 * minus a status; the first plan of a process also applies the file named by
 * the environment variable PSDPROJ_TUNE_CACHE. psdproj_tune("class_choices_clear",
 * 0) drops all per-class policies. */
int psdproj_autotune(int mode, const int64_t *sizes, int count, const char *cache_path,
                     psdproj_stream_t stream);
int psdproj_tune_load(const char *path);

/* ---- serving: a continuous-batching request loop -------------------------
 * A server owns `slots` HIP streams (default priority) and a scheduler thread.
 * Requests are admitted in arrival order as soon as a slot is free and the
 * workspace the request needs fits under hbm_budget_bytes together with the
 * workspaces already held by the slots (later, smaller requests may pass a
 * blocked head request at most `max_bypass` times). Admitted work runs on the
 * slot's stream, so requests that arrive while others are on the GPU overlap
 * with them. Iterates stay in caller-owned HBM: X and out are device pointers
 * that must stay valid until the request completes. Results of a request do
 * not depend on the mix it runs in (tile shapes are a function of (n, mode)
 * only). Timestamps are host CLOCK_MONOTONIC nanoseconds; a request's latency
 * is end_ns - submit_ns, where end_ns is when the scheduler observed the
 * completion event. */
typedef struct psdproj_server psdproj_server;

typedef struct {
    size_t hbm_budget_bytes; /* 0 -> 200 GB */
    int slots;               /* concurrent streams, 0 -> 4 */
    int max_bypass;          /* 0 -> 8 */
    int fake_executor;       /* 1: no GPU work; a request "runs" for a modelled
                                time (tests of the scheduling logic on a CPU) */
    double fake_tflops;      /* fake executor speed (0 -> 500) */
    int coalesce_max_n;      /* requests of order <= this (0 -> 1024; < 0: never)
                                are admitted together with the queued requests of
                                the same mode and order <= this, up to 32 per
                                group, as one batched projection (results are
                                bitwise those of the request alone) */
} psdproj_serve_config;

typedef struct {
    int64_t n, ld;
    const float *X;  /* device, upper triangle read */
    float *out;      /* device */
    double target;   /* accuracy target when mode < 0: <= 1e-4 -> FP32_EMU,
                        otherwise FP8_FP16_SPLIT */
    int mode;        /* psdproj_mode, or -1 to choose from target */
    uint64_t tag;    /* caller's tag, echoed in the result */
} psdproj_request;

typedef struct {
    int status;      /* PSDPROJ_OK, _NONFINITE (input held Inf/NaN; out is NaN),
                        _REJECTED, _CANCELLED, _HIP, ... */
    int mode;
    uint64_t tag;
    int64_t submit_ns, start_ns, end_ns;
    int slot;
} psdproj_result;

typedef struct {
    uint64_t submitted, completed, rejected, cancelled, pending, running;
    double p50_ms, p99_ms, mean_ms, max_ms; /* latency of completed requests */
    double throughput_per_s;                /* completed / (last end - first submit) */
    size_t bytes_held, peak_bytes_held;     /* workspace held by the slots */
} psdproj_serve_statistics;

/* Create a server on the current device. NULL config -> defaults. */
int psdproj_serve_create(const psdproj_serve_config *cfg, psdproj_server **out);
/* Queue a request; *ticket identifies it. A request whose workspace alone
 * exceeds the budget is rejected (PSDPROJ_ERR_REJECTED, no ticket issued). */
int psdproj_serve_submit(psdproj_server *s, const psdproj_request *r, uint64_t *ticket);
/* Wait up to timeout_ns (< 0: forever) for a request; PSDPROJ_ERR_TIMEOUT if
 * it has not finished, PSDPROJ_ERR_NOT_FOUND for an unknown ticket. The
 * result is returned (and forgotten) once finished. */
int psdproj_serve_wait(psdproj_server *s, uint64_t ticket, int64_t timeout_ns, psdproj_result *res);
/* Non-blocking: PSDPROJ_ERR_PENDING while queued or running. */
int psdproj_serve_poll(psdproj_server *s, uint64_t ticket, psdproj_result *res);
/* Cancel a request that has not started (PSDPROJ_ERR_PENDING if it is running). */
int psdproj_serve_cancel(psdproj_server *s, uint64_t ticket);
int psdproj_serve_stats(psdproj_server *s, psdproj_serve_statistics *st);
/* Drain running work, cancel queued requests, free streams and workspaces. */
int psdproj_serve_destroy(psdproj_server *s);

/* ---- ADMM for SDP: the elementwise steps --------------------------------
 * The three-step ADMM of Section 4.2 (its ADMM equation) for SDPs whose
 * constraint map is the diagonal, A X = diag(X), so that A A^T = I and
 * A^T y = Diag(y) (the Max-Cut family):
 *     y = b / sigma - diag(X / sigma + S - C),   W = C - Diag(y) - X / sigma,
 *     S = Pi(W)  (any psdproj_project* call),    X = X + sigma (S + Diag(y) - C).
 * X, S, C, W: device FP32 n x n, column-major, leading dimension ld, both
 * triangles (caller-owned; the projection reads W's upper triangle and writes
 * both triangles of S). b, y: device FP64 vectors of n. Queued on `stream`;
 * the return value reports argument and launch errors only.
 * psdproj_admm_dual writes y and W (n <= 65535).
 * psdproj_admm_primal updates X in place and writes to res (device, at least
 * PSDPROJ_ADMM_RES_DOUBLES doubles; entries 8.. are its scratch):
 *     res[0] = ||diag(X) - b||_2, res[1] = ||Diag(y) + S - C||_F,
 *     res[2] = <C, X>, res[3] = b^T y, res[4] = ||b||_2, res[5] = ||C||_F,
 * from which the paper's surrogate residual (its three-term stopping test
 * before the precision switch) follows. Sums are FP64 in a fixed order. */
#define PSDPROJ_ADMM_GROUPS 512
#define PSDPROJ_ADMM_RES_DOUBLES (8 + 4 * PSDPROJ_ADMM_GROUPS)
int psdproj_admm_dual(int64_t n, int64_t ld, const float *X, const float *S, const float *C,
                      const double *b, double sigma, double *y, float *W, psdproj_stream_t stream);
int psdproj_admm_primal(int64_t n, int64_t ld, float *X, const float *S, const float *C,
                        const double *y, const double *b, double sigma, double *res,
                        psdproj_stream_t stream);

/* ---- product timing (tooling) ---------------------------------------------
 * psdproj_gemm_timing_start clears earlier records and brackets the launches
 * of every filter product of later projections (any stream, the device
 * current at the call) with two HIP events. psdproj_gemm_timing_stop stops
 * recording, waits for the recorded events and returns per product class
 * (index below, out[cap]) the number of products and their summed event time
 * in ms. The events add no device work; a product of a batched projection is
 * one bracket around all its matrices. */
enum {
    PSDPROJ_GEMM_PLAIN = 0,           /* unsplit operands, work-precision output */
    PSDPROJ_GEMM_PLAIN_SPLIT_OUT = 1, /* unsplit operands, split output          */
    PSDPROJ_GEMM_PAIR = 2,            /* split operands, work-precision output   */
    PSDPROJ_GEMM_PAIR_SPLIT_OUT = 3,  /* split operands, split output            */
    PSDPROJ_GEMM_FINAL = 4,           /* final product, unsplit                  */
    PSDPROJ_GEMM_PAIR_FINAL = 5,      /* final product, split                    */
    PSDPROJ_GEMM_CLASSES = 6
};
typedef struct {
    int64_t launches;
    double total_ms;
} psdproj_gemm_timing_entry;
int psdproj_gemm_timing_start(void);
int psdproj_gemm_timing_stop(psdproj_gemm_timing_entry *out, int cap);

/* ---- kernel-level entry points (used by tests and tooling) ---------------
 * psdproj_sym_gemm: D = alpha C0 + beta (L R) + gamma I on n_p x n_p
 * symmetric work matrices (column-major, leading dimension ld >= n_p,
 * n_p a multiple of 128) in dtype 0 = FP32, 1 = FP16, 2 = BF16. Only the upper
 * tiles are computed and mirrored. *lo arguments may be NULL (unsplit);
 * Dlo != NULL requests a split output. The product is queued on `stream` and
 * the call returns at once (launch errors only). The library keeps the
 * operand descriptor of the last call per device: a call whose pointers,
 * sizes or tile schedule differ synchronises the device before replacing it,
 * so repeated calls on the same buffers are bare kernel launches. */
int psdproj_sym_gemm(int dtype, int64_t n_p, int64_t ld, const void *L, const void *Llo,
                     const void *R, const void *Rlo, const void *C0, const void *C0lo,
                     float alpha, float beta, float gamma, void *D, void *Dlo,
                     psdproj_stream_t stream);

/* psdproj_sym_gemm_pair8: the same product on FP16 matrices whose split parts
 * are FP8 pairs (the PSDPROJ_MODE_FP8_FP16_SPLIT storage). For a split matrix
 * M with FP16 part M_hi, the code buffer (device, ld bytes per column, n_p
 * columns) holds the e4m3 codes of (M - M_hi) 2^(11+e), so that
 * M = M_hi + 2^-(11+e) decode(codes). The code of element (row i, column j)
 * is at byte 4 ld (j / 4) + 128 (i / 32) + 32 (j mod 4) + 16 ((i / 8) mod 2)
 * + 8 ((i / 16) mod 2) + (i mod 8): 32 rows of 4 columns fill one 128-byte
 * line, and each 16-byte chunk holds the K values one lane half of an FP16
 * MFMA fragment pair covers. The buffer holds n_p ld bytes. e_l, e_r, e_c0, e_d are the pair exponents of L, R,
 * C0 and D (|e| <= 40). Lx and Rx are both given (pair product: L_hi R_hi on
 * FP16 MFMAs plus both cross terms on FP8 MFMAs, with the codes of M_hi 2^e
 * formed in registers), Lx alone (one-sided product: L_hi R_hi plus the single
 * cross term L_lo R_hi, whose FP8 MFMAs take 64 K per instruction), or both
 * NULL; Rx without Lx is PSDPROJ_ERR_UNSUPPORTED. C0x != NULL adds the pair
 * correction of C0; Dx != NULL writes D's codes. Queued on `stream` like
 * psdproj_sym_gemm. */
int psdproj_sym_gemm_pair8(int64_t n_p, int64_t ld, const void *L, const void *Lx,
                           const void *R, const void *Rx, const void *C0, const void *C0x,
                           float alpha, float beta, float gamma, void *D, void *Dx,
                           int e_l, int e_r, int e_c0, int e_d, psdproj_stream_t stream);

/* psdproj_sym_gemm_pair8_bf16: the same on BF16 hi parts (the
 * PSDPROJ_MODE_FP8_BF16_SPLIT storage): the codes hold e4m3((M - M_hi)
 * 2^(8+e)), so that M = M_hi + 2^-(8+e) decode(codes); arguments, layout and
 * errors as psdproj_sym_gemm_pair8. */
int psdproj_sym_gemm_pair8_bf16(int64_t n_p, int64_t ld, const void *L, const void *Lx,
                                const void *R, const void *Rx, const void *C0, const void *C0x,
                                float alpha, float beta, float gamma, void *D, void *Dx,
                                int e_l, int e_r, int e_c0, int e_d, psdproj_stream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* PSDPROJ_H */

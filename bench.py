#!/usr/bin/env python3
"""Benchmark of the PSD-cone projection on one MI355X.

Workload: one dense symmetric n = 10,000 matrix (the paper's headline size),
GOE spectrum X = (G + G^T) / sqrt(2n), G seeded N(0, 1) (or the rank-500 PSD +
noise matrix with --input lowrank), FP32 in HBM before the timed region.
A "step" is one full projection: Lanczos bound, rescale/cast, T filter stages,
final combine, in the chosen precision form.

Printed (one JSON line): ms per projection, its relative error against an
FP64 eigen-projection (rocSOLVER dsyevd on the same GPU), the roofline of the
dominant kernel (the plain symmetric stage GEMM, its launches inside one more
projection bracketed by HIP events on the projection's stream), the rocSOLVER
ssyevd/dsyevd projection times, and the FP64 CPU oracle timed on a bounded
sample of the same n = 10,000 input (its bound, one filter stage and the final
combine, measured; the other stages counted at the measured stage time).
"""
from __future__ import annotations

import argparse
import ctypes
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "ms per n=10k PSD projection at ≤1e-3 rel err; batched proj/s + p99 latency"
PEAK = {"fp16": 2.5e15, "bf16": 2.5e15, "fp16_split": 2.5e15, "fp8_fp16_split": 2.5e15, "fp32_emu": 2.5e15,
        "fp32": 157.3e12, "ns_fp16": 2.5e15, "ns_fp32": 157.3e12, "fp8_bf16_split": 2.5e15}
DTYPE_NAME = {"fp16": "fp16", "bf16": "bf16", "fp16_split": "fp16", "fp8_fp16_split": "fp16+fp8",
              "fp32_emu": "fp16", "fp32": "fp32", "ns_fp16": "fp16", "ns_fp32": "fp32",
              "fp8_bf16_split": "bf16+fp8"}


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


# ---------------------------------------------------------------------------
# rocSOLVER eigen-projection (comparison leg, library calls)
# ---------------------------------------------------------------------------
class RocSolver:
    def __init__(self, stream):
        self.blas = ctypes.CDLL("librocblas.so")
        self.sol = ctypes.CDLL("librocsolver.so")
        self.h = ctypes.c_void_p()
        assert self.blas.rocblas_create_handle(ctypes.byref(self.h)) == 0
        assert self.blas.rocblas_set_stream(self.h, ctypes.c_void_p(stream.cuda_stream)) == 0

    def projection(self, X, dtype):
        """Q diag(max(w, 0)) Q^T with syevd (rocblas_evect_original, upper)."""
        import torch
        n = X.shape[0]
        A = X.to(dtype).contiguous().clone()
        w = torch.empty(n, dtype=dtype, device=X.device)
        E = torch.empty(n, dtype=dtype, device=X.device)
        info = torch.zeros(1, dtype=torch.int32, device=X.device)
        fn = self.sol.rocsolver_dsyevd if dtype == torch.float64 else self.sol.rocsolver_ssyevd
        st = fn(self.h, 211, 121, n, ctypes.c_void_p(A.data_ptr()), n, ctypes.c_void_p(w.data_ptr()),
                ctypes.c_void_p(E.data_ptr()), ctypes.c_void_p(info.data_ptr()))
        assert st == 0, st
        # A holds eigenvectors in columns of the column-major buffer = rows of A
        Q = A  # row i of the torch tensor = eigenvector i
        P = (Q.t() * torch.clamp(w, min=0)) @ Q
        return P, int(info.item())


def time_rocsolver(rs, X, dtype, reps=1):
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        P, info = rs.projection(X, dtype)
    torch.cuda.synchronize()
    return P, (time.perf_counter() - t0) / reps * 1e3, info


# ---------------------------------------------------------------------------
def measured_traffic(kernel_mode):
    """HBM bytes per launch of the plain stage product from the committed
    counter summary (FETCH_SIZE and WRITE_SIZE passes, each scaled by the same
    counter on a device copy of known size), or None when the summary is for
    another mode or the kernel's sources changed since it was taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "gemm_plain_n10000_traffic.json")
    if kernel_mode != "fp8_fp16_split" or not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    h = hashlib.md5()
    for src in rec["kernel_sources"]:
        with open(os.path.join(ROOT, src), "rb") as f:
            h.update(f.read())
    if h.hexdigest() != rec["kernel_sources_md5"]:
        return None
    return rec


def gemm_roofline(X, out, opts, n, mode, stream):
    """Roofline of the dominant kernel, the plain symmetric stage GEMM, measured
    on the projection's own launches: one more projection runs with every
    filter product bracketed by HIP events on its stream; achieved = the
    algorithmic n^2 (n + 1) flops of one product (the upper triangle of an
    n x n product) / the average event time of the plain stage products.
    The other product classes are reported beside it."""
    import torch
    from paper_2507_09165_amd import psdproj as P
    P.gemm_timing_start()
    P.project_ex(X, out, stream=stream, info=False, **opts)
    cls = P.gemm_timing_stop()
    torch.cuda.synchronize()
    ms = cls["plain"]["avg_ms"]
    flops = float(n) * n * (n + 1)
    achieved = flops / (ms * 1e-3)
    peak = PEAK[mode]
    dt = DTYPE_NAME[mode]
    classes = {k: v for k, v in cls.items() if v["launches"]}
    for v in classes.values():
        v["tflops_per_product_equivalent"] = flops / (v["avg_ms"] * 1e-3) / 1e12
    tr = measured_traffic(mode) if n == 10000 else None
    res = {"kernel": f"gemm_sym_kernel<{dt}, plain stage product> (in-projection products; from n = 5633 one "
                     "product is a launch of 256 x 256 tiles over whole rounds, a launch of the last round's "
                     "tiles cut into K-chunks, and their fixup)",
           "bound": "mfma",
           "achieved": achieved / 1e12, "peak": peak / 1e12, "unit": "TFLOP/s", "frac": achieved / peak,
           "traffic": tr["traffic_bytes_per_launch"] if tr else None, "ms_per_launch": ms, "flops_per_launch": flops,
           "launches": cls["plain"]["launches"], "product_classes": classes}
    if tr:
        res["traffic_detail"] = {"unit": "bytes per launch", "fetch": tr["fetch_bytes_per_launch"],
                                 "write": tr["write_bytes_per_launch"],
                                 "algorithmic": tr["algorithmic_bytes_per_launch"],
                                 "source": "profiles/gemm_plain_n10000_traffic.md"}
    return res


def _host_cpu():
    """Threads this process may run on (nproc) and the host's CPU model."""
    import subprocess
    try:
        nproc = len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        nproc = os.cpu_count() or 1
    model = ""
    try:
        for line in subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout.splitlines():
            if line.startswith("Model name:"):
                model = line.split(":", 1)[1].strip()
    except Exception:  # noqa: BLE001
        pass
    return nproc, model


def cpu_baseline(mode, X32, stages_timed=1):
    """The FP64 oracle (Algorithm 2 in numpy) timed on the host on the timed
    input itself, as a bounded sample: its whole spectral bound, `stages_timed`
    of its T filter stages and its final combine, each measured; the other
    stages are the same three n x n products on the same sizes and are counted
    at the measured per-stage time. value = t_bound + T t_stage + t_final."""
    import oracle
    try:
        from threadpoolctl import threadpool_info
        threads = max([int(d.get("num_threads", 1)) for d in threadpool_info()] or [1])
    except Exception:  # noqa: BLE001
        threads = None
    nproc, model = _host_cpu()
    Xs = oracle.sym_from_upper(X32.astype(np.float64))
    t0 = time.perf_counter()
    b = oracle.spectral_bound(Xs)
    t_bound = time.perf_counter() - t0
    lam = b["lam"]
    rows = oracle.stage_rows(mode)
    X0 = Xs / lam
    Y = X0
    t_st = []
    for a_, b_, c_ in rows[:stages_timed]:
        t0 = time.perf_counter()
        Y = oracle.filter_stage(Y, a_, b_, c_)
        t_st.append(time.perf_counter() - t0)
    t0 = time.perf_counter()
    oracle.final_combine(X0, Y, lam)
    t_final = time.perf_counter() - t0
    T = rows.shape[0]
    t_stage = sum(t_st) / len(t_st)
    total = t_bound + T * t_stage + t_final
    n = X32.shape[0]
    return {"value": total * 1e3, "unit": "ms", "cores": threads if threads else nproc, "kind": "oracle",
            "nproc": nproc, "cpu_model": model,
            "sample": f"FP64 oracle on the timed n={n} input: spectral bound {t_bound:.2f} s, "
                      f"{stages_timed} of {T} filter stages {sum(t_st):.2f} s (3 products each), final combine "
                      f"{t_final:.2f} s, all measured; the other {T - stages_timed} stages counted at the "
                      f"measured per-stage time"}


def batched_leg(steps=3, warmup=1, count=256, mode="fp8_bf16_split"):
    """256 independent GOE blocks, n log-uniform in [32, 1024] (seed 7): one
    psdproj_project_batched call per step; projections per second. BF16 bulk
    with the stage 1-4 corrections as FP8 codes (every block within 5e-3 of
    the FP64 oracle, tested)."""
    import torch
    from paper_2507_09165_amd import inputs
    from paper_2507_09165_amd import psdproj as P
    sizes = inputs.batch_sizes(count, 7)
    Xs = [torch.from_numpy(B).cuda() for B in inputs.batch_blocks(sizes, 7)]
    outs = [torch.empty_like(X) for X in Xs]
    st = torch.cuda.current_stream()
    for _ in range(warmup):
        P.project_batched(Xs, outs, mode=mode, stream=st)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record(st)
    for _ in range(steps):
        P.project_batched(Xs, outs, mode=mode, stream=st)
    ev1.record(st)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / steps
    wall = (time.perf_counter() - t0) * 1e3 / steps
    # the same call captured once in a HIP graph and replayed; every replay's
    # outputs are checked bitwise against the eager call's
    ref = [o.clone() for o in outs]
    gs = torch.cuda.Stream()
    P.project_batched(Xs, outs, mode=mode, stream=gs)
    gs.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=gs):
        P.project_batched(Xs, outs, mode=mode, stream=gs)
    for o in outs:
        o.fill_(float("nan"))
    torch.cuda.synchronize()
    graph.replay()
    torch.cuda.synchronize()
    replay_equal = all(torch.equal(o, r) for o, r in zip(outs, ref))
    # replays timed by the host clock around a device synchronisation (events
    # recorded on the launch stream have bracketed less than the replayed
    # graph's work when it forks to other streams); the event time beside it
    t0 = time.perf_counter()
    ev0.record(gs)
    for _ in range(steps):
        with torch.cuda.stream(gs):
            graph.replay()
    ev1.record(gs)
    torch.cuda.synchronize()
    gms = (time.perf_counter() - t0) * 1e3 / steps
    gms_ev = ev0.elapsed_time(ev1) / steps
    replay_equal = replay_equal and all(torch.equal(o, r) for o, r in zip(outs, ref))
    del graph
    flops = sum(P.gemm_count(mode) * float(n) * n * (n + 1) for n in sizes)
    return {"workload": f"{count} GOE blocks, n log-uniform in [32, 1024] (seed 7), {mode}",
            "ms_per_batch": ms, "host_ms_per_batch": wall, "proj_per_s": count / (ms * 1e-3),
            "algorithmic_tflops": flops / (ms * 1e-3) / 1e12, "n_min": int(sizes.min()),
            "n_max": int(sizes.max()), "steps": steps,
            "graph": {"ms_per_batch": gms, "proj_per_s": count / (gms * 1e-3), "event_ms_per_batch": gms_ev,
                      "outputs_equal_eager": replay_equal}}


def serving_leg(num=2000, rho=(0.5, 0.8, 0.95), slots=4, seed=11, sat_num=400):
    """Serving stream: Poisson arrivals at rho * mu (mu: the measured
    saturated throughput of the same stream). Every request draws its own
    order n log-uniform in [64, 8192] and projects an ADMM-like iterate
    Y_1 = Y_0 + sqrt(1e-3) GOE_1 of a GOE start Y_0 of that order (all iterates
    and outputs resident in HBM before the run); its accuracy target is 1e-3
    (FP8_FP16_SPLIT) or 1e-5 (FP32_EMU), drawn 70/30; admission under a 200 GB
    budget, queued requests of order <= 1024 coalesced into batched launches.
    Reports p50/p99 latency and projections/s per rho."""
    import torch
    from paper_2507_09165_amd import psdproj as P
    rng = np.random.default_rng(seed)
    g = torch.Generator(device="cuda").manual_seed(seed)
    ns = np.clip(np.rint(np.exp(rng.uniform(np.log(64), np.log(8192), size=num))), 64, 8192).astype(int)
    targets = np.where(rng.uniform(size=num) < 0.7, 1e-3, 1e-5)

    def goe_dev(n):
        G = torch.randn(n, n, device="cuda", generator=g)
        return (G + G.t()) * (1.0 / np.sqrt(2.0 * n))

    Xs = [goe_dev(int(n)) + np.sqrt(1e-3) * goe_dev(int(n)) for n in ns]
    outs = [torch.empty_like(X) for X in Xs]
    torch.cuda.synchronize()

    def run(k, rate):
        gaps = rng.exponential(1.0 / rate, size=k) if rate else np.zeros(k)
        with P.Server(slots=slots) as srv:
            tks = []
            t0 = time.perf_counter()
            due = t0
            for i in range(k):
                due += gaps[i]
                dt = due - time.perf_counter()
                if dt > 0:
                    time.sleep(dt)
                tks.append(srv.submit(X=Xs[i], out=outs[i], target=float(targets[i]), tag=i))
            res = [srv.wait(tk, timeout_s=600) for tk in tks]
            stt = srv.stats()
        assert all(r["status"] == 0 for r in res)
        stt["launches"] = len({(r["slot"], r["start_ns"]) for r in res})
        return stt

    run(64, 0)  # warm the slots' workspaces and plans
    sat = run(sat_num, 0)
    mu = sat["throughput_per_s"]
    res = {"workload": f"{num} requests per rate, each an ADMM-like iterate of its own order n log-uniform in "
                       f"[64, 8192] (seed {seed}), Poisson arrivals, 70% target 1e-3 (fp8_fp16_split) / "
                       f"30% 1e-5 (fp32_emu), {slots} slots, 200 GB budget, coalescing n <= 1024",
           "n_median": int(np.median(ns)), "n_max": int(ns.max()),
           "saturated_proj_per_s": mu, "saturated_requests": sat_num, "runs": []}
    for r_ in rho:
        log(f"serving rho {r_}")
        stt = run(num, r_ * mu)
        res["runs"].append({"rho": r_, "offered_per_s": r_ * mu, "proj_per_s": stt["throughput_per_s"],
                            "p50_ms": stt["p50_ms"], "p99_ms": stt["p99_ms"], "mean_ms": stt["mean_ms"],
                            "max_ms": stt["max_ms"], "requests": int(stt["completed"]),
                            "launches": stt["launches"], "peak_workspace_gb": stt["peak_bytes_held"] / 1e9})
    del Xs, outs
    torch.cuda.empty_cache()
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=10000)
    ap.add_argument("--mode", default="fp8_fp16_split", choices=sorted(PEAK))
    ap.add_argument("--input", default="goe", choices=["goe", "lowrank"])
    ap.add_argument("--split-mask", type=lambda s: int(s, 0), default=None)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-rocsolver", action="store_true")
    ap.add_argument("--no-check", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--batched-only", action="store_true",
                    help="run only the batched leg (256 blocks) and print its JSON")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--serve-requests", type=int, default=2000)
    ap.add_argument("--no-compare", action="store_true",
                    help="skip the other forms (plain FP32, FP32_EMU, FP16, Newton-Schulz) at the same n")
    ap.add_argument("--copy-probe", type=int, default=0,
                    help="only copy this many bytes device-to-device 3 times (counter calibration) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one MI355X; this build has no multi-GPU path (--gpus must be 1).",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2507_09165_amd import inputs
    from paper_2507_09165_amd import psdproj as P

    if args.copy_probe:
        # a plain device copy of known size: the reference point that scales
        # the FETCH_SIZE / WRITE_SIZE counters to bytes
        a = torch.empty(args.copy_probe // 4, dtype=torch.float32, device="cuda").fill_(1.0)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": args.copy_probe, "launches": 3}), flush=True)
        return

    P.lib()
    if args.batched_only:
        print(json.dumps(batched_leg()), flush=True)
        return
    dev = torch.device("cuda:0")
    n = args.n
    log("generating input", args.input, n)
    if args.input == "goe":
        X32 = inputs.goe(n, 4)
    else:
        X32 = inputs.lowrank_noise(n, 5, 6)
    X = torch.from_numpy(X32).to(dev)
    X32_host = X32 if not args.no_cpu else None
    del X32
    out = torch.empty_like(X)
    st = torch.cuda.current_stream()
    opts = {"mode": args.mode, "split_mask": args.split_mask}

    log("warmup", args.warmup)
    for _ in range(args.warmup):
        P.project_ex(X, out, stream=st, info=False, **opts)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(st)
    for _ in range(args.steps):
        P.project_ex(X, out, stream=st, info=False, **opts)
    ev1.record(st)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) * 1e3 / args.steps
    ms = ev0.elapsed_time(ev1) / args.steps
    log(f"projection: {ms:.3f} ms/step (wall {wall:.3f})")

    _, info_t = P.project_ex(X, out, stream=st, **opts)
    torch.cuda.synchronize()
    info = P.read_info(info_t)

    res = {"metric": METRIC, "value": ms, "unit": "ms", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": False, "scaling": "weak",
           "vs_baseline": None, "dtype": DTYPE_NAME[args.mode], "data": "synthetic",
           "config": {"workload": f"single dense symmetric n={n} projection, "
                                  f"{'GOE (seed 4)' if args.input == 'goe' else 'rank-500 PSD + noise (seeds 5, 6)'}",
                      "n": n, "mode": args.mode, "input": args.input,
                      "gemm_equivalents": P.gemm_count(**opts)},
           "lambda": info["lambda"], "lanczos_steps": info["lanczos_steps"]}
    flops = P.gemm_count(**opts) * float(n) * n * (n + 1)
    res["algorithmic_tflops"] = flops / (ms * 1e-3) / 1e12

    log("gemm roofline")
    res["roofline"] = gemm_roofline(X, out, opts, n, args.mode, st)

    if not args.no_rocsolver or not args.no_check:
        rs = RocSolver(st)
        log("rocsolver dsyevd")
        P64, t64, inf64 = time_rocsolver(rs, X, torch.float64)
        roc = {"dsyevd_projection_ms": t64, "dsyevd_info": inf64}
        if not args.no_check:
            err = torch.linalg.norm(out.double() - P64) / torch.linalg.norm(P64)
            res["rel_err_vs_fp64_evd"] = float(err)
            log("rel err vs FP64 EVD", float(err))
        if not args.no_compare:
            # the other forms on the same input and GPU: ms per projection and
            # relative error against the FP64 eigen-projection
            cmp = {}
            for m in ("fp32", "fp32_emu", "fp16", "fp16_split", "bf16", "fp8_bf16_split", "ns_fp16", "ns_fp32"):
                log("compare", m)
                P.project_ex(X, out, stream=st, info=False, mode=m)
                torch.cuda.synchronize()
                reps = 2
                ev0.record(st)
                for _ in range(reps):
                    P.project_ex(X, out, stream=st, info=False, mode=m)
                ev1.record(st)
                torch.cuda.synchronize()
                e = torch.linalg.norm(out.double() - P64) / torch.linalg.norm(P64)
                cmp[m] = {"ms": ev0.elapsed_time(ev1) / reps, "rel_err_vs_fp64_evd": float(e),
                          "gemm_equivalents": P.gemm_count(mode=m)}
            res["forms"] = cmp
        del P64
        if not args.no_rocsolver:
            log("rocsolver ssyevd")
            P32, t32, inf32 = time_rocsolver(rs, X, torch.float32)
            roc.update({"ssyevd_projection_ms": t32, "ssyevd_info": inf32})
            del P32
        res["rocsolver"] = roc
    res["paper_context"] = {"b200_fp16_ms": 54.8, "b200_fp32_emulated_ms": 416.0, "n": 10000}
    del X, out
    torch.cuda.empty_cache()
    if not args.no_batched:
        log("batched leg")
        res["batched"] = batched_leg()
    if not args.no_serve:
        log("serving leg")
        res["serving"] = serving_leg(num=args.serve_requests)
    if not args.no_cpu:
        log("cpu baseline")
        res["cpu_baseline"] = cpu_baseline(args.mode, X32_host)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()

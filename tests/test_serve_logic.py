"""Scheduling logic of the serving loop on the CPU (fake executor: requests
'run' for a modelled time, no GPU work). Covers admission under the HBM
budget, slot concurrency, FIFO order with bounded bypass, rejection,
cancellation, polling and the latency statistics."""
import time

import pytest

from paper_2507_09165_amd import psdproj as P

GB = 1 << 30


def test_all_requests_complete_and_stats():
    with P.Server(slots=4, fake_executor=True, fake_tflops=50.0) as s:
        tks = [s.submit(n=200 + 10 * i, target=1e-3, tag=i) for i in range(40)]
        res = [s.wait(t, timeout_s=30) for t in tks]
        assert all(r["status"] == 0 for r in res)
        assert [r["tag"] for r in res] == list(range(40))
        assert all(r["submit_ns"] <= r["start_ns"] <= r["end_ns"] for r in res)
        st = s.stats()
        assert st["completed"] == 40 and st["pending"] == 0 and st["running"] == 0
        assert 0 < st["p50_ms"] <= st["p99_ms"] <= st["max_ms"]
        assert st["throughput_per_s"] > 0


def test_slots_bound_concurrency_and_overlap():
    with P.Server(slots=3, fake_executor=True, fake_tflops=2.0, coalesce_max_n=-1) as s:  # ~10-20 ms each
        tks = [s.submit(n=1000, target=1e-3) for _ in range(9)]
        res = [s.wait(t, timeout_s=60) for t in tks]
    events = sorted([(r["start_ns"], 1) for r in res] + [(r["end_ns"], -1) for r in res])
    live = peak = 0
    for _, d in events:
        live += d
        peak = max(peak, live)
    assert peak == 3                      # never more than the slot count
    assert res[1]["start_ns"] < res[0]["end_ns"]   # later arrivals overlap running work
    assert {r["slot"] for r in res} == {0, 1, 2}


def test_fifo_order_when_unconstrained():
    with P.Server(slots=1, fake_executor=True, fake_tflops=100.0) as s:
        tks = [s.submit(n=300, tag=i) for i in range(10)]
        res = [s.wait(t, timeout_s=30) for t in tks]
    starts = [r["start_ns"] for r in res]
    assert starts == sorted(starts)


def test_request_larger_than_budget_is_rejected():
    ws = P.workspace_bytes(4000, "fp16_split")
    with P.Server(hbm_budget_bytes=ws - 1, fake_executor=True) as s:
        with pytest.raises(P.PsdprojError) as e:
            s.submit(n=4000, target=1e-3)
        assert e.value.status == 5
        t = s.submit(n=100, target=1e-3)
        assert s.wait(t, timeout_s=10)["status"] == 0
        assert s.stats()["rejected"] == 1


def test_budget_limits_held_workspace():
    ws_big = P.workspace_bytes(3000, "fp16_split")
    budget = int(2.5 * ws_big)
    with P.Server(hbm_budget_bytes=budget, slots=8, fake_executor=True, fake_tflops=5.0) as s:
        tks = [s.submit(n=3000, target=1e-3) for _ in range(8)]
        res = [s.wait(t, timeout_s=120) for t in tks]
        st = s.stats()
    assert all(r["status"] == 0 for r in res)
    assert st["peak_bytes_held"] <= budget
    # at most two of these fit at once
    events = sorted([(r["start_ns"], 1) for r in res] + [(r["end_ns"], -1) for r in res])
    live = peak = 0
    for _, d in events:
        live += d
        peak = max(peak, live)
    assert peak <= 2


def test_small_requests_bypass_blocked_head_boundedly():
    ws_big = P.workspace_bytes(6000, "fp16_split")
    with P.Server(hbm_budget_bytes=ws_big, slots=4, max_bypass=3, fake_executor=True,
                  fake_tflops=20.0) as s:
        first = s.submit(n=3000, tag=0)            # holds part of the budget
        big = s.submit(n=6000, tag=1)              # must wait for `first`
        smalls = [s.submit(n=64, tag=10 + i) for i in range(10)]
        r_big = s.wait(big, timeout_s=120)
        r_small = [s.wait(t, timeout_s=120) for t in smalls]
        s.wait(first, timeout_s=120)
    passed = [r for r in r_small if r["start_ns"] < r_big["start_ns"]]
    assert len(passed) <= 3


def test_cancel_pending_and_poll():
    with P.Server(slots=1, fake_executor=True, fake_tflops=1.0) as s:
        a = s.submit(n=2000)        # long
        b = s.submit(n=2000, tag=7)
        t0 = time.time()
        while s.stats()["running"] < 1:  # wait until the scheduler admitted `a`
            assert time.time() - t0 < 10
            time.sleep(0.001)
        assert s.poll(a) is None    # running
        assert s.cancel(b) == 0
        rb = s.wait(b, timeout_s=5)
        assert rb["status"] == 6 and rb["tag"] == 7
        assert s.cancel(a) == 9     # running: cannot cancel
        assert s.wait(a, timeout_s=60)["status"] == 0
        with pytest.raises(P.PsdprojError):
            s.wait(a)               # already collected


def test_wait_timeout():
    with P.Server(slots=1, fake_executor=True, fake_tflops=0.5) as s:
        a = s.submit(n=2500)
        with pytest.raises(P.PsdprojError) as e:
            s.wait(a, timeout_s=0.001)
        assert e.value.status == 7
        s.wait(a, timeout_s=120)


def test_destroy_cancels_queued():
    s = P.Server(slots=1, fake_executor=True, fake_tflops=1.0)
    for _ in range(5):
        s.submit(n=1500)
    t0 = time.time()
    s.close()
    assert time.time() - t0 < 30


def test_mode_from_target():
    with P.Server(slots=2, fake_executor=True) as s:
        a = s.submit(n=100, target=1e-5)
        b = s.submit(n=100, target=1e-3)
        assert s.wait(a, 10)["mode"] == 4      # FP32_EMU (FP32-level operands on FP16 pairs)
        assert s.wait(b, 10)["mode"] == 5      # FP8_FP16_SPLIT


def test_small_queued_requests_coalesce_into_one_launch():
    """Requests queued behind a long one, of order <= coalesce_max_n and one
    mode, start together on one slot (one batched projection); a request of
    another mode or a larger order is not taken into the group."""
    with P.Server(slots=1, fake_executor=True, fake_tflops=5.0) as s:
        big = s.submit(n=3000, target=1e-3)
        time.sleep(0.05)                      # the big request is running
        small = [s.submit(n=100 + 7 * i, target=1e-3, tag=i) for i in range(10)]
        other = s.submit(n=150, target=1e-5)  # another mode
        large = s.submit(n=1500, target=1e-3)  # above coalesce_max_n
        rb = s.wait(big, timeout_s=60)
        rs = [s.wait(t, timeout_s=60) for t in small]
        ro, rl = s.wait(other, timeout_s=60), s.wait(large, timeout_s=60)
    assert all(r["status"] == 0 for r in rs + [rb, ro, rl])
    assert len({r["start_ns"] for r in rs}) == 1 and rs[0]["start_ns"] >= rb["end_ns"]
    assert len({r["end_ns"] for r in rs}) == 1
    assert ro["start_ns"] != rs[0]["start_ns"] and rl["start_ns"] != rs[0]["start_ns"]


def test_coalescing_off_and_group_cap():
    with P.Server(slots=1, fake_executor=True, fake_tflops=5.0, coalesce_max_n=-1) as s:
        big = s.submit(n=3000, target=1e-3)
        time.sleep(0.05)
        rs = [s.wait(t, timeout_s=60) for t in [s.submit(n=100, target=1e-3) for _ in range(5)]]
        s.wait(big, timeout_s=60)
    assert len({r["start_ns"] for r in rs}) == 5
    with P.Server(slots=1, fake_executor=True, fake_tflops=5.0) as s:
        big = s.submit(n=3000, target=1e-3)
        time.sleep(0.05)
        rs = [s.wait(t, timeout_s=60) for t in [s.submit(n=64, target=1e-3) for _ in range(40)]]
        s.wait(big, timeout_s=60)
    starts = sorted({r["start_ns"] for r in rs})
    assert len(starts) == 2   # 32 per group at most: 32 + 8


def test_group_shrinks_to_fit_the_budget():
    ws1 = P.workspace_bytes(1000, "fp8_fp16_split")
    with P.Server(slots=1, fake_executor=True, fake_tflops=5.0, hbm_budget_bytes=int(2.5 * ws1)) as s:
        big = s.submit(n=1000, target=1e-3)
        time.sleep(0.02)
        rs = [s.wait(t, timeout_s=60) for t in [s.submit(n=1000, target=1e-3) for _ in range(8)]]
        s.wait(big, timeout_s=60)
        assert s.stats()["peak_bytes_held"] <= int(2.5 * ws1)
    assert all(r["status"] == 0 for r in rs)
    assert len({r["start_ns"] for r in rs}) >= 4   # groups of at most two

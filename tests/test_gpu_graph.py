"""Projections captured in a HIP graph (through torch.cuda.graph): every
replay, with eager library work between replays, gives the eager result
bitwise; calls that would need a host-side wait (new batch pointers, a new
plan) are refused while capturing."""
import pytest

from paper_2507_09165_amd import inputs
from paper_2507_09165_amd import psdproj as P
from gpu_util import say, to_dev

pytestmark = pytest.mark.gpu


def test_graph_replays_batched_and_single():
    import torch
    say("graph capture")
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    sizes = [40, 129, 300, 700]
    Xs = [to_dev(inputs.goe(n, 90 + n)) for n in sizes]
    outs = [torch.empty_like(X) for X in Xs]
    X1 = to_dev(inputs.goe(900, 98))
    o1 = torch.empty_like(X1)
    Xe = to_dev(inputs.goe(500, 99))
    oe = torch.empty_like(Xe)
    torch.cuda.synchronize()
    # uncaptured first (plans, workspaces and the batch's I/O table); each
    # stream keeps the plan of its own call
    P.project_batched(Xs, outs, mode="bf16", stream=s1)
    P.project(X1, o1, mode="fp8_fp16_split", stream=s2)
    torch.cuda.synchronize()
    ref = [o.clone() for o in outs]
    ref1 = o1.clone()
    g1, g2 = torch.cuda.CUDAGraph(), torch.cuda.CUDAGraph()
    with torch.cuda.graph(g1, stream=s1):
        P.project_batched(Xs, outs, mode="bf16", stream=s1)
    with torch.cuda.graph(g2, stream=s2):
        P.project(X1, o1, mode="fp8_fp16_split", stream=s2)
    for rep in range(3):
        for o in outs + [o1]:
            o.fill_(-1.0)
        torch.cuda.synchronize()
        g1.replay()
        g2.replay()
        torch.cuda.synchronize()
        for o, r in zip(outs, ref):
            assert torch.equal(o, r), rep
        assert torch.equal(o1, ref1), rep
        # eager projections on another stream between replays
        P.project(Xe, oe, mode="fp16")
        torch.cuda.synchronize()
    say("  3 replays equal")


def test_capture_refuses_new_batch_pointers():
    import torch
    s = torch.cuda.Stream()
    Xs = [to_dev(inputs.goe(n, 60 + n)) for n in (64, 200)]
    outs = [torch.empty_like(X) for X in Xs]
    torch.cuda.synchronize()
    P.project_batched(Xs, outs, mode="fp16", stream=s)
    s.synchronize()
    new_outs = [torch.empty_like(X) for X in Xs]
    g = torch.cuda.CUDAGraph()
    with pytest.raises(P.PsdprojError):
        with torch.cuda.graph(g, stream=s):
            P.project_batched(Xs, new_outs, mode="fp16", stream=s)
    torch.cuda.synchronize()
    # a call that would build a new plan (another size) is refused as well
    g2 = torch.cuda.CUDAGraph()
    with pytest.raises(P.PsdprojError):
        with torch.cuda.graph(g2, stream=s):
            P.project_batched(Xs[:1], outs[:1], mode="fp16", stream=s)
    torch.cuda.synchronize()
    # the stream still works uncaptured, with the new pointers
    P.project_batched(Xs, new_outs, mode="fp16", stream=s)
    s.synchronize()
    for a, b in zip(outs, new_outs):
        assert torch.equal(a, b)


def test_graph_survives_eager_calls_with_other_pointers():
    """Ping-pong buffers: a graph captured on outputs A keeps writing A after
    an eager call on the same stream wrote outputs B (other pointers, same
    sizes): the eager call must not overwrite the table the graph reads."""
    import torch
    s = torch.cuda.Stream()
    sizes = [64, 200, 333]
    Xs = [to_dev(inputs.goe(n, 80 + n)) for n in sizes]
    A = [torch.empty_like(X) for X in Xs]
    B = [torch.empty_like(X) for X in Xs]
    torch.cuda.synchronize()
    P.project_batched(Xs, A, mode="fp16", stream=s)
    s.synchronize()
    ref = [a.clone() for a in A]
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        P.project_batched(Xs, A, mode="fp16", stream=s)
    for rep in range(3):
        P.project_batched(Xs, B, mode="fp16", stream=s)  # eager, new pointers
        s.synchronize()
        for b, r in zip(B, ref):
            assert torch.equal(b, r), rep
        for b in B:
            b.fill_(-7.0)
        for a in A:
            a.fill_(-1.0)
        torch.cuda.synchronize()
        with torch.cuda.stream(s):
            g.replay()
        s.synchronize()
        for a, r in zip(A, ref):
            assert torch.equal(a, r), rep
        for b in B:
            assert torch.all(b == -7.0), rep
    say("  graph kept its pointers across 3 eager calls with others")

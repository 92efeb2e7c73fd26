"""jk_vjp under HIP graph capture (torch.cuda.graph).  The derivative runs on
the caller's stream and a second stream of the library, joined by events; a
captured call must replay the same products.  The workload is the nao=500,
naux=2000 set of 8 densities of rank 40 (4 derivative chunks, so the event
chain between the two streams repeats).  Each of three replays, with eager
work and synchronisation in between, is compared bit for bit with the eager
call (whose own parity with the oracle is covered by test_gpu_vjp.py and
test_gpu_large.py).
"""
import pytest

from paper_2608_06536_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def test_vjp_graph_capture_replays():
    from paper_2608_06536_amd import jk
    p = synth.config(4)
    B, CL, CR = synth.make_problem(p)
    W, V = synth.make_cotangents(p)
    dev = torch.device("cuda")
    Bd, Ld, Rd, Wd, Vd = (torch.from_numpy(a).to(dev) for a in (B, CL, CR, W, V))
    del B
    ws = torch.empty(jk.workspace_bytes(jk.make_problem(p.nao, p.naux, p.nd, p.r)),
                     dtype=torch.uint8, device=dev)
    ref = jk.jk_vjp(Bd, Ld, Rd, Wd, Vd, ws=ws)
    torch.cuda.synchronize()
    outs = tuple(torch.empty_like(t) for t in ref)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):                          # warm-up off the default stream
        jk.jk_vjp(Bd, Ld, Rd, Wd, Vd, out=outs, ws=ws)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, capture_error_mode="thread_local"):
        jk.jk_vjp(Bd, Ld, Rd, Wd, Vd, out=outs, ws=ws)
    for rep in range(3):
        for t in outs:
            t.fill_(float("nan"))                          # eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for got, want in zip(outs, ref):
            assert torch.equal(got, want), rep
        jk.jk_build(Bd, Ld, Rd, ws=ws)                     # the workspace reused eagerly
        torch.cuda.synchronize()

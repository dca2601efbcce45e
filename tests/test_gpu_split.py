"""GPU tests of two-stream calls (pat_plan_set_split).

A call of at least the plan's split batch runs half its instances on a second
stream of the plan.  Each instance runs the same kernels with the same tiles
either way, so the outputs must be bitwise those of a one-stream call: at an
even and an odd batch, both operators, and from a captured graph replayed
several times with other work on the stream between replays.
"""
import numpy as np
import pytest

from pat_inputs import config_geometry, make_phantom

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_dev():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _inputs(torch, geom, batch, seed):
    rng = np.random.default_rng(seed)
    f = np.stack([make_phantom(geom.n, 20, 3, 4, seed + b) for b in range(batch)])
    g = rng.standard_normal((batch, geom.n_det, geom.n_t))
    return (torch.tensor(f, dtype=torch.float32, device="cuda"),
            torch.tensor(g, dtype=torch.float32, device="cuda"))


def test_split_setting(torch_dev):
    import paper_2604_19176_amd as pat
    plan = pat.PatPlan(config_geometry(1), max_batch=4)
    try:
        assert plan.split == 64
        plan.set_split(2)
        assert plan.split == 2
        plan.set_split(0)
        assert plan.split == 0
        with pytest.raises(pat.PatError):
            plan.set_split(-1)
        assert plan.split == 0
    finally:
        plan.close()


@pytest.mark.parametrize("batch", [64, 17])
def test_split_is_bitwise_one_stream(torch_dev, batch):
    torch = torch_dev
    import paper_2604_19176_amd as pat
    geom = config_geometry(2)
    plan = pat.PatPlan(geom, max_batch=batch)
    try:
        f, g = _inputs(torch, geom, batch, 300 + batch)
        plan.set_split(0)
        g1, f1 = plan.forward(f), plan.adjoint(g)
        plan.set_split(2)
        g2, f2 = plan.forward(f), plan.adjoint(g)
        torch.cuda.synchronize()
        assert torch.equal(g1, g2)
        assert torch.equal(f1, f2)
        # the halves cover every instance (no instance left unwritten)
        assert bool(torch.isfinite(g2).all()) and float(g2[batch // 2].abs().max()) > 0
        assert float(f2[-1].abs().max()) > 0
    finally:
        plan.close()


def test_split_in_a_captured_graph(torch_dev):
    torch = torch_dev
    import paper_2604_19176_amd as pat
    geom = config_geometry(2)
    B = 32
    plan = pat.PatPlan(geom, max_batch=B)
    try:
        f, g = _inputs(torch, geom, B, 910)
        plan.set_split(0)
        g_ref, f_ref = plan.forward(f), plan.adjoint(g)
        torch.cuda.synchronize()
        plan.set_split(2)
        go, fo = torch.empty_like(g_ref), torch.empty_like(f_ref)
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):  # warm-up outside the capture
            plan.forward(f, out=go)
            plan.adjoint(g, out=fo)
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            plan.forward(f, out=go)
            plan.adjoint(g, out=fo)
        for r in range(3):
            go.zero_()
            fo.fill_(float("nan"))
            torch.cuda.synchronize()
            graph.replay()
            torch.cuda.synchronize()
            assert torch.equal(go, g_ref), "replay %d (forward)" % r
            assert torch.equal(fo, f_ref), "replay %d (adjoint)" % r
        del graph
    finally:
        plan.close()

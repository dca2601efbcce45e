"""GPU differentiation: autograd through A (backward = A*), the TV-gradient
kernel, the fused projected-gradient update and the TV reconstruction loop
(eq. (4)), against FP64 CPU references (oracle and oracle/tv.py)."""
import math

import numpy as np
import pytest

from oracle import tv as tvref
from pat_inputs import CONFIGS, Geometry, add_noise, config_geometry, make_phantom

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_dev():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _rel(a, b):
    return float(np.linalg.norm(np.ravel(a - b)) / np.linalg.norm(np.ravel(b)))


def test_autograd_backward_is_the_adjoint(torch_dev):
    torch = torch_dev
    import oracle
    import paper_2604_19176_amd as pat
    geom = config_geometry("gradcheck")
    plan = pat.PatPlan(geom)
    f = torch.tensor(make_phantom(geom.n, 5, 1, 0, 41), dtype=torch.float32, device="cuda", requires_grad=True)
    w = torch.tensor(np.random.default_rng(41).standard_normal((geom.n_det, geom.n_t)), dtype=torch.float32,
                     device="cuda")
    loss = (pat.pat_operator(plan, f) * w).sum()
    loss.backward()
    assert torch.equal(f.grad, plan.adjoint(w))
    ref = oracle.adjoint(geom, w.cpu().double().numpy())
    assert _rel(f.grad.cpu().double().numpy(), ref) <= 1e-5
    plan.close()


def test_tv_kernel_matches_reference(torch_dev):
    torch = torch_dev
    import paper_2604_19176_amd as pat
    rng = np.random.default_rng(42)
    for n, eps in [(32, 1e-3), (97, 0.05), (256, 1e-3)]:
        fs = rng.standard_normal((3, n, n)).astype(np.float32)
        g, tv = pat.tv_grad(torch.tensor(fs, device="cuda"), eps, with_value=True)
        for b in range(3):
            ref = tvref.tv_grad(fs[b].astype(np.float64), eps)
            assert _rel(g[b].cpu().double().numpy(), ref) <= 1e-5
            assert float(tv[b]) == pytest.approx(tvref.tv_value(fs[b].astype(np.float64), eps), rel=1e-5)
    c = torch.full((1, 16, 16), 3.0, device="cuda")
    gc = pat.tv_grad(c, 1e-3)
    assert float(gc.abs().max()) == 0.0


def test_pgd_update_and_residual(torch_dev):
    torch = torch_dev
    import paper_2604_19176_amd as pat
    gen = torch.Generator(device="cuda").manual_seed(3)
    f = torch.randn(2, 40, 40, device="cuda", generator=gen)
    a = torch.randn(2, 40, 40, device="cuda", generator=gen)
    t = torch.randn(2, 40, 40, device="cuda", generator=gen)
    exp = torch.clamp(f - 0.3 * (a + 0.7 * t), min=0.0)
    pat.pgd_update(f, a, t, 0.3, 0.7)
    assert torch.allclose(f, exp, rtol=1e-6, atol=1e-6)
    g = torch.randn(2, 5, 7, device="cuda", generator=gen)
    gm = torch.randn(2, 5, 7, device="cuda", generator=gen)
    expr = g - gm
    r, sq = pat.residual(g, gm, with_value=True)
    assert torch.equal(r, expr)
    assert torch.allclose(sq, 0.5 * (expr * expr).sum(dim=(1, 2)), rtol=1e-5)


@pytest.mark.parametrize("cfg", ["gradcheck", 3])
def test_objective_gradient_matches_cpu(torch_dev, cfg):
    """Gradient of 0.5||A f - g||^2 + lam TV_eps(f) on the GPU (autograd through
    A*, TV kernel) against the FP64 oracle transpose plus the TV reference."""
    torch = torch_dev
    import oracle
    import paper_2604_19176_amd as pat
    from paper_2604_19176_amd.recon import autograd_loss
    geom = config_geometry(cfg)
    lam, eps = 1e-3, 1e-3
    f0 = make_phantom(geom.n, 5, 1, 1, 43)
    gm = add_noise(oracle.forward(geom, make_phantom(geom.n, 5, 1, 1, 44)), 0.02, 44)
    plan = pat.PatPlan(geom)
    f = torch.tensor(f0, dtype=torch.float32, device="cuda", requires_grad=True)
    loss = autograd_loss(plan, f, torch.tensor(gm, dtype=torch.float32, device="cuda"), lam, eps)
    loss.backward()
    f32 = f0.astype(np.float32).astype(np.float64)
    ref = oracle.adjoint(geom, oracle.forward(geom, f32) - gm) + lam * tvref.tv_grad(f32, eps)
    err = _rel(f.grad.cpu().double().numpy(), ref)
    print("%s: objective gradient rel L2 %.3e" % (cfg, err))
    assert err <= 1e-5
    plan.close()


def test_tv_loop_graph_matches_eager_and_cpu(torch_dev):
    """Projected-gradient TV iterations: HIP-graph replays equal eager steps
    (checked replay by replay, with eager work in between), and the iterates
    follow an FP64 CPU loop with the same step size."""
    torch = torch_dev
    import oracle
    import paper_2604_19176_amd as pat
    from paper_2604_19176_amd.recon import TVReconstructor
    geom = config_geometry("gradcheck")
    lam, eps = 1e-3, 1e-3
    gm = add_noise(oracle.forward(geom, make_phantom(geom.n, 5, 1, 0, 45)), 0.02, 45)
    plan = pat.PatPlan(geom)
    gmt = torch.tensor(gm, dtype=torch.float32, device="cuda")
    eager = TVReconstructor(plan, gmt, lam, eps)
    graph = TVReconstructor(plan, gmt, lam, eps, tau=eager.tau)
    graph.capture()
    # capture() ran one warm-up step on the graph's state; bring the eager state level
    eager.step()
    torch.cuda.synchronize()
    assert torch.equal(graph.f, eager.f)
    for _ in range(4):
        graph.graph.replay()
        eager.step()
        _ = (eager.f * 2.0).sum()  # unrelated eager work between replays
        torch.cuda.synchronize()
        assert torch.equal(graph.f, eager.f)
    # several iterations per graph: run(7) is two replays of three and one eager step
    multi = TVReconstructor(plan, gmt, lam, eps, tau=eager.tau)
    multi.capture(3)
    multi.run(7)
    level = TVReconstructor(plan, gmt, lam, eps, tau=eager.tau)
    for _ in range(8):
        level.step()
    torch.cuda.synchronize()
    assert torch.equal(multi.f, level.f)
    # FP64 CPU loop, same tau, same number of steps (5)
    fc = np.zeros((geom.n, geom.n))
    for _ in range(5):
        G = oracle.adjoint(geom, oracle.forward(geom, fc) - gm) + lam * tvref.tv_grad(fc, eps)
        fc = np.maximum(fc - eager.tau * G, 0.0)
    err = _rel(graph.f.cpu().double().numpy(), fc)
    print("TV loop after 5 steps: rel L2 vs FP64 %.3e" % err)
    assert err <= 1e-4
    # the objective decreases over further steps
    o0 = float(tvref.objective(geom, graph.f.cpu().double().numpy(), gm, lam, eps, oracle.forward))
    graph.run(40)
    torch.cuda.synchronize()
    o1 = float(tvref.objective(geom, graph.f.cpu().double().numpy(), gm, lam, eps, oracle.forward))
    assert o1 < o0
    plan.close()

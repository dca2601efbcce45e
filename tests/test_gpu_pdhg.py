"""GPU primal-dual TV reconstruction against the FP64 reference (oracle/pdhg.py).

* each kernel (data dual, TV dual with projection, primal step with grad*,
  relative-change norms) against the FP64 formulas of the reference on random data;
* whole iterations: the GPU iterates (FP32 operator pair + kernels) follow the
  FP64 iteration on the oracle operator with the same step sizes;
* a batch of two instances equals the instances run alone; HIP-graph replays
  equal eager steps bitwise;
* the stopping rule (relative change <= 1e-4) fires within a couple of
  iterations of the FP64 reference.
"""
import numpy as np
import pytest

from oracle import pdhg as pdref
from pat_inputs import add_noise, config_geometry, make_phantom

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_dev():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _rel(a, b):
    a, b = np.asarray(a, dtype=np.float64), np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def _stream(torch):
    import ctypes
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def test_pd_kernels_against_reference(torch_dev):
    torch = torch_dev
    import paper_2604_19176_amd as pat
    rng = np.random.default_rng(21)
    n, B, sigma, tau, alpha = 37, 3, 0.3, 0.25, 0.2
    st = _stream(torch)
    # data dual
    y1, ax, g = (rng.standard_normal((B, 11, 13)) for _ in range(3))
    # (inputs held in variables: a temporary's memory could be reused before the kernel runs)
    ty1, tax, tg = (torch.tensor(a, dtype=torch.float32, device="cuda") for a in (y1, ax, g))
    pat.pat_pd_dual_data(ty1.data_ptr(), tax.data_ptr(), tg.data_ptr(), y1.size, sigma, st)
    assert _rel(ty1.cpu(), (y1 + sigma * (ax - g)) / (1 + sigma)) <= 1e-6
    # TV dual
    xbar = rng.standard_normal((B, n, n))
    y2 = 0.1 * rng.standard_normal((B, n, n, 2))
    ty2, txb = (torch.tensor(a, dtype=torch.float32, device="cuda") for a in (y2, xbar))
    pat.pat_pd_dual_tv(ty2.data_ptr(), txb.data_ptr(), n, B, sigma, alpha, st)
    out = ty2.cpu().double().numpy()
    for b in range(B):
        dx, dy = pdref.grad(xbar[b])
        vx, vy = y2[b, ..., 0] + sigma * dx, y2[b, ..., 1] + sigma * dy
        sc = np.maximum(1.0, np.sqrt(vx * vx + vy * vy) / alpha)
        assert _rel(out[b, ..., 0], vx / sc) <= 1e-6 and _rel(out[b, ..., 1], vy / sc) <= 1e-6
    assert np.sqrt(out[..., 0] ** 2 + out[..., 1] ** 2).max() <= alpha * (1 + 1e-6)
    # primal step and change norms
    f = np.abs(rng.standard_normal((B, n, n)))
    aty = rng.standard_normal((B, n, n))
    tf, taty = (torch.tensor(a, dtype=torch.float32, device="cuda") for a in (f, aty))
    tx = torch.empty_like(tf)
    pat.pat_pd_primal(tf.data_ptr(), tx.data_ptr(), taty.data_ptr(), ty2.data_ptr(), n, B, tau, st)
    chg = torch.zeros(B, 2, device="cuda")
    pat.pat_pd_change(tf.data_ptr(), tx.data_ptr(), chg.data_ptr(), n, B, st)
    for b in range(B):
        fn = np.maximum(f[b] - tau * (aty[b] + pdref.grad_adjoint(out[b, ..., 0], out[b, ..., 1])), 0.0)
        assert _rel(tf[b].cpu(), fn) <= 1e-6
        assert _rel(tx[b].cpu(), 2 * fn - f[b]) <= 1e-6
        assert float(chg[b, 0]) == pytest.approx(float(np.sum((fn - f[b]) ** 2)), rel=1e-5)
        assert float(chg[b, 1]) == pytest.approx(float(np.sum(fn ** 2)), rel=1e-5)


def _problem(cfg, seed, eta=0.02):
    import oracle
    geom = config_geometry(cfg)
    g = add_noise(oracle.forward(geom, make_phantom(geom.n, 5, 1, 1, seed)), eta, seed)
    fwd = lambda x: oracle.forward(geom, x)
    adj = lambda y: oracle.adjoint(geom, y)
    s, t = pdref.step_sizes(pdref.op_norm_sq(fwd, adj, geom.n, iters=40))
    return geom, g, fwd, adj, s, t


@pytest.mark.parametrize("cfg,iters", [("gradcheck", 40), (1, 25)])
def test_pdhg_iterates_follow_the_fp64_reference(torch_dev, cfg, iters):
    torch = torch_dev
    import paper_2604_19176_amd as pat
    from paper_2604_19176_amd.recon import PDHGReconstructor
    geom, g, fwd, adj, s, t = _problem(cfg, 31)
    alpha = 0.05 * float(np.abs(g).max())
    ref, hist = pdref.pdhg(fwd, adj, g, geom.n, alpha, s, t, iters)
    plan = pat.PatPlan(geom)
    rec = PDHGReconstructor(plan, torch.tensor(g, dtype=torch.float32, device="cuda"), alpha, sigma=s, tau=t)
    for _ in range(iters):
        rec.step()
    torch.cuda.synchronize()
    err = _rel(rec.f.cpu(), ref)
    print("%s: %d PDHG iterations, rel L2 vs FP64 %.2e; relative change gpu %.3e ref %.3e"
          % (cfg, iters, err, rec.relative_change()[0], hist[-1]))
    assert err <= 1e-4
    assert rec.relative_change()[0] == pytest.approx(hist[-1], rel=1e-2)
    plan.close()


def test_pdhg_batch_and_graph(torch_dev):
    torch = torch_dev
    import paper_2604_19176_amd as pat
    from paper_2604_19176_amd.recon import PDHGReconstructor
    geom, g0, fwd, adj, s, t = _problem("gradcheck", 41)
    _, g1, _, _, _, _ = _problem("gradcheck", 42)
    alpha = 0.05 * float(np.abs(g0).max())
    plan = pat.PatPlan(geom, max_batch=2)
    gb = torch.tensor(np.stack([g0, g1]), dtype=torch.float32, device="cuda")
    both = PDHGReconstructor(plan, gb, alpha, sigma=s, tau=t)
    singles = [PDHGReconstructor(plan, gb[b].contiguous(), alpha, sigma=s, tau=t) for b in range(2)]
    graphed = PDHGReconstructor(plan, gb, alpha, sigma=s, tau=t)
    graphed.capture(3)         # runs one iteration eagerly, records the next three
    for r in [both] + singles:
        r.step()
    torch.cuda.synchronize()
    assert torch.equal(graphed.f, both.f)
    for k in range(4):
        graphed.graph.replay()
        for _ in range(3):
            both.step()
            for r in singles:
                r.step()
        _ = float(both.f.sum())  # unrelated eager work between replays
        torch.cuda.synchronize()
        assert torch.equal(graphed.f, both.f), k
        # the graph reduces the change in its last iteration only
        assert torch.equal(graphed.change, both.change), k
        for b in range(2):
            assert torch.equal(both.f[b], singles[b].f), (k, b)
    # run() with a check interval that is not a multiple of the graph's length
    its = graphed.run(7, tol=None, check_every=5)
    for _ in range(7):
        both.step()
    torch.cuda.synchronize()
    assert its == 1 + 7        # the warm-up and run(); direct replays are not counted
    assert torch.equal(graphed.f, both.f) and torch.equal(graphed.change, both.change)
    plan.close()


def test_pdhg_stopping_rule_matches_reference(torch_dev):
    torch = torch_dev
    import paper_2604_19176_amd as pat
    from paper_2604_19176_amd.recon import PDHGReconstructor
    geom, g, fwd, adj, s, t = _problem("gradcheck", 51, eta=0.0)
    alpha = 0.05 * float(np.abs(g).max())
    _, hist = pdref.pdhg(fwd, adj, g, geom.n, alpha, s, t, 3000, tol=1e-4)
    plan = pat.PatPlan(geom)
    rec = PDHGReconstructor(plan, torch.tensor(g, dtype=torch.float32, device="cuda"), alpha, sigma=s, tau=t)
    k = rec.run(3000, tol=1e-4, check_every=1, use_graph=False)
    print("stopping: gpu %d iterations, FP64 reference %d" % (k, len(hist)))
    assert abs(k - len(hist)) <= max(3, len(hist) // 50)
    plan.close()

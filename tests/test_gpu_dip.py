"""GPU deep image prior (eq. (5), Sec. 2.2) against the FP64 reference.

* The objective ||A f - g||^2 + lam TV_eps(f) and its gradient in the image f,
  through this library's A (backward: A*) and TV kernels, equal the FP64
  oracle (oracle/dip.py): value rel 1e-5, gradient rel L2 1e-4.
* One U-Net step: the seeded float32 GPU network gives the same loss (1e-5)
  and parameter gradients (rel L2 1e-4) with the library's objective as with
  the FP64 oracle objective (an autograd Function over oracle.dip); the same
  network in float64 on the CPU gives the same loss, and its gradients measure
  the float32 network's own error (MIOpen convolutions, batch normalisation;
  reported, bounded at 1e-2).
* Three gradient-descent steps of two identical float32 networks that differ
  only in the objective (library kernels vs FP64 oracle) give the same losses
  (1e-5) and output images (rel L2 1e-4).  The steps are plain gradient
  descent, linear in the gradient, so the trajectories differ by the order of
  the FP32-vs-FP64 gradient difference checked at step 0.  (Adam, the
  optimiser of Sec. 2.2.1, moves each parameter in its first steps by about
  the learning rate times the sign of its gradient, so the ~1e-6 gradient
  difference flips the steps of parameters whose gradient is near zero and
  moves the image by the order of the learning rate whatever the kernels do;
  the Adam loop is checked by the objective-decrease test below.  Networks of
  different precision drift apart likewise, so the trajectory check holds the
  network arithmetic fixed.)
* A short run lowers the objective; the U-Net has the layout of Sec. 2.2.1.
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


def _rel(a, b):
    a, b = np.asarray(a, dtype=np.float64), np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def _problem(seed=8):
    import oracle
    geom = config_geometry("gradcheck")
    truth = make_phantom(geom.n, 4, 1, 1, seed)
    g = oracle.forward(geom, truth)
    g += 0.01 * np.abs(g).max() * np.random.default_rng(seed + 1).standard_normal(g.shape)
    return geom, truth, g


def test_dip_objective_and_image_gradient(torch_dev):
    torch = torch_dev
    import paper_2604_19176_amd as pat
    from oracle import dip as ref
    from paper_2604_19176_amd.dip import dip_objective
    geom, truth, g = _problem()
    f = np.abs(truth + 0.05 * np.random.default_rng(9).standard_normal(truth.shape))
    lam, eps = 0.2, 1e-2
    plan = pat.PatPlan(geom)
    tf = torch.tensor(f, dtype=torch.float32, device="cuda", requires_grad=True)
    tg = torch.tensor(g, dtype=torch.float32, device="cuda")
    val = dip_objective(plan, tf, tg, lam, eps)
    val.backward()
    v_ref = ref.objective(geom, f, g, lam, eps)
    g_ref = ref.gradient(geom, f, g, lam, eps)
    print("objective %.6e (FP64 %.6e), gradient rel L2 %.2e" % (float(val), v_ref, _rel(tf.grad.cpu(), g_ref)))
    assert float(val) == pytest.approx(v_ref, rel=1e-5)
    assert _rel(tf.grad.cpu(), g_ref) <= 1e-4
    plan.close()


def test_dip_steps_track_the_fp64_objective(torch_dev):
    torch = torch_dev
    import paper_2604_19176_amd as pat
    from oracle import dip as ref
    from paper_2604_19176_amd.dip import UNet, dip_objective

    class OracleObjective(torch.autograd.Function):
        """The FP64 oracle objective of an image held on any device (gradient cast back)."""
        @staticmethod
        def forward(ctx, f, geom, g, lam, eps):
            x = f.detach().cpu().double().numpy()
            ctx.grad = torch.tensor(ref.gradient(geom, x, g, lam, eps), dtype=f.dtype, device=f.device)
            return torch.tensor(ref.objective(geom, x, g, lam, eps), dtype=f.dtype, device=f.device)

        @staticmethod
        def backward(ctx, go):
            return go * ctx.grad, None, None, None, None

    geom, truth, g = _problem(10)
    lam, eps, steps = 0.1, 1e-2, 3
    z = np.clip(truth + 0.1 * np.random.default_rng(11).standard_normal(truth.shape), 0, None)
    zg = torch.tensor(z, dtype=torch.float32, device="cuda").reshape(1, 1, geom.n, geom.n)
    tg = torch.tensor(g, dtype=torch.float32, device="cuda")
    plan = pat.PatPlan(geom)
    torch.manual_seed(3)
    net_a = UNet().cuda()
    # (1) step 0, parameter gradients of one float32 GPU network with the library objective (ga)
    # and with the FP64 oracle objective (go): they differ only by the objective; a float64 CPU
    # network with the oracle objective (gc) measures the network's own float32 error
    net_c = UNet().double()
    net_c.load_state_dict({k: v.double() for k, v in net_a.state_dict().items()})

    def grads(net):
        return torch.cat([p.grad.flatten().cpu().double() for p in net.parameters()])
    la = dip_objective(plan, net_a(zg)[0, 0].contiguous(), tg, lam, eps)
    la.backward()
    ga = grads(net_a)
    net_a.zero_grad()
    lo = OracleObjective.apply(net_a(zg)[0, 0], geom, g, lam, eps)
    lo.backward()
    go = grads(net_a)
    net_a.zero_grad()
    zc = torch.tensor(z, dtype=torch.float64).reshape(1, 1, geom.n, geom.n)
    lc = OracleObjective.apply(net_c(zc)[0, 0], geom, g, lam, eps)
    lc.backward()
    gc = grads(net_c)
    e_obj = float((ga - go).norm() / gc.norm())
    e_net = float((go - gc).norm() / gc.norm())
    print("step 0: loss library %.7e oracle %.7e fp64 net %.7e; parameter gradients: library vs oracle "
          "objective %.2e, float32 vs float64 network %.2e" % (float(la), float(lo), float(lc), e_obj, e_net))
    assert float(la) == pytest.approx(float(lo), rel=1e-5)
    assert float(la) == pytest.approx(float(lc), rel=1e-5)
    assert e_obj <= 1e-4
    assert e_net <= 1e-2
    # (2) gradient-descent trajectories of two identical float32 networks that differ only in
    # the objective: the library's kernels vs the FP64 oracle.  The step is linear in the
    # gradient, so the trajectories stay within the order of the step-0 gradient difference
    # (1e-4 bound); lr = 1e-6 moves the image by about 10 % over the three steps here, and a
    # wrong operator gradient would move the trajectories apart by orders of magnitude more.
    lr = 1e-6
    torch.manual_seed(4)
    net_a = UNet().cuda()
    net_b = UNet().cuda()
    net_b.load_state_dict(net_a.state_dict())
    opt_a = torch.optim.SGD(net_a.parameters(), lr=lr)
    opt_b = torch.optim.SGD(net_b.parameters(), lr=lr)
    with torch.no_grad():
        i0 = net_a(zg)[0, 0].cpu().double().numpy()
    for k in range(steps):
        opt_a.zero_grad()
        la = dip_objective(plan, net_a(zg)[0, 0].contiguous(), tg, lam, eps)
        la.backward()
        opt_a.step()
        opt_b.zero_grad()
        lb = OracleObjective.apply(net_b(zg)[0, 0], geom, g, lam, eps)
        lb.backward()
        opt_b.step()
        print("step %d: loss library %.7e  oracle %.7e" % (k, float(la), float(lb)))
        assert float(la) == pytest.approx(float(lb), rel=1e-5)
    with torch.no_grad():
        ia = net_a(zg)[0, 0].cpu().double().numpy()
        ib = net_b(zg)[0, 0].cpu().double().numpy()
    print("image after %d steps: moved %.2e, library vs oracle rel L2 %.2e" % (steps, _rel(ia, i0), _rel(ia, ib)))
    assert _rel(ia, i0) >= 1e-2
    assert _rel(ia, ib) <= 1e-4
    plan.close()


def test_dip_run_lowers_the_objective(torch_dev):
    torch = torch_dev
    import paper_2604_19176_amd as pat
    from paper_2604_19176_amd.dip import DIPReconstructor
    from paper_2604_19176_amd.recon import CGLSReconstructor
    geom, truth, g = _problem(12)
    plan = pat.PatPlan(geom)
    tg = torch.tensor(g, dtype=torch.float32, device="cuda")
    cg = CGLSReconstructor(plan, tg)
    for _ in range(8):
        cg.step()
    rec = DIPReconstructor(plan, tg, cg.f, lam=0.05, iters=40, seed=1)
    # layout of Sec. 2.2.1: 4 encoder stages, 3 decoder stages, 32..256 channels
    convs = [m for m in rec.net.modules() if isinstance(m, torch.nn.Conv2d)]
    assert [m.out_channels for m in convs[:8]] == [32, 32, 64, 64, 128, 128, 256, 256]
    assert sum(isinstance(m, torch.nn.ConvTranspose2d) for m in rec.net.modules()) == 3
    first = float(rec.step())
    hist = rec.run(39, truth=torch.tensor(truth, dtype=torch.float32, device="cuda"), every=13)
    print("DIP objective %.4e -> %.4e; PSNR %s" % (first, float(rec.last_loss), hist))
    assert float(rec.last_loss) < first
    plan.close()

"""GPU parity at the headline workload, in the launch configurations the bench
times: 256x256, 256 detectors on a 180 degree arc, 512 samples, batch 64.

- Every one of the 64 instances is computed with the plan's default batch-64
  shapes and with the shapes the autotuner picks on this device for this
  workload at batch 64 (what bench.py times); launch shapes change no
  result, so both batches are bitwise equal.
- The first, a middle and the last instance are compared element by element
  with the FP64 oracle (relative L2 <= 1e-5, the operator's FP32 tolerance).
- Each instance equals its single-instance call bitwise.
"""
import numpy as np
import pytest

from pat_inputs import CONFIGS, config_geometry, make_phantom

pytestmark = pytest.mark.gpu

TOL = 1e-5
B = 64
SAMPLED = (0, 31, 63)


@pytest.fixture(scope="module")
def torch_dev():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _rel(a, b):
    return float(np.linalg.norm(np.ravel(a - b)) / np.linalg.norm(np.ravel(b)))


def test_headline_batch_in_bench_launch_shapes(torch_dev):
    torch = torch_dev
    import oracle
    import paper_2604_19176_amd as pat
    geom = config_geometry(2)
    nb, nd, nl = CONFIGS[2]["phantom"]
    fs = np.stack([make_phantom(geom.n, nb, nd, nl, 2000 + b) for b in range(B)])
    ds = np.random.default_rng(2001).standard_normal((B, geom.n_det, geom.n_t))
    plan = pat.PatPlan(geom, max_batch=B)
    ft = torch.tensor(fs, dtype=torch.float32, device="cuda")
    dt = torch.tensor(ds, dtype=torch.float32, device="cuda")
    g0, a0 = plan.forward(ft).clone(), plan.adjoint(dt).clone()
    tuned = plan.autotune(batch=B)
    print("tuned launch shapes:", tuned)
    assert plan.launch == tuned
    g1, a1 = plan.forward(ft).clone(), plan.adjoint(dt).clone()
    assert torch.equal(g1, g0) and torch.equal(a1, a0)
    for b in SAMPLED:
        ef = _rel(g1[b].cpu().double().numpy(), oracle.forward(geom, fs[b]))
        ea = _rel(a1[b].cpu().double().numpy(), oracle.adjoint(geom, ds[b]))
        print("instance %d: forward rel L2 %.2e, adjoint rel L2 %.2e" % (b, ef, ea))
        assert ef <= TOL and ea <= TOL
    for b in range(B):
        assert torch.equal(g1[b], plan.forward(ft[b].contiguous())), b
        assert torch.equal(a1[b], plan.adjoint(dt[b].contiguous())), b
    plan.close()

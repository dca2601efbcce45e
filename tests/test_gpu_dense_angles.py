"""GPU parity with explicit detector angles (dense synthesis on the matrix cores).

A plan given D arbitrary angles runs the angular synthesis of eq. (2) as a
dense product of the mode coefficients with a cos/sin table (v_mfma_f32
32x32x2) and its transpose in the adjoint.  Checked against the FP64 oracle
(which sums the plane-wave form at the same angles) element by element at rel
L2 <= 1e-5, at sizes spanning several 64 x 64 tiles with ragged tails:

* random unsorted angles, two separated arcs, a sparse subset of a 270 degree
  ring, and the uniform arc's own angles (which must also agree with the
  transform path of the uniform plan);
* the dot-product identity of the GPU pair; batch = per instance (bitwise);
  a heterogeneous batch mixing explicit-angle and uniform plans equals the
  instances run alone (bitwise).
"""
import math

import numpy as np
import pytest

from pat_inputs import Geometry, make_phantom

pytestmark = pytest.mark.gpu

TOL = 1e-5


def _rel(a, b):
    return float(np.linalg.norm(np.ravel(a - b)) / np.linalg.norm(np.ravel(b)))


def _arc(span_deg, D, center):
    a = math.radians(span_deg)
    return [center - a / 2 + (d + 0.5) * a / D for d in range(D)]


GEOMS = {
    # 37 random unsorted angles on a 40^2 grid, R != 1, c != 1
    "random": Geometry(n=40, n_det=37, n_t=75, dt=2.2 / 75, c=1.3, det_r=1.1, support_r=0.95,
                       det_theta=tuple(np.random.default_rng(11).uniform(-math.pi, math.pi, 37))),
    # two arcs of 50 and 30 elements with a gap: 80 detectors (two detector tiles, ragged)
    "two_arcs": Geometry(n=48, n_det=80, n_t=96, dt=2 / 96,
                         det_theta=tuple(_arc(100, 50, -1.2) + _arc(60, 30, 1.6))),
    # every other element of a 130-element 270 degree ring plus its first 3: 68 detectors
    "sparse_270": Geometry(n=64, n_det=68, n_t=128, dt=2 / 128,
                           det_theta=tuple(_arc(270, 130, -math.pi / 2)[::2] + _arc(270, 130, -math.pi / 2)[1:6:2])),
    # the limited-view 256^2 shape with its 256 uniform angles given explicitly
    "cfg2_explicit": Geometry(n=256, n_det=256, n_t=512, dt=2 / 512,
                              det_theta=tuple(_arc(180, 256, -math.pi / 2))),
}

_cache = {}


@pytest.fixture(scope="module")
def torch_dev():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _case(name):
    if name not in _cache:
        import oracle
        geom = GEOMS[name]
        f = make_phantom(geom.n, 5, 1, 1, 700 + len(_cache))
        d = np.random.default_rng(800 + len(_cache)).standard_normal((geom.n_det, geom.n_t))
        _cache[name] = (geom, f, d, oracle.forward(geom, f), oracle.adjoint(geom, d))
    return _cache[name]


@pytest.mark.parametrize("name", list(GEOMS))
def test_dense_synthesis_matches_oracle(torch_dev, name):
    torch = torch_dev
    import paper_2604_19176_amd as pat
    geom, f, d, Af, Ad = _case(name)
    plan = pat.PatPlan(geom)
    assert plan.info.syn_dense == 1 and plan.info.len_czt == 0
    g = plan.forward(torch.tensor(f, dtype=torch.float32, device="cuda")).cpu().double().numpy()
    a = plan.adjoint(torch.tensor(d, dtype=torch.float32, device="cuda")).cpu().double().numpy()
    ef, ea = _rel(g, Af), _rel(a, Ad)
    print("%s: forward rel L2 %.3e  adjoint rel L2 %.3e" % (name, ef, ea))
    assert ef <= TOL and ea <= TOL
    plan.close()


def test_explicit_uniform_angles_agree_with_the_transform_path(torch_dev):
    torch = torch_dev
    import paper_2604_19176_amd as pat
    geom, f, d, _, _ = _case("cfg2_explicit")
    uni = geom.with_(det_theta=None, arc_span=math.radians(180))
    p_dense, p_uni = pat.PatPlan(geom), pat.PatPlan(uni)
    assert p_uni.info.syn_dense == 0 and p_uni.info.len_czt == 512
    ft = torch.tensor(f, dtype=torch.float32, device="cuda")
    dt = torch.tensor(d, dtype=torch.float32, device="cuda")
    e1 = _rel(p_dense.forward(ft).cpu().double().numpy(), p_uni.forward(ft).cpu().double().numpy())
    e2 = _rel(p_dense.adjoint(dt).cpu().double().numpy(), p_uni.adjoint(dt).cpu().double().numpy())
    print("dense vs transform synthesis: forward %.2e adjoint %.2e" % (e1, e2))
    assert e1 <= 2 * TOL and e2 <= 2 * TOL
    p_dense.close()
    p_uni.close()


def test_dense_dot_identity_and_batch(torch_dev):
    torch = torch_dev
    import paper_2604_19176_amd as pat
    geom = GEOMS["two_arcs"]
    B = 3
    fs = np.stack([make_phantom(geom.n, 4, 1, 1, 900 + b) for b in range(B)])
    ds = np.random.default_rng(901).standard_normal((B, geom.n_det, geom.n_t))
    plan = pat.PatPlan(geom, max_batch=B)
    ft = torch.tensor(fs, dtype=torch.float32, device="cuda")
    dt = torch.tensor(ds, dtype=torch.float32, device="cuda")
    gb, ab = plan.forward(ft).clone(), plan.adjoint(dt).clone()
    for b in range(B):
        assert torch.equal(gb[b], plan.forward(ft[b].contiguous()))
        assert torch.equal(ab[b], plan.adjoint(dt[b].contiguous()))
    lhs = float((gb.double() * dt.double()).sum())
    rhs = float((ft.double() * ab.double()).sum())
    err = abs(lhs - rhs) / (float(gb.double().norm()) * float(dt.double().norm()))
    print("dot identity %.2e" % err)
    assert err <= TOL
    plan.close()


def test_heterogeneous_batch_with_dense_plans(torch_dev):
    torch = torch_dev
    import paper_2604_19176_amd as pat
    geoms = [GEOMS["random"], Geometry(n=48, n_det=40, n_t=96, dt=2 / 96, arc_span=math.radians(90)),
             GEOMS["two_arcs"]]
    plans = [pat.PatPlan(g) for g in geoms]
    batch = pat.PatBatch(plans)
    fs = [torch.tensor(make_phantom(g.n, 4, 1, 1, 950 + i), dtype=torch.float32, device="cuda")
          for i, g in enumerate(geoms)]
    rng = np.random.default_rng(951)
    ds = [torch.tensor(rng.standard_normal((g.n_det, g.n_t)), dtype=torch.float32, device="cuda") for g in geoms]
    gs = batch.forward(fs)
    As = batch.adjoint(ds)
    for i, p in enumerate(plans):
        assert torch.equal(gs[i], p.forward(fs[i])), i
        assert torch.equal(As[i], p.adjoint(ds[i])), i
    batch.close()
    for p in plans:
        p.close()

"""GPU tests of the launch shapes, the heterogeneous batch and the autotuner.

* Any launch shape the library accepts gives bitwise the same operator: every
  output, and the scalar sums of the endpoint term, is a sum in an order that
  does not depend on the tiling or the workgroup size.
* A heterogeneous batch (instances of different N, D, arc and T in one launch
  per stage) gives bitwise the per-instance results, matches the FP64 oracle,
  and replays bitwise from a HIP graph.
* The autotuner picks valid shapes, writes a JSON cache and re-applies it.
"""
import json
import math

import numpy as np
import pytest

from pat_inputs import Geometry, config_geometry, make_phantom
from pat_inputs.geometry import mixed_batch_geometries

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


def _inputs(torch, geom, seed, batch=None):
    rng = np.random.default_rng(seed)
    if batch is None:
        f = make_phantom(geom.n, 5, 1, 1, seed)
        d = rng.standard_normal((geom.n_det, geom.n_t))
    else:
        f = np.stack([make_phantom(geom.n, 5, 1, 1, seed + b) for b in range(batch)])
        d = rng.standard_normal((batch, geom.n_det, geom.n_t))
    return (torch.tensor(f, dtype=torch.float32, device="cuda"),
            torch.tensor(d, dtype=torch.float32, device="cuda"))


SHAPES = [
    dict(col_np=1, row_rpb=1, ring_rt=1, dct_dp=1, gat_cb=64, gat_th=8, spr_cb=64, spr_th=8, gat_ib=1, spr_ib=1),
    dict(col_np=2, row_rpb=16, ring_rt=2, dct_dp=8, gat_cb=128, gat_th=32, spr_cb=192, spr_th=8, gat_ib=1,
         spr_ib=2),
    dict(col_np=16, row_rpb=4, ring_rt=4, dct_dp=2, gat_cb=64, gat_th=16, spr_cb=256, spr_th=8, gat_ib=4,
         spr_ib=4),
    dict(col_np=4, row_rpb=2, ring_rt=3, dct_dp=3, gat_cb=32, gat_th=1, spr_cb=128, spr_th=8, gat_ib=2, spr_ib=4),
]


@pytest.mark.parametrize("cfg", [1, "ragged", 2])
def test_launch_shapes_give_the_same_operator(torch_dev, cfg):
    torch = torch_dev
    import paper_2604_19176_amd as pat
    geom = Geometry(n=40, n_det=37, n_t=70, dt=2.0 / 70, arc_span=math.radians(100.0)) if cfg == "ragged" \
        else config_geometry(cfg)
    plan = pat.PatPlan(geom, max_batch=3)
    f, d = _inputs(torch, geom, 71, batch=3)
    g0, a0 = plan.forward(f).clone(), plan.adjoint(d).clone()
    for shp in SHAPES:
        try:
            plan.set_launch(**shp)
        except pat.PatError:
            continue  # does not fit this geometry (checked on the host)
        assert plan.launch == shp
        g, a = plan.forward(f), plan.adjoint(d)
        eg, ea = _rel(g.cpu(), g0.cpu()), _rel(a.cpu(), a0.cpu())
        print(cfg, shp, "rel diff fwd %.2e adj %.2e" % (eg, ea))
        assert torch.equal(g, g0) and torch.equal(a, a0)
    plan.close()


def test_launch_shapes_against_oracle_and_rejections(torch_dev):
    torch = torch_dev
    import oracle
    import paper_2604_19176_amd as pat
    geom = config_geometry(1)
    plan = pat.PatPlan(geom)
    f, d = _inputs(torch, geom, 72)
    plan.set_launch(**SHAPES[1])
    g, a = plan.forward(f).cpu().numpy(), plan.adjoint(d).cpu().numpy()
    assert _rel(g, oracle.forward(geom, f.cpu().double().numpy())) <= 1e-5
    assert _rel(a, oracle.adjoint(geom, d.cpu().double().numpy())) <= 1e-5
    before = plan.launch
    for bad in [dict(gat_cb=100), dict(gat_cb=24), dict(gat_th=12), dict(gat_cb=256, gat_th=64), dict(spr_cb=320), dict(gat_th=0),
                dict(ring_rt=0), dict(col_np=17), dict(dct_dp=0), dict(row_rpb=17), dict(gat_ib=3),
                dict(spr_ib=0), dict(gat_cb=128, gat_th=16, gat_ib=4), dict(spr_th=16), dict(spr_th=4)]:
        with pytest.raises(pat.PatError) as ei:
            plan.set_launch(**bad)
        assert ei.value.status == -1
        assert plan.launch == before
    plan.close()
    plan2 = pat.PatPlan(config_geometry(2))   # cosine transform of length 2M = 2048
    before = plan2.launch
    with pytest.raises(pat.PatError) as ei:
        plan2.set_launch(dct_dp=16)               # 16 x 2048 complex values: more LDS than a workgroup has
    assert ei.value.status == -2
    assert plan2.launch == before
    plan2.close()


def _mixed(count):
    """`count` distinct instances of the heterogeneous workload (N, D, arc mixed), T = 2N."""
    out, seen = [], set()
    for geom, seed in mixed_batch_geometries(64):
        key = (geom.n, geom.n_det, round(geom.arc_span, 6))
        if key in seen:
            continue
        seen.add(key)
        out.append((geom, seed))
        if len(out) == count:
            break
    return out


def test_batch_equals_per_instance_bitwise(torch_dev):
    torch = torch_dev
    import paper_2604_19176_amd as pat
    inst = _mixed(12)
    assert {g.n for g, _ in inst} == {128, 256, 512}
    plans = [pat.PatPlan(g) for g, _ in inst]
    plans.append(plans[0])  # a plan may serve several instances
    inst.append((inst[0][0], inst[0][1] + 777))
    fs, ds = [], []
    for (g, s) in inst:
        f, d = _inputs(torch, g, s)
        fs.append(f)
        ds.append(d)
    batch = pat.PatBatch(plans)
    gb = [x.clone() for x in batch.forward(fs)]
    ab = [x.clone() for x in batch.adjoint(ds)]
    for i, p in enumerate(plans):
        assert torch.equal(gb[i], p.forward(fs[i])), i
        assert torch.equal(ab[i], p.adjoint(ds[i])), i
    # other batch-wide interpolation / spread shapes: still bitwise the same
    for shp in [dict(gat_cb=64, gat_th=8, spr_cb=64, spr_th=8), dict(gat_cb=128, gat_th=32, spr_cb=192, spr_th=8)]:
        batch.set_launch(**shp)
        assert batch.launch == shp
        g2 = batch.forward(fs)
        a2 = batch.adjoint(ds)
        for i in range(len(plans)):
            assert torch.equal(g2[i], gb[i]) and torch.equal(a2[i], ab[i]), (shp, i)
    batch.close()
    for p in plans[:-1]:
        p.close()


def test_batch_keeps_its_shapes_after_plan_changes(torch_dev):
    """A batch runs each instance with the FFT-stage shapes its plan had at
    batch creation; changing the plan's shapes afterwards (set_launch or
    autotune) must leave the batch's workgroup sizes consistent with the
    shapes it copied, so its results stay bitwise the per-instance ones."""
    torch = torch_dev
    import paper_2604_19176_amd as pat
    geoms = [config_geometry(2), config_geometry(1)]
    wide = dict(col_np=16, row_rpb=16, dct_dp=4)
    plans = [pat.PatPlan(g) for g in geoms]
    for p in plans:
        p.set_launch(**wide)
    batch = pat.PatBatch(plans)
    for p in plans:
        p.set_launch(col_np=1, row_rpb=1, dct_dp=1)
    fs, ds = zip(*[_inputs(torch, g, 300 + i) for i, g in enumerate(geoms)])
    gb = [x.clone() for x in batch.forward(list(fs))]
    ab = [x.clone() for x in batch.adjoint(list(ds))]
    for i, p in enumerate(plans):
        assert torch.equal(gb[i], p.forward(fs[i])), i
        assert torch.equal(ab[i], p.adjoint(ds[i])), i
    batch.close()
    for p in plans:
        p.close()


def test_batch_against_oracle(torch_dev):
    torch = torch_dev
    import oracle
    import paper_2604_19176_amd as pat
    geoms = [config_geometry("gradcheck"), config_geometry(1),
             Geometry(n=48, n_det=40, n_t=96, dt=2.0 / 96, arc_span=math.radians(90.0)),
             Geometry(n=36, n_det=20, n_t=50, dt=2.0 / 50, arc_span=2 * math.pi, arc_center=0.3)]
    plans = [pat.PatPlan(g) for g in geoms]
    batch = pat.PatBatch(plans)
    fs, ds = zip(*[_inputs(torch, g, 90 + i) for i, g in enumerate(geoms)])
    gb, ab = batch.forward(list(fs)), batch.adjoint(list(ds))
    for i, g in enumerate(geoms):
        ef = _rel(gb[i].cpu().numpy(), oracle.forward(g, fs[i].cpu().double().numpy()))
        ea = _rel(ab[i].cpu().numpy(), oracle.adjoint(g, ds[i].cpu().double().numpy()))
        print("batch instance %d (N=%d D=%d): fwd %.2e adj %.2e" % (i, g.n, g.n_det, ef, ea))
        assert ef <= 1e-5 and ea <= 1e-5
    batch.close()
    for p in plans:
        p.close()


def test_batch_graph_replays_bitwise(torch_dev):
    torch = torch_dev
    import paper_2604_19176_amd as pat
    inst = _mixed(6)
    plans = [pat.PatPlan(g) for g, _ in inst]
    batch = pat.PatBatch(plans)
    fs, ds = zip(*[_inputs(torch, g, s) for g, s in inst])
    fs, ds = list(fs), list(ds)
    gout = [torch.empty(p.data_shape, device="cuda") for p in plans]
    aout = [torch.empty(p.image_shape, device="cuda") for p in plans]
    batch.forward(fs, gout)
    batch.adjoint(ds, aout)
    torch.cuda.synchronize()
    g_ref = [x.clone() for x in gout]
    a_ref = [x.clone() for x in aout]
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        batch.forward(fs, gout)
        batch.adjoint(ds, aout)
    torch.cuda.current_stream().wait_stream(s)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        batch.forward(fs, gout)
        batch.adjoint(ds, aout)
    for rep in range(3):
        for x in gout + aout:
            x.fill_(-1.0)
        graph.replay()
        _ = sum(float(x.sum()) for x in fs)  # unrelated eager work between replays
        torch.cuda.synchronize()
        for i in range(len(plans)):
            assert torch.equal(gout[i], g_ref[i]) and torch.equal(aout[i], a_ref[i]), (rep, i)
    del graph
    batch.close()
    for p in plans:
        p.close()


def test_autotune_plan_writes_and_reuses_cache(torch_dev, tmp_path):
    torch = torch_dev
    import paper_2604_19176_amd as pat
    geom = config_geometry(1)
    cache = str(tmp_path / "tune.json")
    plan = pat.PatPlan(geom, max_batch=4)
    f, d = _inputs(torch, geom, 73, batch=4)
    g0, a0 = plan.forward(f).clone(), plan.adjoint(d).clone()
    chosen = plan.autotune(batch=4, cache_path=cache)
    entries = json.load(open(cache))
    assert len(entries) == 1
    (key, stored), = entries.items()
    assert "n=64" in key and "batch=4" in key
    # the shapes, and the two-stream batch the tuner timed (4: two streams won, 0: one)
    split = stored.pop("split")
    assert stored == chosen and split == plan.split and split in (0, 4)
    assert torch.equal(plan.forward(f), g0) and torch.equal(plan.adjoint(d), a0)
    plan2 = pat.PatPlan(geom, max_batch=4)
    assert plan2.autotune(batch=4, cache_path=cache) == chosen       # from the cache
    assert plan2.split == split
    plan2.autotune(batch=1, cache_path=cache)                         # a second key
    assert len(json.load(open(cache))) == 2
    # an entry the shape checks now reject (another spread tile height) is tuned again and replaced
    stale = json.load(open(cache))
    stale[key] = dict(stale[key], spr_th=16)
    with open(cache, "w") as fh:
        json.dump(stale, fh)
    plan3 = pat.PatPlan(geom, max_batch=4)
    again = plan3.autotune(batch=4, cache_path=cache)
    renewed = json.load(open(cache))[key]
    assert again["spr_th"] == 8 and renewed.pop("split") == plan3.split and renewed == again
    assert torch.equal(plan3.forward(f), g0) and torch.equal(plan3.adjoint(d), a0)
    plan.close()
    plan2.close()
    plan3.close()


def test_autotune_batch(torch_dev, tmp_path):
    torch = torch_dev
    import paper_2604_19176_amd as pat
    inst = _mixed(4)
    plans = [pat.PatPlan(g) for g, _ in inst]
    batch = pat.PatBatch(plans)
    fs, ds = zip(*[_inputs(torch, g, s) for g, s in inst])
    g0 = [x.clone() for x in batch.forward(list(fs))]
    a0 = [x.clone() for x in batch.adjoint(list(ds))]
    cache = str(tmp_path / "tune.json")
    chosen = batch.autotune(cache)
    entries = json.load(open(cache))
    (key, stored), = entries.items()
    assert key.startswith("batch count=4")
    assert {k: stored[k] for k in chosen} == chosen
    g1, a1 = batch.forward(list(fs)), batch.adjoint(list(ds))
    for i in range(len(plans)):
        assert torch.equal(g1[i], g0[i]) and torch.equal(a1[i], a0[i])
    batch.close()
    for p in plans:
        p.close()

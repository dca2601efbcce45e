"""pat_forward_noalloc, the forward operator on the library's own device
scratch array (for callers that cannot allocate), against pat_forward with a
caller workspace: same kernels and launch shapes, so the outputs must agree
bitwise.  Two calls in a row, the second on a smaller input (another plan,
fewer instances), so the second runs on whatever the first left in the
shared array; a batch whose workspace exceeds the array is rejected on the
host."""
import numpy as np
import pytest

from pat_inputs import CONFIGS, config_geometry, make_phantom

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_dev():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _stream(torch):
    import ctypes
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def test_forward_noalloc_equals_forward(torch_dev):
    torch = torch_dev
    import paper_2604_19176_amd as pat
    cases = [(config_geometry(2), 4, 2100), (config_geometry(1), 1, 2200)]   # second input smaller
    for geom, B, seed in cases:
        print("noalloc case: N=%d D=%d T=%d batch %d" % (geom.n, geom.n_det, geom.n_t, B), flush=True)
        nb, nd, nl = CONFIGS[2]["phantom"]
        f = torch.tensor(np.stack([make_phantom(geom.n, nb, nd, nl, seed + b) for b in range(B)]),
                         dtype=torch.float32, device="cuda")
        plan = pat.PatPlan(geom, max_batch=B)
        assert plan.workspace_bytes(B) <= pat.PAT_NOALLOC_SCRATCH_BYTES
        ref = plan.forward(f).clone()
        out = torch.full_like(ref, float("nan"))
        pat.pat_forward_noalloc(plan.handle, f.data_ptr(), out.data_ptr(), B, _stream(torch))
        torch.cuda.synchronize()
        assert torch.equal(out, ref)
        plan.close()


def test_forward_noalloc_rejects_oversized_batch(torch_dev):
    torch = torch_dev
    import paper_2604_19176_amd as pat
    geom = config_geometry(2)
    B = 32
    plan = pat.PatPlan(geom, max_batch=B)
    assert plan.workspace_bytes(B) > pat.PAT_NOALLOC_SCRATCH_BYTES
    f = torch.zeros((B, geom.n, geom.n), dtype=torch.float32, device="cuda")
    g = torch.zeros((B, geom.n_det, geom.n_t), dtype=torch.float32, device="cuda")
    with pytest.raises(pat.PatError) as e:
        pat.pat_forward_noalloc(plan.handle, f.data_ptr(), g.data_ptr(), B, _stream(torch))
    assert e.value.status == pat.PAT_ERR_WORKSPACE
    plan.close()


def test_forward_noalloc_two_streams(torch_dev):
    """A two-stream call on the library's array: its halves use disjoint
    instance slices of it, and the output is bitwise the one-stream call's."""
    torch = torch_dev
    import paper_2604_19176_amd as pat
    geom = config_geometry(2)
    B = 6
    print("noalloc two-stream case: N=%d batch %d" % (geom.n, B), flush=True)
    f = torch.tensor(np.stack([make_phantom(geom.n, 20, 3, 4, 2300 + b) for b in range(B)]),
                     dtype=torch.float32, device="cuda")
    plan = pat.PatPlan(geom, max_batch=B)
    plan.set_split(0)
    ref = plan.forward(f).clone()
    plan.set_split(2)
    out = torch.full_like(ref, float("nan"))
    pat.pat_forward_noalloc(plan.handle, f.data_ptr(), out.data_ptr(), B, _stream(torch))
    torch.cuda.synchronize()
    assert torch.equal(out, ref)
    plan.close()

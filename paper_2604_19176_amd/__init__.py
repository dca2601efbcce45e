"""MI355X (gfx950) library for the circular-geometry PAT operator pair.

The forward operator A maps an initial pressure image f (eq. (1), Sec. 2.1) to
the pressure traces g at detectors on a circle or arc (eq. (2)); A* is its
exact discrete transpose, the operator the gradients of eq. (4) and eq. (5)
need (Sec. 2.2).  All computation runs in the HIP kernels of libpat.so; this
package only marshals torch tensors (device memory and streams) into the C-ABI.

    plan = PatPlan(geometry, max_batch=B)        # tables built once (FP64 on the host)
    g = plan.forward(f)                           # f: (B, N, N) or (N, N) float32 on the GPU
    f_adj = plan.adjoint(g)
    g = pat_operator(plan, f)                     # autograd: backward runs A*
"""
from __future__ import annotations

import ctypes

import numpy as np

import torch

from . import _lib
from ._lib import (PatError, PAT_ERR_WORKSPACE, PAT_NOALLOC_SCRATCH_BYTES,  # noqa: F401
                   pat_plan_desc, pat_status_string, pat_plan_create, pat_plan_query,
                   pat_plan_destroy, pat_workspace_size, pat_forward, pat_forward_noalloc, pat_adjoint,
                   pat_stream_copy,
                   pat_tv_grad, pat_pgd_update, pat_residual, pat_plan_derive, pat_bessel_jn_table,
                   pat_profile_enable, pat_profile_read, pat_launch, pat_plan_get_launch, pat_plan_set_launch,
                   pat_plan_set_split, pat_plan_get_split,
                   pat_batch_create, pat_batch_destroy, pat_batch_workspace_size, pat_batch_forward,
                   pat_batch_adjoint, pat_batch_get_launch, pat_batch_set_launch, pat_autotune_plan,
                   pat_autotune_batch, pat_pd_dual_data, pat_pd_dual_tv, pat_pd_primal, pat_pd_change,
                   pat_cg_norm2, pat_cg_step_fr, pat_cg_step_p, pat_sim_create, pat_sim_query, pat_sim_run,
                   pat_sim_destroy)

__all__ = ["PatPlan", "PatBatch", "PatSim", "pat_operator", "PatOperatorFn", "tv_grad", "pgd_update", "residual",
           "PatError", "desc_from_geometry", "library_path"]


def library_path() -> str:
    return _lib.LIB_PATH


def desc_from_geometry(geom, max_batch: int = 1) -> pat_plan_desc:
    """pat_plan_desc from any object with the Geometry fields (explicit
    detector angles `det_theta`, if the object has them, are passed as a host
    array that the descriptor keeps alive)."""
    d = pat_plan_desc(int(geom.n), float(geom.support_r), float(geom.det_r), int(geom.n_det),
                      float(geom.arc_center), float(geom.arc_span), int(geom.n_t), float(geom.dt),
                      float(geom.c), float(geom.lambda_oversample), int(geom.em_correction),
                      int(max_batch), None)
    th = getattr(geom, "det_theta", None)
    if th is not None:
        arr = np.ascontiguousarray(th, dtype=np.float64)
        if arr.shape != (int(geom.n_det),):
            raise ValueError("det_theta needs n_det angles")
        d.det_theta = arr.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        d._keep = arr
    return d


def _stream(device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _check_tensor(t, name, shape_tail, device):
    if not isinstance(t, torch.Tensor):
        raise TypeError("%s must be a torch.Tensor" % name)
    if not t.is_cuda:
        raise ValueError("%s must be a GPU tensor (got device %s)" % (name, t.device))
    if device is not None and t.device != device:
        raise ValueError("%s is on %s but the plan lives on %s" % (name, t.device, device))
    if t.dtype != torch.float32:
        raise TypeError("%s must be float32 (got %s)" % (name, t.dtype))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if tuple(t.shape[-len(shape_tail):]) != tuple(shape_tail) or t.dim() not in (len(shape_tail),
                                                                                  len(shape_tail) + 1):
        raise ValueError("%s must have shape %s or (batch,) + %s, got %s"
                         % (name, tuple(shape_tail), tuple(shape_tail), tuple(t.shape)))
    return 1 if t.dim() == len(shape_tail) else int(t.shape[0])


def _check_out(t, name, shape, device):
    """A caller-supplied output must have exactly the shape the call writes
    (batch included): the kernels write that many floats."""
    if not isinstance(t, torch.Tensor):
        raise TypeError("%s must be a torch.Tensor" % name)
    if tuple(t.shape) != tuple(shape):
        raise ValueError("%s must have shape %s, got %s" % (name, tuple(shape), tuple(t.shape)))
    _check_tensor(t, name, shape[-2:], device)


def _check_like(t, name, ref, ref_name):
    """`t` must match `ref` in shape (checked first) and be a contiguous float32
    tensor on ref's GPU: the elementwise kernels read ref.numel() floats of it."""
    if not isinstance(t, torch.Tensor):
        raise TypeError("%s must be a torch.Tensor" % name)
    if tuple(t.shape) != tuple(ref.shape):
        raise ValueError("%s has shape %s but %s has %s" % (name, tuple(t.shape), ref_name, tuple(ref.shape)))
    _check_tensor(t, name, tuple(ref.shape[-2:]), ref.device)


class PatPlan:
    """A plan for one geometry: device tables plus a workspace for up to
    `max_batch` images, on the current CUDA/HIP device."""

    def __init__(self, geom, max_batch: int = 1, device=None):
        if not torch.cuda.is_available():
            raise RuntimeError("PatPlan needs a GPU: torch.cuda.is_available() is False")
        _lib.load()
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None
                                   else torch.device(device).index or 0)
        self.geom = geom
        self.max_batch = int(max_batch)
        with torch.cuda.device(self.device):
            self.handle = pat_plan_create(desc_from_geometry(geom, max_batch))
        self.info = pat_plan_query(self.handle)
        self._ws = None

    # -- sizes ------------------------------------------------------------------
    @property
    def image_shape(self):
        return (self.geom.n, self.geom.n)

    @property
    def data_shape(self):
        return (self.geom.n_det, self.geom.n_t)

    def workspace_bytes(self, batch: int) -> int:
        return pat_workspace_size(self.handle, batch)

    def workspace(self, batch: int):
        need = self.workspace_bytes(batch)
        if self._ws is None or self._ws.numel() < need:
            self._ws = torch.empty(max(need, self.workspace_bytes(self.max_batch)), dtype=torch.uint8,
                                   device=self.device)
        return self._ws

    # -- operators ----------------------------------------------------------------
    def forward(self, f, out=None):
        """g = A f.  f: (N, N) or (B, N, N) float32 contiguous on the plan's GPU."""
        B = _check_tensor(f, "f", self.image_shape, self.device)
        shape = self.data_shape if f.dim() == 2 else (B,) + self.data_shape
        if out is None:
            out = torch.empty(shape, dtype=torch.float32, device=self.device)
        else:
            _check_out(out, "out", shape, self.device)
        ws = self.workspace(B)
        pat_forward(self.handle, f.data_ptr(), out.data_ptr(), B, ws.data_ptr(), ws.numel(),
                    _stream(self.device))
        return out

    def adjoint(self, g, out=None):
        """f = A* g.  g: (D, T) or (B, D, T) float32 contiguous on the plan's GPU."""
        B = _check_tensor(g, "g", self.data_shape, self.device)
        shape = self.image_shape if g.dim() == 2 else (B,) + self.image_shape
        if out is None:
            out = torch.empty(shape, dtype=torch.float32, device=self.device)
        else:
            _check_out(out, "out", shape, self.device)
        ws = self.workspace(B)
        pat_adjoint(self.handle, g.data_ptr(), out.data_ptr(), B, ws.data_ptr(), ws.numel(),
                    _stream(self.device))
        return out

    # -- launch shapes ---------------------------------------------------------------
    @property
    def launch(self) -> dict:
        """The kernels' tile shapes (pat_launch fields)."""
        return pat_plan_get_launch(self.handle).asdict()

    def set_launch(self, **fields):
        """Change some tile shapes; the library checks them (PatError if they do not fit)."""
        c = pat_plan_get_launch(self.handle)
        for k, v in fields.items():
            if not hasattr(c, k):
                raise KeyError(k)
            setattr(c, k, int(v))
        pat_plan_set_launch(self.handle, c)

    @property
    def split(self) -> int:
        """Smallest batch whose calls run as two half-batches on two streams (0: never)."""
        return pat_plan_get_split(self.handle)

    def set_split(self, min_batch: int):
        """Calls of at least `min_batch` instances run half the batch on a second
        stream of the plan (bitwise the same outputs); 0 turns it off."""
        pat_plan_set_split(self.handle, min_batch)

    def autotune(self, batch: int | None = None, cache_path: str | None = None) -> dict:
        """Time candidate tile shapes at `batch` instances (default max_batch) and keep
        the fastest per stage; cached in the JSON file `cache_path` when given."""
        with torch.cuda.device(self.device):
            torch.cuda.synchronize(self.device)
            pat_autotune_plan(self.handle, self.max_batch if batch is None else int(batch), cache_path)
        return self.launch

    def close(self):
        if getattr(self, "handle", None):
            pat_plan_destroy(self.handle)
            self.handle = None
        self._ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class PatBatch:
    """A heterogeneous batch: instance i is evaluated with plans[i] (grid size,
    detector count, arc and time samples may differ).  forward/adjoint launch
    each stage of the operator once for all instances; the calls allocate
    nothing on the device once the pointer tables of a given set of tensors
    exist, so they can be recorded into a CUDA/HIP graph."""

    def __init__(self, plans):
        if not plans:
            raise ValueError("PatBatch needs at least one plan")
        self.plans = list(plans)
        self.device = self.plans[0].device
        for p in self.plans:
            if p.device != self.device:
                raise ValueError("all plans of a batch must live on one GPU")
        with torch.cuda.device(self.device):
            self.handle = pat_batch_create([p.handle for p in self.plans])
        self.count = len(self.plans)
        self._ws = torch.empty(max(pat_batch_workspace_size(self.handle), 256), dtype=torch.uint8,
                               device=self.device)
        self._ptr_tables = {}

    def _ptr_table(self, tensors, shapes, name):
        if len(tensors) != self.count:
            raise ValueError("%s: expected %d tensors, got %d" % (name, self.count, len(tensors)))
        for i, (t, shp) in enumerate(zip(tensors, shapes)):
            _check_tensor(t, "%s[%d]" % (name, i), shp, self.device)
            if t.dim() != 2:
                raise ValueError("%s[%d] must have shape %s" % (name, i, tuple(shp)))
        key = tuple(t.data_ptr() for t in tensors)
        tab = self._ptr_tables.get(key)
        if tab is None:
            tab = torch.tensor(key, dtype=torch.int64, device=self.device)
            self._ptr_tables[key] = tab
        return tab

    def forward(self, fs, outs=None):
        """[g_i] = [A_i f_i]; fs: list of (N_i, N_i) float32 GPU tensors."""
        if outs is None:
            outs = [torch.empty(p.data_shape, dtype=torch.float32, device=self.device) for p in self.plans]
        fp = self._ptr_table(fs, [p.image_shape for p in self.plans], "fs")
        gp = self._ptr_table(outs, [p.data_shape for p in self.plans], "outs")
        pat_batch_forward(self.handle, fp.data_ptr(), gp.data_ptr(), self._ws.data_ptr(), self._ws.numel(),
                          _stream(self.device))
        return outs

    def adjoint(self, gs, outs=None):
        """[f_i] = [A_i* g_i]; gs: list of (D_i, T_i) float32 GPU tensors."""
        if outs is None:
            outs = [torch.empty(p.image_shape, dtype=torch.float32, device=self.device) for p in self.plans]
        gp = self._ptr_table(gs, [p.data_shape for p in self.plans], "gs")
        fp = self._ptr_table(outs, [p.image_shape for p in self.plans], "outs")
        pat_batch_adjoint(self.handle, gp.data_ptr(), fp.data_ptr(), self._ws.data_ptr(), self._ws.numel(),
                          _stream(self.device))
        return outs

    @property
    def launch(self) -> dict:
        c = pat_batch_get_launch(self.handle).asdict()
        return {k: c[k] for k in ("gat_cb", "gat_th", "spr_cb", "spr_th")}

    def set_launch(self, **fields):
        c = pat_batch_get_launch(self.handle)
        for k, v in fields.items():
            if k not in ("gat_cb", "gat_th", "spr_cb", "spr_th"):
                raise KeyError(k)
            setattr(c, k, int(v))
        pat_batch_set_launch(self.handle, c)

    def autotune(self, cache_path: str | None = None) -> dict:
        with torch.cuda.device(self.device):
            torch.cuda.synchronize(self.device)
            pat_autotune_batch(self.handle, cache_path)
        return self.launch

    def close(self):
        if getattr(self, "handle", None):
            pat_batch_destroy(self.handle)
            self.handle = None
        self._ptr_tables = {}

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class PatSim:
    """The FFT wave-propagation data simulator for a geometry whose `n` is the
    fine grid side (the simulation study's finer Cartesian grid): run(f) maps
    an (n, n) float32 image on the GPU to (n_det, n_t) data."""

    def __init__(self, geom, device=None):
        if not torch.cuda.is_available():
            raise RuntimeError("PatSim needs a GPU: torch.cuda.is_available() is False")
        _lib.load()
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None
                                   else torch.device(device).index or 0)
        self.geom = geom
        with torch.cuda.device(self.device):
            self.handle = pat_sim_create(desc_from_geometry(geom, 1))
        self.box_side, self.workspace_bytes = pat_sim_query(self.handle)
        self._ws = None

    def run(self, f, out=None):
        _check_tensor(f, "f", (self.geom.n, self.geom.n), self.device)
        if f.dim() != 2:
            raise ValueError("f must be one (n, n) image")
        shape = (self.geom.n_det, self.geom.n_t)
        if out is None:
            out = torch.empty(shape, dtype=torch.float32, device=self.device)
        else:
            _check_tensor(out, "out", shape, self.device)
        if self._ws is None:
            self._ws = torch.empty(max(self.workspace_bytes, 256), dtype=torch.uint8, device=self.device)
        with torch.cuda.device(self.device):
            pat_sim_run(self.handle, f.data_ptr(), out.data_ptr(), self._ws.data_ptr(), self._ws.numel(),
                        _stream(self.device))
        return out

    def close(self):
        if getattr(self, "handle", None):
            pat_sim_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class PatOperatorFn(torch.autograd.Function):
    """A as an autograd Function: forward runs pat_forward, backward runs
    pat_adjoint on the incoming gradient (the gradient of <A f, w> is A* w)."""

    @staticmethod
    def forward(ctx, f, plan):
        ctx.plan = plan
        return plan.forward(f.contiguous())

    @staticmethod
    def backward(ctx, grad_g):
        return ctx.plan.adjoint(grad_g.contiguous()), None


def pat_operator(plan: PatPlan, f):
    """Differentiable g = A f (backward = A* on the GPU)."""
    return PatOperatorFn.apply(f, plan)


def tv_grad(f, eps: float = 1e-3, with_value: bool = False):
    """Gradient (and optionally the value per image) of the smoothed TV of eq. (4)."""
    if f.dim() == 2:
        n, B = f.shape[-1], 1
    else:
        n, B = f.shape[-1], f.shape[0]
    _check_tensor(f, "f", (n, n), f.device)
    grad = torch.empty_like(f)
    tv = torch.empty(B, dtype=torch.float32, device=f.device) if with_value else None
    pat_tv_grad(f.data_ptr(), grad.data_ptr(), tv.data_ptr() if tv is not None else None, n, B, eps,
                _stream(f.device))
    return (grad, tv) if with_value else grad


def pgd_update(f, adj, tvg, tau: float, lam: float):
    """In place: f <- max(f - tau (adj + lam tvg), 0).  f, adj and tvg (if
    given) are contiguous float32 GPU tensors of one shape, (N, N) or (B, N, N)."""
    if not isinstance(f, torch.Tensor) or f.dim() not in (2, 3):
        raise ValueError("f must be an (N, N) or (B, N, N) tensor")
    _check_like(adj, "adj", f, "f")
    if tvg is not None:
        _check_like(tvg, "tvg", f, "f")
    _check_tensor(f, "f", tuple(f.shape[-2:]), None)
    pat_pgd_update(f.data_ptr(), adj.data_ptr(), tvg.data_ptr() if tvg is not None else None, f.numel(),
                   tau, lam, _stream(f.device))
    return f


def residual(g, g_meas, with_value: bool = False):
    """In place: g <- g - g_meas; optionally 0.5 ||r||^2 per instance.  g and
    g_meas are contiguous float32 GPU tensors of one shape, (D, T) or (B, D, T)."""
    if not isinstance(g, torch.Tensor) or g.dim() not in (2, 3):
        raise ValueError("g must be a (D, T) or (B, D, T) tensor")
    _check_like(g_meas, "g_meas", g, "g")
    _check_tensor(g, "g", tuple(g.shape[-2:]), None)
    B = g.shape[0] if g.dim() == 3 else 1
    per = g.numel() // B
    sq = torch.empty(B, dtype=torch.float32, device=g.device) if with_value else None
    pat_residual(g.data_ptr(), g_meas.data_ptr(), sq.data_ptr() if sq is not None else None, per, B,
                 _stream(g.device))
    return (g, sq) if with_value else g


"""TV-regularised reconstruction (eq. (4), Sec. 2.1) driven by the GPU operator pair.

Projected gradient descent on 0.5 ||A f - g||^2 + lam TV_eps(f) with f >= 0:
    r   = A f - g                       (pat_forward + pat_residual)
    G   = A* r + lam grad TV_eps(f)     (pat_adjoint + pat_tv_grad)
    f  <- max(f - tau G, 0)             (pat_pgd_update)
Every step runs in the library's kernels; a run of iterations can be
captured once as a HIP graph and replayed.  The step is tau = 1 / (||A||^2 + 8 lam / eps),
a Lipschitz bound of the objective's gradient, with ||A||^2 from power
iteration on A* A.
"""
from __future__ import annotations

import torch

from . import PatPlan, pat_operator, pgd_update, residual, tv_grad


def operator_norm_sq(plan: PatPlan, iters: int = 30, seed: int = 0) -> float:
    """||A||^2 by power iteration on A* A (on the GPU)."""
    gen = torch.Generator(device=plan.device).manual_seed(seed)
    x = torch.rand(plan.image_shape, generator=gen, device=plan.device, dtype=torch.float32)
    lam = 0.0
    for _ in range(iters):
        x = x / x.norm()
        y = plan.adjoint(plan.forward(x))
        lam = float((x * y).sum())
        x = y
    return lam


class TVReconstructor:
    """State of the projected-gradient TV loop for one or more instances of a plan."""

    def __init__(self, plan: PatPlan, g_meas: torch.Tensor, lam: float, eps: float = 1e-3,
                 tau: float | None = None, f0: torch.Tensor | None = None):
        self.plan = plan
        self.lam = float(lam)
        self.eps = float(eps)
        self.g_meas = g_meas.contiguous()
        batch_shape = g_meas.shape[:-2]
        self.f = (torch.zeros(batch_shape + plan.image_shape, device=plan.device, dtype=torch.float32)
                  if f0 is None else f0.clone().contiguous())
        if tau is None:
            tau = 1.0 / (operator_norm_sq(plan) + 8.0 * self.lam / self.eps)
        self.tau = float(tau)
        self.r = torch.empty_like(self.g_meas)
        self.adj = torch.empty_like(self.f)
        self.graph = None
        self.graph_iters = 0

    def step(self):
        p = self.plan
        p.forward(self.f, out=self.r)
        residual(self.r, self.g_meas)
        p.adjoint(self.r, out=self.adj)
        tg = tv_grad(self.f, self.eps)
        pgd_update(self.f, self.adj, tg, self.tau, self.lam)

    def capture(self, iters: int = 1):
        """Record `iters` iterations as one HIP graph (torch.cuda.CUDAGraph);
        one iteration runs eagerly first (warm-up).  Several iterations per
        graph remove the gap between consecutive graph launches."""
        self.tg = torch.empty_like(self.f)
        s = torch.cuda.Stream(device=self.plan.device)
        s.wait_stream(torch.cuda.current_stream(self.plan.device))
        with torch.cuda.stream(s):
            self._step_static()  # warm-up outside capture
        torch.cuda.current_stream(self.plan.device).wait_stream(s)
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            for _ in range(iters):
                self._step_static()
        self.graph_iters = iters
        return self.graph

    def _step_static(self):
        from . import pat_tv_grad, _stream
        p = self.plan
        p.forward(self.f, out=self.r)
        residual(self.r, self.g_meas)
        p.adjoint(self.r, out=self.adj)
        B = 1 if self.f.dim() == 2 else self.f.shape[0]
        pat_tv_grad(self.f.data_ptr(), self.tg.data_ptr(), None, self.f.shape[-1], B, self.eps,
                    _stream(self.f.device))
        pgd_update(self.f, self.adj, self.tg, self.tau, self.lam)

    def run(self, steps: int, use_graph: bool = True):
        """`steps` iterations: whole graph replays, then the remainder eagerly."""
        if use_graph:
            if self.graph is None:
                self.capture()
            for _ in range(steps // self.graph_iters):
                self.graph.replay()
            for _ in range(steps % self.graph_iters):
                self._step_static()
        else:
            for _ in range(steps):
                self.step()
        return self.f


def tv_objective(plan: PatPlan, f, g_meas, lam: float, eps: float = 1e-3):
    """0.5 ||A f - g||^2 + lam TV_eps(f) per instance (GPU)."""
    r = plan.forward(f.contiguous())
    r, sq = residual(r, g_meas.contiguous(), with_value=True)
    _, tv = tv_grad(f.contiguous(), eps, with_value=True)
    return sq + lam * tv


def autograd_loss(plan: PatPlan, f, g_meas, lam: float, eps: float = 1e-3):
    """The same objective through autograd (backward runs A* on the GPU);
    the TV term's gradient is supplied by the TV kernel."""
    return _TVLoss.apply(pat_operator(plan, f), g_meas, f, lam, eps)


class _TVLoss(torch.autograd.Function):
    @staticmethod
    def forward(ctx, g, g_meas, f, lam, eps):
        r = (g - g_meas).contiguous()
        fc = f.detach().contiguous()
        tg, tv = tv_grad(fc, eps, with_value=True)
        ctx.save_for_backward(r, tg)
        ctx.lam = lam
        return 0.5 * (r * r).sum() + lam * tv.sum()

    @staticmethod
    def backward(ctx, go):
        r, tg = ctx.saved_tensors
        return go * r, None, go * ctx.lam * tg, None, None


class PDHGReconstructor:
    """Primal-dual TV reconstruction (the paper's classical baseline, Sec. 2.1):
    min_{f >= 0} 0.5 ||A f - g||^2 + alpha TV(f) with isotropic, unsmoothed TV,
    by the primal-dual hybrid gradient method with K = (A, grad), theta = 1 and
    sigma = tau = 0.99 / sqrt(||A||^2 + 8).  Stops when the relative change
    ||f_k - f_{k-1}|| / ||f_k|| of every instance is at most `tol` (1e-4, Sec. 2.3).
    One iteration runs the launches of the operator pair plus three small
    kernels, and the change reduction where the stopping rule reads it; a
    run of iterations can be captured as one HIP graph."""

    def __init__(self, plan: PatPlan, g_meas: torch.Tensor, alpha: float, sigma: float | None = None,
                 tau: float | None = None, f0: torch.Tensor | None = None):
        self.plan = plan
        self.alpha = float(alpha)
        self.g_meas = g_meas.contiguous()
        batch_shape = g_meas.shape[:-2]
        self.batch = 1 if g_meas.dim() == 2 else int(g_meas.shape[0])
        shape = batch_shape + plan.image_shape
        dev = plan.device
        self.f = (torch.zeros(shape, device=dev, dtype=torch.float32) if f0 is None
                  else f0.clone().contiguous())
        self.fbar = self.f.clone()
        self.y1 = torch.zeros_like(self.g_meas)
        self.y2 = torch.zeros(shape + (2,), device=dev, dtype=torch.float32)
        self.ax = torch.empty_like(self.g_meas)
        self.aty = torch.empty_like(self.f)
        self.change = torch.zeros(self.batch, 2, device=dev, dtype=torch.float32)
        if sigma is None or tau is None:
            s = 0.99 / (operator_norm_sq(plan) + 8.0) ** 0.5
            sigma = s if sigma is None else sigma
            tau = s if tau is None else tau
        self.sigma, self.tau = float(sigma), float(tau)
        self.graph = None
        self.graph_iters = 0
        self.iterations = 0

    def step(self, change: bool = True):
        """One iteration; `change` also reduces ||f_k - f_{k-1}||^2 and ||f_k||^2
        into self.change (the stopping rule's input)."""
        from . import _stream, pat_pd_change, pat_pd_dual_data, pat_pd_dual_tv, pat_pd_primal
        p, n, B = self.plan, self.plan.geom.n, self.batch
        st = _stream(self.f.device)
        p.forward(self.fbar, out=self.ax)
        pat_pd_dual_data(self.y1.data_ptr(), self.ax.data_ptr(), self.g_meas.data_ptr(), self.y1.numel(),
                         self.sigma, st)
        pat_pd_dual_tv(self.y2.data_ptr(), self.fbar.data_ptr(), n, B, self.sigma, self.alpha, st)
        p.adjoint(self.y1, out=self.aty)
        pat_pd_primal(self.f.data_ptr(), self.fbar.data_ptr(), self.aty.data_ptr(), self.y2.data_ptr(), n, B,
                      self.tau, st)
        if change:
            pat_pd_change(self.f.data_ptr(), self.fbar.data_ptr(), self.change.data_ptr(), n, B, st)

    def capture(self, iters: int = 10):
        """Record `iters` iterations as one HIP graph, the change reduction in
        the last only (runs one iteration eagerly first to warm up).  With
        `iters` equal to run()'s check interval, every check is one replay."""
        s = torch.cuda.Stream(device=self.plan.device)
        s.wait_stream(torch.cuda.current_stream(self.plan.device))
        with torch.cuda.stream(s):
            self.step()
        torch.cuda.current_stream(self.plan.device).wait_stream(s)
        self.iterations += 1
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            for i in range(iters):
                self.step(change=i == iters - 1)
        self.graph_iters = iters
        return self.graph

    def relative_change(self):
        c = self.change.cpu().double()  # copy, then widen on the host: no device kernel
        return (c[:, 0].sqrt() / c[:, 1].sqrt().clamp_min(1e-300)).tolist()

    def run(self, max_iters: int, tol: float | None = 1e-4, check_every: int = 10, use_graph: bool = True):
        """Iterate until every instance's relative change is <= tol (checked
        every `check_every` iterations) or max_iters; returns the iteration count."""
        if use_graph and self.graph is None:
            self.capture(check_every)
        done = 0
        while done < max_iters:
            k = min(check_every, max_iters - done)
            rest = k
            if use_graph:
                for _ in range(k // self.graph_iters):
                    self.graph.replay()
                rest = k % self.graph_iters
            for i in range(rest):
                self.step(change=i == rest - 1)
            done += k
            self.iterations += k
            if tol is not None and max(self.relative_change()) <= tol:
                break
        return self.iterations


class CGLSReconstructor:
    """CGLS (conjugate gradients on A* A f = A* g): the iterative stand-in for
    the fast inverse that gives the deep image prior its input (Sec. 2.2).
    Every scalar stays on the device; two consecutive steps (which alternate
    the two gamma buffers) can be captured as one HIP graph."""

    def __init__(self, plan: PatPlan, g_meas: torch.Tensor, f0: torch.Tensor | None = None):
        from . import _stream, pat_cg_norm2
        self.plan = plan
        self.g_meas = g_meas.contiguous()
        self.batch = 1 if g_meas.dim() == 2 else int(g_meas.shape[0])
        shape = g_meas.shape[:-2] + plan.image_shape
        dev = plan.device
        self.f = (torch.zeros(shape, device=dev, dtype=torch.float32) if f0 is None
                  else f0.clone().contiguous())
        self.nf = plan.geom.n * plan.geom.n
        self.nr = plan.geom.n_det * plan.geom.n_t
        self.r = torch.empty_like(self.g_meas)
        self.q = torch.empty_like(self.g_meas)
        self.s = torch.empty_like(self.f)
        self.gam = torch.zeros(2, self.batch, device=dev, dtype=torch.float32)
        self.qq = torch.zeros(self.batch, device=dev, dtype=torch.float32)
        self.rr = torch.zeros(self.batch, device=dev, dtype=torch.float32)
        # r = g - A f0, s = A* r, p = s, gamma = <s, s>
        self.r.copy_(self.g_meas)
        if f0 is not None:  # r -= 1 * A f0 with the CGLS update kernel (f += 1 * 0 leaves f alone)
            from . import pat_cg_step_fr
            plan.forward(self.f, out=self.q)
            one = torch.ones(self.batch, device=dev, dtype=torch.float32)
            zero = torch.zeros_like(self.f)
            pat_cg_step_fr(self.f.data_ptr(), zero.data_ptr(), self.nf, self.r.data_ptr(), self.q.data_ptr(),
                           self.nr, one.data_ptr(), one.data_ptr(), self.batch, _stream(dev))
        plan.adjoint(self.r, out=self.s)
        self.p = self.s.clone()
        pat_cg_norm2(self.s.data_ptr(), self.gam[0].data_ptr(), self.nf, self.batch, _stream(dev))
        self.cur = 0
        self.graph = None
        self.iterations = 0

    def _step(self, cur):
        from . import _stream, pat_cg_norm2, pat_cg_step_fr, pat_cg_step_p
        st = _stream(self.f.device)
        B = self.batch
        g_cur, g_new = self.gam[cur], self.gam[1 - cur]
        self.plan.forward(self.p, out=self.q)
        pat_cg_norm2(self.q.data_ptr(), self.qq.data_ptr(), self.nr, B, st)
        pat_cg_step_fr(self.f.data_ptr(), self.p.data_ptr(), self.nf, self.r.data_ptr(), self.q.data_ptr(), self.nr,
                       g_cur.data_ptr(), self.qq.data_ptr(), B, st)
        self.plan.adjoint(self.r, out=self.s)
        pat_cg_norm2(self.s.data_ptr(), g_new.data_ptr(), self.nf, B, st)
        pat_cg_step_p(self.p.data_ptr(), self.s.data_ptr(), self.nf, g_new.data_ptr(), g_cur.data_ptr(), B, st)

    def step(self):
        self._step(self.cur)
        self.cur = 1 - self.cur
        self.iterations += 1

    def capture(self):
        """Record two steps as a HIP graph (runs two steps eagerly first)."""
        s = torch.cuda.Stream(device=self.plan.device)
        s.wait_stream(torch.cuda.current_stream(self.plan.device))
        with torch.cuda.stream(s):
            self.step()
            self.step()
        torch.cuda.current_stream(self.plan.device).wait_stream(s)
        cur = self.cur
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            self._step(cur)
            self._step(1 - cur)
        return self.graph

    def residual_norm(self):
        """||g - A f|| per instance (from the recursively updated residual)."""
        from . import _stream, pat_cg_norm2
        pat_cg_norm2(self.r.data_ptr(), self.rr.data_ptr(), self.nr, self.batch, _stream(self.f.device))
        return self.rr.double().sqrt().cpu().tolist()

    def run(self, iters: int, use_graph: bool = True):
        """`iters` more steps (an even count with the graph: it holds two)."""
        if use_graph:
            if self.graph is None:
                self.capture()  # two eager steps
                iters -= 2
            while iters >= 2:
                self.graph.replay()
                self.iterations += 2
                iters -= 2
        for _ in range(iters):
            self.step()
        return self.iterations

"""Deep image prior (DIP) reconstruction, eq. (5) and Sec. 2.2.

    f^ = phi_theta*(z),  theta* = argmin_theta ||A phi_theta(z) - g||^2 + lambda TV(phi_theta(z))

* phi is the U-Net of Sec. 2.2.1: an encoder of four stages with 32, 64, 128
  and 256 feature channels (two 3x3 convolutions with batch normalisation and
  ReLU per stage, 2x2 max pooling between stages), a decoder of three stages
  (2x2 transposed convolution, concatenation with the encoder features of the
  same resolution, two 3x3 convolutions with batch normalisation and ReLU) and
  a final 3x3 convolution to one channel followed by ReLU (non-negativity).
  Stock PyTorch layers; the grid side must be divisible by 8.
* The data term runs A and A* in this library's kernels (`pat_operator`: the
  backward of A is A*); the TV term is the smoothed isotropic TV of the TV
  kernel (value and gradient in one launch).
* Adam with learning rate 5e-4, cosine annealing over the planned number of
  iterations (Sec. 2.2.1).
* The network input z is an approximate inverse of the data.  The paper uses
  a closed-form fast inverse from the cited literature, which it does not
  state; here z comes from a few CGLS steps (recon.CGLSReconstructor).
"""
from __future__ import annotations

import math

import torch
from torch import nn

from . import PatPlan, pat_operator, tv_grad


def _double_conv(cin: int, cout: int) -> nn.Sequential:
    return nn.Sequential(
        nn.Conv2d(cin, cout, 3, padding=1), nn.BatchNorm2d(cout), nn.ReLU(inplace=True),
        nn.Conv2d(cout, cout, 3, padding=1), nn.BatchNorm2d(cout), nn.ReLU(inplace=True))


class UNet(nn.Module):
    """The encoder-decoder of Sec. 2.2.1 (channels 32-64-128-256, three skips)."""

    def __init__(self, channels=(32, 64, 128, 256), in_ch: int = 1):
        super().__init__()
        c = list(channels)
        self.enc = nn.ModuleList([_double_conv(in_ch, c[0])] + [_double_conv(c[i], c[i + 1])
                                                                 for i in range(len(c) - 1)])
        self.pool = nn.MaxPool2d(2)
        self.up = nn.ModuleList([nn.ConvTranspose2d(c[i + 1], c[i], 2, stride=2) for i in reversed(range(len(c) - 1))])
        self.dec = nn.ModuleList([_double_conv(2 * c[i], c[i]) for i in reversed(range(len(c) - 1))])
        self.out = nn.Conv2d(c[0], 1, 3, padding=1)

    def forward(self, x):
        skips = []
        for i, stage in enumerate(self.enc):
            x = stage(x)
            if i < len(self.enc) - 1:
                skips.append(x)
                x = self.pool(x)
        for up, stage in zip(self.up, self.dec):
            x = up(x)
            x = stage(torch.cat([skips.pop(), x], dim=1))
        return torch.relu(self.out(x))


class _TVTerm(torch.autograd.Function):
    """lambda * TV_eps(f) per image, summed; the gradient comes from the TV kernel."""

    @staticmethod
    def forward(ctx, f, lam, eps):
        fc = f.detach().contiguous()
        grad, tv = tv_grad(fc, eps, with_value=True)
        ctx.save_for_backward(grad)
        ctx.lam = lam
        return lam * tv.sum()

    @staticmethod
    def backward(ctx, go):
        (grad,) = ctx.saved_tensors
        return go * ctx.lam * grad, None, None


def dip_objective(plan: PatPlan, f, g_meas, lam: float, eps: float = 1e-3):
    """||A f - g||^2 + lambda TV_eps(f) for an image f ((N, N) or (B, N, N)),
    differentiable in f (A* on the GPU in the backward)."""
    r = pat_operator(plan, f) - g_meas
    return (r * r).sum() + _TVTerm.apply(f, lam, eps)


def psnr(x, ref) -> float:
    """Peak signal-to-noise ratio of x against ref (peak = max |ref|)."""
    mse = float(((x - ref) ** 2).mean())
    peak = float(ref.abs().max())
    return float("inf") if mse == 0 else 10.0 * math.log10(peak * peak / mse)


class DIPReconstructor:
    """Optimises a freshly initialised U-Net for one measurement (eq. (5))."""

    def __init__(self, plan: PatPlan, g_meas: torch.Tensor, z: torch.Tensor, lam: float, iters: int,
                 lr: float = 5e-4, eps: float = 1e-3, seed: int = 0, channels=(32, 64, 128, 256),
                 dtype=torch.float32):
        if plan.geom.n % 8:
            raise ValueError("the U-Net needs a grid side divisible by 8")
        self.plan, self.lam, self.eps = plan, float(lam), float(eps)
        dev = plan.device
        self.g_meas = g_meas.contiguous()
        self.z = z.reshape(1, 1, plan.geom.n, plan.geom.n).to(device=dev, dtype=dtype)
        torch.manual_seed(seed)
        self.net = UNet(channels).to(device=dev, dtype=dtype)
        self.opt = torch.optim.Adam(self.net.parameters(), lr=lr)
        self.sched = torch.optim.lr_scheduler.CosineAnnealingLR(self.opt, T_max=max(int(iters), 1))
        self.iterations = 0
        self.last_loss = None

    def image(self):
        """The current reconstruction phi_theta(z), float32 (N, N)."""
        with torch.no_grad():
            return self.net(self.z)[0, 0].float().contiguous()

    def step(self):
        self.opt.zero_grad(set_to_none=True)
        f = self.net(self.z)[0, 0].float().contiguous()
        loss = dip_objective(self.plan, f, self.g_meas, self.lam, self.eps)
        loss.backward()
        self.opt.step()
        self.sched.step()
        self.iterations += 1
        self.last_loss = loss.detach()
        return self.last_loss

    def run(self, iters: int, truth: torch.Tensor | None = None, every: int = 1):
        """`iters` iterations; with a ground truth, the PSNR of the image before
        each recorded iteration (every `every`) and at the end."""
        hist = []
        for k in range(iters):
            if truth is not None and k % every == 0:
                hist.append((self.iterations, psnr(self.image(), truth)))
            self.step()
        if truth is not None:
            hist.append((self.iterations, psnr(self.image(), truth)))
        return hist

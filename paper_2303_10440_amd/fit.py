"""Staggered shape / PSF fitting driver (paper Sec. 5.2, "staggered" optimisation).

The paper fits a mesh and a Gaussian PSF to a target volume by alternating
two kinds of steps:

* shape steps: the PSF held fixed, the mesh transform evaluated on the narrow
  band of frequencies (Sec. 5.1), loss the weighted L2 distance
  <(I - I_GT)^2, I_GT> (normalised here by sum(I_GT)), vertices updated;
* PSF steps: the mesh held fixed, the exact transform (the full spectrum,
  band threshold 0, since the narrow band biases the PSF), loss the plain L2
  distance mean((I - I_GT)^2), the PSF parameters updated.

This module is a driver around the renderer: every image and every gradient
comes from ``dm.render`` / ``dm.render_vjp`` (the HIP kernels); the loss, its
derivative dL/dI and the optimiser update are a few elementwise torch
operations on device tensors.  The PSF is parameterised as in the benchmark
configurations, Sigma = diag(sigma_xy^2, sigma_xy^2, sigma_z^2), so
dL/dsigma_xy = 2 sigma_xy (dL/dSigma_xx + dL/dSigma_yy) and
dL/dsigma_z = 2 sigma_z dL/dSigma_zz.

Vertex updates: Adam, the paper's uniform Adam (one second-moment scale for
the whole vertex array, its maximum, so every vertex moves by a step of the
same size), or plain gradient steps; optionally on the smoothed gradient
(I + lambda L)^{-2} dL/dV of Sec. 5.2 (``dm.laplace_smooth``, lambda = 50 in
the paper).
"""
from __future__ import annotations

import dataclasses

import paper_2303_10440_amd as dm


def sigma6(sigma_xy: float, sigma_z: float) -> tuple[float, ...]:
    return (sigma_xy * sigma_xy, sigma_xy * sigma_xy, sigma_z * sigma_z, 0.0, 0.0, 0.0)


def weighted_l2(img, target):
    """Loss <(I - I_GT)^2, I_GT> / sum(I_GT) and its derivative in I."""
    w = target / target.sum()
    d = img - target
    return float((d * d * w).sum()), 2.0 * d * w


def plain_l2(img, target):
    """Loss mean((I - I_GT)^2) and its derivative in I."""
    n = img.numel()
    d = img - target
    return float((d * d).sum()) / n, (2.0 / n) * d


class _Adam:
    """Adam on one device tensor (state on the same device)."""

    def __init__(self, like, lr: float, betas=(0.9, 0.999), eps: float = 1e-8):
        self.lr, (self.b1, self.b2), self.eps = lr, betas, eps
        self.m = like.new_zeros(like.shape)
        self.v = like.new_zeros(like.shape)
        self.t = 0

    def step(self, x, g):
        self.t += 1
        self.m.mul_(self.b1).add_(g, alpha=1.0 - self.b1)
        self.v.mul_(self.b2).addcmul_(g, g, value=1.0 - self.b2)
        mh = self.m / (1.0 - self.b1 ** self.t)
        vh = self.v / (1.0 - self.b2 ** self.t)
        x.sub_(self.lr * mh / (vh.sqrt() + self.eps))


class _AdamUniform(_Adam):
    """Adam whose second-moment estimate is replaced by its maximum over the
    array: the update direction is m_hat / sqrt(max v_hat)."""

    def step(self, x, g):
        self.t += 1
        self.m.mul_(self.b1).add_(g, alpha=1.0 - self.b1)
        self.v.mul_(self.b2).addcmul_(g, g, value=1.0 - self.b2)
        mh = self.m / (1.0 - self.b1 ** self.t)
        vmax = self.v.max() / (1.0 - self.b2 ** self.t)
        x.sub_(self.lr * mh / (vmax.sqrt() + self.eps))


class _Sgd:
    def __init__(self, like, lr: float):
        self.lr = lr

    def step(self, x, g):
        x.sub_(self.lr * g)


@dataclasses.dataclass
class FitConfig:
    lr_shape: float = 0.05           # length units per step (Adam) or per unit gradient (sgd)
    lr_psf: float = 0.02
    shape_steps: int = 10            # per round
    psf_steps: int = 2               # per round
    optimizer: str = "adam"          # "adam", "adam_uniform" or "sgd" (vertex steps; PSF steps use Adam or sgd)
    weighted: bool = True            # weighted L2 for the shape steps (plain L2 if False)
    smooth_lambda: float | None = None   # filter dL/dV by (I + lambda L)^{-2} before the vertex step
    smooth_tol: float = 1e-6


class StaggeredFit:
    """Fit vertices and (sigma_xy, sigma_z) to a target image.

    verts: float32 device tensor [n_v, 3] (updated in place); target: float32
    device tensor with the grid's shape.  ``grid.tau`` is the narrow band of
    the shape steps; the PSF steps use the same grid with tau = 0."""

    def __init__(self, handle, topo, verts, sigma_xy: float, sigma_z: float, grid, target,
                 config: FitConfig | None = None):
        import torch
        self.h, self.topo, self.grid, self.target = handle, topo, grid, target
        self.cfg = config or FitConfig()
        self.verts = verts
        self.psf = torch.tensor([sigma_xy, sigma_z], dtype=torch.float64)
        self.grid_exact = dataclasses.replace(grid, tau=0.0)
        opt_v = {"adam": _Adam, "adam_uniform": _AdamUniform, "sgd": _Sgd}[self.cfg.optimizer]
        self.opt_v = opt_v(verts, self.cfg.lr_shape)
        self.opt_p = (_Sgd if self.cfg.optimizer == "sgd" else _Adam)(self.psf, self.cfg.lr_psf)
        self.history: list[tuple[str, float]] = []

    def sigma6(self):
        sxy, sz = (float(x) for x in self.psf)
        return sigma6(sxy, sz)

    def shape_gradient(self):
        """(loss, dL/dverts) for the current state (narrow band, PSF fixed)."""
        S = self.sigma6()
        img, spec = dm.render(self.h, self.verts, self.topo, S, self.grid, spectrum=True)
        loss_fn = weighted_l2 if self.cfg.weighted else plain_l2
        loss, dI = loss_fn(img, self.target)
        dv, _, _ = dm.render_vjp(self.h, self.verts, self.topo, S, self.grid, dI.contiguous(), want_sigma=False,
                                 spectrum_in=spec)
        return loss, dv

    def psf_gradient(self):
        """(loss, dL/d(sigma_xy, sigma_z)) for the current state (full spectrum, shape fixed)."""
        import torch
        S = self.sigma6()
        img, spec = dm.render(self.h, self.verts, self.topo, S, self.grid_exact, spectrum=True)
        loss, dI = plain_l2(img, self.target)
        _, dS, _ = dm.render_vjp(self.h, self.verts, self.topo, S, self.grid_exact, dI.contiguous(),
                                 want_verts=False, spectrum_in=spec)
        dS = dS.double().cpu()
        sxy, sz = self.psf
        g = torch.stack([2.0 * sxy * (dS[0] + dS[1]), 2.0 * sz * dS[2]])
        return loss, g

    def shape_step(self) -> float:
        loss, dv = self.shape_gradient()
        if self.cfg.smooth_lambda is not None:
            dv = dm.laplace_smooth(self.h, self.topo, dv.contiguous(), lam=self.cfg.smooth_lambda,
                                   tol=self.cfg.smooth_tol)
        self.opt_v.step(self.verts, dv)
        self.history.append(("shape", loss))
        return loss

    def psf_step(self) -> float:
        loss, g = self.psf_gradient()
        self.opt_p.step(self.psf, g)
        self.psf.clamp_(min=1e-3)
        self.history.append(("psf", loss))
        return loss

    def run(self, rounds: int):
        for _ in range(rounds):
            for _ in range(self.cfg.shape_steps):
                self.shape_step()
            for _ in range(self.cfg.psf_steps):
                self.psf_step()
        return self.history

"""3D-VAR harness on the GPU: the covariance operator as a differentiable torch
operation, the bilinear observation operator, the cost and its gradient, and a
conjugate-gradient minimiser.

Sec. 2.1 minimises a quadratic cost in the increment through a preconditioned
linear system solved by conjugate gradients, with the background covariance
factored as B = V V^T.  With the control variable v (increment = V v) the cost is
    J(v) = 1/2 v.v + 1/2 (H V v - y).R^-1.(H V v - y),   grad J = v + V^T H^T R^-1 (H V v - y)
and CG solves (I + V^T H^T R^-1 H V) v = V^T H^T R^-1 y, the same minimiser.
Here V = V_H = G_y G_x per level.  Every iteration calls V and V^T once; both,
H, H^T, the weighted innovation R^-1 (H V v - y), the gradient's sum and the CG
vector steps (deterministic FP64 dot products, scalars kept on the device) are
librf3 calls.  torch only holds the vectors.
"""
from __future__ import annotations

import numpy as np
import torch

from . import rf3
from .operator import HorizontalCovariance


class RF3XY(torch.autograd.Function):
    """y = V x with V = G_y G_x; the backward pass applies V^T (no saved activations)."""

    @staticmethod
    def forward(ctx, x, op):
        ctx.op = op
        return op.apply(x)

    @staticmethod
    def backward(ctx, g):
        return ctx.op.adjoint(g.contiguous()), None


def rf3xy(x: torch.Tensor, op: HorizontalCovariance) -> torch.Tensor:
    return RF3XY.apply(x, op)


class Observations:
    """Bilinear observation operator on one [nlev][ny][nx] field (rf_obs_*)."""

    def __init__(self, op: HorizontalCovariance, lev, x, y, device=None):
        self.op = op
        plan, self.nuniq = rf3.rf_obs_plan(op.grid, lev, x, y)
        self.nobs = len(lev)
        self.npts = op.nx * op.ny * op.nlev
        dev = op.device if device is None else device
        # torch's caching allocator returns 512-byte aligned blocks
        self.plan = torch.frombuffer(bytearray(plan), dtype=torch.uint8).to(dev)
        self.shape = (op.nlev, op.ny, op.nx)

    @staticmethod
    def _prec(t):
        if t.dtype == torch.float32:
            return rf3.RF_FP32
        if t.dtype == torch.float64:
            return rf3.RF_FP64
        raise TypeError(f"float32 or float64 expected, got {t.dtype}")

    def apply(self, field, out=None, stream=None):
        field = field.contiguous()
        if field.numel() != self.npts:
            raise ValueError(f"field has {field.numel()} points, the plan {self.npts}")
        out = torch.empty(self.nobs, dtype=field.dtype, device=field.device) if out is None else out
        rf3.rf_obs_apply(self.plan, self.nobs, self.nuniq, self.npts, self._prec(field), field, out, stream)
        return out

    def adjoint(self, obs, out=None, stream=None):
        obs = obs.contiguous()
        if obs.numel() != self.nobs:
            raise ValueError(f"{obs.numel()} values for {self.nobs} observations")
        out = torch.empty(self.shape, dtype=obs.dtype, device=obs.device) if out is None else out
        rf3.rf_obs_adjoint(self.plan, self.nobs, self.nuniq, self.npts, self._prec(obs), obs, out, stream)
        return out


class Var3D:
    """J(v), grad J(v) and CG for the control variable v (shape [nlev][ny][nx])."""

    def __init__(self, op: HorizontalCovariance, obs: Observations, yobs, rinv):
        self.op, self.obs = op, obs
        self.y = yobs
        self.rinv = rinv   # scalar or tensor over the observations
        dev = yobs.device
        self.prec = Observations._prec(yobs)
        self.s = torch.zeros(rf3.RF_CG_SLOTS, dtype=torch.float64, device=dev)   # device scalars
        self.work = torch.empty(rf3.rf_cg_work_bytes() // 8, dtype=torch.float64, device=dev)

    def _dots(self, pairs):
        """FP64 dot products (deterministic, librf3), returned to the host."""
        for k, (a, b) in enumerate(pairs):
            rf3.rf_dot(self.prec, a.numel(), a, b, self.work, self.s, 3 + k)
        return self.s[3:3 + len(pairs)].tolist()

    def _innov(self, field, yobs, scale, d=None):
        """rd = scale * R^-1 (H field - yobs) in observation space (librf3); None drops a term."""
        o = self.obs
        rd = torch.empty(o.nobs, dtype=self.y.dtype, device=self.y.device)
        if torch.is_tensor(self.rinv):
            rinv, sc = self.rinv.to(self.y.dtype).contiguous(), scale
        else:
            rinv, sc = None, scale * float(self.rinv)
        rf3.rf_obs_innovation(o.plan, o.nobs, o.nuniq, o.npts, self.prec, field, yobs, rinv, sc, d, rd)
        return rd

    def cost_grad(self, v):
        d = torch.empty_like(self.y)
        rd = self._innov(self.op.apply(v), self.y, 1.0, d=d)
        vv, drd = self._dots([(v, v), (d, rd)])
        J = 0.5 * vv + 0.5 * drd
        g = self.op.adjoint(self.obs.adjoint(rd))
        rf3.rf_axpy(self.prec, g.numel(), 1.0, v, g)   # g = v + V^T H^T R^-1 (H V v - y)
        return J, g

    def _vthv(self, p):
        """V^T H^T R^-1 H V p."""
        return self.op.adjoint(self.obs.adjoint(self._innov(self.op.apply(p), None, 1.0)))

    def hess(self, p):
        """(I + V^T H^T R^-1 H V) p."""
        w = self._vthv(p)
        rf3.rf_axpy(self.prec, w.numel(), 1.0, p, w)
        return w

    def cg(self, iters, callback=None, track_cost=True):
        """CG from v = 0 on the normal equations; returns v and J after every iteration
        (only J at v = 0 and at the end when track_cost is False).  The iteration's
        scalars stay on the device: no host round trip inside the loop unless J is tracked."""
        n = self.obs.npts
        v = torch.zeros(self.obs.shape, dtype=self.y.dtype, device=self.y.device)
        r = self.op.adjoint(self.obs.adjoint(self._innov(None, self.y, -1.0)))   # V^T H^T R^-1 y
        p = r.clone()
        rf3.rf_dot(self.prec, n, r, r, self.work, self.s, rf3.RF_CG_RR)
        costs = [self.cost_grad(v)[0]]
        for k in range(iters):
            w = self._vthv(p)                                                # A p = p + w
            rf3.rf_cg_q_dot(self.prec, n, p, w, None, self.work, self.s)    # p.(p + w)
            rf3.rf_cg_step_pw(self.prec, n, p, w, v, r, self.work, self.s)  # v += a p, r -= a (p + w), r.r
            rf3.rf_cg_dir(self.prec, n, r, p, self.s)                       # p = r + b p
            if track_cost:
                costs.append(self.cost_grad(v)[0])
            if callback is not None:
                callback(k, v)
        if not track_cost:
            costs.append(self.cost_grad(v)[0])
        return v, costs


def synthetic_problem(w, nobs, device, dtype=torch.float32, op=None, obs_noise=0.5, seed=None):
    """C5-style twin experiment on workload w: v_true ~ N(0,1) on sea, y = H V v_true + noise."""
    from . import synth
    op = op or HorizontalCovariance(w.mask, w.sigma_x, w.sigma_y, w.nlev, n_img=w.n_img, qmode=w.qmode,
                                    device=device)
    lev, xs, ys = synth.c5_observations(w, nobs, seed=seed)
    obs = Observations(op, lev, xs, ys)
    rng = np.random.default_rng(synth.SEEDS["c5"] if seed is None else seed)
    vt = rng.standard_normal((w.nlev, w.ny, w.nx)) * (w.mask[0] != 0)
    vt = torch.from_numpy(vt).to(device=device, dtype=dtype)
    yobs = obs.apply(op.apply(vt)) + obs_noise * torch.from_numpy(rng.standard_normal(nobs)).to(device, dtype)
    return Var3D(op, obs, yobs, 1.0 / obs_noise ** 2), vt

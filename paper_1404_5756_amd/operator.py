"""V_H = G_y G_x on a GPU-resident grid: holds the grid and its coefficient block.

Thin object wrapper over the C ABI (rf3.py); every computation is a librf3 call.
"""
from __future__ import annotations

import numpy as np
import torch

from . import rf3


def _dev_tensor(a, dtype, device):
    if isinstance(a, torch.Tensor):
        return a.to(device=device, dtype=dtype).contiguous()
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device=device)


class HorizontalCovariance:
    """Operator V_H (3rd-RF) with its adjoint and the 1st-RF baseline on one grid.

    mask: [mask_nlev][ny][nx] (nonzero = sea); sigma_x, sigma_y: [sigma_nlev][ny][nx] in grid units.
    periodic_x: zonally periodic rows (RF_PERIODIC_X); exact_ends: exact end conditions of the
    3rd-RF (RF_EXACT_ENDS).
    """

    def __init__(self, mask, sigma_x, sigma_y, nlev, n_img=0, qmode="literal", k1=5, device="cuda",
                 stream=None, periodic_x=False, exact_ends=False):
        mask = np.asarray(mask.cpu() if isinstance(mask, torch.Tensor) else mask)
        if mask.ndim == 2:
            mask = mask[None]
        sx = sigma_x if isinstance(sigma_x, torch.Tensor) else np.asarray(sigma_x, np.float64)
        sy = sigma_y if isinstance(sigma_y, torch.Tensor) else np.asarray(sigma_y, np.float64)
        if sx.ndim == 2:
            sx = sx[None]
        if sy.ndim == 2:
            sy = sy[None]
        ny, nx = mask.shape[1:]
        self.device = torch.device(device)
        flags = (rf3.RF_PERIODIC_X if periodic_x else 0) | (rf3.RF_EXACT_ENDS if exact_ends else 0)
        self.grid = rf3.make_grid(nx, ny, nlev, mask.shape[0], sx.shape[0], n_img, qmode, k1, flags)
        nbytes = rf3.rf_coeffs_bytes(self.grid)
        if nbytes == 0:
            raise rf3.RFError(rf3.RF_E_SHAPE, "rf_coeffs_bytes")
        # 256-byte aligned: torch's caching allocator returns 512-byte aligned blocks
        self.coef = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        m = _dev_tensor((mask != 0).astype(np.uint8), torch.uint8, self.device)
        sxd = _dev_tensor(sx, torch.float64, self.device)
        syd = _dev_tensor(sy, torch.float64, self.device)
        rf3.rf_coeffs(self.grid, m, sxd, syd, self.coef, stream)
        self.nx, self.ny, self.nlev = nx, ny, nlev

    # fields: [nfields][nlev][ny][nx] (or [nlev][ny][nx] / [ny][nx])
    def _shape(self, x):
        if x.dim() == 2:
            return 1, 1
        if x.dim() == 3:
            return 1, x.shape[0]
        return x.shape[0], x.shape[1]

    def _prec(self, x):
        if x.dtype == torch.float32:
            return rf3.RF_FP32
        if x.dtype == torch.float64:
            return rf3.RF_FP64
        raise TypeError(f"fields must be float32 or float64, got {x.dtype}")

    def apply(self, x, out=None, stream=None):
        """out = G_y G_x x."""
        x = x.contiguous()
        out = torch.empty_like(x) if out is None else out
        nf, nl = self._shape(x)
        rf3.rf3_apply_xy(self.grid, self.coef, self._prec(x), x, out, nl, nf, stream)
        return out

    def adjoint(self, x, out=None, stream=None):
        """out = G_x^T G_y^T x."""
        x = x.contiguous()
        out = torch.empty_like(x) if out is None else out
        nf, nl = self._shape(x)
        rf3.rf3_adjoint_xy(self.grid, self.coef, self._prec(x), x, out, nl, nf, stream)
        return out

    def apply_dir(self, x, direction, adjoint=False, out=None, stream=None):
        """One direction only: G_x (direction 0 / 'x') or G_y (1 / 'y'), or its transpose."""
        d = {"x": 0, "y": 1}.get(direction, direction)
        x = x.contiguous()
        out = torch.empty_like(x) if out is None else out
        nf, nl = self._shape(x)
        rf3.rf3_apply_dir(self.grid, self.coef, self._prec(x), d, int(bool(adjoint)), x, out, nl, nf, stream)
        return out

    def rf1(self, x, K=None, out=None, stream=None):
        """1st-RF baseline, K iterations per direction (FP64)."""
        x = x.contiguous()
        out = torch.empty_like(x) if out is None else out
        nf, nl = self._shape(x)
        rf3.rf1_apply_xy(self.grid, self.coef, self._prec(x), self.grid.k1 if K is None else K, x, out,
                         nl, nf, stream)
        return out


    def rf1_fused(self, x, K=None, out=None, stream=None):
        """1st-RF with all K iterations of a direction on chip (FP32 or FP64)."""
        x = x.contiguous()
        out = torch.empty_like(x) if out is None else out
        nf, nl = self._shape(x)
        rf3.rf1_apply_xy_fused(self.grid, self.coef, self._prec(x), self.grid.k1 if K is None else K, x, out,
                               nl, nf, stream)
        return out


class Batch:
    """Several (operator, input, output) items applied together (rf3_apply_batch).

    items: [(HorizontalCovariance, x, y)] with x, y FP32 device tensors
    [nfields][op.nlev][ny][nx] (y may be x).  The work list is built once here
    and kept on the device; build a new Batch when any tensor changes.
    tuning: None (default work-list shape) or (x_groups_max, y_planes[, x_one_launch]),
    see rf_batch_tuning; autotune() picks one by timing.
    """

    # candidate work-list shapes tried by autotune(): (x_groups_max, y_planes, x_one_launch)
    CANDIDATES = tuple((xg, yp, one) for one in (0, 1) for xg in (1, 2, 4, 8, 16) for yp in (1, 2, 3, 4, 6, 8, 16))

    def __init__(self, items, device=None, tuning=None):
        self._items = []
        self._keep = []
        for op, x, y in items:
            if x.dtype != torch.float32 or y.dtype != torch.float32:
                raise TypeError("batched fields must be float32")
            if x.dim() != 4 or tuple(x.shape[1:]) != (op.nlev, op.ny, op.nx) or x.shape != y.shape:
                raise ValueError(f"expected [nfields][{op.nlev}][{op.ny}][{op.nx}], got {tuple(x.shape)}")
            if not (x.is_contiguous() and y.is_contiguous()):
                raise ValueError("batched fields must be contiguous")
            self._items.append((op.grid, op.coef, x, y, x.shape[0]))
            self._keep.append((op, x, y))
        self.device = device if device is not None else self._items[0][2].device
        self._set_tuning(tuning)

    @staticmethod
    def _norm(tuning):
        """(x_groups_max, y_planes, x_one_launch) of a 2- or 3-tuple, or None."""
        return None if tuning is None else (int(tuning[0]), int(tuning[1]), int(tuning[2]) if len(tuning) > 2 else 0)

    def _set_tuning(self, tuning):
        self.tuning = self._norm(tuning)
        host = rf3.rf3_batch_plan(self._items, self.tuning)
        # torch's caching allocator returns 512-byte aligned blocks
        self.plan = torch.frombuffer(bytearray(host), dtype=torch.uint8).to(self.device)

    @property
    def points(self):
        return sum(x.numel() for _, x, _ in self._keep)

    def apply(self, adjoint=False, stream=None):
        rf3.rf3_apply_batch(self._items, rf3.RF_FP32, int(bool(adjoint)), self.plan, self.plan.numel(), stream,
                            self.tuning)

    # autotune results per (device architecture, CU count, item shapes): a batch of
    # the same shapes on the same kind of device reuses the shape found before
    _tuned = {}

    def signature(self):
        """(architecture, CUs, sorted item shapes and flags): what the best work-list shape depends on."""
        props = torch.cuda.get_device_properties(self.device)
        arch = getattr(props, "gcnArchName", props.name)
        shapes = tuple(sorted((g.nx, g.ny, g.nlev, g.mask_nlev, g.sigma_nlev, g.flags, int(nf))
                              for g, _c, _x, _y, nf in self._items))
        return (arch, props.multi_processor_count, shapes)

    def autotune(self, candidates=None, reps=3, cache=True, finalists=4, rounds=3):
        """Time forward + adjoint for each candidate work-list shape on these items
        and keep the fastest.  The batch is applied repeatedly: the items' outputs
        (and inputs, for items applied in place) are overwritten.  Returns
        {shape: ms}, shapes as (x_groups_max, y_planes, x_one_launch), with the
        default shape under the key None.  Shapes a few percent apart are within
        the timing noise, so the fastest `finalists` shapes and the default are
        timed again in `rounds` interleaved rounds, and the best mean over those
        rounds (their entries in the result) wins.  With cache, a batch
        whose signature() was tuned before in this process takes that shape without
        timing (and returns {}); results do not depend on the shape (bitwise)."""
        key = self.signature() if cache and candidates is None else None
        if key is not None and key in Batch._tuned:
            self._set_tuning(Batch._tuned[key])
            return {}
        stream = torch.cuda.current_stream(self.device)

        def timed(t):
            self._set_tuning(t)
            self.apply(False)
            self.apply(True)
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            for _ in range(reps):
                self.apply(False)
                self.apply(True)
            b.record(stream)
            b.synchronize()
            return a.elapsed_time(b) / reps

        times = {}
        for t in [None] + [self._norm(c) for c in (candidates if candidates is not None else self.CANDIDATES)]:
            times[t] = timed(t)
        final = sorted(times, key=times.get)[:finalists]
        if None not in final:
            final.append(None)
        acc = dict.fromkeys(final, 0.0)
        for _ in range(rounds):
            for t in final:
                acc[t] += timed(t)
        for t in final:
            times[t] = acc[t] / rounds
        best = min(final, key=times.get)
        self._set_tuning(best)
        if key is not None:
            Batch._tuned[key] = best
        return times

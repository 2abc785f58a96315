"""Python binding of librf3 (include/rf3.h): argument marshalling only.

Every function here has the name of the C entry point it calls and takes torch
tensors that live on the GPU (torch is used for device memory and streams; all
arithmetic runs in librf3's HIP kernels).  There is no CPU fallback: if
librf3.so is missing the import of this module's functions raises.
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librf3.so")

RF_OK, RF_E_ARG, RF_E_SHAPE, RF_E_SIGMA, RF_E_HIP, RF_E_UNSUPPORTED = 0, -1, -2, -3, -4, -5
RF_FP32, RF_FP64 = 0, 1
RF_Q_LITERAL, RF_Q_VARMATCH, RF_Q_FIT = 0, 1, 2
RF_CG_RR, RF_CG_PQ, RF_CG_RR_NEW, RF_CG_SLOTS = 0, 1, 2, 8
RF_PERIODIC_X, RF_EXACT_ENDS = 1, 2
QMODES = {"literal": RF_Q_LITERAL, "varmatch": RF_Q_VARMATCH, "fit": RF_Q_FIT}


class rf_grid(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int32) for n in
                ("nx", "ny", "nlev", "mask_nlev", "sigma_nlev", "n_img", "qmode", "k1", "flags")]

    def __repr__(self):
        return "rf_grid(" + ", ".join(f"{n}={getattr(self, n)}" for n, _ in self._fields_) + ")"


class rf_batch_item(ctypes.Structure):
    _fields_ = [("g", ctypes.POINTER(rf_grid)), ("coef", ctypes.c_void_p), ("in_", ctypes.c_void_p),
                ("out", ctypes.c_void_p), ("nfields", ctypes.c_int32)]


class rf_batch_tuning(ctypes.Structure):
    _fields_ = [("x_groups_max", ctypes.c_int32), ("y_planes", ctypes.c_int32), ("x_one_launch", ctypes.c_int32)]

    def __repr__(self):
        return (f"rf_batch_tuning(x_groups_max={self.x_groups_max}, y_planes={self.y_planes}, "
                f"x_one_launch={self.x_one_launch})")


class RFError(RuntimeError):
    def __init__(self, status, where):
        super().__init__(f"{where}: {rf_strerror(status)} (status {status})")
        self.status = status


_lib = None


def lib() -> ctypes.CDLL:
    """Load librf3.so (built in-tree by paper_1404_5756_amd.build)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_1404_5756_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        P, I, S = ctypes.c_void_p, ctypes.c_int32, ctypes.c_size_t
        G = ctypes.POINTER(rf_grid)
        B = ctypes.POINTER(rf_batch_item)
        L.rf_coeffs_bytes.restype = S
        L.rf_coeffs_bytes.argtypes = [G]
        L.rf_coeffs.restype = I
        L.rf_coeffs.argtypes = [G, P, P, P, P, P]
        for name in ("rf3_apply_xy", "rf3_adjoint_xy"):
            f = getattr(L, name)
            f.restype = I
            f.argtypes = [G, P, I, P, P, I, I, P]
        L.rf3_apply_dir.restype = I
        L.rf3_apply_dir.argtypes = [G, P, I, I, I, P, P, I, I, P]
        L.rf1_apply_xy.restype = I
        L.rf1_apply_xy.argtypes = [G, P, I, I, P, P, I, I, P]
        L.rf1_apply_xy_fused.restype = I
        L.rf1_apply_xy_fused.argtypes = [G, P, I, I, P, P, I, I, P]
        L.rf3_batch_plan_bytes.restype = S
        L.rf3_batch_plan_bytes.argtypes = [B, I]
        L.rf3_batch_plan.restype = I
        L.rf3_batch_plan.argtypes = [B, I, P, S]
        L.rf3_apply_batch.restype = I
        L.rf3_apply_batch.argtypes = [B, I, I, I, P, S, P]
        T = ctypes.POINTER(rf_batch_tuning)
        L.rf3_batch_plan_bytes_ex.restype = S
        L.rf3_batch_plan_bytes_ex.argtypes = [B, I, T]
        L.rf3_batch_plan_ex.restype = I
        L.rf3_batch_plan_ex.argtypes = [B, I, T, P, S]
        L.rf3_apply_batch_ex.restype = I
        L.rf3_apply_batch_ex.argtypes = [B, I, T, I, I, P, S, P]
        D = ctypes.POINTER(ctypes.c_double)
        IP = ctypes.POINTER(ctypes.c_int32)
        L.rf_obs_plan_bytes.restype = S
        L.rf_obs_plan_bytes.argtypes = [G, I, IP, D, D, IP]
        L.rf_obs_plan.restype = I
        L.rf_obs_plan.argtypes = [G, I, IP, D, D, P, S]
        for name in ("rf_obs_apply", "rf_obs_adjoint"):
            f = getattr(L, name)
            f.restype = I
            f.argtypes = [P, I, I, ctypes.c_int64, I, P, P, P]
        L.rf_cg_work_bytes.restype = S
        L.rf_cg_work_bytes.argtypes = []
        L64 = ctypes.c_int64
        L.rf_dot.restype = I
        L.rf_dot.argtypes = [I, L64, P, P, P, P, I, P]
        L.rf_dot_noalloc_scratch_bytes.restype = S
        L.rf_dot_noalloc_scratch_bytes.argtypes = []
        L.rf_dot_noalloc.restype = I
        L.rf_dot_noalloc.argtypes = [I, L64, P, P, P, I, P]
        L.rf_cg_q_dot.restype = I
        L.rf_cg_q_dot.argtypes = [I, L64, P, P, P, P, P, P]
        L.rf_cg_step.restype = I
        L.rf_cg_step.argtypes = [I, L64, P, P, P, P, P, P, P]
        L.rf_cg_step_pw.restype = I
        L.rf_cg_step_pw.argtypes = [I, L64, P, P, P, P, P, P, P]
        L.rf_cg_dir.restype = I
        L.rf_cg_dir.argtypes = [I, L64, P, P, P, P]
        L.rf_axpy.restype = I
        L.rf_axpy.argtypes = [I, L64, ctypes.c_double, P, P, P]
        L.rf_obs_innovation.restype = I
        L.rf_obs_innovation.argtypes = [P, I, I, ctypes.c_int64, I, P, P, P, ctypes.c_double, P, P, P]
        L.rf_strerror.restype = ctypes.c_char_p
        L.rf_strerror.argtypes = [I]
        _lib = L
    return _lib


def rf_strerror(status: int) -> str:
    return lib().rf_strerror(int(status)).decode()


def _check(status, where):
    if status != RF_OK:
        raise RFError(status, where)


def _ptr(t):
    if t is None:
        return None
    if isinstance(t, int):
        return t
    return t.data_ptr()


def _stream(stream):
    if stream is None:
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def make_grid(nx, ny, nlev, mask_nlev=1, sigma_nlev=1, n_img=0, qmode=RF_Q_LITERAL, k1=5, flags=0) -> rf_grid:
    if isinstance(qmode, str):
        qmode = QMODES[qmode]
    return rf_grid(nx, ny, nlev, mask_nlev, sigma_nlev, n_img, qmode, k1, flags)


def rf_coeffs_bytes(g: rf_grid) -> int:
    return lib().rf_coeffs_bytes(ctypes.byref(g))


def rf_coeffs(g, mask, sigma_x, sigma_y, coef, stream=None):
    _check(lib().rf_coeffs(ctypes.byref(g), _ptr(mask), _ptr(sigma_x), _ptr(sigma_y), _ptr(coef),
                           _stream(stream)), "rf_coeffs")


def rf3_apply_xy(g, coef, prec, inp, out, nlev, nfields, stream=None):
    _check(lib().rf3_apply_xy(ctypes.byref(g), _ptr(coef), int(prec), _ptr(inp), _ptr(out), int(nlev),
                              int(nfields), _stream(stream)), "rf3_apply_xy")


def rf3_adjoint_xy(g, coef, prec, inp, out, nlev, nfields, stream=None):
    _check(lib().rf3_adjoint_xy(ctypes.byref(g), _ptr(coef), int(prec), _ptr(inp), _ptr(out), int(nlev),
                                int(nfields), _stream(stream)), "rf3_adjoint_xy")


def rf3_apply_dir(g, coef, prec, direction, adjoint, inp, out, nlev, nfields, stream=None):
    _check(lib().rf3_apply_dir(ctypes.byref(g), _ptr(coef), int(prec), int(direction), int(adjoint), _ptr(inp),
                               _ptr(out), int(nlev), int(nfields), _stream(stream)), "rf3_apply_dir")


def rf1_apply_xy(g, coef, prec, K, inp, out, nlev, nfields, stream=None):
    _check(lib().rf1_apply_xy(ctypes.byref(g), _ptr(coef), int(prec), int(K), _ptr(inp), _ptr(out),
                              int(nlev), int(nfields), _stream(stream)), "rf1_apply_xy")


def rf1_apply_xy_fused(g, coef, prec, K, inp, out, nlev, nfields, stream=None):
    _check(lib().rf1_apply_xy_fused(ctypes.byref(g), _ptr(coef), int(prec), int(K), _ptr(inp), _ptr(out),
                                    int(nlev), int(nfields), _stream(stream)), "rf1_apply_xy_fused")


def _items(items):
    arr = (rf_batch_item * len(items))()
    keep = []
    for k, (g, coef, inp, out, nf) in enumerate(items):
        keep.append(g)
        arr[k] = rf_batch_item(ctypes.pointer(g), _ptr(coef), _ptr(inp), _ptr(out), int(nf))
    return arr, keep


def _tuning(tuning):
    """None (defaults), an rf_batch_tuning, or (x_groups_max, y_planes[, x_one_launch])."""
    if tuning is None or isinstance(tuning, rf_batch_tuning):
        return tuning
    xg, yp, *rest = tuning
    return rf_batch_tuning(int(xg), int(yp), int(rest[0]) if rest else 0)


def _tptr(t):
    return ctypes.byref(t) if t is not None else None


def rf3_batch_plan_bytes(items, tuning=None) -> int:
    arr, _keep = _items(items)
    t = _tuning(tuning)
    if t is None:
        return lib().rf3_batch_plan_bytes(arr, len(items))
    return lib().rf3_batch_plan_bytes_ex(arr, len(items), _tptr(t))


def rf3_batch_plan(items, tuning=None) -> bytes:
    """Host work list for `items` [(grid, coef, in, out, nfields), ...]; copy it to the device yourself."""
    arr, _keep = _items(items)
    t = _tuning(tuning)
    nb = lib().rf3_batch_plan_bytes_ex(arr, len(items), _tptr(t))
    if nb == 0:
        raise RFError(RF_E_ARG, "rf3_batch_plan_bytes")
    buf = ctypes.create_string_buffer(nb)
    if t is None:
        _check(lib().rf3_batch_plan(arr, len(items), buf, nb), "rf3_batch_plan")
    else:
        _check(lib().rf3_batch_plan_ex(arr, len(items), _tptr(t), buf, nb), "rf3_batch_plan_ex")
    return buf.raw


def rf3_apply_batch(items, prec, adjoint, plan_dev, plan_bytes, stream=None, tuning=None):
    arr, _keep = _items(items)
    t = _tuning(tuning)
    if t is None:
        _check(lib().rf3_apply_batch(arr, len(items), int(prec), int(adjoint), _ptr(plan_dev), int(plan_bytes),
                                     _stream(stream)), "rf3_apply_batch")
    else:
        _check(lib().rf3_apply_batch_ex(arr, len(items), _tptr(t), int(prec), int(adjoint), _ptr(plan_dev),
                                        int(plan_bytes), _stream(stream)), "rf3_apply_batch_ex")


def rf_obs_plan(g, lev, x, y):
    """Host gather tables of the bilinear observation operator: (plan bytes, nuniq)."""
    import numpy as np
    lev = np.ascontiguousarray(lev, dtype=np.int32)
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.ascontiguousarray(y, dtype=np.float64)
    n = len(lev)
    if len(x) != n or len(y) != n:
        raise ValueError("lev, x, y must have the same length")
    IP = ctypes.POINTER(ctypes.c_int32)
    D = ctypes.POINTER(ctypes.c_double)
    nu = ctypes.c_int32(0)
    args = (ctypes.byref(g), n, lev.ctypes.data_as(IP), x.ctypes.data_as(D), y.ctypes.data_as(D))
    nb = lib().rf_obs_plan_bytes(*args, ctypes.byref(nu))
    if nb == 0:
        raise RFError(RF_E_ARG, "rf_obs_plan_bytes")
    buf = ctypes.create_string_buffer(nb)
    _check(lib().rf_obs_plan(*args, buf, nb), "rf_obs_plan")
    return buf.raw, nu.value


def rf_obs_apply(plan_dev, nobs, nuniq, npts, prec, field, obs, stream=None):
    _check(lib().rf_obs_apply(_ptr(plan_dev), int(nobs), int(nuniq), int(npts), int(prec), _ptr(field), _ptr(obs),
                              _stream(stream)), "rf_obs_apply")


def rf_obs_adjoint(plan_dev, nobs, nuniq, npts, prec, obs, field, stream=None):
    _check(lib().rf_obs_adjoint(_ptr(plan_dev), int(nobs), int(nuniq), int(npts), int(prec), _ptr(obs), _ptr(field),
                                _stream(stream)), "rf_obs_adjoint")


def rf_obs_innovation(plan_dev, nobs, nuniq, npts, prec, field, yobs, rinv, scale, d, rd, stream=None):
    _check(lib().rf_obs_innovation(_ptr(plan_dev), int(nobs), int(nuniq), int(npts), int(prec), _ptr(field),
                                   _ptr(yobs), _ptr(rinv), float(scale), _ptr(d), _ptr(rd), _stream(stream)),
           "rf_obs_innovation")


def rf_cg_work_bytes() -> int:
    return lib().rf_cg_work_bytes()


def rf_dot_noalloc_scratch_bytes() -> int:
    return lib().rf_dot_noalloc_scratch_bytes()


def rf_dot_noalloc(prec, n, a, b, s, slot, stream=None):
    _check(lib().rf_dot_noalloc(int(prec), int(n), _ptr(a), _ptr(b), _ptr(s), int(slot), _stream(stream)),
           "rf_dot_noalloc")


def rf_dot(prec, n, a, b, work, s, slot, stream=None):
    _check(lib().rf_dot(int(prec), int(n), _ptr(a), _ptr(b), _ptr(work), _ptr(s), int(slot), _stream(stream)),
           "rf_dot")


def rf_cg_q_dot(prec, n, p, w, q, work, s, stream=None):
    _check(lib().rf_cg_q_dot(int(prec), int(n), _ptr(p), _ptr(w), _ptr(q), _ptr(work), _ptr(s), _stream(stream)),
           "rf_cg_q_dot")


def rf_cg_step(prec, n, p, q, v, r, work, s, stream=None):
    _check(lib().rf_cg_step(int(prec), int(n), _ptr(p), _ptr(q), _ptr(v), _ptr(r), _ptr(work), _ptr(s),
                            _stream(stream)), "rf_cg_step")


def rf_cg_step_pw(prec, n, p, w, v, r, work, s, stream=None):
    _check(lib().rf_cg_step_pw(int(prec), int(n), _ptr(p), _ptr(w), _ptr(v), _ptr(r), _ptr(work), _ptr(s),
                               _stream(stream)), "rf_cg_step_pw")


def rf_cg_dir(prec, n, r, p, s, stream=None):
    _check(lib().rf_cg_dir(int(prec), int(n), _ptr(r), _ptr(p), _ptr(s), _stream(stream)), "rf_cg_dir")


def rf_axpy(prec, n, a, x, y, stream=None):
    _check(lib().rf_axpy(int(prec), int(n), float(a), _ptr(x), _ptr(y), _stream(stream)), "rf_axpy")

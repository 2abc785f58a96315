"""FP64 CPU oracle for the 3rd-RF / 1st-RF horizontal covariance operator.

TEST INFRASTRUCTURE ONLY: used by ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py``.  The product path never imports it.

The arithmetic lives in ``rf_oracle.c`` (plain C, double precision, written from
the paper: Theorem 3.1 and eqs. "fort"/"bact" of Sec. 3.1, the 1st-RF of eqs.
"proc1-1"/"proc1-2" with the Hayden relation, V_H = G_y G_x of Sec. 2.2).  This
module only compiles it with gcc and marshals numpy arrays through ctypes.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "rf_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

LITERAL, VARMATCH, FIT = 0, 1, 2
QMODES = {"literal": LITERAL, "varmatch": VARMATCH, "fit": FIT}
PERIODIC_X, EXACT_ENDS = 1, 2   # grid flags: zonally periodic rows, exact end conditions of the 3rd-RF


def build(force: bool = False) -> str:
    """Compile rf_oracle.c into liboracle.so with gcc (OpenMP over lines)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-fopenmp", "-std=c99",
                               "-D_GNU_SOURCE", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Grid(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int) for n in
                ("nx", "ny", "nlev", "mask_nlev", "sigma_nlev", "n_img", "qmode", "k1", "flags")]


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = ctypes.CDLL(build())
        d, i, p = ctypes.c_double, ctypes.c_int, ctypes.c_void_p
        _lib.orc_qmap.restype = d
        _lib.orc_qmap.argtypes = [i, d]
        _lib.orc_pair_var_coef.restype = d
        _lib.orc_pair_var_coef.argtypes = [i]
        _lib.orc_coef3.argtypes = [i, d, p, p, p, p]
        _lib.orc_coef1.argtypes = [i, d, p, p]
        _lib.orc_segments.restype = i
        _lib.orc_segments.argtypes = [p, ctypes.c_long, i, i, p, p, p, p]
        _lib.orc_segments_cyclic.restype = i
        _lib.orc_segments_cyclic.argtypes = [p, ctypes.c_long, i, i, p, p, p, p, p]
        for name in ("orc_rf3_apply", "orc_rf3_adjoint"):
            getattr(_lib, name).argtypes = [ctypes.POINTER(_Grid), p, p, p, p, p, i, i, i]
        _lib.orc_rf1_apply.argtypes = [ctypes.POINTER(_Grid), p, p, p, i, p, p, i, i, i]
        _lib.orc_apply_dir.argtypes = [ctypes.POINTER(_Grid), i, i, i, p, p, p, i, i]
        _lib.orc_num_threads.restype = i
    return _lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def qmap(mode: int, sigma: float) -> float:
    return lib().orc_qmap(int(mode), float(sigma))


def pair_var_coefs():
    """(B, A) with var(fwd+bwd impulse response) = A q^2 + B q on an infinite line."""
    L = lib()
    return L.orc_pair_var_coef(0), L.orc_pair_var_coef(1)


def coef3(sigma, mode=LITERAL):
    """Per-point 3rd-RF coefficients (alpha1, alpha2, alpha3, beta) for an array of sigma."""
    s = np.asarray(sigma, dtype=np.float64).ravel()
    out = np.zeros((4, s.size))
    a = [ctypes.c_double() for _ in range(4)]
    for k, v in enumerate(s):
        lib().orc_coef3(int(mode), float(v), *[ctypes.byref(x) for x in a])
        out[:, k] = [x.value for x in a]
    return out.reshape((4,) + np.shape(sigma))


def coef1(sigma, K):
    s = np.asarray(sigma, dtype=np.float64).ravel()
    out = np.zeros((2, s.size))
    a, b = ctypes.c_double(), ctypes.c_double()
    for k, v in enumerate(s):
        lib().orc_coef1(int(K), float(v), ctypes.byref(a), ctypes.byref(b))
        out[:, k] = [a.value, b.value]
    return out.reshape((2,) + np.shape(sigma))


def segments(mask_line, n_img):
    """Return (seg, kind, [(start, end), ...]) for one line (kind: 0 land, 1 sea, 2 imaginary)."""
    m = np.ascontiguousarray(mask_line, dtype=np.uint8)
    n = m.size
    seg = np.zeros(n, np.int32)
    kind = np.zeros(n, np.uint8)
    st = np.zeros(max(n, 1), np.int32)
    en = np.zeros(max(n, 1), np.int32)
    nseg = lib().orc_segments(_ptr(m), 1, n, int(n_img), _ptr(seg), _ptr(kind), _ptr(st), _ptr(en))
    return seg, kind, list(zip(st[:nseg].tolist(), en[:nseg].tolist()))


def segments_cyclic(mask_line, n_img):
    """Segments of a periodic line: (seg, kind, [(start, end), ...], whole); a segment may wrap
    (start > end); whole is True for a line with no land (one cyclic line, no segments)."""
    m = np.ascontiguousarray(mask_line, dtype=np.uint8)
    n = m.size
    seg = np.zeros(n, np.int32)
    kind = np.zeros(n, np.uint8)
    st = np.zeros(max(n, 1), np.int32)
    en = np.zeros(max(n, 1), np.int32)
    whole = ctypes.c_int(0)
    nseg = lib().orc_segments_cyclic(_ptr(m), 1, n, int(n_img), _ptr(seg), _ptr(kind), _ptr(st), _ptr(en),
                                     ctypes.byref(whole))
    return seg, kind, list(zip(st[:nseg].tolist(), en[:nseg].tolist())), bool(whole.value)


class Problem:
    """Grid description + mask + sigma fields, the arguments the paper states the problem with.
    flags: PERIODIC_X (zonally periodic rows) and/or EXACT_ENDS (exact end conditions of the
    3rd-RF's anti-causal sweep)."""

    def __init__(self, mask, sigma_x, sigma_y, n_img=0, qmode=LITERAL, k1=5, flags=0):
        mask = np.asarray(mask)
        if mask.ndim == 2:
            mask = mask[None]
        sx = np.asarray(sigma_x, dtype=np.float64)
        sy = np.asarray(sigma_y, dtype=np.float64)
        if sx.ndim == 2:
            sx = sx[None]
        if sy.ndim == 2:
            sy = sy[None]
        self.mask = np.ascontiguousarray(mask != 0, dtype=np.uint8)
        self.sx = np.ascontiguousarray(sx)
        self.sy = np.ascontiguousarray(sy)
        self.ny, self.nx = self.mask.shape[1:]
        assert self.sx.shape[1:] == (self.ny, self.nx) and self.sy.shape == self.sx.shape
        self.n_img, self.qmode, self.k1, self.flags = int(n_img), int(qmode), int(k1), int(flags)

    def grid(self, nlev):
        ml, sl = self.mask.shape[0], self.sx.shape[0]
        assert ml in (1, nlev) and sl in (1, nlev), "mask/sigma level count must be 1 or nlev"
        return _Grid(self.nx, self.ny, nlev, ml, sl, self.n_img, self.qmode, self.k1, self.flags)

    def _prep(self, field):
        f = np.ascontiguousarray(field, dtype=np.float64)
        if f.ndim == 2:
            f = f[None, None]
        elif f.ndim == 3:
            f = f[None]
        assert f.ndim == 4 and f.shape[2:] == (self.ny, self.nx)
        return f

    def _run(self, name, field, threads, *extra):
        f = self._prep(field)
        out = np.empty_like(f)
        nf, nlev = f.shape[:2]
        g = self.grid(nlev)
        fn = getattr(lib(), name)
        if extra:
            fn(ctypes.byref(g), _ptr(self.mask), _ptr(self.sx), _ptr(self.sy), *extra,
               _ptr(f), _ptr(out), nlev, nf, int(threads))
        else:
            fn(ctypes.byref(g), _ptr(self.mask), _ptr(self.sx), _ptr(self.sy),
               _ptr(f), _ptr(out), nlev, nf, int(threads))
        return out.reshape(np.shape(field))

    def rf3(self, field, threads=0):
        """V_H field = G_y G_x field (FP64)."""
        return self._run("orc_rf3_apply", field, threads)

    def rf3_adjoint(self, field, threads=0):
        """V_H^T field = G_x^T G_y^T field (FP64)."""
        return self._run("orc_rf3_adjoint", field, threads)

    def rf1(self, field, K=None, threads=0):
        """1st-RF with K iterations per direction (K along x, then K along y)."""
        K = self.k1 if K is None else int(K)
        return self._run("orc_rf1_apply", field, threads, ctypes.c_int(K))

    def apply_dir(self, field, direction, op="rf3", K=None, threads=0):
        """One direction only: direction 'x' or 'y'; op 'rf3', 'rf3_adj' or 'rf1'."""
        f = self._prep(field).copy()
        nf, nlev = f.shape[:2]
        g = self.grid(nlev)
        opi = {"rf3": 0, "rf3_adj": 1, "rf1": 2}[op]
        d = {"x": 0, "y": 1}[direction]
        sig = self.sx if d == 0 else self.sy
        for k in range(nf):
            sub = np.ascontiguousarray(f[k])
            lib().orc_apply_dir(ctypes.byref(g), d, opi, int(K or self.k1), _ptr(self.mask),
                                _ptr(sig), _ptr(sub), nlev, int(threads))
            f[k] = sub
        return f.reshape(np.shape(field))


def num_threads() -> int:
    return lib().orc_num_threads()

"""FP64 reference of the 3D-VAR harness pieces (TEST INFRASTRUCTURE ONLY).

Used by ``tests/`` only.  Written from Sec. 2.1 (the quadratic cost in the
increment, eq. "functional2", and its preconditioned system, eq. "eight", with
B = V V^T), in the control variable v (increment = V v): the bilinear observation
operator H, its transpose, the cost J(v) = v.v/2 + (HVv - y).R^-1.(HVv - y)/2 and its
gradient v + V^T H^T R^-1 (HVv - y), and a textbook conjugate-gradient solve of
(I + V^T H^T R^-1 H V) v = V^T H^T R^-1 y.  Plain loops and numpy only.
"""
from __future__ import annotations

import numpy as np


def obs_weights(nx, ny, lev, x, y):
    """Flat point indices [nobs][4] and bilinear weights [nobs][4] of each observation.

    Corners (i, j), (i+1, j), (i, j+1), (i+1, j+1) of the cell holding (x, y),
    weights (1-fx)(1-fy), fx(1-fy), (1-fx)fy, fx fy; a point on the last row or
    column uses the cell before it.
    """
    n = len(lev)
    idx = np.zeros((n, 4), np.int64)
    w = np.zeros((n, 4), np.float64)
    for o in range(n):
        i = min(int(np.floor(x[o])), max(nx - 2, 0))
        j = min(int(np.floor(y[o])), max(ny - 2, 0))
        i1, j1 = min(i + 1, nx - 1), min(j + 1, ny - 1)
        fx = x[o] - i if nx > 1 else 0.0
        fy = y[o] - j if ny > 1 else 0.0
        base = int(lev[o]) * nx * ny
        idx[o] = (base + j * nx + i, base + j * nx + i1, base + j1 * nx + i, base + j1 * nx + i1)
        w[o] = ((1 - fx) * (1 - fy), fx * (1 - fy), (1 - fx) * fy, fx * fy)
    return idx, w


def obs_apply(field, idx, w):
    """H f: interpolated values at the observations."""
    f = np.asarray(field, np.float64).ravel()
    out = np.zeros(len(idx))
    for o in range(len(idx)):
        s = 0.0
        for c in range(4):
            s += w[o, c] * f[idx[o, c]]
        out[o] = s
    return out


def obs_adjoint(obs, idx, w, npts):
    """H^T d: each observation's value spread back with its weights."""
    f = np.zeros(npts)
    for o in range(len(idx)):
        for c in range(4):
            f[idx[o, c]] += w[o, c] * obs[o]
    return f


def cost(v, V, Vt, idx, w, yobs, rinv):
    """J(v) and its gradient; V, Vt map a flat control vector to the field and back."""
    d = obs_apply(V(v), idx, w) - yobs
    J = 0.5 * float(v @ v) + 0.5 * float(d @ (rinv * d))
    g = v + Vt(obs_adjoint(rinv * d, idx, w, len(v)))
    return J, g


def cg(V, Vt, idx, w, yobs, rinv, n, iters):
    """Conjugate gradients on (I + V^T H^T R^-1 H V) v = V^T H^T R^-1 y from v = 0; the iterates."""
    def A(p):
        return p + Vt(obs_adjoint(rinv * obs_apply(V(p), idx, w), idx, w, n))
    v = np.zeros(n)
    r = Vt(obs_adjoint(rinv * yobs, idx, w, n))
    p = r.copy()
    rr = float(r @ r)
    out = [v.copy()]
    for _ in range(iters):
        q = A(p)
        a = rr / float(p @ q)
        v = v + a * p
        r = r - a * q
        rr_new = float(r @ r)
        p = r + (rr_new / rr) * p
        rr = rr_new
        out.append(v.copy())
    return out

"""Per-line parity of a GPU output against the FP64 oracle.

A field-wide relative L2 hides a single bad line (one 1440-point row wrong by
1e-3 moves the C3 field norm by ~5e-6).  The FP32 tiled kernels work line by
line (x rows, then y columns, cut into chunks joined by a carry scan), so a
slip in their coast, chunk-carry or guard-row logic shows up as one line with a
large error.  line_check compares every x-row and every y-column of every plane:

    ||gpu - ref||_2 (line) <= TOL_LINE * ||ref||_2 (line) + FLOOR * sqrt(n) * rms(ref over the plane)

TOL_LINE = 1e-5 is the FP32 target applied per line (measured per-line errors
are ~1e-6 and below); the absolute floor (1e-6 of the plane's rms per point)
keeps lines whose reference is nearly zero (mostly land, or cancellation) from
failing on rounding of their neighbours' magnitude.
"""
import numpy as np

TOL_LINE = 1e-5
FLOOR = 1e-6


def line_errors(gpu, ref, tol_line=TOL_LINE):
    """Worst per-line ratio err / allowed over x-rows and y-columns, and where it is."""
    g = np.asarray(gpu, np.float64)
    r = np.asarray(ref, np.float64)
    if g.ndim == 2:
        g, r = g[None], r[None]
    g = g.reshape((-1,) + g.shape[-2:])
    r = r.reshape((-1,) + r.shape[-2:])
    d = g - r
    ny, nx = r.shape[-2:]
    rms = np.sqrt(np.mean(r * r, axis=(1, 2)))[:, None]            # per plane
    worst = (0.0, None)
    for axis, n, name in ((2, nx, "row"), (1, ny, "col")):
        err = np.linalg.norm(d, axis=axis)
        allowed = tol_line * np.linalg.norm(r, axis=axis) + FLOOR * np.sqrt(n) * rms
        allowed = np.maximum(allowed, 1e-300)
        ratio = err / allowed
        k = np.unravel_index(np.argmax(ratio), ratio.shape)
        if ratio[k] > worst[0]:
            worst = (float(ratio[k]), (name, int(k[0]), int(k[1])))
    return worst


def assert_lines(gpu, ref, what="", tol_line=TOL_LINE):
    ratio, where = line_errors(gpu, ref, tol_line)
    assert ratio <= 1.0, f"{what}: line {where} error {ratio:.3g}x its allowance"
    return ratio

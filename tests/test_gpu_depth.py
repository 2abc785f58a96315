"""GPU parity of depth-dependent masks and length scales on the tiled FP32 kernels.

The paper's global configuration (Sec. 5) has land that grows with depth and
length scales that depend on depth: every level then has its own coefficients,
lane masks and scan tables.  Each case runs the tiled kernels (per-level tables)
and the line-sequential ones (RF3_SEQUENTIAL=1) against the FP64 oracle,
field-wide (relative L2 1e-5) and line by line, and against each other line by
line; forward and adjoint, several fields, tile sizes x 23 / y 45, x 33 / y 56 and
x 1 / y 1, mask-only and sigma-only depth dependence, a call on fewer levels
than the grid holds (it takes the first levels' tables), and exact ends with
two fields.
"""
import numpy as np
import pytest
import torch

from paper_1404_5756_amd import synth
from paper_1404_5756_amd.operator import HorizontalCovariance
from parity_util import assert_lines

pytestmark = pytest.mark.gpu
TOL32 = 1e-5


def rel(a, b):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


LCASES = [
    # seed, ny, nx, nlev, nfields, 3-D mask, 3-D sigma
    (61, 720, 1440, 3, 2, True, True),
    (62, 801, 2112, 2, 1, True, True),
    (63, 14, 50, 3, 3, True, False),
    (64, 97, 131, 4, 2, False, True),
]


def _problem(orc, w, nlev):
    m = w.mask[:nlev] if w.mask.shape[0] > 1 else w.mask
    sx = w.sigma_x[:nlev] if w.sigma_x.shape[0] > 1 else w.sigma_x
    sy = w.sigma_y[:nlev] if w.sigma_y.shape[0] > 1 else w.sigma_y
    return orc.Problem(m, sx, sy, n_img=w.n_img, qmode=orc.QMODES[w.qmode], k1=5)


@pytest.mark.parametrize("c", LCASES, ids=lambda c: f"depth_s{c[0]}_{c[2]}x{c[1]}x{c[3]}_f{c[4]}")
def test_depth_tables(c, orc, monkeypatch):
    seed, ny, nx, nlev, nf, m3, s3 = c
    w = synth.random_case(seed, ny, nx, nlev, 0.3, 4, (1.5, 12.0), 3.0, "fit", m3, s3)
    print(f"depth case {w.name} nfields={nf} mask_3d={m3} sigma_3d={s3}", flush=True)
    op = HorizontalCovariance(w.mask, w.sigma_x, w.sigma_y, nlev, n_img=w.n_img, qmode=w.qmode, k1=5)
    x = w.field(np.float32, nfields=nf)
    for nl in (nlev, nlev - 1):
        P = _problem(orc, w, nl)
        xs = np.ascontiguousarray(x[:, :nl])
        for name, fn, ref in (("forward", op.apply, P.rf3), ("adjoint", op.adjoint, P.rf3_adjoint)):
            r = ref(xs.astype(np.float64), threads=16)
            monkeypatch.delenv("RF3_SEQUENTIAL", raising=False)
            got = fn(torch.from_numpy(xs).cuda()).cpu().numpy()
            monkeypatch.setenv("RF3_SEQUENTIAL", "1")
            seq = fn(torch.from_numpy(xs).cuda()).cpu().numpy()
            monkeypatch.delenv("RF3_SEQUENTIAL")
            e, es = rel(got, r), rel(seq, r)
            lr = assert_lines(got, r, f"{w.name} levels {nl} tiled {name}")
            ls = assert_lines(seq, r, f"{w.name} levels {nl} sequential {name}")
            lt = assert_lines(got, seq, f"{w.name} levels {nl} tiled vs sequential {name}")
            print(f"  levels {nl} {name}: rel {e:.2e} (sequential {es:.2e}); worst line {lr:.3f} / {ls:.3f} "
                  f"(tiled vs sequential {lt:.3f}) of allowance", flush=True)
            assert e <= TOL32 and es <= TOL32


# exact ends with depth-dependent tables: the end maps per level, and (two fields) the y units
# that pair the fields of a level exchange the end corrections of both planes; per-line bound
# of the exact-end FP32 paths
TOL_LINE_END = 3e-5
ECASES = [
    # seed, ny, nx, nlev, nfields, 3-D mask, 3-D sigma
    (65, 120, 700, 3, 2, True, True),
    (66, 720, 1440, 2, 2, True, False),
]


@pytest.mark.parametrize("c", ECASES, ids=lambda c: f"depth_end_s{c[0]}_{c[2]}x{c[1]}x{c[3]}_f{c[4]}")
def test_depth_tables_exact_ends(c, orc, monkeypatch):
    seed, ny, nx, nlev, nf, m3, s3 = c
    w = synth.random_case(seed, ny, nx, nlev, 0.3, 4, (1.5, 12.0), 3.0, "fit", m3, s3)
    print(f"depth exact-ends case {w.name} nfields={nf}", flush=True)
    op = HorizontalCovariance(w.mask, w.sigma_x, w.sigma_y, nlev, n_img=w.n_img, qmode=w.qmode, k1=5,
                              exact_ends=True)
    P = orc.Problem(w.mask, w.sigma_x, w.sigma_y, n_img=w.n_img, qmode=orc.QMODES[w.qmode], k1=5,
                    flags=orc.EXACT_ENDS)
    x = w.field(np.float32, nfields=nf)
    for name, fn, ref in (("forward", op.apply, P.rf3), ("adjoint", op.adjoint, P.rf3_adjoint)):
        r = ref(x.astype(np.float64), threads=16)
        monkeypatch.delenv("RF3_SEQUENTIAL", raising=False)
        got = fn(torch.from_numpy(x).cuda()).cpu().numpy()
        monkeypatch.setenv("RF3_SEQUENTIAL", "1")
        seq = fn(torch.from_numpy(x).cuda()).cpu().numpy()
        monkeypatch.delenv("RF3_SEQUENTIAL")
        e = rel(got, r)
        lr = assert_lines(got, r, f"{w.name} exact ends tiled {name}", TOL_LINE_END)
        lt = assert_lines(got, seq, f"{w.name} exact ends tiled vs sequential {name}", TOL_LINE_END)
        print(f"  {name}: rel {e:.2e}; worst line {lr:.3f} (tiled vs sequential {lt:.3f}) of allowance", flush=True)
        assert e <= TOL32

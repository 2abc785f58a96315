"""Batched application (rf3_apply_batch) on the GPU.

Items of different shapes, one with a per-level mask (line-sequential path),
one in place, one with two fields.  The batch must give exactly the per-item
result of rf3_apply_xy / rf3_adjoint_xy (same kernels, same arithmetic) and
match the FP64 oracle; a hipGraph capture of the batch is replayed several
times with eager work in between and every replay is checked.
"""
import numpy as np
import pytest
import torch

from paper_1404_5756_amd import synth
from paper_1404_5756_amd.operator import Batch, HorizontalCovariance

pytestmark = pytest.mark.gpu

# seed, ny, nx, nlev, nfields, mask_3d, in_place
ITEMS = [
    (21, 131, 257, 5, 1, False, False),
    (22, 801, 70, 3, 1, False, True),
    (23, 40, 1100, 1, 2, False, False),
    (24, 60, 90, 3, 1, True, False),
    (25, 200, 333, 7, 1, False, False),
    (26, 24, 1900, 2, 1, False, False),   # x tile 31: the batch's fourth x occupancy class
]


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.fixture(scope="module")
def batch_setup(orc):
    dev = torch.device("cuda:0")
    ws, ops, xs = [], [], []
    for seed, ny, nx, nlev, nf, m3, _ip in ITEMS:
        w = synth.random_case(seed, ny, nx, nlev, 0.3, 4, (1.5, 10.0), 3.0, "fit", m3, False)
        op = HorizontalCovariance(w.mask, w.sigma_x, w.sigma_y, nlev, n_img=w.n_img, qmode=w.qmode, device=dev)
        x = torch.from_numpy(w.field(np.float32, nfields=nf)).to(dev)
        ws.append(w)
        ops.append(op)
        xs.append(x)
    return ws, ops, xs


def _run_batch(ops, xs, adjoint):
    outs, items = [], []
    for (seed, ny, nx, nlev, nf, m3, ip), op, x in zip(ITEMS, ops, xs):
        xi = x.clone()
        y = xi if ip else torch.empty_like(xi)
        items.append((op, xi, y))
        outs.append(y)
    b = Batch(items)
    b.apply(adjoint=adjoint)
    torch.cuda.synchronize()
    return outs


@pytest.mark.parametrize("adjoint", [False, True])
def test_batch_equals_per_item_and_oracle(batch_setup, orc, adjoint):
    ws, ops, xs = batch_setup
    outs = _run_batch(ops, xs, adjoint)
    for k, (w, op, x, y) in enumerate(zip(ws, ops, xs, outs)):
        ref_gpu = op.adjoint(x) if adjoint else op.apply(x)
        torch.cuda.synchronize()
        assert torch.equal(y, ref_gpu), f"item {k}: batch differs from the per-item call"
        P = orc.Problem(w.mask, w.sigma_x, w.sigma_y, n_img=w.n_img, qmode=orc.QMODES[w.qmode], k1=5)
        xh = x.double().cpu().numpy()
        ref = P.rf3_adjoint(xh) if adjoint else P.rf3(xh)
        assert rel(y.double().cpu().numpy(), ref) < 1e-5, f"item {k}"


def test_batch_fp64_path(batch_setup):
    from paper_1404_5756_amd import rf3
    ws, ops, xs = batch_setup
    items, outs = [], []
    for op, x in zip(ops, xs):
        x64 = x.double()
        y = torch.empty_like(x64)
        items.append((op.grid, op.coef, x64, y, x64.shape[0]))
        outs.append((op, x64, y))
    rf3.rf3_apply_batch(items, rf3.RF_FP64, 0, None, 0)
    torch.cuda.synchronize()
    for op, x64, y in outs:
        assert torch.equal(y, op.apply(x64))


def test_batch_graph_replays(batch_setup):
    ws, ops, xs = batch_setup
    dev = xs[0].device
    items, ins, outs = [], [], []
    for (seed, ny, nx, nlev, nf, m3, ip), op, x in zip(ITEMS, ops, xs):
        xi = x.clone()
        y = torch.empty_like(xi)   # out of place: replays must not read their own output
        items.append((op, xi, y))
        ins.append(xi)
        outs.append(y)
    b = Batch(items)
    b.apply()                      # warm up outside the capture
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        b.apply()
    gen = torch.Generator(device=dev).manual_seed(7)
    for rep in range(3):
        for xi in ins:             # eager work between replays: new inputs in the captured buffers
            xi.copy_(torch.randn(xi.shape, generator=gen, device=dev))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        got = [y.clone() for y in outs]
        b.apply()                  # eager result on the same inputs
        torch.cuda.synchronize()
        for k, (a, e) in enumerate(zip(got, outs)):
            assert torch.equal(a, e), f"replay {rep}, item {k}"


def _batch_items(ops, xs):
    items, outs = [], []
    for (seed, ny, nx, nlev, nf, m3, ip), op, x in zip(ITEMS, ops, xs):
        xi = x.clone()
        y = xi if ip else torch.empty_like(xi)
        items.append((op, xi, y))
        outs.append(y)
    return items, outs


@pytest.mark.parametrize("tuning", [(1, 1), (2, 3), (16, 2), (64, 64), (1, 4, 1), (8, 8, 1)])
def test_batch_tuning_is_bitwise_neutral(batch_setup, tuning):
    """Any work-list shape gives exactly the default result (same kernels per line)."""
    ws, ops, xs = batch_setup
    for adjoint in (False, True):
        ref = _run_batch(ops, xs, adjoint)
        items, outs = _batch_items(ops, xs)
        b = Batch(items, tuning=tuning)
        b.apply(adjoint=adjoint)
        torch.cuda.synchronize()
        for k, (a, e) in enumerate(zip(outs, ref)):
            assert torch.equal(a, e), f"tuning {tuning}, adjoint {adjoint}, item {k}"


def test_batch_autotune(batch_setup):
    ws, ops, xs = batch_setup
    items, outs = _batch_items(ops, xs)
    b = Batch(items)
    times = b.autotune(candidates=[(2, 2), (8, 16, 1)], reps=1)
    assert set(times) == {None, (2, 2, 0), (8, 16, 1)} and all(t > 0 for t in times.values())
    assert b.tuning == min(times, key=times.get)
    # the tuned batch still computes V_H: rerun on fresh copies of the inputs
    items2, outs2 = _batch_items(ops, xs)
    b2 = Batch(items2, tuning=b.tuning)
    b2.apply()
    torch.cuda.synchronize()
    ref = _run_batch(ops, xs, False)
    for k, (a, e) in enumerate(zip(outs2, ref)):
        assert torch.equal(a, e), f"item {k}"


def test_batch_autotune_cache(batch_setup):
    """A second batch of the same item shapes on the same device takes the cached shape
    without timing; a batch of other shapes is timed."""
    ws, ops, xs = batch_setup
    Batch._tuned.clear()
    items, _ = _batch_items(ops, xs)
    b = Batch(items)
    times = b.autotune(reps=1)
    assert times and b.signature() in Batch._tuned
    items2, _ = _batch_items(ops, xs)
    b2 = Batch(items2)
    assert b2.autotune(reps=1) == {} and b2.tuning == b.tuning
    items3, _ = _batch_items(ops[:2], xs[:2])
    b3 = Batch(items3)
    assert b3.signature() != b.signature()
    assert b3.autotune(reps=1) != {}

"""rf_dot_noalloc (the allocation-free entry point) against rf_dot, through the C ABI.

Two calls in a row on one GPU, the second on a smaller input, each checked bit
for bit against rf_dot on the same vectors (both run the same reduction in the
same order); FP32 and FP64, a 16-byte-aligned and an unaligned start.
"""
import pytest
import torch

from paper_1404_5756_amd import rf3

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


@pytest.mark.parametrize("offset", [0, 1])
@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_dot_noalloc_matches_dot(dtype, offset):
    prec = rf3.RF_FP32 if dtype == torch.float32 else rf3.RF_FP64
    assert rf3.rf_dot_noalloc_scratch_bytes() >= rf3.rf_cg_work_bytes()
    gen = torch.Generator(device=DEV).manual_seed(41 + offset)
    s = torch.zeros(rf3.RF_CG_SLOTS, dtype=torch.float64, device=DEV)
    work = torch.empty(rf3.rf_cg_work_bytes() // 8, dtype=torch.float64, device=DEV)
    for n in (3_000_017, 1_234):          # second call smaller
        a = torch.randn(n + offset, generator=gen, device=DEV, dtype=dtype)[offset:]
        b = torch.randn(n + offset, generator=gen, device=DEV, dtype=dtype)[offset:]
        print(f"rf_dot_noalloc {dtype} n={n} offset={offset}", flush=True)
        rf3.rf_dot(prec, n, a, b, work, s, 3)
        rf3.rf_dot_noalloc(prec, n, a, b, s, 4)
        torch.cuda.synchronize()
        ref = float((a.double() * b.double()).sum())
        assert float(s[4]) == float(s[3])
        assert abs(float(s[4]) - ref) <= 1e-12 * float((a.double().abs() * b.double().abs()).sum())


def test_dot_noalloc_rejects_bad_arguments():
    a = torch.ones(8, device=DEV)
    s = torch.zeros(rf3.RF_CG_SLOTS, dtype=torch.float64, device=DEV)
    with pytest.raises(rf3.RFError):
        rf3.rf_dot_noalloc(rf3.RF_FP32, 8, a, a, s, rf3.RF_CG_SLOTS)
    with pytest.raises(rf3.RFError):
        rf3.rf_dot_noalloc(rf3.RF_FP32, 0, a, a, s, 0)

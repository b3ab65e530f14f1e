"""The measurement aid behind the roofline of the sweep kernels: the
sustained FP32 VALU rates of the device (qc_valu_rate)."""
import ctypes

import pytest
import torch

pytestmark = pytest.mark.gpu


def _qs():
    import paper_2205_15000_amd as qs
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return qs


def test_valu_rate_probe():
    """Positive rates, transcendentals no faster than fma, and an invalid
    operation rejected before any launch."""
    qs = _qs()
    r = {op: qs.valu_rate(op) for op in ("fma", "rsq", "sqrt", "rcp")}
    print("valu rates (lane ops/s):", r, flush=True)
    assert all(v > 1e12 for v in r.values()), r
    assert all(r[op] <= 1.05 * r["fma"] for op in ("rsq", "sqrt", "rcp")), r
    v = ctypes.c_double()
    assert qs.lib.qc_valu_rate(0, 7, ctypes.byref(v)) == -1

"""The allocation-free sweep entry point (qc_sweep_static) against qc_sweep,
through the C-ABI: two calls in a row on two grains, the second smaller,
sharing the library's per-device scratch array."""
import ctypes
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2205_15000_amd import workloads as wl  # noqa: E402


def _qs():
    import paper_2205_15000_amd as qs
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return qs


def _note(m):
    print(m, flush=True)
    sys.stdout.flush()


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _call(qs, fn, g, d, a):
    dn = torch.empty_like(d)
    j = torch.empty((2,) + tuple(d.shape[1:]), dtype=torch.float64, device=d.device)
    od = torch.empty(tuple(d.shape[1:]), dtype=torch.float64, device=d.device)
    tot = ctypes.c_double(0.0)
    st = torch.cuda.current_stream().cuda_stream
    rc = fn(g._g, _ptr(d), _ptr(a), _ptr(dn), _ptr(j), _ptr(od), ctypes.byref(tot), ctypes.c_void_p(st))
    if rc < 0:
        raise qs.QcError(rc, qs.lib.qc_last_error().decode())
    torch.cuda.synchronize()
    return dn.cpu().numpy(), j.cpu().numpy(), od.cpu().numpy(), tot.value


def _needed(qs, g):
    need = ctypes.c_size_t(0)
    avail = ctypes.c_size_t(0)
    assert qs.lib.qc_sweep_static_bytes(g._g, ctypes.byref(need), ctypes.byref(avail)) == 0
    return need.value, avail.value


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_static_sweep_equals_sweep_on_two_grains(precision):
    qs = _qs()
    names = ["small_d110_field", "small_holed_mixed", "s_disc_32"]
    grains = {}
    for nm in names:
        sp = wl.spec(nm)
        grains[nm] = (sp, qs.Grain(sp, precision), qs.Grain(sp, precision))
    order = sorted(names, key=lambda nm: -_needed(qs, grains[nm][1])[0])
    sizes = [_needed(qs, grains[nm][1])[0] for nm in order]
    assert sizes[0] > sizes[-1] and sizes[0] <= _needed(qs, grains[order[0]][1])[1]
    for nm in order:  # largest first: each later call is smaller
        sp, ga, gb = grains[nm]
        _note("qc_sweep_static vs qc_sweep: %s %s (%d bytes of scratch)" % (nm, precision, _needed(qs, gb)[0]))
        d = torch.as_tensor(wl.initial_delta(nm, sp)).cuda()
        a = torch.as_tensor(wl.initial_A(nm, sp)).cuda()
        for rep in range(2):  # the first from bulk starts, the second through the boundary store
            ref = _call(qs, qs.lib.qc_sweep, ga, d, a)
            fn = qs.lib.qc_sweep if rep == 0 else qs.lib.qc_sweep_static
            got = _call(qs, fn, gb, d, a)
            for x, y in zip(got[:3], ref[:3]):
                scale = max(np.max(np.abs(y)), 1e-300)
                assert np.max(np.abs(x - y)) <= 1e-10 * scale
            assert abs(got[3] - ref[3]) <= 1e-10 * abs(ref[3])
        ga.close()
        gb.close()


def test_static_sweep_rejects_what_it_cannot_hold():
    qs = _qs()
    sp = wl.spec("d_disc_200")
    g = qs.Grain(sp, "fp64")
    need, avail = _needed(qs, g)
    assert need > avail
    d = torch.as_tensor(wl.initial_delta("d_disc_200", sp)).cuda()
    a = torch.as_tensor(wl.initial_A("d_disc_200", sp)).cuda()
    with pytest.raises(qs.QcError) as e:
        _call(qs, qs.lib.qc_sweep_static, g, d, a)
    assert "scratch" in str(e.value)
    g.close()
    sp = wl.spec("s_disc_32")
    g = qs.Grain(sp, "fp64")
    d = torch.as_tensor(wl.initial_delta("s_disc_32", sp)).cuda()
    a = torch.as_tensor(wl.initial_A("s_disc_32", sp)).cuda()
    with pytest.raises(qs.QcError) as e:
        _call(qs, qs.lib.qc_sweep_static, g, d, a)  # no boundary store yet
    assert "boundary store" in str(e.value)
    g.close()

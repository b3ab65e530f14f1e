"""Batched grains: one persistent sweep launch over several grains gives
the same iterates as each grain's own Picard loop; hipGraph replays give
the same as eager iterations (checked on every replay, with eager work in
between); the autotuner keeps a valid lane shape."""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2205_15000_amd import workloads as wl  # noqa: E402

NAMES = ["s_disc_32", "small_d110_field", "small_holed_mixed", "small_polygon_landau"]


def _qs():
    import paper_2205_15000_amd as qs
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return qs


def _note(m):
    print(m, flush=True)
    sys.stdout.flush()


def _fields(name):
    sp = wl.spec(name)
    return sp, torch.as_tensor(wl.initial_delta(name, sp)).cuda(), torch.as_tensor(wl.initial_A(name, sp)).cuda()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_batch_equals_single_grain_picard(precision):
    qs = _qs()
    _note("batch of %d grains, %s: 5 iterations eager" % (len(NAMES), precision))
    grains, refs = [], []
    for nm in NAMES:
        sp, d, a = _fields(nm)
        grains.append(qs.Grain(sp, precision))
        g1 = qs.Grain(sp, precision)
        dd, aa = d.clone(), a.clone()
        g1.scf(dd, aa, 5)
        refs.append((dd.cpu().numpy(), aa.cpu().numpy()))
        g1.close()
    b = qs.Batch(grains)
    for i, nm in enumerate(NAMES):
        _, d, a = _fields(nm)
        b.set_fields(i, d, a)
    b.iterate(5, graph=False)
    for i, nm in enumerate(NAMES):
        d, a = b.get_fields(i)
        tol = 1e-13 if precision == "fp64" else 1e-6
        assert np.max(np.abs(d.cpu().numpy() - refs[i][0])) <= tol * np.max(np.abs(refs[i][0])), nm
        assert np.max(np.abs(a.cpu().numpy() - refs[i][1])) <= tol * max(np.max(np.abs(refs[i][1])), 1e-30), nm
    b.close()
    for g in grains:
        g.close()


def test_batch_graph_replays_equal_eager():
    qs = _qs()
    _note("batch graph replays vs eager")
    res = []
    for graph in (False, True):
        grains = [qs.Grain(_fields(nm)[0], "fp64") for nm in NAMES]
        b = qs.Batch(grains)
        for i, nm in enumerate(NAMES):
            _, d, a = _fields(nm)
            b.set_fields(i, d, a)
        snaps = []
        b.iterate(1, graph=graph)               # first sweep from bulk roots (eager)
        for rep in range(3):
            b.iterate(2, graph=graph)            # one replay of the two-iteration graph
            torch.cuda.synchronize()
            x = torch.zeros(1000, device="cuda").sum()  # eager work between replays
            snaps.append([b.get_fields(i)[0].cpu().numpy() for i in range(len(NAMES))])
            del x
        res.append(snaps)
        b.close()
        for g in grains:
            g.close()
    for rep in range(3):
        for i in range(len(NAMES)):
            assert np.array_equal(res[0][rep][i], res[1][rep][i]), (rep, NAMES[i])


def test_batch_autotune():
    qs = _qs()
    _note("batch autotune")
    grains = [qs.Grain(_fields(nm)[0], "mixed") for nm in NAMES]
    b = qs.Batch(grains)
    for i, nm in enumerate(NAMES):
        _, d, a = _fields(nm)
        b.set_fields(i, d, a)
    e = b.autotune(2)
    assert e in (1, 2, 4, 8)
    assert b.info()["energies_per_lane"] == e
    ms = b.iterate(4, graph=True)
    assert ms > 0
    d, _ = b.get_fields(0)
    assert torch.isfinite(d).all()
    b.close()
    for g in grains:
        g.close()

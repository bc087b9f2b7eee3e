"""Batched stepping of many domains (continuous batching) through the C-ABI.

A domain stepped inside a batch (one launch per kernel kind for all domains,
replayed from a captured graph or launched directly) must be bit for bit the
same as the domain stepped alone; a domain that meets its stop rule freezes
at that step without disturbing the others; domains can be retired and
admitted between steps; the pool budget bounds admission.
"""
import numpy as np
import pytest

from paper_2003_01490_amd import workloads as W

from harness import gpu_domain

pytestmark = pytest.mark.gpu


def _case(msg):
    print(f"[case] {msg}", flush=True)


def _requests(seed, n):
    """Small sphere-wall requests of the serving mix (ramp, release, contact)."""
    reqs = W.serve_requests(seed, n, edge_range=(24, 48), D_range=(6.0, 8.0))
    return [W.serve_workload(r) for r in reqs]


def _make(wl, stream, **over):
    from paper_2003_01490_amd import lbmdem as L

    g = gpu_domain(wl, storage=L.STORE_F32, stream=stream, **over)
    return g


def _bits(g):
    s = g.spheres()
    out = [g.field("pdf"), g.field("flags"), g.field("owner")] + [s[k] for k in sorted(s)]
    st = g.sphere(0)
    out += [np.asarray(st[k]) for k in sorted(st)]
    return out


def _same(a, b):
    return all(np.array_equal(x, y) for x, y in zip(_bits(a), _bits(b)))


@pytest.mark.parametrize("case", ["requests", "agitated"])
def test_overlap_equals_sequential(case):
    """The DEM and the claims beside the sweep on a second stream give the
    same bits as the whole step on one stream (one-workgroup DEM kernels:
    with state in LDS up to 32 spheres, in global memory above)."""
    import torch

    from paper_2003_01490_amd import lbmdem as L

    stream = torch.cuda.Stream()
    if case == "requests":
        wls, steps = _requests(7, 3), 150
    else:
        wls, steps = [W.dense(3, n=48, count=40, D=8.0, min_gap=0.2, u_rms=0.05, nu=0.01)], 60
    _case(f"overlap vs sequential, {case}: " + ", ".join(
        f"{w.params['nx']}x{w.params['ny']}x{w.params['nz']} P={len(w.R)}" for w in wls))
    for w in wls:
        a = _make(w, stream, overlap=1)
        b = _make(w, stream, overlap=0)
        for _ in range(3):
            a.step(steps // 3)
            b.step(steps // 3)
        assert a.progress() == b.progress() == (steps // 3 * 3, False)
        assert _same(a, b), "overlapped step differs from the sequential one"
        a.close()
        b.close()


@pytest.mark.parametrize("use_graph", [True, False])
def test_batch_equals_alone(use_graph):
    import torch

    from paper_2003_01490_amd import lbmdem as L

    stream = torch.cuda.Stream()
    wls = _requests(3, 4)
    _case(f"batch of {len(wls)} domains vs alone, graph {use_graph}: "
          + ", ".join(f"{w.params['nx']}x{w.params['ny']}x{w.params['nz']}" for w in wls))
    alone = [_make(w, stream) for w in wls]
    for g in alone:
        g.step(60)
    mixed = [_make(w, stream) for w in wls]
    b = L.Batch(stream, pool_bytes=1 << 40, use_graph=use_graph)
    for g in mixed:
        b.admit(g)
    b.step(25)
    b.step(35)
    for k, (a, m) in enumerate(zip(alone, mixed)):
        assert a.progress() == (60, False) and m.progress() == (60, False)
        assert _same(a, m), f"domain {k} differs between batch and alone"
    b.close()


def test_batch_stop_retire_admit():
    import torch

    from paper_2003_01490_amd import lbmdem as L

    stream = torch.cuda.Stream()
    wls = _requests(5, 3)
    _case("stop rule, retire and admit in a running batch")
    ref = [_make(w, stream) for w in wls]
    ref[0].step(25)
    ref[1].step(70)
    ref[2].step(30)
    ds = [_make(w, stream) for w in wls]
    ds[0].set_stop_rule(L.STOP_NONE, max_steps=25)
    b = L.Batch(stream, pool_bytes=1 << 40)
    s0, s1 = b.admit(ds[0]), b.admit(ds[1])
    b.step(40)
    st = b.status()
    assert st[s0] == (25, True) and st[s1] == (40, False), st
    assert b.done() == [s0]
    b.retire(s0)
    s2 = b.admit(ds[2])
    b.step(30)
    st = b.status()
    assert st[s1] == (70, False) and st[s2] == (30, False), st
    assert _same(ref[0], ds[0]), "stopped domain differs from 25 steps alone"
    assert _same(ref[1], ds[1]), "domain kept in the batch differs"
    assert _same(ref[2], ds[2]), "domain admitted later differs"
    # the frozen domain does not move when stepped again alone
    ds[0].step(5)
    assert ds[0].progress() == (25, True)
    assert _same(ref[0], ds[0])
    b.close()


def test_batch_pool_budget():
    import torch

    from paper_2003_01490_amd import lbmdem as L

    stream = torch.cuda.Stream()
    wls = _requests(7, 3)
    ds = sorted((_make(w, stream) for w in wls), key=lambda g: -g.nbytes)  # largest first
    budget = ds[0].nbytes + ds[1].nbytes
    _case(f"pool budget {budget} bytes")
    b = L.Batch(stream, pool_bytes=budget)
    assert b.try_admit(ds[0]) is not None
    assert b.try_admit(ds[1]) is not None
    assert b.try_admit(ds[2]) is None
    with pytest.raises(L.LbmdemError):
        ds[0].step(1)  # stepped only through its batch
    b.retire(0)
    assert b.try_admit(ds[2]) is not None
    b.close()


def test_rebound_stop_rule():
    """The rule stops at the first apex after the first contact has ended;
    the step is found independently from the trajectory of the same domain
    stepped alone."""
    import torch

    from paper_2003_01490_amd import lbmdem as L

    stream = torch.cuda.Stream()
    n = (24, 24, 40)
    wl = W.Workload("rebound", W.base_params(nx=n[0], ny=n[1], nz=n[2], nu=0.02, tc=20.0, e_dry=0.97,
                                             gravity=(0, 0, -1e-4), max_spheres=1),
                    np.array([[12.3, 11.8, 1.0 + 4.0 + 0.6]]), np.array([4.0]), np.array([8.0]),
                    np.array([[0.0, 0.0, -0.06]]), np.zeros((1, 3)), 0)
    _case("rebound stop rule")
    a = _make(wl, stream)
    phase, stop_at = 0, None
    for k in range(1, 400):
        a.step(1)
        s = a.sphere(0)
        contact = bool(np.abs(s["F_col"]).max() > 0)
        uz = s["u"][2]
        if phase == 0 and contact:
            phase = 1
        elif phase == 1 and not contact:
            phase = 2
        elif phase == 2 and uz > 0:
            phase = 3
        elif phase == 3 and uz <= 0:
            stop_at = k
            break
    assert stop_at is not None, "no rebound apex in 400 steps"
    print(f"  apex after step {stop_at}", flush=True)
    g = _make(wl, stream)
    g.set_stop_rule(L.STOP_REBOUND, max_steps=0)
    b = L.Batch(stream, pool_bytes=1 << 40)
    b.admit(g)
    b.step(stop_at + 20)
    assert g.progress() == (stop_at, True)
    ref = _make(wl, stream)
    ref.step(stop_at)
    assert _same(ref, g)
    b.close()

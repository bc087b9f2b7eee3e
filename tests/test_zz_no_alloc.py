"""The allocation-free probe (lbmdem_probe_density_static) against the probe
that stages in the domain region (lbmdem_probe_density): same points, same
results bit for bit, on two calls in a row (the second smaller), and the size
limit of the static scratch.  Calls go through the C-ABI."""
import numpy as np
import pytest

from harness import gpu_domain, random_pdf
from paper_2003_01490_amd import workloads as W

pytestmark = pytest.mark.gpu


def test_static_probe_matches_region_probe():
    import torch

    from paper_2003_01490_amd import lbmdem as L

    n = (40, 36, 44)
    print(f"[case] static probe {n}", flush=True)
    wl = W.Workload("probe", W.base_params(nx=n[0], ny=n[1], nz=n[2], nu=0.02, max_spheres=2),
                    np.array([[12.3, 17.9, 20.2], [30.1, 8.4, 30.7]]), np.array([4.2, 3.6]),
                    np.array([2.0, 2.5]), np.array([[0.01, -0.005, 0.002], [0.0, 0.004, -0.003]]),
                    np.zeros((2, 3)), 0)
    g = gpu_domain(wl, storage=1)
    g.set_pdf(random_pdf(n, seed=4, u0=(0.01, 0.0, -0.005)))
    g.step(5)
    g.sync()
    rng = np.random.default_rng(9)
    for npts in (12000, 1500):  # second call smaller: no stale values may show (n <= N/4)
        xyz = np.column_stack([rng.uniform(-2, n[a] + 2, npts) for a in range(3)])
        ref = g.probe_density(xyz)
        xd = torch.from_numpy(xyz).to("cuda:0")
        out = torch.full((npts,), -7.0, dtype=torch.float64, device="cuda:0")
        g.probe_density_static(xd, out)
        g.sync()
        got = out.cpu().numpy()
        nan = np.isnan(ref)
        assert 0 < nan.sum() < npts
        assert np.array_equal(np.isnan(got), nan)
        assert np.array_equal(got[~nan], ref[~nan])
    big = torch.zeros((65537, 3), dtype=torch.float64, device="cuda:0")
    res = torch.zeros(65537, dtype=torch.float64, device="cuda:0")
    with pytest.raises(L.LbmdemError) as e:
        g.probe_density_static(big, res)
    assert e.value.code == L.EINVAL
    g.close()

"""The row-chord culling of the mapping kernels, restated on the CPU with the
same formulas and checked against brute force (host logic; no GPU).

For one x-row of a box, the kernels visit only the cells near the ends of
the x-chords of a ball around an old and a new centre: the union of the two
chords widened by 1e-3, minus the part both balls surely hold (chords
narrowed by 1e-3).  Every cell whose membership (d^2 <= r^2, computed as the
kernels' cell_d2 does) differs between the two centres must be visited, and
so must every cell inside either ball when only one centre is given."""
import numpy as np
import pytest

EPS = 1e-3


def cell_d2(i, j, k, c):
    dx, dy, dz = (i + 0.5) - c[0], (j + 0.5) - c[1], (k + 0.5) - c[2]
    return (dx * dx + dy * dy) + dz * dz


def visited(jj, kk, xo, xn, r2, lo0, ext0):
    """Box x indices the kernels visit on row (jj, kk): two segments."""
    us, ue, is_, ie = ext0, -1, 0, ext0 - 1
    for c in (xo, xn):
        dy, dz = (jj + 0.5) - c[1], (kk + 0.5) - c[2]
        rho = r2 - (dy * dy + dz * dz)
        if rho >= -EPS:
            a = np.sqrt(max(rho, 0.0)) + EPS
            us = min(us, int(np.ceil(c[0] - a - 0.5)) - lo0)
            ue = max(ue, int(np.floor(c[0] + a - 0.5)) - lo0)
        ain = np.sqrt(rho) - EPS if rho > 0.0 else -1.0
        if ain > 0.0:
            is_ = max(is_, int(np.floor(c[0] - ain - 0.5)) + 1 - lo0)
            ie = min(ie, int(np.ceil(c[0] + ain - 0.5)) - 1 - lo0)
        else:
            is_, ie = 1, 0
    s0, e0 = max(us, 0), min(ue, ext0 - 1)
    if is_ <= ie:
        return set(range(s0, min(e0, is_ - 1) + 1)) | set(range(max(s0, ie + 1), e0 + 1))
    return set(range(s0, e0 + 1))


def check(xo, xn, R, rng_extra=2):
    r2 = R * R
    lo = [int(np.floor(min(xo[a], xn[a]) - R)) - rng_extra for a in range(3)]
    hi = [int(np.floor(max(xo[a], xn[a]) + R)) + rng_extra for a in range(3)]
    ext0 = hi[0] - lo[0] + 1
    missed = 0
    for kk in range(lo[2], hi[2] + 1):
        for jj in range(lo[1], hi[1] + 1):
            v = visited(jj, kk, xo, xn, r2, lo[0], ext0)
            for g in range(ext0):
                ii = lo[0] + g
                if (cell_d2(ii, jj, kk, xo) <= r2) != (cell_d2(ii, jj, kk, xn) <= r2) and g not in v:
                    missed += 1
    return missed


def test_moves_of_random_spheres_miss_no_changed_cell():
    rng = np.random.default_rng(7)
    for _ in range(200):
        R = rng.uniform(1.0, 8.0)
        xo = rng.uniform(20.0, 21.0, 3)
        step = rng.normal(0.0, 1.0, 3) * 10.0 ** rng.uniform(-6, 0)
        assert check(xo, xo + step, R) == 0


@pytest.mark.parametrize("R", [5.0, 3.0, 13.0])
def test_exact_ties_on_the_surface_and_at_chord_ends(R):
    """Centres on cell centres with Pythagorean radii put cell centres
    exactly on the surface (d^2 == R^2 in floating point) and rows exactly
    tangent to it; tiny moves in every direction flip exactly those cells."""
    base = np.array([10.5, 10.5, 10.5])
    for d in [(1e-9, 0, 0), (0, -1e-9, 0), (0, 0, 1e-12), (3e-7, -2e-7, 1e-7), (0.25, 0, 0), (0, 0.5, -0.5)]:
        assert check(base, base + np.array(d), R) == 0
        assert check(base + np.array(d), base, R) == 0


def test_shell_radius_and_shrunk_inside():
    """The shell radius R + delta_aB (= R + 2) with a centre moving along a
    diagonal, and a radius below one cell (empty sure inside)."""
    for R in (0.6, 6.0 + 2.0):
        xo = np.array([15.3, 15.7, 15.1])
        for t in np.linspace(1e-6, 0.9, 7):
            assert check(xo, xo + t * np.array([0.577, -0.577, 0.577]), R) == 0

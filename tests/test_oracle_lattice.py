"""Pins of the oracle's lattice, moment matrix and collision operator.

Each test checks the oracle against something other than itself: the algebraic
structure the paper's moment matrix must have (App. A), the equilibrium moments
printed in App. A, the textbook BGK and TRT operators the paper says its MRT
reduces to (Sec. 2.1.2, Eqs. SRTmatrix, TRTmatrix, TRTbulkmatrix), and exact
conservation laws of the lattice Boltzmann step (Sec. 2.1).
"""
import numpy as np
import pytest

import oracle as O


def test_velocity_set_is_d3q19_and_opposites():
    c, w, opp = O.lattice()
    vecs = {tuple(v) for v in c.tolist()}
    expect = {(a, b, d) for a in (-1, 0, 1) for b in (-1, 0, 1) for d in (-1, 0, 1)
              if a * a + b * b + d * d <= 2}
    assert vecs == expect and len(c) == 19
    assert tuple(c[0]) == (0, 0, 0)
    for q in range(19):
        assert np.array_equal(c[opp[q]], -c[q])
    # App. A: rows 2-4 of M are the velocity components
    M = O.moment_matrix()
    assert np.array_equal(M[1:4].T.astype(int), c)


def test_weights_follow_from_orthogonality_of_M():
    """C1: M W M^T diagonal fixes the weight classes; solve for them here."""
    c, w, _ = O.lattice()
    M = O.moment_matrix()
    c2 = (c * c).sum(1)
    # unknowns (w0, w1, w2) for |c|^2 = 0, 1, 2: rows 0/4 and 0/5 orthogonal, sum 1
    A = np.zeros((3, 3))
    b = np.array([0.0, 0.0, 1.0])
    for cls in range(3):
        sel = c2 == cls
        A[0, cls] = (M[0, sel] * M[4, sel]).sum()
        A[1, cls] = (M[0, sel] * M[5, sel]).sum()
        A[2, cls] = sel.sum()
    wcls = np.linalg.solve(A, b)
    np.testing.assert_allclose(w, wcls[c2], rtol=0, atol=1e-16)
    np.testing.assert_allclose(wcls, [1 / 3, 1 / 18, 1 / 36], atol=1e-16)
    G = M @ np.diag(w) @ M.T
    assert np.abs(G - np.diag(np.diag(G))).max() < 1e-15
    norms = [1, 1 / 3, 1 / 3, 1 / 3, 2 / 3, 2, 2 / 3, 2 / 3, 2 / 3, 4 / 3, 4 / 9, 1 / 9, 1 / 9,
             1 / 9, 4 / 3, 4 / 9, 2 / 9, 2 / 9, 2 / 9]
    np.testing.assert_allclose(np.diag(G), norms, atol=1e-15)


def test_inverse_of_M():
    M = O.moment_matrix()
    Mi = O.moment_inverse()
    assert np.abs(M @ Mi - np.eye(19)).max() < 1e-14
    _, w, _ = O.lattice()
    N = np.diag(M @ np.diag(w) @ M.T)
    assert np.abs(Mi - np.diag(w) @ M.T @ np.diag(1 / N)).max() < 1e-15


@pytest.mark.parametrize("seed", range(5))
def test_equilibrium_moments_match_appendix(seed):
    """C2: M f^eq equals the equilibrium moments printed in App. A."""
    rng = np.random.default_rng(seed)
    rho = 1 + 0.1 * rng.standard_normal()
    u = 0.05 * rng.standard_normal(3)
    ux, uy, uz = u
    meq = np.array([rho, ux, uy, uz, ux * ux + uy * uy + uz * uz, 0, 0, 0, 0,
                    2 * ux * ux - uy * uy - uz * uz, uy * uy - uz * uz, ux * uy, uy * uz, ux * uz,
                    0, 0, 0, 0, 0])
    feq = O.equilibrium(rho, u)
    np.testing.assert_allclose(O.moment_matrix() @ feq, meq, rtol=0, atol=1e-15)


def _random_f(rng, amp=0.01):
    u = 0.05 * rng.standard_normal(3)
    return O.equilibrium(1.0 + 0.05 * rng.standard_normal(), u) + amp * rng.standard_normal(19) / 19


@pytest.mark.parametrize("coll", [O.TRT_AB, O.TRT_B, O.TRT, O.SRT])
@pytest.mark.parametrize("shell", [0, 1])
def test_collision_conserves_mass_momentum_and_fixes_equilibrium(coll, shell):
    """C3: rows 0-3 of S are zero (Eq. RelaxationRateMatrix)."""
    rng = np.random.default_rng(10 + coll)
    cfg = O.make_config(nu=0.02, collision=coll)
    c, _, _ = O.lattice()
    for _ in range(4):
        f = _random_f(rng)
        out = O.collide(cfg, f, shell)
        assert abs(out.sum() - f.sum()) < 1e-15
        np.testing.assert_allclose(out @ c, f @ c, atol=1e-16)
        feq = O.equilibrium(f.sum(), f @ c)
        np.testing.assert_allclose(O.collide(cfg, feq, shell), feq, atol=1e-16)


def test_srt_reduces_to_bgk():
    """C4: all rates equal s_nu gives f - s_nu (f - f^eq) (Eq. SRTmatrix)."""
    rng = np.random.default_rng(3)
    c, w, _ = O.lattice()
    for nu in (0.005, 0.05, 1 / 6, 0.4):
        cfg = O.make_config(nu=nu, collision=O.SRT)
        s = 1.0 / (3 * nu + 0.5)
        for _ in range(3):
            f = _random_f(rng)
            rho, u = f.sum(), f @ c
            cu = c @ u
            feq = w * (rho + 3 * cu + 4.5 * cu * cu - 1.5 * (u @ u))
            np.testing.assert_allclose(O.collide(cfg, f), f - s * (f - feq), atol=1e-16)


def _velocity_space_trt(f, c, w, opp, sp, sm):
    rho, u = f.sum(), f @ c
    cu = c @ u
    feq = w * (rho + 3 * cu + 4.5 * cu * cu - 1.5 * (u @ u))
    fp, fm = 0.5 * (f + f[opp]), 0.5 * (f - f[opp])
    ep, em = 0.5 * (feq + feq[opp]), 0.5 * (feq - feq[opp])
    return f - sp * (fp - ep) - sm * (fm - em)


def test_trt_reduces_to_ginzburg_two_relaxation_time():
    """C4: S_TRT in moment space equals the velocity-space TRT operator."""
    rng = np.random.default_rng(4)
    c, w, opp = O.lattice()
    for nu in (0.01, 0.1, 0.3):
        cfg = O.make_config(nu=nu, collision=O.TRT)
        snu = 1.0 / (3 * nu + 0.5)
        sm = 1.0 / (0.5 + (3 / 16) / (1 / snu - 0.5))  # Eq. (MagicParameter)
        for _ in range(3):
            f = _random_f(rng)
            np.testing.assert_allclose(O.collide(cfg, f), _velocity_space_trt(f, c, w, opp, snu, sm),
                                       atol=2e-16)


def test_trt_b_variants_reduce_to_trt():
    """Lambda_b = 1 is TRT (Sec. 2.1.3); TRT+aB outside the shell is TRT and
    inside it is TRT+B (Sec. 2.3.2)."""
    rng = np.random.default_rng(5)
    f = _random_f(rng)
    trt = O.collide(O.make_config(nu=0.03, collision=O.TRT), f)
    np.testing.assert_allclose(O.collide(O.make_config(nu=0.03, collision=O.TRT_B, lambda_b=1.0), f),
                               trt, atol=2e-16)
    ab = O.make_config(nu=0.03, collision=O.TRT_AB, lambda_b=100.0)
    np.testing.assert_allclose(O.collide(ab, f, 0), trt, atol=2e-16)
    np.testing.assert_allclose(O.collide(ab, f, 1),
                               O.collide(O.make_config(nu=0.03, collision=O.TRT_B), f), atol=2e-16)
    assert np.abs(O.collide(ab, f, 1) - trt).max() > 1e-8


def test_stream_direction_moves_mass_centre_by_momentum():
    """One LBM step moves the centre of mass of a localised perturbation by
    exactly the total momentum (Eq. LBM_Stream sends f_q along +c_q)."""
    n = 16
    cfg = O.make_config(nx=n, ny=n, nz=n, walls=(0, 0, 0), nu=0.05, max_spheres=1)
    d = O.RefDomain(cfg)
    c, w, _ = O.lattice()
    f = np.tile(w[:, None, None, None], (1, n, n, n)).astype(np.float64)
    rng = np.random.default_rng(7)
    f[:, 6:10, 6:10, 6:10] += 0.01 * rng.random((19, 4, 4, 4))
    d.set_pdf(f)
    rho0 = d.field("rho")
    j0 = np.einsum("qzyx,qa->a", d.field("pdf"), c.astype(float))
    d.step(1)
    rho1 = d.field("rho")
    zz, yy, xx = np.meshgrid(*(np.arange(n) + 0.5,) * 3, indexing="ij")
    for a, X in enumerate((xx, yy, zz)):
        shift = ((rho1 - rho0) * X).sum()
        assert abs(shift - j0[a]) < 1e-12, (a, shift, j0[a])

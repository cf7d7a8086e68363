"""Pins of the oracle's Dirichlet solve (GMRES and right-hand side) and of the
projected Dirichlet data.

* GMRES against numpy.linalg.solve, its finite termination on a matrix with
  three distinct eigenvalues, and the reported residual estimates against the
  true residuals of the iterates;
* the projected source datum and its normal flux against closed forms of
  their integrals over the whole lateral boundary per step (face-wise erf
  products and the divergence theorem);
* the pFMM solve against a dense direct solve (no spatial cut, high degree);
* a manufactured solution: the Neumann datum of a heat source outside the
  cube is recovered with a decreasing error under refinement.
"""
import numpy as np
import pytest
from scipy import integrate, special

from oracle.dense import dense_matrix, mass_diag, geometry, toeplitz_blocks
from oracle.fmm import FMMOracle
from oracle.solve import gmres, dirichlet_rhs
from oracle.tree import Tree
from workloads import cube_surface_mesh, uniform_time_nodes
from workloads.dirichlet import project_source_datum, project_source_flux


def _rand_matrix(n, seed):
    rng = np.random.default_rng(seed)
    return 3.0 * np.eye(n) + rng.standard_normal((n, n)) / np.sqrt(n), rng.standard_normal(n)


def test_gmres_matches_direct_solve():
    A, b = _rand_matrix(60, 0)
    x, k, hist = gmres(lambda v: A @ v, b, rtol=1e-13, max_iter=60)
    ref = np.linalg.solve(A, b)
    assert np.linalg.norm(x - ref) / np.linalg.norm(ref) < 1e-11
    assert k < 60 and hist[-1] <= 1e-13


def test_gmres_terminates_after_three_distinct_eigenvalues():
    rng = np.random.default_rng(1)
    Q, _ = np.linalg.qr(rng.standard_normal((40, 40)))
    lam = np.array([1.0, 2.0, 5.0])[rng.integers(0, 3, 40)]
    A = Q @ np.diag(lam) @ Q.T
    b = rng.standard_normal(40)
    x, k, hist = gmres(lambda v: A @ v, b, rtol=1e-12, max_iter=40)
    assert k == 3
    assert hist[2] > 1e-6
    assert np.linalg.norm(A @ x - b) / np.linalg.norm(b) < 1e-12


@pytest.mark.parametrize("k", [1, 2, 3, 5, 8])
def test_gmres_estimates_are_true_residuals(k):
    A, b = _rand_matrix(30, 2)
    x, kk, hist = gmres(lambda v: A @ v, b, rtol=0.0, max_iter=k)
    assert kk == k
    true = np.linalg.norm(b - A @ x) / np.linalg.norm(b)
    assert abs(true - hist[-1]) <= 1e-12 + 1e-10 * true
    assert all(hist[i + 1] <= hist[i] * (1 + 1e-14) for i in range(len(hist) - 1))
    # GMRES minimises the residual over the Krylov space: no other combination does better
    K = np.empty((30, k))
    v = b.copy()
    for i in range(k):
        K[:, i] = v
        v = A @ v
    c, *_ = np.linalg.lstsq(A @ K, b, rcond=None)
    assert true <= np.linalg.norm(b - A @ K @ c) / np.linalg.norm(b) * (1 + 1e-8)


def _face_integral(y, s, alpha, flux):
    """Integral over the surface of [-1,1]^3 of G(x - y, s) (flux=False) or of
    alpha dG/dn_x (flux=True; equals d/ds of the volume integral, y outside)."""
    y = np.asarray(y, dtype=np.float64)
    c = 2.0 * np.sqrt(alpha * s)
    I1 = [0.5 * (special.erf((1 - y[j]) / c) - special.erf((-1 - y[j]) / c)) for j in range(3)]
    if flux:
        # d/ds of prod_j I1_j
        dI = [(-(1 - y[j]) * np.exp(-((1 - y[j]) / c) ** 2) + (-1 - y[j]) * np.exp(-((-1 - y[j]) / c) ** 2))
              / (2.0 * c * s * np.sqrt(np.pi)) for j in range(3)]
        return dI[0] * I1[1] * I1[2] + I1[0] * dI[1] * I1[2] + I1[0] * I1[1] * dI[2]
    tot = 0.0
    g1 = lambda z: (4 * np.pi * alpha * s) ** -0.5 * np.exp(-z * z / (4 * alpha * s))
    for a in range(3):
        others = [I1[j] for j in range(3) if j != a]
        tot += (g1(1 - y[a]) + g1(-1 - y[a])) * others[0] * others[1]
    return tot


@pytest.mark.parametrize("flux", [False, True])
def test_projected_datum_integrates_to_closed_form(flux):
    v, t = cube_surface_mesh(4)
    tn = uniform_time_nodes(8, 1.0)
    ys, ts, alpha = (2.5, 0.3, -0.2), -0.1, 0.8
    fn = project_source_flux if flux else project_source_datum
    g = fn(v, t, tn, ys, ts, alpha, q=8, q_t=8).reshape(8, len(t))
    area = geometry(v, t)[0]
    h = tn[1] - tn[0]
    for j in (0, 3, 7):
        got = (g[j] * area).sum() * h
        ref = integrate.quad(lambda s: _face_integral(ys, s - ts, alpha, flux), tn[j], tn[j + 1],
                             epsabs=0, epsrel=1e-12)[0]
        assert abs(got - ref) <= 2e-4 * abs(ref), (j, got, ref)


def _problem(n, n_steps):
    v, t = cube_surface_mesh(n)
    return v, t, uniform_time_nodes(n_steps, 1.0)


def test_pfmm_gmres_against_dense_solve():
    v, t, tn = _problem(2, 8)
    h = tn[1] - tn[0]
    ys, ts = (2.5, 0.0, 0.0), -0.1
    g = project_source_datum(v, t, tn, ys, ts)
    M = mass_diag(v, t, 8, h)
    BV = toeplitz_blocks(v, t, 8, h, 1.0, "V")
    BK = toeplitz_blocks(v, t, 8, h, 1.0, "K")
    Vd = dense_matrix(v, t, 8, h, 1.0, "V", B=BV)
    Kd = dense_matrix(v, t, 8, h, 1.0, "K", B=BK)
    rhs = dirichlet_rhs(g, M, lambda x: Kd @ x)
    ref = np.linalg.solve(Vd, rhs)
    tr = Tree(v, t, tn, 1.0, n_max=16, c_st=0.9, n_tr=-1)
    oV = FMMOracle(tr, 4, 4, "V")
    oK = FMMOracle(tr, 4, 4, "K")
    oV.set_toeplitz_blocks(BV)
    oK.set_toeplitz_blocks(BK)
    rhs_f = dirichlet_rhs(g, M, oK.apply)
    rhs_err = np.linalg.norm(rhs_f - rhs) / np.linalg.norm(rhs)
    x, k, hist = gmres(oV.apply, rhs_f, rtol=1e-10, max_iter=200)
    assert hist[-1] <= 1e-10
    assert np.linalg.norm(rhs_f - oV.apply(x)) / np.linalg.norm(rhs_f) < 1e-9
    # GMRES on the dense system reproduces the direct solve
    xd, _, _ = gmres(lambda z: Vd @ z, rhs, rtol=1e-12, max_iter=400)
    assert np.linalg.norm(xd - ref) / np.linalg.norm(ref) < 1e-9
    # the pFMM solve differs from the dense one by at most the operator and
    # right-hand-side errors times the condition number (perturbation bound)
    app_err = np.linalg.norm(oV.apply(ref) - Vd @ ref) / np.linalg.norm(Vd @ ref)
    cond = np.linalg.cond(Vd)
    err = np.linalg.norm(x - ref) / np.linalg.norm(ref)
    assert err <= cond * (app_err + rhs_err) / (1 - cond * app_err), (err, cond, app_err, rhs_err)


@pytest.mark.slow
def test_manufactured_neumann_datum_converges():
    # u = G(x - y*, t) with y* outside the cube vanishes at t = 0 inside, so the
    # boundary integral equation holds without an initial term (Section 2) and
    # its solution is w = alpha du/dn.  The parabolic ratio h_t / h_x^2 is fixed.
    ys = (2.5, 0.0, 0.0)
    errs = []
    for n, et in ((2, 4), (3, 9), (4, 16)):
        v, t, tn = _problem(n, et)
        h = tn[1] - tn[0]
        g = project_source_datum(v, t, tn, ys, 0.0)
        w_ex = project_source_flux(v, t, tn, ys, 0.0)
        M = mass_diag(v, t, et, h)
        Vd = dense_matrix(v, t, et, h, 1.0, "V")
        Kd = dense_matrix(v, t, et, h, 1.0, "K")
        w = np.linalg.solve(Vd, dirichlet_rhs(g, M, lambda x: Kd @ x))
        errs.append(np.sqrt(((w - w_ex) ** 2 * M).sum() / ((w_ex ** 2) * M).sum()))
    assert errs[1] < 0.8 * errs[0] and errs[2] < 0.95 * errs[1], errs

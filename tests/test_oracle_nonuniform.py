"""Pins of the oracle on time grids whose steps differ in length (CPU only).

* The double time integral of G (and of G / (2 s)) over two steps of
  different lengths, closed form and trapezoid branch (separated steps at
  r = 0.002), against brute-force two-dimensional quadrature of the kernel
  over the time rectangle.
* On a uniform grid the general (absolute step pair) assembly equals the
  Toeplitz one.
* The double-layer identity (1/2 M_h + K_h) 1 = Galerkin projection of the
  volume heat potential of 1, and V_h 1 against the face-wise erf formula,
  on a graded grid.
* Algorithm 1 splits at the node nearest to the time midpoint (the earlier
  of two equally near); with no spatial cut every causal element pair lies
  in exactly one nearfield or admissible block.
* The pFMM product converges to the dense product as the degrees grow.
"""
import numpy as np
import pytest
from scipy.integrate import dblquad
from scipy.special import erf

from oracle import fmm as F
from oracle.dense import (dense_matrix, dense_matrix_steps, geometry, mass_diag_steps, toeplitz_blocks)
from oracle.quadrature import gauss_legendre01, triangle_rule
from oracle.timeint import G, time_factor_steps
from oracle.tree import Tree
from workloads import cube_surface_mesh, densities

ALPHA = 0.7


def graded_nodes(n, T=1.0, p=1.7):
    """Steps growing from the start: t_j = T (j / n)^p."""
    return T * (np.arange(n + 1) / n) ** p


@pytest.mark.parametrize("kind", ["V", "K"])
@pytest.mark.parametrize("r", [0.002, 0.05, 0.3])
@pytest.mark.parametrize("steps", [((0.40, 0.43), (0.40, 0.43)), ((0.45, 0.47), (0.40, 0.45)),
                                   ((0.80, 0.83), (0.40, 0.45)), ((0.61, 0.62), (0.20, 0.26))])
def test_time_factor_steps_brute_force(kind, r, steps):
    (tk0, tk1), (tj0, tj1) = steps
    d = 0 if tk0 == tj0 else (1 if tk0 == tj1 else 2)
    if d < 2 and r < 0.01:
        pytest.skip("touching steps at r << step: the brute-force reference itself is inaccurate")
    g = (lambda s: G(r, s, ALPHA)) if kind == "V" else (lambda s: G(r, s, ALPHA) / (2 * s))
    ref = dblquad(lambda tau, t: g(t - tau) if t > tau else 0.0, tk0, tk1, tj0, lambda t: min(t, tj1),
                  epsabs=0, epsrel=1e-12)[0]
    val = float(time_factor_steps(np.array([r]), tk0, tk1, tj0, tj1, d, ALPHA, kind)[0])
    tol = 1e-9 if kind == "V" else 1e-7
    assert abs(val - ref) <= tol * abs(ref) + 1e-300, (val, ref)


def test_uniform_grid_general_equals_toeplitz():
    v, t = cube_surface_mesh(2)
    E_t = 4
    tn = np.arange(E_t + 1) * 0.25
    for kind in ("V", "K"):
        A = dense_matrix(v, t, E_t, 0.25, ALPHA, kind, B=toeplitz_blocks(v, t, E_t, 0.25, ALPHA, kind))
        Bm = dense_matrix_steps(v, t, tn, ALPHA, kind)
        assert np.abs(A - Bm).max() <= 1e-11 * np.abs(A).max()


def _element_points(v, t, qx):
    s, tt, w = triangle_rule(qx)
    area, _, _ = geometry(v, t)
    P = v[t]
    x = P[:, 0, None, :] + s[None, :, None] * (P[:, 1] - P[:, 0])[:, None, :] \
        + tt[None, :, None] * (P[:, 2] - P[:, 1])[:, None, :]
    return x, w, area


def test_double_layer_identity_graded_grid():
    v, t = cube_surface_mesh(2)
    tn = graded_nodes(5)
    K = dense_matrix_steps(v, t, tn, ALPHA, "K", q_reg=7, q_sing=10)
    lhs = 0.5 * mass_diag_steps(v, t, tn) + K.sum(axis=1)
    x, w, area = _element_points(v, t, 12)
    g, wg = gauss_legendre01(16)
    nt = len(t)
    ref = np.zeros(len(lhs))
    for kt in range(len(tn) - 1):
        h = tn[kt + 1] - tn[kt]
        T = tn[kt] + g * h
        val = np.ones(x.shape[:2] + (len(T),))
        for j in range(3):
            xj = x[:, :, j][..., None]
            val *= 0.5 * (erf((1 - xj) / (2 * np.sqrt(ALPHA * T))) + erf((1 + xj) / (2 * np.sqrt(ALPHA * T))))
        ref[kt * nt:(kt + 1) * nt] = np.einsum("epq,p,q->e", val, w, wg) * 2 * area * h
    assert np.abs(lhs - ref).max() <= 1e-4 * np.abs(ref).max()


def _v_one(x, T, alpha, nu=64):
    g, wg = gauss_legendre01(nu)
    sq = np.sqrt(T)[None, :, None]
    s = (sq * g[None, None, :]) ** 2
    x = x[:, None, None, :]
    tot = 0.0
    for a in range(3):
        for sig in (-1.0, 1.0):
            z = x[..., a] - sig
            fac = 2.0 * np.exp(-z * z / (4 * alpha * s)) / np.sqrt(4 * np.pi * alpha)
            for j in range(3):
                if j == a:
                    continue
                xi = x[..., j]
                fac = fac * 0.5 * (erf((xi + 1) / (2 * np.sqrt(alpha * s))) - erf((xi - 1) / (2 * np.sqrt(alpha * s))))
            tot = tot + np.sum(wg * fac, axis=-1) * sq[..., 0]
    return tot


def test_single_layer_constant_density_graded_grid():
    v, t = cube_surface_mesh(2)
    tn = graded_nodes(4)
    A = dense_matrix_steps(v, t, tn, ALPHA, "V", q_reg=7, q_sing=10)
    lhs = A.sum(axis=1)
    x, w, area = _element_points(v, t, 8)
    g, wg = gauss_legendre01(8)
    nt = len(t)
    ref = np.zeros(len(lhs))
    for kt in range(len(tn) - 1):
        h = tn[kt + 1] - tn[kt]
        if kt == 0:      # (V 1)(x, t) ~ sqrt(t): integrate in v, t = h v^2
            tp, wt = h * g * g, wg * 2.0 * g
        else:
            tp, wt = tn[kt] + g * h, wg
        for e in range(nt):
            ref[kt * nt + e] = (w @ _v_one(x[e], tp, ALPHA) @ wt) * 2 * area[e] * h
    assert np.abs(lhs - ref).max() <= 1e-4 * np.abs(ref).max()


def test_split_at_nearest_node_and_coverage():
    v, t = cube_surface_mesh(2)
    tn = graded_nodes(11)
    tr = Tree(v, t, tn, 1.0, 8, 0.9, -1)
    assert not tr.uniform
    for lev in tr.levels:
        for b in lev:
            if b.children:
                mids = sorted(set(c.s0 for c in b.children) | set(c.s1 for c in b.children))
                split = mids[1]
                tm = 0.5 * (tn[b.s0] + tn[b.s1])
                best = min(abs(tn[j] - tm) for j in range(b.s0 + 1, b.s1))
                assert abs(tn[split] - tm) <= best + 1e-12
                assert all(abs(tn[j] - tm) > best + 1e-12 for j in range(b.s0 + 1, split))
    N = tr.E_t * tr.E_x
    cnt = np.zeros((N, N), dtype=np.int32)
    memo = {}
    for Z in tr.leaves:
        for S in tr.nearfield(Z, memo):
            cnt[np.ix_(tr.elements(Z), tr.elements(S))] += 1
    for Z in tr.boxes:
        for S in tr.interaction(Z):
            rows, cols = tr.elements(Z), tr.elements(S)
            assert np.all(cols[None, :] // tr.E_x <= rows[:, None] // tr.E_x)
            cnt[np.ix_(rows, cols)] += 1
    kt = np.arange(N) // tr.E_x
    causal = kt[:, None] >= kt[None, :]
    assert np.all(cnt[causal] == 1)


def test_pfmm_converges_to_dense_on_graded_grid():
    """The pFMM on a graded grid approaches the dense product as the
    expansion degree grows (nearfield exact, so only the farfield changes
    with m; on this mesh the errors are close to those of a uniform grid:
    about 7e-2, 3e-2 and 1.1e-2 for m = 2, 4, 6)."""
    v, t = cube_surface_mesh(2)
    tn = graded_nodes(12)
    tr = Tree(v, t, tn, 1.0, 8, 0.9, -1)
    w = densities(12 * len(t), 3)
    fd = dense_matrix_steps(v, t, tn, 1.0, "V") @ w
    near = None
    errs = []
    for m in (2, 4, 6):
        o = F.FMMOracle(tr, m, m, "V")
        if near is None:
            near = o.nearfield(w)
        errs.append(np.linalg.norm(o.farfield(w) + near - fd) / np.linalg.norm(fd))
    assert errs[0] > errs[1] > errs[2], errs
    assert errs[2] < 2e-2 and errs[2] < 0.25 * errs[0], errs

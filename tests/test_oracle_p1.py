"""Pins of the oracle's double layer with p1-continuous trial functions (CPU only).

* The p1-weighted touching-pair rules integrate f(x - y) lambda_i(y)
  exactly for polynomial f (against the tensor Gauss rule of high order),
  and the 1/r kernel with a linear weight on coplanar touching pairs
  against a closed form: lambda_i(y) = lambda_i(x) + grad lambda_i . (y - x),
  int_T dy / |x - y| in closed form and int_T (y - x) / |y - x| dy as a sum
  of closed-form edge integrals of |y - x| (divergence theorem).
* K_h 1 (p1, all vertex values one) equals K_h 1 of the p0 double layer.
* Green's identity for the caloric function u = a.x + b on the cube: with
  zero flux data the interior trace gives (1/2 I + K) u = U0 u0 + V (alpha
  du/dn), U0 u0 the initial potential of u0 = u; u's p1 interpolant and its
  normal derivative (constant per face) are exact in the discrete spaces,
  so (1/2 M_h + K_h) u_h - V_h (alpha a.n) equals the p0 tests of U0 u0 up
  to quadrature error.
* The FMM with p1 trial functions converges to the dense product.
"""
import numpy as np
import pytest
from scipy import integrate
from scipy.special import erf

from oracle import quadrature as Q
from oracle.dense import dense_matrix_steps, geometry
from oracle.p1 import FMMOracleP1, dense_matrix_K1, mixed_mass, p1_mass
from oracle.quadrature import gauss_legendre01, triangle_rule
from oracle.tree import Tree
from workloads import cube_surface_mesh, uniform_time_nodes

V8 = np.array([[0, 0, 0], [1, 0, 0], [0.3, 0.9, 0], [1.2, 0.8, 0], [-0.6, 0.4, 0],
               [0.2, 0.1, 0.8], [1.0, -0.7, 0.0], [1.7, 0.1, 0.0]], dtype=float)
CASES = {"edge": ([0, 1, 2], [1, 0, 6]), "vertex": ([0, 1, 2], [1, 3, 7]),
         "edge90": ([0, 1, 2], [1, 0, 5]), "vertex90": ([0, 1, 2], [0, 5, 4]),
         "edge_rev": ([0, 1, 2], [6, 0, 1]), "vertex_rot": ([0, 1, 2], [3, 7, 1])}


@pytest.mark.parametrize("case", sorted(CASES))
def test_p1_rules_polynomials(case):
    tris = np.array(CASES[case])
    d, W, lam = Q.pair_rule_p1(V8, tris, 0, 1, True, 4, 6)
    d2, W2, lam2 = Q.regular_rule_p1(V8[tris[0]], V8[tris[1]], 8)
    assert np.allclose(lam.sum(1), 1.0)
    for f in (lambda x: np.ones(len(x)), lambda x: (x ** 2).sum(1), lambda x: x[:, 0] * x[:, 1] ** 2 + x[:, 2]):
        for i in range(3):
            a, b = np.sum(W * f(d) * lam[:, i]), np.sum(W2 * f(d2) * lam2[:, i])
            assert abs(a - b) < 1e-13 * max(1.0, abs(b)), (i, a, b)


def _pot(T, x):
    """int_T dy / |x - y|, x in the plane of the 2D ccw triangle T."""
    tot = 0.0
    for e in range(3):
        A, B = T[e], T[(e + 1) % 3]
        L = np.linalg.norm(B - A)
        t = (B - A) / L
        n = np.array([t[1], -t[0]])
        de = np.dot(A - x, n)
        if abs(de) < 1e-14:
            continue
        lm, lp = np.dot(A - x, t), np.dot(B - x, t)
        tot += de * np.log((lp + np.linalg.norm(B - x)) / (lm + np.linalg.norm(A - x)))
    return tot


def _edge_dist_integral(A, B, x):
    """int over the segment AB of |y - x| ds (closed form in the arc
    coordinate l along the line, distance d to it: int sqrt(l^2 + d^2) dl)."""
    L = np.linalg.norm(B - A)
    t = (B - A) / L
    l0, l1 = np.dot(A - x, t), np.dot(B - x, t)
    d2 = max(np.dot(A - x, A - x) - l0 * l0, 0.0)
    if d2 < 1e-28:          # x on the segment's line: int |l| dl
        return 0.5 * (np.sign(l1) * l1 * l1 - np.sign(l0) * l0 * l0)
    F = lambda l: 0.5 * (l * np.sqrt(l * l + d2) + d2 * np.log(l + np.sqrt(l * l + d2)))
    return F(l1) - F(l0)


def _grad_term(T, x):
    """int_T (y - x) / |y - x| dy = sum_e n_e int_e |y - x| ds (ccw T)."""
    out = np.zeros(2)
    for e in range(3):
        A, B = T[e], T[(e + 1) % 3]
        t = (B - A) / np.linalg.norm(B - A)
        out += np.array([t[1], -t[0]]) * _edge_dist_integral(A, B, x)
    return out


@pytest.mark.parametrize("case", ["edge", "vertex", "edge_rev", "vertex_rot"])
def test_p1_rules_one_over_r_linear_weight(case):
    tris = np.array(CASES[case])
    P1, P2 = V8[tris[0]][:, :2], V8[tris[1]][:, :2]
    cross2 = lambda u, w: u[0] * w[1] - u[1] * w[0]
    ccw = lambda P: P if cross2(P[1] - P[0], P[2] - P[0]) > 0 else P[[0, 2, 1]]
    T2 = ccw(P2)
    # barycentric coordinate of vertex i of the source: lambda_i(y) = c_i + g_i . y
    M = np.column_stack([P2, np.ones(3)])
    coef = np.linalg.solve(M, np.eye(3))          # column i: (g_i, c_i)
    d, W, lam = Q.pair_rule_p1(V8, tris, 0, 1, True, 4, 12)
    A1, B1, C1 = ccw(P1)
    area2 = abs(cross2(B1 - A1, C1 - A1))
    for i in range(3):
        g, c = coef[:2, i], coef[2, i]

        def f(v, u):
            x = A1 + u * (B1 - A1) + v * (C1 - A1)
            return (c + g @ x) * _pot(T2, x) + g @ _grad_term(T2, x)
        ref = area2 * integrate.dblquad(f, 0, 1, lambda u: 0, lambda u: 1 - u, epsabs=1e-13, epsrel=1e-10)[0]
        val = np.sum(W * lam[:, i] / np.linalg.norm(d, axis=1))
        assert abs(val - ref) < 1e-8 * abs(ref), (i, val, ref)


def test_K1_of_one_equals_p0_double_layer():
    v, t = cube_surface_mesh(2)
    tn = uniform_time_nodes(3)
    K1 = dense_matrix_K1(v, t, tn, 0.7)
    K0 = dense_matrix_steps(v, t, tn, 0.7, "K")
    a = K1 @ np.ones(3 * len(v))
    b = K0 @ np.ones(3 * len(t))
    assert np.abs(a - b).max() <= 1e-12 * np.abs(b).max()
    # and M_h 1 = the p0 mass diagonal; the p1 mass of 1 = the vertex areas
    M = mixed_mass(v, t, tn)
    area = geometry(v, t)[0]
    assert np.allclose(M @ np.ones(3 * len(v)), np.tile(area, 3) / 3.0)
    assert abs(p1_mass(v, t).sum() - area.sum()) < 1e-13


def _initial_potential_linear(x, T, a, b, alpha):
    """int_{[-1,1]^3} G(x - y, T) (a.y + b) dy (closed form, separable)."""
    s = 2.0 * np.sqrt(alpha * T)
    I0 = [0.5 * (erf((1 - x[..., j]) / s) + erf((1 + x[..., j]) / s)) for j in range(3)]
    I1 = [x[..., j] * I0[j] + np.sqrt(alpha * T / np.pi) * (np.exp(-((1 + x[..., j]) / s) ** 2)
                                                           - np.exp(-((1 - x[..., j]) / s) ** 2)) for j in range(3)]
    out = b * I0[0] * I0[1] * I0[2]
    out = out + a[0] * I1[0] * I0[1] * I0[2] + a[1] * I0[0] * I1[1] * I0[2] + a[2] * I0[0] * I0[1] * I1[2]
    return out


def test_green_identity_linear_caloric():
    alpha = 0.7
    a, b = np.array([1.0, 2.0, -0.5]), 0.3
    v, t = cube_surface_mesh(2)
    tn = np.array([0.0, 0.15, 0.35, 0.6])
    E_t, nt = len(tn) - 1, len(t)
    u = np.tile(v @ a + b, E_t)
    area, nrm, _ = geometry(v, t)
    flux = np.tile(alpha * (nrm @ a), E_t)
    K1 = dense_matrix_K1(v, t, tn, alpha, q_reg=7, q_sing=10)
    Vh = dense_matrix_steps(v, t, tn, alpha, "V", q_reg=7, q_sing=10)
    lhs = 0.5 * mixed_mass(v, t, tn) @ u + K1 @ u - Vh @ flux
    s, tt, w = triangle_rule(12)
    P = v[t]
    x = P[:, 0, None, :] + s[None, :, None] * (P[:, 1] - P[:, 0])[:, None, :] \
        + tt[None, :, None] * (P[:, 2] - P[:, 1])[:, None, :]
    g, wg = gauss_legendre01(16)
    ref = np.zeros(E_t * nt)
    for kt in range(E_t):
        h = tn[kt + 1] - tn[kt]
        for T, wt in zip(tn[kt] + g * h, wg * h):
            ref[kt * nt:(kt + 1) * nt] += wt * (_initial_potential_linear(x, T, a, b, alpha) @ w) * 2 * area
    # residual 1.7e-4 at (q_reg, q_sing) = (4, 5) and 3.5e-5 at (7, 10): quadrature error
    assert np.abs(lhs - ref).max() <= 1e-4 * np.abs(ref).max()


def test_fmm_p1_converges_to_dense():
    v, t = cube_surface_mesh(2)
    tn = uniform_time_nodes(8)
    tr = Tree(v, t, tn, 1.0, 8, 0.9, -1)
    rng = np.random.default_rng(5)
    u = rng.uniform(-1.0, 1.0, 8 * len(v))
    fd = dense_matrix_K1(v, t, tn, 1.0) @ u
    near = None
    errs = []
    for m in (2, 4, 6):
        o = FMMOracleP1(tr, m, m)
        if near is None:
            near = o.nearfield(u)
        errs.append(np.linalg.norm(o.farfield(u) + near - fd) / np.linalg.norm(fd))
    assert errs[0] > errs[1] > errs[2], errs
    assert errs[2] < 0.25 * errs[0], errs
    # sampled rows through the ancestor chains equal the full apply (the
    # nearfield does not depend on the degrees)
    o = FMMOracleP1(tr, 3, 3)
    full = o.farfield(u) + near
    rows = np.array([0, 5, 77, 200, 383])
    vals, _ = o.apply_rows(u, rows)
    assert np.abs(vals - full[rows]).max() <= 1e-13 * np.abs(full).max()

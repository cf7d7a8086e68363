"""Pins of the oracle's dense Galerkin matrices (CPU only).

* Causality and the Toeplitz structure of V_h for uniform steps (Section 2).
* Symmetry of the blocks of V_h (the kernel depends on |x - y|) and positive
  definiteness of the diagonal block.
* V_h 1 against a semi-analytic evaluation of the single-layer potential of
  the constant density on the cube: the surface integral factorises per face
  into erf products, leaving a 1D time integral.
* Double-layer identity: (1/2 M_h + K_h) 1 equals the Galerkin projection of
  the volume heat potential of the constant 1, which on (-1,1)^3 is
  prod_j 1/2 [erf((1 - x_j)/(2 sqrt(alpha t))) + erf((1 + x_j)/(2 sqrt(alpha t)))]
  (the divergence theorem applied to G for t > 0).
"""
import numpy as np
import pytest
from scipy.special import erf

from oracle.dense import toeplitz_blocks, dense_matrix, mass_diag, geometry
from oracle.quadrature import triangle_rule, gauss_legendre01
from workloads import cube_surface_mesh

ALPHA = 1.0


@pytest.fixture(scope="module")
def small():
    v, t = cube_surface_mesh(2)
    E_t = 4
    h = 1.0 / E_t
    BV = toeplitz_blocks(v, t, E_t, h, ALPHA, "V")
    BK = toeplitz_blocks(v, t, E_t, h, ALPHA, "K")
    return v, t, E_t, h, BV, BK


def _element_points(v, t, E_t, h, qx=7, qt=6):
    s, tt, w = triangle_rule(qx)
    g, wg = gauss_legendre01(qt)
    area, _, _ = geometry(v, t)
    P = v[t]
    x = P[:, 0, None, :] + s[None, :, None] * (P[:, 1] - P[:, 0])[:, None, :] \
        + tt[None, :, None] * (P[:, 2] - P[:, 1])[:, None, :]
    return x, w * 1.0, g, wg, area


def test_causal_toeplitz_structure(small):
    v, t, E_t, h, BV, BK = small
    A = dense_matrix(v, t, E_t, h, ALPHA, "V", B=BV)
    nt = len(t)
    for kt in range(E_t):
        for jt in range(E_t):
            blk = A[kt * nt:(kt + 1) * nt, jt * nt:(jt + 1) * nt]
            if jt > kt:
                assert np.all(blk == 0.0)
            elif kt + 1 < E_t:
                nxt = A[(kt + 1) * nt:(kt + 2) * nt, (jt + 1) * nt:(jt + 2) * nt]
                assert np.array_equal(blk, nxt)


def test_regular_entries_from_absolute_times(small):
    """Entries of the dense V_h for panel pairs that do not touch, computed
    from the definition with the absolute time nodes t_j = j h: the double
    time integral of G over steps k and j is the four-term combination
    G2(t_k - t_{j-1}) - G2(t_k - t_j) - G2(t_{k-1} - t_{j-1}) + G2(t_{k-1} - t_j)
    of the second antiderivative G2 (zero for s <= 0; pinned separately by
    brute-force quadrature), summed over the regular space rule.  This does
    not use the step-difference form the oracle assembles from, so it checks
    causality (j > k gives 0) and the Toeplitz structure independently."""
    from oracle.quadrature import classify
    from oracle.timeint import G2
    v, t, E_t, h, BV, BK = small
    A = dense_matrix(v, t, E_t, h, ALPHA, "V", B=BV)
    nt = len(t)
    s_, t_, w_ = triangle_rule(4)
    area, _, _ = geometry(v, t)
    P = v[t]
    rng = np.random.default_rng(3)
    pairs = [(k, j) for k in range(nt) for j in range(nt) if classify(t[k], t[j]) == 0]
    tn = np.arange(E_t + 1) * h

    def g2(r, s):
        return np.where(s > 0, G2(r, np.maximum(s, 1e-300), ALPHA), 0.0)

    for i in rng.choice(len(pairs), 12, replace=False):
        k, j = pairs[i]
        xk = P[k, 0] + s_[:, None] * (P[k, 1] - P[k, 0]) + t_[:, None] * (P[k, 2] - P[k, 1])
        xj = P[j, 0] + s_[:, None] * (P[j, 1] - P[j, 0]) + t_[:, None] * (P[j, 2] - P[j, 1])
        W = (2 * area[k] * w_)[:, None] * (2 * area[j] * w_)[None, :]
        r = np.linalg.norm(xk[:, None, :] - xj[None, :, :], axis=-1)
        for kt in range(E_t):
            for jt in range(E_t):
                tf = (g2(r, tn[kt + 1] - tn[jt]) - g2(r, tn[kt + 1] - tn[jt + 1])
                      - g2(r, tn[kt] - tn[jt]) + g2(r, tn[kt] - tn[jt + 1]))
                ref = np.sum(W * tf)
                got = A[kt * nt + k, jt * nt + j]
                if jt > kt:
                    assert got == 0.0 and ref == 0.0
                else:
                    assert abs(got - ref) <= 1e-10 * abs(ref), (k, j, kt, jt, got, ref)


def test_block_symmetry_and_spd(small):
    v, t, E_t, h, BV, BK = small
    for d in range(2, E_t):
        # d >= 2 uses the symmetric regular rule for every non-identical pair
        assert np.abs(BV[d] - BV[d].T).max() <= 1e-14 * np.abs(BV[d]).max()
    # d = 0, 1 touching pairs use parametrisation-dependent rules: symmetric to quadrature accuracy
    assert np.abs(BV[0] - BV[0].T).max() <= 1e-4 * np.abs(BV[0]).max()
    np.linalg.cholesky(0.5 * (BV[0] + BV[0].T))


def _v_one(x, T, alpha, nu=64):
    """(V 1)(x, T) for points x (n,3) on the cube surface and times T (m,).

    Face-wise erf formula; the inner time integral uses s = u^2.
    """
    g, wg = gauss_legendre01(nu)
    sq = np.sqrt(T)[None, :, None]                 # (1, m, 1)
    s = (sq * g[None, None, :]) ** 2               # (1, m, nu)
    x = x[:, None, None, :]                        # (n, 1, 1, 3)
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
    return tot                                      # (n, m)


@pytest.mark.parametrize("orders,tol", [((4, 5), 5e-4), ((7, 10), 1e-4)])
def test_single_layer_constant_density(orders, tol):
    v, t = cube_surface_mesh(2)
    E_t, h = 4, 0.25
    B = toeplitz_blocks(v, t, E_t, h, ALPHA, "V", q_reg=orders[0], q_sing=orders[1])
    A = dense_matrix(v, t, E_t, h, ALPHA, "V", B=B)
    lhs = A.sum(axis=1)
    x, w, g, wg, area = _element_points(v, t, E_t, h, qx=8, qt=8)
    nt = len(t)
    ref = np.zeros(E_t * nt)
    for kt in range(E_t):
        # (V 1)(x, t) ~ sqrt(t) as t -> 0: on the first step integrate in v, t = h v^2
        if kt == 0:
            tp, wt = h * g * g, wg * 2.0 * g
        else:
            tp, wt = (kt + g) * h, wg
        for e in range(nt):
            val = _v_one(x[e], tp, ALPHA)
            ref[kt * nt + e] = (w @ val @ wt) * 2 * area[e] * h
    assert np.abs(lhs - ref).max() <= tol * np.abs(ref).max()


@pytest.mark.parametrize("orders,tol", [((4, 5), 5e-4), ((7, 10), 1e-4)])
def test_double_layer_identity(orders, tol):
    v, t = cube_surface_mesh(2)
    E_t, h = 4, 0.25
    B = toeplitz_blocks(v, t, E_t, h, ALPHA, "K", q_reg=orders[0], q_sing=orders[1])
    K = dense_matrix(v, t, E_t, h, ALPHA, "K", B=B)
    lhs = 0.5 * mass_diag(v, t, E_t, h) + K.sum(axis=1)
    x, w, g, wg, area = _element_points(v, t, E_t, h, qx=12, qt=16)
    nt = len(t)
    ref = np.zeros(E_t * nt)
    for kt in range(E_t):
        T = (kt + g) * h
        val = np.ones(x.shape[:2] + (len(T),))
        for j in range(3):
            xj = x[:, :, j][..., None]
            val *= 0.5 * (erf((1 - xj) / (2 * np.sqrt(ALPHA * T))) + erf((1 + xj) / (2 * np.sqrt(ALPHA * T))))
        ref[kt * nt:(kt + 1) * nt] = np.einsum("epq,p,q->e", val, w, wg) * 2 * area * h
    assert np.abs(lhs - ref).max() <= tol * np.abs(ref).max()


def test_coplanar_double_layer_zero(small):
    v, t, E_t, h, BV, BK = small
    _, nrm, _ = geometry(v, t)
    same_face = np.abs(nrm @ nrm.T - 1.0) < 1e-12
    for d in range(E_t):
        assert np.all(BK[d][same_face] == 0.0)

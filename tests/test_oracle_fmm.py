"""Pins of the oracle's FMM operators and apply (CPU only).

* S2M / L2T tables integrate polynomials exactly (a rule of much higher
  order gives the same values).
* M2M and L2L are exact re-expansions: moments of a parent obtained from its
  children equal moments computed directly with the parent's basis; locals
  passed down and evaluated in a child equal the parent's locals evaluated
  there (eqs. temp_m2m, st_m2m and their transposes).
* The expansion of eq. kernel_approx approximates the heat kernel on
  admissible box pairs with the expected error per degree (independent
  brute-force values, within a factor 2) and converges as the degrees grow.
* The pFMM product converges to the dense product V_h w (and K_h w) as the
  degrees grow, with no spatial cut (Algorithm 2 vs Section 2).
"""
import numpy as np
import pytest

from oracle import fmm as F
from oracle.dense import toeplitz_blocks, dense_matrix
from oracle.quadrature import triangle_rule, gauss_legendre01
from oracle.timeint import G
from oracle.tree import Tree
from workloads import cube_surface_mesh, uniform_time_nodes, densities


@pytest.fixture(scope="module")
def c1():
    v, t = cube_surface_mesh(4)
    E_t = 16
    tr = Tree(v, t, uniform_time_nodes(E_t), 1.0, 64, 0.9, -1)
    h = 1.0 / E_t
    BV = toeplitz_blocks(v, t, E_t, h, 1.0, "V")
    BK = toeplitz_blocks(v, t, E_t, h, 1.0, "K")
    w = densities(E_t * len(t), 1)
    return v, t, E_t, h, tr, BV, BK, w


def test_tables_exact(c1):
    v, t, E_t, h, tr, BV, BK, w = c1
    o = F.FMMOracle(tr, 6, 6, "V")
    b = tr.levels[3][17]
    A = o.A_x(b, "V")
    AK = o.A_x(b, "K")
    # same integrals with a much finer triangle rule
    s, tt, wq = triangle_rule(12)
    P = tr.verts[tr.tri[b.tris]]
    y = P[:, 0, None, :] + s[None, :, None] * (P[:, 1] - P[:, 0])[:, None, :] \
        + tt[None, :, None] * (P[:, 2] - P[:, 1])[:, None, :]
    yh, H = o._ref_coords(b, y.reshape(-1, 3))
    T = [F.cheb_T(6, yh[:, j]) for j in range(3)]
    dT = [F.cheb_dT(6, yh[:, j]) / H for j in range(3)]
    mi = o.mi
    val = (T[0][mi[:, 0]] * T[1][mi[:, 1]] * T[2][mi[:, 2]]).reshape(len(mi), len(b.tris), -1)
    ref = np.einsum("kiq,q,i->ik", val, wq, 2 * o.area[b.tris])
    assert np.abs(A - ref).max() < 1e-14
    nrm = np.repeat(o.normal[b.tris], len(wq), axis=0)
    valK = sum(nrm[:, j] * dT[j][mi[:, j]] * T[(j + 1) % 3][mi[:, (j + 1) % 3]] * T[(j + 2) % 3][mi[:, (j + 2) % 3]]
               for j in range(3)).reshape(len(mi), len(b.tris), -1)
    refK = np.einsum("kiq,q,i->ik", valK, wq, 2 * o.area[b.tris])
    assert np.abs(AK - refK).max() < 1e-12
    # temporal table: integral of each Lagrange polynomial over the whole interval
    At = o.A_t(b)
    g, wg = gauss_legendre01(12)
    ta, tb = tr.interval(b)
    ref_t = F.lagrange(o.tnodes(b), ta + (tb - ta) * g) @ (wg * (tb - ta))
    assert np.abs(At.sum(0) - ref_t).max() < 1e-15


@pytest.mark.parametrize("kind", ["V", "K"])
def test_m2m_l2l_exact(kind):
    v, t = cube_surface_mesh(4)
    tr = Tree(v, t, uniform_time_nodes(16), 1.0, 64, 0.9, -1)
    o = F.FMMOracle(tr, 5, 5, kind)
    rng = np.random.default_rng(0)
    w = rng.uniform(-1, 1, tr.E_t * tr.E_x)
    W = w.reshape(tr.E_t, tr.E_x)
    for l in (1, 2):           # level 1 -> 2 is temporal, level 2 -> 3 space-time
        p = tr.levels[l][3]
        direct = o.A_t(p).T @ W[p.s0:p.s1][:, p.tris] @ o.A_x(p)
        via = sum(o.qt(c, p).T @ (o.A_t(c).T @ W[c.s0:c.s1][:, c.tris] @ o.A_x(c)) @ o.qx(c, p)
                  for c in p.children)
        assert np.abs(direct - via).max() < 1e-13 * np.abs(direct).max()
        lam_p = rng.uniform(-1, 1, (o.m_t + 1, o.Nk))
        for c in p.children:
            pos = [list(p.tris).index(i) for i in c.tris]
            rows = np.arange(c.s0, c.s1) - p.s0
            parent_eval = (o.A_t(p) @ lam_p @ o.A_x(p, "V").T)[np.ix_(rows, pos)]
            child_eval = o.l2t(c, o.l2l(c, p, lam_p))
            assert np.abs(parent_eval - child_eval).max() < 1e-12 * np.abs(parent_eval).max()


# Relative kernel-approximation error max|G - expansion| / max|G| on
# admissible box pairs with spatial offsets (0,0,0), (1,0,0), (1,1,0) and
# time offsets of 2 and 3 intervals, for box-size ratios
# c = H^2 / (4 alpha h_t) = 0.25 and 0.5 (H, h_t the spatial and temporal
# half-sizes, the ratio of eq. rel_h_t_h_x), m_t = m_x = m: values of an
# independent brute-force evaluation of the truncated Chebyshev x Lagrange
# interpolant of the heat kernel (eqs. kernel_approx, exp_coeffs_3d,
# exp_coeffs_1d) against the kernel itself.
P10_EXPECTED = {0.25: {2: 7e-2, 4: 8e-3, 6: 8e-4, 8: 6e-5}, 0.5: {2: 1.7e-1, 4: 2.9e-2, 6: 5.5e-3, 8: 6.4e-4}}


def _expansion_error(o, tr, Z, S, rng, npts=200):
    m = o.m_x
    op = o.m2l_operator(Z, S)
    lo_x, lo_y = tr.box_lower(Z), tr.box_lower(S)
    H = tr.hx_padded(Z.level)
    x = lo_x + 2 * H * rng.uniform(size=(npts, 3))
    y = lo_y + 2 * H * rng.uniform(size=(npts, 3))
    ta, tb = tr.interval(Z)
    sa, sb = tr.interval(S)
    tt = ta + (tb - ta) * rng.uniform(size=npts)
    tau = sa + (sb - sa) * rng.uniform(size=npts)
    exact = G(np.linalg.norm(x - y, axis=1), tt - tau, 1.0)
    Tx = [F.cheb_T(m, (x[:, j] - lo_x[j]) / H - 1) for j in range(3)]
    Ty = [F.cheb_T(m, (y[:, j] - lo_y[j]) / H - 1) for j in range(3)]
    mi = o.mi
    TX = Tx[0][mi[:, 0]] * Tx[1][mi[:, 1]] * Tx[2][mi[:, 2]]     # (N, npts)
    TY = Ty[0][mi[:, 0]] * Ty[1][mi[:, 1]] * Ty[2][mi[:, 2]]
    Lt = F.lagrange(o.tnodes(Z), tt)
    Ltau = F.lagrange(o.tnodes(S), tau)
    approx = np.einsum("bvak,vi,ki,bi,ai->i", op, TX, TY, Lt, Ltau)
    return np.abs(approx - exact).max() / np.abs(exact).max()


def test_kernel_expansion_error_values():
    """The oracle's M2L operator, read as the kernel expansion it is, has the
    expected approximation error (within a factor 2 either way, so a
    misplaced scale factor such as lambda_k or C_ab fails) and converges as
    m grows.  Cube 4 x 4 squares per face, 16 steps on [0, 1]: level 3 boxes
    have c = 0.25, level 2 boxes c = 0.5."""
    v, t = cube_surface_mesh(4)
    tr = Tree(v, t, uniform_time_nodes(16), 1.0, 64, 0.9, -1)
    for level, c in ((3, 0.25), (2, 0.5)):
        b0 = tr.levels[level][0]
        ta, tb = tr.interval(b0)
        assert abs(tr.hx_padded(level) ** 2 / (4 * 1.0 * (tb - ta) / 2) - c) < 1e-12
        pairs = []
        for off in ((0, 0, 0), (1, 0, 0), (1, 1, 0)):
            for D in (2, 3):
                found = None
                for Z in tr.levels[level]:
                    for S in tr.interaction(Z):
                        if tuple(np.subtract(Z.ix, S.ix)) == off and Z.k - S.k == D:
                            found = (Z, S)
                            break
                    if found:
                        break
                assert found, (level, off, D)
                pairs.append(found)
        errs = []
        for m in (2, 4, 6, 8):
            o = F.FMMOracle(tr, m, m, "V")
            rng = np.random.default_rng(1)
            e = max(_expansion_error(o, tr, Z, S, rng) for Z, S in pairs)
            errs.append(e)
            ratio = e / P10_EXPECTED[c][m]
            assert 0.5 <= ratio <= 2.0, (c, m, e, P10_EXPECTED[c][m])
        assert all(errs[i] > 5 * errs[i + 1] for i in range(3)), errs


def test_pfmm_converges_to_dense_V(c1):
    v, t, E_t, h, tr, BV, BK, w = c1
    fd = dense_matrix(v, t, E_t, h, 1.0, "V", B=BV) @ w
    errs = []
    for m in (2, 3, 4, 5):
        o = F.FMMOracle(tr, m, m, "V")
        o.set_toeplitz_blocks(BV)
        errs.append(np.linalg.norm(o.apply(w) - fd) / np.linalg.norm(fd))
    assert all(errs[i] > errs[i + 1] for i in range(len(errs) - 1)), errs
    assert errs[2] < 2e-3


def test_pfmm_converges_to_dense_K(c1):
    v, t, E_t, h, tr, BV, BK, w = c1
    fd = dense_matrix(v, t, E_t, h, 1.0, "K", B=BK) @ w
    errs = []
    for m in (2, 3, 4):
        o = F.FMMOracle(tr, m, m, "K")
        o.set_toeplitz_blocks(BK)
        errs.append(np.linalg.norm(o.apply(w) - fd) / np.linalg.norm(fd))
    assert all(errs[i] > errs[i + 1] for i in range(len(errs) - 1)), errs
    assert errs[2] < 1e-2


def test_rows_match_full_apply(c1):
    v, t, E_t, h, tr, BV, BK, w = c1
    o = F.FMMOracle(tr, 3, 3, "V")
    o.set_toeplitz_blocks(BV)
    full = o.apply(w)
    rows = np.array([0, 5, 1000, 2047, 3071])
    vals, _ = o.apply_rows(w, rows)
    assert np.abs(vals - full[rows]).max() < 1e-13 * np.abs(full).max()

"""The double layer with p1-continuous trial functions in space (oracle, test-only).

Section 2 discretises the Dirichlet datum by functions that are piecewise
linear and continuous in space (nodal hat functions phi_v at the mesh
vertices) and piecewise constant in time, and tests with p0 x p0 functions:

    K_h[(k_t, k_x), (j_t, v)] = int_{step k_t} int_{gamma_kx} int_{step j_t}
                                int_Gamma alpha dG/dn_y(x - y, t - tau) phi_v(y),
    M_h[(k_t, k_x), (j_t, v)] = delta_{k_t j_t} int_{step k_t} int_{gamma_kx} phi_v
                              = delta_{k_t j_t} h_{k_t} |gamma_kx| / 3  (v a vertex of k_x),

and the system V_h w = (1/2 M_h + K_h) g_h of Section 2 takes g_h as the
coefficients (per step and vertex) of the L2 projection of the datum.

On each source triangle phi_v is the barycentric coordinate of v, so an
entry is a sum over the triangles around v of panel integrals weighted by
lambda_i(y) (``quadrature.pair_rule_p1``) with the double-layer time factors
of ``timeint``; coplanar panel pairs vanish as for p0.  Vertex vectors are
time-major: index j_t n_v + v.

The FMM (Section 3.4) differs from the p0 double layer only in S2M: the
moments of a leaf take sum_i u(j_t, vertex i of j_x) A_x^{(i)}[j_x, kappa]
with A_x^{(i)} = alpha int_{gamma} lambda_i n.grad T_kappa; the nearfield
blocks carry three columns (the local vertices) per source element.

Parity: pinned by tests/test_oracle_p1.py -- the p1-weighted singular rules
against exact polynomial integrals and a closed-form in-plane 1/r potential
with a linear weight; K_h 1 against the p0 double layer of 1; and the
Galerkin-tested Green identity (1/2 M_h + K_h) u_h - V_h (alpha du/dn) =
the initial potential of u for the linear caloric function u = a.x + b,
whose p1 interpolant and normal derivative are exact in the discrete spaces.
"""
import numpy as np

from . import quadrature as Q
from .dense import _TimeSpec, coplanar, geometry
from .fmm import FMMOracle, cheb_T, cheb_dT
from .quadrature import triangle_rule
from .timeint import needs_singular_rule


def panel_integrals_K1(verts, tris, ks, js, dmax, h, alpha, q_reg=4, q_sing=5, tnodes=None, pairs=None):
    """Entries B[k, j][time][i] = int int alpha dG/dn_y lambda_i(y) for the
    panel pairs (ks[n], js[n]) and the local vertex i of js[n]; time offsets
    d = 0..dmax of uniform steps h, or the step pairs `pairs` of `tnodes`.

    Returns an array (len(ks), n_time, 3)."""
    ts = _TimeSpec(dmax, h, tnodes, pairs)
    ks = np.asarray(ks, dtype=np.int64)
    js = np.asarray(js, dtype=np.int64)
    out = np.zeros((len(ks), ts.n, 3))
    _, nrm, _ = geometry(verts, tris)
    for n, (k, j) in enumerate(zip(ks, js)):
        k, j = int(k), int(j)
        if coplanar(verts, tris, k, j):
            continue
        touching = Q.classify(tris[k], tris[j]) > 0
        for singular in (False, True):
            il = [i for i in range(ts.n) if touching and singular == needs_singular_rule(ts.offset(i))]
            if not touching:
                il = list(range(ts.n)) if not singular else []
            if not il:
                continue
            d, W, lam = Q.pair_rule_p1(verts, tris, k, j, singular, q_reg, q_sing)
            r = np.linalg.norm(d, axis=1)
            dn = d @ nrm[j]
            for i in il:
                tf = ts.factor(r, i, alpha, "K") * dn
                out[n, i] = (W * tf) @ lam
    return out


def dense_matrix_K1(verts, tris, tnodes, alpha, q_reg=4, q_sing=5):
    """K_h with p1 trial functions: (E_t E_x) x (E_t n_v), time-major."""
    tn = np.asarray(tnodes, dtype=np.float64)
    E_t, nt, nv = len(tn) - 1, len(tris), len(verts)
    pairs = [(kt, jt) for kt in range(E_t) for jt in range(kt + 1)]
    kk, jj = np.meshgrid(np.arange(nt), np.arange(nt), indexing="ij")
    kk, jj = kk.ravel(), jj.ravel()
    vals = panel_integrals_K1(verts, tris, kk, jj, 0, 0.0, alpha, q_reg, q_sing, tnodes=tn, pairs=pairs)
    A = np.zeros((E_t * nt, E_t * nv))
    for p, (kt, jt) in enumerate(pairs):
        for i in range(3):
            np.add.at(A, (kt * nt + kk, jt * nv + tris[jj, i]), vals[:, p, i])
    return A


def mixed_mass(verts, tris, tnodes):
    """M_h (p0 test x p1 trial): (E_t E_x) x (E_t n_v), time-major."""
    tn = np.asarray(tnodes, dtype=np.float64)
    E_t, nt, nv = len(tn) - 1, len(tris), len(verts)
    area = geometry(verts, tris)[0]
    M = np.zeros((E_t * nt, E_t * nv))
    for kt in range(E_t):
        h = tn[kt + 1] - tn[kt]
        for i in range(3):
            np.add.at(M, (kt * nt + np.arange(nt), kt * nv + tris[:, i]), h * area / 3.0)
    return M


def p1_mass(verts, tris):
    """int_Gamma phi_v phi_w (n_v x n_v): |gamma| (1 + delta_ij) / 12 per triangle."""
    area = geometry(verts, tris)[0]
    M = np.zeros((len(verts), len(verts)))
    for i in range(3):
        for j in range(3):
            np.add.at(M, (tris[:, i], tris[:, j]), area * (2.0 if i == j else 1.0) / 12.0)
    return M


class FMMOracleP1(FMMOracle):
    """Algorithm 2 for K_h with p1 trial functions: vectors u of length
    E_t n_v in, E_t E_x out (p0 test functions)."""

    def __init__(self, tree, m_t, m_x, q_reg=4, q_sing=5):
        super().__init__(tree, m_t, m_x, "K", q_reg, q_sing)
        self.n_v = len(tree.verts)

    def _local(self, u):
        """u per (step, triangle, local vertex)."""
        return np.asarray(u).reshape(self.tr.E_t, self.n_v)[:, self.tr.tri]

    def A_x_local(self, b):
        """A[i, c, kappa] = alpha int_{gamma_c} lambda_i n.grad T_kappa for triangle c of b."""
        key = (b.level, b.ix, "K1")
        if key in self._ax_cache:
            return self._ax_cache[key]
        s, t, w = triangle_rule(self.m_x // 2 + 2)
        P = self.tr.verts[self.tr.tri[b.tris]]
        y = (P[:, 0, None, :] + s[None, :, None] * (P[:, 1] - P[:, 0])[:, None, :]
             + t[None, :, None] * (P[:, 2] - P[:, 1])[:, None, :])
        yh, H = self._ref_coords(b, y.reshape(-1, 3))
        Tj = [cheb_T(self.m_x, yh[:, j]) for j in range(3)]
        dT = [cheb_dT(self.m_x, yh[:, j]) / H for j in range(3)]
        mi = self.mi
        nrm = np.repeat(self.normal[b.tris], len(w), axis=0)
        vals = self.alpha * (nrm[:, 0] * dT[0][mi[:, 0]] * Tj[1][mi[:, 1]] * Tj[2][mi[:, 2]]
                             + nrm[:, 1] * Tj[0][mi[:, 0]] * dT[1][mi[:, 1]] * Tj[2][mi[:, 2]]
                             + nrm[:, 2] * Tj[0][mi[:, 0]] * Tj[1][mi[:, 1]] * dT[2][mi[:, 2]])
        vals = vals.reshape(self.Nk, len(b.tris), len(w))
        lam = np.stack([1.0 - s, s - t, t])                                  # (3, q)
        A = np.einsum("kcq,iq,q,c->ick", vals, lam, w, 2.0 * self.area[b.tris])
        self._ax_cache[key] = A
        return A

    def moments(self, u):
        tr = self.tr
        U = self._local(u)
        mu = {}
        for b in tr.leaves:
            Ab = self.A_x_local(b)
            Ub = U[b.s0:b.s1][:, b.tris]                                     # (steps, c, 3)
            mu[b.id] = sum(self.A_t(b).T @ Ub[:, :, i] @ Ab[i] for i in range(3))
        for l in range(tr.depth - 1, 1, -1):
            for p in tr.levels[l]:
                if p.leaf:
                    continue
                acc = np.zeros((self.m_t + 1, self.Nk))
                for c in p.children:
                    acc += self.qt(c, p).T @ mu[c.id] @ self.qx(c, p)
                mu[p.id] = acc
        return mu

    def entries(self, kx, jx, dmax):
        return panel_integrals_K1(self.tr.verts, self.tr.tri, kx, jx, dmax, self.h, self.alpha, self.q_reg,
                                  self.q_sing)

    def entries_steps(self, kx, jx, pairs):
        return panel_integrals_K1(self.tr.verts, self.tr.tri, kx, jx, 0, 0.0, self.alpha, self.q_reg,
                                  self.q_sing, tnodes=self.tr.t, pairs=pairs)

    def near_contrib(self, Z, S, u):
        """Nearfield block of (Z, S) times the source values: rows (k_t, Z.tris)."""
        U = self._local(u)
        kt = np.arange(Z.s0, Z.s1)
        out = np.zeros((len(kt), len(Z.tris)))
        kx = np.repeat(Z.tris, len(S.tris))
        jx = np.tile(S.tris, len(Z.tris))
        if self.tr.uniform:
            dmax = int(max(Z.s1 - 1 - S.s0, 0))
            ent = self.entries(kx, jx, dmax).reshape(len(Z.tris), len(S.tris), dmax + 1, 3)
            for a in kt:
                for b in range(S.s0, min(S.s1, a + 1)):
                    out[a - Z.s0] += np.einsum("zsi,si->z", ent[:, :, a - b], U[b][S.tris])
        else:
            pairs = [(a, b) for a in kt for b in range(S.s0, S.s1) if b <= a]
            if pairs:
                ent = self.entries_steps(kx, jx, pairs).reshape(len(Z.tris), len(S.tris), len(pairs), 3)
                for p, (a, b) in enumerate(pairs):
                    out[a - Z.s0] += np.einsum("zsi,si->z", ent[:, :, p], U[b][S.tris])
        return out.ravel()

    def near_row(self, kt, kx, srcs, u):
        """Nearfield part of row (k_t, k_x) from the source boxes srcs."""
        U = self._local(u)
        tot = 0.0
        for S in srcs:
            js = list(range(S.s0, min(S.s1, kt + 1)))
            if not js:
                continue
            pairs = [(kt, b) for b in js]
            if self.tr.uniform:
                ent = self.entries(np.full(len(S.tris), kx), S.tris, kt - S.s0)       # (n, d, 3)
                for b in js:
                    tot += np.sum(ent[:, kt - b, :] * U[b][S.tris])
            else:
                ent = self.entries_steps(np.full(len(S.tris), kx), S.tris, pairs)
                for p, b in enumerate(js):
                    tot += np.sum(ent[:, p, :] * U[b][S.tris])
        return tot

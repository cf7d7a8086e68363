"""Space-time FMM apply of V_h and K_h (oracle, test-only).

Follows Section 3 step by step:

* temporal interpolation at transformed Chebyshev nodes (roots of T_{m_t+1})
  with Lagrange polynomials L_{I,b}, b = 0..m_t (0-based);
* spatial tensor Chebyshev polynomials T_{X,kappa} on the padded box,
  truncated to |kappa + nu| <= m_x (eq. kernel_approx);
* expansion coefficients eqs. exp_coeffs_3d, def_r_j, def_d_ab,
  exp_coeffs_1d, with xi_n tied to the target (nu) and xi_m to the source
  (kappa);
* S2M (eq. s2m), M2L (eq. m2l), L2T (eq. l2t), temporal and space-time M2M
  (eqs. temp_m2m, st_m2m), L2L as their transposes;
* Algorithm 2 order: S2M on leaves, M2M for levels p-1..2, M2L for every box
  from its interaction list, L2L for levels 3..p, L2T on leaves, nearfield
  product over the stored inadmissible blocks of every leaf.

Double layer (the paper says "with slight modifications"): the kernel
alpha dG/dn_y is expanded by applying alpha n_y . grad_y to the source
Chebyshev basis, so only S2M changes (moments of alpha n . grad T_{Y,kappa});
the nearfield uses the K_h entries.

Parity: pinned against the dense product (convergence as the degrees grow,
with no spatial cut), against exact polynomial integration for the S2M/L2T
tables, against direct evaluation for the M2M/L2L re-expansions, and against
pointwise kernel values for the expansion coefficients.
"""
import numpy as np

from .quadrature import gauss_legendre01, triangle_rule
from .dense import panel_integrals


# ------------------------------------------------------------ 1D bases

def cheb_nodes(m):
    k = np.arange(m + 1, dtype=np.float64)
    return np.cos((2.0 * k + 1.0) * np.pi / (2.0 * (m + 1)))


def cheb_T(kmax, x):
    """T_0..T_kmax at x by the three-term recurrence; shape (kmax+1,)+x.shape."""
    x = np.asarray(x, dtype=np.float64)
    out = np.empty((kmax + 1,) + x.shape)
    out[0] = 1.0
    if kmax >= 1:
        out[1] = x
    for k in range(2, kmax + 1):
        out[k] = 2.0 * x * out[k - 1] - out[k - 2]
    return out


def cheb_dT(kmax, x):
    """Derivatives T_k'(x) = k U_{k-1}(x); shape (kmax+1,)+x.shape."""
    x = np.asarray(x, dtype=np.float64)
    U = np.empty((kmax + 1,) + x.shape)
    U[0] = 1.0
    if kmax >= 1:
        U[1] = 2.0 * x
    for k in range(2, kmax + 1):
        U[k] = 2.0 * x * U[k - 1] - U[k - 2]
    out = np.zeros((kmax + 1,) + x.shape)
    for k in range(1, kmax + 1):
        out[k] = k * U[k - 1]
    return out


def lagrange(nodes, t):
    """L_b(t) for all b; shape (len(nodes),)+t.shape."""
    t = np.asarray(t, dtype=np.float64)
    m = len(nodes)
    out = np.ones((m,) + t.shape)
    for b in range(m):
        for k in range(m):
            if k != b:
                out[b] = out[b] * (t - nodes[k]) / (nodes[b] - nodes[k])
    return out


def multi_indices(m):
    return np.array([(a, b, c) for a in range(m + 1) for b in range(m + 1 - a)
                     for c in range(m + 1 - a - b)], dtype=np.int64)


def lam(k):
    return np.where(np.asarray(k) == 0, 1.0, 2.0)


def E1d(r, d, m):
    """Eq. exp_coeffs_1d: E[..., k, l](r, d), k <-> source node xi_m, l <-> target xi_n.

    ``d`` may be an array; the result has shape d.shape + (m+1, m+1).
    """
    xi = cheb_nodes(m)
    d = np.asarray(d, dtype=np.float64)
    T = cheb_T(m, xi).T                     # T[n, l] = T_l(xi_n)
    K = np.exp(-((r + xi[:, None] - xi[None, :]) ** 2)[None] / d.reshape(-1, 1, 1))   # [., n, m]
    core = np.einsum("nl,inm,mk->ikl", T, K, T)   # [., k, l] = sum_nm T_l(xi_n) K[n,m] T_k(xi_m)
    lk = lam(np.arange(m + 1))
    out = (lk[:, None] * lk[None, :] / (m + 1) ** 2)[None] * core
    return out.reshape(d.shape + (m + 1, m + 1))


# ------------------------------------------------------------ the oracle FMM

class FMMOracle:
    def __init__(self, tree, m_t, m_x, kind="V", q_reg=4, q_sing=5):
        self.tr = tree
        self.m_t, self.m_x, self.kind = m_t, m_x, kind
        self.q_reg, self.q_sing = q_reg, q_sing
        self.alpha = tree.alpha
        self.mi = multi_indices(m_x)
        self.Nk = len(self.mi)
        self.xt = cheb_nodes(m_t)
        self.xx = cheb_nodes(m_x)
        self.h = (tree.t[-1] - tree.t[0]) / tree.E_t
        P = tree.verts[tree.tri]
        n = np.cross(P[:, 1] - P[:, 0], P[:, 2] - P[:, 0])
        a2 = np.linalg.norm(n, axis=1)
        self.area, self.normal = 0.5 * a2, n / a2[:, None]
        self._ax_cache = {}
        self._op_cache = {}
        self._e1_cache = {}
        self._at_cache = {}
        self._qt_cache = {}
        self._qx_cache = {}
        self._B = None
        # index set of eq. m2l: all (nu, kappa) with |kappa + nu| <= m_x
        deg = self.mi.sum(1)
        pn, pk = np.nonzero(deg[:, None] + deg[None, :] <= m_x)
        self._pn, self._pk = pn, pk

    def _time_key(self, Z, S):
        """What the M2L operator's time dependence sees of a box pair: the
        step offsets and lengths for uniform steps, else the node
        differences (rounded to 2^-40 T)."""
        tr = self.tr
        if tr.uniform:
            return (Z.s0 - S.s0, Z.s1 - Z.s0, S.s1 - S.s0)
        q = lambda x: int(round(x / tr.T * 2.0 ** 40))
        return (q(tr.t[Z.s0] - tr.t[S.s0]), q(tr.t[Z.s1] - tr.t[Z.s0]), q(tr.t[S.s1] - tr.t[S.s0]))

    # ---------------- temporal tables
    def tnodes(self, b):
        ta, tb = self.tr.interval(b)
        return 0.5 * (ta + tb) + 0.5 * (tb - ta) * self.xt

    def A_t(self, b):
        """A_t[j, a] = int_{step j} L_{J,a}(tau) dtau for the steps of box b."""
        key = (b.level, b.k)
        if key in self._at_cache:
            return self._at_cache[key]
        g, w = gauss_legendre01(self.m_t // 2 + 2)
        nodes = self.tnodes(b)
        rows = []
        for j in range(b.s0, b.s1):
            t0, t1 = self.tr.t[j], self.tr.t[j + 1]
            tau = t0 + (t1 - t0) * g
            rows.append(lagrange(nodes, tau) @ (w * (t1 - t0)))
        self._at_cache[key] = np.array(rows)
        return self._at_cache[key]

    # ---------------- spatial tables
    def _ref_coords(self, b, y):
        lo = self.tr.box_lower(b)
        H = self.tr.hx_padded(b.level)
        return (y - lo[None, :]) / H - 1.0, H

    def A_x(self, b, kind=None):
        """A_x[i, kappa] = int_{gamma_i} T_{Y,kappa} (V) or alpha n.grad T (K)."""
        kind = kind or self.kind
        key = (b.level, b.ix, kind)
        if key in self._ax_cache:
            return self._ax_cache[key]
        s, t, w = triangle_rule(self.m_x // 2 + 2)
        P = self.tr.verts[self.tr.tri[b.tris]]
        y = (P[:, 0, None, :] + s[None, :, None] * (P[:, 1] - P[:, 0])[:, None, :]
             + t[None, :, None] * (P[:, 2] - P[:, 1])[:, None, :])          # (n, q, 3)
        yh, H = self._ref_coords(b, y.reshape(-1, 3))
        Tj = [cheb_T(self.m_x, yh[:, j]) for j in range(3)]                 # (m+1, nq)
        mi = self.mi
        if kind == "V":
            vals = Tj[0][mi[:, 0]] * Tj[1][mi[:, 1]] * Tj[2][mi[:, 2]]      # (Nk, nq)
        else:
            dT = [cheb_dT(self.m_x, yh[:, j]) / H for j in range(3)]
            nrm = np.repeat(self.normal[b.tris], len(w), axis=0)           # (nq, 3)
            vals = (nrm[:, 0] * dT[0][mi[:, 0]] * Tj[1][mi[:, 1]] * Tj[2][mi[:, 2]]
                    + nrm[:, 1] * Tj[0][mi[:, 0]] * dT[1][mi[:, 1]] * Tj[2][mi[:, 2]]
                    + nrm[:, 2] * Tj[0][mi[:, 0]] * Tj[1][mi[:, 1]] * dT[2][mi[:, 2]])
            vals = self.alpha * vals
        vals = vals.reshape(self.Nk, len(b.tris), len(w))
        A = np.einsum("kiq,q,i->ik", vals, w, 2.0 * self.area[b.tris])
        self._ax_cache[key] = A
        return A

    # ---------------- re-expansion coefficients
    def qt(self, c, p):
        """q^(t)[a_c, a_p] = L_{I_p, a_p}(xi_{I_c, a_c}) (eq. temp_m2m)."""
        key = (c.level, c.k)
        if key not in self._qt_cache:
            self._qt_cache[key] = lagrange(self.tnodes(p), self.tnodes(c)).T
        return self._qt_cache[key]

    def qx(self, c, p):
        """q^(x)[kappa, nu] over multi-indices, kappa <= nu componentwise (eq. st_m2m)."""
        key = (c.level, c.ix)
        if key in self._qx_cache:
            return self._qx_cache[key]
        m = self.m_x
        lc, Hc = self.tr.box_lower(c), self.tr.hx_padded(c.level)
        lp, Hp = self.tr.box_lower(p), self.tr.hx_padded(p.level)
        Tn = cheb_T(m, self.xx)                                # T_kappa(xi_n): (m+1, n)
        Q = []
        for j in range(3):
            yc = lc[j] + Hc * (1.0 + self.xx)                  # xi_{X_c, n}
            yp = (yc - lp[j]) / Hp - 1.0
            Tp = cheb_T(m, yp)                                 # T_nu(phi_p^-1(.)), (m+1, n)
            Qj = (lam(np.arange(m + 1))[:, None] / (m + 1)) * (Tn @ Tp.T)   # [kappa, nu]
            Q.append(Qj)
        mi = self.mi
        full = Q[0][mi[:, 0][:, None], mi[:, 0][None, :]] * Q[1][mi[:, 1][:, None], mi[:, 1][None, :]] \
            * Q[2][mi[:, 2][:, None], mi[:, 2][None, :]]
        mask = np.all(mi[:, None, :] <= mi[None, :, :], axis=2)
        self._qx_cache[key] = np.where(mask, full, 0.0)
        return self._qx_cache[key]

    # ---------------- M2L operator
    def m2l_operator(self, Z, S):
        """Op[b, nu, a, kappa] of eq. m2l for target box Z and source box S."""
        tr = self.tr
        key = (Z.level, tuple(np.subtract(Z.ix, S.ix))) + self._time_key(Z, S)
        if key in self._op_cache:
            return self._op_cache[key]
        H = tr.hx_padded(Z.level)
        r = (tr.box_lower(Z) - tr.box_lower(S)) / H
        dt = self.tnodes(Z)[None, :] - self.tnodes(S)[:, None]          # [a, b]
        C = (4.0 * np.pi * self.alpha * dt) ** -1.5
        dab = 4.0 * self.alpha * dt / (H * H)
        m = self.m_x
        nt = self.m_t + 1
        E = np.stack([E1d(r[j], dab, m) for j in range(3)])      # [j, a, b, kappa_j, nu_j]
        mi = self.mi
        K1, N1 = mi[:, 0][None, :], mi[:, 0][:, None]                   # rows nu, cols kappa
        K2, N2 = mi[:, 1][None, :], mi[:, 1][:, None]
        K3, N3 = mi[:, 2][None, :], mi[:, 2][:, None]
        mask = (mi.sum(1)[:, None] + mi.sum(1)[None, :]) <= m             # |kappa + nu| <= m_x
        op = np.empty((nt, self.Nk, nt, self.Nk))
        for a in range(nt):
            for b in range(nt):
                blk = C[a, b] * E[0, a, b][K1, N1] * E[1, a, b][K2, N2] * E[2, a, b][K3, N3]
                op[b, :, a, :] = np.where(mask, blk, 0.0)
        self._op_cache[key] = op
        return op

    # ---------------- upward pass
    def moments(self, w):
        tr = self.tr
        W = w.reshape(tr.E_t, tr.E_x)
        mu = {}
        for b in tr.leaves:
            Wb = W[b.s0:b.s1][:, b.tris]
            mu[b.id] = self.A_t(b).T @ Wb @ self.A_x(b)
        for l in range(tr.depth - 1, 1, -1):
            for p in tr.levels[l]:
                if p.leaf:
                    continue
                acc = np.zeros((self.m_t + 1, self.Nk))
                for c in p.children:
                    acc += self.qt(c, p).T @ mu[c.id] @ self.qx(c, p)
                mu[p.id] = acc
        return mu

    def _e1_tables(self, Z, S):
        """Per axis j: E_{kappa_j, nu_j}(r_j, d_ab) for all (a, b), and C_ab (eq. exp_coeffs_3d)."""
        tr = self.tr
        H = tr.hx_padded(Z.level)
        r = (tr.box_lower(Z) - tr.box_lower(S)) / H
        tkey = (Z.level,) + self._time_key(Z, S)
        dt = self.tnodes(Z)[None, :] - self.tnodes(S)[:, None]          # [a, b]
        C = (4.0 * np.pi * self.alpha * dt) ** -1.5
        dab = 4.0 * self.alpha * dt / (H * H)
        E = []
        for j in range(3):
            key = tkey + (int(Z.ix[j]) - int(S.ix[j]),)
            if key not in self._e1_cache:
                self._e1_cache[key] = E1d(r[j], dab, self.m_x)          # [a, b, kappa_j, nu_j]
            E.append(self._e1_cache[key])
        return C, E

    def m2l(self, Z, mu):
        """lambda_{b,nu}(Z) = sum_S sum_a sum_{|kappa+nu|<=m_x} E_{a,kappa,b,nu} mu_{a,kappa}(S) (eq. m2l)."""
        lam_ = np.zeros((self.m_t + 1, self.Nk))
        pn, pk = self._pn, self._pk
        mi = self.mi
        for S in self.tr.interaction(Z):
            C, E = self._e1_tables(Z, S)
            # coefficient of every admissible (a, b, nu, kappa) of the truncated sum
            coef = (C[:, :, None] * E[0][:, :, mi[pk, 0], mi[pn, 0]] * E[1][:, :, mi[pk, 1], mi[pn, 1]]
                    * E[2][:, :, mi[pk, 2], mi[pn, 2]])                   # [a, b, pair]
            contrib = np.einsum("abp,ap->bp", coef, mu[S.id][:, pk])     # [b, pair]
            for b in range(self.m_t + 1):
                lam_[b] += np.bincount(pn, weights=contrib[b], minlength=self.Nk)
        return lam_

    def l2l(self, c, p, lam_p):
        return self.qt(c, p) @ lam_p @ self.qx(c, p).T

    def l2t(self, b, lam_b):
        """f at the elements of leaf b (time-major, (steps, tris))."""
        return self.A_t(b) @ lam_b @ self.A_x(b, "V").T

    # ---------------- nearfield entries
    def set_toeplitz_blocks(self, B):
        """Use precomputed B[d][k_x, j_x] (exact reuse of identical integrals)."""
        self._B = B

    def entries(self, kx, jx, dmax):
        if self._B is not None:
            return self._B[:dmax + 1][:, kx, jx].T
        return panel_integrals(self.tr.verts, self.tr.tri, kx, jx, dmax, self.h, self.alpha,
                               self.kind, self.q_reg, self.q_sing)

    def entries_steps(self, kx, jx, pairs):
        """Entries of the panel pairs (kx[i], jx[i]) for the step pairs
        (kt, jt), kt >= jt, of a time grid with steps of any length:
        (len(kx), len(pairs))."""
        return panel_integrals(self.tr.verts, self.tr.tri, kx, jx, 0, 0.0, self.alpha, self.kind, self.q_reg,
                               self.q_sing, tnodes=self.tr.t, pairs=pairs)

    def near_block(self, Z, S):
        """Dense causal block V|_{Z x S} in time-major element order."""
        kt = np.arange(Z.s0, Z.s1)
        jt = np.arange(S.s0, S.s1)
        if not self.tr.uniform:
            pairs = [(a, b) for a in kt for b in jt if b <= a]
            kx = np.repeat(Z.tris, len(S.tris))
            jx = np.tile(S.tris, len(Z.tris))
            blk = np.zeros((len(kt), len(Z.tris), len(jt), len(S.tris)))
            if pairs:
                ent = self.entries_steps(kx, jx, pairs).reshape(len(Z.tris), len(S.tris), len(pairs))
                for i, (a, b) in enumerate(pairs):
                    blk[a - Z.s0, :, b - S.s0, :] = ent[:, :, i]
            return blk.reshape(len(kt) * len(Z.tris), len(jt) * len(S.tris))
        D = kt[:, None] - jt[None, :]
        dmax = int(max(D.max(), 0))
        kx = np.repeat(Z.tris, len(S.tris))
        jx = np.tile(S.tris, len(Z.tris))
        ent = self.entries(kx, jx, dmax).reshape(len(Z.tris), len(S.tris), dmax + 1)
        Dc = np.clip(D, 0, None)
        blk = ent[:, :, Dc]                                      # (nZx, nSx, nkt, njt)
        blk = np.where((D >= 0)[None, None], blk, 0.0)
        return blk.transpose(2, 0, 3, 1).reshape(len(kt) * len(Z.tris), len(jt) * len(S.tris))

    # ---------------- full apply (Algorithm 2)
    def apply(self, w, far=True, near=True):
        tr = self.tr
        f = np.zeros(tr.E_t * tr.E_x)
        if far:
            f += self.farfield(w)
        if near:
            f += self.nearfield(w)
        return f

    def farfield(self, w):
        tr = self.tr
        mu = self.moments(w)
        lam_ = {}
        for l in range(2, tr.depth + 1):
            for Z in tr.levels[l]:
                lam_[Z.id] = self.m2l(Z, mu)
        for l in range(3, tr.depth + 1):
            for Z in tr.levels[l]:
                p = Z.parent
                if p.id in lam_:
                    lam_[Z.id] = lam_[Z.id] + self.l2l(Z, p, lam_[p.id])
        f = np.zeros(tr.E_t * tr.E_x)
        for b in tr.leaves:
            if b.id in lam_:
                f[tr.elements(b)] += self.l2t(b, lam_[b.id]).ravel()
        return f

    def near_contrib(self, Z, S, w):
        """Nearfield block of (Z, S) times the source values (rows of Z)."""
        return self.near_block(Z, S) @ w[self.tr.elements(S)]

    def nearfield(self, w):
        tr = self.tr
        f = np.zeros(tr.E_t * tr.E_x)
        memo = {}
        for Z in tr.leaves:
            rows = tr.elements(Z)
            for S in tr.nearfield(Z, memo):
                f[rows] += self.near_contrib(Z, S, w)
        return f

    def near_row(self, kt, kx, srcs, w):
        """Nearfield part of row (k_t, k_x): every source element (j_t <= k_t)
        of the source boxes srcs."""
        tr = self.tr
        dmax = kt - min(S.s0 for S in srcs)
        jx_all = np.unique(np.concatenate([S.tris for S in srcs]))
        if tr.uniform:
            ent = self.entries(np.full(len(jx_all), kx), jx_all, dmax)     # (n, dmax+1)
        else:   # column kt - jt holds the step pair (kt, jt)
            ent = self.entries_steps(np.full(len(jx_all), kx), jx_all, [(kt, kt - d) for d in range(dmax + 1)])
        where = {int(j): i for i, j in enumerate(jx_all)}
        tot = 0.0
        for S in srcs:
            idx = np.array([where[int(j)] for j in S.tris])
            for jt in range(S.s0, min(S.s1, kt + 1)):
                tot += ent[idx, kt - jt] @ w[jt * tr.E_x + S.tris]
        return tot

    # ---------------- row-sampled apply (for meshes too large for a full apply)
    def apply_rows(self, w, rows, mu=None):
        """f[rows] of the pFMM product, computing only what those rows need.

        The upward pass is complete; M2L, L2L and L2T follow the chain of
        ancestors of each sampled row's leaf; the nearfield row is summed
        directly.  Returns (values, mu) so the moments can be reused.
        """
        tr = self.tr
        if mu is None:
            mu = self.moments(w)
        leaf_of = {}
        for b in tr.leaves:
            for e in tr.elements(b):
                leaf_of[int(e)] = b
        memo = {}
        lam_memo = {}
        out = np.zeros(len(rows))
        for i, r in enumerate(rows):
            r = int(r)
            Z = leaf_of[r]
            kt, kx = divmod(r, tr.E_x)
            # far field through the ancestor chain
            chain = [b for b in tr.ancestors(Z) if b.level >= 2]
            lam_ = None
            for b in chain:
                if b.id not in lam_memo:
                    here = self.m2l(b, mu)
                    if lam_ is not None:
                        here = here + self.l2l(b, b.parent, lam_)
                    lam_memo[b.id] = here
                lam_ = lam_memo[b.id]
            if lam_ is not None:
                At = self.A_t(Z)[kt - Z.s0]
                Ax = self.A_x(Z, "V")[list(Z.tris).index(kx)]
                out[i] += At @ lam_ @ Ax
            # nearfield row: every source element (j_t <= k_t) of the leaf's nearfield boxes
            srcs = [S for S in tr.nearfield(Z, memo) if S.s0 <= kt]
            if srcs:
                out[i] += self.near_row(kt, kx, srcs, w)
        return out, mu

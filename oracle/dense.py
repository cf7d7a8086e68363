"""Dense p0 x p0 Galerkin matrices V_h and K_h for tiny meshes (oracle, test-only).

Section 2 (matrix V_h): for uniform steps t_j = j h and 0-based step indices,
    V_h[k_t E_x + k_x, j_t E_x + j_x]
      = int_{step k_t} int_{gamma_kx} int_{step j_t} int_{gamma_jx} G dsy dtau dsx dt
      = B_V[k_t - j_t][k_x, j_x]   for k_t >= j_t, and 0 otherwise
(block lower triangular by causality, block Toeplitz for uniform steps).
K_h is the p0 x p0 double-layer matrix (kernel alpha dG/dn_y) built the same
way; coplanar panel pairs are exactly zero because (x - y).n_y vanishes.

The space integrals use the rules of ``quadrature`` and the time integrals the
closed forms of ``timeint``; touching pairs switch to the singular rules for
time offsets 0 and 1.

Parity: pinned by the structural facts above (causality, Toeplitz, symmetry
of V_h blocks), by the double-layer identity (1/2 M_h + K_h) 1 = the volume
potential of the constant 1, and by V_h 1 against a semi-analytic face-wise
formula (tests/test_oracle_dense.py).
"""
import numpy as np

from . import quadrature as Q
from .timeint import time_factors_all, time_factor, time_factor_steps, needs_singular_rule


class _TimeSpec:
    """The time integrals a set of entries needs: offsets d = 0..dmax of
    uniform steps h (Toeplitz form), or explicit step pairs (kt, jt) of a
    time grid with steps of any length."""

    def __init__(self, dmax, h, tnodes=None, pairs=None):
        self.tn = None if tnodes is None else np.asarray(tnodes, dtype=np.float64)
        self.pairs = None if pairs is None else [(int(a), int(b)) for a, b in pairs]
        self.dmax, self.h = dmax, h
        self.n = len(self.pairs) if self.pairs is not None else dmax + 1

    def offset(self, i):
        return self.pairs[i][0] - self.pairs[i][1] if self.pairs is not None else i

    def factor(self, r, i, alpha, kind):
        if self.pairs is None:
            return time_factor(r, i, self.h, alpha, kind)
        kt, jt = self.pairs[i]
        return time_factor_steps(r, self.tn[kt], self.tn[kt + 1], self.tn[jt], self.tn[jt + 1], kt - jt, alpha, kind)

    def factors_all(self, r, alpha, kind):
        if self.pairs is None:
            return time_factors_all(r, self.dmax, self.h, alpha, kind)
        return np.stack([self.factor(r, i, alpha, kind) for i in range(self.n)])


def geometry(verts, tris):
    P = verts[tris]
    n = np.cross(P[:, 1] - P[:, 0], P[:, 2] - P[:, 0])
    a2 = np.linalg.norm(n, axis=1)
    return 0.5 * a2, n / a2[:, None], P.mean(axis=1)


def coplanar(verts, tris, k, j):
    """Same-plane test used to zero double-layer entries exactly."""
    _, nrm, cen = geometry(verts, tris[[k, j]])
    P = verts[tris[[k, j]]]
    L = max(np.linalg.norm(P[0] - P[0][[1, 2, 0]], axis=1).max(),
            np.linalg.norm(P[1] - P[1][[1, 2, 0]], axis=1).max())
    return (abs(1.0 - abs(np.dot(nrm[0], nrm[1]))) < 1e-10
            and abs(np.dot(cen[0] - cen[1], nrm[1])) < 1e-10 * L)


def _integrand_sum(dvec, W, nrm_j, ilist, ts, alpha, kind):
    r = np.linalg.norm(dvec, axis=1)
    vals = []
    for i in ilist:
        tf = ts.factor(r, i, alpha, kind)
        if kind == "K":
            tf = tf * (dvec @ nrm_j)
        vals.append(np.sum(W * tf))
    return np.array(vals)


def panel_integrals(verts, tris, ks, js, dmax, h, alpha, kind="V", q_reg=4, q_sing=5, tnodes=None, pairs=None):
    """Entries B[d][k, j] for the listed panel pairs and d = 0..dmax
    (uniform steps h); or, with `pairs` a list of step pairs (kt, jt),
    kt >= jt, of the time grid `tnodes` (steps of any length), the entries
    of those step pairs.

    Returns an array of shape (len(ks), dmax + 1) or (len(ks), len(pairs)).
    """
    ts = _TimeSpec(dmax, h, tnodes, pairs)
    ks = np.asarray(ks, dtype=np.int64)
    js = np.asarray(js, dtype=np.int64)
    out = np.zeros((len(ks), ts.n))
    area, nrm, cen = geometry(verts, tris)
    nshared = np.array([Q.classify(tris[k], tris[j]) for k, j in zip(ks, js)])
    copl = np.zeros(len(ks), dtype=bool)
    if kind == "K":
        copl = np.array([coplanar(verts, tris, k, j) for k, j in zip(ks, js)])

    # regular rule (non-touching pairs for all d; touching pairs for d >= 2)
    s, t, w = Q.triangle_rule(q_reg)
    P = verts[tris]
    xq = (P[:, 0, None, :] + s[None, :, None] * (P[:, 1] - P[:, 0])[:, None, :]
          + t[None, :, None] * (P[:, 2] - P[:, 1])[:, None, :])          # (nt, q2, 3)
    wq = (2.0 * area)[:, None] * w[None, :]                               # (nt, q2)
    reg = np.nonzero((nshared < 3) & ~copl)[0]
    chunk = 256
    for c0 in range(0, len(reg), chunk):
        idx = reg[c0:c0 + chunk]
        k, j = ks[idx], js[idx]
        dv = xq[k][:, :, None, :] - xq[j][:, None, :, :]                  # (c, q2, q2, 3)
        r = np.linalg.norm(dv, axis=-1)
        W = wq[k][:, :, None] * wq[j][:, None, :]
        tf = ts.factors_all(r, alpha, kind)                              # (D, c, q2, q2)
        if kind == "K":
            tf = tf * np.einsum("cpqx,cx->cpq", dv, nrm[j])[None]
        vals = np.einsum("dcpq,cpq->cd", tf, W)
        touching = nshared[idx] > 0
        for it in range(ts.n):
            if needs_singular_rule(ts.offset(it)):
                vals[touching, it] = 0.0   # replaced below
        out[idx] = vals

    # touching pairs: singular rules (identical for all d, edge/vertex for d<=1)
    for i in np.nonzero((nshared > 0) & ~copl)[0]:
        k, j = int(ks[i]), int(js[i])
        if nshared[i] == 3:
            il = list(range(ts.n))
        else:
            il = [it for it in range(ts.n) if needs_singular_rule(ts.offset(it))]
        if not il:
            continue
        dvec, W = Q.pair_rule(verts, tris, k, j, True, q_reg, q_sing)
        out[i, il] = _integrand_sum(dvec, W, nrm[j], il, ts, alpha, kind)
    return out


def toeplitz_blocks(verts, tris, n_steps, h, alpha, kind="V", q_reg=4, q_sing=5):
    """B[d] (E_x x E_x) for d = 0..n_steps-1 over all panel pairs."""
    nt = len(tris)
    kk, jj = np.meshgrid(np.arange(nt), np.arange(nt), indexing="ij")
    vals = panel_integrals(verts, tris, kk.ravel(), jj.ravel(), n_steps - 1, h, alpha,
                           kind, q_reg, q_sing)
    return vals.T.reshape(n_steps, nt, nt)


def dense_matrix(verts, tris, n_steps, h, alpha, kind="V", q_reg=4, q_sing=5, B=None):
    """Full V_h or K_h (N x N, natural time-major order) for tiny meshes."""
    nt = len(tris)
    if B is None:
        B = toeplitz_blocks(verts, tris, n_steps, h, alpha, kind, q_reg, q_sing)
    N = n_steps * nt
    A = np.zeros((N, N))
    for kt in range(n_steps):
        for jt in range(kt + 1):
            A[kt * nt:(kt + 1) * nt, jt * nt:(jt + 1) * nt] = B[kt - jt]
    return A


def dense_matrix_steps(verts, tris, tnodes, alpha, kind="V", q_reg=4, q_sing=5):
    """Full V_h or K_h (natural time-major order) on a time grid whose steps
    may differ in length (block (kt, jt) from the absolute step pair; zero
    for jt > kt)."""
    tn = np.asarray(tnodes, dtype=np.float64)
    E_t, nt = len(tn) - 1, len(tris)
    pairs = [(kt, jt) for kt in range(E_t) for jt in range(kt + 1)]
    kk, jj = np.meshgrid(np.arange(nt), np.arange(nt), indexing="ij")
    vals = panel_integrals(verts, tris, kk.ravel(), jj.ravel(), 0, 0.0, alpha, kind, q_reg, q_sing,
                           tnodes=tn, pairs=pairs)                      # (nt*nt, n_pairs)
    A = np.zeros((E_t * nt, E_t * nt))
    for i, (kt, jt) in enumerate(pairs):
        A[kt * nt:(kt + 1) * nt, jt * nt:(jt + 1) * nt] = vals[:, i].reshape(nt, nt)
    return A


def mass_diag_steps(verts, tris, tnodes):
    """Diagonal p0 x p0 mass matrix |gamma_k| (t_{j+1} - t_j) (natural order, length E_t E_x)."""
    area = geometry(verts, tris)[0]
    h = np.diff(np.asarray(tnodes, dtype=np.float64))
    return (h[:, None] * area[None, :]).ravel()


def mass_diag(verts, tris, n_steps, h):
    """Diagonal p0 x p0 mass matrix M_h = |gamma_k| h (natural order)."""
    area = geometry(verts, tris)[0]
    return np.tile(area * h, n_steps)

"""Representation formula at interior points (oracle, test-only).

Section 2: for zero initial data the solution of the heat equation in the
space-time cylinder is recovered from its Cauchy data on the lateral surface,

    u(x, t) = (V~ w)(x, t) - (W u)(x, t),   x inside the domain, 0 < t,

with the single-layer potential V~ (kernel G) of the Neumann trace
w = alpha du/dn and the double-layer potential W (kernel alpha dG/dn_y) of
the Dirichlet trace.  For piecewise-constant data in space and time
(w[j_t, j_x] on step j_t and triangle j_x) the time integral over a step is
closed-form: with G1 the s-antiderivative of G vanishing at s = 0,

    G1(r, s) = erfc(z) / (4 pi alpha r),          z = r / (2 sqrt(alpha s)),
    int_{t_j}^{min(t_{j+1}, t)} G(r, t - tau) dtau = G1(r, t - t_j) - G1(r, max(t - t_{j+1}, 0)),

and for the double layer alpha dG/dn_y = ((x - y).n_y / (2 s)) G, whose
antiderivative is K1 = -(alpha / r) dG1/dr,

    K1(r, s) = [erfc(z) + r exp(-z^2) / sqrt(pi alpha s)] / (4 pi r^3).

Space integrals use the collapsed Gauss rule of `quadrature.triangle_rule`
with q points per direction (the targets are interior points, so the
integrand is smooth; its accuracy falls as a target approaches the surface).
Pinned by tests: G1 and K1 against brute-force quadrature of G and G / (2 s)
in time; V~ applied to the constant density on the cube surface against the
face-wise erf formula integrated in time; W applied to the constant against
the volume heat potential of the constant minus one (the double-layer
identity at interior points).
"""
import numpy as np
from scipy.special import erfc

from .quadrature import triangle_rule


def G1(r, s, alpha):
    """First s-antiderivative of G (r > 0), zero for s <= 0."""
    r = np.asarray(r, dtype=np.float64)
    s = np.asarray(s, dtype=np.float64)
    shape = np.broadcast(r, s).shape
    rb = np.broadcast_to(r, shape)
    sb = np.broadcast_to(s, shape)
    out = np.zeros(shape)
    pos = sb > 0
    z = rb[pos] / (2.0 * np.sqrt(alpha * sb[pos]))
    out[pos] = erfc(z) / (4.0 * np.pi * alpha * rb[pos])
    return out


def K1(r, s, alpha):
    """First s-antiderivative of G / (2 s) (r > 0), zero for s <= 0."""
    r = np.asarray(r, dtype=np.float64)
    s = np.asarray(s, dtype=np.float64)
    shape = np.broadcast(r, s).shape
    rb = np.broadcast_to(r, shape)
    sb = np.broadcast_to(s, shape)
    out = np.zeros(shape)
    pos = sb > 0
    rr, ss = rb[pos], sb[pos]
    z = rr / (2.0 * np.sqrt(alpha * ss))
    out[pos] = (erfc(z) + rr * np.exp(-z * z) / np.sqrt(np.pi * alpha * ss)) / (4.0 * np.pi * rr ** 3)
    return out


def _surface_points(verts, tris, q):
    s, t, w = triangle_rule(q)
    P = verts[tris]
    n = np.cross(P[:, 1] - P[:, 0], P[:, 2] - P[:, 0])
    a2 = np.linalg.norm(n, axis=1)
    y = (P[:, 0, None, :] + s[None, :, None] * (P[:, 1] - P[:, 0])[:, None, :]
         + t[None, :, None] * (P[:, 2] - P[:, 1])[:, None, :])             # (E_x, q^2, 3)
    wq = a2[:, None] * w[None, :]                                            # 2 |gamma| w
    return y, wq, n / a2[:, None]


def potentials(verts, tris, time_nodes, w, u, points, times, alpha=1.0, q=4):
    """(V~ w)(x_i, t_i) and (W u)(x_i, t_i) for p0 x p0 densities w, u
    (natural order: index j_t E_x + j_x; either may be None) at the points
    x_i (M x 3) and times t_i (M,).  Returns two arrays of length M."""
    verts = np.asarray(verts, dtype=np.float64)
    tris = np.asarray(tris, dtype=np.int64)
    tn = np.asarray(time_nodes, dtype=np.float64)
    E_t, E_x = len(tn) - 1, len(tris)
    y, wq, nrm = _surface_points(verts, tris, q)
    W = None if w is None else np.asarray(w, dtype=np.float64).reshape(E_t, E_x)
    U = None if u is None else np.asarray(u, dtype=np.float64).reshape(E_t, E_x)
    pts = np.asarray(points, dtype=np.float64)
    out_v = np.zeros(len(pts))
    out_w = np.zeros(len(pts))
    for i, (x, t) in enumerate(zip(pts, np.asarray(times, dtype=np.float64))):
        d = x[None, None, :] - y                                             # (E_x, q^2, 3)
        r = np.linalg.norm(d, axis=-1)
        dn = np.einsum("epk,ek->ep", d, nrm)                                 # (x - y) . n_y
        for j in range(E_t):
            if tn[j] >= t:
                break
            s0, s1 = t - tn[j], max(t - tn[j + 1], 0.0)
            if W is not None:
                tv = G1(r, s0, alpha) - G1(r, s1, alpha)                     # (E_x, q^2)
                out_v[i] += np.sum(W[j] * np.sum(wq * tv, axis=1))
            if U is not None:
                tk = dn * (K1(r, s0, alpha) - K1(r, s1, alpha))
                out_w[i] += np.sum(U[j] * np.sum(wq * tk, axis=1))
    return out_v, out_w


def representation(verts, tris, time_nodes, w, g, points, times, alpha=1.0, q=4):
    """u(x_i, t_i) = (V~ w)(x_i, t_i) - (W g)(x_i, t_i) (Section 2)."""
    v, dl = potentials(verts, tris, time_nodes, w, g, points, times, alpha, q)
    return v - dl

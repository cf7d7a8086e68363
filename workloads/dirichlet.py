"""Dirichlet data of the paper's model problem, projected onto p0 x p0.

Section 5 (eq. dirdata) prescribes u(x, t) = G(x - y*, t) on the lateral
boundary, the heat fundamental solution with a source point y* outside the
domain.  A source time t* shifts it to G(x - y*, t - t*).  The system of
Section 2 needs the L2 projection g_h of u; in the p0 x p0 setting that is
the element mean over every space-time element sigma = gamma x (t_{j-1}, t_j).

The means are computed with a collapsed tensor Gauss-Legendre rule on each
triangle (q x q points) times q_t Gauss-Legendre points per step.  This is
input preparation (a datum and its projection), not part of the FMM.

The manufactured Neumann datum alpha du/dn (the exact solution w of the
boundary integral equation when u(., 0) = 0 inside the domain) is projected
the same way, for convergence tests.
"""
import numpy as np


def _heat(r2, s, alpha):
    """G for squared distance r2 and time lag s (0 where s <= 0)."""
    s = np.asarray(s, dtype=np.float64)
    out = np.zeros(np.broadcast(r2, s).shape)
    pos = np.broadcast_to(s > 0, out.shape)
    sp = np.where(s > 0, s, 1.0)
    val = (4.0 * np.pi * alpha * sp) ** -1.5 * np.exp(-r2 / (4.0 * alpha * sp))
    out[pos] = np.broadcast_to(val, out.shape)[pos]
    return out


def _points(verts, tris, time_nodes, q, q_t):
    """Quadrature points and weights (normalised to element means)."""
    g, gw = np.polynomial.legendre.leggauss(q)
    g, gw = 0.5 * (g + 1.0), 0.5 * gw
    # collapsed rule on the unit triangle: (s, t s), s, t in (0, 1), Jacobian s
    s = np.repeat(g, q)
    t = np.tile(g, q)
    w_tri = np.repeat(gw, q) * np.tile(gw, q) * s * 2.0      # sums to 1
    P = verts[tris]                                           # (E_x, 3, 3)
    X = (P[:, None, 0] + s[None, :, None] * (P[:, None, 1] - P[:, None, 0])
         + (s * t)[None, :, None] * (P[:, None, 2] - P[:, None, 1]))
    gt, gtw = np.polynomial.legendre.leggauss(q_t)
    gt, gtw = 0.5 * (gt + 1.0), 0.5 * gtw
    t0, t1 = time_nodes[:-1], time_nodes[1:]
    T = t0[:, None] + (t1 - t0)[:, None] * gt[None, :]       # (E_t, q_t)
    return X, w_tri, T, gtw


def _time_chunks(n_steps, per_step, cap=8_000_000):
    """Step ranges holding at most `cap` quadrature values each."""
    step = max(1, cap // max(per_step, 1))
    return [(j, min(j + step, n_steps)) for j in range(0, n_steps, step)]


def _normals(verts, tris):
    P = verts[tris]
    n = np.cross(P[:, 1] - P[:, 0], P[:, 2] - P[:, 0])
    return n / np.linalg.norm(n, axis=1)[:, None]


def project_source_datum(verts, tris, time_nodes, y_star, t_star=0.0, alpha=1.0, q=4, q_t=4):
    """Element means of G(x - y*, t - t*) (natural time-major order, length E_t E_x)."""
    X, w_tri, T, gtw = _points(verts, tris, time_nodes, q, q_t)
    r2 = ((X - np.asarray(y_star, dtype=np.float64)) ** 2).sum(-1)          # (E_x, nq)
    out = np.empty((len(T), len(tris)))
    for j0, j1 in _time_chunks(len(T), r2.size * q_t):
        vals = _heat(r2[None, :, :, None], (T[j0:j1] - t_star)[:, None, None, :], alpha)
        out[j0:j1] = vals.reshape(j1 - j0, len(tris), -1) @ np.kron(w_tri, gtw)
    return out.ravel()


def project_source_flux(verts, tris, time_nodes, y_star, t_star=0.0, alpha=1.0, q=4, q_t=4):
    """Element means of alpha dG(x - y*, t - t*)/dn_x = -(x - y*).n / (2 (t - t*)) G."""
    X, w_tri, T, gtw = _points(verts, tris, time_nodes, q, q_t)
    d = X - np.asarray(y_star, dtype=np.float64)
    r2 = (d ** 2).sum(-1)
    dn = np.einsum("xqk,xk->xq", d, _normals(verts, tris))
    out = np.empty((len(T), len(tris)))
    for j0, j1 in _time_chunks(len(T), r2.size * q_t):
        s = (T[j0:j1] - t_star)[:, None, None, :]
        vals = _heat(r2[None, :, :, None], s, alpha) * (-dn[None, :, :, None]) / (2.0 * np.where(s > 0, s, 1.0))
        out[j0:j1] = vals.reshape(j1 - j0, len(tris), -1) @ np.kron(w_tri, gtw)
    return out.ravel()


def project_source_datum_p1(verts, tris, time_nodes, y_star, t_star=0.0, alpha=1.0, q=4, q_t=4):
    """L2 projection of G(x - y*, t - t*) onto functions piecewise linear and
    continuous in space (nodal hat functions phi_v) and piecewise constant in
    time: per step, the p1 mass system sum_w (phi_v, phi_w) g_w = the step
    mean of (G, phi_v).  Returns g per (step, vertex), time-major (length
    E_t n_v)."""
    import scipy.sparse as sp
    import scipy.sparse.linalg as spla
    X, w_tri, T, gtw = _points(verts, tris, time_nodes, q, q_t)
    nq = len(w_tri)
    s = np.repeat(np.polynomial.legendre.leggauss(q)[0] * 0.5 + 0.5, q)
    t = s * np.tile(np.polynomial.legendre.leggauss(q)[0] * 0.5 + 0.5, q)
    lam = np.stack([1.0 - s, s - t, t])                      # barycentric coordinates of the points
    P = verts[tris]
    area = 0.5 * np.linalg.norm(np.cross(P[:, 1] - P[:, 0], P[:, 2] - P[:, 0]), axis=1)
    nv, nt = len(verts), len(tris)
    rows = np.repeat(tris, 3, axis=1).ravel()
    cols = np.tile(tris, (1, 3)).ravel()
    loc = np.array([[2.0, 1.0, 1.0], [1.0, 2.0, 1.0], [1.0, 1.0, 2.0]]) / 12.0
    M = sp.csr_matrix(((area[:, None, None] * loc[None]).ravel(), (rows, cols)), shape=(nv, nv))
    r2 = ((X - np.asarray(y_star, dtype=np.float64)) ** 2).sum(-1)
    out = np.empty((len(T), nv))
    lu = spla.splu(M.tocsc())
    for j0, j1 in _time_chunks(len(T), r2.size * q_t):
        vals = _heat(r2[None, :, :, None], (T[j0:j1] - t_star)[:, None, None, :], alpha) @ gtw   # (steps, E_x, nq)
        # (G, phi_v) per step mean: sum over the triangles of |gamma| sum_q w_q G lambda_i
        rhs = np.zeros((j1 - j0, nv))
        for i in range(3):
            contrib = (vals * (w_tri * lam[i])[None, None, :]).sum(-1) * area[None, :]          # (steps, E_x)
            for k in range(j1 - j0):
                np.add.at(rhs[k], tris[:, i], contrib[k])
        for k in range(j1 - j0):
            out[j0 + k] = lu.solve(rhs[k])
    return out.ravel()

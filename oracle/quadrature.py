"""Quadrature for the p0 x p0 Galerkin panel integrals (oracle, test-only).

The paper assembles the inadmissible (nearfield) blocks with time integrals
done analytically and space integrals done numerically, deferring the details
to a companion paper (Section 3.4, text after eq. eval_sl_nf_block).  The
spatial rules below are this project's reading of that step:

* regular panel pairs: tensor product of a collapsed (Duffy) Gauss-Legendre
  rule with q_reg x q_reg points per triangle;
* panel pairs that touch (identical, common edge, common vertex) use rules
  that place the singular set at the apex of a radial coordinate, so that the
  1/r (single layer) and 1/r^2 (double layer) singularities are cancelled by
  the Jacobian.  They are derived from the fact that the integrand depends on
  x - y only:
    - identical triangles: integrating out the position leaves the
      autocorrelation area of the reference triangle, which is
      (1/2) (1 - l(z))^2 with l piecewise linear on six sectors; each sector
      is integrated in polar-like coordinates (rho, u);
    - common edge: parametrising both triangles along the shared edge, the
      integrand depends on (y1 - x1, x2, y2) only; the remaining weight is
      1 - l(v) with l piecewise linear on four cones, giving six tetrahedra
      with apex at the singular point, each integrated radially;
    - common vertex: the classical split into two regions s1 >= s2 and
      s2 >= s1 with Jacobian xi^3 eta.

Reference triangle: T = {(s, t): 0 <= t <= s <= 1}, mapped by
x = P0 + s (P1 - P0) + t (P2 - P1) with Jacobian 2 |gamma|.

Parity: pinned by tests against brute-force adaptive quadrature on
subdivided triangles, against exact polynomial integrals and against the
total area (constant integrand).
"""
import numpy as np


def gauss_legendre01(n):
    """Gauss-Legendre nodes/weights on [0, 1] by the Golub-Welsch eigenproblem."""
    if n < 1:
        raise ValueError("n >= 1")
    k = np.arange(1, n, dtype=np.float64)
    beta = k / np.sqrt(4.0 * k * k - 1.0)
    J = np.diag(beta, 1) + np.diag(beta, -1)
    x, V = np.linalg.eigh(J)
    w = 2.0 * V[0, :] ** 2
    order = np.argsort(x)
    x, w = x[order], w[order]
    return 0.5 * (x + 1.0), 0.5 * w


def triangle_rule(q):
    """Collapsed Gauss rule on the reference triangle; weights sum to 1/2."""
    g, w = gauss_legendre01(q)
    s = np.repeat(g, q)
    u = np.tile(g, q)
    t = s * u
    wt = np.repeat(w, q) * np.tile(w, q) * s
    return s, t, wt


def tri_geometry(P):
    """Area, unit normal (right-hand rule) and centroid of a triangle (3,3)."""
    n = np.cross(P[1] - P[0], P[2] - P[0])
    a2 = np.linalg.norm(n)
    return 0.5 * a2, n / a2, (P[0] + P[1] + P[2]) / 3.0


def map_ref(P, s, t):
    return P[0][None, :] + s[:, None] * (P[1] - P[0])[None, :] + t[:, None] * (P[2] - P[1])[None, :]


def classify(ta, tb):
    """Number of shared vertex indices: 3 identical, 2 edge, 1 vertex, 0 regular."""
    return len(set(int(i) for i in ta) & set(int(i) for i in tb))


# ---------------------------------------------------------------- regular

def regular_rule(P, Q, q):
    """Differences x - y and weights of the tensor collapsed-Gauss rule."""
    s, t, w = triangle_rule(q)
    x = map_ref(P, s, t)
    y = map_ref(Q, s, t)
    aP = tri_geometry(P)[0]
    aQ = tri_geometry(Q)[0]
    d = x[:, None, :] - y[None, :, :]
    W = (2 * aP) * (2 * aQ) * w[:, None] * w[None, :]
    return d.reshape(-1, 3), W.reshape(-1)


# ---------------------------------------------------------------- identical

_HEX = np.array([[1.0, 0.0], [1.0, 1.0], [0.0, 1.0], [-1.0, 0.0], [-1.0, -1.0], [0.0, -1.0]])


def identical_rule(P, q):
    """Rule for gamma x gamma with an integrand depending on x - y only.

    int int f(x-y) = (2|g|)^2 * sum_sectors int_0^1 int_0^1
                     f(-M rho w(u)) (1/2) (1-rho)^2 rho drho du,
    with M = [P1-P0, P2-P1] and w(u) on the hexagon edge of the sector.
    """
    g, wg = gauss_legendre01(q)
    area = tri_geometry(P)[0]
    M = np.stack([P[1] - P[0], P[2] - P[1]], axis=1)  # 3x2
    rho = np.repeat(g, q)
    u = np.tile(g, q)
    wr = np.repeat(wg, q) * np.tile(wg, q)
    ds, Ws = [], []
    for k in range(6):
        va, vb = _HEX[k], _HEX[(k + 1) % 6]
        z = rho[:, None] * (va[None, :] + u[:, None] * (vb - va)[None, :])
        ds.append(-(z @ M.T))
        Ws.append((2 * area) ** 2 * 0.5 * (1.0 - rho) ** 2 * rho * wr)
    return np.concatenate(ds), np.concatenate(Ws)


# ---------------------------------------------------------------- common edge

# Far facets (in coordinates v = (y1 - x1, x2, y2)) of the six tetrahedra whose
# cones from the origin tile the support of the weight 1 - l(v).
_EDGE_TETS = np.array([
    [[0, 1, 0], [1, 0, 0], [1, 0, 1]],
    [[0, 1, 0], [1, 0, 1], [0, 1, 1]],
    [[0, 0, 1], [1, 0, 1], [0, 1, 1]],
    [[0, 1, 0], [-1, 1, 0], [0, 1, 1]],
    [[0, 0, 1], [-1, 0, 0], [-1, 1, 0]],
    [[0, 0, 1], [-1, 1, 0], [0, 1, 1]],
], dtype=np.float64)


def edge_order(ta, tb):
    """Reorder two triangles sharing an edge as (E0, E1, P2), (E0, E1, Q2).

    E0, E1 follow the cyclic order of the first triangle after its free vertex.
    """
    ta = [int(i) for i in ta]
    tb = [int(i) for i in tb]
    shared = set(ta) & set(tb)
    i = [k for k in range(3) if ta[k] not in shared][0]
    e0, e1 = ta[(i + 1) % 3], ta[(i + 2) % 3]
    q2 = [v for v in tb if v not in shared][0]
    return (e0, e1, ta[i]), (e0, e1, q2)


def edge_rule(P, Q, q):
    """Rule for two triangles already ordered as (E0,E1,P2), (E0,E1,Q2)."""
    g, wg = gauss_legendre01(q)
    e = P[1] - P[0]
    c1 = P[2] - P[1]
    c2 = Q[2] - Q[1]
    aP = tri_geometry(P)[0]
    aQ = tri_geometry(Q)[0]
    rho = np.repeat(g, q * q)
    u1 = np.tile(np.repeat(g, q), q)
    u2 = np.tile(g, q * q)
    wr = np.repeat(wg, q * q) * np.tile(np.repeat(wg, q), q) * np.tile(wg, q * q)
    ds, Ws = [], []
    for a, b, c in _EDGE_TETS:
        det = abs(np.linalg.det(np.stack([a, b, c])))
        p = rho[:, None] * (a[None, :] + u1[:, None] * (b - a)[None, :]
                            + (u1 * u2)[:, None] * (c - b)[None, :])
        z, x2, y2 = p[:, 0], p[:, 1], p[:, 2]
        d = -z[:, None] * e[None, :] + x2[:, None] * c1[None, :] - y2[:, None] * c2[None, :]
        ds.append(d)
        Ws.append((2 * aP) * (2 * aQ) * det * (1.0 - rho) * rho ** 2 * u1 * wr)
    return np.concatenate(ds), np.concatenate(Ws)


# ---------------------------------------------------------------- common vertex

def vertex_order(ta, tb):
    """Rotate both triangles so that the shared vertex comes first."""
    ta = [int(i) for i in ta]
    tb = [int(i) for i in tb]
    v = (set(ta) & set(tb)).pop()
    ia, ib = ta.index(v), tb.index(v)
    return (v, ta[(ia + 1) % 3], ta[(ia + 2) % 3]), (v, tb[(ib + 1) % 3], tb[(ib + 2) % 3])


def vertex_rule(P, Q, q):
    """Rule for two triangles ordered with the shared vertex first."""
    g, wg = gauss_legendre01(q)
    a1, b1 = P[1] - P[0], P[2] - P[1]
    a2, b2 = Q[1] - Q[0], Q[2] - Q[1]
    aP = tri_geometry(P)[0]
    aQ = tri_geometry(Q)[0]
    n = q ** 4
    idx = np.indices((q, q, q, q)).reshape(4, n)
    xi, eta, u1, u2 = g[idx[0]], g[idx[1]], g[idx[2]], g[idx[3]]
    wr = wg[idx[0]] * wg[idx[1]] * wg[idx[2]] * wg[idx[3]]
    A1 = a1[None, :] + u1[:, None] * b1[None, :]
    A2 = a2[None, :] + u2[:, None] * b2[None, :]
    dA = xi[:, None] * (A1 - eta[:, None] * A2)
    dB = xi[:, None] * (eta[:, None] * A1 - A2)
    W = (2 * aP) * (2 * aQ) * xi ** 3 * eta * wr
    return np.concatenate([dA, dB]), np.concatenate([W, W])


# ---------------------------------------------------------------- dispatch

def pair_rule(verts, tris, k, j, singular, q_reg, q_sing):
    """Differences x - y (N,3) and weights for target triangle k, source j.

    ``singular`` selects the touching-pair rules; the caller decides it from
    the time offset (see timeint.needs_singular_rule).
    """
    ta, tb = tris[k], tris[j]
    nshared = classify(ta, tb)
    if nshared == 3:
        return identical_rule(verts[ta], q_sing)
    if singular and nshared == 2:
        oa, ob = edge_order(ta, tb)
        return edge_rule(verts[list(oa)], verts[list(ob)], q_sing)
    if singular and nshared == 1:
        oa, ob = vertex_order(ta, tb)
        return vertex_rule(verts[list(oa)], verts[list(ob)], q_sing)
    return regular_rule(verts[ta], verts[tb], q_reg)


# ---------------------------------------------------------------- p1 trial weights
# For a trial function that is linear on the source triangle (p1-continuous
# hat functions restricted to one panel) each rule above also needs the
# barycentric coordinates lambda_i(y) of the source point.  With the
# reference map y = Q0 + s (Q1 - Q0) + t (Q2 - Q1), 0 <= t <= s <= 1, they
# are (1 - s, s - t, t).  The common-edge rule integrates the position x1
# along the shared edge in closed form; lambda is affine in it, so its
# average over that segment is its value at the segment's midpoint.  The
# common-vertex rule keeps both points explicit.  The identical-panel rule
# integrates the position out as an area: it is not extended (the double
# layer vanishes on a panel with itself, as on every coplanar pair).

def _bary(s, t):
    return np.stack([1.0 - s, s - t, t], axis=1)


def regular_rule_p1(P, Q, q):
    """(x - y, W, lambda(y)) of the tensor collapsed-Gauss rule."""
    s, t, w = triangle_rule(q)
    x = map_ref(P, s, t)
    y = map_ref(Q, s, t)
    aP = tri_geometry(P)[0]
    aQ = tri_geometry(Q)[0]
    d = x[:, None, :] - y[None, :, :]
    W = (2 * aP) * (2 * aQ) * w[:, None] * w[None, :]
    lam_y = np.broadcast_to(_bary(s, t)[None, :, :], (len(s), len(s), 3))
    return d.reshape(-1, 3), W.reshape(-1), lam_y.reshape(-1, 3)


def edge_rule_p1(P, Q, q):
    """edge_rule plus lambda(y) in the order (E0, E1, Q2) of Q.

    In the variables v = (z, x2, y2) = (y1 - x1, x2, y2) the remaining
    position x1 runs over [max(x2, y2 - z), min(1, 1 - z)] (x and y in the
    reference triangle); y = (y1, y2) with y1 = x1 + z."""
    d, W = edge_rule(P, Q, q)
    g, _ = gauss_legendre01(q)
    rho = np.repeat(g, q * q)
    u1 = np.tile(np.repeat(g, q), q)
    u2 = np.tile(g, q * q)
    lams = []
    for a, b, c in _EDGE_TETS:
        p = rho[:, None] * (a[None, :] + u1[:, None] * (b - a)[None, :] + (u1 * u2)[:, None] * (c - b)[None, :])
        z, x2, y2 = p[:, 0], p[:, 1], p[:, 2]
        lo = np.maximum(x2, y2 - z)
        hi = np.minimum(1.0, 1.0 - z)
        y1 = 0.5 * (lo + hi) + z
        lams.append(_bary(y1, y2))
    return d, W, np.concatenate(lams)


def vertex_rule_p1(P, Q, q):
    """vertex_rule plus lambda(y) in the order (V, Q1, Q2) of Q.

    First region: x = V + xi A1, y = V + xi eta A2 (reference coordinates
    (xi eta, xi eta u2) of y); second: x = V + xi eta A1, y = V + xi A2."""
    d, W = vertex_rule(P, Q, q)
    g, _ = gauss_legendre01(q)
    n = q ** 4
    idx = np.indices((q, q, q, q)).reshape(4, n)
    xi, eta, u2 = g[idx[0]], g[idx[1]], g[idx[3]]
    la = _bary(xi * eta, xi * eta * u2)
    lb = _bary(xi, xi * u2)
    return d, W, np.concatenate([la, lb])


def pair_rule_p1(verts, tris, k, j, singular, q_reg, q_sing):
    """(x - y, W, lambda) for target triangle k and source j, lambda[:, i]
    the barycentric coordinate of y for vertex tris[j][i]."""
    ta, tb = tris[k], tris[j]
    nshared = classify(ta, tb)
    if nshared == 3:
        raise ValueError("identical panels: no p1 rule (the double layer vanishes there)")
    if singular and nshared in (1, 2):
        oa, ob = edge_order(ta, tb) if nshared == 2 else vertex_order(ta, tb)
        rule = edge_rule_p1 if nshared == 2 else vertex_rule_p1
        d, W, lo = rule(verts[list(oa)], verts[list(ob)], q_sing)
        cols = [list(ob).index(int(v)) for v in tb]      # column of each of tris[j]'s vertices
        return d, W, lo[:, cols]
    return regular_rule_p1(verts[ta], verts[tb], q_reg)

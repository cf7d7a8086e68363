"""Cube-surface space-time meshes and seeded densities.

The test problems of the paper (Section 5) are the lateral boundary of a cube
times a time interval, discretised by a fixed triangulated surface and uniform
time steps (tensor-product mesh, Section 2).  The paper does not describe its
triangulation, so the cube faces here are split into n x n squares and each
square into two triangles along a fixed diagonal:

* a face is (normal axis a, side +-1); its in-face axes (u, v) are the two
  other coordinate axes in increasing order;
* square (i, j) spans [u_i, u_{i+1}] x [v_j, v_{j+1}] with u_i = -1 + 2 i / n;
  it is split along the (u_i, v_j) -> (u_{i+1}, v_{j+1}) diagonal into
  (p00, p10, p11) and (p00, p11, p01);
* vertex order is flipped where needed so that (p1 - p0) x (p2 - p0) points
  out of the cube;
* vertices are shared between neighbouring triangles and faces (conforming).

Faces are emitted in the order (x-, x+, y-, y+, z-, z+), squares row-major in
(i, j), two triangles per square.
"""
import numpy as np

# The five workloads used by the tests and the benchmark.  Sizes follow the
# paper's cube experiments in shape (Section 5): surface triangles x uniform
# time steps on a unit time interval, heat capacity alpha = 1.
CONFIGS = {
    1: dict(n=4, n_steps=16, m_t=4, m_x=4, n_max=64, c_st=0.9, n_tr=5, seed=1),
    2: dict(n=16, n_steps=256, m_t=6, m_x=6, n_max=64, c_st=0.9, n_tr=5, seed=2),
    3: dict(n=16, n_steps=1024, m_t=6, m_x=6, n_max=64, c_st=0.9, n_tr=5, seed=3),
    5: dict(n=32, n_steps=512, m_t=6, m_x=6, n_max=64, c_st=0.9, n_tr=3, seed=5),
}


def cube_surface_mesh(n):
    """Return (vertices (nv,3) float64, triangles (nt,3) int32) of [-1,1]^3."""
    if n < 1:
        raise ValueError("n must be >= 1")
    vid = {}
    verts = []

    def vertex(ijk):
        key = tuple(int(c) for c in ijk)
        v = vid.get(key)
        if v is None:
            v = len(verts)
            vid[key] = v
            verts.append([-1.0 + 2.0 * c / n for c in key])
        return v

    tris = []
    for a in range(3):
        u_ax, v_ax = [ax for ax in range(3) if ax != a]
        for side in (0, n):  # -1 face, then +1 face
            outward = 1.0 if side == n else -1.0
            for i in range(n):
                for j in range(n):
                    def g(di, dj):
                        c = [0, 0, 0]
                        c[a] = side
                        c[u_ax] = i + di
                        c[v_ax] = j + dj
                        return c
                    p00, p10, p11, p01 = g(0, 0), g(1, 0), g(1, 1), g(0, 1)
                    for tri in ((p00, p10, p11), (p00, p11, p01)):
                        e1 = np.subtract(tri[1], tri[0])
                        e2 = np.subtract(tri[2], tri[0])
                        nrm = np.cross(e1, e2)
                        if nrm[a] * outward < 0:
                            tri = (tri[0], tri[2], tri[1])
                        tris.append([vertex(p) for p in tri])
    return np.asarray(verts, dtype=np.float64), np.asarray(tris, dtype=np.int32)


def uniform_time_nodes(n_steps, T=1.0):
    """t_j = j * T / n_steps, j = 0..n_steps, each computed directly."""
    j = np.arange(n_steps + 1, dtype=np.float64)
    return (j * T) / n_steps


def densities(n_dofs, seed):
    """i.i.d. U(-1, 1) coefficients in natural (time-major) order."""
    return np.random.default_rng(seed).uniform(-1.0, 1.0, n_dofs)


def config_problem(cfg_id):
    """Mesh, time nodes, parameters and density of one of the named workloads."""
    c = dict(CONFIGS[cfg_id])
    verts, tris = cube_surface_mesh(c["n"])
    t = uniform_time_nodes(c["n_steps"])
    w = densities(c["n_steps"] * len(tris), c["seed"])
    return verts, tris, t, c, w


def batch_sizes(seed=4, count=48):
    """The batched workload: `count` independent cube problems with face grids
    n ~ U{4..32} and step counts E_t ~ U{32..512}, drawn in that order from
    default_rng(seed).  Returns [(n, E_t)]."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        n = int(rng.integers(4, 33))
        e = int(rng.integers(32, 513))
        out.append((n, e))
    return out

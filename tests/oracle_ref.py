"""Oracle reference products for the GPU parity tests (CPU, FP64)."""
import numpy as np

from oracle.dense import toeplitz_blocks
from oracle.fmm import FMMOracle
from oracle.tree import Tree
from workloads import cube_surface_mesh, uniform_time_nodes, densities


def problem(n, E_t, T=1.0, seed=1):
    v, t = cube_surface_mesh(n)
    tn = uniform_time_nodes(E_t, T)
    w = densities(E_t * len(t), seed)
    return v, t, tn, w


def reference(v, t, tn, w, kind, alpha=1.0, m_t=4, m_x=4, n_max=64, c_st=0.9, n_tr=5, q_reg=4, q_sing=5):
    """Oracle pFMM product (Algorithm 2) with exact reuse of identical integrals."""
    E_t = len(tn) - 1
    h = (tn[-1] - tn[0]) / E_t
    tr = Tree(v, t, tn, alpha, n_max, c_st, n_tr)
    o = FMMOracle(tr, m_t, m_x, kind, q_reg, q_sing)
    o.set_toeplitz_blocks(toeplitz_blocks(v, t, E_t, h, alpha, kind, q_reg, q_sing))
    return o.apply(w)


def rel_err(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))

"""Host-side checks of the C ABI (no GPU needed).

* libpfmm.so loads and exports every function declared in include/pfmm.h.
* The C++ planner (Algorithm 1 and the lists of Section 3.3) reproduces the
  oracle's tree and list counts exactly.
* Invalid input is rejected with the documented status codes.
"""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_2106_15911_amd as P
from oracle.tree import Tree
from workloads import cube_surface_mesh, uniform_time_nodes

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_exports_every_declared_symbol():
    lib = ctypes.CDLL(P.lib_path())
    names = set()
    for h in os.listdir(os.path.join(ROOT, "include")):
        src = open(os.path.join(ROOT, "include", h)).read()
        names |= set(re.findall(r"\b(pfmm_[a-z_0-9]+)\s*\(", src))
    assert names, "no declarations found"
    for n in sorted(names):
        assert hasattr(lib, n), n


def graded_nodes(n, T=1.0, p=1.7):
    return T * (np.arange(n + 1) / n) ** p


def _oracle_counts(n, E_t, n_max, n_tr, tn=None):
    v, t = cube_surface_mesh(n)
    tr = Tree(v, t, uniform_time_nodes(E_t) if tn is None else tn, 1.0, n_max, 0.9, n_tr)
    memo = {}
    near = 0
    for Z in tr.leaves:
        kt = np.arange(Z.s0, Z.s1)
        for S in tr.nearfield(Z, memo):
            jt = np.arange(S.s0, S.s1)
            near += int(np.sum(kt[:, None] >= jt[None, :])) * len(Z.tris) * len(S.tris)
    m2l = sum(len(tr.interaction(Z)) for Z in tr.boxes)
    return dict(depth=tr.depth, boxes=len(tr.boxes), leaves=len(tr.leaves), near_entries=near, m2l_pairs=m2l)


@pytest.mark.parametrize("n,E_t,n_max,n_tr", [(4, 16, 64, 5), (4, 16, 64, 1), (2, 8, 8, -1), (8, 64, 64, 2),
                                              (4, 32, 16, 3),
                                              # step counts whose time levels split unevenly (nearest-step
                                              # split points of Algorithm 1; leaves on several levels)
                                              (4, 20, 64, 5), (3, 37, 16, 3), (2, 70, 8, -1), (4, 33, 64, 2),
                                              (5, 47, 32, 3),
                                              # single-step leaves of 96 triangles (refinement stops at one step)
                                              (8, 4, 64, 5), (8, 3, 64, 5)])
def test_planner_counts_match_oracle(n, E_t, n_max, n_tr):
    v, t = cube_surface_mesh(n)
    st = P.plan_stats(v, t, uniform_time_nodes(E_t), P.default_params(n_max=n_max, n_tr=n_tr, m_t=3, m_x=3))
    ref = _oracle_counts(n, E_t, n_max, n_tr)
    for k, val in ref.items():
        assert st[k] == val, (k, st[k], val)


@pytest.mark.parametrize("n,E_t,n_max,n_tr,p", [(4, 16, 64, 5, 1.7), (3, 37, 16, 3, 1.7), (2, 40, 8, -1, 2.5),
                                                (4, 33, 64, 2, 0.6)])
def test_planner_counts_match_oracle_graded_steps(n, E_t, n_max, n_tr, p):
    """Graded steps t_j = (j / E_t)^p: Algorithm 1 splits at the node nearest
    the time midpoint, so the tree differs from the uniform one; the counts
    still match the oracle's, and every level >= 2 with more than one pair
    of intervals has classes beyond the two of a uniform grid."""
    v, t = cube_surface_mesh(n)
    tn = graded_nodes(E_t, p=p)
    st = P.plan_stats(v, t, tn, P.default_params(n_max=n_max, n_tr=n_tr, m_t=3, m_x=3))
    ref = _oracle_counts(n, E_t, n_max, n_tr, tn)
    for k, val in ref.items():
        assert st[k] == val, (k, st[k], val)
    assert st["n_time_classes"] > 2


def test_planner_counts_second_workload():
    """3072 triangles x 256 steps, n_tr = 5: the counts also match an independent tally
    (including the causal K_h entries between panels that are not coplanar)."""
    v, t = cube_surface_mesh(16)
    st = P.plan_stats(v, t, uniform_time_nodes(256), P.default_params())
    assert st["boxes"] == 92273 and st["leaves"] == 76288
    assert st["near_entries"] == 6725369088 and st["m2l_pairs"] == 11126496
    assert st["near_nonzero_K"] == 4804862976
    assert st["n_time_classes"] == 2


def test_nonzero_K_count_matches_oracle():
    """Causal nearfield entries of K_h between panels that are not coplanar:
    the planner's count equals the oracle's tree and coplanarity test
    (192 triangles x 16 steps, no spatial cut; 1,597,440 by an independent tally)."""
    from oracle.dense import coplanar
    v, t = cube_surface_mesh(4)
    tn = uniform_time_nodes(16)
    st = P.plan_stats(v, t, tn, P.default_params(m_t=4, m_x=4))
    tr = Tree(v, t, tn, 1.0, 64, 0.9, 5)
    memo = {}
    cop = {}
    nz = 0
    for Z in tr.leaves:
        kt = np.arange(Z.s0, Z.s1)
        for S in tr.nearfield(Z, memo):
            jt = np.arange(S.s0, S.s1)
            steps = int(np.sum(kt[:, None] >= jt[None, :]))
            pairs = 0
            for k in Z.tris:
                for j in S.tris:
                    key = (int(k), int(j))
                    if key not in cop:
                        cop[key] = coplanar(v, t, int(k), int(j))
                    pairs += 0 if cop[key] else 1
            nz += steps * pairs
    assert st["near_nonzero_K"] == nz == 1597440


def test_p1_double_layer_planning():
    """The p1 double layer stores three columns per source triangle (its
    local vertices) in the stored-block layout of V_h; the Toeplitz mode
    has no such layout and is refused."""
    v, t = cube_surface_mesh(4)
    tn = uniform_time_nodes(16)
    st = P.plan_stats(v, t, tn, P.default_params(operators=P.OP_V | P.OP_K1, m_t=3, m_x=3))
    assert st["near_entries_K1"] == 3 * st["near_entries"]
    assert P.plan_stats(v, t, tn, P.default_params(m_t=3, m_x=3))["near_entries_K1"] == 0
    with pytest.raises(P.PfmmError) as e:
        P.plan_stats(v, t, tn, P.default_params(operators=P.OP_K1, nearfield_mode=P.NF_TOEPLITZ))
    assert e.value.status == -6
    with pytest.raises(P.PfmmError) as e:
        P.plan_stats(v, t, tn, P.default_params(operators=8))
    assert e.value.status == -1


def test_error_codes():
    v, t = cube_surface_mesh(2)
    tn = uniform_time_nodes(8)
    with pytest.raises(P.PfmmError) as e:
        P.plan_stats(v, t[:-1], tn)                      # open surface
    assert e.value.status == -1
    bad = tn.copy()
    bad[3] += 0.01
    P.plan_stats(v, t, bad)                              # steps of different lengths: stored nearfield
    with pytest.raises(P.PfmmError) as e:
        P.plan_stats(v, t, bad, P.default_params(nearfield_mode=P.NF_TOEPLITZ))
    assert e.value.status == -6                          # no Toeplitz structure to use
    bad[3] = bad[2]
    with pytest.raises(P.PfmmError) as e:
        P.plan_stats(v, t, bad)                          # repeated node
    assert e.value.status == -1
    vn = v.copy()
    vn[0, 0] = np.nan
    with pytest.raises(P.PfmmError) as e:
        P.plan_stats(vn, t, tn)
    assert e.value.status == -5
    with pytest.raises(P.PfmmError) as e:
        P.plan_stats(v, t, tn, P.default_params(alpha=-1.0))
    assert e.value.status == -1
    flipped = t.copy()
    flipped[0] = flipped[0][[0, 2, 1]]
    with pytest.raises(P.PfmmError) as e:
        P.plan_stats(v, flipped, tn)                     # inconsistent orientation
    assert e.value.status == -1
    v4, t4 = cube_surface_mesh(4)
    st = P.plan_stats(v4, t4, uniform_time_nodes(20))    # 20 steps: level 3 intervals of 2 and 3 steps
    assert st["n_time_classes"] > 2


def test_solve_entry_points_validate_without_gpu():
    lib = P.load_library()
    o = P.SolveOpts()
    assert lib.pfmm_default_solve_opts(o) == 0 and o.rtol == 1e-8 and o.max_iter == 200
    assert o.inner_precision == P.FP64 and not o.x0_dev and not o.precond and o.precond_path is None
    assert lib.pfmm_default_solve_opts(None) == -1
    info = P.SolveInfo()
    for fn in (lib.pfmm_solve_V, lib.pfmm_solve_dirichlet):
        assert fn(None, None, None, None, None, None) == -1
        assert b"NULL" in lib.pfmm_last_error()

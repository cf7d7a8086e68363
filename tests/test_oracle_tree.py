"""Pins of the oracle's cluster tree and lists (CPU only).

* The temporal lists of the paper's worked example (Section 3.3, text after
  eq. 03:ILtemp): N(I_6^(3)) = {I_5^(3), I_6^(3)} and I(I_6^(3)) = {I_4^(3)}.
* Exact coverage: with no spatial cut (n_tr = -1) every causal element pair
  lies in exactly one inadmissible (nearfield) block of a leaf or one
  admissible (interaction-list) block, and no admissible block holds a
  non-causal pair (Section 3.4, matrix partition).
* Padded boxes contain their children and their elements (Section 3.2).
* Refinement types alternate after the first levels (Section 3.2).
"""
import numpy as np
import pytest

from oracle.tree import Tree
from workloads import cube_surface_mesh, uniform_time_nodes


def _tree(n, E_t, n_max=64, c_st=0.9, n_tr=5):
    v, t = cube_surface_mesh(n)
    return Tree(v, t, uniform_time_nodes(E_t), 1.0, n_max, c_st, n_tr)


def test_worked_example_temporal_lists():
    tr = _tree(4, 16)
    assert tr.tI[3] == set(range(8))
    assert tr.temporal_nearfield(3, 6) == {(3, 5), (3, 6)}
    assert tr.temporal_interaction(3, 6) == {4}
    assert tr.temporal_interaction(3, 7) == {4, 5}
    assert tr.temporal_interaction(3, 1) == set()
    assert tr.temporal_nearfield(3, 0) == {(3, 0)}


def test_refinement_types_alternate():
    tr = _tree(16, 256)
    assert tr.rtype == ["st", "t", "st", "t", "st", "t", "st"]


def _coverage(tr):
    N = tr.E_t * tr.E_x
    cnt = np.zeros((N, N), dtype=np.int32)
    memo = {}
    for Z in tr.leaves:
        rows = tr.elements(Z)
        for S in tr.nearfield(Z, memo):
            cols = tr.elements(S)
            cnt[np.ix_(rows, cols)] += 1
    far_noncausal = 0
    for Z in tr.boxes:
        for S in tr.interaction(Z):
            rows = tr.elements(Z)
            cols = tr.elements(S)
            cnt[np.ix_(rows, cols)] += 1
            kt = rows // tr.E_x
            jt = cols // tr.E_x
            far_noncausal += int(np.sum(jt[None, :] > kt[:, None]))
    kt = np.arange(N) // tr.E_x
    causal = kt[:, None] >= kt[None, :]
    return cnt, causal, far_noncausal


@pytest.mark.parametrize("n,E_t,n_max", [(2, 8, 8), (2, 7, 6), (3, 12, 10), (4, 16, 64)])
def test_exact_coverage_without_cut(n, E_t, n_max):
    tr = _tree(n, E_t, n_max=n_max, n_tr=-1)
    cnt, causal, far_noncausal = _coverage(tr)
    assert far_noncausal == 0
    assert np.all(cnt[causal] == 1)
    # nearfield blocks may include non-causal pairs of the same interval, nothing else
    assert np.all(cnt[~causal] <= 1)


def test_counts_c1():
    """Integer counts of the 192-triangle x 16-step tree (also reproduced by the C++ planner)."""
    tr = _tree(4, 16)
    assert len(tr.leaves) == 448 and len(tr.boxes) == 497 and tr.depth == 3
    memo = {}
    near = 0
    for Z in tr.leaves:
        kt = np.arange(Z.s0, Z.s1)
        for S in tr.nearfield(Z, memo):
            jt = np.arange(S.s0, S.s1)
            near += int(np.sum(kt[:, None] >= jt[None, :])) * len(Z.tris) * len(S.tris)
    m2l = sum(len(tr.interaction(Z)) for Z in tr.boxes)
    far = sum((Z.s1 - Z.s0) * len(Z.tris) * (S.s1 - S.s0) * len(S.tris)
              for Z in tr.boxes for S in tr.interaction(Z))
    assert near == 1916928
    assert m2l == 28416
    assert near + far == 192 * 192 * 16 * 17 // 2


def test_padding_contains_children():
    tr = _tree(3, 8, n_max=8)
    assert max(tr.pad) > 0.0
    P = tr.verts[tr.tri]
    for b in tr.boxes:
        lo = tr.box_lower(b)
        hi = lo + 2 * tr.hx_padded(b.level)
        V = P[b.tris].reshape(-1, 3)
        assert np.all(V >= lo - 1e-12) and np.all(V <= hi + 1e-12)
        for c in b.children:
            clo = tr.box_lower(c)
            chi = clo + 2 * tr.hx_padded(c.level)
            assert np.all(clo >= lo - 1e-12) and np.all(chi <= hi + 1e-12)
            assert tr.t[c.s0] >= tr.t[b.s0] and tr.t[c.s1] <= tr.t[b.s1]

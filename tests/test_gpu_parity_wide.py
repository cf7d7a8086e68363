"""GPU parity on deep time trees: levels with 64, 128 and 256 intervals run
the wide matrix-core M2L (row groups x two or four 32-interval blocks, one or
two column blocks per workgroup).  Rows are sampled across every interval
block (first and last steps included) and computed one by one by the oracle
(complete upward pass, the ancestor chain's M2L/L2L/L2T, the row's
nearfield sum)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_2106_15911_amd as P
from oracle.fmm import FMMOracle
from oracle.tree import Tree
from oracle_ref import problem

pytestmark = pytest.mark.gpu

CASES = [
    # 24 triangles x 1024 steps: depth 7, levels with 64 and 128 intervals
    dict(n=2, E_t=1024, m_t=4, m_x=4, n_max=16, n_tr=3),
    dict(n=2, E_t=1024, m_t=6, m_x=6, n_max=16, n_tr=3),
    # 2048 steps: a level with 256 intervals (two column blocks of 128)
    dict(n=2, E_t=2048, m_t=3, m_x=5, n_max=16, n_tr=2),
]


def _rows(E_t, E_x, rng):
    steps = np.unique(np.concatenate([np.linspace(0, E_t - 1, 48).astype(int), [0, 1, E_t - 1]]))
    tri = rng.integers(0, E_x, len(steps))
    return steps * E_x + tri


@pytest.mark.parametrize("case", CASES)
@pytest.mark.parametrize("kind", ["V", "K"])
def test_deep_time_tree_sampled_rows(case, kind):
    print(f"[parity-wide] {case} kind={kind}", flush=True)
    c = dict(case)
    n, E_t = c.pop("n"), c.pop("E_t")
    v, t, tn, w = problem(n, E_t, seed=23)
    op = 1 if kind == "V" else 2
    tree = P.Tree(v, t, tn, P.default_params(operators=op, **c), device=0)
    st = tree.stats()
    assert st["m2l_matrix_cores"] == 1
    x = torch.from_numpy(w).to("cuda:0")
    f = (tree.apply_V(x) if kind == "V" else tree.apply_K(x)).cpu().numpy()
    tree.close()
    assert np.all(np.isfinite(f))
    tr = Tree(v, t, tn, 1.0, c["n_max"], 0.9, c["n_tr"])
    o = FMMOracle(tr, c["m_t"], c["m_x"], kind)
    rows = _rows(E_t, len(t), np.random.default_rng(29))
    vals, _ = o.apply_rows(w, rows)
    err = np.abs(f[rows] - vals).max() / np.abs(vals).max()
    print(f"[parity-wide] depth {st['depth']} rows {len(rows)} max rel err {err:.3e}", flush=True)
    assert err <= 1e-10

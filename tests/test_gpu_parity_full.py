"""Full-size GPU parity: the 3072-triangle x 256-step workload (786,432 DOFs,
degrees 6/6, n_max 64, c_st 0.9, n_tr 5) in the configuration bench.py times.
The oracle computes sampled rows one by one (complete upward pass, the
ancestor chain's M2L/L2L/L2T, and the row's nearfield sum): 64 random rows
plus the first and last steps and 8 rows from each leaf level."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_2106_15911_amd as P
from oracle.fmm import FMMOracle
from oracle.tree import Tree
from sampling import sample_rows
from workloads import config_problem

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("kind", ["V", "K"])
def test_full_size_sampled_rows(kind):
    print(f"[parity-full] kind={kind}", flush=True)
    v, t, tn, c, w = config_problem(2)
    op = 1 if kind == "V" else 2
    tree = P.Tree(v, t, tn, P.default_params(operators=op), device=0)
    st = tree.stats()
    assert st["m2l_matrix_cores"] == 1
    x = torch.from_numpy(w).to("cuda:0")
    f = (tree.apply_V(x) if kind == "V" else tree.apply_K(x)).cpu().numpy()
    tree.close()
    assert np.all(np.isfinite(f))
    tr = Tree(v, t, tn, 1.0, c["n_max"], c["c_st"], c["n_tr"])
    o = FMMOracle(tr, c["m_t"], c["m_x"], kind)
    rows, levels = sample_rows(tr, 64)
    assert len(levels) == 2          # leaves on levels 6 and 7
    vals, _ = o.apply_rows(w, rows)
    err = np.abs(f[rows] - vals).max() / np.abs(vals).max()
    print(f"[parity-full] kind={kind} {len(rows)} rows, max rel err {err:.3e}", flush=True)
    assert err <= 1e-10

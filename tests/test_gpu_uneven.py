"""Trees whose time levels split unevenly (Algorithm 1 splits an interval at
its middle step, the earlier one on a tie, so step counts that are not
multiples of 2^depth give intervals of different lengths, and leaves then
sit on several levels of one time range): the GPU apply against the oracle
pFMM on the same tree (1e-10 relative, FP64), the mixed farfield against
FP64 on the same tree, the Toeplitz nearfield against the stored one, and a
larger tree with time classes on every level against sampled oracle rows."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_2106_15911_amd as P
from oracle.fmm import FMMOracle
from oracle.tree import Tree
from oracle_ref import problem, reference, rel_err
from sampling import sample_rows

pytestmark = pytest.mark.gpu

CASES = [(4, 20, dict(m_t=4, m_x=4, n_max=64, n_tr=5)), (3, 37, dict(m_t=4, m_x=4, n_max=16, n_tr=3)),
         (2, 70, dict(m_t=3, m_x=3, n_max=8, n_tr=-1))]


@pytest.mark.parametrize("case", range(len(CASES)))
def test_uneven_steps_match_oracle(case):
    n, E_t, prm = CASES[case]
    print(f"[uneven] n={n} E_t={E_t} {prm}", flush=True)
    v, t, tn, w = problem(n, E_t, seed=90 + case)
    tree = P.Tree(v, t, tn, P.default_params(precision=P.MIXED_FP32, **prm), device=0)
    st = tree.stats()
    print(f"[uneven] stats {st}", flush=True)
    assert st["n_time_classes"] > 2
    x = torch.from_numpy(w).to("cuda:0")
    out = {}
    for kind in ("V", "K"):
        tree.set_precision(P.FP64)
        f = (tree.apply_V(x) if kind == "V" else tree.apply_K(x)).cpu().numpy()
        r = reference(v, t, tn, w, kind, **prm)
        e = rel_err(f, r)
        em = np.abs(f - r).max() / np.abs(r).max()
        print(f"[uneven] {kind}: rel err {e:.3e} (max {em:.3e})", flush=True)
        assert np.isfinite(e) and e <= 1e-10 and em <= 1e-10
        out[kind] = f
    tree.set_precision(P.MIXED_FP32)
    f32 = tree.apply_V(x).cpu().numpy()
    e32 = rel_err(f32, out["V"])
    print(f"[uneven] FP32 farfield vs FP64: {e32:.3e}", flush=True)
    assert e32 <= 1e-6
    tree.close()
    # Toeplitz nearfield on the same tree: same sums in another order
    tt = P.Tree(v, t, tn, P.default_params(nearfield_mode=P.NF_TOEPLITZ, **prm), device=0)
    ft = tt.apply_V(x).cpu().numpy()
    tt.close()
    assert np.abs(ft - out["V"]).max() <= 1e-13 * np.abs(out["V"]).max()


def test_uneven_larger_tree_sampled_rows():
    """768 triangles x 479 steps (m = 6, n_max 64, n_tr 5): every level has
    intervals of two lengths; sampled rows (random, first and last steps,
    every leaf level) against the oracle."""
    v, t, tn, w = problem(8, 479, seed=95)
    print(f"[uneven] 768 x 479: build", flush=True)
    tree = P.Tree(v, t, tn, P.default_params(operators=1), device=0)
    st = tree.stats()
    print(f"[uneven] stats {st}", flush=True)
    f = tree.apply_V(torch.from_numpy(w).to("cuda:0")).cpu().numpy()
    tree.close()
    tr = Tree(v, t, tn, 1.0, 64, 0.9, 5)
    o = FMMOracle(tr, 6, 6, "V")
    rows, levels = sample_rows(tr, 24, per_level=4)
    print(f"[uneven] oracle {len(rows)} rows, leaf levels {levels}", flush=True)
    vals, _ = o.apply_rows(w, rows)
    err = np.abs(f[rows] - vals).max() / np.abs(vals).max()
    print(f"[uneven] 768 x 479 rows max rel err {err:.3e}", flush=True)
    assert err <= 1e-10


def test_single_step_leaves_of_more_than_64_triangles():
    """768 triangles x 3 steps: refinement stops at intervals of one step, so
    leaves hold 96 triangles (the nearfield and S2M/L2T kernels take them in
    row chunks of at most 64); V_h and K_h against the oracle."""
    v, t, tn, w = problem(8, 3, seed=97)
    prm = dict(m_t=3, m_x=3)
    tree = P.Tree(v, t, tn, P.default_params(**prm), device=0)
    x = torch.from_numpy(w).to("cuda:0")
    for kind in ("V", "K"):
        f = (tree.apply_V(x) if kind == "V" else tree.apply_K(x)).cpu().numpy()
        r = reference(v, t, tn, w, kind, **prm)
        e = rel_err(f, r)
        print(f"[uneven] 768 x 3 {kind}: rel err {e:.3e}", flush=True)
        assert np.isfinite(e) and e <= 1e-10
    tree.close()

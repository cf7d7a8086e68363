"""Toeplitz nearfield mode (no stored blocks; entries read from the distinct
integrals per (leaf spatial box, step difference)) against the CPU oracle and
against the stored-block mode on the same tree.

The stored blocks are copies of the same distinct values and both products
sum the same terms in the same order per lane, so the two modes must agree
bit for bit; against the oracle the FP64 bar (1e-10 relative) applies."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_2106_15911_amd as P
from oracle.fmm import FMMOracle
from oracle.tree import Tree
from oracle_ref import problem, reference, rel_err
from workloads import config_problem

pytestmark = pytest.mark.gpu
TOL = 1e-10


def _apply(v, t, tn, w, kind, mode, **prm):
    op = 1 if kind == "V" else 2
    tree = P.Tree(v, t, tn, P.default_params(operators=op, nearfield_mode=mode, **prm), device=0)
    x = torch.from_numpy(w).to("cuda:0")
    f = tree.apply_V(x) if kind == "V" else tree.apply_K(x)
    torch.cuda.synchronize()
    st = tree.stats()
    tree.close()
    return f.cpu(), st


@pytest.mark.parametrize("case", [
    dict(n=4, E_t=16, m_t=4, m_x=4),
    dict(n=2, E_t=32, m_t=5, m_x=2, n_max=16, n_tr=-1, alpha=2.0),
    dict(n=2, E_t=16, m_t=2, m_x=5, n_max=12, n_tr=1, alpha=0.5),
])
@pytest.mark.parametrize("kind", ["V", "K"])
def test_toeplitz_vs_oracle_and_stored(case, kind):
    print(f"[toeplitz] {case} kind={kind}", flush=True)
    c = dict(case)
    v, t, tn, w = problem(c.pop("n"), c.pop("E_t"), seed=13)
    ft, st_t = _apply(v, t, tn, w, kind, P.NF_TOEPLITZ, **c)
    fs, st_s = _apply(v, t, tn, w, kind, P.NF_STORED, **c)
    assert torch.equal(ft, fs)
    assert st_t["device_bytes"] < st_s["device_bytes"]
    r = reference(v, t, tn, w, kind, **c)
    g = ft.numpy()
    e = rel_err(g, r)
    m = float(np.abs(g - r).max() / np.abs(r).max())
    assert e <= TOL and m <= TOL, (e, m)


def test_toeplitz_full_size():
    """3072 triangles x 256 steps, degrees 6/6: bitwise equal to the stored
    mode, sampled rows against the oracle, and without the 53.8 GB of blocks."""
    print("[toeplitz] full size", flush=True)
    v, t, tn, c, w = config_problem(2)
    ft, st_t = _apply(v, t, tn, w, "V", P.NF_TOEPLITZ)
    fs, st_s = _apply(v, t, tn, w, "V", P.NF_STORED)
    assert torch.equal(ft, fs)
    assert st_s["device_bytes"] - st_t["device_bytes"] >= 8 * st_s["near_entries"] * 0.99
    tr = Tree(v, t, tn, 1.0, c["n_max"], c["c_st"], c["n_tr"])
    o = FMMOracle(tr, c["m_t"], c["m_x"], "V")
    rows = np.concatenate([np.random.default_rng(41).choice(len(w), 6, replace=False), [0, len(w) - 1]])
    vals, _ = o.apply_rows(w, rows)
    f = ft.numpy()
    err = np.abs(f[rows] - vals).max() / np.abs(vals).max()
    print(f"[toeplitz] full size: device bytes {st_t['device_bytes']} vs {st_s['device_bytes']}; "
          f"sampled rows max rel err {err:.3e}", flush=True)
    assert err <= TOL

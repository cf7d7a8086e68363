"""Mixed-precision farfield (M2L with FP32 moments and operator entries, FP32
matrix-core accumulation; everything else FP64) against the FP64 apply on the
same tree and against the CPU FP64 oracle.

Bar: relative 2-norm difference to the FP64 apply <= 1e-6 (the stated target
of the mixed mode), and sampled oracle rows within 2e-6 of max |f|.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_2106_15911_amd as P
from oracle.fmm import FMMOracle
from oracle.tree import Tree
from oracle_ref import problem
from test_gpu_parity_wide import CASES, _rows
from workloads import config_problem

pytestmark = pytest.mark.gpu
MIXED_TOL = 1e-6


def _both(tree, x, kind):
    fn = tree.apply_V if kind == "V" else tree.apply_K
    tree.set_precision(P.MIXED_FP32)
    fm = fn(x).cpu().numpy()
    tree.set_precision(P.FP64)
    fd = fn(x).cpu().numpy()
    return fm, fd


@pytest.mark.parametrize("case", CASES)
@pytest.mark.parametrize("kind", ["V", "K"])
def test_mixed_deep_time_tree(case, kind):
    print(f"[mixed] {case} kind={kind}", flush=True)
    c = dict(case)
    n, E_t = c.pop("n"), c.pop("E_t")
    v, t, tn, w = problem(n, E_t, seed=23)
    op = 1 if kind == "V" else 2
    tree = P.Tree(v, t, tn, P.default_params(operators=op, precision=P.MIXED_FP32, **c), device=0)
    x = torch.from_numpy(w).to("cuda:0")
    fm, fd = _both(tree, x, kind)
    tree.close()
    assert np.all(np.isfinite(fm))
    e = np.linalg.norm(fm - fd) / np.linalg.norm(fd)
    tr = Tree(v, t, tn, 1.0, c["n_max"], 0.9, c["n_tr"])
    o = FMMOracle(tr, c["m_t"], c["m_x"], kind)
    rows = _rows(E_t, len(t), np.random.default_rng(31))
    vals, _ = o.apply_rows(w, rows)
    eo = np.abs(fm[rows] - vals).max() / np.abs(vals).max()
    print(f"[mixed] rel 2-norm vs FP64 {e:.3e}; sampled rows vs oracle {eo:.3e}", flush=True)
    assert e > 0.0          # the FP32 path really ran
    assert e <= MIXED_TOL
    assert eo <= 2 * MIXED_TOL


@pytest.mark.parametrize("kind", ["V", "K"])
def test_mixed_full_size(kind):
    """3072 triangles x 256 steps, degrees 6/6: the benchmarked configuration."""
    print(f"[mixed] full size kind={kind}", flush=True)
    v, t, tn, c, w = config_problem(2)
    op = 1 if kind == "V" else 2
    tree = P.Tree(v, t, tn, P.default_params(operators=op, precision=P.MIXED_FP32), device=0)
    x = torch.from_numpy(w).to("cuda:0")
    fm, fd = _both(tree, x, kind)
    tree.close()
    e = np.linalg.norm(fm - fd) / np.linalg.norm(fd)
    m = np.abs(fm - fd).max() / np.abs(fd).max()
    print(f"[mixed] full size {kind}: rel 2-norm {e:.3e}, max {m:.3e}", flush=True)
    assert 0.0 < e <= MIXED_TOL


def test_precision_switch_errors():
    v, t, tn, w = problem(2, 64, seed=3)
    tree = P.Tree(v, t, tn, P.default_params(m_t=3, m_x=3, n_max=8, operators=1), device=0)
    with pytest.raises(P.PfmmError) as e:
        tree.set_precision(P.MIXED_FP32)
    assert e.value.status == -1
    with pytest.raises(P.PfmmError):
        tree.set_precision(7)
    tree.set_precision(P.FP64)
    tree.close()


@pytest.mark.parametrize("kind", ["V", "K"])
def test_bf16_inputs_error_reported(kind):
    """BF16 moments / operator entries (exact products, FP32 accumulation): the
    error against FP64 is that of 8-bit significands; it is reported, and it is
    checked to lie between the FP32 mode's and a loose upper bound."""
    c = dict(CASES[1])
    n, E_t = c.pop("n"), c.pop("E_t")
    v, t, tn, w = problem(n, E_t, seed=23)
    op = 1 if kind == "V" else 2
    tree = P.Tree(v, t, tn, P.default_params(operators=op, precision=P.MIXED_BF16, **c), device=0)
    x = torch.from_numpy(w).to("cuda:0")
    fn = tree.apply_V if kind == "V" else tree.apply_K
    out = {}
    for name, code in (("fp64", P.FP64), ("fp32", P.MIXED_FP32), ("bf16", P.MIXED_BF16)):
        tree.set_precision(code)
        out[name] = fn(x).cpu().numpy()
    tree.close()
    e32 = np.linalg.norm(out["fp32"] - out["fp64"]) / np.linalg.norm(out["fp64"])
    e16 = np.linalg.norm(out["bf16"] - out["fp64"]) / np.linalg.norm(out["fp64"])
    print(f"[mixed] {kind}: rel 2-norm vs FP64: fp32 {e32:.3e}, bf16 {e16:.3e}", flush=True)
    assert np.all(np.isfinite(out["bf16"]))
    assert e32 <= MIXED_TOL
    assert 10 * e32 < e16 < 1e-2

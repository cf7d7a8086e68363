"""Parity on the 3072-triangle x 1024-step workload (3,145,728 DOFs, degrees
6/6, n_max 64, c_st 0.9, n_tr 5; the configuration bench.py times): one tree
holding the FP64 and the reduced-precision farfields, stored FP64 nearfield.

* FP64: sampled rows (32 random rows, the first and last steps, rows of the
  leaf level) against the oracle's rows at 1e-10 relative to the largest.
* FP32 farfield (FP32 M2L inputs and accumulation): relative 2-norm error
  against the FP64 apply on the same tree <= 1e-6 (the mixed-precision bar);
  the FP32 result's sampled rows against the oracle within the same bound.
* BF16-input farfield: relative 2-norm error against FP64 <= 1e-2.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_2106_15911_amd as P
from oracle.fmm import FMMOracle
from oracle.tree import Tree
from sampling import sample_rows
from workloads import config_problem

pytestmark = pytest.mark.gpu


def test_c3_parity_all_precisions():
    v, t, tn, c, w = config_problem(3)
    print(f"[parity-c3] build {len(t)} x {len(tn) - 1}", flush=True)
    tree = P.Tree(v, t, tn, P.default_params(operators=1, precision=P.MIXED_FP32), device=0)
    st = tree.stats()
    assert st["m2l_matrix_cores"] == 1 and st["near_entries_V"] == 12941813760
    x = torch.from_numpy(w).to("cuda:0")
    out = {}
    for name, prec in (("fp64", P.FP64), ("fp32", P.MIXED_FP32), ("bf16", P.MIXED_BF16)):
        tree.set_precision(prec)
        out[name] = tree.apply_V(x).cpu().numpy()
        print(f"[parity-c3] {name} apply done", flush=True)
    tree.close()
    f64 = out["fp64"]
    assert np.all(np.isfinite(f64))
    e32 = np.linalg.norm(out["fp32"] - f64) / np.linalg.norm(f64)
    e16 = np.linalg.norm(out["bf16"] - f64) / np.linalg.norm(f64)
    print(f"[parity-c3] fp32 vs fp64 {e32:.3e}, bf16 vs fp64 {e16:.3e}", flush=True)
    assert e32 <= 1e-6
    assert e16 <= 1e-2
    tr = Tree(v, t, tn, 1.0, c["n_max"], c["c_st"], c["n_tr"])
    o = FMMOracle(tr, c["m_t"], c["m_x"], "V")
    rows, levels = sample_rows(tr, 32)
    print(f"[parity-c3] oracle: {len(rows)} rows, leaf levels {levels}", flush=True)
    vals, _ = o.apply_rows(w, rows)
    scale = np.abs(vals).max()
    err = np.abs(f64[rows] - vals).max() / scale
    err32 = np.abs(out["fp32"][rows] - vals).max() / scale
    print(f"[parity-c3] fp64 rows max rel err {err:.3e}; fp32 rows {err32:.3e}", flush=True)
    assert err <= 1e-10
    assert err32 <= 1e-6

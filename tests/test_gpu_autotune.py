"""M2L autotuner (pfmm_autotune): timing the launch choices per level and
precision changes the product only by the summation order of list shares;
the cache written is a JSON object whose entries a second tree of the same
shape takes without timing."""
import json
import os
import tempfile

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_2106_15911_amd as P
from oracle_ref import problem

pytestmark = pytest.mark.gpu


def test_autotune_keeps_results_and_caches():
    v, t, tn, w = problem(4, 256, seed=31)
    prm = P.default_params(operators=1, m_t=4, m_x=4, precision=P.MIXED_FP32)
    print("[autotune] 192 x 256, m = 4", flush=True)
    tree = P.Tree(v, t, tn, prm, device=0)
    x = torch.from_numpy(w).to("cuda:0")
    before = {}
    for name, prec in (("fp64", P.FP64), ("fp32", P.MIXED_FP32)):
        tree.set_precision(prec)
        before[name] = tree.apply_V(x).cpu().numpy()
    with tempfile.TemporaryDirectory() as d:
        cache = os.path.join(d, "tune.json")
        n_t, n_c = tree.autotune(cache)
        print(f"[autotune] timed {n_t}, cached {n_c}", flush=True)
        assert n_t > 0 and n_c == 0
        entries = json.load(open(cache))
        assert len(entries) == n_t
        for k, e in entries.items():
            assert e["kernel"] in ("k_m2l_wide", "k_m2l_mfma") and e["shares"] >= 1 and e["ms"] > 0, (k, e)
        for name, prec in (("fp64", P.FP64), ("fp32", P.MIXED_FP32)):
            tree.set_precision(prec)
            after = tree.apply_V(x).cpu().numpy()
            d_ = np.abs(after - before[name]).max() / np.abs(before[name]).max()
            print(f"[autotune] {name}: max rel change {d_:.2e}", flush=True)
            assert d_ <= (1e-13 if name == "fp64" else 1e-6)
        tree.close()
        # a second tree of the same shape takes every choice from the cache
        tree2 = P.Tree(v, t, tn, prm, device=0)
        n_t2, n_c2 = tree2.autotune(cache)
        assert n_t2 == 0 and n_c2 == n_t
        tree2.set_precision(P.FP64)
        f2 = tree2.apply_V(x).cpu().numpy()
        tree2.close()
        tree.close()
        d2 = np.abs(f2 - before["fp64"]).max() / np.abs(before["fp64"]).max()
        assert d2 <= 1e-13

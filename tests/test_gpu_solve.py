"""GPU Dirichlet solve through the C ABI vs the oracle's GMRES.

The GPU solve (pfmm_solve_dirichlet / pfmm_solve_V: FP64 pFMM operators,
GMRES without restart, CGS2 Arnoldi on the GPU) is compared with the oracle's
GMRES (modified Gram-Schmidt) driven by the oracle pFMM operators on the same
tree, degrees and quadrature.  In exact arithmetic both produce the same
iterates; the operators agree to ~1e-15, so the iteration counts must agree
and the solutions within a small multiple of the stopping tolerance.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_2106_15911_amd as P
from oracle.dense import mass_diag, toeplitz_blocks
from oracle.fmm import FMMOracle
from oracle.solve import gmres, dirichlet_rhs
from oracle.tree import Tree
from oracle_ref import problem, rel_err
from workloads.dirichlet import project_source_datum

pytestmark = pytest.mark.gpu


def _oracle_ops(v, t, tn, m, n_max, n_tr, kinds=("V", "K")):
    E_t = len(tn) - 1
    h = tn[1] - tn[0]
    tr = Tree(v, t, tn, 1.0, n_max, 0.9, n_tr)
    out = {}
    for k in kinds:
        o = FMMOracle(tr, m, m, k)
        o.set_toeplitz_blocks(toeplitz_blocks(v, t, E_t, h, 1.0, k))
        out[k] = o
    return out


def test_dirichlet_solve_matches_oracle_gmres():
    print("[solve] dirichlet n=2 E_t=8 m=4 n_max=16 n_tr=-1", flush=True)
    v, t, tn, _ = problem(2, 8)
    g = project_source_datum(v, t, tn, (2.5, 0.0, 0.0), -0.1)
    ops = _oracle_ops(v, t, tn, 4, 16, -1)
    M = mass_diag(v, t, 8, tn[1] - tn[0])
    rhs = dirichlet_rhs(g, M, ops["K"].apply)
    x_ref, k_ref, hist_ref = gmres(ops["V"].apply, rhs, rtol=1e-10, max_iter=300)

    tree = P.Tree(v, t, tn, P.default_params(m_t=4, m_x=4, n_max=16, n_tr=-1), device=0)
    x, info = tree.solve_dirichlet(torch.from_numpy(g).to("cuda:0"), rtol=1e-10, max_iter=300)
    x = x.cpu().numpy()
    tree.close()
    assert info["converged"] and info["iters"] == k_ref, (info["iters"], k_ref)
    h = np.array(info["history"])
    assert len(h) == k_ref + 1
    # residual estimates agree while they are far above rounding
    big = np.array(hist_ref) > 1e-7
    assert np.allclose(h[big], np.array(hist_ref)[big], rtol=1e-6, atol=0)
    assert info["true_rel_residual"] <= 2e-10
    assert rel_err(x, x_ref) <= 1e-8, rel_err(x, x_ref)
    # the oracle operator confirms the residual of the GPU solution
    assert np.linalg.norm(rhs - ops["V"].apply(x)) / np.linalg.norm(rhs) <= 2e-10


def test_solve_V_c1_workload():
    """192 triangles x 16 steps, degrees 4/4, n_max 64, n_tr 5: V_h w = b for a random b."""
    print("[solve] V n=4 E_t=16 m=4", flush=True)
    v, t, tn, b = problem(4, 16, seed=1)
    tree = P.Tree(v, t, tn, P.default_params(m_t=4, m_x=4, operators=1), device=0)
    x, info = tree.solve_V(torch.from_numpy(b).to("cuda:0"), rtol=1e-8, max_iter=400)
    x = x.cpu().numpy()
    tree.close()
    assert info["converged"] and info["rel_residual"] <= 1e-8
    h = info["history"]
    assert all(h[i + 1] <= h[i] * (1 + 1e-12) for i in range(len(h) - 1))
    ops = _oracle_ops(v, t, tn, 4, 64, 5, kinds=("V",))
    r = np.linalg.norm(b - ops["V"].apply(x)) / np.linalg.norm(b)
    assert r <= 1.5e-8 and abs(r - info["true_rel_residual"]) <= 1e-12, (r, info["true_rel_residual"])


def test_solve_deterministic_and_errors():
    print("[solve] determinism / errors n=2 E_t=8", flush=True)
    v, t, tn, b = problem(2, 8, seed=3)
    prm = P.default_params(m_t=3, m_x=3, n_max=8)
    tree = P.Tree(v, t, tn, prm, device=0)
    bd = torch.from_numpy(b).to("cuda:0")
    x1, i1 = tree.solve_V(bd, rtol=1e-9)
    x2, i2 = tree.solve_V(bd, rtol=1e-9)
    assert torch.equal(x1, x2) and i1["history"] == i2["history"]
    # max_iter reached: PFMM_ENOTCONV, last iterate and info still returned
    with pytest.raises(P.PfmmError) as ex:
        tree.solve_V(bd, rtol=1e-12, max_iter=2)
    assert ex.value.status == -4
    x3, i3 = tree.solve_V(bd, rtol=1e-12, max_iter=2, raise_on_notconv=False)
    assert i3["iters"] == 2 and not i3["converged"] and i3["history"] == i1["history"][:3]
    # zero right-hand side: zero solution without iterations
    x0, i0 = tree.solve_V(torch.zeros_like(bd))
    assert i0["iters"] == 0 and float(x0.abs().max()) == 0.0
    # non-finite right-hand side
    bad = bd.clone()
    bad[5] = float("nan")
    with pytest.raises(P.PfmmError) as ex:
        tree.solve_V(bad)
    assert ex.value.status == -5
    # invalid options
    with pytest.raises(P.PfmmError) as ex:
        tree.solve_V(bd, max_iter=0)
    assert ex.value.status == -1
    tree.close()
    # Dirichlet solve needs K_h
    treeV = P.Tree(v, t, tn, P.default_params(m_t=3, m_x=3, n_max=8, operators=1), device=0)
    with pytest.raises(P.PfmmError) as ex:
        treeV.solve_dirichlet(bd)
    assert ex.value.status == -1
    treeV.close()


def test_split_trees_match_single_tree_dirichlet_solve():
    """RHS on a K-only tree + solve on a V-only tree equals the one-tree solve bitwise."""
    print("[solve] split trees n=2 E_t=8", flush=True)
    v, t, tn, _ = problem(2, 8)
    g = torch.from_numpy(project_source_datum(v, t, tn, (2.5, 0.0, 0.0), -0.1)).to("cuda:0")
    kw = dict(m_t=3, m_x=3, n_max=8)
    both = P.Tree(v, t, tn, P.default_params(**kw), device=0)
    x1, i1 = both.solve_dirichlet(g, rtol=1e-9)
    b1 = both.dirichlet_rhs(g)
    both.close()
    tk = P.Tree(v, t, tn, P.default_params(operators=2, **kw), device=0)
    b = tk.dirichlet_rhs(g)
    tk.close()
    tv = P.Tree(v, t, tn, P.default_params(operators=1, **kw), device=0)
    x2, i2 = tv.solve_V(b, rtol=1e-9)
    tv.close()
    assert torch.equal(b, b1)
    assert torch.equal(x1, x2) and i1["iters"] == i2["iters"]


def test_initial_iterate_and_resume():
    """Solve options: an initial iterate that already meets the tolerance is
    returned unchanged after 0 iterations; a solve stopped at max_iter and
    resumed in place from its last iterate reaches the same solution as an
    uninterrupted one (both to a relative residual of 1e-14 on a 384-DOF
    problem, where GMRES without restart ends within N steps)."""
    print("[solve] x0 / resume n=2 E_t=8", flush=True)
    v, t, tn, b = problem(2, 8, seed=4)
    tree = P.Tree(v, t, tn, P.default_params(m_t=3, m_x=3, n_max=8, operators=1), device=0)
    bd = torch.from_numpy(b).to("cuda:0")
    w, i1 = tree.solve_V(bd, rtol=1e-10)
    w_again, i0 = tree.solve_V(bd, rtol=1e-8, x0=w)
    print(f"[solve] from the solution: {i0['iters']} iterations, residual {i0['true_rel_residual']:.2e}", flush=True)
    assert i0["iters"] == 0 and i0["converged"] and torch.equal(w_again, w)
    assert i0["true_rel_residual"] <= 1e-8
    # interrupted + resumed (in place) vs uninterrupted
    n = len(b)
    w_full, i_full = tree.solve_V(bd, rtol=1e-14, max_iter=n)
    wk, ik = tree.solve_V(bd, rtol=1e-14, max_iter=10, raise_on_notconv=False)
    assert not ik["converged"] and ik["iters"] == 10
    w_res, i_res = tree.solve_V(bd, out=wk, rtol=1e-14, max_iter=n, x0=wk)
    d = (torch.linalg.norm(w_res - w_full) / torch.linalg.norm(w_full)).item()
    print(f"[solve] full {i_full['iters']} iterations; 10 + {i_res['iters']} resumed; diff {d:.2e}; "
          f"residuals {i_full['true_rel_residual']:.2e} {i_res['true_rel_residual']:.2e}", flush=True)
    assert i_res["converged"] and i_res["true_rel_residual"] <= 1e-13
    assert d <= 1e-12
    # the first history entry of the resumed solve is the relative residual of x0
    assert abs(i_res["history"][0] - ik["history"][-1]) <= 1e-6 * ik["history"][-1] + 1e-15
    # a non-finite initial iterate is rejected
    bad = w.clone()
    bad[3] = float("inf")
    with pytest.raises(P.PfmmError) as ex:
        tree.solve_V(bd, x0=bad)
    assert ex.value.status == -5
    tree.close()


def test_dirichlet_solve_with_preconditioner_options():
    """pfmm_solve_dirichlet with a preconditioner and FP32 inner applies
    (through the solve options) reaches the FP64 residual bar and the plain
    solution, and an initial iterate is honoured there too."""
    print("[solve] dirichlet + precond options n=3 E_t=64", flush=True)
    v, t, tn, _ = problem(3, 64)
    g = torch.from_numpy(project_source_datum(v, t, tn, (2.5, 0.0, 0.0), -0.1)).to("cuda:0")
    tree = P.Tree(v, t, tn, P.default_params(m_t=4, m_x=4, n_max=16, n_tr=3, precision=P.MIXED_FP32), device=0)
    tree.set_precision(P.FP64)
    w_ref, i_ref = tree.solve_dirichlet(g, rtol=1e-8, max_iter=300)
    pc = P.Precond(device=0, features=8, hidden=0)
    b = tree.dirichlet_rhs(g)
    pc.train(tree, b, n_snap=6, steps=0, batch=4096)
    w, info = tree.solve_dirichlet(g, rtol=1e-8, max_iter=300, precond=pc, inner_precision=P.MIXED_FP32)
    d = (torch.linalg.norm(w - w_ref) / torch.linalg.norm(w_ref)).item()
    print(f"[solve] plain {i_ref['iters']} iterations; preconditioned + FP32 inner {info['iters']} "
          f"({info['outer']} refinement steps), residual {info['true_rel_residual']:.2e}, diff {d:.2e}", flush=True)
    assert info["converged"] and info["true_rel_residual"] <= 1e-8 and not info["precond_fallback"]
    assert info["iters"] < i_ref["iters"]
    assert d <= 1e-5
    w2, info2 = tree.solve_dirichlet(g, rtol=1e-8, x0=w_ref, precond=pc)
    assert info2["iters"] == 0 and torch.equal(w2, w_ref)
    # FP32 inner applies need a mixed tree: a plain FP64 tree refuses them
    tk = P.Tree(v, t, tn, P.default_params(m_t=4, m_x=4, n_max=16, n_tr=3), device=0)
    with pytest.raises(P.PfmmError) as ex:
        tk.solve_dirichlet(g, inner_precision=P.MIXED_FP32)
    assert ex.value.status == -1
    tk.close()
    pc.close()
    tree.close()

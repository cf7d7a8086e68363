"""Learned temporal-block preconditioner: its inference kernel (both layers
in FP32) matches a float64 numpy evaluation of the same weights and
features to FP32 rounding (adjacency built here from the triangle list, the
diagonal of V_h from the oracle's panel integrals); training on pairs from
the library's own FP64 GMRES solves lowers the fit loss; FP64 iterative
refinement around flexible GMRES reaches the FP64 residual bar with and
without the preconditioner and with FP32 inner applies, the trained
preconditioner in use (no fallback) and fewer iterations than plain GMRES;
its solution matches plain GMRES; weights survive a save / load round trip;
useless, non-finite or overflowing weights trigger the fallback to plain
GMRES, which still meets the bar."""
import os
import tempfile

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_2106_15911_amd as P
from oracle.dense import panel_integrals
from oracle_ref import problem

pytestmark = pytest.mark.gpu
PRM = dict(m_t=4, m_x=4, n_max=16, n_tr=3)


def _tree(n, E_t, seed, precision=P.FP64):
    v, t, tn, w = problem(n, E_t, seed=seed)
    tree = P.Tree(v, t, tn, P.default_params(operators=1, precision=precision, **PRM), device=0)
    return tree, torch.from_numpy(w).to("cuda:0")


def _read_weights(path):
    raw = open(path, "rb").read()
    magic, version, FT, H = np.frombuffer(raw[:16], "<i4")
    assert magic == 0x4D4C5031 and version == 4
    w = np.frombuffer(raw[16:], "<f4").astype(np.float64)
    F = 3 * FT
    assert w.size == F + F * H + H * H + H
    c, w = w[:F], w[F:]
    return FT, c, w[:F * H].reshape(F, H), w[F * H:F * H + H * H].reshape(H, H), w[F * H + H * H:]


def _write_weights(path, FT, H, rng):
    """A weights file in the library's format with random stencil and perceptron."""
    F = 3 * FT
    c = rng.uniform(-0.5, 0.5, F)
    W1 = rng.uniform(-1, 1, (F, H)) * np.sqrt(6 / (F + H)) if H else np.zeros((F, 0))
    W2 = rng.uniform(-1, 1, (H, H)) * np.sqrt(3 / H) if H else np.zeros((0, 0))
    w3 = rng.uniform(-1, 1, H) * np.sqrt(6 / (H + 1)) if H else np.zeros(0)
    with open(path, "wb") as f:
        f.write(np.array([0x4D4C5031, 4, FT, H], "<i4").tobytes())
        for a in (c, W1, W2, w3):
            f.write(np.ascontiguousarray(a, "<f4").tobytes())


def _rings(tris):
    """Edge neighbours from undirected edges; second ring with multiplicity, without the triangle itself."""
    owners = {}
    for k, tr in enumerate(tris):
        for e in range(3):
            owners.setdefault(frozenset((int(tr[e]), int(tr[(e + 1) % 3]))), []).append(k)
    nb = [[] for _ in range(len(tris))]
    for ks in owners.values():
        assert len(ks) == 2
        nb[ks[0]].append(ks[1])
        nb[ks[1]].append(ks[0])
    second = [[q2 for q in nb[k] for q2 in nb[q] if q2 != k] for k in range(len(tris))]
    return nb, second


def _mlp_ref(path, v, tris, D, E_t):
    """c . x + N(x) in float64 from the file's FP32 weights.  The kernel runs
    both layers in FP32 (FP32 features, FP32 matrix-core products and
    accumulation, tanh through the hardware exponential), so the two agree to
    FP32 rounding."""
    FT, cl, W1, W2, w3 = _read_weights(path)
    ex = len(tris)
    u = v.reshape(E_t, ex) / D[None, :]
    s = np.sqrt(np.mean(u * u))
    u = u / s
    nb, second = _rings(tris)
    r1 = np.stack([u[:, nb[k]].mean(axis=1) for k in range(ex)], axis=1)
    r2 = np.stack([u[:, second[k]].mean(axis=1) for k in range(ex)], axis=1)
    X = np.zeros((E_t, ex, 3 * FT))
    for f in range(FT):
        for ring, a in enumerate((u, r1, r2)):
            X[f:, :, 3 * f + ring] = a[:E_t - f]
    z = np.tanh(np.tanh(X @ W1) @ W2) @ w3 + X @ cl
    return s * z.reshape(-1)


def test_inference_matches_numpy(tmp_path):
    n, E_t = 3, 64
    print(f"[precond] inference parity n={n} E_t={E_t}", flush=True)
    v, t, tn, w = problem(n, E_t, seed=65)
    tree = P.Tree(v, t, tn, P.default_params(operators=1, **PRM), device=0)
    h = (tn[-1] - tn[0]) / E_t
    ks = np.arange(len(t))
    D = panel_integrals(v, t, ks, ks, 0, h, 1.0)[:, 0]
    rng = np.random.default_rng(14)
    for FT, H in ((1, 8), (6, 64), (8, 256), (8, 0), (3, 0)):
        path = tmp_path / f"pc_{FT}_{H}.bin"
        _write_weights(path, FT, H, rng)
        pc = P.Precond(device=0, path=path)
        z = pc.apply(tree, torch.from_numpy(w).to("cuda:0")).cpu().numpy()
        ref = _mlp_ref(path, w, t, D, E_t)
        d = np.abs(z - ref)
        zmax = np.max(np.abs(ref))
        print(f"[precond] features {FT} hidden {H}: max error {np.max(d) / zmax:.2e}, median "
              f"{np.median(d) / zmax:.2e}", flush=True)
        # FP32 features and two FP32 layers of width <= 256: a few FP32 ulps
        # per accumulated term
        assert np.max(d) <= 2e-5 * zmax
        assert np.median(d) <= 1e-6 * zmax
        pc.close()
    tree.close()


def test_training_lowers_the_loss_and_solves_converge():
    print("[precond] train + solve", flush=True)
    tree_a, b_a = _tree(2, 256, 61)
    pc = P.Precond(device=0, features=8, hidden=64, seed=3)
    l0 = pc.train(tree_a, b_a, n_snap=6, steps=1, batch=2048, lr=1e-3)
    l1 = pc.train(tree_a, b_a, n_snap=6, steps=400, batch=2048, lr=1e-3)
    print(f"[precond] loss after 1 step {l0:.4e}, after 400 more {l1:.4e}", flush=True)
    assert np.isfinite(l1) and l1 < l0
    tree_a.close()
    # a different problem (mesh and steps) with the mixed farfield available
    tree, b = _tree(3, 128, 62, precision=P.MIXED_FP32)
    w_ref, i_ref = tree.solve_V(b, rtol=1e-8, max_iter=300)
    for label, pcx, inner in (("none", None, P.FP64), ("learned", pc, P.FP64), ("learned+fp32", pc, P.MIXED_FP32)):
        w, info = tree.solve_V_precond(b, precond=pcx, inner_precision=inner, rtol=1e-8, max_iter=300)
        d = (torch.linalg.norm(w - w_ref) / torch.linalg.norm(w_ref)).item()
        print(f"[precond] {label}: {info['iters']} inner iterations, {info['outer']} refinement steps, "
              f"fallback {info['precond_fallback']}, residual {info['true_rel_residual']:.2e}, "
              f"diff to plain GMRES {d:.2e} (plain: {i_ref['iters']} iterations)", flush=True)
        assert info["converged"] and info["true_rel_residual"] <= 1e-8
        assert d <= 1e-5
        if pcx is not None:
            # the learned preconditioner is used, not bypassed, and pays off
            assert not info["precond_fallback"]
            assert info["iters"] < i_ref["iters"]
    # the stencil alone (hidden width 0) is deterministic and converges too
    st0 = P.Precond(device=0, features=8, hidden=0, seed=1)
    tree_b, b_b = _tree(2, 256, 61)
    l_s = st0.train(tree_b, b_b, n_snap=6, steps=0, batch=4096)
    tree_b.close()
    w0, i0 = tree.solve_V_precond(b, precond=st0, rtol=1e-8, max_iter=300)
    print(f"[precond] stencil alone: fit residual {l_s:.3e}, {i0['iters']} inner iterations", flush=True)
    assert np.isfinite(l_s) and i0["converged"] and i0["true_rel_residual"] <= 1e-8
    st0.close()
    # save / load: the same weights give the same iterations
    with tempfile.TemporaryDirectory() as td:
        path = os.path.join(td, "pc.bin")
        pc.save(path)
        pc2 = P.Precond(device=0, path=path)
        w1, i1 = tree.solve_V_precond(b, precond=pc, rtol=1e-8, max_iter=300)
        w2, i2 = tree.solve_V_precond(b, precond=pc2, rtol=1e-8, max_iter=300)
        assert i1["iters"] == i2["iters"] and torch.equal(w1, w2)
        pc2.close()
    pc.close()
    tree.close()


def test_precond_errors():
    tree, b = _tree(2, 32, 63)
    with pytest.raises(P.PfmmError):
        P.Precond(device=0, features=0)
    with pytest.raises(P.PfmmError):
        P.Precond(device=0, hidden=4096)
    with pytest.raises(P.PfmmError) as e:   # FP32 inner applies need a mixed tree
        tree.solve_V_precond(b, inner_precision=P.MIXED_FP32)
    assert e.value.status == -1
    with pytest.raises(P.PfmmError):
        P.Precond(device=0, path="/nonexistent/pc.bin")
    tree.close()


@pytest.mark.parametrize("kind", ["zero", "nan", "overflow"])
def test_forced_fallback_still_converges(tmp_path, kind):
    """A preconditioner whose output is useless (all weights zero: z = 0) or
    non-finite (NaN weights; weights of 3e38, whose FP32 sums overflow) must
    not break the solve: the refinement detects it, falls back to plain
    FP64 GMRES from the current iterate, and still meets the FP64 bar."""
    print(f"[precond] forced fallback: {kind}", flush=True)
    tree, b = _tree(3, 64, 66)
    FT, H = 4, 64
    path = tmp_path / f"bad_{kind}.bin"
    F = 3 * FT
    val = {"zero": 0.0, "nan": np.nan, "overflow": 3e38}[kind]
    with open(path, "wb") as f:
        f.write(np.array([0x4D4C5031, 4, FT, H], "<i4").tobytes())
        f.write(np.full(F + F * H + H * H + H, val, "<f4").tobytes())
    pc = P.Precond(device=0, path=path)
    w_ref, i_ref = tree.solve_V(b, rtol=1e-8, max_iter=300)
    w, info = tree.solve_V_precond(b, precond=pc, rtol=1e-8, max_iter=300)
    d = (torch.linalg.norm(w - w_ref) / torch.linalg.norm(w_ref)).item()
    print(f"[precond] {kind}: fallback {info['precond_fallback']}, {info['iters']} iterations, "
          f"residual {info['true_rel_residual']:.2e}, diff to plain {d:.2e}", flush=True)
    assert info["precond_fallback"]
    assert info["converged"] and info["true_rel_residual"] <= 1e-8
    assert torch.all(torch.isfinite(w))
    assert d <= 1e-5
    # the same file through the solve options (loaded for the call)
    w2, info2 = tree.solve_V(b, precond_path=path, rtol=1e-8, max_iter=300)
    assert info2["precond_fallback"] and info2["converged"] and info2["true_rel_residual"] <= 1e-8
    pc.close()
    tree.close()

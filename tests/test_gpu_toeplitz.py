"""Toeplitz nearfield mode (no stored blocks; entries read from the distinct
integrals per (leaf spatial box, step difference)) against the CPU oracle and
against the stored-block mode on the same tree.

The stored blocks are copies of the same distinct values.  Groups whose
leaves are time translates run as GEMMs on the matrix cores (another
summation order: the modes agree to 1e-13 relative); the others, and all
groups with nearfield_gemm = 0, use a kernel with the stored mode's order
(bit for bit equal).  Against the oracle the FP64 bar (1e-10 relative)
applies."""
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
TOL_MODES = 1e-13   # Toeplitz vs stored: same terms, FP64, summation order of the GEMM path


def _mode_diff(a, b):
    return float((a - b).abs().max() / b.abs().max())


def _apply(v, t, tn, w, kind, mode, gemm=1, **prm):
    op = 1 if kind == "V" else 2
    tree = P.Tree(v, t, tn, P.default_params(operators=op, nearfield_mode=mode, nearfield_gemm=gemm, **prm), device=0)
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
    fv, st_v = _apply(v, t, tn, w, kind, P.NF_TOEPLITZ, gemm=0, **c)
    assert st_v["near_gemm_groups"] == 0 and torch.equal(fv, fs)
    dm = _mode_diff(ft, fs)
    print(f"[toeplitz] GEMM groups {st_t['near_gemm_groups']}, leaves {st_t['leaves']}: "
          f"max rel diff to stored {dm:.2e}", flush=True)
    assert dm <= TOL_MODES
    assert st_s["near_gemm_groups"] == 0
    assert st_t["device_bytes"] < st_s["device_bytes"]
    r = reference(v, t, tn, w, kind, **c)
    g = ft.numpy()
    e = rel_err(g, r)
    m = float(np.abs(g - r).max() / np.abs(r).max())
    assert e <= TOL and m <= TOL, (e, m)


@pytest.mark.parametrize("n,E_t,n_max", [(4, 64, 4), (6, 128, 8), (8, 64, 16), (4, 256, 64)])
def test_stored_bitwise_equal_to_toeplitz_vector_kernel(n, E_t, n_max):
    """Leaves of 1 to 64 triangles (n_max from 4 to 64): the stored-block
    product (densities staged per wave in LDS) and the Toeplitz matrix-vector
    kernel (one density gather per lane and column) take the same products
    in the same order, so they agree bit for bit, V and K."""
    print(f"[toeplitz] stored vs vector kernel n={n} E_t={E_t} n_max={n_max}", flush=True)
    v, t, tn, w = problem(n, E_t, seed=29)
    for kind in ("V", "K"):
        fs, _ = _apply(v, t, tn, w, kind, P.NF_STORED, m_t=3, m_x=3, n_max=n_max)
        fv, st = _apply(v, t, tn, w, kind, P.NF_TOEPLITZ, gemm=0, m_t=3, m_x=3, n_max=n_max)
        assert st["near_gemm_groups"] == 0
        assert torch.equal(fs, fv), (kind, _mode_diff(fs, fv))


def test_toeplitz_full_size():
    """3072 triangles x 256 steps, degrees 6/6: equal to the stored mode to
    1e-13 (GEMM path in use) and bit for bit with nearfield_gemm = 0, sampled
    rows against the oracle, and without the 53.8 GB of blocks."""
    print("[toeplitz] full size", flush=True)
    v, t, tn, c, w = config_problem(2)
    ft, st_t = _apply(v, t, tn, w, "V", P.NF_TOEPLITZ)
    fs, st_s = _apply(v, t, tn, w, "V", P.NF_STORED)
    fv, _ = _apply(v, t, tn, w, "V", P.NF_TOEPLITZ, gemm=0)
    assert torch.equal(fv, fs)   # same products, same order per lane
    dm = _mode_diff(ft, fs)
    print(f"[toeplitz] full size: GEMM groups {st_t['near_gemm_groups']}: max rel diff to stored {dm:.2e}", flush=True)
    assert dm <= TOL_MODES and st_t["near_gemm_groups"] > 0
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


@pytest.mark.parametrize("n,E_t,n_max,n_tr", [(4, 40, 32, 2), (8, 24, 64, 3)])
def test_gemm_ragged_step_blocks(n, E_t, n_max, n_tr):
    """Step counts that are not multiples of the GEMM's 16-step blocks (the
    last block has lanes past the final step, whose densities shift into no
    valid lane): the GEMM path equals the matrix-vector kernel (bit for bit
    the stored mode) to 1e-13, V and K."""
    print(f"[toeplitz] ragged blocks n={n} E_t={E_t} n_max={n_max} n_tr={n_tr}", flush=True)
    v, t, tn, w = problem(n, E_t, seed=31)
    for kind in ("V", "K"):
        ft, st = _apply(v, t, tn, w, kind, P.NF_TOEPLITZ, m_t=3, m_x=3, n_max=n_max, n_tr=n_tr)
        fv, _ = _apply(v, t, tn, w, kind, P.NF_TOEPLITZ, gemm=0, m_t=3, m_x=3, n_max=n_max, n_tr=n_tr)
        dm = _mode_diff(ft, fv)
        print(f"[toeplitz] {kind}: GEMM groups {st['near_gemm_groups']}, max rel diff {dm:.2e}", flush=True)
        assert st["near_gemm_groups"] > 0
        assert dm <= TOL_MODES


def test_gemm_solve_workload():
    """12,288 triangles x 512 steps, n_tr = 3 (the Dirichlet solve's tree,
    whose largest leaf boxes need two 16-row tiles): the GEMM path against
    the matrix-vector kernel (1e-13) and sampled rows, from both leaf levels
    and the first and last steps, against the oracle (1e-10)."""
    from sampling import sample_rows
    print("[toeplitz] 12,288 x 512, n_tr = 3", flush=True)
    v, t, tn, c, w = config_problem(5)
    prm = dict(m_t=c["m_t"], m_x=c["m_x"], n_max=c["n_max"], c_st=c["c_st"], n_tr=c["n_tr"])
    ft, st = _apply(v, t, tn, w, "V", P.NF_TOEPLITZ, **prm)
    fv, _ = _apply(v, t, tn, w, "V", P.NF_TOEPLITZ, gemm=0, **prm)
    dm = _mode_diff(ft, fv)
    print(f"[toeplitz] GEMM groups {st['near_gemm_groups']}: max rel diff to the vector kernel {dm:.2e}", flush=True)
    assert st["near_gemm_groups"] > 0 and dm <= TOL_MODES
    tr = Tree(v, t, tn, 1.0, c["n_max"], c["c_st"], c["n_tr"])
    rows, levels = sample_rows(tr, 4, per_level=2)
    vals, _ = FMMOracle(tr, c["m_t"], c["m_x"], "V").apply_rows(w, rows)
    f = ft.numpy()
    err = np.abs(f[rows] - vals).max() / np.abs(vals).max()
    print(f"[toeplitz] {len(rows)} rows (leaf levels {levels}): max rel err {err:.3e}", flush=True)
    assert err <= TOL


@pytest.mark.parametrize("n,E_t,n_max,n_tr", [(4, 23, 16, 2), (4, 45, 32, 3)])
def test_gemm_unequal_leaves(n, E_t, n_max, n_tr):
    """Step counts whose time tree has leaves of unequal lengths (the split at
    the step nearest the midpoint, Algorithm 1): the GEMM path, with per-leaf
    source ranges and leaf starts, equals the matrix-vector kernel to 1e-13
    and the dense oracle to 1e-10, V and K."""
    print(f"[toeplitz] unequal leaves n={n} E_t={E_t} n_max={n_max} n_tr={n_tr}", flush=True)
    v, t, tn, w = problem(n, E_t, seed=37)
    prm = dict(m_t=3, m_x=3, n_max=n_max, n_tr=n_tr)
    for kind in ("V", "K"):
        ft, st = _apply(v, t, tn, w, kind, P.NF_TOEPLITZ, **prm)
        fv, _ = _apply(v, t, tn, w, kind, P.NF_TOEPLITZ, gemm=0, **prm)
        dm = _mode_diff(ft, fv)
        r = reference(v, t, tn, w, kind, **prm)
        e = float(np.abs(ft.numpy() - r).max() / np.abs(r).max())
        print(f"[toeplitz] {kind}: GEMM groups {st['near_gemm_groups']}, diff to vector kernel {dm:.2e}, "
              f"max rel err vs dense {e:.2e}", flush=True)
        assert st["near_gemm_groups"] > 0
        assert dm <= TOL_MODES and e <= TOL


def test_gemm_unequal_leaves_larger_tree():
    """3072 triangles x 479 steps (leaves of 3 and 4 steps, as in the batch's
    largest drawn problems): GEMM path against the matrix-vector kernel
    (1e-13) and sampled rows against the oracle (1e-10)."""
    from sampling import sample_rows
    from workloads import cube_surface_mesh, densities, uniform_time_nodes
    print("[toeplitz] 3072 x 479", flush=True)
    v, t = cube_surface_mesh(16)
    tn = uniform_time_nodes(479)
    w = densities(479 * len(t), 11)
    prm = dict(m_t=4, m_x=4, n_max=64, n_tr=5)
    ft, st = _apply(v, t, tn, w, "V", P.NF_TOEPLITZ, **prm)
    fv, _ = _apply(v, t, tn, w, "V", P.NF_TOEPLITZ, gemm=0, **prm)
    dm = _mode_diff(ft, fv)
    print(f"[toeplitz] GEMM groups {st['near_gemm_groups']}: max rel diff to the vector kernel {dm:.2e}", flush=True)
    assert st["near_gemm_groups"] > 0 and dm <= TOL_MODES
    tr = Tree(v, t, tn, 1.0, prm["n_max"], 0.9, prm["n_tr"])
    rows, levels = sample_rows(tr, 4, per_level=2)
    vals, _ = FMMOracle(tr, prm["m_t"], prm["m_x"], "V").apply_rows(w, rows)
    err = np.abs(ft.numpy()[rows] - vals).max() / np.abs(vals).max()
    print(f"[toeplitz] {len(rows)} rows (leaf levels {levels}): max rel err {err:.3e}", flush=True)
    assert err <= TOL

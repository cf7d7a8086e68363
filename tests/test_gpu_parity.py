"""GPU parity: the HIP path through the C ABI vs the CPU FP64 oracle.

Bar (FP64 mode): relative 2-norm error <= 1e-10 and max-abs error
<= 1e-10 * max|f| against the oracle pFMM product on the same seeded input.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_2106_15911_amd as P
from oracle_ref import problem, reference, rel_err

pytestmark = pytest.mark.gpu
TOL = 1e-10


def _gpu_apply(v, t, tn, w, kind, **prm):
    tree = P.Tree(v, t, tn, P.default_params(**prm), device=0)
    x = torch.from_numpy(w).to("cuda:0")
    f = tree.apply_V(x) if kind == "V" else tree.apply_K(x)
    torch.cuda.synchronize()
    out = f.cpu().numpy()
    tree.close()
    return out


def _check(g, r):
    assert np.all(np.isfinite(g))
    e = rel_err(g, r)
    m = float(np.abs(g - r).max() / np.abs(r).max())
    assert e <= TOL and m <= TOL, (e, m)


@pytest.mark.parametrize("kind", ["V", "K"])
def test_c1_workload(kind):
    """192 triangles x 16 steps, degrees 4/4, n_max 64, c_st 0.9, n_tr 5."""
    print(f"[parity] c1 kind={kind}", flush=True)
    v, t, tn, w = problem(4, 16, seed=1)
    g = _gpu_apply(v, t, tn, w, kind, m_t=4, m_x=4)
    r = reference(v, t, tn, w, kind, m_t=4, m_x=4)
    _check(g, r)


@pytest.mark.parametrize("case", [
    dict(n=2, E_t=8, m_t=3, m_x=3, n_max=8, n_tr=-1, alpha=1.0, T=1.0),
    dict(n=2, E_t=16, m_t=2, m_x=5, n_max=12, n_tr=1, alpha=0.5, T=0.5),
    dict(n=2, E_t=32, m_t=5, m_x=2, n_max=16, n_tr=-1, alpha=2.0, T=2.0),
])
@pytest.mark.parametrize("kind", ["V", "K"])
def test_variants(case, kind):
    print(f"[parity] variant {case} kind={kind}", flush=True)
    c = dict(case)
    v, t, tn, w = problem(c.pop("n"), c.pop("E_t"), T=c.pop("T"), seed=7)
    g = _gpu_apply(v, t, tn, w, kind, **c)
    r = reference(v, t, tn, w, kind, **c)
    _check(g, r)


def test_deterministic_and_errors():
    print("[parity] determinism", flush=True)
    v, t, tn, w = problem(4, 16, seed=3)
    tree = P.Tree(v, t, tn, P.default_params(m_t=4, m_x=4, operators=1), device=0)
    x = torch.from_numpy(w).to("cuda:0")
    a = tree.apply_V(x)
    b = tree.apply_V(x)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    with pytest.raises(P.PfmmError) as e:
        tree.apply_K(x)
    assert e.value.status == -1
    with pytest.raises(ValueError):
        tree.apply_V(x[:-1])
    tree.close()


@pytest.mark.parametrize("mode", ["stored", "toeplitz"])
def test_nearfield_beside_farfield_equals_in_order(mode):
    """The default apply (Toeplitz mode: nearfield on a side stream; stored
    mode: in order) and the in-order apply with stage timing on give bitwise
    equal results, for V and K, on a tree with a deep farfield (m = 6,
    matrix-core M2L on several levels)."""
    print(f"[parity] side-stream nearfield vs in order, {mode}", flush=True)
    v, t, tn, w = problem(6, 128, seed=9)
    nf = P.NF_TOEPLITZ if mode == "toeplitz" else P.NF_STORED
    tree = P.Tree(v, t, tn, P.default_params(m_t=6, m_x=6, operators=3, nearfield_mode=nf), device=0)
    x = torch.from_numpy(w).to("cuda:0")
    a, c = tree.apply_V(x), tree.apply_K(x)
    tree.profile_enable(True)
    b, d = tree.apply_V(x), tree.apply_K(x)
    tree.profile_enable(False)
    torch.cuda.synchronize()
    assert torch.equal(a, b) and torch.equal(c, d)
    tree.close()


@pytest.mark.parametrize("kind", ["V", "K"])
def test_c1_mesh_degree6_matrix_cores(kind):
    """Degrees 6/6 on the 192 x 16 mesh: exercises the FP64 matrix-core M2L
    (split-K segments, split interaction lists) against the oracle."""
    print(f"[parity] c1 m=6 kind={kind}", flush=True)
    v, t, tn, w = problem(4, 16, seed=5)
    tree = P.Tree(v, t, tn, P.default_params(m_t=6, m_x=6), device=0)
    assert tree.stats()["m2l_matrix_cores"] == 1
    x = torch.from_numpy(w).to("cuda:0")
    g = (tree.apply_V(x) if kind == "V" else tree.apply_K(x)).cpu().numpy()
    tree.close()
    r = reference(v, t, tn, w, kind, m_t=6, m_x=6)
    _check(g, r)


def test_vector_unit_m2l_above_matrix_core_limits():
    """Degrees 7/7 exceed the LDS budget of the matrix-core M2L; the vector-unit
    M2L with explicit operators must give the same product as the oracle."""
    print("[parity] m=7 vector-unit M2L", flush=True)
    v, t, tn, w = problem(2, 8, seed=9)
    prm = dict(m_t=7, m_x=7, n_max=8, n_tr=-1)
    tree = P.Tree(v, t, tn, P.default_params(**prm), device=0)
    assert tree.stats()["m2l_matrix_cores"] == 0
    x = torch.from_numpy(w).to("cuda:0")
    g = tree.apply_V(x).cpu().numpy()
    tree.close()
    _check(g, reference(v, t, tn, w, "V", **prm))

"""The no-allocation preconditioner application (pfmm_precond_apply_noalloc,
for callers that cannot allocate device memory) against the allocating
pfmm_precond_apply on the same inputs: two calls in a row on one device, the
second on a smaller tree, each equal to the allocating entry point's result.
Both run the same kernels on the same inputs, so the results are bitwise
equal; the bar of the kernels' own parity tests (1e-12 relative) is checked
as well for the message."""
import os
import tempfile

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_2106_15911_amd as P
from oracle_ref import problem

pytestmark = pytest.mark.gpu
PRM = dict(m_t=4, m_x=4, n_max=16, n_tr=3)


def _weights(path, FT, H, seed):
    """A weights file in the library's format with a random stencil and perceptron."""
    rng = np.random.default_rng(seed)
    F = 3 * FT
    c = rng.uniform(-0.5, 0.5, F)
    W1 = rng.uniform(-1, 1, (F, H)) * np.sqrt(6 / (F + H))
    W2 = rng.uniform(-1, 1, (H, H)) * np.sqrt(3 / H)
    w3 = rng.uniform(-1, 1, H) * np.sqrt(6 / (H + 1))
    with open(path, "wb") as f:
        f.write(np.array([0x4D4C5031, 4, FT, H], "<i4").tobytes())
        for a in (c, W1, W2, w3):
            f.write(np.ascontiguousarray(a, "<f4").tobytes())


@pytest.mark.parametrize("hidden", [0, 64])
def test_noalloc_matches_allocating_entry_point(hidden):
    dev = "cuda:0"
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "w.bin")
        _weights(path, 8, hidden if hidden else 1, 3)
        if hidden == 0:
            # the stencil alone: rewrite with hidden width 0
            raw = np.fromfile(path, "<f4", offset=16)[:24]
            with open(path, "wb") as f:
                f.write(np.array([0x4D4C5031, 4, 8, 0], "<i4").tobytes())
                f.write(raw.astype("<f4").tobytes())
        pc = P.Precond(device=0, path=path)
    try:
        # two calls in a row, the second on a smaller tree (fewer DOFs)
        for n, E_t, seed in ((4, 32, 21), (2, 8, 22)):
            v, t, tn, w = problem(n, E_t, seed=seed)
            print(f"[noalloc] hidden={hidden} mesh n={n} steps={E_t} dofs={len(w)}", flush=True)
            tree = P.Tree(v, t, tn, P.default_params(operators=1, **PRM), device=0)
            x = torch.from_numpy(w).to(dev)
            z_ref = pc.apply(tree, x)
            z = torch.full_like(x, float("nan"))
            pc.apply_noalloc(tree, x, z)
            torch.cuda.synchronize()
            zr, zn = z_ref.cpu().numpy(), z.cpu().numpy()
            assert np.all(np.isfinite(zn))
            err = np.abs(zn - zr).max() / np.abs(zr).max()
            print(f"[noalloc] max rel diff {err:.3e}", flush=True)
            assert err <= 1e-12
            assert np.array_equal(zn, zr)
            tree.close()
    finally:
        pc.close()

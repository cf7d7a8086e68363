"""Batched applies: independent problems applied in one captured HIP graph
must give, bit for bit, what each tree's own apply gives; the graph is
replayed several times with eager work in between (every replay checked),
re-captured when the vectors change, and rejects misuse."""
import pytest

torch = pytest.importorskip("torch")

import paper_2106_15911_amd as P
from oracle_ref import problem

pytestmark = pytest.mark.gpu

SIZES = [(4, 32, dict(m_t=4, m_x=4)), (2, 64, dict(m_t=3, m_x=3, n_max=8)), (3, 16, dict(m_t=4, m_x=4)),
         (2, 16, dict(m_t=2, m_x=5, n_max=12, n_tr=1))]


def _trees(mode):
    trees, ws = [], []
    for i, (n, E_t, prm) in enumerate(SIZES):
        v, t, tn, w = problem(n, E_t, seed=50 + i)
        trees.append(P.Tree(v, t, tn, P.default_params(operators=1, nearfield_mode=mode, **prm), device=0))
        ws.append(torch.from_numpy(w).to("cuda:0"))
    return trees, ws


@pytest.mark.parametrize("mode", [P.NF_STORED, P.NF_TOEPLITZ])
def test_batch_matches_single_applies(mode):
    print(f"[batch] nearfield mode {mode}", flush=True)
    trees, ws = _trees(mode)
    ref = [t.apply_V(w) for t, w in zip(trees, ws)]
    torch.cuda.synchronize()
    b = P.Batch(trees)
    outs = [torch.empty_like(w) for w in ws]
    for rep in range(4):
        for y in outs:
            y.fill_(float("nan"))
        b.apply_V(ws, outs)
        torch.cuda.synchronize()
        for r, y in zip(ref, outs):
            assert torch.equal(r, y), rep
        # eager work between replays
        z = trees[0].apply_V(ws[0])
        torch.cuda.synchronize()
        assert torch.equal(z, ref[0])
    # new output tensors: re-captured graph, same results
    outs2 = b.apply_V(ws)
    torch.cuda.synchronize()
    for r, y in zip(ref, outs2):
        assert torch.equal(r, y)
    b.close()
    for t in trees:
        t.close()


def test_batch_errors():
    trees, ws = _trees(P.NF_TOEPLITZ)
    with pytest.raises(P.PfmmError):
        P.Batch([trees[0], trees[0]])
    b = P.Batch(trees[:2])
    trees[1].profile_enable(True)
    with pytest.raises(P.PfmmError) as e:
        b.apply_V(ws[:2])
    assert e.value.status == -1
    trees[1].profile_enable(False)
    with pytest.raises(ValueError):
        b.apply_V(ws[:1])
    b.close()
    for t in trees:
        t.close()


def test_batch_recaptures_on_precision_change():
    """A batch captured while its trees ran the FP32 farfield must not keep
    replaying FP32 after the trees are switched back to FP64."""
    print("[batch] precision change", flush=True)
    trees, ws = [], []
    for i, (n, E_t) in enumerate(((4, 64), (2, 64))):
        v, t, tn, w = problem(n, E_t, seed=70 + i)
        trees.append(P.Tree(v, t, tn, P.default_params(operators=1, m_t=4, m_x=4, n_max=16,
                                                       precision=P.MIXED_FP32), device=0))
        ws.append(torch.from_numpy(w).to("cuda:0"))
    ref64 = []
    for t, w in zip(trees, ws):
        t.set_precision(P.FP64)
        ref64.append(t.apply_V(w))
        t.set_precision(P.MIXED_FP32)
    ref32 = [t.apply_V(w) for t, w in zip(trees, ws)]
    torch.cuda.synchronize()
    b = P.Batch(trees)
    outs = [torch.empty_like(w) for w in ws]
    b.apply_V(ws, outs)
    torch.cuda.synchronize()
    assert all(torch.equal(r, y) for r, y in zip(ref32, outs))
    for t in trees:
        t.set_precision(P.FP64)
    b.apply_V(ws, outs)        # same vectors, new precision: must re-capture
    torch.cuda.synchronize()
    assert all(torch.equal(r, y) for r, y in zip(ref64, outs))
    assert not all(torch.equal(r, y) for r, y in zip(ref32, outs))
    b.close()
    for t in trees:
        t.close()


def test_batch_matches_oracle():
    """Every batched result against the CPU oracle pFMM on the same tree
    (face grids of 3 and 5 squares: cube boxes that do not align with the
    squares, so the padded boxes of Algorithm 1 are exercised; 21 steps:
    time levels with intervals of different lengths)."""
    import numpy as np
    from oracle_ref import reference, rel_err
    cases = [(3, 24, dict(m_t=4, m_x=4, n_max=16, n_tr=2)), (5, 8, dict(m_t=3, m_x=3, n_max=32, n_tr=3)),
             (2, 32, dict(m_t=3, m_x=3, n_max=8, n_tr=-1)),
             # a step count whose time levels split unevenly
             (3, 21, dict(m_t=3, m_x=3, n_max=16, n_tr=2))]
    trees, ws, refs = [], [], []
    for i, (n, E_t, prm) in enumerate(cases):
        v, t, tn, w = problem(n, E_t, seed=80 + i)
        print(f"[batch-oracle] n={n} E_t={E_t} {prm}", flush=True)
        trees.append(P.Tree(v, t, tn, P.default_params(operators=1, nearfield_mode=P.NF_TOEPLITZ, **prm), device=0))
        ws.append(torch.from_numpy(w).to("cuda:0"))
        refs.append(reference(v, t, tn, w, "V", **prm))
    b = P.Batch(trees)
    outs = b.apply_V(ws)
    torch.cuda.synchronize()
    for (n, E_t, _), y, r in zip(cases, outs, refs):
        e = rel_err(y.cpu().numpy(), r)
        print(f"[batch-oracle] n={n} E_t={E_t}: rel err {e:.3e}", flush=True)
        assert np.isfinite(e) and e <= 1e-10
    b.close()
    for t in trees:
        t.close()


@pytest.mark.parametrize("mode", [P.NF_STORED, P.NF_TOEPLITZ])
def test_cross_problem_m2l_equals_single_applies(mode):
    """Trees with unequal time intervals (21, 37, 47 and 70 steps) and one
    with equal ones: the batch's cross-problem M2L launch gives, bit for bit,
    each tree's own apply, in FP64 and with the FP32 farfield, and so does
    the batch with the cross-problem launch switched off."""
    sizes = [(3, 21, dict(m_t=4, m_x=4, n_max=16)), (2, 37, dict(m_t=4, m_x=4, n_max=8)),
             (4, 47, dict(m_t=4, m_x=4)), (2, 70, dict(m_t=4, m_x=4, n_max=8, n_tr=-1)),
             (4, 32, dict(m_t=4, m_x=4))]
    trees, ws = [], []
    for i, (n, E_t, prm) in enumerate(sizes):
        v, t, tn, w = problem(n, E_t, seed=60 + i)
        trees.append(P.Tree(v, t, tn, P.default_params(operators=1, nearfield_mode=mode, precision=P.MIXED_FP32,
                                                       **prm), device=0))
        ws.append(torch.from_numpy(w).to("cuda:0"))
    print(f"[batch-xm] mode {mode}: time classes {[tr.stats()['n_time_classes'] for tr in trees]}", flush=True)
    b = P.Batch(trees)
    for prec in (P.FP64, P.MIXED_FP32):
        for tr in trees:
            tr.set_precision(prec)
        ref = [tr.apply_V(w) for tr, w in zip(trees, ws)]
        torch.cuda.synchronize()
        for cross in (True, False, True):
            b.set_cross_m2l(cross)
            outs = [torch.full_like(w, float("nan")) for w in ws]
            for rep in range(2):
                b.apply_V(ws, outs)
                torch.cuda.synchronize()
                for r, y in zip(ref, outs):
                    assert torch.equal(r, y), (prec, cross, rep)
    b.close()
    for tr in trees:
        tr.close()

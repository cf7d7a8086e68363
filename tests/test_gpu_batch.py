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

"""Row samples for the full-size parity tests: random rows plus rows of the
first and last time steps and rows from every leaf level of the tree."""
import numpy as np


def sample_rows(tr, n_random, per_level=8, seed=17):
    rng = np.random.default_rng(seed)
    N = tr.E_t * tr.E_x
    rows = set(int(r) for r in rng.choice(N, n_random, replace=False))
    rows |= {0, tr.E_x - 1, N - tr.E_x, N - 1}              # first and last steps
    level_of_box = np.zeros(max(b.id for b in tr.boxes) + 1, dtype=np.int64)
    for b in tr.boxes:
        level_of_box[b.id] = b.level
    row_level = level_of_box[tr.leaf_of_element()]
    levels = sorted(set(int(b.level) for b in tr.leaves))
    for l in levels:
        cand = np.nonzero(row_level == l)[0]
        rows |= set(int(r) for r in rng.choice(cand, min(per_level, len(cand)), replace=False))
    return np.array(sorted(rows)), levels

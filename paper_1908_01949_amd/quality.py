"""Track-finding quality of turn partitions (section 3.1, Eqs. 2-3).

For the n'-th true turn partition, C_{n'} is its number of hits and C_{i->n'} the
number of hits of true partition i classified to the partition found for n':
efficiency eps = C_{n'->n'} / C_{n'}, purity pi = C_{n'->n'} / sum_i C_{i->n'} (the
sum runs over true turn partitions, so noise hits do not enter it). Reading: a found
partition stands for the true partition that contributes most of its hits (ties to
the lower index); when several stand for the same one, the one holding most of its
hits is taken.
"""
from __future__ import annotations

import numpy as np


def turn_quality(true_turn, found_turn):
    """Per true partition n': dict(n_hits=C_{n'}, eps, pi, found=index or -1).

    true_turn: int [H], the hit's true partition (-1 noise); found_turn: int [H],
    the partition the hit was classified to (-1 none).
    """
    t = np.asarray(true_turn, np.int64)
    f = np.asarray(found_turn, np.int64)
    n_true = int(t.max()) + 1 if t.size and t.max() >= 0 else 0
    n_found = int(f.max()) + 1 if f.size and f.max() >= 0 else 0
    C = np.zeros((max(n_true, 1), max(n_found, 1)), np.int64)
    sel = (t >= 0) & (f >= 0)
    np.add.at(C, (t[sel], f[sel]), 1)
    owner = np.full(n_found, -1)
    for p in range(n_found):
        if C[:, p].sum() > 0:
            owner[p] = int(np.argmax(C[:, p]))
    out = []
    for n in range(n_true):
        cn = int((t == n).sum())
        cand = [p for p in range(n_found) if owner[p] == n]
        if not cand:
            out.append(dict(n_hits=cn, eps=0.0, pi=float("nan"), found=-1))
            continue
        p = max(cand, key=lambda q: (C[n, q], -q))
        out.append(dict(n_hits=cn, eps=C[n, p] / cn, pi=C[n, p] / C[:, p].sum(), found=p))
    return out

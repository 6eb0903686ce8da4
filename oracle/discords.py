"""Oracle of discord discovery -- TEST INFRASTRUCTURE ONLY.

A discord is the window with the largest matrix-profile value (Sec. 2, the
discord footnote).  For more than one discord the paper gives no rule; the
reading used here: take the largest finite value (ties: smallest index), drop
every row within ``excl`` of it (|r - r*| <= excl; excl = m - 1 by default, so
no two discords overlap), and repeat.

Certification (Sec. 2, after the max-error guarantee): the dictionary join
P_hat and the exact join P satisfy P_hat - e_max <= P <= P_hat (Lemmas 1 and
2), so when the largest P_hat exceeds the runner-up by more than e_max the
top row needs no exact computation.  Literally the runner-up is the
second-largest value of P_hat; with overlapping windows that is almost always
a neighbour of the top row, so the test is also offered with the runner-up
taken as the second discord (outside the top row's zone), which places the
exact discord within that zone.
"""
from __future__ import annotations

import numpy as np

from . import ab_join


def topk_discords(P, K, excl):
    """Greedy top-K over the finite entries of P; returns (rows, values)."""
    P = np.asarray(P, dtype=np.float64)
    alive = np.isfinite(P)
    rows, vals = [], []
    for _ in range(K):
        if not alive.any():
            break
        r = int(np.argmax(np.where(alive, P, -np.inf)))
        rows.append(r)
        vals.append(float(P[r]))
        alive[max(0, r - excl):r + excl + 1] = False
    return np.array(rows, dtype=np.int64), np.array(vals)


def top_certified(P_hat, e_max, excl=None):
    """True when the largest P_hat beats the runner-up by more than e_max.

    excl=None: runner-up = second-largest finite value (the literal test);
    otherwise the second greedy discord with that exclusion."""
    P_hat = np.asarray(P_hat, dtype=np.float64)
    if excl is None:
        v = np.sort(P_hat[np.isfinite(P_hat)])[::-1]
    else:
        _, v = topk_discords(P_hat, 2, excl)
    if v.size == 0:
        return False
    return bool(v.size == 1 or v[0] - v[1] > e_max)


def exact_discords(query, ref, ref_bounds, m, K, excl=None):
    """Top-K discords of query under the exact join against ref (Def. 8 windows)."""
    P, I = ab_join(query, ref, ref_bounds, m)
    rows, vals = topk_discords(P, K, m - 1 if excl is None else excl)
    return rows, vals, I[rows] if rows.size else rows

"""Oracle of the learning phase (Sec. 3.1, Alg. 1) -- TEST INFRASTRUCTURE ONLY.

``learn_dictionary(T, m, ...)`` returns the greedy dictionary of a training
series: the merged [start, end) pieces of T that form it, the window starts it
chose (in order), their concatenation with segment offsets and original
starts, its e_max (Def. 10) and the self-join profile it started from.

What the greedy choice does (Sec. 3.1, Fig. 4): every window is ranked by its
self-join distance (its distance to its own nearest non-trivial match) minus
its distance to the closest window chosen so far, and the lowest-ranked window
is taken next.  Motifs therefore come first, and the repeats of a motif that
is already in the dictionary sink down the ranking.  The rules this oracle
applies, with the readings taken where the paper leaves a choice (each listed
in the design notes):

* self-join: trivial matches are the windows within floor(m/2) of a window;
* a chosen window and the windows within floor(m/2) of it are never chosen
  again, nor are windows whose self-join distance is not finite; the loop ends
  when no window is left; ties go to the smallest index;
* the "distance to the chosen windows" is the element-wise minimum of their
  distance profiles (Def. 4), zero before the first choice;
* each choice adds ``element_of``: ceil(k m) samples in total (k = 1.5 in the
  paper), bounded by [m, n], the window in the middle (the odd sample after
  it), shifted back inside the series at the ends; pieces that overlap or touch
  merge into one segment;
* stopping: for the memory condition, as soon as the merged pieces hold at
  least (1 - space_saving) n samples; for the accuracy condition, as soon as
  e_max of the current dictionary (computed with the exact join) is at most the
  target; the piece added in the step that meets the condition is kept;
  ``max_iters`` caps the number of choices.

``forced`` replays a given sequence of choices (lockstep checks against the
GPU): at each step the forced index must rank lowest within ``tie_tol`` and is
used in place of the oracle's own choice.
"""
from __future__ import annotations

import math

import numpy as np

from . import ab_join, dist_profile, self_join


def merge_elements(elements):
    """Merge [start, end) intervals that overlap or touch; sorted by start."""
    out = []
    for a, b in sorted(elements):
        if out and a <= out[-1][1]:
            out[-1][1] = max(out[-1][1], b)
        else:
            out.append([a, b])
    return [tuple(e) for e in out]


def element_of(j, n, m, k):
    L = min(n, max(m, int(math.ceil(k * m))))
    c0 = j - (L - m) // 2
    c0 = min(max(c0, 0), n - L)
    return c0, c0 + L


def dictionary_of(T, segs):
    d = np.concatenate([T[a:b] for a, b in segs]) if segs else np.zeros(0)
    bounds = np.concatenate([[0], np.cumsum([b - a for a, b in segs])]).astype(np.int64)
    return d, bounds, np.array([a for a, _ in segs], dtype=np.int64)


def e_max_of(T, segs, m):
    """Def. 10: max over the windows of T of the distance to the dictionary's windows."""
    d, bounds, _ = dictionary_of(T, segs)
    if len(d) < m:
        return math.inf
    P, _ = ab_join(T, d, bounds, m)
    return float(np.max(P))


def learn_dictionary(T, m, k=1.5, stop="space_saving", value=0.9, max_iters=None, forced=None, tie_tol=1e-6):
    """Returns dict(segments, chosen, dictionary, bounds, orig_start, e_max, p_b)."""
    T = np.asarray(T, dtype=np.float64)
    n = len(T)
    W = n - m + 1
    excl = m // 2
    P_B, _ = self_join(T, m, excl)
    S = np.zeros(W)
    first = True
    blocked = np.zeros(W, dtype=bool)
    chosen, elements = [], []
    max_iters = W if max_iters is None else max_iters
    for it in range(max_iters):
        if forced is not None and it >= len(forced):
            raise AssertionError(f"the replayed run stopped after {len(forced)} steps; the oracle continues")
        Pp = P_B - S
        Pp[blocked] = np.inf
        Pp[~np.isfinite(P_B)] = np.inf
        if not np.isfinite(Pp).any():
            break
        j = int(np.argmin(Pp))
        if forced is not None:
            jf = int(forced[it])
            if not (Pp[jf] <= Pp[j] + tie_tol):
                raise AssertionError(f"step {it}: forced {jf} (P'={Pp[jf]}) is not an argmin (P'[{j}]={Pp[j]})")
            j = jf
        chosen.append(j)
        blocked[max(0, j - excl):min(W, j + excl + 1)] = True
        elements.append(element_of(j, n, m, k))
        segs = merge_elements(elements)
        size = sum(b - a for a, b in segs)
        if stop == "space_saving" and size >= (1.0 - value) * n:
            break
        if stop == "e_max" and e_max_of(T, segs, m) <= value:
            break
        Sp = dist_profile(T, m, T[j:j + m])
        S = Sp if first else np.minimum(S, Sp)
        first = False
    segs = merge_elements(elements)
    d, bounds, orig = dictionary_of(T, segs)
    return dict(segments=segs, chosen=chosen, dictionary=d, bounds=bounds, orig_start=orig,
                e_max=e_max_of(T, segs, m), p_b=P_B)

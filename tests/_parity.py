"""Parity checks between the HIP path and the FP64 oracle (shared by GPU tests)."""
import numpy as np


def compare(P_gpu, I_gpu, P_or, I_or, P2_or, tol, orc, q, d, m, bounds, rows=None):
    """Assert the parity bar and return error statistics.

    * P: |P_gpu - P_or| <= tol elementwise (inf and NaN must match exactly);
    * I: equal wherever the oracle's best-to-second gap exceeds tol;
    * every finite row: I_gpu[i] is a window of the reference in the sense of
      Def. 8 (inside one segment of ``bounds``) with finite samples, its
      oracle distance d(i, I_gpu[i]) is within tol of the best (the returned
      index is a valid near-optimal neighbour even where several are within
      tol), and P_gpu[i] is within tol of d(i, I_gpu[i]) (the reported value
      belongs to the reported index).
    """
    P_gpu = np.asarray(P_gpu, dtype=np.float64)
    I_gpu = np.asarray(I_gpu)
    rows = np.arange(len(P_or)) if rows is None else np.asarray(rows)
    nan_or, nan_g = np.isnan(P_or), np.isnan(P_gpu)
    assert np.array_equal(nan_or, nan_g), f"NaN rows differ: {np.flatnonzero(nan_or != nan_g)[:10]}"
    inf_or, inf_g = np.isinf(P_or), np.isinf(P_gpu)
    assert np.array_equal(inf_or, inf_g), f"inf rows differ: {np.flatnonzero(inf_or != inf_g)[:10]}"
    assert np.all(I_gpu[nan_or | inf_or] == -1)
    fin = ~(nan_or | inf_or)
    err = np.abs(P_gpu[fin] - P_or[fin])
    worst = int(np.argmax(err)) if err.size else 0
    assert err.size == 0 or err.max() <= tol, (
        f"max |P err| {err.max():.3e} > {tol} at row {rows[fin][worst]} "
        f"(gpu {P_gpu[fin][worst]!r}, oracle {P_or[fin][worst]!r})")
    gap = P2_or - P_or
    with np.errstate(invalid="ignore"):
        clear = fin & (gap > tol)
    bad = np.flatnonzero(clear & (I_gpu != I_or))
    assert bad.size == 0, f"I differs on clear rows {rows[bad][:10]}: gpu {I_gpu[bad][:10]} oracle {I_or[bad][:10]}"
    if fin.any():
        sel = I_gpu[fin]
        WB = len(d) - m + 1
        assert np.all((sel >= 0) & (sel < WB)), f"index out of range: {sel[(sel < 0) | (sel >= WB)][:10]}"
        valid = orc.valid_windows(bounds, len(d), m)
        inside = valid[sel]
        assert inside.all(), f"index crosses a segment break: rows {rows[fin][~inside][:10]}, I {sel[~inside][:10]}"
        dsel = orc.pair_dists(q, d, m, rows[fin], sel)
        assert np.all(np.isfinite(dsel)), f"index holds a non-finite sample: rows {rows[fin][~np.isfinite(dsel)][:10]}"
        slack = dsel - P_or[fin]
        assert slack.max() <= tol, f"chosen neighbour {slack.max():.3e} worse than the best"
        own = np.abs(P_gpu[fin] - dsel)
        assert own.max() <= tol, (f"P does not belong to I: |P - d(i, I)| = {own.max():.3e} at row "
                                  f"{rows[fin][int(np.argmax(own))]}")
    return dict(max_abs=float(err.max()) if err.size else 0.0, mean_abs=float(err.mean()) if err.size else 0.0,
                rows=int(len(P_or)), clear_rows=int(clear.sum()))

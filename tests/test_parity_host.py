"""The parity helper itself, on the CPU: it accepts the oracle's own result and
rejects each kind of wrong answer a kernel could give (an index that crosses a
segment break, an index on a window with a non-finite sample, a value that
does not belong to its index, a far neighbour on a row whose best is not
unique, a wrong index on a clear row)."""
import numpy as np
import pytest

import _parity

M = 16


@pytest.fixture(scope="module")
def case(orc):
    """A reference of two segments [0, 120) and [120, 300).  A period-10
    pattern over samples 100..135 makes windows 100 (valid), 110 (crosses the
    break) and 120 (valid) identical, and query row 40 an affine copy of them:
    its best distance 0 is reached twice (100 and 120), so the row is not
    clear.  Sample 250 is NaN (windows 235..250 are not windows)."""
    rng = np.random.default_rng(314)
    q = np.cumsum(rng.standard_normal(400))
    d = np.cumsum(rng.standard_normal(300))
    pat = rng.standard_normal(10)
    d[100:136] = np.tile(pat, 4)[:36]
    q[40:40 + M] = 2.0 * d[100:100 + M] - 3.0
    d[250] = np.nan
    bounds = [0, 120, 300]
    P, I, P2 = orc.ab_join(q, d, bounds, M, second=True)
    assert P[40] < 1e-9 and P2[40] < 1e-9 and I[40] == 100
    return q, d, bounds, P, I, P2


def cmp(orc, case, P_gpu, I_gpu):
    q, d, bounds, P, I, P2 = case
    return _parity.compare(P_gpu, I_gpu, P, I, P2, 1e-3, orc, q, d, M, bounds)


def test_accepts_oracle_result_and_the_other_best(orc, case):
    q, d, bounds, P, I, P2 = case
    st = cmp(orc, case, P.astype(np.float32), I)
    assert st["clear_rows"] > 0
    I2 = I.copy()
    I2[40] = 120  # the other valid window at distance 0
    cmp(orc, case, P, I2)


def test_rejects_segment_crossing_index(orc, case):
    q, d, bounds, P, I, P2 = case
    I_bad = I.copy()
    I_bad[40] = 110  # also at distance 0, but it crosses the break at 120
    with pytest.raises(AssertionError, match="segment break"):
        cmp(orc, case, P, I_bad)


def test_rejects_nonfinite_window(orc, case):
    q, d, bounds, P, I, P2 = case
    unclear = np.flatnonzero((P2 - P) <= 1e-3)
    I_bad = I.copy()
    I_bad[unclear] = 240  # holds the NaN sample
    with pytest.raises(AssertionError, match="non-finite"):
        cmp(orc, case, P, I_bad)


def test_rejects_value_not_belonging_to_index(orc, case):
    q, d, bounds, P, I, P2 = case
    # row 40: the true best value 0 reported with a valid index whose distance is not 0
    far = int(np.argmax(orc.pair_dists(q, d, M, [40] * 50, np.arange(50))))
    I_bad = I.copy()
    I_bad[40] = far
    with pytest.raises(AssertionError, match="worse than the best|does not belong"):
        cmp(orc, case, P, I_bad)


def test_rejects_value_beyond_tolerance(orc, case):
    q, d, bounds, P, I, P2 = case
    P_bad = P.copy()
    P_bad[7] += 5e-4  # inside the tolerance: accepted
    cmp(orc, case, P_bad, I)
    P_bad[7] += 1e-3
    with pytest.raises(AssertionError, match="max \\|P err\\|"):
        cmp(orc, case, P_bad, I)


def test_rejects_wrong_index_on_clear_row(orc, case):
    q, d, bounds, P, I, P2 = case
    clear = np.flatnonzero((P2 - P) > 1e-3)
    r = int(clear[0])
    I_bad = I.copy()
    I_bad[r] = I[r] + 1 if I[r] + 1 < 120 - M else I[r] - 1
    with pytest.raises(AssertionError, match="differs on clear rows"):
        cmp(orc, case, P, I_bad)


def test_rejects_inf_nan_mismatch(orc, case):
    q, d, bounds, P, I, P2 = case
    P_bad = P.copy()
    P_bad[0] = np.inf
    with pytest.raises(AssertionError, match="inf rows differ"):
        cmp(orc, case, P_bad, I)

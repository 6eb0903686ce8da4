"""The paper's two guarantees on the GPU path, at the shape of its Fig. 8
experiment: dictionaries learned from an 8,000-sample ECG-like series at
several space-saving factors, joined with a long held-out ECG-like series.

With E = P_hat - P (dictionary join minus join against the whole training
series): no false negatives (Lemma 1, E >= 0) and the max-error guarantee
(Lemma 2, E <= e_max).  Both joins are the FP32 tier, whose distances are
FP64 re-checks of real windows (never below the true minimum, at most 1e-3
above it), so the test allows 1e-3 on each side.  Sampled rows are checked
against the FP64 oracle.
"""
import numpy as np
import pytest
import torch

from paper_2112_12965_amd import abjoin, synth

pytestmark = pytest.mark.gpu
TOL = 1e-3


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).cuda()


@pytest.fixture(scope="module")
def series():
    rng = np.random.default_rng(2112)
    TB = synth.ecg_like(8000, rng)
    TA = synth.ecg_like(400_000, rng, n_anomalies=40)
    return TB, TA


@pytest.mark.parametrize("s", [0.3, 0.5, 0.8, 0.9, 0.99])
def test_guarantees_hold(orc, series, s):
    TB, TA = series
    m = 128
    print(f"[case] guarantees s={s} n_B={len(TB)} n_A={len(TA)} m={m}", flush=True)
    g = abjoin.dict_build(dev(TB), m, stop="space_saving", value=s)
    qa = dev(TA)
    Ph, _ = abjoin.ab_join(qa, g["dictionary"], g["bounds"], m)
    P, _ = abjoin.ab_join(qa, dev(TB), [0, len(TB)], m)
    Ph, P = Ph.cpu().numpy().astype(np.float64), P.cpu().numpy().astype(np.float64)
    E = Ph - P
    em = g["e_max"]
    print(f"s={s} dict={int(g['bounds'][-1])} e_max={em:.4f} E mean={E.mean():.4f} std={E.std():.4f} "
          f"max={E.max():.4f} min={E.min():.4f}", flush=True)
    assert E.min() >= -TOL
    assert E.max() <= em + TOL
    rows = np.random.default_rng(7).choice(len(P), 48, replace=False)
    Po, _ = orc.ab_join(TA, TB, [0, len(TB)], m, rows=rows)
    Pho, _ = orc.ab_join(TA, g["dictionary"].cpu().numpy(), g["bounds"], m, rows=rows)
    assert np.abs(P[rows] - Po).max() <= TOL and np.abs(Ph[rows] - Pho).max() <= TOL

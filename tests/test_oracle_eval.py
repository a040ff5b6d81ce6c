"""Pins of the oracle's threshold (eq. 12) and ROC AUC (Sec. 5.3.1).

The references are scikit-learn's roc_auc_score, brute-force pair counting and closed forms.
"""
import numpy as np
import pytest

import oracle


def test_auc_against_sklearn_and_pairs():
    sk = pytest.importorskip("sklearn.metrics")
    rng = np.random.default_rng(0)
    s = np.round(rng.standard_normal(400), 1)       # many ties
    t = (rng.random(400) < 0.2).astype(np.uint8)
    a = oracle.auc(s, t)
    assert a == pytest.approx(sk.roc_auc_score(t, s), abs=1e-15)
    pos, neg = s[t == 1], s[t == 0]
    gt = (pos[:, None] > neg[None, :]).sum()
    eq = (pos[:, None] == neg[None, :]).sum()
    assert oracle.auc_counts(s, t)[:2] == (gt, eq)
    assert a == (gt + 0.5 * eq) / (pos.size * neg.size)


def test_auc_special_cases():
    t = np.array([0, 0, 1, 1, 0], dtype=np.uint8)
    assert oracle.auc(np.array([0.1, 0.2, 0.9, 0.8, 0.3]), t) == 1.0
    assert oracle.auc(np.full(5, 2.0), t) == 0.5
    assert oracle.auc(-np.array([0.1, 0.2, 0.9, 0.8, 0.3]), t) == 0.0


def test_threshold_closed_form():
    n, a, z = 10, 5.0, 3.0
    s = np.zeros(n)
    s[-1] = a
    tau = oracle.threshold(s, z)
    assert tau == pytest.approx(a / n + z * a * np.sqrt(n - 1) / n, rel=1e-15)
    m = oracle.mask(s, tau)
    assert m.dtype == np.uint8 and m.sum() == (1 if a > tau else 0)


def test_threshold_ignores_non_finite():
    s = np.array([1.0, 2.0, 3.0, np.inf, np.nan])
    assert oracle.threshold(s, 0.0) == pytest.approx(2.0)
    assert oracle.mask(s, 2.5).tolist() == [0, 0, 1, 1, 0]

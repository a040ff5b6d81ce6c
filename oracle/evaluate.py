"""Post-processing of an anomaly map (oracle side).

Test infrastructure only.

* ``threshold``: the adaptive cut-off of eq. (12), tau = mu_d + Z * sigma_d.  mu_d and
  sigma_d are the mean and the population standard deviation of the anomaly matrix
  (Sec. 5.3.2).  Z is left open by the paper and defaults to 3.0 here.  Non-finite
  scores are left out of mu_d and sigma_d.
* ``auc``: the area under the ROC curve (Sec. 5.3.1).  ROC points are counted per
  pixel.  The area equals the Mann-Whitney probability
  P(s_pos > s_neg) + 1/2 P(s_pos = s_neg).
"""
from __future__ import annotations

import numpy as np


def threshold(scores: np.ndarray, z_alpha: float = 3.0) -> float:
    s = np.asarray(scores, dtype=np.float64).ravel()
    s = s[np.isfinite(s)]
    if s.size == 0:
        return float("nan")
    mu = s.sum() / s.size
    var = ((s - mu) ** 2).sum() / s.size
    return float(mu + z_alpha * np.sqrt(var))


def mask(scores: np.ndarray, tau: float) -> np.ndarray:
    """Pixels declared anomalous: s > tau (NaN never is)."""
    return (np.asarray(scores) > tau).astype(np.uint8)


def auc_counts(scores: np.ndarray, truth: np.ndarray) -> tuple[int, int, int, int]:
    """(greater, equal, n_pos, n_neg): pairs (positive, negative) with s_p > s_n, with
    s_p == s_n.  Sorting the negatives once and binary-searching each positive counts
    every pair exactly."""
    s = np.asarray(scores, dtype=np.float64).ravel()
    t = np.asarray(truth).ravel().astype(bool)
    pos, neg = s[t], np.sort(s[~t])
    lo = np.searchsorted(neg, pos, side="left")
    hi = np.searchsorted(neg, pos, side="right")
    return int(lo.sum()), int((hi - lo).sum()), int(pos.size), int(neg.size)


def auc(scores: np.ndarray, truth: np.ndarray) -> float:
    g, e, npos, nneg = auc_counts(scores, truth)
    if npos == 0 or nneg == 0:
        return float("nan")
    return (g + 0.5 * e) / (npos * nneg)

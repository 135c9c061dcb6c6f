"""Oracle of the Risky Gate's trust metrics, the measurement-cost model and its
break-even point (arXiv 2512.19750, Sec. III-C Eqs. 1-4 and Sec. V).

TEST INFRASTRUCTURE ONLY, like the rest of `oracle/`: the product library
never imports or runs it, and it imports nothing of the product.

Written from the definitions:
  Eq. 1  D = |NDV_hist - NDV_est| / NDV_hist, a risk when D >= 0.25;
  Eq. 2  a risk when |S_est - S_probe| > 0.01, with S_probe = count / n;
  Eq. 3  PCS = P(A,B) / (P(A) P(B)), a breach when PCS > 1.6 or PCS < 0.7;
  Eq. 4  the measurement cost, here a linear model in the bytes read and the
         row-terms evaluated whose coefficients are fitted, non-negative, to
         measured latencies (the paper's 0.85 ms constant is the prior).
Readings (the paper gives thresholds, not arithmetic):
  * D and the selectivity error are computed in IEEE binary64 in the order the
    formulas are written, so that a decision at a threshold is the same in
    every implementation;
  * PCS is compared with 8/5 and 7/10 exactly, as rationals of the counts;
  * a signal without a value (no sampled rows; P(A) or P(B) zero) raises no
    flag.
"""
from __future__ import annotations

import math
from fractions import Fraction
from typing import Dict, Optional, Sequence, Tuple

import numpy as np

DRIFT, SELERR, PCS_HI, PCS_LO = 1, 2, 4, 8
PCS = 4
DRIFT_MIN = 0.25                     # Sec. III-C, Eq. 1
SEL_ERR_MAX = 0.01                   # Eq. 2
PCS_HI_T = Fraction(8, 5)            # Eq. 3: 1.6
PCS_LO_T = Fraction(7, 10)           # Eq. 3: 0.7
PRIOR_MS = 0.85                      # Eq. 4


def drift(ndv_hist: float, ndv_est: float) -> float:
    """Eq. 1."""
    return abs(ndv_hist - ndv_est) / ndv_hist


def sel_error(s_est: float, count: int, n: int) -> float:
    """Eq. 2 with S_probe = count / n (Sec. III-C)."""
    return abs(s_est - count / n)


def pcs_exact(c_ab: int, c_a: int, c_b: int, n: int) -> Fraction:
    """Eq. 3 from the counts of one sample of n rows: P(X) = c_X / n."""
    p_ab, p_a, p_b = Fraction(c_ab, n), Fraction(c_a, n), Fraction(c_b, n)
    return p_ab / (p_a * p_b)


def gate(ndv: Optional[Tuple[float, float]] = None, sel: Optional[Tuple[float, int, int]] = None,
         pcs: Optional[Tuple[int, int, int, int]] = None, drift_min: float = DRIFT_MIN,
         sel_err_max: float = SEL_ERR_MAX, pcs_hi: Fraction = PCS_HI_T, pcs_lo: Fraction = PCS_LO_T) -> Dict:
    """Flags of the three signals (Sec. III-A): the gate triggers when any is set."""
    flags = undefined = 0
    out = dict(drift=math.nan, sel_err=math.nan, pcs=None)
    if ndv is not None:
        out["drift"] = drift(*ndv)
        if out["drift"] >= drift_min:
            flags |= DRIFT
    if sel is not None:
        s_est, count, n = sel
        if n == 0:
            undefined |= SELERR
        else:
            out["sel_err"] = sel_error(s_est, count, n)
            if out["sel_err"] > sel_err_max:
                flags |= SELERR
    if pcs is not None:
        c_ab, c_a, c_b, n = pcs
        if c_a == 0 or c_b == 0:
            undefined |= PCS
        else:
            v = pcs_exact(c_ab, c_a, c_b, n)
            out["pcs"] = v
            if v > pcs_hi:
                flags |= PCS_HI
            if v < pcs_lo:
                flags |= PCS_LO
    out.update(flags=flags, undefined=undefined, trigger=flags != 0)
    return out


# ---------------------------------------------------------------- cost model
def design(obs: Sequence[Tuple[float, float, float, float]]) -> Tuple[np.ndarray, np.ndarray]:
    """Rows (1, N * row_bytes, N * terms) and latencies of observations
    (n_rows, row_bytes, terms, ms)."""
    X = np.array([[1.0, n * b, n * t] for n, b, t, _ in obs], dtype=np.float64)
    y = np.array([ms for *_, ms in obs], dtype=np.float64)
    return X, y


def cost_fit(obs: Sequence[Tuple[float, float, float, float]], prior_ms: float = PRIOR_MS) -> np.ndarray:
    """Non-negative least squares for ms = c0 + c1 N b + c2 N t (scipy's NNLS on
    columns scaled to unit RMS); the prior (prior_ms, 0, 0) below 3
    observations."""
    from scipy.optimize import nnls
    if len(obs) < 3:
        return np.array([prior_ms, 0.0, 0.0])
    X, y = design(obs)
    s = np.sqrt((X * X).mean(axis=0))
    s[s == 0] = 1.0
    beta, _ = nnls(X / s, y)
    return beta / s


def cost_predict(coef, n_rows: float, row_bytes: float, terms: float) -> float:
    return coef[0] + coef[1] * (n_rows * row_bytes) + coef[2] * (n_rows * terms)


def breakeven(dev, host, row_bytes: float, terms: float) -> float:
    """Smallest N from which the device model never predicts more than the
    host model: the crossing of the two lines in N (Sec. V, item 2)."""
    sg = dev[1] * row_bytes + dev[2] * terms
    sh = host[1] * row_bytes + host[2] * terms
    if sg < sh:
        return max(0.0, (dev[0] - host[0]) / (sh - sg))
    if sg == sh and dev[0] <= host[0]:
        return 0.0
    return math.inf

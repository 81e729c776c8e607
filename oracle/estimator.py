"""Oracle of the energy estimator with correcting factors.  TEST INFRASTRUCTURE.

Per generation n the projection yields the mean weight w_bar_n (as log) and
the weighted mean local energy e_bar_n.  The population-control bias is
removed by the correcting factors G_n = prod_{k=0}^{p} w_bar_{n-k}:
E_p = sum_n G_n e_bar_n / sum_n G_n (computed in log space).  The error bar
comes from Flyvbjerg-Petersen blocking (J. Chem. Phys. 91, 461 (1989)) of
the weighted series.
"""
from __future__ import annotations

import numpy as np


def correcting_log_factors(log_wbar: np.ndarray, p: int) -> np.ndarray:
    lw = np.asarray(log_wbar, dtype=np.float64)
    n = lw.shape[0]
    out = np.full(n, -np.inf)
    for i in range(p, n):
        out[i] = float(np.sum(lw[i - p:i + 1]))
    return out


def energy(log_wbar, ebar, p: int = 0, n0: int = 0) -> float:
    lg = correcting_log_factors(log_wbar, p)[n0:]
    e = np.asarray(ebar, dtype=np.float64)[n0:]
    ok = np.isfinite(lg)
    lg, e = lg[ok], e[ok]
    g = np.exp(lg - np.max(lg))
    return float(np.sum(g * e) / np.sum(g))


def blocking_error(x: np.ndarray) -> float:
    """Standard error of the mean of a correlated series by blocking: the
    maximum over block levels with at least 16 blocks."""
    x = np.asarray(x, dtype=np.float64)
    best = 0.0
    while x.shape[0] >= 16:
        n = x.shape[0]
        err = np.std(x, ddof=1) / np.sqrt(n)
        best = max(best, err)
        m = n // 2
        x = 0.5 * (x[0:2 * m:2] + x[1:2 * m:2])
    return float(best)


def energy_and_error(log_wbar, ebar, p: int = 0, n0: int = 0):
    """E_p and its blocking error; the error uses the normalized-weight
    series G_n e_n / <G>."""
    lg = correcting_log_factors(log_wbar, p)[n0:]
    e = np.asarray(ebar, dtype=np.float64)[n0:]
    ok = np.isfinite(lg)
    lg, e = lg[ok], e[ok]
    g = np.exp(lg - np.max(lg))
    E = float(np.sum(g * e) / np.sum(g))
    y = g * (e - E) / np.mean(g)
    return E, blocking_error(y)

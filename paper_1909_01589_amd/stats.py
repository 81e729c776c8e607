"""Energy estimator of the projection records (host statistics, numpy).

Per generation the library reports log(w_bar_n) and e_bar_n.  The mixed
estimate with population-control correction over the last p generations is
E_p = sum_n G_n e_bar_n / sum_n G_n, G_n = prod_{k=0}^{p} w_bar_{n-k}; its
statistical error comes from reblocking the normalized series (Flyvbjerg &
Petersen, J. Chem. Phys. 91, 461 (1989)).
"""
from __future__ import annotations

import numpy as np


def _log_gamma(log_wbar: np.ndarray, p: int) -> np.ndarray:
    lw = np.asarray(log_wbar, dtype=np.float64)
    c = np.concatenate([[0.0], np.cumsum(lw)])
    out = np.full(lw.shape, -np.inf)
    if lw.size > p:
        out[p:] = c[p + 1:] - c[:-p - 1]
    return out


def reblock_error(y: np.ndarray, min_blocks: int = 16) -> float:
    y = np.asarray(y, dtype=np.float64)
    errs = []
    while y.size >= min_blocks:
        errs.append(np.std(y, ddof=1) / np.sqrt(y.size))
        y = 0.5 * (y[: y.size // 2 * 2 : 2] + y[1: y.size // 2 * 2 : 2])
    return float(max(errs)) if errs else float("nan")


def estimate(log_wbar, ebar, p=None, skip: int = 0):
    """(E, sigma) from generation records, skipping the first `skip`.
    p=None: plain mean of e_bar_n (no correcting factors); p >= 0: E_p."""
    if p is None:
        e = np.asarray(ebar, dtype=np.float64)[skip:]
        if e.size == 0:
            return float("nan"), float("nan")
        return float(e.mean()), reblock_error(e)
    lg = _log_gamma(np.asarray(log_wbar)[skip:], p)
    e = np.asarray(ebar, dtype=np.float64)[skip:]
    keep = np.isfinite(lg)
    lg, e = lg[keep], e[keep]
    if e.size == 0:
        return float("nan"), float("nan")
    g = np.exp(lg - lg.max())
    E = float(np.dot(g, e) / g.sum())
    return E, reblock_error(g * (e - E) / g.mean())

"""Test infrastructure (oracle): the learned Jastrow correction, tabulated in
plain numpy FP64 from the network weights.

The correction of a pair term at distance r is f(r) = w(r) g(r) for r < r_c
and 0 beyond, with the envelope w(r) = r^2 (1 - r/r_c)^3 (so f and f' vanish
at r = 0, leaving the Pade cusps alone, and f, f', f'' vanish at r_c) and
g(r) = w3 . silu(W2 silu(W1 x + b1) + b2) + b3 at x = r / r_c,
silu(z) = z / (1 + e^-z).  The table holds f, f', f'' at the nodes
r_k = k r_c / (G - 1); the trial function's correction is the quintic
Hermite interpolant of that table (oracle function orc_corr), so the table,
not the network, defines Psi.  Derivatives are carried through the layers by
the chain rule (value, d/dr, d^2/dr^2).  Only tests and the CPU baseline use
this module.
"""
from __future__ import annotations

import numpy as np


def silu3(z):
    """silu(z), silu'(z), silu''(z)."""
    s = 1.0 / (1.0 + np.exp(-z))
    return z * s, s * (1.0 + z * (1.0 - s)), s * (1.0 - s) * (2.0 + z * (1.0 - 2.0 * s))


def network(p: dict, r: np.ndarray, r_c: float):
    """g, g', g'' (r-derivatives) of one network at distances r."""
    r = np.asarray(r, dtype=np.float64)
    x = r / r_c
    z1 = np.outer(x, p["W1"]) + p["b1"]
    dz1 = np.broadcast_to(p["W1"] / r_c, z1.shape)
    a1, s1, t1 = silu3(z1)
    h1, dh1, d2h1 = a1, s1 * dz1, t1 * dz1 * dz1
    z2 = h1 @ p["W2"].T + p["b2"]
    dz2, d2z2 = dh1 @ p["W2"].T, d2h1 @ p["W2"].T
    a2, s2, t2 = silu3(z2)
    h2, dh2, d2h2 = a2, s2 * dz2, t2 * dz2 * dz2 + s2 * d2z2
    w3 = p["w3"]
    return h2 @ w3 + float(p["b3"]), dh2 @ w3, d2h2 @ w3


def envelope(r, r_c: float):
    """w, w', w'' of w(r) = r^2 (1 - r/r_c)^3."""
    r = np.asarray(r, dtype=np.float64)
    q = 1.0 - r / r_c
    w = r * r * q ** 3
    dw = 2.0 * r * q ** 3 - 3.0 * r * r * q * q / r_c
    d2w = 2.0 * q ** 3 - 12.0 * r * q * q / r_c + 6.0 * r * r * q / (r_c * r_c)
    return w, dw, d2w


def correction(p: dict, r, r_c: float):
    """f, f', f'' of one correction at distances r < r_c."""
    g, dg, d2g = network(p, r, r_c)
    w, dw, d2w = envelope(r, r_c)
    return w * g, dw * g + w * dg, d2w * g + 2.0 * dw * dg + w * d2g


def tabulate(weights: dict, n_nodes: int, r_c: float) -> np.ndarray:
    """Table [2][n_nodes][3] = {f, f', f''} at r_k = k r_c / (n_nodes - 1),
    type 0 from weights["ee"], type 1 from weights["en"]."""
    r = np.linspace(0.0, r_c, n_nodes)
    tab = np.zeros((2, n_nodes, 3))
    for t, kind in enumerate(("ee", "en")):
        f, df, d2f = correction(weights[kind], r, r_c)
        tab[t, :, 0], tab[t, :, 1], tab[t, :, 2] = f, df, d2f
    return tab

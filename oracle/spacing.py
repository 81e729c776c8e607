"""Oracle for the paper's choice of r_c and a'/a.  TEST INFRASTRUCTURE.

* r_c(Z) = beta Z^(-5/7), beta = 0.75 (main text, after Eq. (10)).
* r_c(a, Z) = beta (kappa alpha^-2 + 1)/(alpha^-2 + 1) Z^(-5/7), with
  alpha = 1/(a Z) and kappa = 2.5 (supplement Eq. (S-13)).
* N_core(r_c) = int 4 pi r^2 rho(r) exp(-r^2 / 2 r_c^2) dr (main text Eq. (7))
  with a Slater-type atomic density.  The paper takes Clementi's exponents;
  those tables are not at hand, so Slater's own screening rules are used.
* a'/a = sqrt((Z - N_core)/N_core) (main text Eq. (6)).
* speedup^-1 = N_core/Z + (N_val/Z)(a'/a)^-2 (main text Eq. (5)).
"""
from __future__ import annotations

import math

import numpy as np
from scipy import integrate, special

BETA = 0.75
KAPPA = 2.5

# n* of Slater's rules for principal quantum numbers 1..6
_NSTAR = {1: 1.0, 2: 2.0, 3: 3.0, 4: 3.7, 5: 4.0, 6: 4.2}


def rc_of_z(Z: float, beta: float = BETA) -> float:
    return beta * Z ** (-5.0 / 7.0)


def rc_of_a(a: float, Z: float, beta: float = BETA, kappa: float = KAPPA) -> float:
    alpha = 1.0 / (a * Z)
    x = alpha ** -2
    return beta * (kappa * x + 1.0) / (x + 1.0) * Z ** (-5.0 / 7.0)


def rc_of_alpha(alpha: float, Z: float, beta: float = BETA, kappa: float = KAPPA) -> float:
    x = alpha ** -2
    return beta * (kappa * x + 1.0) / (x + 1.0) * Z ** (-5.0 / 7.0)


def aufbau(Z: int):
    """Ground-state subshell occupations (n, l, occ) in Madelung order."""
    subshells = sorted(((n, l) for n in range(1, 8) for l in range(0, n)),
                       key=lambda t: (t[0] + t[1], t[0]))
    left = int(Z)
    out = []
    for n, l in subshells:
        if left <= 0:
            break
        occ = min(left, 2 * (2 * l + 1))
        out.append((n, l, occ))
        left -= occ
    return out


def slater_groups(Z: int):
    """Slater groups [(n, kind, occ)], kind 'sp', 'd' or 'f', in Slater order."""
    groups = {}
    for n, l, occ in aufbau(Z):
        key = (n, "sp") if l <= 1 else (n, "d" if l == 2 else "f")
        groups[key] = groups.get(key, 0) + occ
    rank = {"sp": 0, "d": 1, "f": 2}
    return [(n, k, o) for (n, k), o in sorted(groups.items(), key=lambda t: (t[0][0], rank[t[0][1]]))]


def slater_exponents(Z: int):
    """[(n*, zeta, occ)] from Slater's screening rules (Phys. Rev. 36, 57)."""
    gs = slater_groups(Z)
    out = []
    for gi, (n, kind, occ) in enumerate(gs):
        s = (occ - 1) * (0.30 if n == 1 else 0.35)
        for gj in range(gi):
            n2, k2, o2 = gs[gj]
            if kind == "sp":
                if n2 == n - 1:
                    s += 0.85 * o2
                elif n2 <= n - 2:
                    s += 1.00 * o2
            else:
                s += 1.00 * o2
        nstar = _NSTAR[n]
        out.append((nstar, (Z - s) / nstar, occ))
    return out


def n_core(Z: int, r_c: float) -> float:
    """Main text Eq. (7) with the Slater density: sum over groups of
    occ * int_0^inf r^2 R(r)^2 exp(-r^2/2r_c^2) dr, R = N r^(n*-1) e^(-zeta r)."""
    total = 0.0
    for nstar, zeta, occ in slater_exponents(Z):
        lognorm = (2 * nstar + 1) * math.log(2 * zeta) - special.gammaln(2 * nstar + 1)

        def f(r, nstar=nstar, zeta=zeta, lognorm=lognorm):
            if r <= 0.0:
                return 0.0
            return math.exp(lognorm + 2 * nstar * math.log(r) - 2 * zeta * r - r * r / (2 * r_c * r_c))

        peak = nstar / zeta
        val, _ = integrate.quad(f, 0.0, np.inf, points=None, limit=200, epsabs=1e-14, epsrel=1e-12)
        if not np.isfinite(val):
            val, _ = integrate.quad(f, 0.0, 50 * peak, limit=400)
        total += occ * val
    return total


def a_prime_ratio(Z: int, r_c: float) -> float:
    nc = n_core(Z, r_c)
    return math.sqrt((Z - nc) / nc)


def speedup(Z: float, nc: float, ratio: float) -> float:
    """Main text Eq. (5)."""
    return 1.0 / (nc / Z + (Z - nc) / Z * ratio ** -2)


def spacing(Z: int, a: float, beta: float = BETA, kappa: float = KAPPA):
    """(r_c, a', N_core) for small spacing a and heaviest charge Z."""
    rc = rc_of_a(a, Z, beta, kappa)
    nc = n_core(Z, rc)
    return rc, a * math.sqrt((Z - nc) / nc), nc


def spacing_pade(Z: float, a: float):
    """(r_c, a') of the earlier parametrization the paper compares against:
    r_c = Z/2 in the Pade switch of main text Eq. (2), and
    a'/a = sqrt(Z^2/4 + 1) (main text Eq. (4))."""
    return 0.5 * Z, a * math.sqrt(Z * Z / 4.0 + 1.0)

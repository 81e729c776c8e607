"""Algorithmic FP64 operation counts of the projection, per unit of work.

Counting convention: one add, subtract, multiply, compare-select, exp, log,
sqrt or division is one operation; a fused multiply-add is two.  These counts
belong to the algorithm as formulated (orbital-projected inverse Y = C Ainv,
one exponential per (nucleus, exponent) group), not to the instructions the
compiler emits: an exp, sqrt or division costs gfx950 ten to twenty FP64
instructions, so a fraction of the FP64 peak computed from these counts is a
lower bound on how busy the vector units are.

Units:
* a table evaluation: the ratios, coefficients and heat-bath weights of all
  M = 12N moves of one walker (done once per move plus once per walker and
  generation for the final holding time);
* an accepted move: new orbital row with derivatives, Sherman-Morrison
  update of Ainv and Y, determinant derivatives, the Jastrow derivative
  terms of the moved electron's pairs at its new and old position (the
  other electrons' sums change only by those), local energy;
* a generation start: Slater matrices with derivatives, Gauss-Jordan
  inversion, Y, derivatives and local energy of one walker.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class Shape:
    N: int
    n_up: int
    n_dn: int
    K: int
    n_nuc: int
    n_heavy: int
    groups: list      # per (nucleus, exponent) group: tuple of angular momenta present

    @property
    def ns(self) -> int:
        return max(self.n_up, self.n_dn)

    @property
    def M(self) -> int:
        return 12 * self.N


def shape_of(system, z_heavy=None) -> Shape:
    zh = float(np.max(system.Z)) if z_heavy is None else float(z_heavy)
    groups = {}
    order = []
    for nuc, l, al in zip(system.shell_nuc, system.shell_l, system.shell_alpha):
        key = (int(nuc), float(al))
        if key not in groups or l in groups[key]:
            if key in groups:
                key = (int(nuc), float(al), len(order))
            groups[key] = []
            order.append(key)
        groups[key].append(int(l))
    return Shape(N=system.n_elec, n_up=system.n_up, n_dn=system.n_dn, K=system.n_basis,
                 n_nuc=system.n_nuc, n_heavy=int(np.sum(system.Z >= zh)),
                 groups=[tuple(groups[k]) for k in order])


# per group of the ratio dot product: d (3), |d|^2 (5), alpha*d^2 and exp (2),
# accumulate (2), plus the polynomial part for each angular momentum present
_POLY = {0: 1, 1: 6, 2: 20}
# per basis function with gradient and Laplacian: value 1, gradient 9, Laplacian 2
_FULL_PER_FN = 12
_FULL_PER_GROUP = 12
_PAIR = 14          # one Pade pair term at a displaced point (incl. sqrt and division)
_PAIR_DERIV = 25    # one Pade pair with gradient and Laplacian (incl. sqrt, divisions)


def table_ops(s: Shape) -> float:
    per_group = sum(12 + sum(_POLY[l] for l in g) for g in s.groups)
    entry = (15                      # displaced point and midpoint
             + 8 * s.n_heavy + 2     # nearest heavy nucleus and exp of the switch
             + 2                     # coefficient k
             + per_group             # determinant ratio via Y
             + _PAIR * (s.N - 1 + s.n_nuc) + 3  # Jastrow ratio and its exp
             + 3)                    # T = k max(rho, 0) / 2
    return float(s.M * entry + 2 * s.M)     # plus the cumulative sum


def _orbital_rows(s: Shape, n: int) -> float:
    full = _FULL_PER_FN * s.K + _FULL_PER_GROUP * len(s.groups)
    return float(full + 5 * s.K * n * 2)


def accept_ops(s: Shape) -> float:
    n = s.ns
    return (_orbital_rows(s, n)
            + 2 * n * n              # w = phi(r') Ainv
            + 3 * n * n              # Ainv rank-1 update
            + 3 * n * s.K            # Y rank-1 update
            + 4 * n * n * 2          # grad/lap D/D of the moved spin
            + _PAIR_DERIV * 2 * (s.N - 1 + s.n_nuc)     # the moved electron's pair terms, new and old
            + 14 * s.N)              # local energy


def setup_ops(s: Shape) -> float:
    ops = 0.0
    for n in (s.n_up, s.n_dn):
        if n == 0:
            continue
        ops += n * _orbital_rows(s, n)
        ops += 2 * n * (2 * n) * n * 2 / 2  # Gauss-Jordan on [A | I]
        ops += n * s.K * n * 2               # Y = C Ainv
        ops += 4 * n * n * 2                 # grad/lap D/D
    return ops + _PAIR_DERIV * s.N * (s.N - 1 + s.n_nuc) + 14 * s.N


def projection_ops(s: Shape, walker_launches: int, moves: int, setups: int) -> float:
    """Operations of projection launches with `moves` accepted moves in total,
    `walker_launches` = walkers x launches (each walker evaluates one table
    per accepted move plus one for the holding time that ends its
    generation) and `setups` generation starts (refresh generations)."""
    return setups * setup_ops(s) + (moves + walker_launches) * table_ops(s) + moves * accept_ops(s)


def state_bytes(s: Shape) -> float:
    """HBM bytes of one projection launch per walker: positions in and out,
    log w, e_L and the move count out (the MO matrix and basis constants are
    shared and cache resident)."""
    return 8.0 * (3 * s.N) * 2 + 8 + 8 + 4

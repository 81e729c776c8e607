"""Pins of the small-grid drop rule: a move of the small grid whose switch p
at the midpoint is below 2^-52 has heat-bath weight T = 0.

* On a heavy atom (Z = 54 at a = 1/(3.5 Z)) many small-grid moves of valence
  electrons are dropped, every dropped one has p < 2^-52 (k a^2 < 2^-52) and
  no large-grid move is dropped.
* Delta with the rule differs from the full sum of k max(rho, 0) / 2 by less
  than 1e-13 relative, and the lattice e_L still equals the analytic E_L to
  the same order.
* The Pade switch (p >= 1 / (1 + r_c^2 d^2), never that small) and the single
  grid drop nothing.
"""
import numpy as np
import pytest

import oracle
from oracle import spacing
from paper_1909_01589_amd import inputs


def _table(o, pos, Rm):
    rho, k, d = o.eval_moves(pos, Rm)
    full = 0.5 * (k * np.maximum(rho, 0.0)).sum()
    return rho, k, d, full


def test_heavy_atom_drops_only_negligible_small_grid_moves(oracle_lib):
    s = inputs.zsweep_atom(54, 0)
    a = 1.0 / (3.5 * 54)
    rc, ap, _ = spacing.spacing(54.0, a)
    o = oracle.Oracle(s, a, ap, rc, seed=1)
    pos = inputs.initial_walkers(s, 2, 3)
    n_drop = 0
    for w in range(2):
        Rm = o.move_rotation(w, 0, 0)
        rho, k, d, full = _table(o, pos[w], Rm)
        g = (np.arange(o.M) // 6) % 2
        p = k * a * a                       # small grid: k = p / a^2
        small = (g == 0) & (p < 2.0 ** -52 * (1 + 1e-12))
        T = 0.5 * k * np.maximum(rho, 0.0)
        dropped_sum = T[small].sum()
        n_drop += int(small.sum())
        assert abs(d["delta"] - (full - dropped_sum)) <= 1e-12 * full
        assert dropped_sum <= 1e-13 * full
        assert abs(d["e_lattice"] - d["e_l"]) <= 1e-9 * (abs(d["e_l"]) + abs(d["lap_exact"]))
    assert n_drop > 100


@pytest.mark.parametrize("mode", ["pade", "single"])
def test_nothing_dropped_without_the_gaussian_switch(oracle_lib, mode):
    s = inputs.zsweep_atom(54, 0)
    a = 1.0 / (3.5 * 54)
    if mode == "pade":
        rc, ap = spacing.spacing_pade(54.0, a)
        o = oracle.Oracle(s, a, ap, rc, seed=1, switch_form=1)
    else:
        o = oracle.Oracle(s, a, a, 1.0, seed=1, grids=1)
    pos = inputs.initial_walkers(s, 1, 3)[0]
    rho, k, d, full = _table(o, pos, o.move_rotation(0, 0, 0))
    assert d["delta"] == pytest.approx(full, rel=1e-14)

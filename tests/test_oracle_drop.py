"""The GPU kernels' skip of negligible small-grid moves, judged against the
oracle's plain Eq. (1) heat bath.

The oracle sums every move of both grids.  The large-system kernels leave
out of the heat bath the small-grid moves whose switch p at the midpoint is
below 2^-52 (their weight p/a^2 is below 2^-52 (a'/a)^2 of the large-grid
weight of the same electron and direction).  Measured here on the oracle's
own tables of a heavy atom (Z = 54 at a = 1/(3.5 Z)), where hundreds of
moves per table fall under that rule:

* every cumulative sum C_m of the table, and Delta itself, moves by less
  than 1e-13 of Delta when those moves are left out;
* so a heat-bath choice of the kernel can differ from the oracle's only
  where the oracle's decision margin is below 1e-13, inside the 1e-12 tie
  rule under which the parity tests accept a differing index (and count it);
* the Pade switch (p >= 1 / (1 + r_c^2 d^2)) and the single grid have no
  such moves.
"""
import numpy as np
import pytest

import oracle
from oracle import spacing
from paper_1909_01589_amd import inputs

P_SKIP = 2.0 ** -52       # the kernels' rule
TIE = 1e-12               # the parity tests' tie margin


def test_skip_rule_moves_every_cumulative_sum_below_the_tie_margin(oracle_lib):
    s = inputs.zsweep_atom(54, 0)
    a = 1.0 / (3.5 * 54)
    rc, ap, _ = spacing.spacing(54.0, a)
    o = oracle.Oracle(s, a, ap, rc, seed=1)
    pos = inputs.initial_walkers(s, 3, 3)
    n_skip, worst = 0, 0.0
    for w in range(3):
        Rm = o.move_rotation(w, 0, 0)
        rho, k, d = o.eval_moves(pos[w], Rm)
        T = 0.5 * k * np.maximum(rho, 0.0)
        # the oracle's Delta is the plain sum over every move
        assert d["delta"] == pytest.approx(T.sum(), rel=1e-13)
        g = (np.arange(o.M) // 6) % 2
        p = k * a * a                       # small grid: k = p / a^2
        skip = (g == 0) & (p < P_SKIP)
        n_skip += int(skip.sum())
        T_skip = np.where(skip, 0.0, T)
        C, C_skip = np.cumsum(T), np.cumsum(T_skip)
        worst = max(worst, float(np.max(np.abs(C - C_skip)) / C[-1]))
        # the lattice e_L still equals the analytic E_L
        assert abs(d["e_lattice"] - d["e_l"]) <= 1e-9 * (abs(d["e_l"]) + abs(d["lap_exact"]))
    assert n_skip > 100
    assert worst < 1e-13 < TIE
    print(f"Z=54: {n_skip} small-grid moves under the skip rule in 3 tables; "
          f"largest shift of a cumulative sum {worst:.2e} of Delta")


@pytest.mark.parametrize("mode", ["pade", "single"])
def test_nothing_under_the_rule_without_the_gaussian_switch(oracle_lib, mode):
    s = inputs.zsweep_atom(54, 0)
    a = 1.0 / (3.5 * 54)
    if mode == "pade":
        rc, ap = spacing.spacing_pade(54.0, a)
        o = oracle.Oracle(s, a, ap, rc, seed=1, switch_form=1)
    else:
        o = oracle.Oracle(s, a, a, 1.0, seed=1, grids=1)
    pos = inputs.initial_walkers(s, 1, 3)[0]
    rho, k, d = o.eval_moves(pos, o.move_rotation(0, 0, 0))
    if mode == "pade":
        g = (np.arange(o.M) // 6) % 2
        assert np.all(k[g == 0] * a * a >= P_SKIP)
    assert d["delta"] == pytest.approx(0.5 * (k * np.maximum(rho, 0.0)).sum(), rel=1e-14)

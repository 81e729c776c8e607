"""Oracle pins for the earlier double-grid scheme and the single grid the
paper compares against.

* Earlier switch, main text Eq. (2): p = 1/(1 + r_c^2 d^2) at the midpoint,
  with the same lattice Laplacian of Eq. (1).  Pinned by properties that do
  not restate the formula: p = 1 at the heavy nucleus and p = 1/2 at
  distance 1/r_c (from the positions of a one-nucleus system), the symmetry
  k(x -> x') = k(x' -> x), O(a^2) convergence of the lattice kinetic term,
  r_c = 0 reducing the scheme to the single grid, and the exact hydrogenic
  trial function keeping a zero-variance local energy.
* Single grid (p = 1, spacing a, 6N moves): equals the standard 7-point
  finite-difference Laplacian built here from full Psi evaluations, and the
  double grid with a' = a summed over the two grids.
* Earlier spacing rule, main text Eq. (4): a'/a = sqrt(Z^2/4 + 1) with
  r_c = Z/2; closed forms at Z = 2 and the large-Z limit.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import spacing
from paper_1909_01589_amd import inputs


@pytest.fixture(scope="module")
def tiny(oracle_lib):
    s = inputs.tiny_mixed(seed=2, n_up=2, n_dn=2)
    return oracle.Oracle(s, a=0.05, a_prime=0.09, r_c=1.7, z_heavy=3.0, switch_form=1)


def _fd7(o, pos, a, R=np.eye(3)):
    l0, s0 = o.log_psi(pos)
    tot = 0.0
    for i in range(pos.shape[0]):
        for ax in range(3):
            for sg in (1, -1):
                p = pos.copy()
                p[i] = p[i] + sg * a * R[:, ax]
                l1, s1 = o.log_psi(p)
                tot += (s0 * s1 * np.exp(l1 - l0) - 1.0) / a ** 2
    return tot


def test_pade_switch_half_point(oracle_lib):
    """One heavy nucleus at R: p = 1 on it, 1/2 at distance 1/r_c, 1/5 at
    distance 2/r_c, monotone in between."""
    s = inputs.atom(10, (4, 2, 1), 0.1, 2.5, seed=0)
    s.R[0] = [0.3, -0.2, 0.1]
    rc = 2.5
    o = oracle.Oracle(s, a=0.02, a_prime=0.05, r_c=rc, switch_form=1)
    rng = np.random.default_rng(1)
    for _ in range(5):
        u = rng.normal(size=3)
        u /= np.linalg.norm(u)
        assert o.p_switch(s.R[0]) == 1.0
        assert o.p_switch(s.R[0] + u / rc) == pytest.approx(0.5, rel=1e-13)
        assert o.p_switch(s.R[0] + 2 * u / rc) == pytest.approx(0.2, rel=1e-13)
        d = np.linspace(0.0, 3.0 / rc, 20)
        vals = [o.p_switch(s.R[0] + t * u) for t in d]
        assert np.all(np.diff(vals) < 0)


def test_pade_switch_coefficients_are_symmetric(tiny):
    rng = np.random.default_rng(4)
    pos = inputs.initial_walkers(tiny.system, 1, 4)[0] * 0.3
    R = tiny.rotation(rng.uniform(size=3))
    for m in range(tiny.M):
        rp, k = tiny.move(pos, R, m)
        back = m + 1 if m % 2 == 0 else m - 1
        p2 = pos.copy()
        p2[m // 12] = rp
        r_back, k_back = tiny.move(p2, R, back)
        assert np.allclose(r_back, pos[m // 12], atol=1e-14)
        assert k_back == pytest.approx(k, rel=1e-12, abs=1e-300)


def test_pade_switch_laplacian_converges_as_a_squared(tiny):
    pos = inputs.initial_walkers(tiny.system, 1, 3)[0]
    exact = tiny.local_energy(pos)[1]
    ratios = []
    for a in (0.04, 0.02, 0.01):
        o = tiny.with_params(a=a, a_prime=1.8 * a)
        ratios.append((o.eval_moves(pos)[2]["lap_lattice"] - exact) / a ** 2)
    assert ratios[0] != 0.0
    assert ratios[1] == pytest.approx(ratios[0], rel=0.05)
    assert ratios[2] == pytest.approx(ratios[1], rel=0.05)


def test_single_grid_is_seven_point_laplacian(tiny):
    o = tiny.with_params(grids=1)
    assert o.M == 6 * o.N
    pos = inputs.initial_walkers(o.system, 1, 1)[0]
    R = o.rotation([0.3, 0.6, 0.1])
    rho, k, d = o.eval_moves(pos, R)
    assert np.all(k == 1.0 / o.prm.a ** 2)
    assert d["lap_lattice"] == pytest.approx(_fd7(o, pos, o.prm.a, R), rel=1e-10)
    assert d["e_lattice"] == pytest.approx(d["e_l"], rel=1e-10, abs=1e-10)


def test_single_grid_equals_double_grid_with_equal_spacings(tiny):
    pos = inputs.initial_walkers(tiny.system, 1, 2)[0]
    R = tiny.rotation([0.2, 0.5, 0.8])
    a = 0.07
    r1, k1, d1 = tiny.with_params(a=a, a_prime=a, grids=1).eval_moves(pos, R)
    for form, rc in ((0, 0.3), (1, 2.0)):
        r2, k2, d2 = tiny.with_params(a=a, a_prime=a, switch_form=form, r_c=rc).eval_moves(pos, R)
        kk = k2.reshape(-1, 2, 6)
        assert np.allclose(kk.sum(axis=1).reshape(-1), k1, rtol=1e-13)
        assert np.array_equal(r2.reshape(-1, 2, 6)[:, 0, :].reshape(-1), r1)
        assert d2["lap_lattice"] == pytest.approx(d1["lap_lattice"], rel=1e-12)


def test_pade_switch_with_zero_rc_is_single_grid(tiny):
    pos = inputs.initial_walkers(tiny.system, 1, 5)[0]
    o = tiny.with_params(r_c=0.0)
    rho, k, d = o.eval_moves(pos)
    kk = k.reshape(-1, 2, 6)
    assert np.all(kk[:, 0, :] == 1.0 / o.prm.a ** 2) and np.all(kk[:, 1, :] == 0.0)
    single = tiny.with_params(grids=1).eval_moves(pos)[2]
    assert d["lap_lattice"] == pytest.approx(single["lap_lattice"], rel=1e-12)


@pytest.mark.parametrize("switch_form,grids", [(1, 2), (0, 1)])
def test_exact_hydrogenic_local_energy_in_every_mode(oracle_lib, switch_form, grids):
    Z = 2.0
    s = inputs.hydrogenic(Z)
    o = oracle.Oracle(s, a=0.15, a_prime=0.25, r_c=1.0, switch_form=switch_form, grids=grids)
    rng = np.random.default_rng(7)
    for _ in range(5):
        pos = rng.normal(size=(1, 3)) * 0.8
        d = o.eval_moves(pos, o.rotation(rng.uniform(size=3)))[2]
        assert d["e_lattice"] == pytest.approx(-Z * Z / 2, rel=1e-12)
        assert d["e_l"] == pytest.approx(-Z * Z / 2, rel=1e-12)


def test_earlier_spacing_rule():
    rc, ap = spacing.spacing_pade(2.0, 0.1)
    assert rc == 1.0
    assert ap == pytest.approx(0.1 * math.sqrt(2.0), rel=1e-15)
    for Z in (18.0, 54.0, 1e4):
        rc, ap = spacing.spacing_pade(Z, 1.0)
        assert rc == Z / 2
        assert ap / (Z / 2) == pytest.approx(1.0, rel=2.0 / Z ** 2)
        assert ap > Z / 2

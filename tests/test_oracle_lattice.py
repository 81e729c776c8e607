"""Oracle pins: the double-grid lattice Laplacian (main text Eq. (1)) with the
Gaussian switch (Eq. (3)).

* p = 1 everywhere reduces Eq. (1) to the standard 7-point finite-difference
  Laplacian at spacing a, computed here from full Psi evaluations.
* a' = a reduces it to the single grid for any p.
* The lattice kinetic term converges to the analytic Laplacian as O(a^2) at
  fixed a'/a.
* Midpoint evaluation of p makes the coefficient of x -> x' equal that of
  x' -> x (a symmetric H^a).
* R_c runs over the heaviest nuclei only ("Application to large systems").
* Cost model of Eq. (5): the single-grid move rate over the double-grid
  move rate tends to N/(N_c + (N - N_c)(a/a')^2), N_c = sum_i p(r_i).
"""
import numpy as np
import pytest

import oracle
from paper_1909_01589_amd import inputs


@pytest.fixture(scope="module")
def tiny(oracle_lib):
    s = inputs.tiny_mixed(seed=2, n_up=2, n_dn=2)
    return oracle.Oracle(s, a=0.05, a_prime=0.09, r_c=0.6, z_heavy=3.0)


def _fd7(o, pos, a, R=np.eye(3)):
    """sum_i sum_{mu,+-} [Psi(r_i + a e_mu) - Psi(r_i)] / (a^2 Psi)."""
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


def test_p_one_gives_seven_point_laplacian(tiny):
    o = tiny.with_params(r_c=1e300)          # p = exp(-0) = 1 everywhere
    pos = inputs.initial_walkers(o.system, 1, 1)[0]
    R = o.rotation([0.3, 0.6, 0.1])
    rho, k, d = o.eval_moves(pos, R)
    kk = k.reshape(-1, 2, 6)
    assert np.all(kk[:, 0, :] == 1.0 / o.prm.a ** 2)
    assert np.all(kk[:, 1, :] == 0.0)
    assert d["lap_lattice"] == pytest.approx(_fd7(o, pos, o.prm.a, R), rel=1e-10)


def test_equal_spacings_give_single_grid(tiny):
    pos = inputs.initial_walkers(tiny.system, 1, 2)[0]
    a = 0.07
    single = tiny.with_params(a=a, a_prime=a, r_c=1e300).eval_moves(pos)[2]["lap_lattice"]
    for rc in (0.05, 0.3, 1.0):
        dbl = tiny.with_params(a=a, a_prime=a, r_c=rc).eval_moves(pos)[2]["lap_lattice"]
        assert dbl == pytest.approx(single, rel=1e-12)


def test_lattice_laplacian_converges_as_a_squared(tiny):
    pos = inputs.initial_walkers(tiny.system, 1, 3)[0]
    exact = tiny.local_energy(pos)[1]
    ratios = []
    for a in (0.04, 0.02, 0.01):
        o = tiny.with_params(a=a, a_prime=1.8 * a, r_c=0.6)
        err = o.eval_moves(pos)[2]["lap_lattice"] - exact
        ratios.append(err / a ** 2)
    assert ratios[0] != 0.0
    assert ratios[1] == pytest.approx(ratios[0], rel=0.05)
    assert ratios[2] == pytest.approx(ratios[1], rel=0.05)


def test_hopping_coefficients_are_symmetric(tiny):
    """k(x -> x') for move (i, grid, axis, +) equals k(x' -> x) for the move
    (i, grid, axis, -) from x'."""
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


def test_switch_uses_heaviest_nuclei_only(oracle_lib):
    s = inputs.molecule(0)
    o = oracle.Oracle(s, a=1 / 28, a_prime=0.08, r_c=0.3, z_heavy=8.0)
    for I in range(4, 12):          # on top of a hydrogen
        x = s.R[I]
        dO = min(np.linalg.norm(x - s.R[J]) for J in range(4))
        assert o.p_switch(x) == pytest.approx(np.exp(-dO ** 2 / (2 * 0.3 ** 2)), rel=1e-12)
    for I in range(4):
        assert o.p_switch(s.R[I]) == 1.0


def test_coefficients_weight_by_p_at_midpoint(tiny):
    pos = inputs.initial_walkers(tiny.system, 1, 9)[0] * 0.5
    R = tiny.rotation([0.9, 0.2, 0.7])
    a, ap = tiny.prm.a, tiny.prm.a_prime
    for m in range(tiny.M):
        i, g, dr = m // 12, (m // 6) % 2, m % 6
        h = a if g == 0 else ap
        sgn = 1 if dr % 2 == 0 else -1
        mid = pos[i] + sgn * 0.5 * h * R[:, dr // 2]
        p = tiny.p_switch(mid)
        _, k = tiny.move(pos, R, m)
        assert k == pytest.approx(p / a ** 2 if g == 0 else (1 - p) / ap ** 2, rel=1e-14)


def test_move_rate_ratio_follows_eq5(oracle_lib):
    """Delta = sum_m k_m max(rho_m,0)/2 -> 3 sum_i [p_i/a^2 + (1-p_i)/a'^2] as
    a -> 0, so Delta_single/Delta_double -> N/(N_c + (N-N_c)(a/a')^2)."""
    s = inputs.be_like(0)
    a, ap, rc = 0.002, 0.0035, 0.44
    dbl = oracle.Oracle(s, a=a, a_prime=ap, r_c=rc)
    sgl = dbl.with_params(a_prime=a)
    for seed in range(3):
        pos = inputs.initial_walkers(s, 1, 40 + seed)[0] * 0.5
        Nc = sum(dbl.p_switch(r) for r in pos)
        pred = s.n_elec / (Nc + (s.n_elec - Nc) * (a / ap) ** 2)
        ratio = sgl.eval_moves(pos)[2]["delta"] / dbl.eval_moves(pos)[2]["delta"]
        assert ratio == pytest.approx(pred, rel=0.02)

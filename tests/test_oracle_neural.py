"""Oracle pins for the learned Jastrow correction.

* The network's chain-rule derivatives against central finite differences of
  its own value; the envelope's closed-form zeros at r = 0 (f, f') and r = r_c
  (f, f', f'').
* The quintic Hermite interpolant reproduces any quintic polynomial exactly
  from its values and first two derivatives at the nodes, is C^2 across
  nodes, and vanishes beyond the cutoff.
* With a table in the trial function: analytic gradient and Laplacian of
  log Psi against central finite differences of log Psi, a zero table giving
  the Pade trial function, and a finite local energy at electron-electron
  and electron-nucleus coalescence (cusps untouched).
"""
import numpy as np
import pytest

import oracle
from oracle import neural
from paper_1909_01589_amd import inputs

RC = 6.0


@pytest.fixture(scope="module")
def weights():
    return inputs.neural_weights(seed=1, out_scale=1.0)


def test_network_derivatives_match_finite_differences(weights):
    r = np.linspace(0.05, RC - 0.05, 37)
    for kind in ("ee", "en"):
        for fn in (neural.network, neural.correction):
            v, d1, d2 = fn(weights[kind], r, RC)
            h = 1e-4
            vp, _, _ = fn(weights[kind], r + h, RC)
            vm, _, _ = fn(weights[kind], r - h, RC)
            dp = fn(weights[kind], r + h, RC)[1]
            dm = fn(weights[kind], r - h, RC)[1]
            assert np.allclose(d1, (vp - vm) / (2 * h), rtol=1e-6, atol=1e-8)
            assert np.allclose(d2, (dp - dm) / (2 * h), rtol=1e-6, atol=1e-7)


def test_envelope_zeros(weights):
    f0 = neural.correction(weights["ee"], np.array([0.0]), RC)
    fc = neural.correction(weights["ee"], np.array([RC]), RC)
    assert f0[0][0] == 0.0 and f0[1][0] == 0.0 and f0[2][0] != 0.0
    assert all(abs(x[0]) < 1e-15 for x in fc)


def _orc(system=None, tab=None, rc=RC):
    s = system if system is not None else inputs.tiny_mixed(seed=3, n_up=2, n_dn=2)
    return oracle.Oracle(s, a=0.1, a_prime=0.15, r_c=0.4, ftab=tab, ftab_rcut=rc)


def test_hermite_reproduces_quintics(oracle_lib):
    rng = np.random.default_rng(2)
    c = rng.normal(size=6)
    p = np.polynomial.Polynomial(c)
    G = 13
    r = np.linspace(0.0, RC, G)
    tab = np.zeros((2, G, 3))
    tab[0, :, 0], tab[0, :, 1], tab[0, :, 2] = p(r), p.deriv(1)(r), p.deriv(2)(r)
    tab[1] = -tab[0]
    o = _orc(tab=tab)
    for x in rng.uniform(0, RC, 50):
        got = o.corr(0, x)
        ref = np.array([p(x), p.deriv(1)(x), p.deriv(2)(x)])
        assert np.allclose(got, ref, rtol=1e-11, atol=1e-11 * np.abs(c).sum() * RC ** 5)
        assert np.allclose(o.corr(1, x), -got, rtol=0, atol=0)
    assert np.all(o.corr(0, RC) == 0.0) and np.all(o.corr(0, RC + 1.0) == 0.0)


def test_interpolant_is_c2_across_nodes(oracle_lib, weights):
    G = 41
    tab = neural.tabulate(weights, G, RC)
    o = _orc(tab=tab)
    h = RC / (G - 1)
    for k in range(1, G - 1):
        left, right = o.corr(0, k * h - 1e-10), o.corr(0, k * h + 1e-10)
        assert np.allclose(left, right, rtol=1e-7, atol=1e-7)
        assert np.allclose(o.corr(0, k * h), tab[0, k], rtol=1e-12, atol=1e-13)


def test_zero_table_is_the_pade_trial_function(oracle_lib):
    s = inputs.tiny_mixed(seed=3, n_up=2, n_dn=2)
    pos = inputs.initial_walkers(s, 1, 4)[0]
    plain = _orc(s)
    zero = _orc(s, np.zeros((2, 9, 3)))
    assert zero.log_psi(pos) == plain.log_psi(pos)
    assert zero.local_energy(pos) == plain.local_energy(pos)


def test_derivatives_of_log_psi_with_correction(oracle_lib, weights):
    """sum_i lap_i Psi / Psi from the analytic path against central FD of
    Psi built from log Psi (the same check the Pade trial function passes)."""
    s = inputs.tiny_mixed(seed=3, n_up=2, n_dn=2)
    tab = neural.tabulate(weights, 601, RC)
    o = _orc(s, tab)
    rng = np.random.default_rng(5)
    for _ in range(3):
        pos = inputs.initial_walkers(s, 1, int(rng.integers(100)))[0]
        lap_exact = o.local_energy(pos)[1]
        l0, s0 = o.log_psi(pos)
        tot = 0.0
        for h in (2e-3, 1e-3):
            acc = 0.0
            for i in range(s.n_elec):
                for ax in range(3):
                    for sg in (1, -1):
                        p = pos.copy()
                        p[i, ax] += sg * h
                        l1, s1 = o.log_psi(p)
                        acc += (s0 * s1 * np.exp(l1 - l0) - 1.0) / h ** 2
            tot = acc if h == 2e-3 else (4 * acc - tot) / 3
        assert tot == pytest.approx(lap_exact, rel=2e-6, abs=1e-5)


def test_cusps_untouched(oracle_lib, weights):
    """E_L stays finite when an electron sits on another or on a nucleus."""
    s = inputs.tiny_mixed(seed=3, n_up=2, n_dn=2)
    o = _orc(s, neural.tabulate(weights, 301, RC))
    pos = inputs.initial_walkers(s, 1, 7)[0]
    for eps in (1e-3, 1e-5, 1e-7):
        p = pos.copy()
        p[1] = p[0] + eps * np.array([0.6, 0.0, 0.8])
        assert np.isfinite(o.local_energy(p)[0])
        q = pos.copy()
        q[2] = s.R[0] + eps * np.array([0.0, 1.0, 0.0])
        assert np.isfinite(o.local_energy(q)[0])
    e1 = o.local_energy(_shift(pos, 1e-6, s))[0]
    e2 = o.local_energy(_shift(pos, 1e-7, s))[0]
    assert abs(e1 - e2) < 1e-2 * (1 + abs(e1))


def _shift(pos, eps, s):
    p = pos.copy()
    p[1] = p[0] + eps * np.array([0.6, 0.0, 0.8])
    return p


def test_last_interval_up_to_the_cutoff(oracle_lib):
    """Just below r_c (where r/h can round up to the last node index) the
    interpolant still uses the last interval: it returns the end node's
    values of a quintic, not a neighbouring table entry."""
    rng = np.random.default_rng(4)
    p = np.polynomial.Polynomial(rng.normal(size=6))
    G = 10                                  # RC / (G - 1) is inexact here
    r = np.linspace(0.0, RC, G)
    tab = np.zeros((2, G, 3))
    for t in (0, 1):
        tab[t, :, 0], tab[t, :, 1], tab[t, :, 2] = p(r), p.deriv(1)(r), p.deriv(2)(r)
        tab[t] *= (1.0, -3.0)[t]
    o = _orc(tab=tab)
    x = np.nextafter(RC, 0.0)
    assert x / (RC / (G - 1)) == G - 1      # the rounding case
    for t in (0, 1):
        ref = (1.0, -3.0)[t] * np.array([p(RC), p.deriv(1)(RC), p.deriv(2)(RC)])
        assert np.allclose(o.corr(t, x), ref, rtol=1e-9, atol=1e-9)

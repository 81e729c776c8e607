"""Oracle pins: the whole projection (generation start, lattice moves, heat
bath, weights, reconfiguration, estimator) against exact energies.

* One electron, nodeless trial: the fixed-node constraint is void, so the
  lattice-regularized ground state tends to -1/2 as O(a^2).  The trial used
  here has a VMC energy of -0.451 Ha, far from the target.
* He with a nodeless orbital (positive coefficients) times the Pade
  Jastrow: fixed node is exact, so the a -> 0 extrapolation of
  E(a) = E0 + k1 a^2 must reach the exact -2.903724 Ha (supplement Table S-II).
  The double grid uses r_c(a, Z) of Eq. (S-13) and a'/a of Eq. (6).
"""
import os

import numpy as np
import pytest

import oracle
from oracle import estimator, spacing
from paper_1909_01589_amd import inputs

HERE = os.path.dirname(os.path.abspath(__file__))


def _fit_a2(a, E, err):
    """Weighted least squares E = E0 + k a^2; returns (E0, sigma_E0)."""
    A = np.stack([np.ones_like(a), a ** 2], axis=1)
    Wt = 1.0 / err ** 2
    cov = np.linalg.inv(A.T @ (A * Wt[:, None]))
    coef = cov @ (A.T @ (Wt * E))
    return coef[0], np.sqrt(cov[0, 0])


def _energy(o, system, W, n_eq, n_prod, seed):
    pos = inputs.initial_walkers(system, W, seed)
    r = o.run(pos, n_eq, gen0=0, want_idx=False)
    r = o.run(r["pos"], n_prod, gen0=n_eq, want_idx=False)
    return estimator.energy_and_error(r["log_wbar"], r["ebar"], p=8)


@pytest.mark.slow
def test_hydrogen_nodeless_gaussian_extrapolates_to_exact(oracle_lib):
    s = inputs.System(Z=np.array([1.0]), R=np.zeros((1, 3)), n_up=1, n_dn=0,
                      shell_nuc=[0], shell_l=[0], shell_alpha=[0.1], mo=np.ones((1, 1)),
                      b_ee=1.0, b_en=0.5)
    a_vals = np.array([0.6, 0.4, 0.3])
    E, err = [], []
    for a in a_vals:
        o = oracle.Oracle(s, a=a, a_prime=1.4 * a, r_c=0.8, tau=0.3, seed=3, rotate=1)
        e, de = _energy(o, s, 1024, 40, 800, 1)
        E.append(e)
        err.append(de)
    E, err = np.array(E), np.array(err)
    assert np.all(E < -0.49)                   # far below the VMC -0.451
    E0, sE0 = _fit_a2(a_vals, E, err)
    assert abs(E0 + 0.5) < 3 * sE0 + 2e-4, (E, err, E0, sE0)
    assert sE0 < 2e-3


@pytest.mark.slow
def test_helium_nodeless_extrapolates_to_exact(oracle_lib):
    exact = float(open(os.path.join(HERE, "golden", "exact_energies.txt")).read().split()[-1])
    s = inputs.helium_nodeless(alphas=(0.25, 0.9, 3.0), coefs=(0.3, 0.5, 0.2))
    a_vals = np.array([0.3, 0.2])
    E, err = [], []
    for a in a_vals:
        rc, ap, nc = spacing.spacing(2, a)
        assert ap > a
        o = oracle.Oracle(s, a=a, a_prime=ap, r_c=rc, tau=0.3, seed=5, rotate=1)
        e, de = _energy(o, s, 1024, 30, 500, 2)
        E.append(e)
        err.append(de)
    E, err = np.array(E), np.array(err)
    E0, sE0 = _fit_a2(a_vals, E, err)
    assert abs(E0 - exact) < 3 * sE0 + 2e-4, (E, err, E0, sE0)
    assert sE0 < 2.5e-3

"""Oracle pins: the energy estimator with correcting factors and its
blocking error (the paper states neither).

Correcting factors G_n = prod_{k=0}^{p} wbar_{n-k} (p + 1 factors, the
generation's own mean weight included), E_p = sum_n G_n ebar_n / sum_n G_n
over the generations with a full window (n >= p):
* a constant mean weight gives the plain mean of ebar for every p;
* five records with mean weights (2, 1, 4, 1/2, 1) and energies (1, ..., 5),
  worked out by hand for p = 0, 1, 2 (a window of p factors, or one shifted
  by a generation, gives another number in each case).
Blocking error (Flyvbjerg & Petersen, J. Chem. Phys. 91, 461 (1989)):
* white noise: the plain standard error;
* an AR(1) series x_t = phi x_{t-1} + e_t: the error of the mean tends to
  sigma_e / ((1 - phi) sqrt(n)), about 4.4x the naive value at phi = 0.9.
The package's host estimator must give the same numbers as the oracle's.
"""
import numpy as np
import pytest

from oracle import estimator
from paper_1909_01589_amd import stats

WBAR = np.array([2.0, 1.0, 4.0, 0.5, 1.0])
EBAR = np.array([1.0, 2.0, 3.0, 4.0, 5.0])


def test_constant_weight_gives_plain_mean():
    rng = np.random.default_rng(0)
    e = rng.normal(size=50) - 7.0
    for p in (0, 1, 3, 10):
        E = estimator.energy(np.full(50, 0.3), e, p=p)
        assert E == pytest.approx(e[p:].mean(), rel=1e-14)


@pytest.mark.parametrize("p,expected", [
    # p = 0: G = wbar_n: (2*1 + 1*2 + 4*3 + 0.5*4 + 1*5) / 8.5 = 23 / 8.5
    (0, 23.0 / 8.5),
    # p = 1: G_1..4 = 2*1, 1*4, 4*0.5, 0.5*1 = 2, 4, 2, 0.5:
    # (2*2 + 4*3 + 2*4 + 0.5*5) / 8.5 = 26.5 / 8.5
    (1, 26.5 / 8.5),
    # p = 2: G_2..4 = 2*1*4, 1*4*0.5, 4*0.5*1 = 8, 2, 2: (8*3 + 2*4 + 2*5) / 12
    (2, 42.0 / 12.0),
])
def test_hand_computed_records(p, expected):
    E = estimator.energy(np.log(WBAR), EBAR, p=p)
    assert E == pytest.approx(expected, rel=1e-14)
    E2, _ = estimator.energy_and_error(np.log(WBAR), EBAR, p=p)
    assert E2 == pytest.approx(expected, rel=1e-14)


def test_log_factors_window():
    lg = estimator.correcting_log_factors(np.log(WBAR), 2)
    assert np.all(np.isneginf(lg[:2]))
    assert np.allclose(np.exp(lg[2:]), [8.0, 2.0, 2.0], rtol=1e-14)


def test_blocking_error_white_noise():
    rng = np.random.default_rng(3)
    errs = []
    for _ in range(20):
        x = rng.normal(size=4096)
        errs.append(estimator.blocking_error(x) / (1.0 / np.sqrt(4096)))
    # the maximum over levels sits a little above the true error
    assert 0.9 < np.mean(errs) < 1.3


def test_blocking_error_ar1():
    rng = np.random.default_rng(4)
    phi, n = 0.9, 1 << 16
    exact = 1.0 / ((1.0 - phi) * np.sqrt(n))
    ratios = []
    for _ in range(8):
        e = rng.normal(size=n)
        x = np.empty(n)
        x[0] = e[0] / np.sqrt(1 - phi * phi)
        for t in range(1, n):
            x[t] = phi * x[t - 1] + e[t]
        naive = np.std(x, ddof=1) / np.sqrt(n)
        assert naive < 0.3 * exact
        ratios.append(estimator.blocking_error(x) / exact)
    assert 0.85 < np.mean(ratios) < 1.2, ratios


def test_package_estimator_matches_oracle():
    rng = np.random.default_rng(5)
    lw = rng.normal(size=300) * 0.05 + 0.2
    e = rng.normal(size=300) * 0.3 - 14.0
    for p in (0, 1, 4, 16):
        E_o, s_o = estimator.energy_and_error(lw, e, p=p)
        E_g, s_g = stats.estimate(lw, e, p=p)
        assert E_g == pytest.approx(E_o, rel=1e-13)
        assert s_g == pytest.approx(s_o, rel=1e-9)
    assert stats.reblock_error(e) == pytest.approx(estimator.blocking_error(e), rel=1e-12)

"""Oracle pins: heat-bath move choice, holding times and reconfiguration.

* The heat-bath choice picks move m with probability T_m / Delta (chi^2).
* Holding times tau_d = -ln(u)/Delta are exponential with mean 1/Delta.
* Systematic resampling: equal weights give the identity; each walker is
  copied floor(M w_j/W) or ceil(M w_j/W) times; the copies add up to M.
* Exact trial function (hydrogenic): every walker gets the same weight, the
  reconfiguration is the identity and every generation's energy is -Z^2/2.
"""
import numpy as np
import pytest
from scipy import stats

import oracle
from paper_1909_01589_amd import inputs


@pytest.fixture(scope="module")
def orc(oracle_lib):
    return oracle.Oracle(inputs.hydrogenic(1.0), a=0.1, a_prime=0.1, r_c=1.0, seed=11)


def test_select_frequencies(orc):
    rng = np.random.default_rng(0)
    T = rng.uniform(size=24) * (rng.uniform(size=24) > 0.3)
    n = 40000
    counts = np.zeros(24)
    for j in range(n):
        u2 = orc.draw(j, 0, 0, 0)[1]
        counts[orc.select(T, u2)] += 1
    assert np.all(counts[T == 0] == 0)
    nz = T > 0
    expected = n * T[nz] / T.sum()
    chi2 = np.sum((counts[nz] - expected) ** 2 / expected)
    assert stats.chi2.sf(chi2, nz.sum() - 1) > 0.001


def test_select_edges(orc):
    T = np.array([0.0, 1.0, 0.0, 2.0, 0.0])
    assert orc.select(T, 1e-300) == 1
    assert orc.select(T, 0.3334) == 3
    assert orc.select(T, 1.0 - 2 ** -53) == 3
    assert orc.select(np.zeros(4), 0.5) == -1


def test_holding_time_mean(orc):
    u = np.array([orc.draw(j, 1, 2, 0)[0] for j in range(20000)])
    Delta = 37.0
    td = -np.log(u) / Delta
    assert td.mean() == pytest.approx(1 / Delta, rel=0.03)
    assert stats.kstest(td * Delta, "expon").pvalue > 0.001


def test_reconfigure_equal_weights_identity(orc):
    for W in (1, 7, 512):
        for xi in (1e-9, 0.5, 1 - 1e-9):
            idx, lwb, eb = orc.reconfigure(np.full(W, 0.37), np.arange(W, dtype=float), xi)
            assert np.array_equal(idx, np.arange(W))
            assert lwb == pytest.approx(0.37, rel=1e-14)


def test_reconfigure_copy_counts(orc):
    rng = np.random.default_rng(5)
    for trial in range(20):
        W = int(rng.integers(2, 300))
        lw = rng.normal(size=W) * 2.0
        xi = rng.uniform()
        idx, lwb, eb = orc.reconfigure(lw, rng.normal(size=W), xi)
        assert np.all(np.diff(idx) >= 0)
        w = np.exp(lw - lw.max())
        target = W * w / w.sum()
        copies = np.bincount(idx, minlength=W)
        assert copies.sum() == W
        assert np.all(copies >= np.floor(target - 1e-9)) and np.all(copies <= np.ceil(target + 1e-9))
        assert lwb == pytest.approx(np.log(np.mean(np.exp(lw))), rel=1e-12)


def test_reconfigure_weighted_energy(orc):
    lw = np.log(np.array([1.0, 3.0, 0.0 + 1e-300, 4.0]))
    e = np.array([1.0, 2.0, 100.0, -1.0])
    idx, lwb, eb = orc.reconfigure(lw, e, 0.5)
    assert eb == pytest.approx((1 + 6 - 4) / 8, rel=1e-14)


def test_hydrogenic_run_is_exact(oracle_lib):
    """Zero-variance trial: E_L = -Z^2/2 for every walker, so all weights
    agree, reconfiguration is the identity and ebar_n = -Z^2/2."""
    Z = 2.0
    s = inputs.hydrogenic(Z)
    o = oracle.Oracle(s, a=0.15, a_prime=0.25, r_c=0.4, tau=0.05, seed=3, rotate=1)
    pos = inputs.initial_walkers(s, 64, 0) * 0.5
    r = o.run(pos, 6)
    assert np.allclose(r["ebar"], -Z * Z / 2, rtol=1e-12)
    assert np.allclose(r["log_wbar"], 0.05 * Z * Z / 2, rtol=1e-10)
    assert np.all(r["idx"] == np.arange(64)[None, :])
    assert np.all(r["n_moves"] > 0)


def test_generation_is_deterministic_and_moves_one_electron_per_step(oracle_lib):
    s = inputs.be_like(0)
    o = oracle.Oracle(s, a=0.2, a_prime=0.2813, r_c=0.4417, tau=0.02, seed=1)
    pos = inputs.initial_walkers(s, 1, 0)[0]
    a = o.generation(pos, 3, 5)
    b = o.generation(pos, 3, 5)
    assert np.array_equal(a[0], b[0]) and a[1:] == b[1:]
    c = o.generation(pos, 4, 5)
    assert not np.array_equal(a[0], c[0]) or a[3] == 0
    moved = np.sum(np.any(a[0] != pos, axis=1))
    assert moved <= a[3]


def test_reconfigure_is_unbiased_over_xi(orc):
    """Averaged over the uniform offset xi, walker j is copied M w_j / sum w
    times (systematic resampling is unbiased)."""
    rng = np.random.default_rng(8)
    W = 13
    lw = rng.normal(size=W)
    w = np.exp(lw - lw.max())
    target = W * w / w.sum()
    xs = (np.arange(4000) + 0.5) / 4000
    mean = np.zeros(W)
    for xi in xs:
        idx, _, _ = orc.reconfigure(lw, np.zeros(W), xi)
        mean += np.bincount(idx, minlength=W)
    mean /= len(xs)
    assert np.allclose(mean, target, atol=2e-3)

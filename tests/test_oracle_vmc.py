"""Pins of the oracle's Metropolis sampler of |Psi|^2.

* Hydrogenic trial function Psi = exp(-Z r) (exact ground state): the
  sampled density is r^2 exp(-2 Z r), so <r> = 3/(2Z), <r^2> = 3/Z^2, each
  Cartesian second moment is 1/Z^2 and first moment 0; E_L = -Z^2/2 at every
  configuration.  Means from a long chain, errors by reblocking.
* Two independent hydrogenic electrons (no electron-electron Jastrow,
  opposite spins): the same marginals per electron.
* The chain is a deterministic function of (seed, slot, generation).
"""
import numpy as np
import pytest

import oracle
from paper_1909_01589_amd import inputs


def _blocked_error(x):
    x = np.asarray(x, dtype=np.float64)
    errs = []
    while x.size >= 32:
        errs.append(x.std(ddof=1) / np.sqrt(x.size))
        x = 0.5 * (x[: x.size // 2 * 2: 2] + x[1: x.size // 2 * 2: 2])
    return max(errs)


def _chain(o, pos, n_samples, stride, step, slot=0):
    out, acc = [], 0
    for g in range(n_samples):
        pos, a, el = o.vmc(pos, slot, g, stride, step)
        acc += a
        out.append(pos.copy())
    return np.array(out), acc / (n_samples * stride), el


@pytest.mark.parametrize("Z,step", [(1.0, 1.2), (2.0, 0.6)])
def test_hydrogenic_moments(oracle_lib, Z, step):
    s = inputs.hydrogenic(Z)
    o = oracle.Oracle(s, 0.1, 0.1, 1.0, seed=5)
    pos = np.array([[0.3, -0.2, 0.4]]) / Z
    pos, _, _ = o.vmc(pos, 0, 10 ** 6, 2000, step)      # equilibrate
    xs, acc, el = _chain(o, pos, 20000, 10, step)
    assert 0.2 < acc < 0.9
    assert el == pytest.approx(-0.5 * Z * Z, abs=1e-12)
    x = xs[:, 0, :]
    r = np.linalg.norm(x, axis=1)
    for val, ref in ((r, 1.5 / Z), (r * r, 3.0 / Z ** 2)):
        assert abs(val.mean() - ref) < 4.5 * _blocked_error(val), (val.mean(), ref)
    for c in range(3):
        assert abs(x[:, c].mean()) < 4.5 * _blocked_error(x[:, c])
        assert abs((x[:, c] ** 2).mean() - 1.0 / Z ** 2) < 4.5 * _blocked_error(x[:, c] ** 2)


def test_two_independent_electrons(oracle_lib):
    s = inputs.hydrogenic(1.0)
    s2 = inputs.System(Z=s.Z, R=s.R, n_up=1, n_dn=1, shell_nuc=[0], shell_l=[0], shell_alpha=[0.0],
                       mo=np.ones((1, 1)), b_ee=1.0, b_en=0.0, name="two")
    o = oracle.Oracle(s2, 0.1, 0.1, 1.0, seed=2)
    # |Psi|^2 = exp(-2 r1 - 2 r2 + 2 J_ee): reweighting by exp(-2 J_ee)
    # gives the product density, whose marginals have <r> = 3/2
    pos = np.array([[0.5, 0.0, 0.0], [-0.5, 0.2, 0.0]])
    pos, _, _ = o.vmc(pos, 0, 10 ** 6, 2000, 1.0)
    xs, acc, _ = _chain(o, pos, 12000, 10, 1.0)
    r12 = np.linalg.norm(xs[:, 0] - xs[:, 1], axis=1)
    w = np.exp(-2.0 * 0.5 * r12 / (1.0 + r12))          # |Psi_0|^2 / |Psi|^2 with J_ee = r/(2(1+r))
    for e in (0, 1):
        r = np.linalg.norm(xs[:, e], axis=1)
        est = (w * r).sum() / w.sum()
        assert est == pytest.approx(1.5, abs=0.06)


def test_chain_is_deterministic(oracle_lib):
    s = inputs.tiny_mixed(seed=1, n_up=2, n_dn=1)
    o = oracle.Oracle(s, 0.1, 0.15, 0.4, seed=3)
    pos = inputs.initial_walkers(s, 1, 0)[0]
    a = o.vmc(pos, 4, 7, 50, 0.5)
    b = o.vmc(pos, 4, 7, 50, 0.5)
    c = o.vmc(pos, 5, 7, 50, 0.5)
    assert np.array_equal(a[0], b[0]) and a[1] == b[1]
    assert not np.array_equal(a[0], c[0])

"""Oracle pins: trial wave function, move ratios and local energy.

Each check uses a route independent of the oracle's own arithmetic:
central finite differences, numpy's determinant and inverse, the exact
hydrogenic solution, and the cusp conditions of the Coulomb Hamiltonian.
"""
import numpy as np
import pytest

import oracle
from paper_1909_01589_amd import inputs


@pytest.fixture(scope="module")
def tiny(oracle_lib):
    s = inputs.tiny_mixed(seed=1, n_up=3, n_dn=2)
    return oracle.Oracle(s, a=0.05, a_prime=0.08, r_c=0.5, z_heavy=3.0)


@pytest.fixture(scope="module")
def be(oracle_lib):
    return oracle.Oracle(inputs.be_like(0), a=0.2, a_prime=0.2813, r_c=0.4417)


def _fd_basis(o, r, h=1e-5):
    g = np.zeros((o.K, 3))
    lap = np.zeros(o.K)
    v0 = o.basis(r)[0]
    for c in range(3):
        e = np.zeros(3)
        e[c] = h
        vp, vm = o.basis(r + e)[0], o.basis(r - e)[0]
        g[:, c] = (vp - vm) / (2 * h)
        lap += (vp - 2 * v0 + vm) / h ** 2
    return v0, g, lap


def test_basis_derivatives_match_finite_differences(tiny):
    rng = np.random.default_rng(3)
    for _ in range(10):
        r = rng.normal(size=3) * 0.8
        v, g, l = tiny.basis(r)
        v0, gf, lf = _fd_basis(tiny, r)
        scale = np.max(np.abs(v)) + 1.0
        assert np.allclose(g, gf, atol=2e-8 * scale)
        assert np.allclose(l, lf, atol=5e-4 * scale)


def test_d_shell_components_are_harmonic(tiny):
    """The five l=2 forms are harmonic polynomials: with alpha -> 0 their
    Laplacian vanishes."""
    s = inputs.System(Z=np.array([1.0]), R=np.zeros((1, 3)), n_up=1, n_dn=0,
                      shell_nuc=[0], shell_l=[2], shell_alpha=[0.0], mo=np.eye(5)[:, :1])
    o = oracle.Oracle(s, a=0.1, a_prime=0.1, r_c=1.0)
    rng = np.random.default_rng(0)
    for _ in range(5):
        v, g, l = o.basis(rng.normal(size=3))
        assert np.allclose(l, 0.0, atol=1e-13)


def test_log_psi_determinant_against_numpy(tiny):
    """det A_up det A_dn from the oracle's LU equals numpy's determinant of
    the orbital matrices built from the oracle's basis values."""
    s = tiny.system
    pos = inputs.initial_walkers(s, 1, 5)[0]
    la, sg = tiny.log_psi(pos)
    J = tiny.jastrow(pos)
    det = 1.0
    for i0, n in ((0, s.n_up), (s.n_up, s.n_dn)):
        A = np.array([tiny.basis(pos[i0 + i])[0] @ s.mo[:, :n] for i in range(n)])
        det *= np.linalg.det(A)
    assert np.sign(det) == sg
    assert la - J == pytest.approx(np.log(abs(det)), abs=1e-11)


def test_move_ratios_match_determinant_lemma(tiny):
    """Psi(x')/Psi(x) = (phi(r') . Ainv[:, i]) * exp(J(x') - J(x)), with the
    inverse and J difference taken from numpy and the oracle's J."""
    s = tiny.system
    pos = inputs.initial_walkers(s, 1, 6)[0]
    rho, k, d = tiny.eval_moves(pos)
    J0 = tiny.jastrow(pos)
    for m in range(0, tiny.M, 5):
        i = m // 12
        sg0, n = (0, s.n_up) if i < s.n_up else (s.n_up, s.n_dn)
        A = np.array([tiny.basis(pos[sg0 + q])[0] @ s.mo[:, :n] for q in range(n)])
        rp, _ = tiny.move(pos, np.eye(3), m)
        phi = tiny.basis(rp)[0] @ s.mo[:, :n]
        det_ratio = phi @ np.linalg.inv(A)[:, i - sg0]
        p2 = pos.copy()
        p2[i] = rp
        expect = det_ratio * np.exp(tiny.jastrow(p2) - J0)
        assert rho[m] == pytest.approx(expect, rel=1e-10, abs=1e-12)


def _fd_lap_psi(o, pos, h=2e-4):
    """sum_i lap_i Psi / Psi = sum (lap log Psi + |grad log Psi|^2), central
    differences with one Richardson step (error O(h^4))."""
    return (4.0 * _fd_lap_psi_h(o, pos, h / 2) - _fd_lap_psi_h(o, pos, h)) / 3.0


def _fd_lap_psi_h(o, pos, h):
    l0, _ = o.log_psi(pos)
    tot = 0.0
    for i in range(pos.shape[0]):
        for c in range(3):
            p = pos.copy(); p[i, c] += h
            m = pos.copy(); m[i, c] -= h
            lp, _ = o.log_psi(p)
            lm, _ = o.log_psi(m)
            g = (lp - lm) / (2 * h)
            tot += (lp - 2 * l0 + lm) / h ** 2 + g * g
    return tot


@pytest.mark.parametrize("fixture", ["tiny", "be"])
def test_local_energy_laplacian_matches_finite_differences(fixture, request):
    o = request.getfixturevalue(fixture)
    for seed in range(3):
        pos = inputs.initial_walkers(o.system, 1, 10 + seed)[0]
        e, lap, v = o.local_energy(pos)
        fd = _fd_lap_psi(o, pos)
        assert lap == pytest.approx(fd, rel=2e-5, abs=2e-5)
        assert e == pytest.approx(-0.5 * lap + v, rel=1e-14)


def test_potential_brute_force(tiny):
    s = tiny.system
    pos = inputs.initial_walkers(s, 1, 2)[0]
    V = 0.0
    for i in range(s.n_elec):
        for j in range(i + 1, s.n_elec):
            V += 1 / np.linalg.norm(pos[i] - pos[j])
        for I in range(s.n_nuc):
            V -= s.Z[I] / np.linalg.norm(pos[i] - s.R[I])
    V += s.Z[0] * s.Z[1] / np.linalg.norm(s.R[0] - s.R[1])
    assert tiny.potential(pos) == pytest.approx(V, rel=1e-13)


@pytest.mark.parametrize("Z", [1.0, 2.0, 3.0, 7.5])
def test_hydrogenic_zero_variance(oracle_lib, Z):
    """Psi = exp(-Z r) is the exact ground state of one electron around
    charge Z: E_L = -Z^2/2 everywhere, for the analytic and the lattice-
    assembled local energy at any spacing."""
    o = oracle.Oracle(inputs.hydrogenic(Z), a=0.11, a_prime=0.23, r_c=0.4)
    rng = np.random.default_rng(int(Z * 10))
    for _ in range(20):
        pos = rng.normal(size=(1, 3)) * 1.5 / Z
        e, lap, v = o.local_energy(pos)
        assert e == pytest.approx(-Z * Z / 2, rel=1e-13)
        rho, k, d = o.eval_moves(pos, o.rotation(rng.uniform(size=3)))
        assert d["e_lattice"] == pytest.approx(-Z * Z / 2, rel=1e-10)
        assert np.all(rho > 0)


def test_lattice_local_energy_equals_analytic(tiny, be):
    """With V^a = V + (L^a - lap Psi/Psi)/2 the fixed-node lattice local
    energy sum k/2 + V^a + V_sf - Delta equals E_L identically."""
    for o in (tiny, be):
        for seed in range(4):
            pos = inputs.initial_walkers(o.system, 1, 30 + seed)[0]
            rho, k, d = o.eval_moves(pos, o.rotation(np.random.default_rng(seed).uniform(size=3)))
            scale = d["sum_k"] + abs(d["e_l"])
            assert abs(d["e_lattice"] - d["e_l"]) < 1e-11 * scale


def test_electron_electron_cusp(oracle_lib):
    """The Jastrow cusps (1/2 antiparallel, 1/4 parallel) cancel the 1/r
    divergence of the e-e Coulomb term: E_L stays bounded as r_12 -> 0."""
    for n_up, n_dn in ((1, 1), (2, 0)):
        s = inputs.System(Z=np.array([2.0]), R=np.zeros((1, 3)), n_up=n_up, n_dn=n_dn,
                          shell_nuc=[0, 0], shell_l=[0, 1], shell_alpha=[0.5, 0.5],
                          mo=np.array([[1.0, 0.0], [0.0, 1.0], [0.3, 0.0], [0.0, 0.2]]))
        o = oracle.Oracle(s, a=0.1, a_prime=0.1, r_c=1.0)
        base = np.array([[0.4, 0.3, 0.2], [0.4, 0.3, 0.2]])
        d = np.array([0.3, -0.5, 0.8]) / np.linalg.norm([0.3, -0.5, 0.8])
        vals = []
        for r in (1e-3, 1e-4, 1e-5, 1e-6):
            p = base.copy()
            p[1] += r * d
            vals.append(o.local_energy(p)[0])
        assert max(vals) - min(vals) < 0.05, vals


def test_electron_nucleus_cusp(oracle_lib):
    """The e-n Pade factor -Z r/(1+b r) supplies the nuclear cusp that the
    Gaussian orbitals lack: E_L stays bounded as r_iI -> 0."""
    s = inputs.be_like(0)
    o = oracle.Oracle(s, a=0.2, a_prime=0.28, r_c=0.44)
    pos = inputs.initial_walkers(s, 1, 4)[0]
    d = np.array([0.6, 0.0, -0.8])
    vals = []
    for r in (1e-3, 1e-4, 1e-5, 1e-6):
        p = pos.copy()
        p[0] = r * d
        vals.append(o.local_energy(p)[0])
    assert max(vals) - min(vals) < 0.05 * (1 + abs(vals[0])), vals

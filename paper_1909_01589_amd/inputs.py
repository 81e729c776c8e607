"""Seeded synthetic inputs for the double-grid LRDMC projection step.

This module is shared by the HIP path and by the CPU oracle's tests.  It only
lays out systems (nuclei, Gaussian shells, a random orthonormal MO matrix,
Pade Jastrow constants) and draws initial electron positions.  It holds none
of the method's arithmetic: no wave-function values, no lattice spacings
derived from the paper's formulas, no energies.

Every system stands in for the paper's all-electron atoms (He...Xe, main-text
Table I) and for a benzene-sized molecule (main-text Table II).  The paper's
own basis sets and optimized JAGP wave functions are not available, so the
shapes follow the paper (atomic number Z, electron count, a basis size close to
the paper's determinant basis, lattice spacing a = (3.5 Z)^-1 for the
Z-sweep) while the coefficients are seeded random numbers.

Basis convention: each shell is an uncontracted, unnormalized Cartesian-
harmonic Gaussian P_l(d) exp(-alpha |d|^2), d = r - R_nucleus, with l in
{0, 1, 2} contributing 1, 3 and 5 functions.  Functions are ordered by
nucleus, then by shell (all s, then all p, then all d), then by exponent.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace
from typing import Dict, Optional

import numpy as np

__all__ = [
    "System", "basis_alloc", "atom", "be_like", "ar_like", "zsweep_atom",
    "molecule", "hydrogenic", "helium_nodeless", "initial_walkers", "CONFIGS",
    "Config", "get_config",
]


@dataclass
class System:
    """One trial-function system: nuclei, basis shells, MO matrix, Jastrow."""

    Z: np.ndarray            # [n_nuc] nuclear charges
    R: np.ndarray            # [n_nuc, 3] nuclear positions (bohr)
    n_up: int
    n_dn: int
    shell_nuc: np.ndarray    # [n_shell] int32 nucleus of each shell
    shell_l: np.ndarray      # [n_shell] int32 angular momentum 0, 1, 2
    shell_alpha: np.ndarray  # [n_shell] float64 Gaussian exponent
    mo: np.ndarray           # [K, n_orb] MO coefficients, shared by both spins
    b_ee: float = 1.0
    b_en: float = 1.0
    name: str = ""

    def __post_init__(self):
        self.Z = np.ascontiguousarray(self.Z, dtype=np.float64)
        self.R = np.ascontiguousarray(np.reshape(self.R, (-1, 3)), dtype=np.float64)
        self.shell_nuc = np.ascontiguousarray(self.shell_nuc, dtype=np.int32)
        self.shell_l = np.ascontiguousarray(self.shell_l, dtype=np.int32)
        self.shell_alpha = np.ascontiguousarray(self.shell_alpha, dtype=np.float64)
        self.mo = np.ascontiguousarray(self.mo, dtype=np.float64)

    @property
    def n_nuc(self) -> int:
        return int(self.Z.shape[0])

    @property
    def n_elec(self) -> int:
        return int(self.n_up + self.n_dn)

    @property
    def n_shell(self) -> int:
        return int(self.shell_l.shape[0])

    @property
    def n_basis(self) -> int:
        return int(np.sum(2 * self.shell_l + 1))

    @property
    def n_orb(self) -> int:
        return int(self.mo.shape[1])

    @property
    def z_max(self) -> float:
        return float(np.max(self.Z))

    @property
    def n_moves(self) -> int:
        """Lattice moves per walker: 2 grids x 6 directions per electron."""
        return 12 * self.n_elec


def basis_alloc(K: int):
    """Split a total basis size K into (K_s, K_p, K_d) shells of one nucleus."""
    K_d = int(math.floor(K / 16.0 + 0.5))
    K_p = int(math.floor((K - 5 * K_d) / 4.0))
    K_s = K - 5 * K_d - 3 * K_p
    return K_s, K_p, K_d


def _even_tempered(alpha0: float, beta: float, n: int) -> np.ndarray:
    return alpha0 * beta ** np.arange(n, dtype=np.float64)


def _shells_for(nuc: int, counts, alpha0: float, beta: float):
    nuc_l, l_l, a_l = [], [], []
    for l, n in enumerate(counts):
        for alpha in _even_tempered(alpha0, beta, n):
            nuc_l.append(nuc)
            l_l.append(l)
            a_l.append(alpha)
    return nuc_l, l_l, a_l


def _random_mo(rng: np.random.Generator, K: int, n_orb: int) -> np.ndarray:
    """First n_orb columns of Q from QR of a K x K N(0,1) matrix, diag(R) > 0."""
    G = rng.standard_normal((K, K))
    Q, Rm = np.linalg.qr(G)
    Q = Q * np.sign(np.diag(Rm))[None, :]
    return np.ascontiguousarray(Q[:, :n_orb])


def _streams(seed: int, n: int = 3):
    return [np.random.default_rng(s) for s in np.random.SeedSequence(seed).spawn(n)]


def atom(Z: int, counts, alpha0: float, beta: float, seed: int = 0,
         b_ee: float = 1.0, b_en: float = 1.0, name: str = "") -> System:
    """Neutral closed-shell-like atom at the origin with Z/2 up and Z/2 down."""
    n_up = (Z + 1) // 2
    n_dn = Z // 2
    nuc_l, l_l, a_l = _shells_for(0, counts, alpha0, beta)
    K = int(sum((2 * l + 1) for l in l_l))
    mo_rng, _, _ = _streams(seed)
    mo = _random_mo(mo_rng, K, max(n_up, n_dn))
    return System(Z=np.array([float(Z)]), R=np.zeros((1, 3)), n_up=n_up, n_dn=n_dn,
                  shell_nuc=nuc_l, shell_l=l_l, shell_alpha=a_l, mo=mo,
                  b_ee=b_ee, b_en=b_en, name=name or f"Z{Z}")


def be_like(seed: int = 0) -> System:
    """Be-like atom: Z=4, 2 up 2 down, 8 even-tempered s Gaussians 0.1*3^k."""
    return atom(4, (8, 0, 0), 0.1, 3.0, seed=seed, name="be")


def ar_like(seed: int = 0) -> System:
    """Ar-like atom: Z=18, 9 up 9 down, K=64 s/p/d Gaussians 0.05*2.5^k."""
    return atom(18, basis_alloc(64), 0.05, 2.5, seed=seed, name="ar")


def zsweep_atom(Z: int, seed: int = 0) -> System:
    """Z-sweep atom with K = 8*ceil(Z/4) s/p/d Gaussians on 0.05*2.5^k."""
    K = 8 * int(math.ceil(Z / 4.0))
    return atom(Z, basis_alloc(K), 0.05, 2.5, seed=seed, name=f"zsweep{Z}")


def molecule(seed: int = 0) -> System:
    """4 nuclei Z=8 and 8 nuclei Z=1 in a 4-bohr ball, 20 up / 20 down."""
    mo_rng, geo_rng, _ = _streams(seed)
    pts = []
    while len(pts) < 12:
        p = geo_rng.uniform(-4.0, 4.0, size=3)
        if np.dot(p, p) > 16.0:
            continue
        if all(np.linalg.norm(p - q) >= 1.8 for q in pts):
            pts.append(p)
    Z = np.array([8.0] * 4 + [1.0] * 8)
    nuc_l, l_l, a_l = [], [], []
    for I in range(12):
        counts = (11, 8, 3) if Z[I] == 8.0 else (4, 1, 0)
        a, b, c = _shells_for(I, counts, 0.05, 2.5)
        nuc_l += a
        l_l += b
        a_l += c
    K = int(sum((2 * l + 1) for l in l_l))
    mo = _random_mo(mo_rng, K, 20)
    return System(Z=Z, R=np.array(pts), n_up=20, n_dn=20, shell_nuc=nuc_l,
                  shell_l=l_l, shell_alpha=a_l, mo=mo, name="molecule")


def hydrogenic(Z: float = 1.0) -> System:
    """One electron, one constant s function (alpha=0), b_en=0: Psi = exp(-Z r)."""
    return System(Z=np.array([float(Z)]), R=np.zeros((1, 3)), n_up=1, n_dn=0,
                  shell_nuc=[0], shell_l=[0], shell_alpha=[0.0], mo=np.ones((1, 1)),
                  b_ee=1.0, b_en=0.0, name=f"hydrogenic{Z:g}")


def helium_nodeless(alphas=(0.3, 1.0, 3.5), coefs=(0.3, 0.5, 0.25),
                    b_ee: float = 1.0, b_en: float = 1.0) -> System:
    """He, 1 up 1 down, one nodeless s orbital (positive coefficients) x Pade."""
    return System(Z=np.array([2.0]), R=np.zeros((1, 3)), n_up=1, n_dn=1,
                  shell_nuc=[0] * len(alphas), shell_l=[0] * len(alphas),
                  shell_alpha=list(alphas), mo=np.array(coefs, dtype=np.float64)[:, None],
                  b_ee=b_ee, b_en=b_en, name="helium")


def tiny_mixed(seed: int = 1, n_up: int = 2, n_dn: int = 1) -> System:
    """Two nuclei with s/p/d shells and few electrons: small test system."""
    mo_rng, geo_rng, _ = _streams(seed)
    R = np.array([[0.0, 0.0, 0.0], [0.3, -0.4, 1.4]]) + 0.01 * geo_rng.standard_normal((2, 3))
    Z = np.array([3.0, 1.0])
    nuc_l, l_l, a_l = [], [], []
    for I, counts in enumerate(((2, 2, 1), (2, 1, 0))):
        a, b, c = _shells_for(I, counts, 0.4, 3.0)
        nuc_l += a
        l_l += b
        a_l += c
    K = int(sum((2 * l + 1) for l in l_l))
    mo = _random_mo(mo_rng, K, max(n_up, n_dn, 1))
    return System(Z=Z, R=R, n_up=n_up, n_dn=n_dn, shell_nuc=nuc_l, shell_l=l_l,
                  shell_alpha=a_l, mo=mo, b_ee=1.0, b_en=1.0, name="tiny_mixed")


def initial_walkers(system: System, W: int, seed: int = 0) -> np.ndarray:
    """Initial positions [W, N, 3]: each electron at its nucleus + N(0, 1 bohr^2).

    Electrons are assigned to nuclei so that nucleus I receives Z_I electrons
    (rounded), up electrons first: the up list visits nuclei in order, taking
    ceil(Z_I/2) from each, the down list floor(Z_I/2); hydrogen-like nuclei
    alternate between the two lists.  Surplus or missing electrons go to the
    heaviest nucleus.
    """
    _, _, w_rng = _streams(seed)
    up_sites, dn_sites = [], []
    odd_toggle = 0
    for I in range(system.n_nuc):
        z = int(round(system.Z[I]))
        nu, nd = z // 2, z // 2
        if z % 2:
            if odd_toggle == 0:
                nu += 1
            else:
                nd += 1
            odd_toggle ^= 1
        up_sites += [I] * nu
        dn_sites += [I] * nd
    heavy = int(np.argmax(system.Z))
    up_sites = (up_sites + [heavy] * system.n_up)[: system.n_up]
    dn_sites = (dn_sites + [heavy] * system.n_dn)[: system.n_dn]
    sites = np.array(up_sites + dn_sites, dtype=np.int64)
    centers = system.R[sites] if len(sites) else np.zeros((0, 3))
    pos = centers[None, :, :] + w_rng.standard_normal((W, system.n_elec, 3))
    return np.ascontiguousarray(pos, dtype=np.float64)


@dataclass
class Config:
    """A named workload: system, small spacing a, walkers, generations, tau."""

    name: str
    system: System
    a: float
    walkers: int
    generations: int
    tau: float                 # projection time per generation (1/Ha)
    rotate: int = 1
    seed: int = 0
    refresh: int = 8           # generations between full walker-state recomputations
    extra: Dict = field(default_factory=dict)


def _configs() -> Dict[str, Config]:
    # tau follows the rule "about one move per electron per generation":
    # tau = N / <Delta>, <Delta> = mean total move rate of 512 walkers after
    # 60 generations of equilibration on the MI355X, frozen here with three
    # significant figures.
    out = {
        "be": Config("be", be_like(0), a=0.2, walkers=512, generations=500, tau=0.0217),
        "ar_a0.2": Config("ar_a0.2", ar_like(0), a=0.2, walkers=4096, generations=2000, tau=0.0375),
        "ar_a0.1": Config("ar_a0.1", ar_like(0), a=0.1, walkers=4096, generations=2000, tau=0.00842),
        "molecule": Config("molecule", molecule(0), a=1.0 / 28.0, walkers=16384, generations=100, tau=0.00179),
    }
    for Z, tau in ((10, 0.00115), (18, 0.000473), (36, 0.000167), (54, 0.0000912)):
        out[f"zsweep{Z}"] = Config(f"zsweep{Z}", zsweep_atom(Z, 0), a=1.0 / (3.5 * Z),
                                   walkers=8192, generations=100, tau=tau)
    return out


CONFIGS = _configs()


def get_config(name: str, **overrides) -> Config:
    c = CONFIGS[name]
    return replace(c, **overrides) if overrides else c


def neural_weights(seed: int = 0, hidden: int = 64, out_scale: float = 0.1) -> dict:
    """Seeded weights of the two correction networks (electron pairs "ee",
    electron-nucleus pairs "en"), each 1 -> hidden -> hidden -> 1: W1[h],
    b1[h], W2[h][h], b2[h], w3[h], b3 (float64 arrays; scaled normal draws,
    the output layer damped by out_scale)."""
    rng = np.random.default_rng([seed, 77])
    out = {}
    for kind in ("ee", "en"):
        out[kind] = {
            "W1": rng.normal(size=hidden) * 2.0,
            "b1": rng.normal(size=hidden) * 0.5,
            "W2": rng.normal(size=(hidden, hidden)) / np.sqrt(hidden),
            "b2": rng.normal(size=hidden) * 0.1,
            "w3": rng.normal(size=hidden) / np.sqrt(hidden) * out_scale,
            "b3": np.array(0.0),
        }
    return out


def jastrow_table(seed: int = 0, n_nodes: int = 33, r_cut: float = 4.0, scale: float = 0.2) -> np.ndarray:
    """Node table [2][n_nodes][3] = {F, F', F''} at r_k = k r_cut / (n_nodes - 1)
    of a smooth random radial function per pair type (0: electron pairs,
    1: electron-nucleus): F(r) = scale r^2 (1 - r/r_cut)^3 P(r/r_cut) with P
    a random cubic; values and derivatives exact (numpy polynomials)."""
    P = np.polynomial.Polynomial
    rng = np.random.default_rng([seed, 91])
    r = np.linspace(0.0, r_cut, n_nodes)
    env = P([0.0, 0.0, 1.0]) * P([1.0, -1.0 / r_cut]) ** 3
    tab = np.zeros((2, n_nodes, 3))
    for t in range(2):
        f = scale * env * P(rng.normal(size=4))(P([0.0, 1.0 / r_cut]))
        tab[t, :, 0], tab[t, :, 1], tab[t, :, 2] = f(r), f.deriv(1)(r), f.deriv(2)(r)
    return tab


# Occupied orbitals of the closed s/p shells in filling order: (n, l, axis);
# axis 0/1/2 = x/y/z for p.
_SP_ORBITALS = ((1, 0, 0), (2, 0, 0), (2, 1, 0), (2, 1, 1), (2, 1, 2), (3, 0, 0), (3, 1, 0), (3, 1, 1), (3, 1, 2))


def _slater_zeff(Z: int, n: int) -> float:
    """Slater's screening rules for an s/p electron of shell n of the neutral
    atom with closed s/p shells filled in the order 1s 2s2p 3s3p."""
    cap = {1: 2, 2: 8, 3: 8}
    occ, left = {}, Z
    for m in (1, 2, 3):
        occ[m] = min(cap[m], left)
        left -= occ[m]
    s = (occ[n] - 1) * (0.30 if n == 1 else 0.35)
    if n >= 2:
        s += 0.85 * occ[n - 1]
    if n >= 3:
        s += 1.0 * sum(occ[m] for m in range(1, n - 1))
    return Z - s


def _hydrogenic_radial(n: int, l: int, zeta: float, r: np.ndarray) -> np.ndarray:
    """g(r) with orbital = g(r) for s and x_axis g(r) for p: screened
    hydrogenic shapes of shells 1 to 3 (unnormalized)."""
    x = zeta * r
    if (n, l) == (1, 0):
        return np.exp(-x)
    if (n, l) == (2, 0):
        return (2.0 - x) * np.exp(-x / 2.0)
    if (n, l) == (2, 1):
        return np.exp(-x / 2.0)
    if (n, l) == (3, 0):
        return (27.0 - 18.0 * x + 2.0 * x * x) * np.exp(-x / 3.0)
    if (n, l) == (3, 1):
        return (6.0 - x) * np.exp(-x / 3.0)
    raise ValueError("shells 1s to 3p only")


def atom_screened(Z: int, counts, alpha0: float, beta: float, b_ee: float = 1.0, b_en: float = 3.0,
                  name: str = "") -> System:
    """Closed-shell atom (Z in 2, 4, 10, 12, 18) whose determinant, times the
    electron-nucleus Pade factor exp(-Z r / (1 + b_en r)), approximates
    Slater-screened hydrogenic orbitals: each MO column is the weighted
    least-squares fit (weight r^(2 + 2l) on a radial grid) of
    g(r) exp(+Z r / (1 + b_en r)) by the basis functions of its angular type.
    A trial function with physically placed nodes, in the same even-tempered
    basis as `atom`."""
    if Z not in (2, 4, 10, 12, 18):
        raise ValueError("closed s/p shells only: Z in 2, 4, 10, 12, 18")
    n_up = n_dn = Z // 2
    nuc_l, l_l, a_l = _shells_for(0, counts, alpha0, beta)
    K = int(sum((2 * l + 1) for l in l_l))
    # first function index of every shell
    first, at = [], 0
    for l in l_l:
        first.append(at)
        at += 2 * l + 1
    r = np.geomspace(1e-5, 20.0, 6000)
    dr = np.gradient(r)
    jen = np.exp(-Z * r / (1.0 + b_en * r))
    mo = np.zeros((K, n_up))
    for j, (n, l, axis) in enumerate(_SP_ORBITALS[:n_up]):
        g = _hydrogenic_radial(n, l, _slater_zeff(Z, n), r)
        cols = [q for q, ll in enumerate(l_l) if ll == l]
        Bm = np.stack([jen * np.exp(-a_l[q] * r * r) for q in cols], axis=1)
        w = np.sqrt(r ** (2 + 2 * l) * dr)
        c, *_ = np.linalg.lstsq(Bm * w[:, None], g * w, rcond=1e-13)
        c /= np.max(np.abs(c))
        for q, cq in zip(cols, c):
            mo[first[q] + (axis if l == 1 else 0), j] = cq
    return System(Z=np.array([float(Z)]), R=np.zeros((1, 3)), n_up=n_up, n_dn=n_dn,
                  shell_nuc=nuc_l, shell_l=l_l, shell_alpha=a_l, mo=mo,
                  b_ee=b_ee, b_en=b_en, name=name or f"Z{Z}_screened")


def ar_screened() -> System:
    """Ar (Z=18, 9 up 9 down) in the Ar-like basis (K=64 s/p/d Gaussians
    0.05*2.5^k) with screened hydrogenic orbitals (1s 2s 2p 3s 3p)."""
    return atom_screened(18, basis_alloc(64), 0.05, 2.5, name="ar_screened")

"""CPU oracle for the double-grid LRDMC projection step (arXiv:1909.01589).

TEST INFRASTRUCTURE.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  It shares no
code with the HIP library ``paper_1909_01589_amd``; the two meet only through
the seeded inputs of ``paper_1909_01589_amd.inputs``.

``lrdmc_oracle.c`` (plain C, FP64) holds the projection step; ``spacing.py``
the host-side parameter choice of the paper (r_c and a'/a); ``estimator.py``
the energy estimator and its error bar; ``neural.py`` the learned Jastrow
correction's network and tabulation.

Every function is pinned by the CPU tests (closed forms, brute force, the
paper's printed values, statistical limits).  Parity unpinned: the absolute
energies of the random-MO workloads, which have no reference value and are
checked only through parity with the GPU path.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from typing import Optional, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lrdmc_oracle.c")
_LIB = os.path.join(_HERE, "liblrdmc_oracle.so")

__all__ = ["build", "load", "Oracle"]


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, OpenMP).  Returns the .so path."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-std=gnu11", "-fPIC", "-shared", "-fopenmp",
               "-Wall", "-Wno-unused-function", _SRC, "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


class _Sys(C.Structure):
    _fields_ = [
        ("n_nuc", C.c_int32), ("Z", C.c_void_p), ("R", C.c_void_p),
        ("n_up", C.c_int32), ("n_dn", C.c_int32),
        ("n_shell", C.c_int32), ("shell_nuc", C.c_void_p), ("shell_l", C.c_void_p),
        ("shell_alpha", C.c_void_p),
        ("n_orb", C.c_int32), ("mo", C.c_void_p),
        ("b_ee", C.c_double), ("b_en", C.c_double),
        ("ftab", C.c_void_p), ("ftab_n", C.c_int32), ("ftab_rcut", C.c_double),
    ]


class _Prm(C.Structure):
    _fields_ = [
        ("a", C.c_double), ("a_prime", C.c_double), ("r_c", C.c_double),
        ("z_heavy", C.c_double), ("tau", C.c_double),
        ("seed", C.c_uint64), ("rotate", C.c_int32),
        ("switch_form", C.c_int32), ("grids", C.c_int32), ("pad", C.c_int32),
    ]


_lib = None


def load():
    """Load the oracle library (LRDMC_ORACLE_LIB names another build of the
    same source, e.g. one with sanitizers)."""
    global _lib
    if _lib is None:
        path = os.environ.get("LRDMC_ORACLE_LIB") or _LIB
        if path == _LIB and not os.path.exists(_LIB):
            build()
        lib = C.CDLL(path)
        P = C.c_void_p
        lib.orc_philox4x64_10.argtypes = [P, P, P]
        lib.orc_u01.argtypes = [C.c_uint64]
        lib.orc_u01.restype = C.c_double
        lib.orc_draw.argtypes = [C.c_uint64] * 5 + [P]
        lib.orc_rotation.argtypes = [P, P]
        lib.orc_nbasis.argtypes = [P]
        lib.orc_nbasis.restype = C.c_int
        lib.orc_basis.argtypes = [P, P, P, P, P]
        lib.orc_jastrow.argtypes = [P, P]
        lib.orc_jastrow.restype = C.c_double
        lib.orc_log_psi.argtypes = [P, P, P, P]
        lib.orc_log_psi.restype = C.c_int
        lib.orc_potential.argtypes = [P, P]
        lib.orc_potential.restype = C.c_double
        lib.orc_local_energy.argtypes = [P, P, P, P, P]
        lib.orc_local_energy.restype = C.c_int
        lib.orc_jastrow_param_grad.argtypes = [P, P, P, P]
        lib.orc_corr.argtypes = [P, C.c_int, C.c_double, P]
        lib.orc_corr.restype = None
        lib.orc_jastrow_param_grad.restype = C.c_int
        lib.orc_p_switch.argtypes = [P, P, P]
        lib.orc_p_switch.restype = C.c_double
        lib.orc_move.argtypes = [P, P, P, P, C.c_int, P, P]
        lib.orc_eval_moves.argtypes = [P, P, P, P, P, P, P]
        lib.orc_eval_moves.restype = C.c_int
        lib.orc_select.argtypes = [P, C.c_int, C.c_double]
        lib.orc_select.restype = C.c_int
        lib.orc_select_margin.argtypes = [P, C.c_int, C.c_double, P]
        lib.orc_select_margin.restype = C.c_int
        lib.orc_generation.argtypes = [P, P, C.c_uint64, C.c_uint64, P, P, P, P, P]
        lib.orc_generations.argtypes = [P, P, C.c_int, P, C.c_uint64, P, P, P, P, C.c_int]
        lib.orc_generations.restype = C.c_int
        lib.orc_vmc.argtypes = [P, P, C.c_uint64, C.c_uint64, C.c_int, C.c_double, P, P, P]
        lib.orc_generation.restype = C.c_int
        lib.orc_reconfigure.argtypes = [P, P, C.c_int, C.c_double, P, P, P, P]
        lib.orc_reconfigure.restype = C.c_int
        lib.orc_xi.argtypes = [C.c_uint64, C.c_uint64]
        lib.orc_xi.restype = C.c_double
        lib.orc_run.argtypes = [P, P, C.c_int, P, C.c_uint64, C.c_int, P, P, P, P, P, C.c_int]
        lib.orc_run.restype = C.c_int
        _lib = lib
    return _lib


def _ptr(a: np.ndarray) -> int:
    return a.ctypes.data


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


class OracleError(RuntimeError):
    pass


def _check(rc: int, what: str):
    if rc != 0:
        raise OracleError(f"{what} failed with code {rc}")


class Oracle:
    """One system plus lattice parameters, bound to the C oracle."""

    def __init__(self, system, a: float, a_prime: float, r_c: float,
                 z_heavy: Optional[float] = None, tau: float = 0.01,
                 seed: int = 0, rotate: int = 1, switch_form: int = 0, grids: int = 2,
                 ftab: Optional[np.ndarray] = None, ftab_rcut: float = 0.0):
        """ftab: optional learned Jastrow correction, [2][G][3] = {F, F', F''}
        at G nodes on [0, ftab_rcut] (type 0: electron pairs, 1: electron-
        nucleus pairs, scaled by Z)."""
        self.lib = load()
        self.system = system
        self.ftab = None if ftab is None else np.ascontiguousarray(ftab, dtype=np.float64)
        self.ftab_rcut = float(ftab_rcut)
        if self.ftab is not None and (self.ftab.ndim != 3 or self.ftab.shape[0] != 2 or self.ftab.shape[2] != 3
                                      or self.ftab.shape[1] < 2 or not self.ftab_rcut > 0):
            raise ValueError("ftab must be [2][G>=2][3] with ftab_rcut > 0")
        # keep arrays alive for the lifetime of the struct
        self._keep = [system.Z, system.R, system.shell_nuc, system.shell_l,
                      system.shell_alpha, system.mo, self.ftab]
        self.sys = _Sys(system.n_nuc, _ptr(system.Z), _ptr(system.R), system.n_up,
                        system.n_dn, system.n_shell, _ptr(system.shell_nuc),
                        _ptr(system.shell_l), _ptr(system.shell_alpha), system.n_orb,
                        _ptr(system.mo), system.b_ee, system.b_en,
                        None if self.ftab is None else self.ftab.ctypes.data,
                        0 if self.ftab is None else self.ftab.shape[1], self.ftab_rcut)
        zh = float(np.max(system.Z)) if z_heavy is None else float(z_heavy)
        if switch_form not in (0, 1) or grids not in (1, 2):
            raise ValueError("switch_form must be 0 (Gaussian) or 1 (Pade), grids 1 or 2")
        self.prm = _Prm(a, a_prime, r_c, zh, tau, seed, rotate, switch_form, grids, 0)
        self.N = system.n_elec
        self.M = (12 if grids == 2 else 6) * self.N
        self.K = self.lib.orc_nbasis(C.byref(self.sys))

    # -- parameters -------------------------------------------------------
    def with_params(self, **kw) -> "Oracle":
        d = {f: getattr(self.prm, f) for f, _ in _Prm._fields_ if f != "pad"}
        d.update(kw)
        return Oracle(self.system, d["a"], d["a_prime"], d["r_c"], d["z_heavy"],
                      d["tau"], d["seed"], d["rotate"], d["switch_form"], d["grids"],
                      self.ftab, self.ftab_rcut)

    def corr(self, kind: int, r: float) -> np.ndarray:
        """Learned correction of type kind (0 e-e, 1 e-n) at r: (F, F', F'')."""
        out = np.zeros(3)
        self.lib.orc_corr(C.byref(self.sys), int(kind), C.c_double(r), _ptr(out))
        return out

    # -- random numbers ---------------------------------------------------
    def philox(self, ctr, key) -> np.ndarray:
        c = np.ascontiguousarray(ctr, dtype=np.uint64)
        k = np.ascontiguousarray(key, dtype=np.uint64)
        o = np.zeros(4, dtype=np.uint64)
        self.lib.orc_philox4x64_10(_ptr(c), _ptr(k), _ptr(o))
        return o

    def draw(self, slot, gen, it, purpose) -> np.ndarray:
        u = np.zeros(4)
        self.lib.orc_draw(self.prm.seed, slot, gen, it, purpose, _ptr(u))
        return u

    def rotation(self, u3) -> np.ndarray:
        u = _f64(u3)
        Rm = np.zeros(9)
        self.lib.orc_rotation(_ptr(u), _ptr(Rm))
        return Rm.reshape(3, 3)

    def move_rotation(self, slot, gen, it) -> np.ndarray:
        if not self.prm.rotate:
            return np.eye(3)
        return self.rotation(self.draw(slot, gen, it, 1)[:3])

    def xi(self, gen) -> float:
        return float(self.lib.orc_xi(self.prm.seed, gen))

    # -- wave function ----------------------------------------------------
    def basis(self, r) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
        r = _f64(r)
        v = np.zeros(self.K)
        g = np.zeros((self.K, 3))
        l = np.zeros(self.K)
        self.lib.orc_basis(C.byref(self.sys), _ptr(r), _ptr(v), _ptr(g), _ptr(l))
        return v, g, l

    def log_psi(self, pos) -> Tuple[float, int]:
        pos = _f64(pos)
        la = C.c_double()
        sg = C.c_int()
        self.lib.orc_log_psi(C.byref(self.sys), _ptr(pos), C.byref(la), C.byref(sg))
        return la.value, sg.value

    def jastrow(self, pos) -> float:
        return float(self.lib.orc_jastrow(C.byref(self.sys), _ptr(_f64(pos))))

    def jastrow_param_grad(self, pos) -> Tuple[np.ndarray, np.ndarray]:
        """(dJ/dtheta, dE_L/dtheta) for theta = (b_ee, b_en) at fixed positions."""
        dJ, dE = np.zeros(2), np.zeros(2)
        rc = self.lib.orc_jastrow_param_grad(C.byref(self.sys), _ptr(_f64(pos)), _ptr(dJ), _ptr(dE))
        _check(rc, "jastrow_param_grad")
        return dJ, dE

    def potential(self, pos) -> float:
        return float(self.lib.orc_potential(C.byref(self.sys), _ptr(_f64(pos))))

    def local_energy(self, pos) -> Tuple[float, float, float]:
        pos = _f64(pos)
        e, lap, v = C.c_double(), C.c_double(), C.c_double()
        rc = self.lib.orc_local_energy(C.byref(self.sys), _ptr(pos), C.byref(e), C.byref(lap), C.byref(v))
        _check(rc, "local_energy")
        return e.value, lap.value, v.value

    # -- lattice ------------------------------------------------------------
    def p_switch(self, x) -> float:
        return float(self.lib.orc_p_switch(C.byref(self.sys), C.byref(self.prm), _ptr(_f64(x))))

    def move(self, pos, Rm, m) -> Tuple[np.ndarray, float]:
        rp = np.zeros(3)
        k = C.c_double()
        Rf = _f64(Rm).reshape(9)
        self.lib.orc_move(C.byref(self.sys), C.byref(self.prm), _ptr(_f64(pos)), _ptr(Rf),
                          int(m), _ptr(rp), C.byref(k))
        return rp, k.value

    DIAG = ("e_l", "e_lattice", "lap_lattice", "lap_exact", "v_a", "v_sf", "delta", "v", "sum_k")

    def eval_moves(self, pos, Rm=None):
        """rho[M], k[M] and a dict of diagnostics at frozen positions."""
        pos = _f64(pos)
        Rf = _f64(np.eye(3) if Rm is None else Rm).reshape(9)
        rho = np.zeros(self.M)
        k = np.zeros(self.M)
        diag = np.zeros(10)
        rc = self.lib.orc_eval_moves(C.byref(self.sys), C.byref(self.prm), _ptr(pos), _ptr(Rf),
                                     _ptr(rho), _ptr(k), _ptr(diag))
        _check(rc, "eval_moves")
        return rho, k, dict(zip(self.DIAG, diag[:9]))

    def select(self, T, u2) -> int:
        T = _f64(T)
        return int(self.lib.orc_select(_ptr(T), int(T.shape[0]), float(u2)))

    def select_margin(self, T, u2) -> Tuple[int, float]:
        """Heat-bath choice and its relative margin (distance of u2 * Delta to
        the nearer end of the chosen cumulative interval, over Delta)."""
        T = _f64(T)
        mg = C.c_double()
        m = self.lib.orc_select_margin(_ptr(T), int(T.shape[0]), float(u2), C.byref(mg))
        return int(m), mg.value

    # -- projection -------------------------------------------------------
    def generation(self, pos, slot: int, gen: int, with_margin: bool = False):
        """One walker, one generation.  Returns (pos', log_w, e_L, n_moves),
        plus the smallest relative margin of its integer decisions when
        with_margin."""
        p = _f64(pos).copy()
        lw, el, mg = C.c_double(), C.c_double(), C.c_double()
        nm = C.c_int64()
        rc = self.lib.orc_generation(C.byref(self.sys), C.byref(self.prm), int(slot), int(gen),
                                     _ptr(p), C.byref(lw), C.byref(el), C.byref(nm), C.byref(mg))
        _check(rc, "generation")
        if with_margin:
            return p, lw.value, el.value, nm.value, mg.value
        return p, lw.value, el.value, nm.value

    def generations(self, pos, gen: int, nthreads: int = 0):
        """One generation of every walker slot of pos [W][N][3] (no
        reconfiguration), slots in parallel.  Returns dict(pos, log_w, e_l,
        n_moves, margin) per slot."""
        p = _f64(pos).copy()
        W = p.shape[0]
        lw, el, mg = np.zeros(W), np.zeros(W), np.zeros(W)
        nm = np.zeros(W, dtype=np.int64)
        rc = self.lib.orc_generations(C.byref(self.sys), C.byref(self.prm), W, _ptr(p), int(gen),
                                      _ptr(lw), _ptr(el), _ptr(nm), _ptr(mg), int(nthreads))
        _check(rc, "generations")
        return dict(pos=p, log_w=lw, e_l=el, n_moves=nm, margin=mg)

    def vmc(self, pos, slot: int, gen: int, n_steps: int, step: float):
        """Metropolis chain of n_steps single-electron moves from pos:
        (pos, accepted steps, E_L at the end)."""
        p = np.array(pos, dtype=np.float64, copy=True).reshape(self.N, 3)
        acc, el = C.c_int64(), C.c_double()
        rc = self.lib.orc_vmc(C.byref(self.sys), C.byref(self.prm), int(slot), int(gen),
                              int(n_steps), float(step), _ptr(p), C.byref(acc), C.byref(el))
        _check(rc, "orc_vmc")
        return p, int(acc.value), float(el.value)

    def reconfigure(self, log_w, e_l, xi, with_margin: bool = False):
        """Systematic resampling: (idx, log_wbar, ebar), plus per destination
        slot the relative margin of its choice when with_margin."""
        lw = _f64(log_w)
        el = _f64(e_l)
        W = lw.shape[0]
        idx = np.zeros(W, dtype=np.int32)
        mg = np.zeros(W)
        lwb, eb = C.c_double(), C.c_double()
        rc = self.lib.orc_reconfigure(_ptr(lw), _ptr(el), W, float(xi), _ptr(idx),
                                      C.byref(lwb), C.byref(eb), _ptr(mg))
        _check(rc, "reconfigure")
        if with_margin:
            return idx, lwb.value, eb.value, mg
        return idx, lwb.value, eb.value

    def run(self, pos, n_gen: int, gen0: int = 0, nthreads: int = 0, want_idx: bool = True):
        """Whole projection.  Returns dict(pos, log_wbar, ebar, n_moves, idx,
        margin); margin [n_gen][2][W]: per slot the smallest decision margin of
        its projection, then per destination slot that of its resampling."""
        p = _f64(pos).copy()
        W = p.shape[0]
        lwb = np.zeros(n_gen)
        eb = np.zeros(n_gen)
        nm = np.zeros(n_gen, dtype=np.int64)
        idx = np.zeros((n_gen, W), dtype=np.int32) if want_idx else None
        mg = np.zeros((n_gen, 2, W)) if want_idx else None
        rc = self.lib.orc_run(C.byref(self.sys), C.byref(self.prm), W, _ptr(p), int(gen0), int(n_gen),
                              _ptr(lwb), _ptr(eb), _ptr(nm), _ptr(idx) if want_idx else None,
                              _ptr(mg) if want_idx else None, int(nthreads))
        _check(rc, "run")
        return dict(pos=p, log_wbar=lwb, ebar=eb, n_moves=nm, idx=idx, margin=mg)

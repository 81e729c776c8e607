"""Thin Python binding of liblrdmc.so (include/lrdmc.h) for MI355X.

Argument marshalling only: every step of the projection runs in the HIP
kernels of the library.  torch supplies device memory (cuda tensors on ROCm)
and the stream handle.  There is no CPU fallback: if the library is not built
or no GPU is present, the calls raise.

Module-level functions carry the C names (lrdmc_create, lrdmc_project, ...);
the class ``LRDMC`` bundles a context with the system it was made for.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Tuple

import numpy as np
import torch  # imported before the library so that both share one HIP runtime

_HERE = os.path.dirname(os.path.abspath(__file__))
# LRDMC_LIB names another build of the same sources (e.g. with host sanitizers)
LIB_PATH = os.environ.get("LRDMC_LIB") or os.path.join(_HERE, "liblrdmc.so")

LRDMC_NDIAG = 9
DIAG_NAMES = ("e_l", "e_lattice", "lap_lattice", "lap_exact", "v_a", "v_sf", "delta", "v", "sum_k")

ERRORS = {-1: "EINVAL", -2: "ESINGULAR", -3: "ENONFINITE", -4: "ENOMEM", -5: "EDEVICE", -6: "ECOLLAPSE",
          -7: "EITERCAP"}


class LRDMCError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


class lrdmc_system(C.Structure):
    _fields_ = [
        ("n_nuc", C.c_int32), ("Z", C.c_void_p), ("R", C.c_void_p),
        ("n_up", C.c_int32), ("n_dn", C.c_int32),
        ("n_shell", C.c_int32), ("shell_nuc", C.c_void_p), ("shell_l", C.c_void_p),
        ("shell_alpha", C.c_void_p),
        ("n_orb", C.c_int32), ("mo", C.c_void_p),
        ("b_ee", C.c_double), ("b_en", C.c_double),
    ]


class lrdmc_params(C.Structure):
    _fields_ = [
        ("a", C.c_double), ("a_prime", C.c_double), ("r_c", C.c_double),
        ("z_heavy", C.c_double), ("tau", C.c_double),
        ("seed", C.c_uint64), ("rotate", C.c_int32), ("refresh", C.c_int32),
        ("switch_form", C.c_int32), ("grids", C.c_int32),
    ]


_lib = None
EXPORTS = ("lrdmc_spacing", "lrdmc_spacing_pade", "lrdmc_create", "lrdmc_set_walkers", "lrdmc_project", "lrdmc_branch",
           "lrdmc_run", "lrdmc_get_walkers", "lrdmc_eval_moves", "lrdmc_reconfigure",
           "lrdmc_reconfigure_noalloc", "lrdmc_inverse_residual", "lrdmc_jastrow_grad", "lrdmc_set_jastrow", "lrdmc_set_jastrow_table", "lrdmc_jastrow_table_grad",
           "lrdmc_vmc", "lrdmc_net_param_count", "lrdmc_net_workspace_size", "lrdmc_net_tabulate", "lrdmc_net_tabulate_backward",
           "lrdmc_use_generic", "lrdmc_is_specialized", "lrdmc_set_precision", "lrdmc_set_timing", "lrdmc_timing",
           "lrdmc_set_collapse_threshold", "lrdmc_set_move_cap", "lrdmc_generation",
           "lrdmc_last_error", "lrdmc_destroy")


def load():
    """Load liblrdmc.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
    lib = C.CDLL(LIB_PATH)
    P, I32, I64, U64, D = C.c_void_p, C.c_int32, C.c_int64, C.c_uint64, C.c_double
    lib.lrdmc_spacing.argtypes = [D, D, D, D, P, P, P]
    lib.lrdmc_spacing_pade.argtypes = [D, D, P, P]
    lib.lrdmc_create.argtypes = [P, P, I32, P]
    lib.lrdmc_set_walkers.argtypes = [P, P, U64, P]
    lib.lrdmc_project.argtypes = [P, P]
    lib.lrdmc_branch.argtypes = [P, P, P, P, P, P, P]
    lib.lrdmc_run.argtypes = [P, I32, P, P, P, P, P, P]
    lib.lrdmc_get_walkers.argtypes = [P, P, P, P, P, P]
    lib.lrdmc_eval_moves.argtypes = [P, P, P, P, P, P]
    lib.lrdmc_reconfigure.argtypes = [P, P, I32, D, P, P, P]
    lib.lrdmc_reconfigure_noalloc.argtypes = [P, P, I32, D, P, P, P]
    lib.lrdmc_inverse_residual.argtypes = [P, P, P]
    lib.lrdmc_jastrow_grad.argtypes = [P, P, P, P]
    lib.lrdmc_set_jastrow.argtypes = [P, D, D]
    lib.lrdmc_set_jastrow_table.argtypes = [P, P, I32, D, I32, P]
    lib.lrdmc_jastrow_table_grad.argtypes = [P, P, P, P, P, P]
    lib.lrdmc_vmc.argtypes = [P, I32, D, P]
    lib.lrdmc_net_param_count.argtypes = [I32]
    lib.lrdmc_net_param_count.restype = I32
    lib.lrdmc_net_workspace_size.argtypes = [I32, I32]
    lib.lrdmc_net_workspace_size.restype = C.c_int64
    lib.lrdmc_net_tabulate.argtypes = [P, I32, I32, D, P, P]
    lib.lrdmc_net_tabulate_backward.argtypes = [P, I32, I32, D, P, P, P, P]
    lib.lrdmc_use_generic.argtypes = [P, I32]
    lib.lrdmc_set_precision.argtypes = [P, I32]
    lib.lrdmc_set_collapse_threshold.argtypes = [P, D]
    lib.lrdmc_set_move_cap.argtypes = [P, I32]
    lib.lrdmc_is_specialized.argtypes = [P]
    lib.lrdmc_is_specialized.restype = I32
    lib.lrdmc_set_timing.argtypes = [P, I32]
    lib.lrdmc_timing.argtypes = [P, P]
    lib.lrdmc_generation.argtypes = [P]
    lib.lrdmc_generation.restype = U64
    lib.lrdmc_last_error.argtypes = [P]
    lib.lrdmc_last_error.restype = C.c_char_p
    lib.lrdmc_destroy.argtypes = [P]
    lib.lrdmc_destroy.restype = None
    for name in ("lrdmc_spacing", "lrdmc_spacing_pade", "lrdmc_create", "lrdmc_set_walkers", "lrdmc_project", "lrdmc_branch",
                 "lrdmc_run", "lrdmc_get_walkers", "lrdmc_eval_moves", "lrdmc_reconfigure",
                 "lrdmc_reconfigure_noalloc", "lrdmc_inverse_residual", "lrdmc_jastrow_grad", "lrdmc_set_jastrow", "lrdmc_set_jastrow_table",
                 "lrdmc_jastrow_table_grad", "lrdmc_vmc", "lrdmc_net_tabulate", "lrdmc_net_tabulate_backward",
                 "lrdmc_use_generic", "lrdmc_set_precision", "lrdmc_set_collapse_threshold", "lrdmc_set_move_cap",
                 "lrdmc_set_timing",
                 "lrdmc_timing"):
        getattr(lib, name).restype = C.c_int
    _lib = lib
    return lib


def _check(rc: int, ctx=None):
    if rc != 0:
        msg = load().lrdmc_last_error(ctx).decode()
        raise LRDMCError(rc, msg)


def _dptr(t: Optional[torch.Tensor], dtype=None) -> Optional[int]:
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("device tensor expected")
    if not t.is_contiguous():
        raise ValueError("contiguous tensor expected")
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"{dtype} tensor expected, got {t.dtype}")
    return t.data_ptr()


def _stream(stream=None) -> int:
    s = torch.cuda.current_stream() if stream is None else stream
    return s.cuda_stream


# -- the C entry points -------------------------------------------------------

def lrdmc_spacing(Z: float, a: float, beta: float = 0.75, kappa: float = 2.5) -> Tuple[float, float, float]:
    rc, ap, nc = C.c_double(), C.c_double(), C.c_double()
    _check(load().lrdmc_spacing(float(Z), float(a), float(beta), float(kappa),
                                C.byref(rc), C.byref(ap), C.byref(nc)))
    return rc.value, ap.value, nc.value


def lrdmc_spacing_pade(Z: float, a: float) -> Tuple[float, float]:
    """Earlier parametrization (Eq. (2) switch with r_c = Z/2, Eq. (4) a'/a)."""
    rc, ap = C.c_double(), C.c_double()
    _check(load().lrdmc_spacing_pade(float(Z), float(a), C.byref(rc), C.byref(ap)))
    return rc.value, ap.value


def _pack_system(system):
    keep = [np.ascontiguousarray(system.Z, dtype=np.float64),
            np.ascontiguousarray(system.R, dtype=np.float64).reshape(-1),
            np.ascontiguousarray(system.shell_nuc, dtype=np.int32),
            np.ascontiguousarray(system.shell_l, dtype=np.int32),
            np.ascontiguousarray(system.shell_alpha, dtype=np.float64),
            np.ascontiguousarray(system.mo, dtype=np.float64)]
    s = lrdmc_system(len(keep[0]), keep[0].ctypes.data, keep[1].ctypes.data, int(system.n_up),
                     int(system.n_dn), len(keep[2]), keep[2].ctypes.data, keep[3].ctypes.data,
                     keep[4].ctypes.data, int(keep[5].shape[1]), keep[5].ctypes.data,
                     float(system.b_ee), float(system.b_en))
    return s, keep


def lrdmc_create(system, a: float, a_prime: float, r_c: float, tau: float, n_walkers: int,
                 z_heavy: Optional[float] = None, seed: int = 0, rotate: int = 1, refresh: int = 1,
                 switch_form: int = 0, grids: int = 2) -> int:
    s, keep = _pack_system(system)
    zh = float(np.max(system.Z)) if z_heavy is None else float(z_heavy)
    p = lrdmc_params(a, a_prime, r_c, zh, tau, seed, rotate, refresh, switch_form, grids)
    ctx = C.c_void_p()
    _check(load().lrdmc_create(C.byref(s), C.byref(p), int(n_walkers), C.byref(ctx)))
    del keep
    return ctx.value


def lrdmc_set_walkers(ctx, pos: torch.Tensor, generation: int = 0, stream=None):
    _check(load().lrdmc_set_walkers(ctx, _dptr(pos, torch.float64), int(generation), _stream(stream)), ctx)


def lrdmc_project(ctx, stream=None):
    _check(load().lrdmc_project(ctx, _stream(stream)), ctx)


def lrdmc_branch(ctx, log_wbar=None, ebar=None, n_moves=None, idx=None, ess=None, stream=None):
    _check(load().lrdmc_branch(ctx, _stream(stream), _dptr(log_wbar, torch.float64),
                               _dptr(ebar, torch.float64), _dptr(n_moves, torch.int64),
                               _dptr(idx, torch.int32), _dptr(ess, torch.float64)), ctx)


def lrdmc_run(ctx, n_gen: int, log_wbar=None, ebar=None, n_moves=None, idx=None, ess=None, stream=None):
    _check(load().lrdmc_run(ctx, int(n_gen), _stream(stream), _dptr(log_wbar, torch.float64),
                            _dptr(ebar, torch.float64), _dptr(n_moves, torch.int64),
                            _dptr(idx, torch.int32), _dptr(ess, torch.float64)), ctx)


def lrdmc_get_walkers(ctx, pos=None, log_w=None, e_loc=None, n_moves=None, stream=None):
    _check(load().lrdmc_get_walkers(ctx, _dptr(pos, torch.float64), _dptr(log_w, torch.float64),
                                    _dptr(e_loc, torch.float64), _dptr(n_moves, torch.int32),
                                    _stream(stream)), ctx)


def lrdmc_eval_moves(ctx, pos, rho=None, k=None, diag=None, stream=None):
    _check(load().lrdmc_eval_moves(ctx, _dptr(pos, torch.float64), _dptr(rho, torch.float64),
                                   _dptr(k, torch.float64), _dptr(diag, torch.float64),
                                   _stream(stream)), ctx)


def lrdmc_reconfigure(log_w, e_loc, xi: float, idx, stats=None, stream=None):
    """idx[W] (int32) and stats[2] = (log w_bar, e_bar) from log_w[W], e_loc[W]."""
    W = int(log_w.numel())
    if e_loc.numel() != W or idx.numel() != W or (stats is not None and stats.numel() < 2):
        raise ValueError("log_w, e_loc and idx must hold W elements each, stats at least 2")
    _check(load().lrdmc_reconfigure(_dptr(log_w, torch.float64), _dptr(e_loc, torch.float64),
                                    W, float(xi), _dptr(idx, torch.int32),
                                    _dptr(stats, torch.float64), _stream(stream)))


NOALLOC_MAX_WALKERS = 1 << 20


def lrdmc_reconfigure_noalloc(log_w, e_loc, xi: float, idx, stats=None, stream=None):
    """lrdmc_reconfigure with its scratch in the library's fixed device array
    (no allocation; calls that overlap on one GPU race)."""
    W = int(log_w.numel())
    if e_loc.numel() != W or idx.numel() != W or (stats is not None and stats.numel() < 2):
        raise ValueError("log_w, e_loc and idx must hold W elements each, stats at least 2")
    _check(load().lrdmc_reconfigure_noalloc(_dptr(log_w, torch.float64), _dptr(e_loc, torch.float64),
                                            W, float(xi), _dptr(idx, torch.int32),
                                            _dptr(stats, torch.float64), _stream(stream)))


def lrdmc_inverse_residual(ctx, res, stream=None):
    """res[W] (device float64) = max |A Ainv - I| of each walker's carried inverse."""
    _check(load().lrdmc_inverse_residual(ctx, _dptr(res, torch.float64), _stream(stream)), ctx)


def lrdmc_jastrow_grad(ctx, pos, out, stream=None):
    _check(load().lrdmc_jastrow_grad(ctx, _dptr(pos, torch.float64), _dptr(out, torch.float64),
                                     _stream(stream)), ctx)


def lrdmc_set_jastrow(ctx, b_ee: float, b_en: float):
    _check(load().lrdmc_set_jastrow(ctx, float(b_ee), float(b_en)), ctx)


MAX_TABLE_NODES = 4096


def lrdmc_set_jastrow_table(ctx, tab, r_cut: float = 0.0, stream=None):
    """tab: [2][G][3] float64 (host array or device tensor), or None to remove."""
    if tab is None:
        _check(load().lrdmc_set_jastrow_table(ctx, None, 0, 0.0, 0, _stream(stream)), ctx)
        return
    if isinstance(tab, torch.Tensor) and tab.is_cuda:
        if tab.dim() != 3 or tab.shape[0] != 2 or tab.shape[2] != 3:
            raise ValueError("table must be [2][n_nodes][3]")
        _check(load().lrdmc_set_jastrow_table(ctx, _dptr(tab, torch.float64), int(tab.shape[1]), float(r_cut), 1,
                                              _stream(stream)), ctx)
        return
    a = np.ascontiguousarray(np.asarray(tab, dtype=np.float64))
    if a.ndim != 3 or a.shape[0] != 2 or a.shape[2] != 3:
        raise ValueError("table must be [2][n_nodes][3]")
    _check(load().lrdmc_set_jastrow_table(ctx, a.ctypes.data, int(a.shape[1]), float(r_cut), 0, _stream(stream)), ctx)


def lrdmc_jastrow_table_grad(ctx, pos, c_j, c_e, gtab, stream=None):
    _check(load().lrdmc_jastrow_table_grad(ctx, _dptr(pos, torch.float64), _dptr(c_j, torch.float64),
                                           _dptr(c_e, torch.float64), _dptr(gtab, torch.float64),
                                           _stream(stream)), ctx)


def lrdmc_vmc(ctx, n_steps: int, step: float, stream=None):
    _check(load().lrdmc_vmc(ctx, int(n_steps), float(step), _stream(stream)), ctx)


def lrdmc_net_param_count(hidden: int) -> int:
    return int(load().lrdmc_net_param_count(int(hidden)))


def lrdmc_net_workspace_size(hidden: int, n_nodes: int) -> int:
    return int(load().lrdmc_net_workspace_size(int(hidden), int(n_nodes)))


def lrdmc_net_tabulate(params, hidden: int, n_nodes: int, r_cut: float, tab, stream=None):
    _check(load().lrdmc_net_tabulate(_dptr(params, torch.float64), int(hidden), int(n_nodes), float(r_cut),
                                     _dptr(tab, torch.float64), _stream(stream)))


def lrdmc_net_tabulate_backward(params, hidden: int, n_nodes: int, r_cut: float, gtab, gparams, work,
                                stream=None):
    _check(load().lrdmc_net_tabulate_backward(_dptr(params, torch.float64), int(hidden), int(n_nodes), float(r_cut),
                                              _dptr(gtab, torch.float64), _dptr(gparams, torch.float64),
                                              _dptr(work, torch.float64), _stream(stream)))


def lrdmc_use_generic(ctx, enable=True):
    """0/False automatic, 1/True the general kernel, 2 the general kernel with
    the orbital-projected inverse in device memory."""
    _check(load().lrdmc_use_generic(ctx, int(enable)), ctx)


def lrdmc_set_precision(ctx, mode: int):
    """0 FP64 move table; 1 mixed precision (FP32 estimates of 1/r and of the
    Pade denominators' reciprocal in the table's Jastrow pair terms)."""
    _check(load().lrdmc_set_precision(ctx, int(mode)), ctx)


def lrdmc_set_collapse_threshold(ctx, min_fraction: float):
    """Population-collapse check: LRDMC_ECOLLAPSE when a generation's
    effective sample size falls below min_fraction * W (0 turns it off)."""
    _check(load().lrdmc_set_collapse_threshold(ctx, float(min_fraction)), ctx)


def lrdmc_set_move_cap(ctx, max_moves: int):
    """Moves per walker and generation before LRDMC_EITERCAP (1..2^22)."""
    _check(load().lrdmc_set_move_cap(ctx, int(max_moves)), ctx)


def lrdmc_is_specialized(ctx) -> bool:
    return bool(load().lrdmc_is_specialized(ctx))


def lrdmc_set_timing(ctx, enable: bool = True):
    _check(load().lrdmc_set_timing(ctx, 1 if enable else 0), ctx)


def lrdmc_timing(ctx):
    """(projection ms, projection launches, reconfiguration ms, launches)."""
    out = (C.c_double * 4)()
    _check(load().lrdmc_timing(ctx, out), ctx)
    return tuple(out)


def lrdmc_generation(ctx) -> int:
    return int(load().lrdmc_generation(ctx))


def lrdmc_last_error(ctx=None) -> str:
    return load().lrdmc_last_error(ctx).decode()


def lrdmc_destroy(ctx):
    if ctx:
        load().lrdmc_destroy(ctx)


# -- convenience object -----------------------------------------------------

class LRDMC:
    """A context bound to one system and walker count, with torch buffers."""

    def __init__(self, system, a: float, a_prime: float, r_c: float, tau: float, n_walkers: int,
                 z_heavy: Optional[float] = None, seed: int = 0, rotate: int = 1, refresh: int = 1,
                 device: str = "cuda:0", switch_form: int = 0, grids: int = 2):
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU: the LRDMC projection runs only on the HIP device")
        self.device = torch.device(device)
        if self.device.index is None:
            self.device = torch.device("cuda", torch.cuda.current_device())
        torch.cuda.set_device(self.device)
        self.system = system
        self.W = int(n_walkers)
        self.N = system.n_elec
        self.M = (6 if grids == 1 else 12) * self.N
        self.table_nodes = 0
        self.ctx = lrdmc_create(system, a, a_prime, r_c, tau, n_walkers, z_heavy, seed, rotate, refresh,
                                switch_form, grids)

    def close(self):
        if self.ctx:
            lrdmc_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _f64(self, *shape):
        return torch.empty(*shape, dtype=torch.float64, device=self.device)

    def positions(self, pos) -> torch.Tensor:
        """pos as the contiguous float64 device tensor [W][N][3] the kernels
        read for this context (the C entry points take bare pointers)."""
        t = torch.as_tensor(pos, dtype=torch.float64).to(self.device).contiguous()
        if tuple(t.shape) != (self.W, self.N, 3):
            raise ValueError(f"positions must be [{self.W}, {self.N}, 3]")
        return t

    def set_walkers(self, pos, generation: int = 0):
        lrdmc_set_walkers(self.ctx, self.positions(pos), generation)

    @property
    def generation(self) -> int:
        return lrdmc_generation(self.ctx)

    def project(self):
        lrdmc_project(self.ctx)

    def branch(self):
        lwb, eb = self._f64(1), self._f64(1)
        nm = torch.empty(1, dtype=torch.int64, device=self.device)
        idx = torch.empty(self.W, dtype=torch.int32, device=self.device)
        ess = self._f64(1)
        lrdmc_branch(self.ctx, lwb, eb, nm, idx, ess)
        return dict(log_wbar=float(lwb.item()), ebar=float(eb.item()), n_moves=int(nm.item()), idx=idx,
                    ess=float(ess.item()))

    def run(self, n_gen: int, want_idx: bool = False, out=None):
        if out is None:
            out = dict(log_wbar=self._f64(n_gen), ebar=self._f64(n_gen),
                       n_moves=torch.empty(n_gen, dtype=torch.int64, device=self.device),
                       idx=(torch.empty(n_gen, self.W, dtype=torch.int32, device=self.device)
                            if want_idx else None),
                       ess=self._f64(n_gen))
        lrdmc_run(self.ctx, n_gen, out["log_wbar"], out["ebar"], out["n_moves"], out["idx"], out.get("ess"))
        return out

    def get_walkers(self):
        pos = self._f64(self.W, self.N, 3)
        lw, el = self._f64(self.W), self._f64(self.W)
        nm = torch.empty(self.W, dtype=torch.int32, device=self.device)
        lrdmc_get_walkers(self.ctx, pos, lw, el, nm)
        return dict(pos=pos, log_w=lw, e_l=el, n_moves=nm)

    def set_jastrow(self, b_ee: float, b_en: float):
        lrdmc_set_jastrow(self.ctx, b_ee, b_en)

    def vmc(self, n_steps: int, step: float):
        """Metropolis sampling of |Psi|^2: n_steps single-electron moves per
        walker (one generation index); get_walkers() then has the samples."""
        lrdmc_vmc(self.ctx, n_steps, step)

    def set_jastrow_table(self, tab, r_cut: float = 0.0):
        """Learned correction from its node table [2][G][3] (None removes it)."""
        lrdmc_set_jastrow_table(self.ctx, tab, r_cut)
        self.table_nodes = 0 if tab is None else int(tab.shape[1])

    def jastrow_table_grad(self, pos, c_j=None, c_e=None):
        """[2][G][3]: d/dtab sum_w (c_j[w] J_w + c_e[w] E_L,w)."""
        t = self.positions(pos)
        cj = None if c_j is None else torch.as_tensor(c_j, dtype=torch.float64).to(self.device).contiguous()
        ce = None if c_e is None else torch.as_tensor(c_e, dtype=torch.float64).to(self.device).contiguous()
        for c in (cj, ce):
            if c is not None and tuple(c.shape) != (self.W,):
                raise ValueError(f"coefficients must be [{self.W}]")
        if not getattr(self, "table_nodes", 0):
            raise ValueError("no correction table is set")
        g = self._f64(2, self.table_nodes, 3)
        lrdmc_jastrow_table_grad(self.ctx, t, cj, ce, g)
        return g

    def jastrow_grad(self, pos):
        """[W][6]: E_L, J, dJ/db_ee, dJ/db_en, dE_L/db_ee, dE_L/db_en."""
        t = self.positions(pos)
        out = self._f64(self.W, 6)
        lrdmc_jastrow_grad(self.ctx, t, out)
        return out

    def eval_moves(self, pos):
        t = self.positions(pos)
        rho, k = self._f64(self.W, self.M), self._f64(self.W, self.M)
        diag = self._f64(self.W, LRDMC_NDIAG)
        lrdmc_eval_moves(self.ctx, t, rho, k, diag)
        return rho, k, diag

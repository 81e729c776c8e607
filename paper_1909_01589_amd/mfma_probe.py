"""Measurement prototype behind the choice of the table's contraction.

Binding of libmfma_probe.so (csrc/mfma_probe.hip): the determinant ratios of
the fixed-axis move table of every walker, computed either as the FP64 dot
of each move point's basis values with the moved electron's row of
Y = C Ainv (the formulation of the projection kernels), or as the BF16x3
matrix-core product Phi' = B' C (C shared by every walker, FP32
accumulation) followed by the FP64 dot with the inverse Slater matrix.  Not
part of the projection path: it times the two contractions on the same
inputs so that the choice rests on a measurement.

The host side prepares the inputs of a walker population: the basis
function table, the two-term BF16 split of C in the matrix-core operand
layout, and (in numpy, FP64) the inverse Slater matrices and Y.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmfma_probe.so")

FN_DTYPE = np.dtype([("R", np.float64, 3), ("alpha", np.float64), ("l", np.int32), ("comp", np.int32),
                     ("pad", np.int32, 2)])

_lib = None


def load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        lib = C.CDLL(LIB_PATH)
        P, I, D = C.c_void_p, C.c_int, C.c_double
        lib.mfma_probe_ratios.argtypes = [I, I, I, I, I, D, D, P, P, P, P, P, P, P]
        lib.mfma_probe_ratios.restype = I
        lib.mfma_probe_fn_bytes.restype = I
        assert lib.mfma_probe_fn_bytes() == FN_DTYPE.itemsize
        _lib = lib
    return _lib


def basis_table(system) -> np.ndarray:
    """One record per basis function in the system's order (shells, then
    components p: x, y, z; d: xy, yz, zx, x^2 - y^2, 2 z^2 - x^2 - y^2)."""
    rows = []
    for q in range(system.n_shell):
        l = int(system.shell_l[q])
        for c in range(2 * l + 1):
            rows.append((system.R[int(system.shell_nuc[q])], float(system.shell_alpha[q]), l, c, (0, 0)))
    return np.array(rows, dtype=FN_DTYPE)


def basis_values(fns: np.ndarray, pts: np.ndarray) -> np.ndarray:
    """g_mu at the points pts [..., 3] -> [..., K] (FP64)."""
    d = pts[..., None, :] - fns["R"]                      # [..., K, 3]
    x, y, z = d[..., 0], d[..., 1], d[..., 2]
    e = np.exp(-fns["alpha"] * (x * x + y * y + z * z))
    l, c = fns["l"], fns["comp"]
    P = np.ones_like(e)
    p1 = np.choose(np.where(l == 1, c, 0), [x, y, z])
    p2 = np.choose(np.where(l == 2, c, 0), [x * y, y * z, z * x, x * x - y * y, 2 * z * z - x * x - y * y])
    P = np.where(l == 1, p1, np.where(l == 2, p2, P))
    return P * e


def split_c(mo: np.ndarray, Kpad: int) -> np.ndarray:
    """C = hi + lo + rest with hi, lo BF16 by truncation of the FP32 value,
    laid out as the B operand of v_mfma_f32_16x16x32_bf16: for chunk kc,
    tile t (orbitals 16 t .. 16 t + 15), term h (hi, lo) and lane l, the 8
    values C[32 kc + 8 (l / 16) + j][16 t + l % 16], j = 0..7.  Orbitals
    beyond 32 are not supported."""
    K, n_orb = mo.shape
    if n_orb > 32:
        raise ValueError("at most 32 orbitals")
    Cp = np.zeros((Kpad, 32), dtype=np.float32)
    Cp[:K, :n_orb] = mo
    bits = Cp.view(np.uint32)
    hi_f = (bits & np.uint32(0xFFFF0000)).view(np.float32)
    lo_f = Cp - hi_f
    terms = [(hi_f.view(np.uint32) >> 16).astype(np.uint16), (lo_f.view(np.uint32) >> 16).astype(np.uint16)]
    n_kc = Kpad // 32
    out = np.zeros((n_kc, 2, 2, 64, 8), dtype=np.uint16)
    lane = np.arange(64)
    for kc in range(n_kc):
        for t in range(2):
            for h in range(2):
                for j in range(8):
                    out[kc, t, h, :, j] = terms[h][32 * kc + 8 * (lane // 16) + j, 16 * t + lane % 16]
    return out


def prepare(system, pos: np.ndarray):
    """Host inputs for W walkers at pos [W][N][3]: basis table, C split,
    inverse Slater matrices Ainv [W][2][32][32] (orbital row, electron
    column, zero padded) and Y [W][N][Kpad], all FP64 from numpy."""
    fns = basis_table(system)
    K = len(fns)
    Kpad = (K + 31) // 32 * 32
    W, N, _ = pos.shape
    nu, nd = system.n_up, system.n_dn
    Ainv = np.zeros((W, 2, 32, 32))
    Y = np.zeros((W, N, Kpad))
    for w0 in range(0, W, 512):
        sl = slice(w0, min(W, w0 + 512))
        phi = basis_values(fns, pos[sl]) @ system.mo       # [w][N][n_orb]
        for s, (i0, n) in enumerate(((0, nu), (nu, nd))):
            if n == 0:
                continue
            inv = np.linalg.inv(phi[:, i0:i0 + n, :n])     # A[electron][orbital] -> [orbital][electron]
            Ainv[sl, s, :n, :n] = inv
            Y[sl, i0:i0 + n, :K] = np.einsum("mj,wji->wim", system.mo[:, :n], inv)
    return dict(fns=fns, K=K, Kpad=Kpad, Cb=split_c(system.mo, Kpad), Ainv=Ainv, Y=Y)


def move_points(pos: np.ndarray, a: float, ap: float) -> np.ndarray:
    """Displaced points of the fixed-axis table, m = 12 i + 6 g + d -> [W][12 N][3]."""
    W, N, _ = pos.shape
    pts = np.repeat(pos, 12, axis=1).reshape(W, N, 12, 3).copy()
    for g, h in ((0, a), (1, ap)):
        for d in range(6):
            pts[:, :, 6 * g + d, d // 2] += h if d % 2 == 0 else -h
    return pts.reshape(W, 12 * N, 3)


def bf16x3_bound(prep, system, pos, a, ap) -> np.ndarray:
    """Bound on |rho_D(BF16x3) - rho_D| per move [W][12 N]: each operand's
    two-term split leaves at most 2^-16 of it, the neglected lo.lo term
    2^-16 more, FP32 products and the accumulation over K terms K 2^-24, so
    |dPhi'_mj| <= (3 2^-16 + K 2^-24) sum_mu |g_mu C_mj| (plus the rounding
    of g to FP32); rho_D adds sum_j |dPhi'_mj| |Ainv_ji|."""
    g = basis_values(prep["fns"], move_points(pos, a, ap))            # [W][M][K]
    S = np.abs(g) @ np.abs(system.mo)                                 # [W][M][n_orb]
    eps = 4 * 2.0 ** -16 + prep["K"] * 2.0 ** -24
    W, M = S.shape[:2]
    N = system.n_elec
    out = np.zeros((W, M))
    for m in range(M):
        i = m // 12
        s, col = (0, i) if i < system.n_up else (1, i - system.n_up)
        n = system.n_up if s == 0 else system.n_dn
        out[:, m] = eps * np.sum(S[:, m, :n] * np.abs(prep["Ainv"][:, s, :n, col]), axis=1)
    return out


class Probe:
    """Device copies of a prepared population; ratios(variant) -> [W][12 N]."""

    def __init__(self, system, pos: np.ndarray, a: float, ap: float, device="cuda"):
        self.lib = load()
        prep = prepare(system, pos)
        self.prep = prep
        self.W, self.N = pos.shape[:2]
        self.n_up, self.K = system.n_up, prep["K"]
        self.a, self.ap = float(a), float(ap)
        t = lambda x, dt=torch.float64: torch.tensor(np.ascontiguousarray(x), dtype=dt, device=device)
        self.pos = t(pos)
        self.fns = torch.tensor(np.frombuffer(prep["fns"].tobytes(), dtype=np.uint8), device=device)
        self.Y = t(prep["Y"])
        self.Cb = torch.tensor(prep["Cb"].view(np.int16), dtype=torch.int16, device=device)
        self.Ainv = t(prep["Ainv"])
        self.rho = torch.empty(self.W, 12 * self.N, dtype=torch.float64, device=device)

    def ratios(self, variant: int, stream=None) -> torch.Tensor:
        st = (torch.cuda.current_stream() if stream is None else stream).cuda_stream
        rc = self.lib.mfma_probe_ratios(int(variant), self.W, self.N, self.n_up, self.K, self.a, self.ap,
                                        self.pos.data_ptr(), self.fns.data_ptr(), self.Y.data_ptr(),
                                        self.Cb.data_ptr(), self.Ainv.data_ptr(), self.rho.data_ptr(), st)
        if rc != 0:
            raise RuntimeError(f"mfma_probe_ratios failed with code {rc}")
        return self.rho

"""Learned Jastrow correction behind torch.autograd.

The trial function's Jastrow exponent gets, on top of the Pade terms, a
radial function per pair type, f(r) = r^2 (1 - r/r_cut)^3 g(r/r_cut) with g
a network 1 -> H -> H -> 1 (SiLU), F_ee for electron pairs and Z_I F_en for
electron-nucleus pairs.  The projection kernels read f from a node table
{f, f', f''} (C^2 quintic interpolation between nodes), so one training step
is, all in the library's kernels:

  params --lrdmc_net_tabulate--> table --lrdmc_set_jastrow_table-->
  lrdmc_jastrow_grad --> (J_w, E_L,w)                        (forward)
  lrdmc_jastrow_table_grad --> d/dtable --lrdmc_net_tabulate_backward-->
  d/dparams                                                  (backward)

torch holds the parameters, the scalar objective over the walkers and the
optimizer state; the per-walker physics and the network run in HIP.

Variance minimisation over fixed configurations x_w sampled from a density
proportional to |Psi_0|^p (p = 2: |Psi_0|^2; p = 1: the mixed density Psi_0
Phi_0 of the projection's walkers, whose E_L variance sets the projection's
statistical error): weights exp(p (J - J_0)) correct for the change of the
trial function (the determinant is fixed, so Psi / Psi_0 = exp(J - J_0)).
"""
from __future__ import annotations

from typing import Dict, Optional

import numpy as np
import torch

from .lrdmc import (LRDMC, lrdmc_jastrow_grad, lrdmc_jastrow_table_grad, lrdmc_net_param_count,
                    lrdmc_net_tabulate, lrdmc_net_tabulate_backward, lrdmc_net_workspace_size,
                    lrdmc_set_jastrow_table)

_ORDER = ("W1", "b1", "W2", "b2", "w3", "b3")


def pack(weights: Dict[str, Dict[str, np.ndarray]]) -> np.ndarray:
    """[2][P] parameter vector from {"ee": {...}, "en": {...}} with arrays
    W1[H], b1[H], W2[H][H] (row = output unit), b2[H], w3[H], b3."""
    rows = []
    for kind in ("ee", "en"):
        p = weights[kind]
        rows.append(np.concatenate([np.asarray(p[k], dtype=np.float64).ravel() for k in _ORDER]))
    out = np.stack(rows)
    H = np.asarray(weights["ee"]["W1"]).size
    if out.shape[1] != H * H + 4 * H + 1:
        raise ValueError("inconsistent network shapes")
    return out


def unpack(params: np.ndarray, hidden: int) -> Dict[str, Dict[str, np.ndarray]]:
    H = hidden
    sizes = (H, H, H * H, H, H, 1)
    out = {}
    for t, kind in enumerate(("ee", "en")):
        row, d, o = np.asarray(params[t], dtype=np.float64), {}, 0
        for k, n in zip(_ORDER, sizes):
            d[k] = row[o:o + n].copy()
            o += n
        d["W2"] = d["W2"].reshape(H, H)
        d["b3"] = d["b3"].reshape(())
        out[kind] = d
    return out


def init_params(hidden: int = 64, seed: int = 0, device="cuda") -> torch.Tensor:
    """Random hidden layers and a zero output layer: the correction starts at
    zero (the trial function is the Pade one)."""
    rng = np.random.default_rng(seed)
    H = hidden
    w = {}
    for kind in ("ee", "en"):
        w[kind] = dict(W1=rng.normal(size=H) * 2.0, b1=rng.normal(size=H) * 0.5,
                       W2=rng.normal(size=(H, H)) / np.sqrt(H), b2=rng.normal(size=H) * 0.1,
                       w3=np.zeros(H), b3=np.zeros(()))
    return torch.tensor(pack(w), dtype=torch.float64, device=device)


class NetTable(torch.autograd.Function):
    """params [2][P] -> node table [2][n_nodes][3]."""

    @staticmethod
    def forward(ctx, params: torch.Tensor, hidden: int, n_nodes: int, r_cut: float):
        p = params.detach().contiguous()
        if tuple(p.shape) != (2, lrdmc_net_param_count(hidden)):
            raise ValueError(f"params must be [2, {lrdmc_net_param_count(hidden)}]")
        tab = torch.empty(2, n_nodes, 3, dtype=torch.float64, device=p.device)
        lrdmc_net_tabulate(p, hidden, n_nodes, r_cut, tab)
        ctx.save_for_backward(p)
        ctx.cfg = (hidden, n_nodes, r_cut)
        return tab

    @staticmethod
    def backward(ctx, gtab):
        (p,) = ctx.saved_tensors
        hidden, n_nodes, r_cut = ctx.cfg
        g = torch.empty_like(p)
        work = torch.empty(lrdmc_net_workspace_size(hidden, n_nodes), dtype=torch.float64, device=p.device)
        lrdmc_net_tabulate_backward(p, hidden, n_nodes, r_cut, gtab.contiguous(), g, work)
        return g, None, None, None


class TableJastrow(torch.autograd.Function):
    """node table -> (J[W], E_L[W]) at the configurations pos of an LRDMC
    context (the forward pass sets the context's table)."""

    @staticmethod
    def forward(ctx, tab: torch.Tensor, engine: LRDMC, pos: torch.Tensor, r_cut: float):
        t = tab.detach().contiguous()
        pos = engine.positions(pos)
        lrdmc_set_jastrow_table(engine.ctx, t, r_cut)
        engine.table_nodes = int(t.shape[1])
        out = torch.empty(engine.W, 6, dtype=torch.float64, device=engine.device)
        lrdmc_jastrow_grad(engine.ctx, pos, out)
        ctx.engine, ctx.pos = engine, pos
        ctx.n_nodes = int(t.shape[1])
        return out[:, 1].clone(), out[:, 0].clone()

    @staticmethod
    def backward(ctx, g_j, g_e):
        engine = ctx.engine
        g = torch.empty(2, ctx.n_nodes, 3, dtype=torch.float64, device=engine.device)
        cj = None if g_j is None else g_j.contiguous()
        ce = None if g_e is None else g_e.contiguous()
        lrdmc_jastrow_table_grad(engine.ctx, ctx.pos, cj, ce, g)
        return g, None, None, None


def weighted_moments(j: torch.Tensor, e: torch.Tensor, j0: torch.Tensor, power: float):
    """Weighted mean and variance of E_L with weights exp(power (J - J0))."""
    lw = power * (j - j0)
    w = torch.exp(lw - lw.max())
    w = w / w.sum()
    mean = (w * e).sum()
    return mean, (w * (e - mean) ** 2).sum()


class NeuralJastrow:
    """Network parameters on the device plus the table geometry."""

    def __init__(self, hidden: int = 64, n_nodes: int = 257, r_cut: float = 6.0, params=None, seed: int = 0,
                 device="cuda"):
        self.hidden, self.n_nodes, self.r_cut = int(hidden), int(n_nodes), float(r_cut)
        if params is None:
            params = init_params(hidden, seed, device)
        self.params = torch.as_tensor(params, dtype=torch.float64).to(device).contiguous().requires_grad_(True)

    def table(self) -> torch.Tensor:
        return NetTable.apply(self.params, self.hidden, self.n_nodes, self.r_cut)

    def attach(self, engine: LRDMC):
        """Set the current table on a context (projection, evaluation)."""
        with torch.no_grad():
            engine.set_jastrow_table(self.table().detach(), self.r_cut)

    def energies(self, engine: LRDMC, pos: torch.Tensor):
        """(J[W], E_L[W]) with the current parameters, differentiable."""
        return TableJastrow.apply(self.table(), engine, pos, self.r_cut)

    def train(self, engine: LRDMC, pos, steps: int = 100, lr: float = 1e-3, power: float = 0.0,
              log: Optional[list] = None):
        """Variance minimisation of E_L over the configurations pos (device
        [W][N][3], sampled with the current trial function) with Adam.
        power = 0: the plain variance over the fixed sample (robust when the
        trial function moves far from the sampling one); power > 0: the
        correlated-sampling weights exp(power (J - J0)).  Returns the
        (mean, variance) history as floats."""
        pos = engine.positions(pos)
        with torch.no_grad():
            j0, _ = self.energies(engine, pos)
        opt = torch.optim.Adam([self.params], lr=lr)
        hist = [] if log is None else log
        for _ in range(steps):
            opt.zero_grad()
            j, e = self.energies(engine, pos)
            mean, var = weighted_moments(j, e, j0, power)
            var.backward()
            opt.step()
            hist.append((float(mean.detach()), float(var.detach())))
        self.attach(engine)
        return hist


def fit_vmc(nj: NeuralJastrow, engine: LRDMC, rounds: int = 8, steps: int = 60, lr: float = 1e-3,
            vmc_steps: int = 300, step: float = 0.25, power: float = 0.0, log=None):
    """Rounds of variance minimisation on Metropolis samples of |Psi|^2 from
    the engine's walkers (lrdmc_vmc), each followed by a fresh sample with the
    updated trial function; the parameters with the lowest variance of E_L
    on a fresh sample (held out from their own training) are kept and set on
    the engine.  The engine's walkers must be equilibrated samples.  Returns
    one dict per round."""
    out = engine.get_walkers()
    best_var = float(out["e_l"].var())
    best = nj.params.detach().clone()
    hist = [dict(round=-1, vmc_E=float(out["e_l"].mean()), vmc_var=best_var)]
    pos = out["pos"]
    for r in range(rounds):
        h = nj.train(engine, pos, steps=steps, lr=lr, power=power)
        engine.vmc(vmc_steps, step)
        out = engine.get_walkers()
        e = out["e_l"]
        row = dict(round=r, train_var_start=h[0][1], train_var_end=h[-1][1], vmc_E=float(e.mean()),
                   vmc_var=float(e.var()), acceptance=float(out["n_moves"].double().mean()) / vmc_steps)
        hist.append(row)
        if log is not None:
            log(row)
        if row["vmc_var"] < best_var:
            best_var, best = row["vmc_var"], nj.params.detach().clone()
        pos = out["pos"]
    with torch.no_grad():
        nj.params.copy_(best)
    nj.attach(engine)
    return hist

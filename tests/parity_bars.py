"""Bars of the GPU parity tests against the oracle, the tie rule for
indices, and a record of the differences observed in a session.

Indices (moves per generation, heat-bath choices, resampling indices) must be
bit-exact, except where the oracle's decision margin (its relative distance
of the threshold to the nearer end of the chosen cumulative interval, or of
the holding time to the time left) is below TIE: there the summation order
decides, and either index is accepted.  Such ties
are counted and reported; the trajectories that follow a tie are not
compared.

Every comparison records the largest difference it saw; the session summary
(tests/conftest.py) prints them, so the headroom under each bar is visible
in the test log.
"""
from __future__ import annotations

import numpy as np

TIE = 1e-12
OBSERVED: dict = {}

# FP64 bars.  Generation records (ebar, log wbar):
# the 1e-10 Ha target plus about 900 eps |E| for the synthetic atoms whose
# energies reach thousands of Ha (cancellation in E_L of tight Gaussians).
# Per-walker E_L (and sum_i lap_i Psi/Psi) relative to 1 + |E_L| (+ |lap|),
# log w relative to 1 + |log w|: these carry kappa(A) eps from the inverse
# and the Sherman-Morrison updates carried since the last refresh.  Move
# ratios: relative to |rho| plus a share of the walker's largest |rho| (a
# ratio near a node is a difference of large terms).


def record_bar(E):
    return 1e-10 + 2e-13 * np.abs(E)


WALKER_E_REL = 2e-10
WALKER_LOGW_REL = 2e-11


def ratio_bar(rho, scale):
    return 1e-11 * np.abs(rho) + 2e-12 * scale
TIES = {"count": 0, "where": []}


def record(name: str, value: float) -> None:
    v = float(value)
    if name not in OBSERVED or v > OBSERVED[name]:
        OBSERVED[name] = v


def check(name: str, got, ref, bar, scale=None) -> float:
    """Assert |got - ref| <= bar elementwise (bar broadcasts); record the
    largest |got - ref| under `name`, its largest share of the bar under
    `name/bar` and, given a magnitude `scale`, the largest |got - ref|/scale
    under `name/rel`.  Returns the largest difference."""
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    d = np.abs(got - ref)
    bar = np.broadcast_to(np.asarray(bar, dtype=np.float64), d.shape)
    dmax = float(d.max()) if d.size else 0.0
    record(name, dmax)
    if d.size:
        record(name + "/bar", float(np.max(d / bar)))
        if scale is not None:
            sc = np.broadcast_to(np.asarray(scale, dtype=np.float64), d.shape)
            record(name + "/rel", float(np.max(d / sc)))
    assert np.all(d <= bar), f"{name}: max |d| = {dmax:.3e}, worst share of the bar {np.max(d / bar):.3g}"
    print(f"{name}: max |d| = {dmax:.3e}", flush=True)
    return dmax


def tie(label: str, margin: float) -> None:
    assert margin < TIE, f"{label}: index differs from the oracle's at margin {margin:.3e} >= {TIE}"
    TIES["count"] += 1
    TIES["where"].append(f"{label} (margin {margin:.2e})")
    print(f"tolerated tie: {label}, oracle margin {margin:.2e}", flush=True)


def slot_agrees(label: str, n_gpu, n_orc, pos_gpu, pos_orc, margin, atol=1e-11) -> bool:
    """One walker slot after one generation: True when its move count and
    positions agree with the oracle's; otherwise the difference must come
    from a tie (asserted and counted) and the slot is not compared further."""
    if int(n_gpu) == int(n_orc) and np.allclose(pos_gpu, pos_orc, rtol=0, atol=atol):
        return True
    tie(f"{label}: moves {int(n_gpu)} vs {int(n_orc)}", margin)
    return False


def run_agrees(label: str, n_moves_gpu, idx_gpu, ref) -> int:
    """Whole projections: the number of leading generations whose records
    (log wbar, ebar) are comparable.  Move totals and resampling indices must
    agree up to the first tie; after a tie the trajectories differ."""
    nm_g = np.asarray(n_moves_gpu)
    nm_o = ref["n_moves"]
    mg = ref["margin"]
    n_gen = nm_o.shape[0]
    for g in range(n_gen):
        if nm_g[g] != nm_o[g]:
            tie(f"{label} generation {g}: moves {nm_g[g]} vs {nm_o[g]}", float(mg[g, 0].min()))
            return g
        if idx_gpu is not None:
            bad = np.nonzero(np.asarray(idx_gpu[g]) != ref["idx"][g])[0]
            if bad.size:
                tie(f"{label} generation {g}: {bad.size} resampling indices", float(mg[g, 1, bad].max()))
                return g + 1
    return n_gen

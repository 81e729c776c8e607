#!/usr/bin/env python
"""Benchmark of the double-grid LRDMC projection on one MI355X.

One step = one generation: a continuous-time projection of every walker over
projection time tau (all moves: table of 12N lattice moves, heat-bath choice,
Sherman-Morrison update) followed by the fixed-population reconfiguration.
The timed region runs `--steps` generations through lrdmc_run with the
walkers resident in HBM, bracketed by device synchronizations.

Workload (default): the largest configuration that fits one GPU, the
synthetic molecule: 4 nuclei Z = 8 and 8 nuclei Z = 1 at seeded positions
(minimum separation 1.8 bohr), 20 up / 20 down electrons, K = 256
even-tempered s/p/d Gaussians 0.05 * 2.5^k with a seeded orthonormal MO
matrix, Pade Jastrow b = 1, a = 1/28 bohr with r_c(a, Z = 8) and a' from the
paper's rule, R_c over the Z = 8 nuclei, 16384 walkers, FP64.  The same line
reports the molecule with the mixed-precision move table and the Ar-like atom
(Z = 18, K = 64, a = 0.1 bohr, 4096 walkers) on its fixed-size and on the
general kernel.

Prints one JSON line.  Runs on one GPU only (the walker population is not
sharded over several GPUs).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP64_PEAK_TFLOPS = 78.6       # MI355X FP64 vector peak (vendor figure)
METRIC = "LRDMC electron-moves/s"


def kernel_source_hash() -> str:
    """SHA-256 over the kernel sources and the build script (flags)."""
    h = hashlib.sha256()
    for rel in ("paper_1909_01589_amd/csrc/lrdmc.hip", "paper_1909_01589_amd/csrc/lrdmc_device.h",
                "paper_1909_01589_amd/build.py"):
        h.update(open(os.path.join(ROOT, rel), "rb").read())
    return h.hexdigest()


def _traffic_record(workload: str):
    """HBM bytes per projection launch measured with rocprofv3 counters
    (profiles/traffic_project_kernel.md), if they were taken on the current
    kernel sources."""
    path = os.path.join(ROOT, "profiles", "traffic_project_kernel.md")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m = re.search(r"^source_sha256 = ([0-9a-f]{64})$", text, re.M)
    if not m or m.group(1) != kernel_source_hash():
        return None
    m = re.search(r"^" + re.escape(workload) + r" bytes_per_launch = ([0-9.eE+]+)$", text, re.M)
    return float(m.group(1)) if m else None


HE_EXACT = -2.903724        # nonrelativistic He ground state, the value the paper quotes


def _switch_sum(pos, R, r_c, form):
    """Sum over electrons of the switch p at the electrons, averaged over
    walkers (the sampled N_core of Eq. (7))."""
    d2 = ((pos - R[None, None, :]) ** 2).sum(axis=2)
    p = 1.0 / (1.0 + r_c * r_c * d2) if form == 1 else np.exp(-d2 / (2.0 * r_c * r_c))
    return float(p.sum(axis=1).mean())


def _fit_e0(a, E, sig):
    """Weighted least squares E(a) = E0 + k1 a^2 + k2 a^4; (E0, sigma E0,
    chi^2 per degree of freedom)."""
    a, E, sig = (np.asarray(x, dtype=np.float64) for x in (a, E, sig))
    X = np.stack([np.ones_like(a), a ** 2, a ** 4], axis=1) / sig[:, None]
    y = E / sig
    coef, *_ = np.linalg.lstsq(X, y, rcond=None)
    cov = np.linalg.inv(X.T @ X)
    chi2 = float(((X @ coef - y) ** 2).sum()) / max(1, len(a) - 3)
    return float(coef[0]), float(np.sqrt(cov[0, 0])), chi2


def ascan(walkers=16384, t_equil=5.0, t_prod=20.0, alphas=(1.0, 1.25, 1.5, 1.75, 2.0, 2.5, 3.0, 3.5), seed=0,
          moves_per_electron=4.0):
    """The paper's spacing scan on helium with a nodeless trial function
    (fixed node exact): for the double grid of this paper (Gaussian switch,
    r_c from Eq. (S-13), a' from Eq. (6)), the earlier double grid (Pade
    switch, r_c = Z/2, a' from Eq. (4)) and the single grid, at
    a = 1/(alpha Z): LRDMC energies, moves per unit projection time, the
    single/double move-rate ratio beside Eq. (5) with the sampled N_core,
    and E0 from the fit E0 + k1 a^2 + k2 a^4.  Each run equilibrates for
    projection time t_equil and averages over t_prod (1/Ha), with tau per
    generation set for about `moves_per_electron` moves per electron."""
    import torch
    from paper_1909_01589_amd import inputs, stats
    from paper_1909_01589_amd.lrdmc import LRDMC, lrdmc_spacing, lrdmc_spacing_pade
    s = inputs.helium_nodeless()
    Z, N = float(s.Z[0]), s.n_elec
    pos0 = inputs.initial_walkers(s, walkers, seed)
    modes = {"double_grid": (0, 2), "double_grid_previous": (1, 2), "single_grid": (0, 1)}
    res = {}
    t0 = time.perf_counter()
    for mode, (form, grids) in modes.items():
        rows = []
        for al in alphas:
            a = 1.0 / (al * Z)
            if form == 1:
                rc, ap = lrdmc_spacing_pade(Z, a)
            elif grids == 2:
                rc, ap, _ = lrdmc_spacing(Z, a)
                ap = max(ap, a)    # Eq. (6) gives a'/a < 1 when N_core > Z/2
            else:
                rc, ap = 1.0, a
            kw = dict(seed=seed, switch_form=form, grids=grids, refresh=8)
            g = LRDMC(s, a, ap, rc, 1.0, walkers, **kw)
            delta = float(g.eval_moves(pos0)[2][:, 6].mean())
            g.close()
            tau = moves_per_electron * N / delta
            equil, gens = int(np.ceil(t_equil / tau)), int(np.ceil(t_prod / tau))
            g = LRDMC(s, a, ap, rc, tau, walkers, **kw)
            g.set_walkers(pos0, 0)
            g.run(equil)
            out = g.run(gens)
            torch.cuda.synchronize()
            lwb, eb = out["log_wbar"].cpu().numpy(), out["ebar"].cpu().numpy()
            E, sig = stats.estimate(lwb, eb, p=None)
            moves = int(out["n_moves"].sum())
            nc = _switch_sum(g.get_walkers()["pos"].cpu().numpy(), s.R[0], rc, form) if grids == 2 else float(N)
            g.close()
            rows.append(dict(alpha=al, a=a, a_prime=ap, r_c=rc, tau=tau, generations=gens, E=E, sigma=sig,
                             move_rate=moves / (walkers * tau * gens), n_core=nc))
        E0, s0, chi2 = _fit_e0([r["a"] for r in rows], [r["E"] for r in rows], [r["sigma"] for r in rows])
        res[mode] = dict(rows=rows, E0=E0, sigma_E0=s0, chi2_dof=chi2)
    speed = {}
    for mode in ("double_grid", "double_grid_previous"):
        lst = []
        for r1, r2 in zip(res["single_grid"]["rows"], res[mode]["rows"]):
            nc, ratio = r2["n_core"], r2["a_prime"] / r2["a"]
            lst.append(dict(alpha=r2["alpha"], measured=r1["move_rate"] / r2["move_rate"],
                            eq5=1.0 / (nc / N + (N - nc) / N * ratio ** -2)))
        speed[mode] = lst
    return {"ascan": {"system": "He, nodeless s orbital x Pade Jastrow (fixed node exact)",
                      "walkers": walkers, "equilibration_time": t_equil, "production_time": t_prod,
                      "energy": "mean of the generation energies, reblocked error",
                      "reference_E": HE_EXACT, "modes": res, "speedup": speed,
                      "wall_s": time.perf_counter() - t0}}


def jastrow_grad_bench(name="ar_a0.1", reps=50):
    """Throughput of the Jastrow-parameter gradient kernel on the walkers of a
    workload (one call = E_L, J and both parameter derivatives of every
    walker), timed with device synchronization around `reps` calls."""
    import torch
    from paper_1909_01589_amd import inputs
    from paper_1909_01589_amd.lrdmc import LRDMC, lrdmc_spacing
    cfg = inputs.get_config(name)
    s = cfg.system
    rc, ap, _ = lrdmc_spacing(s.z_max, cfg.a)
    g = LRDMC(s, cfg.a, ap, rc, cfg.tau, cfg.walkers, seed=cfg.seed, refresh=cfg.refresh)
    g.set_walkers(inputs.initial_walkers(s, cfg.walkers, cfg.seed), 0)
    g.run(20)
    pos = g.get_walkers()["pos"].clone()
    g.jastrow_grad(pos)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        g.jastrow_grad(pos)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    g.close()
    return {"jastrow_grad": {"workload": name, "walkers": cfg.walkers, "ms_per_call": 1e3 * dt,
                             "walker_gradients_per_s": cfg.walkers / dt}}


def neural_bench(system="ar", walkers=16384, rounds=8, train_steps=60, lr=1e-3, gens=1200, seed=0,
                 train_walkers=131072, spacings=None, forms=("pade", "neural"), gens_inverse_a=False,
                 runs_out=None, t_equil=None, t_prod=None):
    """Learned Jastrow correction against the Pade trial function alone.
    Metropolis samples of |Psi_Pade|^2 (lrdmc_vmc), rounds of variance
    minimisation of the 2 x 64 SiLU networks (tabulated on 257 nodes up to
    r_cut = 6 bohr) on `train_walkers` configurations per round (8 rounds:
    about 10^6 samples), each round followed by a fresh sample (the
    parameters with the lowest fresh-sample variance are kept), then LRDMC
    with `walkers` walkers and both trial
    functions at three spacings: energies with reblocked errors, move rates,
    the time to sigma(E) = 1 mHa extrapolated from each run
    (wall x (sigma / 1 mHa)^2), and E0 of the fit E0 + k a^2 (the lattice
    bias of LRDMC depends on the trial function; the fixed-node limits must
    agree, the determinant and hence the nodes being the same).
    system "ar": Ar with screened hydrogenic orbitals in the Ar-like basis;
    "he": He with a nodeless s orbital (fixed node exact).
    spacings: override the spacings; forms: the trial functions to run
    ("pade", "neural"); gens_inverse_a: `gens` at the largest spacing and
    gens x a_max / a at the others (the projection time per generation
    shrinks as a^2); t_prod: instead, the same projection time (Ha^-1) at
    every spacing; t_equil: projection time discarded before the timed
    production (default 2 Ha^-1 for Ar, 10 for He); runs_out: a file that
    receives one JSON line per LRDMC run (neural_summarize combines such
    files).  Each run also records the energies of the two halves of its
    production (a check that the discarded part was long enough)."""
    import torch
    from paper_1909_01589_amd import inputs, neural, stats
    from paper_1909_01589_amd.lrdmc import LRDMC, lrdmc_spacing
    if system == "ar":
        s, sp0, step, E_ref = inputs.ar_screened(), (0.06, 0.045, 0.035, 0.025, 0.0175), 0.25, None
        moves_per_electron, t_equil0 = 8.0, 2.0
    elif system == "he":
        s, sp0, step, E_ref = inputs.helium_nodeless(), (0.25, 0.15, 0.1), 0.6, HE_EXACT
        moves_per_electron, t_equil0 = 20.0, 10.0
    else:
        raise ValueError(system)
    t_equil = t_equil0 if t_equil is None else float(t_equil)
    spacings = tuple(spacings) if spacings else sp0
    a_max = max(spacings)
    Z, N = s.z_max, s.n_elec
    pos0 = inputs.initial_walkers(s, walkers, seed)
    t0 = time.perf_counter()

    def note(msg):
        print(f"[neural {system} {time.perf_counter() - t0:6.1f}s] {msg}", file=sys.stderr, flush=True)

    g = LRDMC(s, spacings[0], spacings[0], 1.0, 0.01, train_walkers, seed=seed + 3, rotate=1, refresh=8)
    g.set_walkers(inputs.initial_walkers(s, train_walkers, seed + 1), 0)
    g.vmc(3000, step)

    def spread(n_snap=4):
        """E_L over n_snap Metropolis snapshots 300 steps apart: mean, mean of
        the snapshot variances, and (1.4826 MAD)^2, a width the heavy tails of
        E_L do not dominate."""
        es = []
        for _ in range(n_snap):
            g.vmc(300, step)
            es.append(g.get_walkers()["e_l"].cpu().numpy())
        e = np.concatenate(es)
        mad = 1.4826 * np.median(np.abs(e - np.median(e)))
        return dict(E=float(e.mean()), var=float(np.mean([x.var() for x in es])), robust_var=float(mad * mad))

    vmc_pade = spread()
    nj = neural.NeuralJastrow(64, 257, 6.0, seed=seed)
    hist, t_train, vmc_neural = [], 0.0, None
    if "neural" in forms:
        t_train = time.perf_counter()
        hist = neural.fit_vmc(nj, g, rounds=rounds, steps=train_steps, lr=lr, vmc_steps=300, step=step,
                              log=lambda r: note(f"round {r['round']}: VMC E={r['vmc_E']:.4f} "
                                                 f"var={r['vmc_var']:.3f}"))
        t_train = time.perf_counter() - t_train
        vmc_neural = spread()
    g.close()

    def projection(with_net, a):
        rc, ap, _ = lrdmc_spacing(Z, a)
        ap = max(ap, a)
        g = LRDMC(s, a, ap, rc, 1.0, walkers, seed=seed + 11, rotate=1, refresh=8)
        if with_net:
            nj.attach(g)
        g.set_walkers(pos0, 0)
        g.vmc(2000, step)
        p = g.get_walkers()["pos"]
        delta = float(g.eval_moves(p)[2][:, 6].mean())
        g.close()
        tau = moves_per_electron * N / delta
        g = LRDMC(s, a, ap, rc, tau, walkers, seed=seed + 11, rotate=1, refresh=8)
        if with_net:
            nj.attach(g)
        g.set_walkers(p, 0)
        form = "neural" if with_net else "pade"
        chunk = max(1, int(round(2.0 / tau)))          # 2 Ha^-1 of projection per call
        n_eq = int(t_equil / tau) + 20
        for c0 in range(0, n_eq, chunk):
            g.run(min(chunk, n_eq - c0))
        n_gen = int(round(gens * a_max / a)) if gens_inverse_a else gens
        if t_prod is not None:
            n_gen = int(round(t_prod / tau))
        note(f"{form} a={a}: {n_eq} generations discarded, {n_gen} timed")
        parts = []
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        t_note = t1
        for c0 in range(0, n_gen, 4 * chunk):
            parts.append(g.run(min(4 * chunk, n_gen - c0)))
            torch.cuda.synchronize()
            if time.perf_counter() - t_note > 30.0:
                t_note = time.perf_counter()
                note(f"  {min(n_gen, c0 + 4 * chunk)} of {n_gen} generations")
        dt = time.perf_counter() - t1
        lw = torch.cat([q["log_wbar"] for q in parts]).cpu().numpy()
        eb = torch.cat([q["ebar"] for q in parts]).cpu().numpy()
        E, sig = stats.estimate(lw, eb, p=None)
        h = n_gen // 2
        halves = [stats.estimate(lw[:h], eb[:h], p=None), stats.estimate(lw[h:], eb[h:], p=None)]
        moves = int(sum(int(q["n_moves"].sum()) for q in parts))
        g.close()
        row = dict(form=form, a=a, a_prime=ap, r_c=rc, tau=tau, generations=n_gen, E=E,
                   sigma=sig, wall_s=dt, moves_per_s=moves / dt, t_1mHa_s=dt * (sig / 1e-3) ** 2,
                   t_equil=t_equil, t_prod=n_gen * tau, E_halves=[list(x) for x in halves])
        if runs_out:
            with open(runs_out, "a") as f:
                f.write(json.dumps(row) + "\n")
        note(f"{form} a={a}: E={E:.5f} +- {sig:.5f} t(1mHa)={row['t_1mHa_s']:.1f}s, halves "
             f"{halves[0][0]:.5f} +- {halves[0][1]:.5f} and {halves[1][0]:.5f} +- {halves[1][1]:.5f}")
        return row

    rows = []
    for label, net in (("pade", False), ("neural", True)):
        if label in forms:
            rows += [projection(net, a) for a in spacings]
    out = neural_summarize(rows)
    out.update({
        "system": s.name, "walkers": walkers, "training_walkers": train_walkers,
        "network": "2 x 64 SiLU per pair type, 257-node table, r_cut 6",
        "training": dict(rounds=rounds, steps_per_round=train_steps, lr=lr, wall_s=t_train, history=hist),
        "vmc": dict(pade=vmc_pade, neural=vmc_neural), "reference_E": E_ref, "wall_s": time.perf_counter() - t0})
    return {"neural": out}


NEURAL_FITS = (("E0 + k1 a^2 + k2 a^4", (2, 4)), ("E0 + k1 a^2 + k2 a^4 + k3 a^6", (2, 4, 6)),
               ("E0 + k1 a + k2 a^2", (1, 2)), ("E0 + k1 a + k2 a^2 + k3 a^3", (1, 2, 3)))


def _fit_poly(a, E, sig, powers):
    """Weighted fit E = E0 + sum_p k_p a^p: (E0, sigma_E0, chi2 per degree of
    freedom, degrees of freedom)."""
    a = np.asarray(a, dtype=np.float64)
    E = np.asarray(E, dtype=np.float64)
    w = 1.0 / np.asarray(sig, dtype=np.float64) ** 2
    X = np.stack([np.ones_like(a)] + [a ** q for q in powers], axis=1)
    cov = np.linalg.inv(X.T @ (X * w[:, None]))
    beta = cov @ (X.T @ (w * E))
    r = E - X @ beta
    dof = len(E) - X.shape[1]
    return float(beta[0]), float(np.sqrt(cov[0, 0])), float((w * r * r).sum() / max(dof, 1)), dof


def neural_summarize(rows):
    """Per trial function (rows: per-run dicts with form, a, E, sigma,
    t_1mHa_s) the fit of E(a) (E0 + k1 a^2 + k2 a^4 from four spacings on,
    else E0 + k1 a^2) and, with both forms, the difference of the limits
    and the time-to-1 mHa ratios at the common spacings.  With five
    spacings or more, every model of NEURAL_FITS that leaves a degree of
    freedom is fitted as well ("fits"), with the difference of the limits
    per model: whether E(a) is in its a^2 regime decides which limit means
    anything."""
    res = {}
    for label in ("pade", "neural"):
        rs = sorted((r for r in rows if r["form"] == label), key=lambda r: -r["a"])
        if not rs:
            continue
        a_, E_, s_ = [r["a"] for r in rs], [r["E"] for r in rs], [r["sigma"] for r in rs]
        if len(rs) >= 4:
            E0, s0, chi2 = _fit_e0(a_, E_, s_)           # E0 + k1 a^2 + k2 a^4
            fit = "E0 + k1 a^2 + k2 a^4"
        else:
            E0, s0, chi2 = _fit_e0_linear(a_, E_, s_)    # E0 + k1 a^2
            fit = "E0 + k1 a^2"
        res[label] = dict(rows=rs, fit=fit, E0=E0, sigma_E0=s0, chi2_dof=chi2)
        if len(rs) >= 5:
            res[label]["fits"] = {}
            for name, powers in NEURAL_FITS:
                if len(rs) > len(powers) + 1:
                    e0, se0, c2, dof = _fit_poly(a_, E_, s_, powers)
                    res[label]["fits"][name] = dict(E0=e0, sigma_E0=se0, chi2_dof=c2, dof=dof)
    out = {"lrdmc": res}
    if "pade" in res and "neural" in res:
        by_a = {r["a"]: r for r in res["neural"]["rows"]}
        out["time_to_1mHa_ratio_pade_over_neural"] = {str(r["a"]): r["t_1mHa_s"] / by_a[r["a"]]["t_1mHa_s"]
                                                     for r in res["pade"]["rows"] if r["a"] in by_a}
        out["E0_difference"] = res["neural"]["E0"] - res["pade"]["E0"]
        out["E0_difference_sigma"] = float(np.hypot(res["pade"]["sigma_E0"], res["neural"]["sigma_E0"]))
        fp, fn = res["pade"].get("fits", {}), res["neural"].get("fits", {})
        out["E0_difference_per_fit"] = {k: dict(diff=fn[k]["E0"] - fp[k]["E0"],
                                                sigma=float(np.hypot(fn[k]["sigma_E0"], fp[k]["sigma_E0"])))
                                        for k in fp if k in fn}
    return out


def _fit_e0_linear(a, E, sig):
    """Weighted fit E = E0 + k a^2: (E0, sigma_E0, chi2 per degree of freedom)."""
    a2 = np.asarray(a, dtype=np.float64) ** 2
    E = np.asarray(E, dtype=np.float64)
    w = 1.0 / np.asarray(sig, dtype=np.float64) ** 2
    X = np.stack([np.ones_like(a2), a2], axis=1)
    cov = np.linalg.inv(X.T @ (X * w[:, None]))
    beta = cov @ (X.T @ (w * E))
    r = E - X @ beta
    dof = max(1, len(E) - 2)
    return float(beta[0]), float(np.sqrt(cov[0, 0])), float((w * r * r).sum() / dof)


def zscan(Zs=(10, 18, 36, 54), walkers=8192, gens=20, warmup=10, moves_per_electron=2.0, seed=0):
    """Cost of the projection against the atomic number at a = 1/(3.5 Z)
    (the spacing of the paper's Table I and its CPU-time scaling figure) on
    the Z-sweep atoms, for the single grid and this paper's double grid
    (Eq. (3), r_c from Eq. (S-13), a' from Eq. (6)).  Walkers are first
    brought to the trial function's |Psi|^2 by Metropolis sampling
    (30 N steps).  Reported per Z and grid: projection time per second
    W tau n_gen / wall (what the double grid improves), GPU seconds per walker
    and unit projection time, electron-moves/s, the kernel time per
    generation; per Z the acceleration (ratio of costs), the single/double
    move-rate ratio Delta_s / Delta_d beside Eq. (5) with the sampled
    N_core = <sum_i p(r_i)>; and power-law exponents of the cost in Z.  tau
    per generation is set for about `moves_per_electron` moves per electron."""
    import torch
    from paper_1909_01589_amd import inputs
    from paper_1909_01589_amd.lrdmc import LRDMC, lrdmc_spacing, lrdmc_set_timing, lrdmc_timing
    rows, per_z = [], []
    for Z in Zs:
        s = inputs.zsweep_atom(Z, seed)
        N = s.n_elec
        a = 1.0 / (3.5 * Z)
        g = LRDMC(s, a, a, 1.0, 1.0, walkers, seed=seed, rotate=1, refresh=8, grids=1)
        g.set_walkers(inputs.initial_walkers(s, walkers, seed), 0)
        g.vmc(30 * N, 0.2)
        out = g.get_walkers()
        pos0 = out["pos"].clone()
        acc = float(out["n_moves"].double().mean()) / (30 * N)
        g.close()
        rc_d, ap_d, nc_model = lrdmc_spacing(float(Z), a)
        ap_d = max(ap_d, a)
        nc_sampled = _switch_sum(pos0.cpu().numpy(), s.R[0], rc_d, 0)
        deltas = {}
        for mode in ("single_grid", "double_grid"):
            if mode == "double_grid":
                rc, ap, kw = rc_d, ap_d, dict(grids=2)
            else:
                rc, ap, kw = 1.0, a, dict(grids=1)
            g = LRDMC(s, a, ap, rc, 1.0, walkers, seed=seed, rotate=1, refresh=8, **kw)
            delta = float(g.eval_moves(pos0)[2][:, 6].mean())
            g.close()
            deltas[mode] = delta
            tau = moves_per_electron * N / delta
            g = LRDMC(s, a, ap, rc, tau, walkers, seed=seed, rotate=1, refresh=8, **kw)
            g.set_walkers(pos0, 0)
            g.run(warmup)
            torch.cuda.synchronize()
            print(f"[zscan] Z={Z} {mode}: tau={tau:.3e}, warm", file=sys.stderr, flush=True)
            lrdmc_set_timing(g.ctx, 1)
            t0 = time.perf_counter()
            out = g.run(gens)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            tm = lrdmc_timing(g.ctx)
            moves = int(out["n_moves"].sum())
            g.close()
            rows.append(dict(Z=Z, mode=mode, electrons=N, basis=s.n_basis, a=a, a_prime=ap, r_c=rc, tau=tau,
                             delta=delta, moves_per_s=moves / dt,
                             kernel_ms_per_generation=tm[0] / max(1.0, tm[1]),
                             projection_time_per_s=walkers * tau * gens / dt,
                             cost_s_per_walker_per_unit_time=dt / (walkers * gens * tau)))
            print(f"[zscan] Z={Z} {mode}: a'={ap:.4f} {moves / dt / 1e6:.1f} M moves/s, "
                  f"{rows[-1]['projection_time_per_s']:.3g} walker-Ha^-1 per s", file=sys.stderr, flush=True)
        c = {x["mode"]: x["cost_s_per_walker_per_unit_time"] for x in rows if x["Z"] == Z}
        ratio = ap_d / a
        per_z.append(dict(Z=Z, vmc_acceptance=acc, n_core_model=nc_model, n_core_sampled=nc_sampled,
                          a_prime_over_a=ratio, acceleration=c["single_grid"] / c["double_grid"],
                          move_rate_ratio=deltas["single_grid"] / deltas["double_grid"],
                          eq5_sampled=1.0 / (nc_sampled / N + (N - nc_sampled) / N * ratio ** -2),
                          eq5_model=1.0 / (nc_model / N + (N - nc_model) / N * ratio ** -2)))
    fits = {}
    for mode in ("single_grid", "double_grid"):
        r = [x for x in rows if x["mode"] == mode]
        fits[mode] = float(np.polyfit(np.log([x["Z"] for x in r]),
                                      np.log([x["cost_s_per_walker_per_unit_time"] for x in r]), 1)[0])
    return {"zscan": {"walkers": walkers, "generations": gens, "rows": rows, "per_Z": per_z,
                      "cost_exponent": fits,
                      "cost": "GPU seconds per walker per unit projection time (1/Ha), at a = 1/(3.5 Z)"}}


SWEEP = (("be", 300, 30), ("ar_a0.2", 300, 30), ("ar_a0.1", 300, 30), ("zsweep10", 100, 10), ("zsweep18", 100, 10),
         ("zsweep36", 30, 5), ("zsweep54", 20, 5), ("molecule", 20, 5))


# Acceleration column of Table S-I (ratio of accepted off-diagonal moves,
# single over double grid) at a = 1/(alpha Z), for the rows measured here.
TABLE_S1_ACCELERATION = {("Be", 3.33): 2.0, ("Be", 2.0): 1.8, ("Be", 1.0): 1.4,
                         ("Ne", 3.33): 3.5, ("Ne", 2.0): 3.1, ("Ne", 1.0): 2.4}


def _production(s, a, ap, rc, grids, tau, pos0, walkers, t_equil, t_prod, ms_per_gen, seed, tag):
    """Equilibrate for projection time t_equil, then run t_prod on the general
    kernel in chunks of about 20 s (a progress line each): (E, sigma) of the
    generation energies (reblocked), generations and production wall time."""
    import torch
    from paper_1909_01589_amd import stats
    from paper_1909_01589_amd.lrdmc import LRDMC, lrdmc_use_generic
    g = LRDMC(s, a, ap, rc, tau, walkers, seed=seed, rotate=1, refresh=8, grids=grids)
    lrdmc_use_generic(g.ctx, 1)
    g.set_walkers(pos0, 0)
    chunk = max(100, int(20e3 / ms_per_gen))
    n_eq, n_prod = int(np.ceil(t_equil / tau)), int(np.ceil(t_prod / tau))
    while n_eq > 0:
        g.run(min(chunk, n_eq))
        n_eq -= chunk
    torch.cuda.synchronize()
    lw, eb, done, wall = [], [], 0, 0.0
    while done < n_prod:
        n = min(chunk, n_prod - done)
        t0 = time.perf_counter()
        out = g.run(n)
        torch.cuda.synchronize()
        wall += time.perf_counter() - t0
        lw.append(out["log_wbar"].cpu().numpy())
        eb.append(out["ebar"].cpu().numpy())
        done += n
        print(f"[zscan-phys] {tag}: {done}/{n_prod} generations", file=sys.stderr, flush=True)
    g.close()
    lw, eb = np.concatenate(lw), np.concatenate(eb)
    E, sig = stats.estimate(lw, eb, p=None)
    h = n_prod // 2
    (E1, s1), (E2, s2) = stats.estimate(lw[:h], eb[:h], p=None), stats.estimate(lw[h:], eb[h:], p=None)
    return dict(E=E, sigma=sig, t_prod=t_prod, generations=n_prod, wall_s=wall,
                time_to_1mHa_s=wall * (sig / 1e-3) ** 2, E_first_half=E1, sigma_first_half=s1,
                E_second_half=E2, sigma_second_half=s2)


def zscan_phys(walkers=8192, gens=100, warmup=20, moves_per_electron=2.0, seed=0, t_equil=5.0,
               t_prod=None, alpha_prod=3.5):
    """Single vs double grid for Be, Ne and Ar with screened hydrogenic
    orbitals (physical core densities, unlike the random-MO Z-sweep atoms) at
    a = 1/(alpha Z): the move-rate ratio beside Eq. (5) with the sampled
    N_core and beside the acceleration column of Table S-I (Be and Ne), and
    the ratio of GPU cost per unit projection time, both grids on the general
    kernel (the kernels built for fixed sizes exist for the double grid only;
    where one serves the system, its ratio is reported beside).  Single and double grid
    share the trial function and its nodes, so to first order the cost ratio
    is the ratio of times to a fixed error (the paper's CPU-time
    accelerations at alpha = 3.5: Be 1.4, Ne 2.3, Ar 3.3).  At alpha_prod
    both grids also run a production of projection time t_prod[atom] for the
    time to sigma(E) = 1 mHa, its single/double ratio and the double - single
    energy difference (the bias column of Table S-I)."""
    import torch
    from paper_1909_01589_amd import inputs
    from paper_1909_01589_amd.lrdmc import LRDMC, lrdmc_is_specialized, lrdmc_spacing, lrdmc_use_generic
    t_prod = dict(Be=80.0, Ne=40.0, Ar=8.0) if t_prod is None else t_prod
    systems = (("Be", inputs.atom_screened(4, (8, 0, 0), 0.1, 3.0, name="be_screened"), 0.5,
                (3.33, 3.5, 2.0, 1.0)),
               ("Ne", inputs.atom_screened(10, (11, 6, 0), 0.05, 2.5, name="ne_screened"), 0.3,
                (3.33, 3.5, 2.0, 1.0)),
               ("Ar", inputs.ar_screened(), 0.25, (3.33, 3.5)))
    out = []
    for label, s, step, alphas in systems:
        Z, N = s.z_max, s.n_elec
        g = LRDMC(s, 0.01, 0.01, 1.0, 1.0, walkers, seed=seed, rotate=1, refresh=8, grids=1)
        g.set_walkers(inputs.initial_walkers(s, walkers, seed), 0)
        g.vmc(100 * N, step)
        pos0 = g.get_walkers()["pos"].clone()
        g.close()
        for alpha in alphas:
            a = 1.0 / (alpha * Z)
            rc_d, ap_d, nc_model = lrdmc_spacing(float(Z), a)
            ap_d = max(ap_d, a)
            nc = _switch_sum(pos0.cpu().numpy(), s.R[0], rc_d, 0)
            cost, delta, taus, ms, jumps = {}, {}, {}, {}, {}
            specialized = False
            for mode, (rc, ap, grids, generic) in (("single_grid", (1.0, a, 1, 1)), ("double_grid", (rc_d, ap_d, 2, 1)),
                                                   ("double_grid_auto", (rc_d, ap_d, 2, 0))):
                if mode == "double_grid_auto":
                    delta[mode] = delta["double_grid"]
                else:
                    g = LRDMC(s, a, ap, rc, 1.0, walkers, seed=seed, rotate=1, refresh=8, grids=grids)
                    delta[mode] = float(g.eval_moves(pos0)[2][:, 6].mean())
                    g.close()
                tau = moves_per_electron * N / delta[mode]
                g = LRDMC(s, a, ap, rc, tau, walkers, seed=seed, rotate=1, refresh=8, grids=grids)
                lrdmc_use_generic(g.ctx, generic)
                if mode == "double_grid_auto":
                    specialized = lrdmc_is_specialized(g.ctx)
                    if not specialized:
                        g.close()
                        continue
                g.set_walkers(pos0, 0)
                g.run(warmup)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                rec = g.run(gens)
                torch.cuda.synchronize()
                wall = time.perf_counter() - t0
                jumps[mode] = float(rec["n_moves"].double().mean()) / walkers
                cost[mode] = wall / (walkers * gens * tau)
                taus[mode], ms[mode] = tau, 1e3 * wall / gens
                g.close()
            ratio = ap_d / a
            row = dict(atom=label, Z=Z, alpha=alpha, a=a, a_prime=ap_d, r_c=rc_d, n_core_model=nc_model,
                       n_core_sampled=nc, move_rate_ratio=delta["single_grid"] / delta["double_grid"],
                       eq5_sampled=1.0 / (nc / N + (N - nc) / N * ratio ** -2),
                       eq5_model=1.0 / (nc_model / N + (N - nc_model) / N * ratio ** -2),
                       tau_single=taus["single_grid"], tau_double=taus["double_grid"],
                       ms_per_gen_single=ms["single_grid"], ms_per_gen_double=ms["double_grid"],
                       moves_per_walker_gen_single=jumps["single_grid"],
                       moves_per_walker_gen_double=jumps["double_grid"],
                       cost_single=cost["single_grid"], cost_double=cost["double_grid"],
                       acceleration=cost["single_grid"] / cost["double_grid"],
                       ms_per_gen_double_specialized=ms["double_grid_auto"] if specialized else None,
                       acceleration_specialized_double=(cost["single_grid"] / cost["double_grid_auto"]
                                                        if specialized else None),
                       paper_acceptance=TABLE_S1_ACCELERATION.get((label, alpha)))
            if alpha == alpha_prod:
                prod = {}
                for mode, (rc, ap, grids) in (("single_grid", (1.0, a, 1)), ("double_grid", (rc_d, ap_d, 2))):
                    prod[mode] = _production(s, a, ap, rc, grids, taus[mode], pos0, walkers, t_equil,
                                             t_prod[label], ms[mode], seed, f"{label} {mode}")
                ps, pd = prod["single_grid"], prod["double_grid"]
                row["production"] = prod
                row["time_to_error_acceleration"] = ps["time_to_1mHa_s"] / pd["time_to_1mHa_s"]
                row["bias_mHa"] = 1e3 * (pd["E"] - ps["E"])
                row["bias_sigma_mHa"] = 1e3 * float(np.hypot(pd["sigma"], ps["sigma"]))
            print(f"[zscan-phys] {label} alpha={alpha}: N_core {nc:.3f} (model {nc_model:.3f}), move-rate ratio "
                  f"{row['move_rate_ratio']:.3f} (Eq. 5: {row['eq5_sampled']:.3f}), acceleration {row['acceleration']:.2f}",
                  file=sys.stderr, flush=True)
            out.append(row)
    return {"zscan_phys": {"walkers": walkers, "generations": gens, "rows": out,
                           "paper_cpu_time_alpha_3.5": {"Be": 1.4, "Ne": 2.3, "Ar": 3.3}}}


def mixed_bench(walkers=16384, gens=1200, seed=0):
    """FP64 against the mixed-precision move table (lrdmc_set_precision 1):
    throughput on the benchmark workload (same kernel otherwise), and on two
    physical trial functions (helium with a nodeless orbital, fixed node
    exact; Ar with screened hydrogenic orbitals) the energy, its reblocked
    error over `gens` generations after equilibration from the same walkers,
    and the time to sigma(E) = 1 mHa, both as measured and from the pooled
    variance per unit projection time of the two runs (the same process up to
    rounding of the transition probabilities, so the pooled figure isolates
    the speed); last, the throughput of both tables on the screened Ar atom
    with and without a learned-correction table."""
    import torch
    from paper_1909_01589_amd import inputs, stats
    from paper_1909_01589_amd.lrdmc import LRDMC, lrdmc_set_precision, lrdmc_spacing
    out = {"throughput": {}, "systems": []}
    for p in (0, 1):
        cfg, r = run_workload("ar_a0.1", 1000, 100, False, 0.0, precision=p)
        out["throughput"]["fp64" if p == 0 else "mixed"] = dict(value=r["value"], ms_per_step=r["ms_per_step"],
                                                                 frac=r["roofline"]["frac"])
        print(f"[mixed] ar_a0.1 precision={p}: {r['value'] / 1e6:.2f} M electron-moves/s", file=sys.stderr, flush=True)
    out["throughput_z54"] = {}
    for p in (0, 1):
        cfg, r = run_workload("zsweep54", 20, 5, False, 0.0, precision=p)
        out["throughput_z54"]["fp64" if p == 0 else "mixed"] = dict(value=r["value"], ms_per_step=r["ms_per_step"])
        print(f"[mixed] zsweep54 precision={p}: {r['value'] / 1e6:.2f} M electron-moves/s", file=sys.stderr, flush=True)
    for label, s, a, step, mpe, t_equil in (("He nodeless", inputs.helium_nodeless(), 0.1, 0.6, 20.0, 10.0),
                                             ("Ar screened", inputs.ar_screened(), 0.035, 0.25, 8.0, 2.0)):
        rc, ap, _ = lrdmc_spacing(s.z_max, a)
        ap = max(ap, a)
        g = LRDMC(s, a, ap, rc, 1.0, walkers, seed=seed + 11, rotate=1, refresh=8)
        g.set_walkers(inputs.initial_walkers(s, walkers, seed), 0)
        g.vmc(2000, step)
        pos = g.get_walkers()["pos"].clone()
        delta = float(g.eval_moves(pos)[2][:, 6].mean())
        g.close()
        tau = mpe * s.n_elec / delta
        rows = {}
        for p in (0, 1):
            g = LRDMC(s, a, ap, rc, tau, walkers, seed=seed + 11, rotate=1, refresh=8)
            lrdmc_set_precision(g.ctx, p)
            g.set_walkers(pos, 0)
            g.run(int(t_equil / tau) + 20)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            rec = g.run(gens)
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            E, sig = stats.estimate(rec["log_wbar"].cpu().numpy(), rec["ebar"].cpu().numpy(), p=None)
            rows["fp64" if p == 0 else "mixed"] = dict(
                E=E, sigma=sig, wall_s=wall, moves_per_s=float(rec["n_moves"].sum()) / wall,
                time_to_1mHa_s=wall * (sig / 1e-3) ** 2)
            g.close()
            print(f"[mixed] {label} precision={p}: E={E:.5f} +- {sig:.5f}, {wall:.1f} s", file=sys.stderr, flush=True)
        f, m = rows["fp64"], rows["mixed"]
        pooled = 0.5 * (f["sigma"] ** 2 + m["sigma"] ** 2) / 1e-6
        out["systems"].append(dict(
            system=label, a=a, a_prime=ap, tau=tau, walkers=walkers, generations=gens, runs=rows,
            energy_difference=m["E"] - f["E"], energy_difference_sigma=float(np.hypot(f["sigma"], m["sigma"])),
            speed_ratio=f["wall_s"] / m["wall_s"],
            time_to_1mHa_ratio_measured=f["time_to_1mHa_s"] / m["time_to_1mHa_s"],
            time_to_1mHa_pooled_s={"fp64": f["wall_s"] * pooled, "mixed": m["wall_s"] * pooled}))
    # throughput with and without a learned-correction table on the screened Ar atom
    s = inputs.ar_screened()
    a, tau = 0.05, 0.02
    rc, ap, _ = lrdmc_spacing(s.z_max, a)
    ap = max(ap, a)
    pos0 = inputs.initial_walkers(s, walkers, seed)
    tab = inputs.jastrow_table(seed=1, n_nodes=257, r_cut=6.0, scale=0.05)
    out["correction"] = []
    for table in (False, True):
        row = dict(table=table, a=a, tau=tau, walkers=walkers)
        for p in (0, 1):
            g = LRDMC(s, a, ap, rc, tau, walkers, seed=1, rotate=1, refresh=8)
            if table:
                g.set_jastrow_table(tab, 6.0)
            lrdmc_set_precision(g.ctx, p)
            g.set_walkers(pos0, 0)
            g.run(40)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            rec = g.run(60)
            torch.cuda.synchronize()
            row["fp64" if p == 0 else "mixed"] = float(rec["n_moves"].sum()) / (time.perf_counter() - t0)
            g.close()
        print(f"[mixed] screened Ar table={table}: {row['fp64'] / 1e6:.1f} -> {row['mixed'] / 1e6:.1f} M electron-moves/s",
              file=sys.stderr, flush=True)
        out["correction"].append(row)
    return {"mixed_precision": out}


def mixed_molecule(gens=400, equil=100, vmc_steps=800, step=0.3, seed=0):
    """FP64 against the mixed-precision move table on the benchmark molecule
    (16384 walkers, a = 1/28): both projections start from the same
    Metropolis sample of |Psi|^2 with the same random keys, run `equil`
    untimed and `gens` timed generations; reported per table the energy with
    its reblocked error, the wall rate and the smallest effective sample size,
    and the energy difference.  The random orbitals make these energies a
    property of this synthetic trial function only, not of a physical
    system."""
    import torch
    from paper_1909_01589_amd import inputs, stats
    from paper_1909_01589_amd.lrdmc import LRDMC, lrdmc_set_precision, lrdmc_spacing
    cfg = inputs.get_config("molecule")
    s, W = cfg.system, cfg.walkers
    rc, ap, _ = lrdmc_spacing(s.z_max, cfg.a)
    g = LRDMC(s, cfg.a, ap, rc, cfg.tau, W, seed=cfg.seed, rotate=cfg.rotate, refresh=cfg.refresh)
    g.set_walkers(inputs.initial_walkers(s, W, seed), 0)
    g.vmc(vmc_steps, step)
    pos = g.get_walkers()["pos"].clone()
    g.close()
    rows = {}
    for p in (0, 1):
        g = LRDMC(s, cfg.a, ap, rc, cfg.tau, W, seed=cfg.seed, rotate=cfg.rotate, refresh=cfg.refresh)
        lrdmc_set_precision(g.ctx, p)
        g.set_walkers(pos, 0)
        g.run(equil)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rec = g.run(gens)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        E, sig = stats.estimate(rec["log_wbar"].cpu().numpy(), rec["ebar"].cpu().numpy(), p=None)
        rows["fp64" if p == 0 else "mixed"] = dict(E=E, sigma=sig, wall_s=wall,
                                                   moves_per_s=float(rec["n_moves"].sum()) / wall,
                                                   ess_min=float(rec["ess"].min()) / W)
        g.close()
        print(f"[mixed molecule] precision={p}: E={E:.4f} +- {sig:.4f}, {wall:.1f} s", file=sys.stderr, flush=True)
    f, m = rows["fp64"], rows["mixed"]
    return {"mixed_molecule": dict(walkers=W, a=cfg.a, a_prime=ap, tau=cfg.tau, equilibration_generations=equil,
                                   generations=gens, vmc_steps=vmc_steps, runs=rows,
                                   energy_difference=m["E"] - f["E"],
                                   energy_difference_sigma=float(np.hypot(f["sigma"], m["sigma"])),
                                   speed_ratio=f["wall_s"] / m["wall_s"])}


def tsigma_bench(seeds=8, walkers=16384, a=0.035, gens=1000, moves_per_electron=8.0, t_equil=2.0, seed0=0,
                 rounds=8, train_steps=60, lr=1e-3, train_walkers=131072, step=0.25, first_seed=0, runs_out=None):
    """Time to sigma(E) = 1 mHa of four forms of the projection on the same
    physical system (Ar with screened hydrogenic orbitals in the Ar-like
    basis, a = 0.035 bohr, `walkers` walkers): Pade FP64, Pade with the
    mixed-precision move table, the learned Jastrow correction (trained once
    by variance minimisation on about 10^6 Metropolis samples), and both.
    Each form runs `seeds` independent projections (own start walkers and
    random keys), each `gens` generations after t_equil of equilibration.
    Per run: c = wall time per unit projection time, v = sigma(E)^2 x
    projection time (the variance per unit projection time, reblocked).
    Per form: the means of c and v over the seeds with their standard errors;
    time to 1 mHa = mean(c) mean(v) / 1e-6; the ratio of FP64 to each form
    with a 95 % interval from the spread over seeds (delta method on log c
    and log v).  The energies of the forms are compared with their errors.
    first_seed: index of the first seed (so that the seeds can be split over
    several calls); runs_out: a file that receives one JSON line per run as
    it ends (tsigma_summary combines such files)."""
    import torch
    from paper_1909_01589_amd import inputs, neural, stats
    from paper_1909_01589_amd.lrdmc import LRDMC, lrdmc_set_precision, lrdmc_spacing
    s = inputs.ar_screened()
    N = s.n_elec
    rc, ap, _ = lrdmc_spacing(s.z_max, a)
    ap = max(ap, a)
    t0 = time.perf_counter()

    def note(msg):
        print(f"[tsigma {time.perf_counter() - t0:7.1f}s] {msg}", file=sys.stderr, flush=True)

    # the learned correction, trained once
    g = LRDMC(s, a, a, 1.0, 0.01, train_walkers, seed=seed0 + 3, rotate=1, refresh=8)
    g.set_walkers(inputs.initial_walkers(s, train_walkers, seed0 + 1), 0)
    g.vmc(3000, step)
    nj = neural.NeuralJastrow(64, 257, 6.0, seed=seed0)
    t_train = time.perf_counter()
    neural.fit_vmc(nj, g, rounds=rounds, steps=train_steps, lr=lr, vmc_steps=300, step=step,
                   log=lambda r: note(f"training round {r['round']}: VMC var={r['vmc_var']:.2f}"))
    t_train = time.perf_counter() - t_train
    g.close()

    def start(net, sd):
        """VMC-equilibrated start walkers of seed sd and tau for the form's
        trial function (moves_per_electron moves per electron and generation)."""
        g = LRDMC(s, a, ap, rc, 1.0, walkers, seed=1000 + sd, rotate=1, refresh=8)
        if net:
            nj.attach(g)
        g.set_walkers(inputs.initial_walkers(s, walkers, 100 + sd), 0)
        g.vmc(2000, step)
        pos = g.get_walkers()["pos"].clone()
        delta = float(g.eval_moves(pos)[2][:, 6].mean())
        g.close()
        return pos, delta

    forms = (("fp64", False, 0), ("mixed", False, 1), ("neural", True, 0), ("neural+mixed", True, 1))
    taus = {}
    for net in (False, True):
        _, delta = start(net, 0)
        taus[net] = float(f"{moves_per_electron * N / delta:.3g}")
    runs = {f: [] for f, _, _ in forms}
    for sd in range(first_seed, first_seed + seeds):
        starts = {net: start(net, sd)[0] for net in (False, True)}
        for label, net, prec in forms:
            tau = taus[net]
            g = LRDMC(s, a, ap, rc, tau, walkers, seed=seed0 + 17 * sd + 5, rotate=1, refresh=8)
            if net:
                nj.attach(g)
            lrdmc_set_precision(g.ctx, prec)
            g.set_walkers(starts[net], 0)
            g.run(int(t_equil / tau) + 20)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            rec = g.run(gens)
            torch.cuda.synchronize()
            wall = time.perf_counter() - t1
            E, sig = stats.estimate(rec["log_wbar"].cpu().numpy(), rec["ebar"].cpu().numpy(), p=None)
            ess = rec["ess"].cpu().numpy() / walkers
            T = gens * tau
            row = dict(form=label, seed=sd, tau=tau, generations=gens, E=E, sigma=sig, wall_s=wall, c=wall / T,
                       v=sig * sig * T, moves_per_s=float(rec["n_moves"].sum()) / wall, ess_min=float(ess.min()))
            runs[label].append(row)
            if runs_out:
                with open(runs_out, "a") as f:
                    f.write(json.dumps(row) + "\n")
            g.close()
            note(f"{label} seed {sd}: E={E:.4f} +- {sig:.4f}, {wall:.1f} s")

    res = tsigma_summarize(runs)
    res.update(system=s.name, a=a, a_prime=ap, r_c=rc, walkers=walkers, generations=gens, seeds=seeds,
               first_seed=first_seed, tau=dict(pade=taus[False], neural=taus[True]), train_wall_s=t_train,
               wall_s=time.perf_counter() - t0)
    for f, q in res["against_fp64"].items():
        note(f"{f}: time-to-1mHa ratio FP64/{f} = {q['ratio']:.3f} [{q['ci95'][0]:.3f}, {q['ci95'][1]:.3f}], "
             f"dE = {1e3 * q['dE']:.2f} +- {1e3 * q['dE_sigma']:.2f} mHa")
    return {"tsigma": res}


def tsigma_summarize(runs):
    """Per form (runs: form -> list of per-run dicts with c, v, E, sigma):
    means and standard errors of c and v, time to 1 mHa = mean(c) mean(v) /
    1e-6, inverse-variance mean energy; against FP64 the time-to-1 mHa ratio
    with a 95 % interval (delta method on log c and log v), the speed and
    variance ratios and the energy difference."""
    forms = ("fp64", "mixed", "neural", "neural+mixed")

    def summary(rs):
        c = np.array([r["c"] for r in rs])
        v = np.array([r["v"] for r in rs])
        E = np.array([r["E"] for r in rs])
        sg = np.array([r["sigma"] for r in rs])
        n = len(rs)
        w = 1.0 / sg ** 2
        Em = float(np.sum(w * E) / np.sum(w))
        return dict(c=float(c.mean()), c_se=float(c.std(ddof=1) / np.sqrt(n)), v=float(v.mean()),
                    v_se=float(v.std(ddof=1) / np.sqrt(n)), time_to_1mHa_s=float(c.mean() * v.mean() / 1e-6),
                    E=Em, E_sigma=float(1.0 / np.sqrt(np.sum(w))),
                    E_scatter_chi2_dof=float(np.sum(w * (E - Em) ** 2) / max(n - 1, 1)),
                    moves_per_s=float(np.mean([r["moves_per_s"] for r in rs])),
                    ess_min=float(min(r["ess_min"] for r in rs)))

    summ = {f: summary(runs[f]) for f in forms if runs.get(f)}
    base = summ["fp64"]
    comp = {}
    for f in forms[1:]:
        if f not in summ:
            continue
        q = summ[f]
        ratio = base["time_to_1mHa_s"] / q["time_to_1mHa_s"]
        var_log = sum((x[k + "_se"] / x[k]) ** 2 for x in (base, q) for k in ("c", "v"))
        half = 1.96 * np.sqrt(var_log)
        comp[f] = dict(ratio=ratio, ci95=[ratio * float(np.exp(-half)), ratio * float(np.exp(half))],
                       speed_ratio=base["c"] / q["c"], variance_ratio=base["v"] / q["v"],
                       dE=q["E"] - base["E"], dE_sigma=float(np.hypot(q["E_sigma"], base["E_sigma"])))
        # paired by seed (same start walkers and random keys in both forms):
        # the mean over seeds of log(c v)_fp64 - log(c v)_form
        by_seed = {r["seed"]: r for r in runs["fp64"] if "seed" in r}
        d = [np.log(by_seed[r["seed"]]["c"] * by_seed[r["seed"]]["v"] / (r["c"] * r["v"]))
             for r in runs[f] if r.get("seed") in by_seed]
        if len(d) >= 2:
            m, se = float(np.mean(d)), float(np.std(d, ddof=1) / np.sqrt(len(d)))
            comp[f]["paired"] = dict(ratio=float(np.exp(m)), ci95=[float(np.exp(m - 1.96 * se)),
                                                                   float(np.exp(m + 1.96 * se))], seeds=len(d))
    return dict(forms=summ, against_fp64=comp, runs=runs)


def mfma_probe_bench(reps=10, names=("molecule", "zsweep54")):
    """The table's contraction two ways on the same walkers (the measurement
    prototype libmfma_probe.so): determinant ratios of every move of the
    fixed-axis table by the FP64 dot with Y = C Ainv and by the BF16x3
    matrix-core product Phi' = B' C followed by the FP64 dot with Ainv; both
    evaluate the basis functions with the same code.  Walkers after 20
    projection generations of the workload; kernel times by HIP events over
    `reps` launches; the BF16x3 ratios against the FP64 ones (relative to the
    walker's largest |rho_D|, and the moves whose sign changes); for context
    the projection kernel's time per table of the same population."""
    import torch
    from paper_1909_01589_amd import inputs
    from paper_1909_01589_amd import mfma_probe as mp
    from paper_1909_01589_amd.lrdmc import LRDMC, lrdmc_set_timing, lrdmc_spacing, lrdmc_timing
    rows = []
    for name in names:
        cfg = inputs.get_config(name)
        s = cfg.system
        rc, ap, _ = lrdmc_spacing(s.z_max, cfg.a)
        W = cfg.walkers
        g = LRDMC(s, cfg.a, ap, rc, cfg.tau, W, seed=cfg.seed, rotate=cfg.rotate, refresh=cfg.refresh)
        g.set_walkers(inputs.initial_walkers(s, W, cfg.seed), 0)
        g.run(10)
        lrdmc_set_timing(g.ctx, True)
        rec = g.run(10)
        proj_ms, proj_n, _, _ = lrdmc_timing(g.ctx)
        tables = W * 10 + int(rec["n_moves"].sum())
        pos = g.get_walkers()["pos"].cpu().numpy()
        g.close()
        t0 = time.perf_counter()
        probe = mp.Probe(s, pos, cfg.a, ap)
        prep_s = time.perf_counter() - t0
        ms = {}
        for v in (0, 1):
            probe.ratios(v)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(reps):
                probe.ratios(v)
            e1.record()
            torch.cuda.synchronize()
            ms[v] = e0.elapsed_time(e1) / reps
        r64 = probe.ratios(0).cpu().numpy().copy()
        r16 = probe.ratios(1).cpu().numpy().copy()
        scale = np.max(np.abs(r64), axis=1, keepdims=True)
        rel = np.abs(r16 - r64) / scale
        relm = np.abs(r16 - r64) / np.maximum(np.abs(r64), 1e-300)
        M = 12 * s.n_elec
        row = dict(workload=name, walkers=W, moves_per_table=M, basis=s.n_basis,
                   fp64_ydot_ms=ms[0], bf16x3_mfma_ms=ms[1], mfma_over_fp64=ms[1] / ms[0],
                   table_evaluations_per_s={"fp64_ydot": W / (ms[0] * 1e-3), "bf16x3_mfma": W / (ms[1] * 1e-3)},
                   projection_kernel_ms_per_table=proj_ms / tables, projection_ms_per_launch=proj_ms / max(proj_n, 1),
                   error_over_max_rho={"median": float(np.median(rel)), "p99": float(np.quantile(rel, 0.99)),
                                       "max": float(rel.max())},
                   relative_error_median=float(np.median(relm)),
                   sign_changes=int(np.sum(np.sign(r16) != np.sign(r64))), moves=int(r64.size),
                   host_prep_s=prep_s)
        print(f"[mfma-probe] {name}: FP64 Y-dot {ms[0]:.2f} ms, BF16x3 MFMA {ms[1]:.2f} ms per launch of {W} "
              f"tables; error/max|rho| median {row['error_over_max_rho']['median']:.2e}", file=sys.stderr,
              flush=True)
        rows.append(row)
        del probe
        torch.cuda.empty_cache()
    return {"mfma_probe": rows}


def sweep():
    """Throughput of every configured workload (generations, warm-up) as in
    the benchmark line: electron-moves/s, ms per generation, the kernel's
    HIP-event time and its fraction of the FP64 peak by the algorithmic count
    (which counts every move of the table, also those the large-system kernels
    skip under the small-grid drop rule)."""
    out = []
    for name, steps, warm in SWEEP:
        cfg, r = run_workload(name, steps, warm, False, 0.0)
        s = cfg.system
        row = dict(workload=name, electrons=s.n_elec, basis=s.n_basis, nuclei=int(s.n_nuc), walkers=r["walkers"],
                   a=r["a"], a_prime=r["a_prime"], generations=steps, value=r["value"],
                   ms_per_step=r["ms_per_step"], moves_per_walker_gen=r["moves_per_walker_gen"],
                   kernel_ms=r["roofline"]["avg_launch_ms"], achieved_tflops=r["roofline"]["achieved"],
                   frac=r["roofline"]["frac"], ess_fraction=r["ess_fraction"])
        print(f"[sweep] {name}: {r['value'] / 1e6:.2f} M electron-moves/s, frac {row['frac']:.3f}",
              file=sys.stderr, flush=True)
        out.append(row)
    return {"sweep": out}


def copy_probe():
    """A plain device copy of 512 MiB: the reference for scaling the HBM byte
    counters (FETCH_SIZE, WRITE_SIZE) of a profiled run."""
    import torch
    n = 64 * 1024 * 1024
    x = torch.ones(n, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": n * 8}), flush=True)


def cpu_baseline(system, a, ap, rc, tau, seed, pos, gen0, seconds, threads=None):
    """The CPU oracle, as it stands, on a bounded sample of the workload:
    chunks of 64 walkers of the equilibrated population, one generation each,
    until `seconds` of wall time have passed, on `threads` host threads (all
    by default: OMP_NUM_THREADS, else the CPU count)."""
    import oracle
    oracle.build(force=False)
    if threads is None:
        threads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or os.cpu_count()
    o = oracle.Oracle(system, a, ap, rc, tau=tau, seed=seed)
    W = pos.shape[0]
    moves, chunks = 0, 0
    t0 = time.perf_counter()
    while True:
        lo = (chunks * 64) % W
        r = o.run(pos[lo:lo + 64], 1, gen0=gen0 + chunks, want_idx=False, nthreads=threads)
        moves += int(r["n_moves"].sum())
        chunks += 1
        if time.perf_counter() - t0 >= seconds:
            break
    dt = time.perf_counter() - t0
    return {"value": moves / dt, "unit": "electron-moves/s", "cores": threads, "kind": "oracle",
            "sample": f"{chunks} x (64 walkers x 1 generation) of the equilibrated population, "
                      f"{moves} moves in {dt:.1f} s"}


def population_scan(name, walker_counts, steps, warmup, gens=20):
    """Throughput of one workload (its system, spacing and tau) against the
    number of walkers.  A generation ends with its slowest walker, and the
    number of moves of a walker in a generation is Poisson-like, so with few
    walkers per resident workgroup slot the end of the launch runs on a part
    of the machine; the scan shows how much of the kernel's rate that costs.
    Also reports the variance-to-mean ratio of the moves per walker and
    generation at the workload's own walker count, and the correlation of a
    walker's count with its parent's in the generation before (None where
    every walker descends from one parent)."""
    import torch
    from paper_1909_01589_amd import inputs
    from paper_1909_01589_amd.lrdmc import LRDMC, lrdmc_spacing
    rows = []
    for W in walker_counts:
        _, r = run_workload(name, steps, warmup, False, 0.0, walkers=W)
        rows.append(dict(walkers=W, value=r["value"], ms_per_step=r["ms_per_step"],
                         kernel_ms=r["roofline"]["avg_launch_ms"], achieved=r["roofline"]["achieved"],
                         frac=r["roofline"]["frac"], kernel=r["roofline"]["kernel"],
                         moves_per_walker_gen=r["moves_per_walker_gen"]))
        print(f"[population] {name} W={W}: {r['value'] / 1e6:.2f} M electron-moves/s, "
              f"kernel {r['roofline']['avg_launch_ms']:.4f} ms, frac {r['roofline']['frac']:.3f}",
              file=sys.stderr, flush=True)
    cfg = inputs.get_config(name)
    s = cfg.system
    rc, ap, _ = lrdmc_spacing(s.z_max, cfg.a)
    gpu = LRDMC(s, cfg.a, ap, rc, cfg.tau, cfg.walkers, seed=cfg.seed, rotate=cfg.rotate, refresh=cfg.refresh)
    gpu.set_walkers(inputs.initial_walkers(s, cfg.walkers, cfg.seed), 0)
    if warmup:
        gpu.run(warmup)
    disp, mx, corr, prev = [], [], [], None
    for _ in range(gens):
        gpu.project()
        nm = gpu.get_walkers()["n_moves"].cpu().numpy().astype(float)
        disp.append(nm.var() / nm.mean())
        mx.append(nm.max() / nm.mean())
        if prev is not None and prev.std() > 0:
            corr.append(float(np.corrcoef(nm, prev)[0, 1]))
        idx = gpu.branch()["idx"].cpu().numpy()
        prev = nm[idx]   # the parent's count, per slot of the next generation
    torch.cuda.synchronize()
    gpu.close()
    return {"population_scan": {"workload": name, "default_walkers": cfg.walkers, "steps": steps, "warmup": warmup,
                                "rows": rows, "moves_var_over_mean": float(np.mean(disp)),
                                "moves_max_over_mean": float(np.mean(mx)), "generations_sampled": gens,
                                "parent_child_moves_corr": float(np.mean(corr)) if corr else None,
                                "generations_with_distinct_parents": len(corr)}}


def run_workload(name, steps, warmup, want_cpu, cpu_seconds, precision=0, generic=0, walkers=None):
    import torch
    from paper_1909_01589_amd import inputs, stats, workcount
    from paper_1909_01589_amd.lrdmc import (LRDMC, lrdmc_is_specialized, lrdmc_set_precision, lrdmc_set_timing,
                                            lrdmc_spacing, lrdmc_timing, lrdmc_use_generic)

    cfg = inputs.get_config(name, walkers=walkers) if walkers else inputs.get_config(name)
    s = cfg.system
    rc, ap, nc = lrdmc_spacing(s.z_max, cfg.a)
    W = cfg.walkers
    gpu = LRDMC(s, cfg.a, ap, rc, cfg.tau, W, seed=cfg.seed, rotate=cfg.rotate, refresh=cfg.refresh)
    lrdmc_set_precision(gpu.ctx, precision)
    lrdmc_use_generic(gpu.ctx, generic)
    kernel = "project_kernel_fixed" if lrdmc_is_specialized(gpu.ctx) else "project_kernel"
    gpu.set_walkers(inputs.initial_walkers(s, W, cfg.seed), 0)
    if warmup:
        gpu.run(warmup)
    torch.cuda.synchronize()
    lrdmc_set_timing(gpu.ctx, True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = gpu.run(steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    proj_ms, proj_n, br_ms, br_n = lrdmc_timing(gpu.ctx)
    lrdmc_set_timing(gpu.ctx, False)
    wall = t1 - t0
    n_moves = out["n_moves"].cpu().numpy()
    moves = int(n_moves.sum())
    lwb = out["log_wbar"].cpu().numpy()
    eb = out["ebar"].cpu().numpy()
    ess = out["ess"].cpu().numpy() / W
    E, sig = stats.estimate(lwb, eb, p=None)

    shp = workcount.shape_of(s)
    # generation starts: every walker on refresh generations (multiples of
    # `refresh`, counted from the first generation after set_walkers)
    R = max(1, int(cfg.refresh))
    n_refresh = sum(1 for gen in range(warmup, warmup + steps) if R == 1 or gen % R == 0)
    ops = workcount.projection_ops(shp, W * steps, moves, W * n_refresh) if proj_n else 0.0
    avg_ms = proj_ms / max(proj_n, 1)
    ops_per_launch = ops / max(proj_n, 1)
    achieved = ops_per_launch / (avg_ms * 1e-3) / 1e12 if proj_n else 0.0
    traffic = _traffic_record(name)
    res = {
        "value": moves / wall, "ms_per_step": 1e3 * wall / steps, "moves": moves, "wall_s": wall,
        "moves_per_walker_gen": moves / (W * steps),
        "projection_time_per_s": W * cfg.tau * steps / wall,
        "E_Ha": E, "sigma_E_Ha": sig,
        "ess_fraction": {"median": float(np.median(ess)), "min": float(ess.min())},
        "time_to_sigma_1mHa_s": wall * (sig / 1e-3) ** 2 if np.isfinite(sig) else None,
        "a": cfg.a, "a_prime": ap, "r_c": rc, "n_core": nc, "tau": cfg.tau, "walkers": W,
        "refresh": cfg.refresh,
        "roofline": {"bound": "alu", "achieved": achieved, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / FP64_PEAK_TFLOPS, "traffic": traffic,
                     "kernel": kernel, "avg_launch_ms": avg_ms,
                     "ops_per_launch": ops_per_launch,
                     "reconfigure_avg_ms": br_ms / max(br_n, 1)},
    }
    if want_cpu:
        pos = gpu.get_walkers()["pos"].cpu().numpy()
        res["cpu_baseline"] = cpu_baseline(s, cfg.a, ap, rc, cfg.tau, cfg.seed, pos, 10_000_000, cpu_seconds)
        one = cpu_baseline(s, cfg.a, ap, rc, cfg.tau, cfg.seed, pos, 10_000_000, cpu_seconds / 2, threads=1)
        res["cpu_baseline"]["single_core"] = {"value": one["value"], "sample": one["sample"]}
    gpu.close()
    return cfg, res


WORKLOAD_TEXT = {
    "molecule": "synthetic molecule: 4 nuclei Z=8 + 8 nuclei Z=1 at seeded positions (min separation 1.8 bohr), "
                "20 up / 20 down electrons, K={K} even-tempered s/p/d Gaussians 0.05*2.5^k, seeded orthonormal MOs, "
                "Pade Jastrow b=1, a={a:.5f} bohr, a'={ap:.5f}, r_c={rc:.5f} (R_c over the Z=8 nuclei), "
                "{W} walkers, tau={tau} per generation, FP64",
    "ar_a0.1": "Ar-like atom Z=18 (9 up, 9 down), K={K} even-tempered s/p/d Gaussians 0.05*2.5^k, seeded "
               "orthonormal MOs, Pade Jastrow b=1, a={a} bohr, a'={ap:.5f}, r_c={rc:.5f}, {W} walkers, "
               "tau={tau} per generation, FP64",
}


def _describe(cfg, res):
    t = WORKLOAD_TEXT.get(cfg.name, cfg.name + ": a={a} bohr, a'={ap:.5f}, {W} walkers, tau={tau}")
    return cfg.name + ": " + t.format(K=cfg.system.n_basis, a=cfg.a, ap=res["a_prime"], rc=res["r_c"],
                                      W=cfg.walkers, tau=cfg.tau)


def _mixed_bound(system) -> float:
    """The derived bound on the mixed-precision ratios: exp(dJ) - 1 with
    dJ = 2^-20 (sum_j c_ij / b_ee + sum_I Z_I / b_en) for the electron with the
    largest sum (cusp coefficients 1/2 and 1/4)."""
    s = system
    worst = 0.0
    for up in (True, False):
        same, other = (s.n_up, s.n_dn) if up else (s.n_dn, s.n_up)
        if same == 0:
            continue
        ee = (0.25 * (same - 1) + 0.5 * other) / s.b_ee
        en = float(np.sum(s.Z)) / s.b_en
        worst = max(worst, ee + en)
    return float(np.expm1(2.0 ** -20 * worst))


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=300, help="timed generations")
    ap.add_argument("--warmup", type=int, default=50, help="untimed generations before timing")
    ap.add_argument("--workload", default="molecule")
    ap.add_argument("--second", default="ar_a0.1", help="second workload line ('' to skip)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true", help="skip the mixed-precision line of the benchmark")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a 512 MiB device copy (counter calibration) and exit")
    ap.add_argument("--source-hash", action="store_true", help="print the kernel source hash and exit")
    ap.add_argument("--jastrow-grad", action="store_true",
                    help="only time the Jastrow-parameter gradient kernel and exit")
    ap.add_argument("--neural", choices=["ar", "he"], default=None,
                    help="only run the learned-Jastrow comparison (VMC, training, LRDMC scan) and exit")
    ap.add_argument("--neural-gens", type=int, default=1200, help="timed generations per spacing for --neural")
    ap.add_argument("--neural-spacings", type=float, nargs="+", default=None, help="spacings for --neural")
    ap.add_argument("--neural-forms", nargs="+", default=["pade", "neural"], choices=["pade", "neural"],
                    help="trial functions for --neural")
    ap.add_argument("--neural-gens-inverse-a", action="store_true",
                    help="--neural: --neural-gens at the largest spacing, scaled as 1/a at the others")
    ap.add_argument("--neural-equil", type=float, default=None,
                    help="--neural: projection time (Ha^-1) discarded before each timed run")
    ap.add_argument("--neural-time", type=float, default=None,
                    help="--neural: projection time (Ha^-1) of every timed run (instead of generations)")
    ap.add_argument("--neural-summary", nargs="+", default=None, metavar="FILE",
                    help="fit the per-run lines of --neural --runs-out files (no GPU) and exit")
    ap.add_argument("--sweep", action="store_true",
                    help="only time every configured workload (Be-like, Ar-like, Z-sweep, molecule) and exit")
    ap.add_argument("--mixed-molecule", action="store_true",
                    help="FP64 against the mixed-precision table on the benchmark molecule: energies (JSON on stdout)")
    ap.add_argument("--mixed", action="store_true",
                    help="FP64 against the mixed-precision move table: throughput, energies, time to 1 mHa")
    ap.add_argument("--zscan-phys", action="store_true",
                    help="only run the single/double-grid comparison for Ne and Ar with screened orbitals and exit")
    ap.add_argument("--zscan", action="store_true",
                    help="only run the single/double-grid cost scan over Z = 10, 18, 36, 54 and exit")
    ap.add_argument("--population", type=int, nargs="+", default=None, metavar="W",
                    help="throughput of --workload at these walker counts (JSON on stdout)")
    ap.add_argument("--ascan", action="store_true",
                    help="only run the spacing scan on helium for the three lattice schemes and exit")
    ap.add_argument("--tsigma", action="store_true",
                    help="only measure the time to sigma(E) = 1 mHa of FP64, mixed, neural and neural+mixed over "
                         "independent seeds on screened Ar and exit")
    ap.add_argument("--seeds", type=int, default=8, help="independent runs per form for --tsigma")
    ap.add_argument("--first-seed", type=int, default=0, help="first seed index for --tsigma")
    ap.add_argument("--tsigma-gens", type=int, default=1000, help="generations per --tsigma run")
    ap.add_argument("--runs-out", default=None, help="--tsigma: append one JSON line per run to this file")
    ap.add_argument("--tsigma-summary", nargs="+", default=None, metavar="FILE",
                    help="combine the per-run lines of --tsigma --runs-out files (no GPU) and exit")
    ap.add_argument("--mfma-probe", action="store_true",
                    help="only time the table's contraction as FP64 Y-dot and as BF16x3 MFMA (prototype) and exit")
    args = ap.parse_args()
    if args.source_hash:
        print(kernel_source_hash())
        return
    if args.neural_summary:
        rows = [json.loads(line) for path in args.neural_summary for line in open(path) if line.strip()]
        print(json.dumps({"neural": neural_summarize(rows)}), flush=True)
        return
    if args.tsigma_summary:
        runs = {}
        for path in args.tsigma_summary:
            for line in open(path):
                if line.strip():
                    r = json.loads(line)
                    runs.setdefault(r["form"], []).append(r)
        print(json.dumps({"tsigma": tsigma_summarize(runs)}), flush=True)
        return

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: runs on exactly one GPU; --gpus must be 1 "
              "(the walker population is not sharded over several GPUs)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(1)
    if args.copy_probe:
        copy_probe()
        return
    if args.ascan:
        print(json.dumps(ascan()), flush=True)
        return
    if args.population:
        print(json.dumps(population_scan(args.workload, args.population, args.steps, args.warmup)), flush=True)
        return
    if args.tsigma:
        print(json.dumps(tsigma_bench(seeds=args.seeds, first_seed=args.first_seed, gens=args.tsigma_gens,
                                      runs_out=args.runs_out)), flush=True)
        return
    if args.mfma_probe:
        print(json.dumps(mfma_probe_bench()), flush=True)
        return
    if args.sweep:
        print(json.dumps(sweep()), flush=True)
        return
    if args.mixed:
        print(json.dumps(mixed_bench()), flush=True)
        return
    if args.mixed_molecule:
        print(json.dumps(mixed_molecule()), flush=True)
        return
    if args.zscan_phys:
        print(json.dumps(zscan_phys()), flush=True)
        return
    if args.zscan:
        print(json.dumps(zscan()), flush=True)
        return
    if args.neural:
        print(json.dumps(neural_bench(args.neural, gens=args.neural_gens, spacings=args.neural_spacings,
                                      forms=tuple(args.neural_forms), gens_inverse_a=args.neural_gens_inverse_a,
                                      runs_out=args.runs_out, t_equil=args.neural_equil,
                                      t_prod=args.neural_time)), flush=True)
        return
    if args.jastrow_grad:
        print(json.dumps(jastrow_grad_bench()), flush=True)
        return

    cfg, main_res = run_workload(args.workload, args.steps, args.warmup, not args.no_cpu_baseline,
                                 args.cpu_seconds)
    print(f"[bench] {args.workload}: {main_res['value'] / 1e6:.2f} M electron-moves/s", file=sys.stderr, flush=True)
    mixed = None
    if not args.no_mixed:
        _, mixed = run_workload(args.workload, args.steps, args.warmup, False, 0.0, precision=1)
    second = second_gen = None
    if args.second:
        cfg2, second = run_workload(args.second, args.steps, args.warmup, False, 0.0)
        _, second_gen = run_workload(args.second, args.steps, args.warmup, False, 0.0, generic=1)

    s = cfg.system
    line = {
        "metric": METRIC, "value": main_res["value"], "unit": "electron-moves/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": main_res["ms_per_step"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {
            "workload": _describe(cfg, main_res),
            "walkers": cfg.walkers, "electrons": s.n_elec, "basis": s.n_basis, "nuclei": int(s.n_nuc),
            "a": cfg.a, "a_prime": main_res["a_prime"], "r_c": main_res["r_c"], "tau": cfg.tau,
            "refresh": cfg.refresh,
        },
        "roofline": main_res["roofline"],
        "moves_per_walker_gen": main_res["moves_per_walker_gen"],
        "projection_time_per_s": main_res["projection_time_per_s"],
        "E_Ha": main_res["E_Ha"], "sigma_E_Ha": main_res["sigma_E_Ha"],
        "time_to_sigma_1mHa_s": main_res["time_to_sigma_1mHa_s"],
        "ess_fraction": main_res["ess_fraction"],
        "energy_note": "seeded random MOs: a throughput workload whose nodes are not physical; E_Ha and its "
                       "sigma only record the run (physical energies and times to 1 mHa: --ascan, --zscan-phys, "
                       "--neural, --mixed)",
    }
    if "cpu_baseline" in main_res:
        line["cpu_baseline"] = main_res["cpu_baseline"]
    if mixed is not None:
        line["mixed_precision_table"] = {
            "value": mixed["value"], "ms_per_step": mixed["ms_per_step"], "dtype": "f64 with f32 Jastrow estimates",
            "speedup": mixed["value"] / main_res["value"],
            "note": f"lrdmc_set_precision 1: same workload and steps; ratios within a derived "
                    f"{_mixed_bound(s):.2g} of FP64"}
    if second is not None:
        line["second_workload"] = {
            "workload": _describe(cfg2, second), "value": second["value"], "ms_per_step": second["ms_per_step"],
            "kernel": second["roofline"]["kernel"], "roofline_frac": second["roofline"]["frac"],
            "avg_launch_ms": second["roofline"]["avg_launch_ms"],
            "moves_per_walker_gen": second["moves_per_walker_gen"],
            "general_kernel": {"value": second_gen["value"], "ms_per_step": second_gen["ms_per_step"],
                               "roofline_frac": second_gen["roofline"]["frac"],
                               "avg_launch_ms": second_gen["roofline"]["avg_launch_ms"]},
        }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()

"""The mixed-precision move table (lrdmc_set_precision(ctx, 1)): the Jastrow
pair terms of the ratios take 1/r and 1/(1/r + b) from FP32 hardware
estimates; everything else stays FP64.

Bound on the ratios, derived from the arithmetic: each pair term
u = c / (1/r + b) gets a relative error of at most about 3 * 2^-22 (two FP32
estimates and the FP32 rounding of the denominators and their product), and
|u| < |c| / b, so the Jastrow exponent of a displaced configuration is off by
at most dJ = 2^-20 * (sum_j |c_ij| / b_ee + sum_I Z_I / b_en), and the ratio
by the factor exp(dJ); with the learned correction, F is evaluated at an r
carried by the FP32 1/r, which adds |F'| r 2^-22 per pair term.  The test
adds the FP64 bar of the main parity tests.
Move indices then follow the FP64 path until such a difference decides one,
so runs are compared statistically, on helium (fixed node exact)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from oracle import spacing  # noqa: E402
from paper_1909_01589_amd import inputs  # noqa: E402

HE_EXACT = -2.903724


def _jastrow_bound(s):
    N, nu = s.n_elec, s.n_up
    worst = 0.0
    for i in range(N):
        c = sum((0.25 if (j < nu) == (i < nu) else 0.5) for j in range(N) if j != i)
        worst = max(worst, c / s.b_ee + float(np.sum(s.Z)) / s.b_en)
    return 2.0 ** -20 * worst


@pytest.mark.parametrize("name", ["be", "ar"])
@pytest.mark.parametrize("generic", [0, 1])
@pytest.mark.parametrize("table", [False, True])
def test_mixed_ratios_within_the_derived_bound(name, generic, table):
    from paper_1909_01589_amd.lrdmc import LRDMC, lrdmc_is_specialized, lrdmc_set_precision, lrdmc_use_generic
    s, a, tau = (inputs.be_like(0), 0.2, 0.0161) if name == "be" else (inputs.ar_like(0), 0.1, 0.00318)
    rc, ap, _ = spacing.spacing(s.z_max, a)
    W, rcut = 16, 5.0
    tab = inputs.jastrow_table(seed=5, n_nodes=257, r_cut=rcut, scale=0.3) if table else None
    pos = inputs.initial_walkers(s, W, 7)
    out = {}
    for mode in (0, 1):
        gpu = LRDMC(s, a, ap, rc, tau, W, seed=3, rotate=1, refresh=8)
        if table:
            gpu.set_jastrow_table(tab, rcut)
        lrdmc_use_generic(gpu.ctx, generic)
        lrdmc_set_precision(gpu.ctx, mode)
        assert lrdmc_is_specialized(gpu.ctx) == (generic == 0)
        out[mode] = [x.cpu().numpy() for x in gpu.eval_moves(pos)]
        gpu.close()
    orc = oracle.Oracle(s, a, ap, rc, tau=tau, seed=3, rotate=1, ftab=tab, ftab_rcut=rcut)
    dJ = _jastrow_bound(s)
    if table:
        # the correction is evaluated at r = d^2 * (1/r) with the FP32 1/r:
        # |dF| <= |F'| r 2^-22 per term, r < r_cut, nucleus terms scaled by Z
        dJ += 2.0 ** -21 * rcut * float(np.abs(tab[:, :, 1]).max()) * (s.n_elec + float(np.sum(s.Z)))
    rho_m, k_m, diag_m = out[1]
    worst = 0.0
    for w in range(W):
        print(f"mixed precision case={name} generic={generic} table={table} walker={w}", flush=True)
        r_o, k_o, d_o = orc.eval_moves(pos[w], orc.move_rotation(w, 0, 0))
        scale = np.max(np.abs(r_o))
        err = np.abs(rho_m[w] - r_o)
        assert np.all(err <= 1e-9 * (np.abs(r_o) + scale) + np.expm1(dJ) * np.abs(r_o))
        worst = max(worst, float(np.max(err / (np.abs(r_o) + 1e-300 + 1e-9 * scale))))
        assert np.allclose(k_m[w], k_o, rtol=1e-12, atol=0)
        assert abs(diag_m[w, 6] - d_o["delta"]) <= (1e-9 + np.expm1(dJ)) * d_o["delta"]
    # the local energy does not use the table's ratios: identical to FP64
    assert np.array_equal(out[0][2][:, 0], diag_m[:, 0])
    assert np.array_equal(out[0][2][:, 3], diag_m[:, 3])
    print(f"largest relative ratio error {worst:.2e} (bound {np.expm1(dJ):.2e})", flush=True)


def test_mixed_projection_energies_agree_with_fp64():
    """Helium with a nodeless orbital at a = 0.1 (fixed node exact), 8192
    walkers: the FP64 and the mixed-precision projection from the same start
    give the same energy within error bars, both at the exact value within
    the lattice bias of this spacing."""
    from paper_1909_01589_amd import stats
    from paper_1909_01589_amd.lrdmc import LRDMC, lrdmc_set_precision, lrdmc_spacing
    s = inputs.helium_nodeless()
    W, a = 8192, 0.1
    rc, ap, _ = lrdmc_spacing(s.z_max, a)
    ap = max(ap, a)
    g = LRDMC(s, a, ap, rc, 1.0, W, seed=21, rotate=1)
    g.set_walkers(inputs.initial_walkers(s, W, 0), 0)
    g.vmc(2000, 0.6)
    pos = g.get_walkers()["pos"].clone()
    delta = float(g.eval_moves(pos)[2][:, 6].mean())
    g.close()
    tau = 20.0 * s.n_elec / delta
    res = {}
    for mode in (0, 1):
        g = LRDMC(s, a, ap, rc, tau, W, seed=21, rotate=1, refresh=8)
        lrdmc_set_precision(g.ctx, mode)
        g.set_walkers(pos, 0)
        g.run(int(10.0 / tau))
        out = g.run(1500)
        res[mode] = stats.estimate(out["log_wbar"].cpu().numpy(), out["ebar"].cpu().numpy(), p=None)
        g.close()
    (e0, s0), (e1, s1) = res[0], res[1]
    print(f"FP64 {e0:.6f} +- {s0:.6f}; mixed {e1:.6f} +- {s1:.6f}", flush=True)
    assert abs(e1 - e0) < 3.5 * np.hypot(s0, s1)
    for e, sg in ((e0, s0), (e1, s1)):
        assert abs(e - HE_EXACT) < 4.0 * sg + 1e-3


@pytest.mark.parametrize("name,W", [("zsweep54", 2), ("molecule", 2)])
def test_mixed_ratios_large_systems(name, W):
    """The same bound for the kernels with the orbital-projected inverse in
    device memory: the Z = 54 atom and the molecule (twelve nuclei, each
    electron-nucleus term in the two-point form of the shared reciprocal)."""
    from paper_1909_01589_amd.lrdmc import LRDMC, lrdmc_set_precision
    cfg = inputs.get_config(name)
    s = cfg.system
    rc, ap, _ = spacing.spacing(s.z_max, cfg.a)
    gpu = LRDMC(s, cfg.a, ap, rc, cfg.tau, W, seed=4, rotate=1, refresh=8)
    lrdmc_set_precision(gpu.ctx, 1)
    pos = inputs.initial_walkers(s, W, 5)
    rho, k, diag = (x.cpu().numpy() for x in gpu.eval_moves(pos))
    gpu.close()
    orc = oracle.Oracle(s, cfg.a, ap, rc, tau=cfg.tau, seed=4, rotate=1)
    dJ = _jastrow_bound(s)
    for w in range(W):
        print(f"mixed precision large case={name} walker={w}", flush=True)
        r_o, k_o, d_o = orc.eval_moves(pos[w], orc.move_rotation(w, 0, 0))
        scale = np.max(np.abs(r_o))
        assert np.all(np.abs(rho[w] - r_o) <= 1e-9 * (np.abs(r_o) + scale) + np.expm1(dJ) * np.abs(r_o))
        assert abs(diag[w, 0] - d_o["e_l"]) <= 1e-9 * (1 + abs(d_o["e_l"]) + abs(d_o["lap_exact"]))


@pytest.mark.parametrize("name,W,generic", [("ar_a0.1", 64, 0), ("ar_a0.1", 32, 1), ("zsweep54", 24, 0),
                                            ("molecule", 16, 0)])
def test_mixed_projection_against_the_oracle(name, W, generic):
    """One generation of the mixed-precision projection kernels against the
    FP64 oracle, slot by slot: the fixed-size kernel of the Ar-like atom
    (generic 0) and the general one, the Z = 54 atom (compacted table,
    inverse in device memory) and the molecule.  A move index may differ from
    the oracle's only where the oracle's decision margin is within the
    derived ratio bound eta (the relative change of the rates that the FP32
    estimates can cause: 2 eta for a heat-bath choice; a move-or-stay
    comparison also carries the perturbations of the generation's earlier
    holding times, at most eta tau against tau_d, so the bar is 20 eta for
    about twenty moves per generation); elsewhere the walker follows the
    oracle exactly:
    same moves, positions to 1e-11, E_L to the FP64 bar (the local energy
    does not use the table), log w to the FP64 bar plus the rate bound times
    |log w| (each holding time tau_d = -ln u / Delta moves by at most that
    relative amount)."""
    from paper_1909_01589_amd.lrdmc import LRDMC, lrdmc_is_specialized, lrdmc_set_precision, lrdmc_use_generic
    cfg = inputs.get_config(name)
    s = cfg.system
    rc, ap, _ = spacing.spacing(s.z_max, cfg.a)
    gpu = LRDMC(s, cfg.a, ap, rc, cfg.tau, W, seed=6, rotate=1, refresh=8)
    lrdmc_use_generic(gpu.ctx, generic)
    lrdmc_set_precision(gpu.ctx, 1)
    if name == "ar_a0.1":
        assert lrdmc_is_specialized(gpu.ctx) == (generic == 0)
    pos = inputs.initial_walkers(s, W, 8)
    gpu.set_walkers(pos, 0)
    gpu.project()
    out = {k: v.cpu().numpy() for k, v in gpu.get_walkers().items()}
    gpu.close()
    orc = oracle.Oracle(s, cfg.a, ap, rc, tau=cfg.tau, seed=6, rotate=1)
    ref = orc.generations(pos, 0)
    eta = float(np.expm1(_jastrow_bound(s)))
    differ = 0
    for w in range(W):
        same = (out["n_moves"][w] == ref["n_moves"][w]
                and np.allclose(out["pos"][w], ref["pos"][w], rtol=0, atol=1e-11))
        if not same:
            assert ref["margin"][w] < 20.0 * eta, (w, ref["margin"][w], eta)
            differ += 1
            continue
        el_o, lw_o = ref["e_l"][w], ref["log_w"][w]
        assert np.isfinite(out["e_l"][w]) and np.isfinite(out["log_w"][w])
        assert abs(out["e_l"][w] - el_o) <= 1e-9 * (1 + abs(el_o))
        assert abs(out["log_w"][w] - lw_o) <= 1e-9 * (1 + abs(lw_o)) + 2.0 * eta * abs(lw_o)
    print(f"mixed projection {name} generic={generic}: {differ} of {W} slots took another move "
          f"(oracle margin < {20 * eta:.1e}); {ref['n_moves'].sum()} moves", flush=True)
    assert differ <= W // 8

"""The general kernels with the orbital-projected inverse Y in the walker's
device-memory state (chosen automatically for large systems, forced here on
small ones with lrdmc_use_generic(ctx, 2)) against the oracle: move tables,
whole runs resuming the stored state, a switch between the two placements
inside a run, the Metropolis sampler, the gradient kernels and the learned
correction.  Bars as in the main parity tests."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from parity_bars import check, record_bar, run_agrees  # noqa: E402
from oracle import spacing  # noqa: E402
from paper_1909_01589_amd import inputs  # noqa: E402


def _system(name):
    return {"be": (inputs.be_like(0), 0.2, 0.0161), "ar": (inputs.ar_like(0), 0.1, 0.00318),
            "tiny": (inputs.tiny_mixed(seed=1, n_up=3, n_dn=2), 0.06, 0.02)}[name]


def _pair(name, W, seed=3, refresh=1, tab=None):
    from paper_1909_01589_amd.lrdmc import LRDMC, lrdmc_use_generic
    s, a, tau = _system(name)
    rc, ap, _ = spacing.spacing(s.z_max, a)
    gpu = LRDMC(s, a, ap, rc, tau, W, seed=seed, rotate=1, refresh=refresh)
    lrdmc_use_generic(gpu.ctx, 2)
    if tab is not None:
        gpu.set_jastrow_table(tab, 4.0)
    orc = oracle.Oracle(s, a, ap, rc, tau=tau, seed=seed, rotate=1, ftab=tab, ftab_rcut=4.0)
    return s, gpu, orc


@pytest.mark.parametrize("name,W", [("be", 8), ("tiny", 6), ("ar", 4)])
def test_eval_moves_y_in_hbm(name, W):
    s, gpu, orc = _pair(name, W)
    pos = inputs.initial_walkers(s, W, 7)
    rho, k, diag = (x.cpu().numpy() for x in gpu.eval_moves(pos))
    for w in range(W):
        r_o, k_o, d_o = orc.eval_moves(pos[w], orc.move_rotation(w, 0, 0))
        assert np.all(np.abs(rho[w] - r_o) <= 1e-9 * (np.abs(r_o) + np.max(np.abs(r_o))))
        assert abs(diag[w, 0] - d_o["e_l"]) <= 1e-9 * (1 + abs(d_o["e_l"]) + abs(d_o["lap_exact"]))
    gpu.close()


@pytest.mark.parametrize("name,W,n_gen,refresh,table", [("be", 64, 5, 4, False), ("tiny", 32, 4, 3, True),
                                                        ("ar", 16, 3, 2, False), ("ar", 16, 3, 1, True)])
def test_run_y_in_hbm(name, W, n_gen, refresh, table):
    tab = inputs.jastrow_table(seed=2, n_nodes=65, r_cut=4.0, scale=0.3) if table else None
    s, gpu, orc = _pair(name, W, seed=9, refresh=refresh, tab=tab)
    pos = inputs.initial_walkers(s, W, 2)
    gpu.set_walkers(pos, 0)
    out = gpu.run(n_gen, want_idx=True)
    ref = orc.run(pos, n_gen, gen0=0)
    print(f"y-hbm run case={name} refresh={refresh} table={table}", flush=True)
    n = run_agrees(f"y-hbm run {name} refresh {refresh} table {table}", out["n_moves"].cpu().numpy(),
                   out["idx"].cpu().numpy(), ref)
    eb = out["ebar"].cpu().numpy()
    check(f"y-hbm run ebar ({name})", eb[:n], ref["ebar"][:n], record_bar(ref["ebar"][:n]),
          scale=np.abs(ref["ebar"][:n]))
    if n == n_gen:
        check(f"y-hbm run final positions ({name})", gpu.get_walkers()["pos"].cpu().numpy(), ref["pos"], 1e-10)
    gpu.close()


def test_switching_placement_inside_a_run():
    """Two generations with Y in LDS (fixed-size kernel), two with Y in
    device memory resuming the stored state, two back in LDS: the same
    records as the oracle's uninterrupted run."""
    from paper_1909_01589_amd.lrdmc import LRDMC, lrdmc_is_specialized, lrdmc_use_generic
    s, a, tau = _system("be")
    rc, ap, _ = spacing.spacing(s.z_max, a)
    W = 64
    gpu = LRDMC(s, a, ap, rc, tau, W, seed=5, rotate=1, refresh=8)
    orc = oracle.Oracle(s, a, ap, rc, tau=tau, seed=5, rotate=1)
    pos = inputs.initial_walkers(s, W, 3)
    gpu.set_walkers(pos, 0)
    idx, eb, nm = [], [], []
    for mode in (0, 2, 0):
        lrdmc_use_generic(gpu.ctx, mode)
        assert lrdmc_is_specialized(gpu.ctx) == (mode == 0)
        out = gpu.run(2, want_idx=True)
        idx.append(out["idx"].cpu().numpy())
        eb.append(out["ebar"].cpu().numpy())
        nm.append(out["n_moves"].cpu().numpy())
    ref = orc.run(pos, 6, gen0=0)
    n = run_agrees("y-hbm placement switch", np.concatenate(nm), np.concatenate(idx), ref)
    check("y-hbm placement switch ebar", np.concatenate(eb)[:n], ref["ebar"][:n],
          record_bar(ref["ebar"][:n]), scale=np.abs(ref["ebar"][:n]))
    gpu.close()


def test_vmc_and_gradients_y_in_hbm():
    tab = inputs.jastrow_table(seed=3, n_nodes=33, r_cut=4.0, scale=0.3)
    s, gpu, orc = _pair("tiny", 6, seed=4, tab=tab)
    pos = inputs.initial_walkers(s, 6, 5)
    gpu.set_walkers(pos, 0)
    gpu.vmc(40, 0.3)
    out = {k: v.cpu().numpy() for k, v in gpu.get_walkers().items()}
    for w in range(6):
        p, acc, el = orc.vmc(pos[w], w, 0, 40, 0.3)
        assert out["n_moves"][w] == acc
        assert np.allclose(out["pos"][w], p, rtol=0, atol=1e-10)
    g = gpu.jastrow_grad(pos).cpu().numpy()
    for w in range(6):
        e_o = orc.local_energy(pos[w])[0]
        assert abs(g[w, 0] - e_o) <= 1e-9 * (1 + abs(e_o))
        assert abs(g[w, 1] - orc.jastrow(pos[w])) <= 1e-11 * (1 + abs(g[w, 1]))
    gt = gpu.jastrow_table_grad(pos, np.ones(6), np.ones(6)).cpu().numpy()
    from paper_1909_01589_amd.lrdmc import lrdmc_use_generic
    lrdmc_use_generic(gpu.ctx, 1)
    gt_lds = gpu.jastrow_table_grad(pos, np.ones(6), np.ones(6)).cpu().numpy()
    assert np.allclose(gt, gt_lds, rtol=1e-12, atol=1e-12 * np.abs(gt).max())
    gpu.close()


def test_mode_errors():
    from paper_1909_01589_amd.lrdmc import LRDMC, LRDMCError, lrdmc_use_generic
    s, a, tau = _system("be")
    gpu = LRDMC(s, a, 0.3, 0.4, tau, 4, seed=1)
    for bad in (-1, 3):
        with pytest.raises(LRDMCError, match="EINVAL"):
            lrdmc_use_generic(gpu.ctx, bad)
    gpu.close()


def test_compacted_table_run():
    """44 electrons (264 move pairs > 256 threads): the table runs compacted,
    with the small-grid moves of valence electrons dropped (p < 2^-52); three
    generations against the oracle, indices bit-exact."""
    from paper_1909_01589_amd.lrdmc import LRDMC, lrdmc_use_generic
    s = inputs.atom(44, (12, 10, 2), 0.08, 2.0, seed=0)   # Slater matrices well conditioned
    a = 1.0 / (3.5 * 44)
    rc, ap, _ = spacing.spacing(44.0, a)
    W, tau = 8, 4e-5
    gpu = LRDMC(s, a, ap, rc, tau, W, seed=6, rotate=1, refresh=2)
    lrdmc_use_generic(gpu.ctx, 2)
    orc = oracle.Oracle(s, a, ap, rc, tau=tau, seed=6, rotate=1)
    pos = inputs.initial_walkers(s, W, 4)
    # the rule drops moves here
    _, k, d = orc.eval_moves(pos[0], orc.move_rotation(0, 0, 0))
    g = (np.arange(orc.M) // 6) % 2
    assert np.sum((g == 0) & (k * a * a < 2.0 ** -52)) > 50
    gpu.set_walkers(pos, 0)
    out = gpu.run(3, want_idx=True)
    ref = orc.run(pos, 3, gen0=0)
    print(f"compacted run moves={ref['n_moves'].sum()}", flush=True)
    assert ref["n_moves"].sum() > 3 * W
    n = run_agrees("compacted run", out["n_moves"].cpu().numpy(), out["idx"].cpu().numpy(), ref)
    eb = out["ebar"].cpu().numpy()
    check("compacted run ebar", eb[:n], ref["ebar"][:n], record_bar(ref["ebar"][:n]),
          scale=np.abs(ref["ebar"][:n]))
    if n == 3:
        check("compacted run final positions", gpu.get_walkers()["pos"].cpu().numpy(), ref["pos"], 1e-10)
    gpu.close()


def _shell_mix():
    """Three nuclei whose groups (shells of one nucleus and exponent) take
    every combination of s, p and d: a beta = 2.5 chain with flags s, p, sp,
    d, sd, pd, spd and five trailing s-only groups; a beta = 2 chain sp, sp,
    s; a beta = 3 chain spd and four s-only groups; a stand-alone p group."""
    rng = np.random.default_rng(11)
    shells = []   # (nucleus, l, alpha)
    flags0 = [(0,), (1,), (0, 1), (2,), (0, 2), (1, 2), (0, 1, 2)] + [(0,)] * 5
    for k, ls in enumerate(flags0):
        shells += [(0, l, 0.2 * 2.5 ** k) for l in ls]
    for k, ls in enumerate([(0, 1), (0, 1), (0,)]):
        shells += [(1, l, 0.3 * 2.0 ** k) for l in ls]
    for k, ls in enumerate([(0, 1, 2)] + [(0,)] * 4):
        shells += [(2, l, 0.5 * 3.0 ** k) for l in ls]
    shells.append((2, 1, 200.0))
    nuc, l, al = (list(x) for x in zip(*shells))
    K = sum(2 * q + 1 for q in l)
    mo = np.linalg.qr(rng.standard_normal((K, K)))[0][:, :3]
    R = np.array([[0.0, 0.0, 0.0], [0.3, -0.4, 1.4], [-1.0, 0.5, -0.6]])
    return inputs.System(Z=np.array([3.0, 1.0, 2.0]), R=R, n_up=3, n_dn=3, shell_nuc=nuc, shell_l=l,
                         shell_alpha=al, mo=mo, name="shell_mix")


def test_every_shell_combination_y_in_hbm():
    """The device-memory table loads each group's coefficients by its shell
    combination (and the trailing s-only groups four at a time): move
    tables against the oracle and against the same kernels with Y in LDS,
    then a run against the oracle."""
    from paper_1909_01589_amd.lrdmc import LRDMC, lrdmc_use_generic
    s = _shell_mix()
    a, tau, W = 0.05, 0.01, 8
    rc, ap, _ = spacing.spacing(s.z_max, a)
    gpu = LRDMC(s, a, ap, rc, tau, W, seed=2, rotate=1, refresh=2)
    orc = oracle.Oracle(s, a, ap, rc, tau=tau, seed=2, rotate=1)
    pos = inputs.initial_walkers(s, W, 6)
    lrdmc_use_generic(gpu.ctx, 2)
    rho = gpu.eval_moves(pos)[0].cpu().numpy().copy()
    lrdmc_use_generic(gpu.ctx, 1)
    rho_lds = gpu.eval_moves(pos)[0].cpu().numpy().copy()
    for w in range(W):
        r_o = orc.eval_moves(pos[w], orc.move_rotation(w, 0, 0))[0]
        check("shell mix y-hbm rho", rho[w], r_o, 1e-11 * np.abs(r_o) + 2e-12 * np.max(np.abs(r_o)),
              scale=np.abs(r_o))
    check("shell mix y-hbm against y-lds rho", rho, rho_lds, 1e-13 * np.abs(rho_lds).max(),
          scale=np.abs(rho_lds))
    lrdmc_use_generic(gpu.ctx, 2)
    gpu.set_walkers(pos, 0)
    out = gpu.run(3, want_idx=True)
    ref = orc.run(pos, 3, gen0=0)
    n = run_agrees("shell mix y-hbm run", out["n_moves"].cpu().numpy(), out["idx"].cpu().numpy(), ref)
    eb = out["ebar"].cpu().numpy()
    check("shell mix y-hbm run ebar", eb[:n], ref["ebar"][:n], record_bar(ref["ebar"][:n]),
          scale=np.abs(ref["ebar"][:n]))
    gpu.close()

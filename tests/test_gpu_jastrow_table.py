"""GPU parity of the learned Jastrow correction (a radial function per pair
type given by its node table, interpolated by C^2 quintics) against the
oracle through the C ABI: move tables and local energies, whole generations,
J and E_L of the gradient kernel, and the table gradient of
sum_w (c_j J_w + c_e E_L,w) against central differences of the oracle (exact
up to rounding: J is linear and E_L quadratic in the table).  Bars as in the
main parity tests: indices bit-exact, ratios and coefficients to FP64
rounding headroom, energies within 1e-9 relative."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from parity_bars import check, record_bar, run_agrees  # noqa: E402
from oracle import spacing  # noqa: E402
from paper_1909_01589_amd import inputs  # noqa: E402


def _system(name):
    if name == "be":
        return inputs.be_like(0), 0.2, 0.0161
    if name == "ar":
        return inputs.ar_like(0), 0.1, 0.00318
    if name == "tiny":
        return inputs.tiny_mixed(seed=1, n_up=3, n_dn=2), 0.06, 0.02
    raise KeyError(name)


def _pair(name, W, tab, rcut, seed=3, rotate=1, refresh=1):
    from paper_1909_01589_amd.lrdmc import LRDMC
    s, a, tau = _system(name)
    rc, ap, _ = spacing.spacing(s.z_max, a)
    gpu = LRDMC(s, a, ap, rc, tau, W, seed=seed, rotate=rotate, refresh=refresh)
    if tab is not None:
        gpu.set_jastrow_table(tab, rcut)
    orc = oracle.Oracle(s, a, ap, rc, tau=tau, seed=seed, rotate=rotate, ftab=tab, ftab_rcut=rcut)
    return s, gpu, orc


@pytest.mark.parametrize("name,W,G,rcut", [("be", 16, 33, 4.0), ("tiny", 8, 9, 2.5), ("ar", 6, 257, 5.0)])
def test_eval_moves_with_table_matches_oracle(name, W, G, rcut):
    tab = inputs.jastrow_table(seed=5, n_nodes=G, r_cut=rcut, scale=0.3)
    s, gpu, orc = _pair(name, W, tab, rcut)
    pos = inputs.initial_walkers(s, W, 7)
    rho, k, diag = (x.cpu().numpy() for x in gpu.eval_moves(pos))
    plain = oracle.Oracle(s, orc.prm.a, orc.prm.a_prime, orc.prm.r_c, tau=orc.prm.tau, seed=3, rotate=1)
    for w in range(W):
        print(f"table eval case={name} walker={w}", flush=True)
        r_o, k_o, d_o = orc.eval_moves(pos[w], orc.move_rotation(w, 0, 0))
        scale = np.max(np.abs(r_o))
        assert np.all(np.abs(rho[w] - r_o) <= 1e-9 * (np.abs(r_o) + scale))
        assert np.allclose(k[w], k_o, rtol=1e-12, atol=0)
        assert abs(diag[w, 0] - d_o["e_l"]) <= 1e-9 * (1 + abs(d_o["e_l"]) + abs(d_o["lap_exact"]))
        assert abs(diag[w, 3] - d_o["lap_exact"]) <= 1e-9 * (1 + abs(d_o["lap_exact"]))
        assert abs(diag[w, 6] - d_o["delta"]) <= 1e-9 * d_o["delta"]
        # the table changes the trial function
        assert abs(plain.local_energy(pos[w])[0] - d_o["e_l"]) > 1e-6
    gpu.close()


@pytest.mark.parametrize("name,W,n_gen,refresh", [("be", 64, 5, 1), ("be", 32, 5, 4), ("tiny", 32, 4, 3),
                                                  ("ar", 16, 3, 2)])
def test_run_with_table_matches_oracle(name, W, n_gen, refresh):
    rcut = 4.0
    tab = inputs.jastrow_table(seed=2, n_nodes=65, r_cut=rcut, scale=0.3)
    s, gpu, orc = _pair(name, W, tab, rcut, seed=9, refresh=refresh)
    pos = inputs.initial_walkers(s, W, 2)
    gpu.set_walkers(pos, 0)
    out = gpu.run(n_gen, want_idx=True)
    ref = orc.run(pos, n_gen, gen0=0)
    print(f"table run case={name} W={W} refresh={refresh}", flush=True)
    n = run_agrees(f"table run {name} refresh {refresh}", out["n_moves"].cpu().numpy(),
                   out["idx"].cpu().numpy(), ref)
    eb, eb_o = out["ebar"].cpu().numpy(), ref["ebar"]
    check(f"table run ebar ({name})", eb[:n], eb_o[:n], record_bar(eb_o[:n]), scale=np.abs(eb_o[:n]))
    if n == n_gen:
        p = gpu.get_walkers()["pos"].cpu().numpy()
        check(f"table run final positions ({name})", p, ref["pos"], 1e-10)
    gpu.close()


def test_fixed_and_general_kernels_agree_with_table():
    """The Be-sized fixed kernel (selected with refresh > 1) and the general
    kernel give the same generation with a table."""
    from paper_1909_01589_amd.lrdmc import LRDMC, lrdmc_is_specialized, lrdmc_use_generic
    s, a, tau = _system("be")
    rc, ap, _ = spacing.spacing(s.z_max, a)
    tab = inputs.jastrow_table(seed=4, n_nodes=33, r_cut=4.0, scale=0.3)
    pos = inputs.initial_walkers(s, 64, 1)
    res = []
    for generic in (False, True):
        gpu = LRDMC(s, a, ap, rc, tau, 64, seed=1, rotate=1, refresh=4)
        gpu.set_jastrow_table(tab, 4.0)
        lrdmc_use_generic(gpu.ctx, generic)
        assert lrdmc_is_specialized(gpu.ctx) == (not generic)
        gpu.set_walkers(pos, 0)
        out = gpu.run(3, want_idx=True)
        res.append((out["idx"].cpu().numpy(), out["ebar"].cpu().numpy(), gpu.get_walkers()["pos"].cpu().numpy()))
        gpu.close()
    assert np.array_equal(res[0][0], res[1][0])
    assert np.allclose(res[0][1], res[1][1], rtol=1e-12, atol=1e-12)
    assert np.allclose(res[0][2], res[1][2], rtol=0, atol=1e-11)


def test_zero_table_and_removal_give_pade():
    from paper_1909_01589_amd.lrdmc import LRDMC
    s, a, tau = _system("be")
    rc, ap, _ = spacing.spacing(s.z_max, a)
    W = 16
    pos = inputs.initial_walkers(s, W, 3)
    gpu = LRDMC(s, a, ap, rc, tau, W, seed=1, rotate=1)
    base = gpu.eval_moves(pos)[2].cpu().numpy()
    gpu.set_jastrow_table(np.zeros((2, 17, 3)), 3.0)
    zero = gpu.eval_moves(pos)[2].cpu().numpy()
    gpu.set_jastrow_table(inputs.jastrow_table(seed=1, n_nodes=17, r_cut=3.0, scale=0.3), 3.0)
    other = gpu.eval_moves(pos)[2].cpu().numpy()
    gpu.set_jastrow_table(None)
    back = gpu.eval_moves(pos)[2].cpu().numpy()
    assert np.allclose(zero, base, rtol=1e-13, atol=1e-13)
    assert not np.allclose(other[:, 0], base[:, 0], rtol=1e-6, atol=0)
    assert np.array_equal(back, base)
    gpu.close()


def test_device_table_equals_host_table():
    from paper_1909_01589_amd.lrdmc import LRDMC
    s, a, tau = _system("tiny")
    rc, ap, _ = spacing.spacing(s.z_max, a)
    W = 8
    tab = inputs.jastrow_table(seed=8, n_nodes=21, r_cut=3.0, scale=0.3)
    pos = inputs.initial_walkers(s, W, 3)
    gpu = LRDMC(s, a, ap, rc, tau, W, seed=1, rotate=1)
    gpu.set_jastrow_table(tab, 3.0)
    host = gpu.eval_moves(pos)[0].cpu().numpy()
    gpu.set_jastrow_table(torch.tensor(tab, device=gpu.device), 3.0)
    dev = gpu.eval_moves(pos)[0].cpu().numpy()
    assert np.array_equal(host, dev)
    gpu.close()


def test_table_errors():
    from paper_1909_01589_amd.lrdmc import LRDMC, LRDMCError
    s, a, tau = _system("tiny")
    rc, ap, _ = spacing.spacing(s.z_max, a)
    gpu = LRDMC(s, a, ap, rc, tau, 4, seed=1)
    pos = inputs.initial_walkers(s, 4, 3)
    with pytest.raises(ValueError):
        gpu.jastrow_table_grad(pos, np.ones(4), np.ones(4))
    for bad, rcut in ((np.zeros((2, 1, 3)), 1.0), (np.zeros((2, 5, 3)), 0.0), (np.zeros((2, 5, 3)), np.inf),
                      (np.zeros((2, 4097, 3)), 1.0)):
        with pytest.raises(LRDMCError, match="EINVAL"):
            gpu.set_jastrow_table(bad, rcut)
    t = inputs.jastrow_table(seed=1, n_nodes=9, r_cut=2.0)
    t[1, 3, 2] = np.nan
    with pytest.raises(LRDMCError, match="non-finite table entry"):
        gpu.set_jastrow_table(t, 2.0)
    # the failed call removed the correction: the Pade trial function is back
    base = oracle.Oracle(s, a, ap, rc, tau=tau, seed=1, rotate=1)
    e = gpu.eval_moves(pos)[2].cpu().numpy()[:, 0]
    assert np.allclose(e, [base.local_energy(p)[0] for p in pos], rtol=1e-10, atol=1e-10)
    gpu.close()


@pytest.mark.parametrize("name,W,G,rcut", [("tiny", 6, 9, 2.5), ("be", 5, 7, 3.0)])
def test_jastrow_and_energy_with_table(name, W, G, rcut):
    tab = inputs.jastrow_table(seed=6, n_nodes=G, r_cut=rcut, scale=0.3)
    s, gpu, orc = _pair(name, W, tab, rcut)
    pos = inputs.initial_walkers(s, W, 4)
    out = gpu.jastrow_grad(pos).cpu().numpy()
    for w in range(W):
        e_o = orc.local_energy(pos[w])[0]
        assert abs(out[w, 0] - e_o) <= 1e-9 * (1 + abs(e_o))
        assert abs(out[w, 1] - orc.jastrow(pos[w])) <= 1e-11 * (1 + abs(out[w, 1]))
        dj, de = orc.jastrow_param_grad(pos[w])
        assert np.allclose(out[w, 2:4], dj, rtol=1e-10, atol=1e-12)
        assert np.allclose(out[w, 4:6], de, rtol=1e-9, atol=1e-10)
    gpu.close()


@pytest.mark.parametrize("name,W,G,rcut", [("tiny", 6, 9, 2.5), ("be", 5, 7, 3.0)])
def test_table_gradient_matches_oracle_differences(name, W, G, rcut):
    tab = inputs.jastrow_table(seed=6, n_nodes=G, r_cut=rcut, scale=0.3)
    s, gpu, orc = _pair(name, W, tab, rcut)
    pos = inputs.initial_walkers(s, W, 4)
    rng = np.random.default_rng(0)
    cj, ce = rng.normal(size=W), rng.normal(size=W)
    g = gpu.jastrow_table_grad(pos, cj, ce).cpu().numpy()
    gj = gpu.jastrow_table_grad(pos, cj, None).cpu().numpy()

    def objective(t, with_e=True):
        o = oracle.Oracle(s, orc.prm.a, orc.prm.a_prime, orc.prm.r_c, ftab=t, ftab_rcut=rcut)
        return sum(cj[w] * o.jastrow(pos[w]) + (ce[w] * o.local_energy(pos[w])[0] if with_e else 0.0)
                   for w in range(W))

    h = 1e-3
    ref, ref_j = np.zeros_like(tab), np.zeros_like(tab)
    for idx in np.ndindex(*tab.shape):
        tp, tm = tab.copy(), tab.copy()
        tp[idx] += h
        tm[idx] -= h
        ref[idx] = (objective(tp) - objective(tm)) / (2 * h)
        ref_j[idx] = (objective(tp, False) - objective(tm, False)) / (2 * h)
    print(f"table grad case={name} max|g|={np.abs(ref).max():.3e}", flush=True)
    scale = np.abs(ref).max()
    assert np.allclose(g, ref, rtol=1e-6, atol=1e-8 * scale)
    assert np.allclose(gj, ref_j, rtol=1e-8, atol=1e-10 * np.abs(ref_j).max())
    gpu.close()

"""GPU parity of the learned Jastrow network path against the oracle.

* Tabulation kernel (value, f', f'' by forward-mode derivatives through the
  layers) against the numpy oracle's tabulation of the same weights.
* Reverse pass (parameter gradient of a loss on the table) against central
  differences of the oracle's tabulation.
* The whole chain params -> table -> (J, E_L) -> weighted variance: its
  autograd gradient against central differences of the same objective
  computed by the oracle alone.
* Variance minimisation lowers the weighted variance, and the trained
  trial function's E_L matches the oracle's with the same weights.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from oracle import neural as oneural  # noqa: E402
from oracle import spacing  # noqa: E402
from paper_1909_01589_amd import inputs  # noqa: E402


@pytest.mark.parametrize("H,G,rc", [(8, 33, 4.0), (64, 257, 6.0), (100, 65, 5.0)])
def test_net_table_matches_oracle(H, G, rc):
    from paper_1909_01589_amd import neural
    from paper_1909_01589_amd.lrdmc import lrdmc_net_tabulate
    w = inputs.neural_weights(seed=3, hidden=H, out_scale=1.0)
    p = torch.tensor(neural.pack(w), device="cuda")
    tab = torch.empty(2, G, 3, dtype=torch.float64, device="cuda")
    lrdmc_net_tabulate(p, H, G, rc, tab)
    got = tab.cpu().numpy()
    ref = oneural.tabulate(w, G, rc)
    scale = np.abs(ref).max(axis=1, keepdims=True)
    assert np.all(np.abs(got - ref) <= 1e-12 * (np.abs(ref) + scale))
    assert np.all(got[:, 0, :2] == 0.0) and np.all(np.abs(got[:, -1]) <= 1e-13 * scale[:, 0])


@pytest.mark.parametrize("H,G,n_check", [(8, 17, None), (64, 65, 80)])
def test_net_backward_matches_oracle_differences(H, G, n_check):
    from paper_1909_01589_amd import neural
    from paper_1909_01589_amd.lrdmc import lrdmc_net_tabulate_backward, lrdmc_net_workspace_size
    rc = 5.0
    w = inputs.neural_weights(seed=4, hidden=H, out_scale=1.0)
    flat = neural.pack(w)
    rng = np.random.default_rng(1)
    gtab = rng.normal(size=(2, G, 3))
    p = torch.tensor(flat, device="cuda")
    g = torch.empty_like(p)
    work = torch.empty(lrdmc_net_workspace_size(H, G), dtype=torch.float64, device="cuda")
    lrdmc_net_tabulate_backward(p, H, G, rc, torch.tensor(gtab, device="cuda"), g, work)
    got = g.cpu().numpy()

    def loss(x):
        return float((gtab * oneural.tabulate(neural.unpack(x, H), G, rc)).sum())

    idx = list(np.ndindex(*flat.shape))
    if n_check is not None:
        idx = [idx[i] for i in rng.choice(len(idx), n_check, replace=False)]
        idx += [(0, 0), (1, H), (0, 2 * H + 5), (1, 3 * H + H * H), (0, flat.shape[1] - 1)]
    scale = np.abs(got).max()
    for ix in idx:
        vals = []
        for h in (1e-4, 5e-5):
            xp, xm = flat.copy(), flat.copy()
            xp[ix] += h
            xm[ix] -= h
            vals.append((loss(xp) - loss(xm)) / (2 * h))
        ref = (4 * vals[1] - vals[0]) / 3
        assert abs(got[ix] - ref) <= 1e-7 * (abs(ref) + scale), (ix, got[ix], ref)


def _system():
    return inputs.be_like(0), 0.2, 0.0161


def test_table_from_network_matches_oracle():
    from paper_1909_01589_amd import neural
    from paper_1909_01589_amd.lrdmc import LRDMC
    s, a, tau = _system()
    rc_s, ap, _ = spacing.spacing(s.z_max, a)
    H, G, rcut, W = 16, 129, 5.0, 12
    w = inputs.neural_weights(seed=5, hidden=H, out_scale=0.3)
    nj = neural.NeuralJastrow(H, G, rcut, params=neural.pack(w))
    gpu = LRDMC(s, a, ap, rc_s, tau, W, seed=2, rotate=1)
    nj.attach(gpu)
    orc = oracle.Oracle(s, a, ap, rc_s, tau=tau, seed=2, rotate=1, ftab=oneural.tabulate(w, G, rcut),
                        ftab_rcut=rcut)
    pos = inputs.initial_walkers(s, W, 6)
    rho, k, diag = (x.cpu().numpy() for x in gpu.eval_moves(pos))
    for wk in range(W):
        r_o, k_o, d_o = orc.eval_moves(pos[wk], orc.move_rotation(wk, 0, 0))
        assert np.all(np.abs(rho[wk] - r_o) <= 1e-9 * (np.abs(r_o) + np.max(np.abs(r_o))))
        assert abs(diag[wk, 0] - d_o["e_l"]) <= 1e-9 * (1 + abs(d_o["e_l"]) + abs(d_o["lap_exact"]))
    gpu.close()


def _oracle_objective(s, a, ap, rc_s, pos, flat, H, G, rcut, j0, power):
    from paper_1909_01589_amd import neural
    tab = oneural.tabulate(neural.unpack(flat, H), G, rcut)
    o = oracle.Oracle(s, a, ap, rc_s, ftab=tab, ftab_rcut=rcut)
    j = np.array([o.jastrow(p) for p in pos])
    e = np.array([o.local_energy(p)[0] for p in pos])
    lw = power * (j - j0)
    wt = np.exp(lw - lw.max())
    wt /= wt.sum()
    m = (wt * e).sum()
    return (wt * (e - m) ** 2).sum(), j, e


@pytest.mark.parametrize("power", [1.0, 2.0])
def test_chain_gradient_matches_oracle_objective(power):
    from paper_1909_01589_amd import neural
    from paper_1909_01589_amd.lrdmc import LRDMC
    s, a, tau = _system()
    rc_s, ap, _ = spacing.spacing(s.z_max, a)
    H, G, rcut, W = 8, 33, 4.0, 6
    w = inputs.neural_weights(seed=7, hidden=H, out_scale=0.5)
    flat = neural.pack(w)
    pos = inputs.initial_walkers(s, W, 9)
    j0 = np.zeros(W) + 0.1 * np.arange(W)
    gpu = LRDMC(s, a, ap, rc_s, tau, W, seed=2, rotate=1)
    nj = neural.NeuralJastrow(H, G, rcut, params=flat)
    pos_d = torch.tensor(pos, device="cuda")
    j, e = nj.energies(gpu, pos_d)
    _, var = neural.weighted_moments(j, e, torch.tensor(j0, device="cuda"), power)
    var.backward()
    got = nj.params.grad.cpu().numpy()
    var_o, j_o, e_o = _oracle_objective(s, a, ap, rc_s, pos, flat, H, G, rcut, j0, power)
    assert np.allclose(j.detach().cpu().numpy(), j_o, rtol=1e-11, atol=1e-11)
    assert np.allclose(e.detach().cpu().numpy(), e_o, rtol=1e-9, atol=1e-9)
    assert float(var.detach()) == pytest.approx(var_o, rel=1e-8)
    rng = np.random.default_rng(3)
    idx = list(np.ndindex(*flat.shape))
    idx = [idx[i] for i in rng.choice(len(idx), 24, replace=False)] + [(0, 3 * H + H * H), (1, 4 * H + H * H)]
    scale = np.abs(got).max()
    for ix in idx:
        h = 1e-5
        xp, xm = flat.copy(), flat.copy()
        xp[ix] += h
        xm[ix] -= h
        ref = (_oracle_objective(s, a, ap, rc_s, pos, xp, H, G, rcut, j0, power)[0] -
               _oracle_objective(s, a, ap, rc_s, pos, xm, H, G, rcut, j0, power)[0]) / (2 * h)
        assert abs(got[ix] - ref) <= 1e-5 * (abs(ref) + scale), (ix, got[ix], ref)
    gpu.close()


def test_training_lowers_variance_and_matches_oracle():
    from paper_1909_01589_amd import neural
    from paper_1909_01589_amd.lrdmc import LRDMC
    s, a, tau = _system()
    rc_s, ap, _ = spacing.spacing(s.z_max, a)
    W = 2048
    gpu = LRDMC(s, a, ap, rc_s, tau, W, seed=2, rotate=1, refresh=4)
    gpu.set_walkers(inputs.initial_walkers(s, W, 1), 0)
    gpu.run(40)
    pos = gpu.get_walkers()["pos"]
    nj = neural.NeuralJastrow(16, 129, 5.0, seed=1)
    hist = nj.train(gpu, pos, steps=60, lr=3e-3, power=1.0)
    print(f"variance {hist[0][1]:.4f} -> {hist[-1][1]:.4f}", flush=True)
    assert hist[-1][1] < 0.8 * hist[0][1]
    # the trained trial function, evaluated by the oracle from the same weights
    flat = nj.params.detach().cpu().numpy()
    o = oracle.Oracle(s, a, ap, rc_s, ftab=oneural.tabulate(neural.unpack(flat, 16), 129, 5.0), ftab_rcut=5.0)
    out = gpu.jastrow_grad(pos).cpu().numpy()
    pn = pos.cpu().numpy()
    for wk in (0, 1, W // 2, W - 1):
        e_o = o.local_energy(pn[wk])[0]
        assert abs(out[wk, 0] - e_o) <= 1e-9 * (1 + abs(e_o))
    gpu.close()

"""GPU Metropolis sampler against the oracle's chain (same random stream:
accepted counts bit-exact, positions and E_L to rounding) and against the
exact moments of the hydrogenic density r^2 exp(-2 Z r)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from oracle import spacing  # noqa: E402
from paper_1909_01589_amd import inputs  # noqa: E402


@pytest.mark.parametrize("name,W,steps,step,table", [("be", 16, 60, 0.4, False), ("tiny", 8, 50, 0.3, True),
                                                       ("ar", 4, 40, 0.2, False), ("ar", 4, 40, 0.2, True)])
def test_vmc_chain_matches_oracle(name, W, steps, step, table):
    from paper_1909_01589_amd.lrdmc import LRDMC
    s = {"be": inputs.be_like(0), "tiny": inputs.tiny_mixed(seed=1, n_up=3, n_dn=2), "ar": inputs.ar_like(0)}[name]
    a = 0.1
    rc, ap, _ = spacing.spacing(s.z_max, a)
    tab = inputs.jastrow_table(seed=3, n_nodes=65, r_cut=4.0, scale=0.3) if table else None
    gpu = LRDMC(s, a, ap, rc, 0.01, W, seed=4, rotate=1)
    if table:
        gpu.set_jastrow_table(tab, 4.0)
    orc = oracle.Oracle(s, a, ap, rc, tau=0.01, seed=4, rotate=1, ftab=tab, ftab_rcut=4.0)
    pos = inputs.initial_walkers(s, W, 5)
    gpu.set_walkers(pos, 0)
    gpu.vmc(steps, step)
    gpu.vmc(steps, step)          # second call: generation 1, continues from the first
    out = {k: v.cpu().numpy() for k, v in gpu.get_walkers().items()}
    for w in range(W):
        print(f"vmc case={name} table={table} walker={w}", flush=True)
        p, a0, _ = orc.vmc(pos[w], w, 0, steps, step)
        p, a1, el = orc.vmc(p, w, 1, steps, step)
        assert out["n_moves"][w] == a1
        assert np.allclose(out["pos"][w], p, rtol=0, atol=1e-10)
        assert abs(out["e_l"][w] - el) <= 1e-9 * (1 + abs(el))
        assert out["log_w"][w] == 0.0
    gpu.close()


@pytest.mark.parametrize("Z,step", [(1.0, 1.2), (3.0, 0.4)])
def test_hydrogenic_moments(Z, step):
    from paper_1909_01589_amd.lrdmc import LRDMC
    s = inputs.hydrogenic(Z)
    W = 8192
    gpu = LRDMC(s, 0.1, 0.1, 1.0, 0.01, W, seed=7, rotate=1)
    rng = np.random.default_rng(0)
    gpu.set_walkers(rng.normal(size=(W, 1, 3)) / Z, 0)
    gpu.vmc(400, step)
    r, r2, x2 = [], [], []
    for _ in range(8):
        gpu.vmc(20, step)
        out = gpu.get_walkers()
        p = out["pos"].cpu().numpy()[:, 0]
        assert np.allclose(out["e_l"].cpu().numpy(), -0.5 * Z * Z, atol=1e-10)
        rr = np.linalg.norm(p, axis=1)
        r.append(rr.mean()); r2.append((rr * rr).mean()); x2.append((p * p).mean(axis=0))
    # 8 nearly independent batches of 8192 walkers
    for val, ref in ((np.array(r), 1.5 / Z), (np.array(r2), 3.0 / Z ** 2)):
        err = val.std(ddof=1) / np.sqrt(val.size)
        assert abs(val.mean() - ref) < 5 * err + 1e-3 * ref, (val.mean(), ref, err)
    x2 = np.array(x2).mean(axis=0)
    assert np.allclose(x2, 1.0 / Z ** 2, rtol=0.02)
    gpu.close()


def test_vmc_errors():
    from paper_1909_01589_amd.lrdmc import LRDMC, LRDMCError
    s = inputs.be_like(0)
    gpu = LRDMC(s, 0.1, 0.2, 0.5, 0.01, 4, seed=1)
    with pytest.raises(LRDMCError, match="no walkers"):
        gpu.vmc(10, 0.3)
    gpu.set_walkers(inputs.initial_walkers(s, 4, 0), 0)
    for n, st in ((-1, 0.3), (5, 0.0), (5, float("nan"))):
        with pytest.raises(LRDMCError, match="EINVAL"):
            gpu.vmc(n, st)
    gpu.close()

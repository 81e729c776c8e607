"""The check of the Sherman-Morrison-carried state (lrdmc_inverse_residual):
max |A Ainv - I| per walker, A recomputed from the positions, Ainv the
inverse stored in the walker's state.  On the benchmark-size Ar-like atom
(inverse in LDS), the Z = 54 atom and the molecule (inverse with Y in device
memory): small right after the inverse is recomputed at a refresh generation,
larger after several generations of rank-one updates, and well inside the
FP64 parity bars throughout; refused where no state is stored."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from oracle import spacing  # noqa: E402
from paper_1909_01589_amd import inputs  # noqa: E402


def _residual(gpu):
    from paper_1909_01589_amd.lrdmc import lrdmc_inverse_residual
    res = torch.empty(gpu.W, dtype=torch.float64, device="cuda")
    lrdmc_inverse_residual(gpu.ctx, res)
    return res.cpu().numpy()


@pytest.mark.parametrize("name,W", [("ar_a0.1", 512), ("zsweep54", 64), ("molecule", 64)])
def test_inverse_residual_of_the_carried_state(name, W):
    from paper_1909_01589_amd.lrdmc import LRDMC
    cfg = inputs.get_config(name)
    s = cfg.system
    rc, ap, _ = spacing.spacing(s.z_max, cfg.a)
    assert cfg.refresh == 8
    gpu = LRDMC(s, cfg.a, ap, rc, cfg.tau, W, seed=cfg.seed, rotate=1, refresh=cfg.refresh)
    gpu.set_walkers(inputs.initial_walkers(s, W, 3), 0)
    out = {}
    for gen in range(10):
        gpu.project()
        out[gen] = _residual(gpu)           # after generation gen (before its reconfiguration)
        gpu.branch()
    r_after = _residual(gpu)                # slots report the walkers they selected
    gpu.close()
    for gen, r in out.items():
        print(f"{name}: generation {gen}: max |A Ainv - I| = {r.max():.2e} (median {np.median(r):.2e})", flush=True)
        assert np.all(np.isfinite(r)) and np.all(r >= 0.0)
        assert r.max() < 1e-6
    assert np.isfinite(r_after).all()
    # generation 8 recomputes the inverse at its start (refresh 8); 7 carries
    # seven generations of updates since generation 0
    print(f"{name}: median after 7 carried generations {np.median(out[7]):.2e}, "
          f"after the refresh at 8 {np.median(out[8]):.2e}", flush=True)


def test_inverse_residual_refused_without_stored_state():
    from paper_1909_01589_amd.lrdmc import LRDMC, LRDMCError
    s = inputs.be_like(0)
    rc, ap, _ = spacing.spacing(4, 0.2)
    gpu = LRDMC(s, 0.2, ap, rc, 0.02, 8, seed=1, refresh=1)
    gpu.set_walkers(inputs.initial_walkers(s, 8, 0), 0)
    gpu.project()
    with pytest.raises(LRDMCError) as e:
        _residual(gpu)
    assert e.value.code == -1
    gpu.close()
    gpu = LRDMC(s, 0.2, ap, rc, 0.02, 8, seed=1, refresh=4)
    gpu.set_walkers(inputs.initial_walkers(s, 8, 0), 0)
    with pytest.raises(LRDMCError):
        _residual(gpu)                      # no projection yet
    gpu.project()
    assert _residual(gpu).max() < 1e-8
    gpu.close()

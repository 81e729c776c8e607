"""The measurement prototype of the table's contraction (libmfma_probe.so):
determinant ratios of the fixed-axis move table by the FP64 Y-dot and by the
BF16x3 matrix-core product Phi' = B' C with the FP64 inverse, against the
oracle's determinant ratios (Psi ratio over the Jastrow ratio, both
recomputed in full).

Bars: the FP64 variant to the FP64 parity bar of the move ratios; the BF16x3
variant within its derived bound (split and FP32 accumulation errors times
sum_j sum_mu |g_mu C_mu j| |Ainv_j i|), with the observed errors printed."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from oracle import spacing  # noqa: E402
from paper_1909_01589_amd import inputs  # noqa: E402
from parity_bars import check, ratio_bar  # noqa: E402


def _oracle_det_ratios(o, pos):
    rho, _, _ = o.eval_moves(pos, np.eye(3))
    J0 = o.jastrow(pos)
    out = np.zeros(o.M)
    for m in range(o.M):
        rp, _ = o.move(pos, np.eye(3), m)
        p2 = pos.copy()
        p2[m // (o.M // o.N)] = rp
        out[m] = rho[m] / np.exp(o.jastrow(p2) - J0)
    return out


@pytest.mark.parametrize("name,W", [("ar_a0.1", 6), ("molecule", 3), ("zsweep54", 2)])
def test_probe_ratios_against_the_oracle(name, W):
    from paper_1909_01589_amd import mfma_probe as mp
    cfg = inputs.get_config(name)
    s = cfg.system
    rc, ap, _ = spacing.spacing(s.z_max, cfg.a)
    pos = inputs.initial_walkers(s, W, 4)
    probe = mp.Probe(s, pos, cfg.a, ap)
    r64 = probe.ratios(0).cpu().numpy().copy()
    r16 = probe.ratios(1).cpu().numpy().copy()
    bound = mp.bf16x3_bound(probe.prep, s, pos, cfg.a, ap)
    o = oracle.Oracle(s, cfg.a, ap, rc, tau=cfg.tau, seed=1, rotate=0)
    rel = []
    for w in range(W):
        print(f"mfma probe {name} walker {w}", flush=True)
        rd = _oracle_det_ratios(o, pos[w])
        scale = np.max(np.abs(rd))
        check(f"probe FP64 Y-dot ({name})", r64[w], rd, ratio_bar(rd, scale), scale=np.abs(rd) + scale)
        check(f"probe BF16x3 MFMA ({name})", r16[w], rd, bound[w] + 1e-9 * scale, scale=np.abs(rd) + scale)
        rel.append(np.abs(r16[w] - rd) / scale)
    rel = np.concatenate(rel)
    print(f"BF16x3 {name}: error / max|rho_D| median {np.median(rel):.2e}, max {rel.max():.2e}; "
          f"sign changes {int(np.sum(np.sign(r16) != np.sign(r64)))} of {r16.size}", flush=True)

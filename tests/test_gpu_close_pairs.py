"""GPU parity of the move table where a displaced point lands next to
another electron or next to the nucleus, at distances from 1e-3 down to
1e-7 bohr.  The table's Jastrow terms of two electrons at both points of a
move pair share one reciprocal of the product of their denominators
1/r + b, which then span up to seven orders of magnitude.  Lattice axes are
fixed (no rotation), so the constructed geometry is exact.  Padé and
learned-correction Jastrow, fixed-size and general kernels; bars as in the
main parity tests."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from oracle import spacing  # noqa: E402
from paper_1909_01589_amd import inputs  # noqa: E402

_EPS = (1e-3, 1e-5, 1e-7)
_DIRS = np.array([[0.3, -0.5, 0.8], [-0.6, 0.2, 0.1], [0.1, 0.9, -0.4]])


def _close_walkers(s, W, h_small, h_large, seed=11):
    """Walker w puts, by kind w % 4: the first down electron next to the +x
    small-grid point of electron 0; the same next to the -y large-grid
    point; electron 0 so that its -z small-grid point lies next to the
    nucleus; two down electrons next to the +x and -x small-grid points of
    electron 0.  The distance is _EPS[(w // 4) % 3]."""
    pos = inputs.initial_walkers(s, W, seed).copy()
    nu, R = s.n_up, np.asarray(s.R[0], dtype=np.float64)
    for w in range(W):
        eps, kind = _EPS[(w // 4) % 3], w % 4
        v0, v1 = eps * _DIRS[w % 3], eps * _DIRS[(w + 1) % 3]
        if kind == 0:
            pos[w, nu] = pos[w, 0] + np.array([h_small, 0.0, 0.0]) + v0
        elif kind == 1:
            pos[w, nu] = pos[w, 0] - np.array([0.0, h_large, 0.0]) + v0
        elif kind == 2:
            pos[w, 0] = R + np.array([0.0, 0.0, h_small]) + v0
        else:
            pos[w, nu] = pos[w, 0] + np.array([h_small, 0.0, 0.0]) + v0
            pos[w, nu + 1] = pos[w, 0] - np.array([h_small, 0.0, 0.0]) + v1
    return pos


@pytest.mark.parametrize("name", ["be", "ar"])
@pytest.mark.parametrize("table", [False, True])
@pytest.mark.parametrize("generic", [0, 1])
def test_close_pairs_in_the_move_table(name, table, generic):
    from paper_1909_01589_amd.lrdmc import LRDMC, lrdmc_use_generic
    s, a, tau = (inputs.be_like(0), 0.2, 0.0161) if name == "be" else (inputs.ar_like(0), 0.1, 0.00318)
    rc, ap, _ = spacing.spacing(s.z_max, a)
    W, rcut = 12, 5.0
    tab = inputs.jastrow_table(seed=5, n_nodes=257, r_cut=rcut, scale=0.3) if table else None
    gpu = LRDMC(s, a, ap, rc, tau, W, seed=3, rotate=0)
    if table:
        gpu.set_jastrow_table(tab, rcut)
    lrdmc_use_generic(gpu.ctx, generic)
    orc = oracle.Oracle(s, a, ap, rc, tau=tau, seed=3, rotate=0, ftab=tab, ftab_rcut=rcut)
    pos = _close_walkers(s, W, a, ap)
    rho, k, diag = (x.cpu().numpy() for x in gpu.eval_moves(pos))
    for w in range(W):
        print(f"close pairs case={name} table={table} generic={generic} walker={w}", flush=True)
        r_o, k_o, d_o = orc.eval_moves(pos[w], np.eye(3))
        scale = np.max(np.abs(r_o))
        assert np.all(np.abs(rho[w] - r_o) <= 1e-9 * (np.abs(r_o) + scale))
        assert np.allclose(k[w], k_o, rtol=1e-12, atol=0)
        assert abs(diag[w, 0] - d_o["e_l"]) <= 1e-9 * (1 + abs(d_o["e_l"]) + abs(d_o["lap_exact"]))
        assert abs(diag[w, 6] - d_o["delta"]) <= 1e-9 * d_o["delta"]
    gpu.close()

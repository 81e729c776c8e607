"""GPU parity of the earlier double-grid scheme (Pade switch of main text
Eq. (2) with the spacing rule of Eq. (4)) and of the single grid (p = 1,
6N moves), against the oracle through the C ABI.  Same bars as the main
parity tests: move and reconfiguration indices bit-exact, ratios and
coefficients to FP64 rounding headroom, energies within 1e-10 Ha plus a
relative term."""
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


def _pair(name, W, mode, seed=3, rotate=1, refresh=1):
    from paper_1909_01589_amd.lrdmc import LRDMC
    s, a, tau = _system(name)
    if mode == "pade":
        rc, ap = spacing.spacing_pade(s.z_max, a)
        kw = dict(switch_form=1, grids=2)
    else:
        rc, ap, _ = spacing.spacing(s.z_max, a) if name != "tiny" else (0.5, 0.1, 0)
        kw = dict(switch_form=0, grids=1)
    gpu = LRDMC(s, a, ap, rc, tau, W, seed=seed, rotate=rotate, refresh=refresh, **kw)
    orc = oracle.Oracle(s, a, ap, rc, tau=tau, seed=seed, rotate=rotate, **kw)
    return s, gpu, orc


def test_pade_spacing_matches_oracle():
    from paper_1909_01589_amd.lrdmc import lrdmc_spacing_pade
    for Z in (2, 4, 10, 18, 36, 54):
        for a in (0.01, 0.1):
            rc, ap = lrdmc_spacing_pade(Z, a)
            rc_o, ap_o = spacing.spacing_pade(Z, a)
            assert rc == rc_o and ap == pytest.approx(ap_o, rel=1e-15)


@pytest.mark.parametrize("mode", ["pade", "single"])
@pytest.mark.parametrize("name,W", [("be", 16), ("tiny", 8), ("ar", 6)])
@pytest.mark.parametrize("rotate", [0, 1])
def test_eval_moves_matches_oracle(mode, name, W, rotate):
    s, gpu, orc = _pair(name, W, mode, rotate=rotate)
    assert gpu.M == orc.M == (12 if mode == "pade" else 6) * s.n_elec
    pos = inputs.initial_walkers(s, W, 7)
    rho, k, diag = (x.cpu().numpy() for x in gpu.eval_moves(pos))
    for w in range(W):
        print(f"modes eval mode={mode} case={name} walker={w} rotate={rotate}", flush=True)
        r_o, k_o, d_o = orc.eval_moves(pos[w], orc.move_rotation(w, 0, 0))
        scale = np.max(np.abs(r_o))
        assert np.all(np.abs(rho[w] - r_o) <= 1e-9 * (np.abs(r_o) + scale))
        assert np.allclose(k[w], k_o, rtol=1e-12, atol=0)
        assert abs(diag[w, 0] - d_o["e_l"]) <= 1e-9 * (1 + abs(d_o["e_l"]) + abs(d_o["lap_exact"]))
        assert abs(diag[w, 2] - d_o["lap_lattice"]) <= 1e-9 * (1 + abs(d_o["lap_lattice"]))
        assert abs(diag[w, 8] - d_o["sum_k"]) <= 1e-12 * d_o["sum_k"]
        assert abs(diag[w, 6] - d_o["delta"]) <= 1e-9 * d_o["delta"]
    gpu.close()


@pytest.mark.parametrize("mode", ["pade", "single"])
@pytest.mark.parametrize("name,W,n_gen,refresh", [("be", 64, 6, 1), ("tiny", 32, 5, 3), ("ar", 16, 4, 2)])
def test_run_matches_oracle(mode, name, W, n_gen, refresh):
    s, gpu, orc = _pair(name, W, mode, seed=9, refresh=refresh)
    pos = inputs.initial_walkers(s, W, 2)
    gpu.set_walkers(pos, 0)
    out = gpu.run(n_gen, want_idx=True)
    ref = orc.run(pos, n_gen, gen0=0)
    print(f"modes run mode={mode} case={name}", flush=True)
    n = run_agrees(f"modes run {mode} {name}", out["n_moves"].cpu().numpy(), out["idx"].cpu().numpy(), ref)
    e = out["ebar"].cpu().numpy()
    check(f"modes run ebar ({mode}, {name})", e[:n], ref["ebar"][:n], record_bar(ref["ebar"][:n]),
          scale=np.abs(ref["ebar"][:n]))
    lwb = out["log_wbar"].cpu().numpy()
    check(f"modes run log wbar ({mode}, {name})", lwb[:n], ref["log_wbar"][:n],
          record_bar(ref["log_wbar"][:n]), scale=np.abs(ref["log_wbar"][:n]))
    if n == n_gen:
        fin = gpu.get_walkers()["pos"].cpu().numpy()
        check(f"modes run final positions ({mode}, {name})", fin, ref["pos"], 1e-11)
    gpu.close()


def test_kernel_selection_by_mode():
    """With a state kept across generations (refresh > 1, the layout the
    fixed-size kernels are built for), the Pade switch runs the fixed-size
    kernel of the Ar-like atom; the single grid (6N moves) has a different
    layout and runs the general one."""
    from paper_1909_01589_amd.lrdmc import lrdmc_is_specialized
    _, gpu, _ = _pair("ar", 4, "pade", refresh=4)
    assert lrdmc_is_specialized(gpu.ctx)
    gpu.close()
    _, gpu, _ = _pair("ar", 4, "single", refresh=4)
    assert not lrdmc_is_specialized(gpu.ctx)
    gpu.close()


@pytest.mark.parametrize("mode", ["pade", "single"])
def test_exact_hydrogenic_trial_function(mode):
    """Psi = exp(-Z r): every local energy is -Z^2/2, all weights are equal
    and the reconfiguration is the identity, in both modes."""
    from paper_1909_01589_amd.lrdmc import LRDMC
    Z, W = 2.0, 32
    s = inputs.hydrogenic(Z)
    kw = dict(switch_form=1, grids=2) if mode == "pade" else dict(switch_form=0, grids=1)
    rc, ap = spacing.spacing_pade(Z, 0.15) if mode == "pade" else (1.0, 0.15)
    gpu = LRDMC(s, 0.15, ap, rc, 0.05, W, seed=2, **kw)
    gpu.set_walkers(inputs.initial_walkers(s, W, 2) * 0.5, 0)
    out = gpu.run(5, want_idx=True)
    assert np.allclose(out["ebar"].cpu().numpy(), -Z * Z / 2, rtol=1e-12)
    assert np.all(out["idx"].cpu().numpy() == np.arange(W)[None, :])
    gpu.close()


def test_spacing_scan_on_helium():
    """The paper's spacing scan through the GPU path on helium with a nodeless
    trial function (fixed node exact), for the three lattice schemes:
    * the single/double move-rate ratio follows Eq. (5) with the sampled
      N_core = <sum_i p(r_i)> (within 5 %; O(a) terms from rho != 1);
    * E0 of the fit E0 + k1 a^2 + k2 a^4 agrees with the exact helium energy
      within 4 sigma in every scheme."""
    import os
    import sys
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import bench
    res = bench.ascan()["ascan"]
    for mode, lst in res["speedup"].items():
        for x in lst:
            print(f"ascan speedup {mode} alpha={x['alpha']} measured={x['measured']:.4f} eq5={x['eq5']:.4f}",
                  flush=True)
            assert x["measured"] == pytest.approx(x["eq5"], rel=0.05)
    for mode, v in res["modes"].items():
        print(f"ascan {mode} E0={v['E0']:.6f} +- {v['sigma_E0']:.6f}", flush=True)
        assert abs(v["E0"] - bench.HE_EXACT) <= 4 * v["sigma_E0"]
        assert v["sigma_E0"] < 2e-3

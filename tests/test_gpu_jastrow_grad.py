"""GPU derivatives of the Jastrow exponent J and of the local energy with
respect to the Pade parameters (b_ee, b_en), through the C ABI:

* the kernel against the oracle's analytic gradient (itself pinned by
  finite differences of the oracle's J and E_L) and against the oracle's J and
  E_L, on several systems;
* the torch.autograd.Function against central finite differences of its own
  forward pass;
* parameters set on a context reach the projection (run parity with an oracle
  built with the same parameters);
* variance minimisation with the gradients lowers the variance of E_L;
* a non-finite position is reported with its walker slot.
"""
import dataclasses

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from parity_bars import check, record_bar, run_agrees  # noqa: E402
from oracle import spacing  # noqa: E402
from paper_1909_01589_amd import inputs  # noqa: E402


def _system(name):
    return {"be": inputs.be_like(0), "tiny": inputs.tiny_mixed(seed=3, n_up=3, n_dn=2),
            "ar": inputs.ar_like(0), "helium": inputs.helium_nodeless(),
            "molecule": inputs.molecule(0)}[name]


def _engine(s, W, b_ee=None, b_en=None, **kw):
    from paper_1909_01589_amd.lrdmc import LRDMC
    g = LRDMC(s, 0.1, 0.15, 0.3, 0.01, W, **kw)
    if b_ee is not None:
        g.set_jastrow(b_ee, b_en)
    return g


@pytest.mark.parametrize("name,W", [("be", 16), ("tiny", 8), ("ar", 6), ("helium", 16), ("molecule", 2)])
def test_kernel_matches_oracle(name, W):
    s = dataclasses.replace(_system(name), b_ee=0.8, b_en=1.3)
    g = _engine(s, W)
    pos = inputs.initial_walkers(s, W, 31)
    out = g.jastrow_grad(pos).cpu().numpy()
    o = oracle.Oracle(s, a=0.1, a_prime=0.15, r_c=0.3)
    for w in range(W):
        print(f"jastrow grad case={name} walker={w}", flush=True)
        el, lap, _ = o.local_energy(pos[w])
        dJ, dE = o.jastrow_param_grad(pos[w])
        assert abs(out[w, 0] - el) <= 1e-9 * (1 + abs(el) + abs(lap))
        assert out[w, 1] == pytest.approx(o.jastrow(pos[w]), rel=1e-12, abs=1e-12)
        assert np.allclose(out[w, 2:4], dJ, rtol=1e-11, atol=1e-12)
        assert np.all(np.abs(out[w, 4:6] - dE) <= 1e-9 * (1 + np.abs(dE) + abs(lap)))
    g.close()


def test_autograd_matches_finite_differences():
    from paper_1909_01589_amd.jastrow import jastrow_and_local_energy
    s = inputs.tiny_mixed(seed=3, n_up=2, n_dn=2)
    W = 32
    g = _engine(s, W)
    pos = torch.as_tensor(inputs.initial_walkers(s, W, 8), device=g.device)
    wts = torch.linspace(0.5, 1.5, W, dtype=torch.float64, device=g.device)

    def loss(theta):
        j, e = jastrow_and_local_energy(theta, g, pos)
        return (wts * (e * e + 3.0 * j)).sum() / W

    theta = torch.tensor([0.9, 1.2], dtype=torch.float64, requires_grad=True)
    (grad,) = torch.autograd.grad(loss(theta), theta)
    for t in range(2):
        fd = []
        for h in (1e-3, 5e-4):
            tp, tm = theta.detach().clone(), theta.detach().clone()
            tp[t] += h
            tm[t] -= h
            fd.append(float((loss(tp) - loss(tm)) / (2 * h)))
        rich = (4 * fd[1] - fd[0]) / 3
        assert float(grad[t]) == pytest.approx(rich, rel=1e-6)
    g.close()


def test_parameters_reach_the_projection():
    s = inputs.be_like(0)
    rc, ap, _ = spacing.spacing(4, 0.2)
    from paper_1909_01589_amd.lrdmc import LRDMC
    W = 32
    g = LRDMC(s, 0.2, ap, rc, 0.0161, W, seed=4, refresh=3)
    pos = inputs.initial_walkers(s, W, 2)
    g.set_walkers(pos, 0)
    g.run(2)                        # state stored with the original parameters
    g.set_jastrow(0.6, 1.7)
    mid = g.get_walkers()["pos"].cpu().numpy()
    g.set_walkers(mid, 2)
    out = g.run(4, want_idx=True)
    o = oracle.Oracle(dataclasses.replace(s, b_ee=0.6, b_en=1.7), 0.2, ap, rc, tau=0.0161, seed=4)
    ref = o.run(mid, 4, gen0=2)
    n = run_agrees("run after set_jastrow", out["n_moves"].cpu().numpy(), out["idx"].cpu().numpy(), ref)
    e = out["ebar"].cpu().numpy()
    check("run ebar (new Pade parameters)", e[:n], ref["ebar"][:n], record_bar(ref["ebar"][:n]),
          scale=np.abs(ref["ebar"][:n]))
    g.close()


def test_variance_minimisation_lowers_the_variance():
    """Adam on theta from a poor start, configurations fixed (drawn once from
    a short projection at theta0): the weighted variance of E_L drops."""
    from paper_1909_01589_amd.jastrow import jastrow_and_local_energy, weighted_variance
    s = inputs.helium_nodeless()
    W = 4096
    from paper_1909_01589_amd.lrdmc import LRDMC
    g = LRDMC(s, 0.2, 0.2, 1.0, 0.02, W, seed=1, refresh=4)
    theta0 = torch.tensor([3.0, 3.0], dtype=torch.float64)
    g.set_jastrow(3.0, 3.0)
    g.set_walkers(inputs.initial_walkers(s, W, 3), 0)
    g.run(30)
    pos = g.get_walkers()["pos"].clone()
    with torch.no_grad():
        j0, _ = jastrow_and_local_energy(theta0, g, pos)
    theta = theta0.clone().requires_grad_(True)
    opt = torch.optim.Adam([theta], lr=0.1)
    v_start = None
    for step in range(40):
        opt.zero_grad()
        var, _ = weighted_variance(theta, g, pos, j0)
        if v_start is None:
            v_start = float(var.detach())
        var.backward()
        opt.step()
        with torch.no_grad():
            theta.clamp_(min=0.05)
    v_end = float(weighted_variance(theta.detach(), g, pos, j0)[0])
    print(f"variance {v_start:.5f} -> {v_end:.5f} at theta {theta.detach().tolist()}", flush=True)
    assert v_end < 0.7 * v_start
    g.close()


def test_non_finite_position_is_reported():
    from paper_1909_01589_amd.lrdmc import LRDMCError
    s = inputs.be_like(0)
    g = _engine(s, 8)
    pos = inputs.initial_walkers(s, 8, 0)
    pos[3, 0, 1] = np.inf
    with pytest.raises(LRDMCError) as e:
        g.jastrow_grad(pos)
    assert e.value.code == -3 and "slot 3" in str(e.value)
    g.close()

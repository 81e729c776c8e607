"""The reconfiguration entry point that allocates nothing
(lrdmc_reconfigure_noalloc, scratch in the library's fixed device array)
against the allocating one (lrdmc_reconfigure) through the C ABI: two calls
in a row, the second on a smaller population, each with identical indices
and generation record; a non-finite weight is reported and the next call is
clean again (the error flag in the shared array is cleared by every call);
populations beyond the array are refused before any device work."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _pair_call(lw, el, xi):
    from paper_1909_01589_amd.lrdmc import lrdmc_reconfigure, lrdmc_reconfigure_noalloc
    W = lw.numel()
    idx_a = torch.empty(W, dtype=torch.int32, device="cuda")
    idx_b = torch.full((W,), -1, dtype=torch.int32, device="cuda")
    st_a = torch.empty(2, dtype=torch.float64, device="cuda")
    st_b = torch.full((2,), np.nan, dtype=torch.float64, device="cuda")
    lrdmc_reconfigure_noalloc(lw, el, xi, idx_b, st_b)
    lrdmc_reconfigure(lw, el, xi, idx_a, st_a)
    return idx_a.cpu().numpy(), idx_b.cpu().numpy(), st_a.cpu().numpy(), st_b.cpu().numpy()


def test_noalloc_reconfigure_matches_the_allocating_entry_point():
    rng = np.random.default_rng(7)
    for W in (65536, 1000):
        print(f"no-alloc reconfigure W={W}", flush=True)
        lw = torch.tensor(rng.normal(size=W) * 1.5, device="cuda")
        el = torch.tensor(rng.normal(size=W) - 5.0, device="cuda")
        xi = float(rng.uniform())
        ia, ib, sa, sb = _pair_call(lw, el, xi)
        assert np.array_equal(ia, ib)
        assert np.array_equal(sa, sb)
        assert np.all(np.diff(ib) >= 0) and ib[-1] < W


def test_noalloc_reconfigure_errors():
    from paper_1909_01589_amd.lrdmc import LRDMCError, NOALLOC_MAX_WALKERS, lrdmc_reconfigure_noalloc
    W = 512
    lw = torch.zeros(W, dtype=torch.float64, device="cuda")
    lw[7] = float("nan")
    el = torch.zeros(W, dtype=torch.float64, device="cuda")
    idx = torch.empty(W, dtype=torch.int32, device="cuda")
    with pytest.raises(LRDMCError) as e:
        lrdmc_reconfigure_noalloc(lw, el, 0.5, idx)
    assert e.value.code == -3
    lw[7] = 0.0
    lrdmc_reconfigure_noalloc(lw, el, 0.5, idx)          # the flag is clean again
    assert np.array_equal(idx.cpu().numpy(), np.arange(W))
    big = NOALLOC_MAX_WALKERS + 1
    lwb = torch.zeros(big, dtype=torch.float64, device="cuda")
    idxb = torch.empty(big, dtype=torch.int32, device="cuda")
    with pytest.raises(LRDMCError) as e:
        lrdmc_reconfigure_noalloc(lwb, lwb, 0.5, idxb)
    assert e.value.code == -1

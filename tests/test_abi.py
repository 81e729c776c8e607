"""The C-ABI library loads on the CPU and exports every declared symbol; its
host-side logic (parameter choice, argument validation) is checked without a
GPU.  No kernel is launched here."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from oracle import spacing
from paper_1909_01589_amd import inputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lrdmc.h")


@pytest.fixture(scope="module")
def lib():
    from paper_1909_01589_amd import lrdmc
    return lrdmc.load()


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lrdmc_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ("lrdmc_create", "lrdmc_project", "lrdmc_branch", "lrdmc_run", "lrdmc_eval_moves",
              "lrdmc_reconfigure", "lrdmc_spacing", "lrdmc_destroy"):
        assert n in names


def test_library_exports_every_declared_symbol(lib):
    from paper_1909_01589_amd import lrdmc
    for name in declared_functions():
        assert hasattr(lib, name), name
    assert set(declared_functions()) == set(lrdmc.EXPORTS)


@pytest.mark.parametrize("Z,a", [(4, 0.2), (4, 0.075), (10, 1 / 35), (18, 0.2), (18, 0.1), (36, 1 / 126),
                                 (54, 1 / 189), (8, 1 / 28)])
def test_spacing_matches_oracle(lib, Z, a):
    from paper_1909_01589_amd.lrdmc import lrdmc_spacing
    rc, ap, nc = lrdmc_spacing(Z, a)
    rc_o, ap_o, nc_o = spacing.spacing(Z, a)
    assert rc == pytest.approx(rc_o, rel=1e-14)
    assert nc == pytest.approx(nc_o, rel=1e-8)
    assert ap == pytest.approx(ap_o, rel=1e-8)


def test_spacing_rejects_bad_arguments(lib):
    from paper_1909_01589_amd.lrdmc import LRDMCError, lrdmc_spacing
    for Z, a in ((0.5, 0.1), (4, 0.0), (4, -1.0), (100, 0.1)):
        with pytest.raises(LRDMCError) as e:
            lrdmc_spacing(Z, a)
        assert e.value.code == -1


@pytest.mark.parametrize("bad", [
    dict(a_prime=0.1),        # a' < a
    dict(a=0.0),
    dict(r_c=0.0),
    dict(tau=0.0),
    dict(z_heavy=99.0),       # no heavy nucleus
    dict(n_walkers=0),
])
def test_create_validates_before_touching_the_device(lib, bad):
    """Invalid parameters are refused on the host with EINVAL."""
    from paper_1909_01589_amd.lrdmc import LRDMCError, lrdmc_create
    kw = dict(a=0.2, a_prime=0.28, r_c=0.44, tau=0.02, n_walkers=8, z_heavy=None)
    kw.update(bad)
    with pytest.raises(LRDMCError) as e:
        lrdmc_create(inputs.be_like(0), kw["a"], kw["a_prime"], kw["r_c"], kw["tau"], kw["n_walkers"],
                     kw["z_heavy"])
    assert e.value.code == -1


def test_create_validates_system_sizes(lib):
    from paper_1909_01589_amd.lrdmc import LRDMCError, lrdmc_create
    s = inputs.be_like(0)
    bad_l = inputs.System(Z=s.Z, R=s.R, n_up=2, n_dn=2, shell_nuc=s.shell_nuc, shell_l=np.full(8, 3),
                          shell_alpha=s.shell_alpha, mo=s.mo)
    too_few_orb = inputs.System(Z=s.Z, R=s.R, n_up=3, n_dn=2, shell_nuc=s.shell_nuc, shell_l=s.shell_l,
                                shell_alpha=s.shell_alpha, mo=s.mo)
    for sysm in (bad_l, too_few_orb):
        with pytest.raises(LRDMCError) as e:
            lrdmc_create(sysm, 0.2, 0.3, 0.4, 0.02, 4)
        assert e.value.code == -1


def test_product_does_not_reach_the_oracle():
    """The HIP path must not import or load the CPU oracle."""
    pkg = os.path.join(ROOT, "paper_1909_01589_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "from oracle" not in text, f
                assert "lrdmc_oracle" not in text, f


def test_binding_refuses_host_tensors(lib):
    import torch
    from paper_1909_01589_amd.lrdmc import _dptr
    with pytest.raises(ValueError):
        _dptr(torch.zeros(3, dtype=torch.float64))


def test_network_sizes_and_validation(lib):
    """lrdmc_net_*: sizes, and every argument check returns EINVAL before any
    device work (the pointers below are never dereferenced)."""
    assert lib.lrdmc_net_param_count(64) == 64 * 64 + 4 * 64 + 1
    assert lib.lrdmc_net_param_count(0) == 0 and lib.lrdmc_net_param_count(257) == 0
    assert lib.lrdmc_net_workspace_size(64, 257) == 2 * 257 * (9 * 64 + 1)
    for h, g in ((64, 1), (0, 10), (64, 4097), (300, 10)):
        assert lib.lrdmc_net_workspace_size(h, g) == 0
    dummy = C.c_void_p(64)
    for args in ((None, 8, 9, 1.0, dummy), (dummy, 8, 9, 1.0, None), (dummy, 0, 9, 1.0, dummy),
                 (dummy, 8, 1, 1.0, dummy), (dummy, 8, 4097, 1.0, dummy), (dummy, 8, 9, 0.0, dummy),
                 (dummy, 8, 9, float("nan"), dummy), (dummy, 8, 9, float("inf"), dummy)):
        assert lib.lrdmc_net_tabulate(*args, None) == -1
        assert lib.lrdmc_net_tabulate_backward(args[0], args[1], args[2], args[3], dummy, args[4], dummy,
                                               None) == -1
    assert lib.lrdmc_net_tabulate_backward(dummy, 8, 9, 1.0, dummy, dummy, None, None) == -1


def test_context_entry_points_reject_null(lib):
    dummy = C.c_void_p(64)
    assert lib.lrdmc_vmc(None, 10, 0.3, None) == -1
    assert lib.lrdmc_set_jastrow_table(None, dummy, 9, 1.0, 0, None) == -1
    assert lib.lrdmc_jastrow_table_grad(None, dummy, None, None, dummy, None) == -1
    assert lib.lrdmc_jastrow_grad(None, dummy, dummy, None) == -1
    assert lib.lrdmc_set_jastrow(None, 1.0, 1.0) == -1
    assert lib.lrdmc_use_generic(None, 0) == -1
    assert lib.lrdmc_set_precision(None, 1) == -1
    assert lib.lrdmc_is_specialized(None) == 0
    assert lib.lrdmc_set_collapse_threshold(None, 0.01) == -1
    assert lib.lrdmc_set_move_cap(None, 10) == -1
    assert lib.lrdmc_inverse_residual(None, dummy, None) == -1

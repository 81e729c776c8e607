"""Host-side helpers (CPU): the E(a) fits and the sampled N_core of the
benchmark modes, and the packing of the network parameters."""
import numpy as np
import pytest

import bench


def test_fit_e0_recovers_a_polynomial():
    a = np.array([0.06, 0.045, 0.035, 0.025, 0.0175])
    E = -520.4 + 300.0 * a ** 2 - 2.0e4 * a ** 4
    sig = np.full(a.size, 0.01)
    E0, s0, chi2 = bench._fit_e0(a, E, sig)
    assert E0 == pytest.approx(-520.4, abs=1e-9)
    assert chi2 == pytest.approx(0.0, abs=1e-12)
    E0l, s0l, _ = bench._fit_e0_linear(a[2:], -1.0 + 5.0 * a[2:] ** 2, sig[2:])
    assert E0l == pytest.approx(-1.0, abs=1e-12)
    # the error of E0 grows with the error bars
    assert bench._fit_e0(a, E, 2 * sig)[1] == pytest.approx(2 * s0, rel=1e-12)


def test_switch_sum_counts_core_electrons():
    R = np.zeros(3)
    pos = np.zeros((4, 3, 3))
    pos[:, 1, 0] = 10.0          # far electron: p = 0
    pos[:, 2, 0] = 0.1           # near electron: p = exp(-0.01 / (2 r_c^2))
    rc = 0.2
    got = bench._switch_sum(pos, R, rc, 0)
    assert got == pytest.approx(1.0 + 0.0 + np.exp(-0.01 / (2 * rc * rc)), rel=1e-14)
    got_pade = bench._switch_sum(pos, R, rc, 1)
    assert got_pade == pytest.approx(1.0 + 1.0 / (1 + rc * rc * 100.0) + 1.0 / (1 + rc * rc * 0.01), rel=1e-14)


def test_network_packing_round_trip():
    from paper_1909_01589_amd import inputs, neural
    w = inputs.neural_weights(seed=2, hidden=16)
    flat = neural.pack(w)
    assert flat.shape == (2, 16 * 16 + 4 * 16 + 1)
    back = neural.unpack(flat, 16)
    for kind in ("ee", "en"):
        for k, v in w[kind].items():
            assert np.array_equal(np.asarray(back[kind][k]), np.asarray(v))
    with pytest.raises(ValueError):
        bad = {k: dict(v) for k, v in w.items()}
        bad["ee"]["W2"] = np.zeros((16, 15))
        neural.pack(bad)


def test_bench_refuses_more_than_one_gpu():
    """bench.py --gpus N with N > 1 exits with a message, before touching a GPU."""
    import subprocess
    import sys
    r = subprocess.run([sys.executable, "bench.py", "--gpus", "2", "--steps", "1", "--warmup", "0"],
                       cwd=bench.ROOT, capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "exactly one GPU" in r.stderr


def test_bench_source_hash_is_stable():
    import subprocess
    import sys
    a = subprocess.run([sys.executable, "bench.py", "--source-hash"], cwd=bench.ROOT, capture_output=True, text=True,
                       timeout=120)
    assert a.returncode == 0 and len(a.stdout.strip()) == 64
    assert a.stdout.strip() == bench.kernel_source_hash()


def test_work_model_counts_by_hand():
    """One electron, one s function, one nucleus: a table entry is 15 (points)
    + 8 + 2 (switch) + 2 (k) + 13 (one group: 12 + s polynomial 1) + 14 (one
    Pade pair) + 3 (Jastrow exp) + 3 (T) = 60 operations, 12 moves and the
    cumulative sum: 12 * 60 + 24; launches add tables, accepts and starts."""
    from paper_1909_01589_amd import inputs, workcount
    s = workcount.shape_of(inputs.hydrogenic(1.0))
    assert (s.N, s.K, s.n_nuc, s.n_heavy, s.groups) == (1, 1, 1, 1, [(0,)])
    t = workcount.table_ops(s)
    assert t == 12 * 60 + 24
    a, g = workcount.accept_ops(s), workcount.setup_ops(s)
    assert workcount.projection_ops(s, 10, 7, 3) == 3 * g + 17 * t + 7 * a


def test_positions_are_checked_before_a_pointer_is_passed():
    """The C entry points take bare device pointers, so the binding checks the
    walker positions' shape against the context (W, N) before every call;
    here on an instance without a device context."""
    from paper_1909_01589_amd.lrdmc import LRDMC
    eng = object.__new__(LRDMC)
    eng.W, eng.N, eng.device = 4, 3, "cpu"
    t = eng.positions(np.zeros((4, 3, 3)))
    assert t.dtype.is_floating_point and tuple(t.shape) == (4, 3, 3) and t.is_contiguous()
    for bad in (np.zeros((3, 3, 3)), np.zeros((4, 2, 3)), np.zeros((4, 3))):
        with pytest.raises(ValueError):
            eng.positions(bad)


def test_table_s1_accelerations_quoted_by_the_bench_match_the_fixture():
    """The acceleration column the single/double comparison prints beside its
    measured move-rate ratios is the one transcribed (with its citation) in
    tests/golden/table_s1.txt."""
    import os
    rows = np.loadtxt(os.path.join(os.path.dirname(__file__), "golden", "table_s1.txt"))
    names = {4: "Be", 10: "Ne"}
    for (atom, alpha), acc in bench.TABLE_S1_ACCELERATION.items():
        hit = [r for r in rows if names.get(int(r[0])) == atom and abs(r[2] - alpha) < 1e-9]
        assert len(hit) == 1, (atom, alpha)
        assert hit[0][3] == acc


def test_fit_poly_closed_forms():
    """_fit_poly (the E(a) models of the learned-Jastrow comparison): exact
    polynomial data give their constant term with chi2 = 0; with no powers
    the fit is the weighted mean with error 1 / sqrt(sum w); with powers
    (2, 4) it is the fit of _fit_e0."""
    a = np.array([0.06, 0.045, 0.035, 0.025, 0.0175, 0.0125])
    sig = np.array([0.02, 0.01, 0.014, 0.012, 0.017, 0.0125])
    E = -520.1 - 12.0 * a + 90.0 * a ** 2 - 700.0 * a ** 3
    E0, s0, chi2, dof = bench._fit_poly(a, E, sig, (1, 2, 3))
    assert E0 == pytest.approx(-520.1, abs=1e-9)
    assert chi2 == pytest.approx(0.0, abs=1e-12)
    assert dof == a.size - 4
    y = np.array([1.0, 2.0, 4.0])
    s = np.array([1.0, 2.0, 0.5])
    w = 1.0 / s ** 2
    m, sm, c2, d = bench._fit_poly(np.array([0.1, 0.2, 0.3]), y, s, ())
    assert m == pytest.approx(np.sum(w * y) / np.sum(w), rel=1e-14)
    assert sm == pytest.approx(1.0 / np.sqrt(np.sum(w)), rel=1e-14)
    assert c2 == pytest.approx(np.sum(w * (y - m) ** 2) / 2, rel=1e-12)
    assert d == 2
    Eq = -520.4 + 300.0 * a ** 2 - 2.0e4 * a ** 4 + np.array([1, -1, 1, -1, 1, -1]) * sig
    assert bench._fit_poly(a, Eq, sig, (2, 4))[:3] == pytest.approx(bench._fit_e0(a, Eq, sig), rel=1e-12)


def test_tsigma_summary_hand_computed():
    """tsigma_summarize on two seeds per form: time to 1 mHa = mean(c) mean(v)
    / 1e-6; the ratio's 95 % interval from the delta method on log c and
    log v (here only v scatters: se(v) = 1 at v = 4 for both forms, so the
    half-width in log is 1.96 sqrt(2) / 4); the paired ratio of identical
    per-seed ratios has no spread; the energy is the inverse-variance mean."""
    def run(seed, c, v, E, sg):
        return dict(seed=seed, c=c, v=v, E=E, sigma=sg, moves_per_s=1.0, ess_min=0.5)
    runs = {"fp64": [run(0, 2.0, 3.0, 1.0, 1.0), run(1, 2.0, 5.0, 2.0, 1.0)],
            "mixed": [run(0, 1.0, 3.0, 1.5, 1.0), run(1, 1.0, 5.0, 1.5, 1.0)]}
    res = bench.tsigma_summarize(runs)
    f = res["forms"]["fp64"]
    assert f["time_to_1mHa_s"] == pytest.approx(2.0 * 4.0 / 1e-6, rel=1e-14)
    assert f["v_se"] == pytest.approx(1.0, rel=1e-14)
    assert f["E"] == pytest.approx(1.5, rel=1e-14)
    assert f["E_sigma"] == pytest.approx(1.0 / np.sqrt(2.0), rel=1e-14)
    assert f["E_scatter_chi2_dof"] == pytest.approx(0.5, rel=1e-14)
    q = res["against_fp64"]["mixed"]
    assert q["ratio"] == pytest.approx(2.0, rel=1e-14)
    assert q["speed_ratio"] == pytest.approx(2.0, rel=1e-14)
    assert q["variance_ratio"] == pytest.approx(1.0, rel=1e-14)
    half = 1.96 * np.sqrt(2.0) / 4.0
    assert q["ci95"] == pytest.approx([2.0 * np.exp(-half), 2.0 * np.exp(half)], rel=1e-12)
    assert q["paired"]["ratio"] == pytest.approx(2.0, rel=1e-14)
    assert q["paired"]["ci95"] == pytest.approx([2.0, 2.0], rel=1e-14)
    assert q["dE"] == pytest.approx(0.0, abs=1e-14)


def test_neural_summary_ratios_and_limits():
    """neural_summarize: per-spacing time ratios Pade / neural, each form's
    E0 from E0 + k a^2 (three spacings), and the difference of the limits."""
    a = [0.3, 0.2, 0.1]
    rows = [dict(form="pade", a=x, E=-2.9 + 0.5 * x * x, sigma=1e-3, t_1mHa_s=t) for x, t in zip(a, (30.0, 20.0, 10.0))]
    rows += [dict(form="neural", a=x, E=-2.8 + 0.2 * x * x, sigma=1e-3, t_1mHa_s=t) for x, t in zip(a, (10.0, 10.0, 5.0))]
    out = bench.neural_summarize(rows)
    assert out["lrdmc"]["pade"]["fit"] == "E0 + k1 a^2"
    assert out["lrdmc"]["pade"]["E0"] == pytest.approx(-2.9, abs=1e-12)
    assert out["lrdmc"]["neural"]["E0"] == pytest.approx(-2.8, abs=1e-12)
    assert out["E0_difference"] == pytest.approx(0.1, abs=1e-12)
    assert out["time_to_1mHa_ratio_pade_over_neural"] == pytest.approx({"0.3": 3.0, "0.2": 2.0, "0.1": 2.0}, rel=1e-14)


def test_traffic_record_follows_the_source_hash(monkeypatch):
    """The bench line's HBM traffic comes from the committed counter record
    only while the kernel sources hash to the recorded value; any other
    hash gives None (the counters no longer describe the kernel)."""
    import re
    text = open(bench.os.path.join(bench.ROOT, "profiles", "traffic_project_kernel.md")).read()
    recorded = re.search(r"^source_sha256 = ([0-9a-f]{64})$", text, re.M).group(1)
    mol = float(re.search(r"^molecule bytes_per_launch = ([0-9.eE+]+)$", text, re.M).group(1))
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: recorded)
    assert bench._traffic_record("molecule") == mol > 0
    assert bench._traffic_record("no_such_workload") is None
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "0" * 64)
    assert bench._traffic_record("molecule") is None

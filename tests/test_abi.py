"""Host-side checks of the C-ABI library: it loads, exports every symbol the
header declares, validates arguments without a device, and its configuration
selection engine follows the same rules as the oracle's.  CPU only."""
import os
import random
import re

import pytest

from oracle import tuner as orc_tuner
from oracle.tuner import EXPERT, FULL_SEARCH, PREDICTIVE, TunerOracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def M():
    from paper_2505_03438_amd import mdlj
    if not os.path.exists(mdlj.LIB_PATH):
        from paper_2505_03438_amd import build
        build.build(verbose=False)
    mdlj.lib()
    return mdlj


def _declared():
    txt = open(os.path.join(ROOT, "include", "mdlj.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(md_[a-z_]+)\s*\(", txt)))


def test_exports_every_declared_symbol(M):
    names = _declared()
    assert len(names) >= 20
    L = M.lib()
    for name in names:
        assert hasattr(L, name), name
    assert set(names) == set(M._SIGS), "binding and header disagree"


def test_config_default(M):
    c = M.config_default(1000, 12.0)
    assert c.n == 1000 and list(c.box) == [12.0] * 3 and c.rc2[0] == 6.25
    assert c.skin == 0.3 and c.csf == 1.0 and c.rebuild_interval == 10
    assert c.container == M.MD_CONTAINER_VL and c.precision == M.MD_FP32


def _create_rc(M, c):
    import ctypes
    h = ctypes.c_void_p()
    rc = M.lib().md_create(ctypes.byref(c), ctypes.byref(h))
    if rc == 0:
        M.lib().md_destroy(h)
    return rc


def test_create_rejects_bad_configs(M):
    c = M.config_default(100, 12.0)
    assert c.tune_skin == 0
    c.tune_skin = 2
    assert _create_rc(M, c) == M.MD_ERR_INVALID_ARG and "tune_skin" in M.md_last_error()
    c.tune_skin = 0
    c.box[1] = 5.0  # < 2 (r_c + skin)
    assert _create_rc(M, c) == M.MD_ERR_BOX_TOO_SMALL
    assert "box[1]" in M.md_last_error()
    for field, val in (("n_types", 3), ("csf", 0.3), ("rebuild_interval", 0), ("precision", 7),
                       ("container", 9), ("skin", -1.0), ("max_neighbors", 0)):
        c = M.config_default(100, 12.0)
        setattr(c, field, val)
        assert _create_rc(M, c) == M.MD_ERR_INVALID_ARG, field
    c = M.config_default(100, 12.0)
    c.n_types = 2
    c.rc2[1] = 5.0  # rc2[0][1] != rc2[1][0]
    assert _create_rc(M, c) == M.MD_ERR_INVALID_ARG
    assert "symmetric" in M.md_last_error()


def test_batch_counters_null(M):
    assert M.lib().md_batch_get_counters(None, None) == M.MD_ERR_INVALID_ARG


def test_batch_create_rejects_unsupported_configs(M):
    """md_batch_create checks its configuration before it touches a device:
    linked cells or (FP32, systems of at most 65536 particles) Verlet lists,
    gather-only; the reason is in md_last_error."""
    import ctypes
    import numpy as np

    def rc_of(cfg, offs, boxes):
        b = ctypes.c_void_p()
        offs = np.ascontiguousarray(offs, dtype=np.int64)
        boxes = np.ascontiguousarray(boxes, dtype=np.float64)
        rc = M.lib().md_batch_create(ctypes.byref(cfg), len(offs) - 1, ctypes.c_void_p(offs.ctypes.data),
                                     ctypes.c_void_p(boxes.ctypes.data), ctypes.byref(b))
        if rc == 0:
            M.lib().md_batch_destroy(b)
        return rc

    offs, boxes = [0, 500, 900], [[9.0] * 3, [8.0] * 3]
    for container, newton3, prec, what in ((M.MD_CONTAINER_CL, 0, M.MD_FP32, "linked cells or Verlet lists"),
                                          (M.MD_CONTAINER_LC, 1, M.MD_FP32, "gather-only"),
                                          (M.MD_CONTAINER_VL, 0, M.MD_FP64, "FP32")):
        c = M.config_default(900, 9.0)
        c.container, c.newton3, c.precision = container, newton3, prec
        assert rc_of(c, offs, boxes) == M.MD_ERR_INVALID_ARG
        assert what in M.md_last_error()
    c = M.config_default(70000, 40.0)
    c.container, c.precision = M.MD_CONTAINER_VL, M.MD_FP32
    assert rc_of(c, [0, 70000], [[40.0] * 3]) == M.MD_ERR_INVALID_ARG
    assert "65536" in M.md_last_error()


@pytest.mark.skipif(os.environ.get("HIP_VISIBLE_DEVICES") is None and os.path.exists("/dev/kfd"),
                    reason="a device may be present")
def test_create_without_device_fails_cleanly(M):
    c = M.config_default(100, 12.0)
    assert _create_rc(M, c) == M.MD_ERR_NO_DEVICE


def _drive(strategy, n, phases, scores, M):
    """Run the library tuner and the oracle on the same score table."""
    lib_t = M.Tuner(strategy, n, phases)
    orc_t = TunerOracle(strategy, n, phases)
    for p in range(phases):
        a = lib_t.begin_phase()
        b = orc_t.begin_phase()
        assert a == b, (p, a, b)
        for c in a:
            lib_t.report(c, scores[p][c])
            orc_t.report(c, scores[p][c])
        assert lib_t.end_phase() == orc_t.end_phase()
        assert lib_t.blacklisted() == [c for c in range(n) if orc_t.blacklisted[c]]


def test_tuner_matches_oracle_on_hand_trace(M):
    import json
    t = json.load(open(os.path.join(ROOT, "tests", "golden", "tuner_predictive_trace.json")))
    tu = M.Tuner(t["strategy"], t["n_configs"], t["total_phases"])
    for ph in t["phases"]:
        assert tu.begin_phase() == ph["trial"]
        for c in ph["trial"]:
            tu.report(c, ph["scores"][str(c)])
        assert tu.end_phase() == ph["chosen"]
        assert tu.blacklisted() == ph["blacklisted_after"]


@pytest.mark.parametrize("strategy", [FULL_SEARCH, PREDICTIVE])
def test_tuner_matches_oracle_on_random_traces(M, strategy):
    rng = random.Random(1234 + strategy)
    for trial in range(40):
        n = rng.randint(1, 12)
        phases = rng.randint(1, 12)
        base = [rng.uniform(1.0, 30.0) for _ in range(n)]
        drift = [rng.uniform(-2.0, 2.0) for _ in range(n)]
        scores = [[max(0.01, base[c] + drift[c] * p + rng.uniform(-1, 1)) for c in range(n)]
                  for p in range(phases)]
        # occasional ties
        if n > 1 and trial % 5 == 0:
            for p in range(phases):
                scores[p][1] = scores[p][0]
        _drive(strategy, n, phases, scores, M)


def _random_rules(rng, n_configs):
    inf = float("inf")
    rules = []
    for _ in range(rng.randint(1, 12)):
        ants = []
        for _ in range(rng.choice((1, 1, 2))):
            pts = sorted(rng.uniform(0.0, 10.0) for _ in range(4))
            if rng.random() < 0.2:
                pts[0] = pts[1] = -inf
            if rng.random() < 0.2:
                pts[2] = pts[3] = inf
            if rng.random() < 0.1:
                pts[1] = pts[2]  # triangle
            ants.append((rng.randrange(8), tuple(pts)))
        rules.append({"if": ants, "config": rng.randrange(n_configs), "then": rng.randrange(3)})
    return rules


def test_expert_suitability_matches_oracle(M):
    """The library's exact piecewise-linear centre of gravity against the
    oracle's fine-grid integral, on random rule sets and statistics."""
    rng = random.Random(2505)
    for trial in range(60):
        n = rng.randint(1, 8)
        rules = _random_rules(rng, n)
        stats = [rng.uniform(0.0, 10.0) for _ in range(8)]
        got = M.md_expert_suitability(stats, n, rules)
        want = orc_tuner.suitability(rules, stats, n)
        for c in range(n):
            assert abs(got[c] - want[c]) < 1e-8, (trial, c, got[c], want[c])
        assert orc_tuner.expert_trial_set(want) == orc_tuner.expert_trial_set(got) or \
            any(abs(v - max(want) + 0.1) < 1e-8 for v in want)


def test_expert_rules_validated(M):
    inf = float("inf")
    ok = {"if": [(0, (-inf, -inf, 2.0, 4.0))], "config": 0, "then": M.MD_SUIT_GOOD}
    M.md_expert_suitability([1.0] * 8, 1, [ok])
    for bad in ({"if": [(8, (0, 1, 2, 3))], "config": 0, "then": 0},
                {"if": [(0, (0, 2, 1, 3))], "config": 0, "then": 0},
                {"if": [(0, (0, float("nan"), 1, 3))], "config": 0, "then": 0},
                {"if": [(0, (0, 1, 2, 3))], "config": 1, "then": 0},
                {"if": [(0, (0, 1, 2, 3))], "config": 0, "then": 3}):
        with pytest.raises(RuntimeError):
            M.md_expert_suitability([1.0] * 8, 1, [bad])


def test_builtin_expert_rules_select_families(M):
    """The built-in rules (mean particles per CSF-1 bin only): Verlet lists,
    gather-only, always; its N3L variant too at medium means; linked and
    cluster lists never while Verlet lists are suited."""
    def trials(mean):
        s = M.md_expert_suitability([mean, 0.2, mean, 2 * mean, 1e5, 0, 256, 0.3], 7)
        return orc_tuner.expert_trial_set(s)
    assert trials(0.9) == [4]      # droplet
    assert trials(17.7) == [4]     # 1M fluid at density 0.8
    assert trials(6.7) == [4, 5]   # fluid at density 0.3
    assert trials(5.95) == [4, 5]  # slab
    s64 = M.md_expert_suitability([17.7, 0.2, 17.7, 40, 1e5, 0, 256, 0.3], 6)  # FP64 space: no cluster lists
    assert orc_tuner.expert_trial_set(s64) == [4]


def test_expert_tuner_matches_oracle(M):
    rng = random.Random(77)
    for trial in range(30):
        n = rng.randint(1, 9)
        phases = rng.randint(1, 6)
        lib_t = M.Tuner(EXPERT, n, phases)
        orc_t = TunerOracle(EXPERT, n, phases)
        for p in range(phases):
            suit = [rng.choice((0.0, 1.0 / 6.0, 0.5, 0.75, 0.8, 5.0 / 6.0, rng.random())) for _ in range(n)]
            if trial % 7 == 0:
                suit = [0.0] * n
            lib_t.set_suitability(suit)
            a = lib_t.begin_phase()
            b = orc_t.begin_phase(suit)
            assert a == b, (trial, p, suit, a, b)
            for c in a:
                sc = rng.uniform(1.0, 20.0)
                lib_t.report(c, sc)
                orc_t.report(c, sc)
            assert lib_t.end_phase() == orc_t.end_phase()
            assert lib_t.blacklisted() == []
    with pytest.raises(RuntimeError):
        M.Tuner(EXPERT, 2, 2).set_suitability([0.5, 1.5])


def test_random_forest_matches_scikit_learn(M):
    """The library's tree evaluator against scikit-learn's predict for the
    same forest (refitted from the committed data with the same seed), on
    the training scenarios and on perturbed and random statistics; and the
    committed model header is the one that fit writes."""
    import tempfile

    import numpy as np
    from paper_2505_03438_amd import rf_train as R
    X, y = R.load()
    model = R.fit(X, y)
    rng = np.random.default_rng(5)
    rows = [X] + [X * np.exp(rng.normal(0.0, 0.6, size=X.shape)) for _ in range(10)]
    lo, hi = X.min(axis=0), X.max(axis=0)
    rows.append(lo + (hi - lo) * rng.random((500, X.shape[1])))
    XX = np.vstack(rows)
    want = model.predict(XX)
    got = np.array([M.md_rf_predict(x) for x in XX])
    assert np.array_equal(got, want)
    assert set(want) == {4, 6}  # both classes occur, so the test sees both paths
    with tempfile.TemporaryDirectory() as d:
        out = os.path.join(d, "rf_model.h")
        R.write_header(model, out)
        assert open(out).read() == open(R.OUT).read()


def test_random_forest_rejects(M):
    with pytest.raises(RuntimeError, match="NaN"):
        M.md_rf_predict([1.0, float("nan"), 1, 1, 1, 0, 256, 0.3])
    with pytest.raises(RuntimeError, match="no configuration"):
        M.md_rf_predict([32, 0, 32, 32, 27, 0, 256, 0.3], 4)  # classes are 4 and 6
    # with the cluster lists outside the space (FP64) the forest falls back to the other class
    assert M.md_rf_predict([2.32, 0.66, 2, 9, 729, 66, 256, 0.3], 7) == 6
    assert M.md_rf_predict([2.32, 0.66, 2, 9, 729, 66, 256, 0.3], 6) == 4


def test_tuner_rejects_bad_use(M):
    tu = M.Tuner(PREDICTIVE, 3, 4)
    tr = tu.begin_phase()
    with pytest.raises(RuntimeError):
        tu.end_phase()  # nothing reported
    with pytest.raises(RuntimeError):
        tu.report(7, 1.0)
    with pytest.raises(RuntimeError):
        tu.report(tr[0], float("nan"))


def test_probe_library_exports_its_header():
    """The measurement probe (libmdprobe.so) exports what include/mdprobe.h
    declares and counts its work without a device."""
    import ctypes
    from paper_2505_03438_amd import build
    if not os.path.exists(build.PROBE_LIB):
        build.build(verbose=False)
    txt = open(os.path.join(ROOT, "include", "mdprobe.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    names = sorted(set(re.findall(r"\b(mdprobe_[a-z0-9_]+)\s*\(", txt)))
    assert names == ["mdprobe_fma_f32", "mdprobe_fma_f32_flops"]
    L = ctypes.CDLL(build.PROBE_LIB)
    for name in names:
        assert hasattr(L, name), name
    L.mdprobe_fma_f32_flops.restype = ctypes.c_int64
    L.mdprobe_fma_f32_flops.argtypes = [ctypes.c_int32, ctypes.c_int32]
    assert L.mdprobe_fma_f32_flops(4096, 4096) == 4096 * 256 * 4096 * 8 * 2
    L.mdprobe_fma_f32.restype = ctypes.c_int
    L.mdprobe_fma_f32.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p]
    assert L.mdprobe_fma_f32(0, 1, None, None) == -1


def test_bench_config_takes_every_box_side(M):
    # the slab's box is 1:1:3; a cubic configuration would fold two thirds of
    # it onto the edge cells
    import sys
    sys.path.insert(0, ROOT)
    import bench
    for kind in ("auto", "plain", "fixed:vl:1:0:5"):
        c = bench.make_cfg(M, 1000, [12.0, 13.0, 39.0], kind, 100)
        assert list(c.box) == [12.0, 13.0, 39.0], kind

"""The selection-strategy oracle against a hand-computed trace (CPU only)."""
import json
import os

from oracle.tuner import FULL_SEARCH, PREDICTIVE, TunerOracle

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_predictive_hand_trace():
    t = json.load(open(os.path.join(GOLD, "tuner_predictive_trace.json")))
    tu = TunerOracle(t["strategy"], t["n_configs"], t["total_phases"])
    for ph in t["phases"]:
        assert tu.begin_phase() == ph["trial"]
        for c in ph["trial"]:
            tu.report(c, ph["scores"][str(c)])
        assert tu.end_phase() == ph["chosen"]
        assert [c for c in range(t["n_configs"]) if tu.blacklisted[c]] == ph["blacklisted_after"]


def test_full_search_trials_everything():
    tu = TunerOracle(FULL_SEARCH, 3, 4)
    for scores in ([5, 4, 100], [3, 4, 1]):
        assert tu.begin_phase() == [0, 1, 2]
        for c, s in enumerate(scores):
            tu.report(c, s)
        assert tu.end_phase() == scores.index(min(scores))
    assert not any(tu.blacklisted)


def test_predictive_clamps_falling_line():
    tu = TunerOracle(PREDICTIVE, 2, 100)
    for scores in ([10, 10], [10, 2]):
        tu.begin_phase()
        for c, s in enumerate(scores):
            tu.report(c, s)
        tu.end_phase()
    # config 1 falls 10 -> 2: the line predicts -6, clamped to 0.5 * 2 = 1
    tu.phase += 0
    assert tu.begin_phase() == [1]
    assert tu.predict(1) == 1.0

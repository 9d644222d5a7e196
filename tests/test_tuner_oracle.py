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


# ---------------------------------------------------------------- Expert (Sec. 5.2)

import math  # noqa: E402

import pytest  # noqa: E402

from oracle.tuner import (BAD, EXPERT, GOOD, OKAY, expert_trial_set, membership,  # noqa: E402
                          suitability)

INF = math.inf


def _rule(c, then, *ants):
    return {"if": list(ants), "config": c, "then": then}


def test_membership_corners_flanks_shoulders():
    t = (1.0, 3.0, 5.0, 9.0)
    for x, want in ((0.5, 0.0), (1.0, 0.0), (2.0, 0.5), (3.0, 1.0), (4.0, 1.0), (5.0, 1.0), (6.0, 0.75),
                    (9.0, 0.0), (12.0, 0.0)):
        assert membership(x, t) == want, x
    left = (-INF, -INF, 2.0, 4.0)
    right = (10.0, 14.0, INF, INF)
    assert membership(-1e300, left) == 1.0 and membership(3.0, left) == 0.5 and membership(4.0, left) == 0.0
    assert membership(1e300, right) == 1.0 and membership(11.0, right) == 0.25
    assert membership(5.0, (-INF, -INF, INF, INF)) == 1.0


def _good_clipped(h):
    """Centre of gravity of the Good triangle (0 at y = 1/2, 1 at y = 1)
    clipped at height h, integrated by hand: a rising wedge on
    [1/2, 1/2 + h/2] and a flat top of height h on [1/2 + h/2, 1]."""
    area = h * h / 4.0 + h * (0.5 - h / 2.0)
    moment = h ** 3 / 12.0 + h * h / 8.0 + (h / 2.0) * (1.0 - (0.5 + h / 2.0) ** 2)
    return moment / area


@pytest.mark.parametrize("h", [1.0, 0.75, 0.5, 0.25, 0.1])
def test_centre_of_gravity_closed_forms(h):
    everywhere = (0, (-INF, -INF, INF, INF))
    # a term that fires at strength h for stats[0] = 0: flank of (-1, 1, .., ..)
    at_h = (0, (-1.0, -1.0 + 1.0 / h, 1e9, 2e9))
    stats = [0.0] * 8
    s = suitability([_rule(0, GOOD, at_h)], stats, 1)[0]
    assert abs(s - _good_clipped(h)) < 1e-9
    # Bad mirrors Good about 1/2; Okay is symmetric about 1/2
    s = suitability([_rule(0, BAD, at_h)], stats, 1)[0]
    assert abs(s - (1.0 - _good_clipped(h))) < 1e-9
    s = suitability([_rule(0, OKAY, at_h)], stats, 1)[0]
    assert abs(s - 0.5) < 1e-9
    # the whole triangles: centroids 5/6, 1/2 and 1/6
    if h == 1.0:
        for then, want in ((GOOD, 5.0 / 6.0), (OKAY, 0.5), (BAD, 1.0 / 6.0)):
            assert abs(suitability([_rule(0, then, everywhere)], stats, 1)[0] - want) < 1e-9
    assert abs(_good_clipped(0.5) - 29.0 / 36.0) < 1e-15


def test_centre_of_gravity_of_joined_terms_and_and():
    stats = [3.0, 0.25] + [0.0] * 6
    full = (0, (-INF, -INF, INF, INF))
    # Bad and Good fully fired: symmetric about 1/2
    assert abs(suitability([_rule(0, BAD, full), _rule(0, GOOD, full)], stats, 1)[0] - 0.5) < 1e-9
    # AND is the smaller membership: stats[0] = 3 in (2, 4, ..) -> 0.5,
    # stats[1] = 0.25 in (0, 1, ..) -> 0.25
    r = _rule(0, GOOD, (0, (2.0, 4.0, 10.0, 11.0)), (1, (0.0, 1.0, 2.0, 3.0)))
    assert abs(suitability([r], stats, 1)[0] - _good_clipped(0.25)) < 1e-9
    # no rule of configuration 1 fires: suitability 0
    out = suitability([_rule(0, GOOD, full), _rule(1, GOOD, (0, (5.0, 6.0, 7.0, 8.0)))], stats, 2)
    assert out[1] == 0.0 and abs(out[0] - 5.0 / 6.0) < 1e-9


def test_expert_trial_set_and_phase():
    assert expert_trial_set([0.0, 0.0, 0.0]) == [0, 1, 2]
    assert expert_trial_set([0.5, 0.8333, 0.75, 0.0]) == [1, 2]
    assert expert_trial_set([0.5, 0.5, 0.1667]) == [0, 1]
    tu = TunerOracle(EXPERT, 3, 4)
    assert tu.begin_phase([0.8, 0.5, 0.75]) == [0, 2]
    tu.report(0, 5.0)
    tu.report(2, 50.0)
    assert tu.end_phase() == 0 and not any(tu.blacklisted)
    assert tu.begin_phase([0.8, 0.5, 0.75]) == [0, 2]

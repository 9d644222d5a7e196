"""Plain-Python oracle of the configuration-selection strategies.

TEST INFRASTRUCTURE ONLY (imported by tests, never by the product).

Sec. 2.2.5 ("Algorithm Selection"): tuning phases occur after a fixed number
of time steps; in a phase, configurations are trialled for a few iterations and
a weighted average of container-build time and force time is taken; the one
with the smallest value is used until the next phase.  Trialling everything is
the Full Search.

Sec. 5.1 (Predictive strategy), steps in the paper's order:
  1. in the first two tuning phases every configuration is trialled;
  2. afterwards, at the start of each phase, a linear model through the last
     two data points of each configuration predicts its score in this phase;
  3. only configurations predicted within a relative threshold (2x) of the
     predicted optimum are trialled;
  4. configurations not trialled for about a quarter of the simulation are
     retrialled regardless of their prediction;
  5. configurations measured more than 10x worse than the best are
     blacklisted and never trialled again.

Sec. 5.2 (Expert strategy), with the fuzzy logic of Sec. 2.3: rules written
by an expert map live simulation statistics (Sec. 4) through linguistic terms
to a suitability per configuration; the set of degrees of membership is
reduced to a crisp value by its centre of gravity; only the configurations
the rules mark as suited are trialled.

Readings where the paper is silent (each listed in the design notes):
  * a prediction from a single data point is that point's score;
  * predictions are clamped from below at half the configuration's last score
    (a falling line may otherwise cross zero and break the relative test);
  * "within 2x" is inclusive: trial iff prediction <= 2 * min prediction;
  * "a quarter of the simulation" = ceil(total_phases / 4) phases (at least 1);
  * "10x worse than the best" compares against the best score measured in the
    same phase, strictly greater than 10x;
  * ties in score go to the lower configuration index;
  * Expert: input terms are trapezoids; the output variable "suitability"
    on [0, 1] has three triangular terms, Bad / Okay / Good, peaking at 0,
    0.5 and 1 and reaching 0 half a unit from the peak; AND is min; a rule
    clips its output term at its firing strength and a configuration's
    clipped terms are joined by max; a configuration no rule fires for has
    suitability 0; a phase trials every configuration within 0.1 of the
    largest suitability (all if none fires) and never blacklists.
"""
from __future__ import annotations

import math

import numpy as np

FULL_SEARCH = 1
PREDICTIVE = 2
EXPERT = 3

BAD, OKAY, GOOD = 0, 1, 2
EXPERT_MARGIN = 0.1


class TunerOracle:
    def __init__(self, strategy: int, n_configs: int, total_phases: int,
                 rel_threshold: float = 2.0, blacklist_factor: float = 10.0,
                 retrial_fraction: float = 0.25):
        assert strategy in (FULL_SEARCH, PREDICTIVE, EXPERT)
        self.strategy = strategy
        self.n = n_configs
        self.rel = rel_threshold
        self.black = blacklist_factor
        self.retrial = max(1, math.ceil(retrial_fraction * total_phases))
        self.phase = -1
        self.history = [[] for _ in range(n_configs)]  # list of (phase, score)
        self.blacklisted = [False] * n_configs
        self.trial_set: list[int] = []
        self.scores: dict[int, float] = {}
        self.chosen = -1

    def predict(self, c: int) -> float:
        h = self.history[c]
        if len(h) == 1:
            return h[-1][1]
        (p1, s1), (p2, s2) = h[-2], h[-1]
        slope = (s2 - s1) / (p2 - p1)
        pred = s2 + slope * (self.phase - p2)
        return max(pred, 0.5 * s2)

    def begin_phase(self, suitability=None) -> list[int]:
        self.phase += 1
        self.scores = {}
        if self.strategy == EXPERT:
            self.trial_set = expert_trial_set(suitability if suitability is not None else [0.0] * self.n)
            return list(self.trial_set)
        alive = [c for c in range(self.n) if not self.blacklisted[c]]
        if self.strategy == FULL_SEARCH or self.phase < 2:
            self.trial_set = alive
            return list(self.trial_set)
        preds = {c: self.predict(c) for c in alive if self.history[c]}
        best = min(preds.values()) if preds else 0.0
        trial = []
        for c in alive:
            if not self.history[c]:
                trial.append(c)
                continue
            last = self.history[c][-1][0]
            if preds[c] <= self.rel * best or self.phase - last >= self.retrial:
                trial.append(c)
        self.trial_set = trial
        return list(trial)

    def report(self, c: int, score: float) -> None:
        assert c in self.trial_set
        self.scores[c] = float(score)
        self.history[c].append((self.phase, float(score)))

    def end_phase(self) -> int:
        assert set(self.scores) == set(self.trial_set)
        best_c = min(self.scores, key=lambda c: (self.scores[c], c))
        best = self.scores[best_c]
        if self.strategy == PREDICTIVE:
            for c, s in self.scores.items():
                if s > self.black * best:
                    self.blacklisted[c] = True
        self.chosen = best_c
        return best_c


# ---------------------------------------------------------------- Expert (Sec. 5.2)

def membership(x: float, trap) -> float:
    """Degree of membership of x in the trapezoidal term trap = (a, b, c, d):
    full on [b, c], linear on the flanks (a, b) and (c, d), none outside;
    infinite corners make shoulders."""
    a, b, c, d = trap
    if b <= x <= c:
        return 1.0
    if a < x < b:
        return (x - a) / (b - a)
    if c < x < d:
        return (d - x) / (d - c)
    return 0.0


def output_term(term: int, y: np.ndarray) -> np.ndarray:
    """The Bad / Okay / Good terms of "suitability" on [0, 1]."""
    peak = {BAD: 0.0, OKAY: 0.5, GOOD: 1.0}[term]
    return np.maximum(0.0, 1.0 - 2.0 * np.abs(y - peak))


def firing_strength(rule, stats) -> float:
    """rule["if"]: list of (statistic index, trapezoid); AND is min."""
    return min(membership(stats[i], trap) for i, trap in rule["if"])


def suitability(rules, stats, n_configs: int, points: int = 400001) -> list[float]:
    """Crisp suitability of each configuration: the centre of gravity,
    integral(y mu(y)) / integral(mu(y)) over [0, 1], of the union (max) of
    its rules' output terms, each clipped (min) at the rule's firing
    strength; integrals by the trapezoid rule on a fine uniform grid."""
    y = np.linspace(0.0, 1.0, points)
    out = []
    for c in range(n_configs):
        mu = np.zeros_like(y)
        for r in rules:
            if r["config"] != c:
                continue
            s = firing_strength(r, stats)
            mu = np.maximum(mu, np.minimum(s, output_term(r["then"], y)))
        area = np.trapezoid(mu, y)
        out.append(float(np.trapezoid(y * mu, y) / area) if area > 0.0 else 0.0)
    return out


def expert_trial_set(suit) -> list[int]:
    """Configurations a phase trials: within EXPERT_MARGIN of the most
    suitable (and suited at all), or every configuration if no rule fired."""
    top = max(suit) if len(suit) else 0.0
    if top <= 0.0:
        return list(range(len(suit)))
    return [c for c, v in enumerate(suit) if v > 0.0 and v >= top - EXPERT_MARGIN]

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

Readings where the paper is silent (each listed in the design notes):
  * a prediction from a single data point is that point's score;
  * predictions are clamped from below at half the configuration's last score
    (a falling line may otherwise cross zero and break the relative test);
  * "within 2x" is inclusive: trial iff prediction <= 2 * min prediction;
  * "a quarter of the simulation" = ceil(total_phases / 4) phases (at least 1);
  * "10x worse than the best" compares against the best score measured in the
    same phase, strictly greater than 10x;
  * ties in score go to the lower configuration index.
"""
from __future__ import annotations

import math

FULL_SEARCH = 1
PREDICTIVE = 2


class TunerOracle:
    def __init__(self, strategy: int, n_configs: int, total_phases: int,
                 rel_threshold: float = 2.0, blacklist_factor: float = 10.0,
                 retrial_fraction: float = 0.25):
        assert strategy in (FULL_SEARCH, PREDICTIVE)
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

    def begin_phase(self) -> list[int]:
        self.phase += 1
        self.scores = {}
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

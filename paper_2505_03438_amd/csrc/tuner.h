// Configuration-selection strategies (host only): Full Search (Sec. 2.2.5)
// and the Predictive strategy (Sec. 5.1).
#pragma once

#include <vector>

#include "mdlj.h"

namespace mdlj {

class Tuner {
public:
    Tuner(int strategy, int n_configs, int total_phases, double rel_threshold, double blacklist_factor);

    // Start a phase; fills trial[c] = 1 for configurations to trial.
    int begin_phase(std::vector<int> &trial);
    // Score of a trialled configuration (lower is better).
    bool report(int config, double score);
    // Finish the phase; returns the chosen configuration or -1 if a trialled
    // configuration has no score.
    int end_phase();

    int n() const { return n_; }
    bool blacklisted(int c) const { return black_[c] != 0; }
    int phase() const { return phase_; }

private:
    struct Point {
        int phase;
        double score;
    };
    double predict(int c) const;

    int strategy_, n_, retrial_;
    double rel_, black_factor_;
    int phase_ = -1;
    std::vector<std::vector<Point>> hist_;
    std::vector<char> black_, in_trial_, scored_;
    std::vector<double> score_;
};

// The GPU configuration space the autotuner explores for a base config:
// linked cells (CSF 1 and 0.5) and Verlet lists, gather-only or with
// Newton's third law, and cluster lists (gather-only, FP32).  The rebuild
// interval is not a trial dimension: it is derived from the measured
// particle motion (the most steps that keep displacements within the skin).
void tuning_space(const md_config &base, std::vector<md_config> &space);

}  // namespace mdlj

// Configuration-selection strategies (host only): Full Search (Sec. 2.2.5),
// the Predictive strategy (Sec. 5.1), the Expert strategy (Sec. 5.2) and the
// Random Forest strategy (Sec. 5.3).
#pragma once

#include <math.h>

#include <string>
#include <functional>
#include <vector>

#include "mdlj.h"

namespace mdlj {

class Tuner {
public:
    Tuner(int strategy, int n_configs, int total_phases, double rel_threshold, double blacklist_factor);

    // The trial set the next phase would have (trial[c] = 1 for
    // configurations to trial) and its size; changes nothing.
    int plan_phase(std::vector<int> &trial) const;
    // Start a phase; fills trial[c] = 1 for configurations to trial.
    int begin_phase(std::vector<int> &trial);
    // Expert and Random Forest strategies: the suitability of each
    // configuration for the next phase (all 0: trial everything).
    void set_suitability(const std::vector<double> &s) { suit_ = s; }
    const std::vector<double> &suitability() const { return suit_; }
    // Score of a trialled configuration (lower is better).
    bool report(int config, double score);
    // Finish the phase; returns the chosen configuration or -1 if a trialled
    // configuration has no score.
    int end_phase();

    int n() const { return n_; }
    bool blacklisted(int c) const { return black_[c] != 0; }
    int phase() const { return phase_; }
    // Last score measured for configuration c (NaN if never trialled).
    double last_score(int c) const { return hist_[c].empty() ? NAN : hist_[c].back().score; }

private:
    struct Point {
        int phase;
        double score;
    };
    double predict(int c, int phase) const;

    int strategy_, n_, retrial_;
    double rel_, black_factor_;
    int phase_ = -1;
    std::vector<std::vector<Point>> hist_;
    std::vector<char> black_, in_trial_, scored_;
    std::vector<double> score_, suit_;
};

// Expert strategy: margin below the largest suitability within which a
// configuration is trialled.
constexpr double kExpertMargin = 0.1;

// Check a rule set against a tuning space of n_configs entries; "" if valid,
// else the reason.
std::string check_rules(const md_fuzzy_rule *rules, int n_rules, int n_configs);
// Crisp suitability of each of n_configs configurations (Sec. 5.2 with the
// fuzzy logic of Sec. 2.3) for the live statistics stats[8].
void expert_suitability(const md_fuzzy_rule *rules, int n_rules, int n_configs, const double *stats,
                        std::vector<double> &suit);
// Random Forest: the configuration (index below n_configs) the forest of
// rf_model.h predicts for the live statistics stats[8], or -1.
int rf_predict(const double *stats, int n_configs);
// The same with the forest's classes (indices of the FP32 tuning space
// without skin variants) mapped to another space by map (-1: not in it).
int rf_predict_mapped(const double *stats, const std::function<int(int)> &map);
// The built-in rules (written from Full Search scores on MI355X).
const std::vector<md_fuzzy_rule> &builtin_rules();
// Whether a rule set reads statistics that need the bin histogram (relative
// spread, median, maximum, empty bins) rather than counts alone.
bool rules_need_histogram(const std::vector<md_fuzzy_rule> &rules);

// The GPU configuration space the autotuner explores for a base config:
// linked cells (CSF 1 and 0.5) and Verlet lists, gather-only or with
// Newton's third law, cluster lists and pairwise Verlet lists (gather-only,
// FP32), and with tune_skin
// Verlet lists at 2/3, 4/3 and 5/3 of the skin.  The rebuild interval is not
// a trial dimension: it is derived from the measured particle motion (the
// most steps that keep displacements within the configuration's skin).
void tuning_space(const md_config &base, std::vector<md_config> &space);

}  // namespace mdlj

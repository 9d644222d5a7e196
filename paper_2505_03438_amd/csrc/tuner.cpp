// Selection strategies, Sec. 2.2.5 and Sec. 5.1.
//
// Full Search: every live configuration is trialled in every phase and the
// one with the smallest score is kept until the next phase.
//
// Predictive: in the first two phases every configuration is trialled; after
// that each configuration's score in the current phase is predicted by the
// straight line through its last two (phase, score) points, and only those
// predicted within rel_threshold times the best prediction are trialled.  A
// configuration not trialled for a quarter of the run's phases is trialled
// again whatever its prediction, and one measured more than blacklist_factor
// times worse than the phase's best is never trialled again.
//
// Readings where the paper gives no number or is silent: a single point
// predicts its own score; a falling line is clamped from below at half the
// last score; "within" is inclusive; the retrial gap is ceil(total/4) phases;
// ties go to the lower index.
#include "tuner.h"

#include <math.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <string>

namespace mdlj {

int fail(int code, const std::string &msg);

Tuner::Tuner(int strategy, int n_configs, int total_phases, double rel_threshold, double blacklist_factor)
    : strategy_(strategy), n_(n_configs), rel_(rel_threshold), black_factor_(blacklist_factor)
{
    retrial_ = std::max(1, (int)ceil(0.25 * (double)total_phases));
    hist_.resize(n_);
    black_.assign(n_, 0);
    in_trial_.assign(n_, 0);
    scored_.assign(n_, 0);
    score_.assign(n_, 0.0);
}

double Tuner::predict(int c) const
{
    const std::vector<Point> &h = hist_[c];
    const Point &b = h.back();
    if (h.size() == 1) return b.score;
    const Point &a = h[h.size() - 2];
    double slope = (b.score - a.score) / (double)(b.phase - a.phase);
    double p = b.score + slope * (double)(phase_ - b.phase);
    return std::max(p, 0.5 * b.score);
}

int Tuner::begin_phase(std::vector<int> &trial)
{
    phase_++;
    trial.assign(n_, 0);
    std::fill(in_trial_.begin(), in_trial_.end(), 0);
    std::fill(scored_.begin(), scored_.end(), 0);
    bool all = strategy_ == MD_TUNE_FULL || phase_ < 2;
    double best = INFINITY;
    if (!all)
        for (int c = 0; c < n_; c++)
            if (!black_[c] && !hist_[c].empty()) best = std::min(best, predict(c));
    int cnt = 0;
    for (int c = 0; c < n_; c++) {
        if (black_[c]) continue;
        bool t = all || hist_[c].empty();
        if (!t) {
            bool near = predict(c) <= rel_ * best;
            bool stale = phase_ - hist_[c].back().phase >= retrial_;
            t = near || stale;
        }
        if (t) {
            trial[c] = 1;
            in_trial_[c] = 1;
            cnt++;
        }
    }
    return cnt;
}

bool Tuner::report(int c, double score)
{
    if (c < 0 || c >= n_ || !in_trial_[c]) return false;
    if (scored_[c]) hist_[c].pop_back();
    scored_[c] = 1;
    score_[c] = score;
    hist_[c].push_back(Point{phase_, score});
    return true;
}

int Tuner::end_phase()
{
    int best_c = -1;
    for (int c = 0; c < n_; c++) {
        if (!in_trial_[c]) continue;
        if (!scored_[c]) return -1;
        if (best_c < 0 || score_[c] < score_[best_c]) best_c = c;
    }
    if (best_c < 0) return -1;
    if (strategy_ == MD_TUNE_PREDICTIVE)
        for (int c = 0; c < n_; c++)
            if (in_trial_[c] && score_[c] > black_factor_ * score_[best_c]) black_[c] = 1;
    std::fill(in_trial_.begin(), in_trial_.end(), 0);
    return best_c;
}

void tuning_space(const md_config &base, std::vector<md_config> &space)
{
    space.clear();
    md_config c = base;
    c.autotune = MD_TUNE_OFF;
    // linked cells, CSF 1 and 0.5, gather-only and N3L
    for (double csf : {1.0, 0.5})
        for (int n3 : {MD_N3L_OFF, MD_N3L_ON}) {
            c.container = MD_CONTAINER_LC;
            c.csf = csf;
            c.newton3 = n3;
            space.push_back(c);
        }
    // Verlet lists (built from CSF-1 cells)
    for (int n3 : {MD_N3L_OFF, MD_N3L_ON}) {
        c.container = MD_CONTAINER_VL;
        c.csf = 1.0;
        c.newton3 = n3;
        space.push_back(c);
    }
    // cluster-pair lists (FP32, gather-only)
    if (base.precision == MD_FP32) {
        c.container = MD_CONTAINER_CL;
        c.csf = 1.0;
        c.newton3 = MD_N3L_OFF;
        space.push_back(c);
    }
}

}  // namespace mdlj

// ------------------------------------------------------------------ C-ABI

struct md_tuner {
    mdlj::Tuner t;
    std::vector<int> trial;
};

extern "C" int md_tuner_create(int32_t strategy, int32_t n_configs, int32_t total_phases, double rel_threshold,
                               double blacklist_factor, md_tuner **out)
{
    if (!out) return mdlj::fail(MD_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (strategy != MD_TUNE_FULL && strategy != MD_TUNE_PREDICTIVE)
        return mdlj::fail(MD_ERR_INVALID_ARG, "strategy must be MD_TUNE_FULL or MD_TUNE_PREDICTIVE");
    if (n_configs < 1 || total_phases < 1) return mdlj::fail(MD_ERR_INVALID_ARG, "n_configs, total_phases >= 1");
    if (!(rel_threshold >= 1.0) || !(blacklist_factor >= 1.0))
        return mdlj::fail(MD_ERR_INVALID_ARG, "thresholds must be >= 1");
    md_tuner *t = new (std::nothrow)
        md_tuner{mdlj::Tuner(strategy, n_configs, total_phases, rel_threshold, blacklist_factor), {}};
    if (!t) return mdlj::fail(MD_ERR_INVALID_ARG, "out of memory");
    *out = t;
    return MD_OK;
}

extern "C" void md_tuner_destroy(md_tuner *t) { delete t; }

extern "C" int md_tuner_begin_phase(md_tuner *t, int32_t *trial)
{
    if (!t || !trial) return mdlj::fail(MD_ERR_INVALID_ARG, "NULL argument");
    int cnt = t->t.begin_phase(t->trial);
    for (int c = 0; c < t->t.n(); c++) trial[c] = t->trial[c];
    return cnt;
}

extern "C" int md_tuner_report(md_tuner *t, int32_t config, double score)
{
    if (!t) return mdlj::fail(MD_ERR_INVALID_ARG, "NULL tuner");
    if (!(score >= 0.0) || !isfinite(score)) return mdlj::fail(MD_ERR_INVALID_ARG, "score must be finite, >= 0");
    if (!t->t.report(config, score)) return mdlj::fail(MD_ERR_INVALID_ARG, "configuration not in this phase's trials");
    return MD_OK;
}

extern "C" int md_tuner_end_phase(md_tuner *t)
{
    if (!t) return mdlj::fail(MD_ERR_INVALID_ARG, "NULL tuner");
    int c = t->t.end_phase();
    if (c < 0) return mdlj::fail(MD_ERR_INVALID_ARG, "a trialled configuration has no score");
    return c;
}

extern "C" int md_tuner_blacklist(md_tuner *t, int32_t *blacklisted)
{
    if (!t || !blacklisted) return mdlj::fail(MD_ERR_INVALID_ARG, "NULL argument");
    for (int c = 0; c < t->t.n(); c++) blacklisted[c] = t->t.blacklisted(c) ? 1 : 0;
    return MD_OK;
}

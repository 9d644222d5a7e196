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
// Expert: fuzzy rules over the live statistics give each configuration a
// suitability; the configurations within kExpertMargin of the most suitable
// are trialled and the fastest of them is kept (no blacklist).
//
// Random Forest (Sec. 5.3): a forest fitted offline maps the live
// statistics to one configuration, the only one the phase trials.
//
// Readings where the paper gives no number or is silent: a single point
// predicts its own score; a falling line is clamped from below at half the
// last score; "within" is inclusive; the retrial gap is ceil(total/4) phases;
// ties go to the lower index.
#include "tuner.h"

#include "rf_model.h"

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

double Tuner::predict(int c, int phase) const
{
    const std::vector<Point> &h = hist_[c];
    const Point &b = h.back();
    if (h.size() == 1) return b.score;
    const Point &a = h[h.size() - 2];
    double slope = (b.score - a.score) / (double)(b.phase - a.phase);
    double p = b.score + slope * (double)(phase - b.phase);
    return std::max(p, 0.5 * b.score);
}

int Tuner::plan_phase(std::vector<int> &trial) const
{
    int phase = phase_ + 1;
    trial.assign(n_, 0);
    int cnt = 0;
    if (strategy_ == MD_TUNE_EXPERT || strategy_ == MD_TUNE_RF) {
        double top = 0.0;
        for (int c = 0; c < n_ && c < (int)suit_.size(); c++) top = std::max(top, suit_[c]);
        for (int c = 0; c < n_; c++) {
            double sc = c < (int)suit_.size() ? suit_[c] : 0.0;
            trial[c] = top <= 0.0 || (sc > 0.0 && sc >= top - kExpertMargin) ? 1 : 0;
            cnt += trial[c];
        }
        return cnt;
    }
    bool all = strategy_ == MD_TUNE_FULL || phase < 2;
    double best = INFINITY;
    if (!all)
        for (int c = 0; c < n_; c++)
            if (!black_[c] && !hist_[c].empty()) best = std::min(best, predict(c, phase));
    for (int c = 0; c < n_; c++) {
        if (black_[c]) continue;
        bool t = all || hist_[c].empty();
        if (!t) {
            bool near = predict(c, phase) <= rel_ * best;
            bool stale = phase - hist_[c].back().phase >= retrial_;
            t = near || stale;
        }
        trial[c] = t ? 1 : 0;
        cnt += trial[c];
    }
    return cnt;
}

int Tuner::begin_phase(std::vector<int> &trial)
{
    int cnt = plan_phase(trial);
    phase_++;
    std::fill(scored_.begin(), scored_.end(), 0);
    for (int c = 0; c < n_; c++) in_trial_[c] = (char)trial[c];
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

// ------------------------------------------------------------------ fuzzy rules (Sec. 2.3, 5.2)

// Trapezoid membership (a, b, c, d): 1 on [b, c], linear flanks on (a, b)
// and (c, d), 0 elsewhere.  Infinite a = b or c = d make shoulders.
static double trapezoid(double x, const double t[4])
{
    if (x >= t[1] && x <= t[2]) return 1.0;
    if (x > t[0] && x < t[1]) return (x - t[0]) / (t[1] - t[0]);
    if (x > t[2] && x < t[3]) return (t[3] - x) / (t[3] - t[2]);
    return 0.0;
}

// Output terms of "suitability" on [0, 1]: triangles peaking at 0 (Bad),
// 0.5 (Okay) and 1 (Good), each reaching 0 half a unit from its peak.
static double out_term(int term, double y)
{
    double peak = 0.5 * term;
    return std::max(0.0, 1.0 - 2.0 * fabs(y - peak));
}

std::string check_rules(const md_fuzzy_rule *rules, int n_rules, int n_configs)
{
    if (n_rules < 0 || (n_rules > 0 && !rules)) return "rules NULL with n_rules > 0";
    for (int r = 0; r < n_rules; r++) {
        const md_fuzzy_rule &u = rules[r];
        std::string at = "rule " + std::to_string(r) + ": ";
        if (u.config < 0 || u.config >= n_configs) return at + "config outside the tuning space";
        if (u.then < MD_SUIT_BAD || u.then > MD_SUIT_GOOD) return at + "unknown output term";
        for (int k = 0; k < 2; k++) {
            if (k == 1 && u.input[1] == -1) break;
            if (u.input[k] < 0 || u.input[k] > 7) return at + "input outside 0..7";
            const double *t = u.trap[k];
            if (t[0] != t[0] || t[1] != t[1] || t[2] != t[2] || t[3] != t[3]) return at + "NaN in a trapezoid";
            if (!(t[0] <= t[1] && t[1] <= t[2] && t[2] <= t[3])) return at + "trapezoid needs a <= b <= c <= d";
        }
    }
    return "";
}

void expert_suitability(const md_fuzzy_rule *rules, int n_rules, int n_configs, const double *stats,
                        std::vector<double> &suit)
{
    suit.assign(n_configs, 0.0);
    std::vector<double> w(n_rules, 0.0);
    for (int r = 0; r < n_rules; r++) {
        const md_fuzzy_rule &u = rules[r];
        double s = trapezoid(stats[u.input[0]], u.trap[0]);
        if (u.input[1] >= 0) s = std::min(s, trapezoid(stats[u.input[1]], u.trap[1]));
        w[r] = s;
    }
    for (int c = 0; c < n_configs; c++) {
        // the aggregate mu(y) = max over the configuration's rules of
        // min(strength, term(y)) is linear between the points where any two
        // of its pieces cross: the terms' corners and crossings (0, 1/4, 1/2,
        // 3/4, 1) and where a flank meets a strength level
        std::vector<double> ys = {0.0, 0.25, 0.5, 0.75, 1.0};
        bool any = false;
        for (int r = 0; r < n_rules; r++) {
            if (rules[r].config != c || w[r] <= 0.0) continue;
            any = true;
            double h = w[r];
            for (double y : {0.5 * (1.0 - h), 0.5 * h, 1.0 - 0.5 * h, 0.5 * (1.0 + h)}) ys.push_back(y);
        }
        if (!any) continue;
        std::sort(ys.begin(), ys.end());
        auto mu = [&](double y) {
            double m = 0.0;
            for (int r = 0; r < n_rules; r++)
                if (rules[r].config == c && w[r] > 0.0) m = std::max(m, std::min(w[r], out_term(rules[r].then, y)));
            return m;
        };
        // exact integrals of a piecewise-linear function: area and first moment
        double area = 0.0, moment = 0.0;
        double y0 = ys[0], m0 = mu(y0);
        for (size_t k = 1; k < ys.size(); k++) {
            double y1 = ys[k];
            if (y1 <= y0) continue;
            double m1 = mu(y1);
            double dy = y1 - y0;
            area += 0.5 * dy * (m0 + m1);
            moment += dy / 6.0 * (m0 * (2.0 * y0 + y1) + m1 * (y0 + 2.0 * y1));
            y0 = y1;
            m0 = m1;
        }
        suit[c] = area > 0.0 ? moment / area : 0.0;
    }
}

bool rules_need_histogram(const std::vector<md_fuzzy_rule> &rules)
{
    for (const md_fuzzy_rule &u : rules)
        for (int k = 0; k < 2; k++) {
            int i = u.input[k];
            if (i == 1 || i == 2 || i == 3 || i == 5) return true;
        }
    return false;
}

const std::vector<md_fuzzy_rule> &builtin_rules()
{
    static const std::vector<md_fuzzy_rule> rules = [] {
        const double inf = INFINITY;
        auto rule = [&](double a, double b, double c, double d, int config, int then) {
            md_fuzzy_rule u;
            u.input[0] = 0;
            u.input[1] = -1;
            u.trap[0][0] = a;
            u.trap[0][1] = b;
            u.trap[0][2] = c;
            u.trap[0][3] = d;
            for (int k = 0; k < 4; k++) u.trap[1][k] = 0.0;
            u.config = config;
            u.then = then;
            return u;
        };
        // terms of the mean particles per CSF-1 bin; Full Search on MI355X
        // (fluids of 32k-1M particles at densities 0.05-1.0, the droplet and
        // the slab) found Verlet lists, gather-only, fastest in every case
        // but one, where the N3L variant led by 4 % at a mean of 8; linked
        // cells came second in sparse systems (CSF 1) and dense ones (CSF
        // 0.5), cluster lists in small sparse ones
        const double sparse[4] = {-inf, -inf, 2.0, 4.0};
        const double medium[4] = {2.0, 4.0, 10.0, 14.0};
        const double dense[4] = {10.0, 14.0, inf, inf};
        // tuning-space indices: 0 LC CSF 1, 1 LC CSF 1 N3L, 2 LC CSF 0.5,
        // 3 LC CSF 0.5 N3L, 4 VL, 5 VL N3L, 6 cluster lists
        const int then[7][3] = {
            {MD_SUIT_OKAY, MD_SUIT_OKAY, MD_SUIT_BAD},   // per config: sparse, medium, dense
            {MD_SUIT_BAD, MD_SUIT_OKAY, MD_SUIT_BAD},
            {MD_SUIT_BAD, MD_SUIT_BAD, MD_SUIT_OKAY},
            {MD_SUIT_BAD, MD_SUIT_BAD, MD_SUIT_OKAY},
            {MD_SUIT_GOOD, MD_SUIT_GOOD, MD_SUIT_GOOD},
            {MD_SUIT_OKAY, MD_SUIT_GOOD, MD_SUIT_OKAY},
            {MD_SUIT_OKAY, MD_SUIT_OKAY, MD_SUIT_BAD},
        };
        const double *terms[3] = {sparse, medium, dense};
        std::vector<md_fuzzy_rule> v;
        for (int c = 0; c < 7; c++)
            for (int k = 0; k < 3; k++)
                v.push_back(rule(terms[k][0], terms[k][1], terms[k][2], terms[k][3], c, then[c][k]));
        return v;
    }();
    return rules;
}

// ------------------------------------------------------------------ random forest (Sec. 5.3)

int rf_predict(const double *stats, int n_configs)
{
    return rf_predict_mapped(stats, [n_configs](int k) { return k < n_configs ? k : -1; });
}

int rf_predict_mapped(const double *stats, const std::function<int(int)> &map)
{
    double acc[rf::kClasses] = {};
    for (int t = 0; t < rf::kTrees; t++) {
        int k = rf::kRoot[t];
        while (rf::kNodes[k].feature >= 0) {
            const rf::Node &nd = rf::kNodes[k];
            // the trees were fitted on single-precision features
            double x = (double)(float)stats[nd.feature];
            k = x <= nd.threshold ? nd.left : nd.right;
        }
        const double *p = rf::kProba + rf::kNodes[k].proba;
        for (int c = 0; c < rf::kClasses; c++) acc[c] += p[c];
    }
    // mean class fraction over the trees; the first largest among the
    // classes this space holds
    int best = -1;
    for (int c = 0; c < rf::kClasses; c++) {
        acc[c] /= (double)rf::kTrees;
        if (map(rf::kConfig[c]) < 0) continue;
        if (best < 0 || acc[c] > acc[best]) best = c;
    }
    return best < 0 ? -1 : map(rf::kConfig[best]);
}

void tuning_space(const md_config &base, std::vector<md_config> &space)
{
    space.clear();
    md_config c = base;
    c.autotune = MD_TUNE_OFF;
    c.layout = MD_LAYOUT_PACKED;
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
    // pairwise Verlet lists (FP32, gather-only, CSF-1 cells; left out by the
    // caller where the box holds fewer than three such cells per dimension)
    if (base.precision == MD_FP32) {
        c.container = MD_CONTAINER_PVL;
        c.csf = 1.0;
        c.newton3 = MD_N3L_OFF;
        space.push_back(c);
    }
    // Verlet list cells (FP32, Newton's third law through the C08
    // colouring, CSF-1 cells; left out like pairwise lists on small boxes)
    if (base.precision == MD_FP32) {
        c.container = MD_CONTAINER_VLC;
        c.csf = 1.0;
        c.newton3 = MD_N3L_ON;
        space.push_back(c);
    }
    // Verlet lists, gather-only, with the other LDS window layouts (FP32,
    // one particle type)
    if (base.precision == MD_FP32 && base.n_types == 1)
        for (int lay : {MD_LAYOUT_ALIGNED, MD_LAYOUT_SOA}) {
            c.container = MD_CONTAINER_VL;
            c.csf = 1.0;
            c.newton3 = MD_N3L_OFF;
            c.layout = lay;
            space.push_back(c);
        }
    c.layout = MD_LAYOUT_PACKED;
    // linked cells with the C08 colouring (FP32, CSF-1 cells; left out like
    // pairwise lists on small boxes)
    if (base.precision == MD_FP32) {
        c.container = MD_CONTAINER_LC;
        c.csf = 1.0;
        c.newton3 = MD_N3L_C08;
        space.push_back(c);
    }
    // joint skin / rebuild-interval search: Verlet lists at other skins (a
    // larger skin buys a longer interval with longer lists)
    if (base.tune_skin && base.skin > 0.0)
        for (double f : {2.0 / 3.0, 4.0 / 3.0, 5.0 / 3.0}) {
            c.container = MD_CONTAINER_VL;
            c.csf = 1.0;
            c.newton3 = MD_N3L_OFF;
            c.skin = base.skin * f;
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
    if (strategy != MD_TUNE_FULL && strategy != MD_TUNE_PREDICTIVE && strategy != MD_TUNE_EXPERT &&
        strategy != MD_TUNE_RF)
        return mdlj::fail(MD_ERR_INVALID_ARG, "strategy must be one of MD_TUNE_FULL .. MD_TUNE_RF");
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

extern "C" int md_tuner_set_suitability(md_tuner *t, const double *suitability)
{
    if (!t || !suitability) return mdlj::fail(MD_ERR_INVALID_ARG, "NULL argument");
    std::vector<double> s(suitability, suitability + t->t.n());
    for (double v : s)
        if (!(v >= 0.0 && v <= 1.0)) return mdlj::fail(MD_ERR_INVALID_ARG, "suitability must lie in [0, 1]");
    t->t.set_suitability(s);
    return MD_OK;
}

extern "C" int md_rf_predict(const double *stats, int32_t n_configs)
{
    if (!stats || n_configs < 1) return mdlj::fail(MD_ERR_INVALID_ARG, "bad arguments");
    for (int k = 0; k < 8; k++)
        if (!(stats[k] == stats[k])) return mdlj::fail(MD_ERR_INVALID_ARG, "statistics must not be NaN");
    int c = mdlj::rf_predict(stats, n_configs);
    if (c < 0) return mdlj::fail(MD_ERR_INVALID_ARG, "the model predicts no configuration of this space");
    return c;
}

extern "C" int md_expert_suitability(const md_fuzzy_rule *rules, int32_t n_rules, int32_t n_configs,
                                     const double *stats, double *suitability)
{
    if (!stats || !suitability || n_configs < 1) return mdlj::fail(MD_ERR_INVALID_ARG, "bad arguments");
    const md_fuzzy_rule *r = rules;
    int nr = n_rules;
    std::vector<md_fuzzy_rule> keep;
    if (!rules) {
        // the built-in rules that name configurations of this space
        for (const md_fuzzy_rule &u : mdlj::builtin_rules())
            if (u.config < n_configs) keep.push_back(u);
        r = keep.data();
        nr = (int)keep.size();
    }
    std::string why = mdlj::check_rules(r, nr, n_configs);
    if (!why.empty()) return mdlj::fail(MD_ERR_INVALID_ARG, why);
    std::vector<double> s;
    mdlj::expert_suitability(r, nr, n_configs, stats, s);
    for (int c = 0; c < n_configs; c++) suitability[c] = s[c];
    return MD_OK;
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

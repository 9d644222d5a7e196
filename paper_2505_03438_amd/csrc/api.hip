// C-ABI of libmdlj: handle lifecycle, argument validation, cell geometry,
// the rebuild policy of md_step (rebuild every R steps; steps that ran with a
// structure a particle had outgrown by skin/2 are recomputed) and the
// autotuned configuration switching.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <vector>

#include "md_internal.h"
#include "tuner.h"

namespace mdlj {

static thread_local std::string g_err;

int fail(int code, const std::string &msg)
{
    g_err = msg;
    return code;
}

int hip_fail(hipError_t e, const char *what)
{
    g_err = std::string("HIP error ") + hipGetErrorName(e) + " (" + hipGetErrorString(e) + ") in " + what;
    return MD_ERR_HIP;
}

void launch_zero(void *p, int64_t bytes, hipStream_t s);

// Cell geometry for csf and the cutoffs: n_d = floor(L_d / (csf r_l)) (>= 1),
// side L_d / n_d, stencil reach ceil(r_l / side) with duplicate periodic
// images of the same cell removed.
int make_geom(const md_config &c, double csf, Geom &g)
{
    memset(&g, 0, sizeof(g));
    int nt = c.n_types;
    double rcmax2 = 0.0;
    for (int a = 0; a < nt; a++)
        for (int b = 0; b < nt; b++) rcmax2 = std::max(rcmax2, c.rc2[a * nt + b]);
    double rl = sqrt(rcmax2) + c.skin;
    g.rl2 = rl * rl;
    g.nt = nt;
    for (int d = 0; d < 3; d++) {
        if (!(c.box[d] >= 2.0 * rl))
            return fail(MD_ERR_BOX_TOO_SMALL, "box[" + std::to_string(d) + "] = " + std::to_string(c.box[d]) +
                                                  " < 2 (r_c + skin) = " + std::to_string(2.0 * rl));
        double side_min = csf * rl;
        double ndd = floor(c.box[d] / side_min);
        if (ndd > 4096.0) ndd = 4096.0;
        int nd = ndd < 1.0 ? 1 : (int)ndd;
        // the C08 colouring (Verlet list cells, linked cells with
        // MD_N3L_C08): an even count where there are more than three
        // (slightly larger cells), so that it needs two colours per
        // dimension, not three
        if ((c.container == MD_CONTAINER_VLC || c.newton3 == MD_N3L_C08) && nd > 3 && nd % 2) nd--;
        g.nc[d] = nd;
        g.L[d] = c.box[d];
        g.inv_w[d] = (double)nd / c.box[d];
        g.S[d] = 4294967296.0 / c.box[d];
        double w = c.box[d] / nd;
        int reach = 1;
        while (reach * w < rl) reach++;
        if (2 * reach + 1 > kMaxOfs) return fail(MD_ERR_INVALID_ARG, "cell size factor too small (needs csf >= 0.5)");
        int k = 0;
        for (int o = -reach; o <= reach; o++) {
            int sft = ((o % nd) + nd) % nd;
            bool dup = false;
            for (int m = 0; m < k; m++) dup |= g.ofs[d][m] == sft;
            if (!dup) g.ofs[d][k++] = sft;
        }
        g.nofs[d] = k;
        g.reach[d] = reach;
    }
    int64_t ncell = (int64_t)g.nc[0] * g.nc[1] * g.nc[2];
    if (ncell > (int64_t)1 << 30) return fail(MD_ERR_INVALID_ARG, "too many cells");
    g.ncell = (int)ncell;
    g.ry = (float)(c.box[1] / c.box[0]);
    g.rz = (float)(c.box[2] / c.box[0]);
    g.iso = (c.box[0] == c.box[1] && c.box[1] == c.box[2]) ? 1 : 0;
    // y-rows per windowed block: about 256 particles per block at the mean
    // density, in blocks about four times longer (in x) than high (in y)
    double ppc = (double)std::max<int64_t>(c.n, 1) / (double)ncell;
    int band = (int)floor(sqrt(256.0 / ppc / 4.0));
    band = std::max(1, std::min(band, kWinBlkRows));
    band = std::min(band, std::max(1, g.nc[1] - 2 * g.reach[1]));
    g.wband = band;
    g.layout = c.layout;
    double u = c.box[0] / 4294967296.0;
    g.rl2_lo = (float)(g.rl2 / (u * u) * (1.0 - kBand));
    g.rl2_hi = (float)(g.rl2 / (u * u) * (1.0 + kBand));
    double h = 0.5 * c.skin;
    g.disp2 = c.skin > 0.0 ? (float)(h * h * (1.0 - 1e-4) / (u * u)) : INFINITY;
    return MD_OK;
}

}  // namespace mdlj

using namespace mdlj;

// ------------------------------------------------------------------ handle

struct md_handle {
    md_config cfg;           // current configuration (tuning may change it)
    md_config base;          // configuration at creation
    int device = 0;
    Geom g;
    Buffers b;
    int64_t n = 0;
    int64_t ncell_cap = 0;   // allocated cell-array entries
    int64_t scan_cap = 0;
    bool built = false;      // cells (and lists) valid for the staged positions
    bool lists = false;      // neighbour lists built since the last cell build
    int age = 0;             // integrator steps since the last build
    int64_t rebuilds = 0, forced = 0, phases = 0, trials = 0, list_entries = 0;
    int32_t config_index = -1;
    hipEvent_t ev0 = nullptr, ev1 = nullptr, ev2 = nullptr;
    // kernel-class timing (md_timing)
    struct TPair {
        hipEvent_t a, b;
        int kind;  // 0 force, 1 build
    };
    bool timing = false;
    std::vector<hipEvent_t> tpool;
    size_t tnext = 0;
    std::vector<TPair> tpend;
    double tsum[4] = {0, 0, 0, 0};
    // autotuning
    mdlj::Tuner *tuner = nullptr;
    std::vector<md_config> space;
    std::vector<md_fuzzy_rule> rules;  // Expert strategy
    std::vector<int32_t> phase_choices;  // configuration chosen by each tuning phase
    int64_t steps_done = 0;       // md_step steps since creation
    uint32_t sticky = 0;          // flag bits already read back from the device
    bool truncated = false;       // the current lists overflowed max_neighbors
    bool no_window = false;       // a cell neighbourhood overflowed the LDS windows: global kernels only
    bool energy_gather = true;    // the last energy partials saw each pair twice
    int epart_blocks = 0;         // partial slots the last energy force pass wrote
    bool replay_no_log = false;   // the next block replays: its first step's log entry is done
    int64_t next_phase = 0;       // step index of the next tuning phase
    double rate[4] = {0, 0, 0, 0};  // recent largest displacements per step (fixed-point units)
    int rate_pos = 0;
    // fused integrator: the step whose start (first half kick, drift, stage,
    // skin check) the last force pass already did (-1: none), and how many
    // per-workgroup kinetic-energy and displacement partials were written last
    int started = -1;
    int kpart_blocks = 0, dpart_blocks = 0;
};

static size_t real_size(const md_config &c) { return c.precision == MD_FP64 ? 8 : 4; }

// The built-in Expert rules, less those naming configurations outside this
// handle's tuning space (cluster lists are FP32 only).
static void set_builtin_rules(md_handle *h)
{
    h->rules.clear();
    for (const md_fuzzy_rule &u : builtin_rules())
        if (u.config < (int)h->space.size()) h->rules.push_back(u);
}

static void free_buffers(md_handle *h)
{
    Buffers &b = h->b;
    void *ptrs[] = {b.cell_id, b.slot, b.perm, b.perm2, b.cell_count, b.cell_start, b.cell_sorted, b.scan_blocks,
                    b.tmp_pos, b.tmp_vel, b.tmp_force, b.tmp_type, b.tmp_ids, b.stage, b.stage_ref,
                    b.nbr, b.nbr_count, b.partials, b.kpart, b.dpart, b.flags, b.tab, b.cl_start,
                    b.cl_count, b.cl_cell, b.cl_centre, b.cl_half, b.cl_base, b.cl_key, b.cl_nbr,
                    b.cl_nbr_count, b.snap_pos, b.snap_vel,
                    b.snap_force, b.snap_type, b.snap_ids, b.snap_stage, b.gpart, b.stat, b.stat_count, b.pvl_perm, b.pvl_cnt, b.pvl_s, b.pvl_entries, b.vlc_nbr, b.vlc_seg, b.vlc_part, b.pos_alt, b.stage_alt,
                    b.w_blk, b.w_staged, b.w_rown, b.w_rowb, b.w_nbr};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    if (b.host_flags) (void)hipHostFree(b.host_flags);
    b = Buffers();
}

template <typename T>
static int dalloc(T **p, size_t count)
{
    *p = nullptr;
    if (count == 0) count = 1;
    hipError_t e = hipMalloc((void **)p, count * sizeof(T));
    if (e != hipSuccess) return hip_fail(e, "hipMalloc");
    return MD_OK;
}

static int dalloc_bytes(void **p, size_t bytes)
{
    *p = nullptr;
    hipError_t e = hipMalloc(p, bytes ? bytes : 1);
    if (e != hipSuccess) return hip_fail(e, "hipMalloc");
    return MD_OK;
}

// Cell arrays sized for the geometry g (grown on demand, e.g. when tuning
// switches to a smaller cell size factor).
static int ensure_cells(md_handle *h, const Geom &g)
{
    int64_t need = (int64_t)g.ncell + 1;
    if (need <= h->ncell_cap) return MD_OK;
    if (h->b.cell_count) (void)hipFree(h->b.cell_count);
    if (h->b.cell_start) (void)hipFree(h->b.cell_start);
    if (h->b.scan_blocks) (void)hipFree(h->b.scan_blocks);
    h->b.cell_count = h->b.cell_start = h->b.scan_blocks = nullptr;
    int rc;
    if ((rc = dalloc(&h->b.cell_count, need))) return rc;
    if ((rc = dalloc(&h->b.cell_start, need))) return rc;
    int64_t sc = scan_scratch_size(need) + 64;
    if ((rc = dalloc(&h->b.scan_blocks, sc))) return rc;
    h->ncell_cap = need;
    return MD_OK;
}

// Containers that keep neighbour lists (Verlet lists, cluster-pair lists).
static bool has_lists(const md_config &c) { return c.container != MD_CONTAINER_LC; }

// Configurations that need at least three cells per dimension (their
// traversals pair each cell with distinct neighbours).
static bool needs_three_cells(const md_config &c)
{
    return c.container == MD_CONTAINER_PVL || c.container == MD_CONTAINER_VLC || c.newton3 == MD_N3L_C08;
}

static int ensure_list(md_handle *h, int64_t maxn)
{
    if (maxn <= h->b.nbr_cap && h->b.nbr) return MD_OK;
    if (h->b.nbr) (void)hipFree(h->b.nbr);
    h->b.nbr = nullptr;
    int rc = dalloc(&h->b.nbr, (size_t)maxn * (size_t)std::max<int64_t>(h->n, 1));
    if (rc) return rc;
    h->b.nbr_cap = maxn;
    return MD_OK;
}

static int validate_config(const md_config *c)
{
    if (!c) return fail(MD_ERR_INVALID_ARG, "config is NULL");
    if (c->n < 0 || c->n > (int64_t)INT32_MAX / 3) return fail(MD_ERR_INVALID_ARG, "n out of range");
    if (c->n_types < 1 || c->n_types > MD_MAX_TYPES) return fail(MD_ERR_INVALID_ARG, "n_types must be 1 or 2");
    if (c->precision != MD_FP32 && c->precision != MD_FP64) return fail(MD_ERR_INVALID_ARG, "bad precision");
    for (int d = 0; d < 3; d++)
        if (!(c->box[d] > 0.0) || !isfinite(c->box[d])) return fail(MD_ERR_INVALID_ARG, "box must be positive");
    int nt = c->n_types;
    for (int a = 0; a < nt; a++)
        for (int b = 0; b < nt; b++) {
            double v = c->rc2[a * nt + b];
            if (!(v > 0.0) || !isfinite(v)) return fail(MD_ERR_INVALID_ARG, "rc2 must be positive");
            if (v != c->rc2[b * nt + a]) return fail(MD_ERR_INVALID_ARG, "rc2 must be symmetric");
        }
    if (!(c->skin >= 0.0) || !isfinite(c->skin)) return fail(MD_ERR_INVALID_ARG, "skin must be >= 0");
    if (!(c->csf >= 0.5 && c->csf <= 1.0)) return fail(MD_ERR_INVALID_ARG, "csf must lie in [0.5, 1]");
    if (c->container != MD_CONTAINER_LC && c->container != MD_CONTAINER_VL && c->container != MD_CONTAINER_CL &&
        c->container != MD_CONTAINER_PVL && c->container != MD_CONTAINER_VLC)
        return fail(MD_ERR_INVALID_ARG, "bad container");
    if (c->container == MD_CONTAINER_VLC &&
        (c->newton3 != MD_N3L_ON || c->precision != MD_FP32 || c->csf != 1.0))
        return fail(MD_ERR_INVALID_ARG, "Verlet list cells are FP32, with Newton's third law, on CSF-1 cells");
    if (c->container == MD_CONTAINER_PVL &&
        (c->newton3 != MD_N3L_OFF || c->precision != MD_FP32 || c->csf != 1.0))
        return fail(MD_ERR_INVALID_ARG, "pairwise Verlet lists are FP32, gather-only, on CSF-1 cells");
    if (c->newton3 != MD_N3L_OFF && c->newton3 != MD_N3L_ON && c->newton3 != MD_N3L_C08)
        return fail(MD_ERR_INVALID_ARG, "bad newton3");
    if (c->newton3 == MD_N3L_C08 && (c->container != MD_CONTAINER_LC || c->precision != MD_FP32 || c->csf != 1.0))
        return fail(MD_ERR_INVALID_ARG, "the C08 traversal is for FP32 linked cells on CSF-1 cells");
    if (c->layout != MD_LAYOUT_PACKED && c->layout != MD_LAYOUT_ALIGNED && c->layout != MD_LAYOUT_SOA)
        return fail(MD_ERR_INVALID_ARG, "bad layout");
    if (c->layout != MD_LAYOUT_PACKED && (c->container != MD_CONTAINER_VL || c->newton3 != MD_N3L_OFF ||
                                          c->precision != MD_FP32 || c->n_types != 1))
        return fail(MD_ERR_INVALID_ARG, "window layouts other than packed are for FP32 Verlet lists, gather-only, "
                                        "one particle type");
    if (c->container == MD_CONTAINER_CL && c->newton3 != MD_N3L_OFF)
        return fail(MD_ERR_INVALID_ARG, "cluster lists are gather-only (newton3 = MD_N3L_OFF)");
    if (c->container == MD_CONTAINER_CL && c->precision != MD_FP32)
        return fail(MD_ERR_INVALID_ARG, "cluster lists run in FP32 (precision = MD_FP32)");
    if (c->rebuild_interval < 1) return fail(MD_ERR_INVALID_ARG, "rebuild_interval must be >= 1");
    if (c->max_neighbors < 1 || c->max_neighbors > 4096) return fail(MD_ERR_INVALID_ARG, "max_neighbors out of range");
    if (c->autotune != MD_TUNE_OFF && c->autotune != MD_TUNE_FULL && c->autotune != MD_TUNE_PREDICTIVE &&
        c->autotune != MD_TUNE_EXPERT && c->autotune != MD_TUNE_RF)
        return fail(MD_ERR_INVALID_ARG, "bad autotune");
    if (c->autotune != MD_TUNE_OFF && (c->tune_interval < 1 || c->tune_trial_steps < 2))
        return fail(MD_ERR_INVALID_ARG, "tune_interval >= 1 and tune_trial_steps >= 2 required");
    if (c->tune_skin != 0 && c->tune_skin != 1) return fail(MD_ERR_INVALID_ARG, "tune_skin must be 0 or 1");
    if (c->tune_first < 0) return fail(MD_ERR_INVALID_ARG, "tune_first must be >= 0");
    return MD_OK;
}

namespace mdlj {
int validate_md_config(const md_config *c) { return validate_config(c); }
}  // namespace mdlj

extern "C" int md_config_default(md_config *cfg, int64_t n, double L)
{
    if (!cfg) return fail(MD_ERR_INVALID_ARG, "cfg is NULL");
    memset(cfg, 0, sizeof(*cfg));
    cfg->n = n;
    cfg->n_types = 1;
    cfg->precision = MD_FP32;
    cfg->box[0] = cfg->box[1] = cfg->box[2] = L;
    for (int k = 0; k < MD_MAX_TYPES * MD_MAX_TYPES; k++) cfg->rc2[k] = 6.25;
    cfg->skin = 0.3;
    cfg->csf = 1.0;
    cfg->container = MD_CONTAINER_VL;
    cfg->newton3 = MD_N3L_OFF;
    cfg->rebuild_interval = 10;
    cfg->max_neighbors = 128;
    cfg->autotune = MD_TUNE_OFF;
    cfg->tune_interval = 500;
    cfg->tune_trial_steps = 10;
    cfg->total_steps_hint = 1000;
    return MD_OK;
}


extern "C" int md_create(const md_config *cfg, md_handle **out)
{
    if (!out) return fail(MD_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    int rc = validate_config(cfg);
    if (rc) return rc;
    Geom g;
    if ((rc = make_geom(*cfg, cfg->csf, g))) return rc;
    if (needs_three_cells(*cfg) && !pvl_geometry_ok(g))
        return fail(MD_ERR_INVALID_ARG, "pairwise lists, Verlet list cells and the C08 traversal need at least "
                                        "three cells of side r_c + skin per dimension");
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return fail(MD_ERR_NO_DEVICE, "no HIP device");
    md_handle *h = new md_handle();
    h->cfg = *cfg;
    h->base = *cfg;
    h->n = cfg->n;
    h->g = g;
    (void)hipGetDevice(&h->device);
    int64_t n = std::max<int64_t>(cfg->n, 1);
    size_t rs = real_size(*cfg);
    Buffers &b = h->b;
#define ALLOC(expr)                   \
    do {                              \
        if ((rc = (expr))) {          \
            free_buffers(h);          \
            delete h;                 \
            return rc;                \
        }                             \
    } while (0)
    ALLOC(dalloc(&b.cell_id, n));
    ALLOC(dalloc(&b.slot, n));
    ALLOC(dalloc(&b.perm, n));
    ALLOC(dalloc(&b.perm2, n));
    ALLOC(dalloc(&b.cell_sorted, n));
    ALLOC(dalloc(&b.tmp_pos, 3 * n));
    ALLOC(dalloc_bytes(&b.tmp_vel, 3 * n * rs));
    ALLOC(dalloc_bytes(&b.tmp_force, 3 * n * rs));
    ALLOC(dalloc(&b.tmp_type, n));
    ALLOC(dalloc(&b.tmp_ids, n));
    ALLOC(dalloc(&b.stage, n));
    ALLOC(dalloc(&b.stage_ref, n));
    ALLOC(dalloc(&b.nbr_count, n));
    ALLOC(dalloc(&b.partials, (size_t)kMaxPartials * 4));
    ALLOC(dalloc(&b.kpart, (size_t)kMaxPartials));
    ALLOC(dalloc(&b.dpart, (size_t)kMaxPartials));
    ALLOC(dalloc(&b.gpart, (size_t)kMaxPartials * 8));
    ALLOC(dalloc(&b.flags, 8));
    ALLOC(dalloc(&b.tab, 1));
    ALLOC(ensure_cells(h, g));
#undef ALLOC
    if (hipHostMalloc((void **)&b.host_flags, 8 * sizeof(uint32_t), 0) != hipSuccess) {
        free_buffers(h);
        delete h;
        return fail(MD_ERR_HIP, "hipHostMalloc failed");
    }
    (void)hipMemset(b.flags, 0, 8 * sizeof(int32_t));
    int32_t init[8] = {0, INT32_MAX, 0, 0, 0, 0, 0, 0};
    (void)hipMemcpy(b.flags, init, sizeof(init), hipMemcpyHostToDevice);
    (void)hipEventCreate(&h->ev0);
    (void)hipEventCreate(&h->ev1);
    (void)hipEventCreate(&h->ev2);
    if (cfg->autotune != MD_TUNE_OFF) {
        tuning_space(*cfg, h->space);
        // skin variants whose list radius does not fit the box are left out
        std::vector<md_config> fit;
        for (const md_config &k : h->space) {
            Geom gk;
            std::string keep_err = g_err;
            if (make_geom(k, k.csf, gk) == MD_OK && (!needs_three_cells(k) || pvl_geometry_ok(gk)))
                fit.push_back(k);
            g_err = keep_err;
        }
        h->space.swap(fit);
        int total_phases = std::max(1, (int)((cfg->total_steps_hint + cfg->tune_interval - 1) / cfg->tune_interval));
        h->tuner = new Tuner(cfg->autotune, (int)h->space.size(), total_phases, 2.0, 10.0);
        h->next_phase = cfg->tune_first;
        set_builtin_rules(h);
    }
    if (hipDeviceSynchronize() != hipSuccess) {
        md_destroy(h);
        return fail(MD_ERR_HIP, "device initialisation failed");
    }
    *out = h;
    return MD_OK;
}

extern "C" void md_destroy(md_handle *h)
{
    if (!h) return;
    (void)hipSetDevice(h->device);
    (void)hipDeviceSynchronize();
    free_buffers(h);
    if (h->ev0) (void)hipEventDestroy(h->ev0);
    if (h->ev1) (void)hipEventDestroy(h->ev1);
    if (h->ev2) (void)hipEventDestroy(h->ev2);
    for (hipEvent_t e : h->tpool) (void)hipEventDestroy(e);
    delete h->tuner;
    delete h;
}

// ------------------------------------------------------------------ building

static int check_handle(md_handle *h)
{
    if (!h) return fail(MD_ERR_INVALID_ARG, "handle is NULL");
    hipError_t e = hipSetDevice(h->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    return MD_OK;
}

// Counting sort into cells + gather into cell order + copy back in place.
static bool use_window(const md_config &c, const Geom &g);
static bool use_window(const md_handle *h) { return !h->no_window && use_window(h->cfg, h->g); }
static int build_blocks(md_handle *h, hipStream_t s);
static int ensure_cube_part(md_handle *h);

// Where the particle arrays of a time-stepping call currently live.  Inside
// md_step a cell build does not copy the reordered arrays back: the current
// arrays and the build's output buffers trade places (cur points at the
// caller's or the handle's buffers; md_step copies back once at its end).
struct CurArrays {
    double **pos;
    void **vel, **force;
    int32_t **type, **ids;
};

// check_window: when the configuration runs over LDS windows, wait for the
// block packer and read whether some cell neighbourhood exceeds the window
// tile; if so the handle switches to the global kernels (and md_status
// reports MD_FLAG_WINDOW_FALLBACK).  Without it (the rebuilds inside md_step's
// blocks) the flag is read at the block's end and the block is redone.
static int window_overflow_fallback(md_handle *h, hipStream_t s);

static int build_cells_impl(md_handle *h, double *pos, void *vel, void *force, int32_t *type, int32_t *ids,
                            hipStream_t s, const CurArrays *cur = nullptr, bool check_window = true)
{
    const Geom &g = h->g;
    Buffers &b = h->b;
    int n = (int)h->n;
    size_t rs = real_size(h->cfg);
    int rc = ensure_cells(h, g);
    if (rc) return rc;
    launch_fill_i32(b.cell_count, 0, g.ncell, s);
    launch_cell_hist(n, pos, g, b.cell_id, b.slot, b.cell_count, b.flags, s);
    launch_scan(b.cell_count, b.cell_start, g.ncell, b.scan_blocks, s);
    if (h->cfg.container == MD_CONTAINER_CL) {
        launch_scatter(n, b.cell_id, b.slot, b.cell_start, b.perm, s);
        // cluster lists order each cell by position (Morton code), then id
        if (!b.cl_key) {
            int rc2 = dalloc(&b.cl_key, (size_t)std::max<int64_t>(h->n, 1));
            if (rc2) return rc2;
        }
        launch_cl_sort(n, b.cell_start, pos, ids, b.cell_id, b.perm, g, b.cl_key, b.cell_sorted, b.perm2, s);
    } else {
        // every cell ordered by x, then id (the Verlet-list build bisects its
        // stencil rows by x)
        if (!b.cl_key) {
            int rc2 = dalloc(&b.cl_key, (size_t)std::max<int64_t>(h->n, 1));
            if (rc2) return rc2;
        }
        launch_scatter_sort_x(n, b.cell_id, b.slot, b.cell_start, ids, pos, g, b.perm, b.cl_key, b.cell_sorted,
                              b.perm2, s);
    }
    launch_gather(n, h->cfg.precision, b.perm2, pos, vel, force, type, ids, b.tmp_pos, b.tmp_vel, b.tmp_force,
                  b.tmp_type, b.tmp_ids, b.cell_id, b.cell_sorted, g, b.stage, b.stage_ref, s);
    if (cur) {
        // the gathered buffers become the current arrays, the old ones the
        // next build's output buffers (forces only if they were gathered)
        std::swap(*cur->pos, b.tmp_pos);
        if (vel) std::swap(*cur->vel, b.tmp_vel);
        if (force) std::swap(*cur->force, b.tmp_force);
        std::swap(*cur->type, b.tmp_type);
        std::swap(*cur->ids, b.tmp_ids);
    } else if (n > 0) {
        MD_HIP(hipMemcpyAsync(pos, b.tmp_pos, 3 * (size_t)n * sizeof(double), hipMemcpyDeviceToDevice, s));
        if (vel) MD_HIP(hipMemcpyAsync(vel, b.tmp_vel, 3 * (size_t)n * rs, hipMemcpyDeviceToDevice, s));
        if (force) MD_HIP(hipMemcpyAsync(force, b.tmp_force, 3 * (size_t)n * rs, hipMemcpyDeviceToDevice, s));
        MD_HIP(hipMemcpyAsync(type, b.tmp_type, (size_t)n * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
        MD_HIP(hipMemcpyAsync(ids, b.tmp_ids, (size_t)n * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
    }
    launch_fill_i32(b.flags + 1, INT32_MAX, 1, s);
    h->rebuilds++;
    h->age = 0;
    h->built = true;
    h->lists = false;
    if (h->cfg.newton3 == MD_N3L_C08 && (rc = ensure_cube_part(h))) return rc;
    if (!use_window(h)) return MD_OK;
    if ((rc = build_blocks(h, s))) return rc;
    if (!check_window) return MD_OK;
    MD_HIP(hipMemcpyAsync(h->b.host_flags + 3, h->b.flags + 3, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    MD_HIP(hipStreamSynchronize(s));
    if (h->b.host_flags[3] & 1u) return window_overflow_fallback(h, s);
    return MD_OK;
}

// The packer met a cell column whose window exceeds the LDS tile: the
// windowed kernels would skip its blocks, so the handle uses the global
// kernels from now on (the cells are valid for them as they are).
static int window_overflow_fallback(md_handle *h, hipStream_t s)
{
    h->no_window = true;
    h->sticky |= MD_FLAG_WINDOW_FALLBACK;
    h->lists = false;
    launch_fill_i32(h->b.flags + 3, 0, 1, s);
    return MD_OK;
}

namespace mdlj {
// Cluster arrays: clusters <= n/8 + cells; the list rows hold up to
// max_neighbors j-clusters.
static int ensure_clusters(md_handle *h)
{
    Buffers &b = h->b;
    int rc;
    int64_t cap = cluster_cap(h->n, h->g);
    int64_t maxn = h->cfg.max_neighbors;
    if (cap > b.cl_cap || maxn > b.cl_list_cap) {
        void *ptrs[] = {b.cl_start, b.cl_count, b.cl_cell, b.cl_centre, b.cl_half, b.cl_nbr, b.cl_nbr_count};
        for (void *p : ptrs)
            if (p) (void)hipFree(p);
        b.cl_start = b.cl_count = b.cl_cell = b.cl_nbr = b.cl_nbr_count = nullptr;
        b.cl_centre = nullptr;
        b.cl_half = nullptr;
        if ((rc = dalloc(&b.cl_start, cap)) || (rc = dalloc(&b.cl_count, cap)) || (rc = dalloc(&b.cl_cell, cap)) ||
            (rc = dalloc(&b.cl_centre, cap)) || (rc = dalloc(&b.cl_half, cap)) ||
            (rc = dalloc(&b.cl_nbr, (size_t)cap * maxn)) || (rc = dalloc(&b.cl_nbr_count, cap)))
            return rc;
        b.cl_cap = cap;
        b.cl_list_cap = maxn;
    }
    if ((int64_t)h->g.ncell + 1 > b.cl_base_cap) {
        if (b.cl_base) (void)hipFree(b.cl_base);
        b.cl_base = nullptr;
        if ((rc = dalloc(&b.cl_base, (size_t)h->g.ncell + 1))) return rc;
        b.cl_base_cap = (int64_t)h->g.ncell + 1;
    }
    return MD_OK;
}
}

// FP32 linked cells and Verlet lists run over LDS windows (Verlet lists as
// 16-bit window positions): full windows gather-only, half windows with
// Newton's third law.  The FP64 path, cell grids with a reach above one cell
// and half traversals of grids with fewer than three cells per dimension use
// the global kernels (32-bit lists).
static bool use_window(const md_config &c, const Geom &g)
{
    return (c.container == MD_CONTAINER_VL || c.container == MD_CONTAINER_LC) && c.precision == MD_FP32 &&
           c.newton3 != MD_N3L_C08 && window_geometry_ok(g, c.newton3 == MD_N3L_ON);
}

static int ensure_window(md_handle *h, int64_t maxn)
{
    Buffers &b = h->b;
    int rc;
    int64_t cap = window_block_cap(h->n, h->g);
    if (cap > b.w_cap) {
        if (b.w_blk) (void)hipFree(b.w_blk);
        b.w_blk = nullptr;
        b.w_cap = 0;
        if ((rc = dalloc(&b.w_blk, cap))) return rc;
        b.w_cap = cap;
    }
    int64_t staged = window_staged_blocks(h->g);
    if (staged > b.w_staged_cap) {
        if (b.w_staged) (void)hipFree(b.w_staged);
        b.w_staged = nullptr;
        b.w_staged_cap = 0;
        if ((rc = dalloc(&b.w_staged, staged))) return rc;
        b.w_staged_cap = staged;
    }
    int64_t rows = (int64_t)h->g.nc[1] * h->g.nc[2] + 1;
    if (rows > b.w_rows_cap) {
        for (int32_t **p : {&b.w_rown, &b.w_rowb}) {
            if (*p) (void)hipFree(*p);
            *p = nullptr;
            if ((rc = dalloc(p, rows))) return rc;
        }
        b.w_rows_cap = rows;
    }
    if (h->cfg.container == MD_CONTAINER_VL && (maxn > b.w_nbr_cap || !b.w_nbr)) {
        if (b.w_nbr) (void)hipFree(b.w_nbr);
        b.w_nbr = nullptr;
        // entries are stored in chunks of eight, plus one chunk row that the
        // force kernels' prefetch may read past a full list
        int64_t rows8 = (maxn + 7) / 8 * 8 + 8;
        if ((rc = dalloc(&b.w_nbr, (size_t)rows8 * (size_t)std::max<int64_t>(h->n, 1)))) return rc;
        b.w_nbr_cap = maxn;
    }
    return MD_OK;
}

// Blocks of the windowed traversals (after every cell build).
static int build_blocks(md_handle *h, hipStream_t s)
{
    Buffers &b = h->b;
    int rc = ensure_window(h, h->cfg.max_neighbors);
    if (rc) return rc;
    launch_blocks(h->g, b.cell_start, b.w_staged, b.w_rown, b.w_rowb, b.scan_blocks, b.w_blk, (int)b.w_cap,
                  b.flags, h->cfg.newton3 == MD_N3L_ON, s);
    return MD_OK;
}

// Pairwise Verlet lists: 13 sorted orders and projections and 26 prefix
// lengths per particle.
static int ensure_pvl(md_handle *h)
{
    Buffers &b = h->b;
    int64_t n = std::max<int64_t>(h->n, 1);
    if (n > b.pvl_cap) {
        void *ptrs[] = {b.pvl_perm, b.pvl_cnt, b.pvl_s};
        for (void *p : ptrs)
            if (p) (void)hipFree(p);
        b.pvl_perm = b.pvl_cnt = nullptr;
        b.pvl_s = nullptr;
        b.pvl_cap = 0;
        int rc;
        if ((rc = dalloc(&b.pvl_perm, (size_t)13 * n)) || (rc = dalloc(&b.pvl_cnt, (size_t)26 * n)) ||
            (rc = dalloc(&b.pvl_s, (size_t)13 * n)))
            return rc;
        b.pvl_cap = n;
    }
    return MD_OK;
}

// Per-cube energy partials [ncell][4] of the C08 traversals.
static int ensure_cube_part(md_handle *h)
{
    Buffers &b = h->b;
    if ((int64_t)h->g.ncell <= b.vlc_part_cap) return MD_OK;
    if (b.vlc_part) (void)hipFree(b.vlc_part);
    b.vlc_part = nullptr;
    b.vlc_part_cap = 0;
    int rc = dalloc(&b.vlc_part, (size_t)4 * h->g.ncell);
    if (rc) return rc;
    b.vlc_part_cap = h->g.ncell;
    return MD_OK;
}

// Verlet list cells: a row of entries per particle, [n][ld] with ld the
// capacity rounded up to a multiple of 8 (so that a row is whole 16-byte
// chunks), segment ends [4][n], per-cube energy partials [ncell][4].
static int vlc_ld(const md_handle *h) { return (h->cfg.max_neighbors + 7) & ~7; }

static int ensure_vlc(md_handle *h, int32_t maxn)
{
    Buffers &b = h->b;
    int64_t n = std::max<int64_t>(h->n, 1);
    int rc;
    if (n > b.vlc_cap || maxn > b.vlc_maxn) {
        if (b.vlc_nbr) (void)hipFree(b.vlc_nbr);
        if (b.vlc_seg) (void)hipFree(b.vlc_seg);
        b.vlc_nbr = b.vlc_seg = nullptr;
        b.vlc_cap = 0;
        b.vlc_maxn = 0;
        const size_t ld = (size_t)((maxn + 7) & ~7);
        if ((rc = dalloc(&b.vlc_nbr, ld * n)) || (rc = dalloc(&b.vlc_seg, (size_t)4 * n))) return rc;
        b.vlc_cap = n;
        b.vlc_maxn = maxn;
    }
    return ensure_cube_part(h);
}

static int build_lists_impl(md_handle *h, const double *pos, hipStream_t s)
{
    Buffers &b = h->b;
    int n = (int)h->n;
    if (use_window(h) && h->cfg.container == MD_CONTAINER_VL) {
        int rc = ensure_window(h, h->cfg.max_neighbors);
        if (rc) return rc;
        const Geom &g = h->g;
        launch_fill_i32(b.flags + 2, 0, 1, s);
        launch_vlw_build(b.stage, b.cell_start, b.cell_sorted, pos, g, n, b.w_rowb + window_nbands(g), b.w_blk,
                         b.w_nbr, b.nbr_count, h->cfg.max_neighbors, b.flags, h->cfg.newton3 == MD_N3L_ON, s);
    } else if (h->cfg.container == MD_CONTAINER_VL) {
        int rc = ensure_list(h, h->cfg.max_neighbors);
        if (rc) return rc;
        launch_fill_i32(b.flags + 2, 0, 1, s);
        launch_vl_build(n, b.stage, b.cell_start, b.cell_sorted, pos, h->g, h->cfg.newton3, b.nbr, b.nbr_count,
                        n, h->cfg.max_neighbors, b.flags, s);
    } else if (h->cfg.container == MD_CONTAINER_VLC) {
        int rc = ensure_vlc(h, h->cfg.max_neighbors);
        if (rc) return rc;
        launch_fill_i32(b.flags + 2, 0, 1, s);
        launch_vlc_build(n, b.stage, b.cell_start, b.cell_sorted, pos, h->g, b.vlc_nbr, b.vlc_seg, b.nbr_count,
                         vlc_ld(h), b.flags, s);
    } else if (h->cfg.container == MD_CONTAINER_PVL) {
        int rc = ensure_pvl(h);
        if (rc) return rc;
        launch_pvl_build(n, b.stage, b.cell_start, b.cell_sorted, h->g, b.pvl_s, b.pvl_perm, b.pvl_cnt, s);
    } else if (h->cfg.container == MD_CONTAINER_CL) {
        int rc = ensure_clusters(h);
        if (rc) return rc;
        launch_fill_i32(b.flags + 2, 0, 1, s);
        // per-cell cluster counts go to the (free after the build) count buffer
        launch_cluster_build(n, h->g, b.cell_start, b.stage, b.cell_count, b.cl_base, b.scan_blocks, b.cl_start,
                             b.cl_count, b.cl_cell, b.cl_centre, b.cl_half, b.cl_nbr, b.cl_nbr_count, b.cl_cap,
                             h->cfg.max_neighbors, b.flags, s);
    }
    h->lists = true;
    return MD_OK;
}

static int check_particles(md_handle *h, const void *pos, const void *type)
{
    if (h->n > 0 && (!pos || !type)) return fail(MD_ERR_INVALID_ARG, "pos and type must not be NULL");
    return MD_OK;
}

extern "C" int md_build_cells(md_handle *h, double *pos, void *vel, void *force, int32_t *type, int32_t *ids,
                              void *stream)
{
    int rc = check_handle(h);
    if (rc) return rc;
    if ((rc = check_particles(h, pos, type))) return rc;
    if (h->n > 0 && !ids) return fail(MD_ERR_INVALID_ARG, "ids must not be NULL");
    return build_cells_impl(h, pos, vel, force, type, ids, (hipStream_t)stream);
}

extern "C" int md_build_neighbors(md_handle *h, const double *pos, const int32_t *type, void *stream)
{
    int rc = check_handle(h);
    if (rc) return rc;
    if ((rc = check_particles(h, pos, type))) return rc;
    if (!h->built) return fail(MD_ERR_NOT_BUILT, "md_build_cells must be called first");
    hipStream_t s = (hipStream_t)stream;
    launch_stage((int)h->n, pos, type, h->g, h->b.stage, s);
    return build_lists_impl(h, pos, s);
}

// ------------------------------------------------------------------ forces

static ForceArgs force_args(md_handle *h, const double *pos, const int32_t *type, void *force, bool energy)
{
    ForceArgs a;
    memset(&a, 0, sizeof(a));
    a.n = (int)h->n;
    a.precision = h->cfg.precision;
    a.container = h->cfg.container;
    a.newton3 = h->cfg.newton3;
    a.energy = energy;
    a.pos = pos;
    a.type = type;
    a.stage = h->b.stage;
    a.cell_start = h->b.cell_start;
    a.cell_sorted = h->b.cell_sorted;
    a.nbr = h->b.nbr;
    a.nbr_count = h->b.nbr_count;
    a.nbr_ld = h->n;
    a.cl_start = h->b.cl_start;
    a.cl_count = h->b.cl_count;
    a.cl_nbr = h->b.cl_nbr;
    a.cl_nbr_count = h->b.cl_nbr_count;
    a.cl_ld = h->b.cl_cap;
    a.n_clusters = (int)h->b.cl_cap;
    a.cl_ncl = h->b.cl_base ? h->b.cl_base + h->g.ncell : nullptr;
    a.pvl_perm = h->b.pvl_perm;
    a.pvl_cnt = h->b.pvl_cnt;
    a.vlc_nbr = h->b.vlc_nbr;
    a.vlc_seg = h->b.vlc_seg;
    a.vlc_ld = vlc_ld(h);
    a.vlc_part = h->b.vlc_part;
    a.vlc_blocks = vlc_force_blocks(h->g);
    a.tab = h->b.tab;
    a.force = force;
    a.partials = h->b.partials;
    a.flags = h->b.flags;
    a.window = use_window(h);
    if (a.window) {
        a.w_nblk = h->b.w_rowb + window_nbands(h->g);
        a.w_blk = h->b.w_blk;
        a.w_nbr = h->b.w_nbr;
    }
    return a;
}

static int forces_impl(md_handle *h, const double *pos, const int32_t *type, void *force, bool energy,
                       hipStream_t s)
{
    ForceArgs a = force_args(h, pos, type, force, energy);
    if (force_blocks(a) > kMaxPartials) return fail(MD_ERR_INVALID_ARG, "too many particles for the reduction");
    if (h->cfg.newton3 != MD_N3L_OFF) launch_zero(force, 3 * h->n * (int64_t)real_size(h->cfg), s);
    launch_force(a, h->g, s);
    if (energy) {
        h->energy_gather = h->cfg.newton3 == MD_N3L_OFF;
        h->epart_blocks = force_blocks(a);
    }
    return MD_OK;
}

extern "C" int md_compute_forces(md_handle *h, const double *pos, const int32_t *type, const double *lj,
                                 void *force, double *out, void *stream)
{
    int rc = check_handle(h);
    if (rc) return rc;
    if ((rc = check_particles(h, pos, type))) return rc;
    if (!lj || (h->n > 0 && !force)) return fail(MD_ERR_INVALID_ARG, "lj and force must not be NULL");
    if (!h->built) return fail(MD_ERR_NOT_BUILT, "md_build_cells (and md_build_neighbors) must be called first");
    if (has_lists(h->cfg) && !h->lists)
        return fail(MD_ERR_NOT_BUILT, "md_build_neighbors must be called after md_build_cells");
    hipStream_t s = (hipStream_t)stream;
    launch_prepare_tab(lj, h->cfg.rc2, h->g, h->b.tab, s);
    launch_stage((int)h->n, pos, type, h->g, h->b.stage, s);
    if ((rc = forces_impl(h, pos, type, force, out != nullptr, s))) return rc;
    if (out) {
        ForceArgs a = force_args(h, pos, type, force, true);
        launch_reduce_out(h->b.partials, force_blocks(a), h->cfg.newton3 == MD_N3L_OFF, out, s);
    }
    return MD_OK;
}

// ------------------------------------------------------------------ time stepping

struct StepCtx {
    // the current particle arrays: the caller's, or after a cell build the
    // handle's buffers (see CurArrays); shared by every function of the call
    mutable double *pos;
    mutable void *vel, *force;
    mutable int32_t *type, *ids;
    const double *inv_mass, *lj;
    double dt;
    int32_t nsteps, energy_every;
    double *log;
    hipStream_t s;
};

static IntegrateArgs integ_args(md_handle *h, const StepCtx &c, int kick_prev, int start, int energy, int step,
                                bool track = false)
{
    IntegrateArgs a;
    memset(&a, 0, sizeof(a));
    a.n = (int)h->n;
    a.precision = h->cfg.precision;
    a.pos = c.pos;
    a.vel = c.vel;
    a.force = c.force;
    a.type = c.type;
    a.inv_mass = c.inv_mass;
    a.hdt = 0.5 * c.dt;
    a.dt = c.dt;
    a.kick_prev = kick_prev;
    a.start = start;
    a.energy = energy;
    a.step_index = step;
    a.stage = h->b.stage;
    a.stage_ref = h->b.stage_ref;
    a.flags = h->b.flags;
    a.kpart = h->b.kpart;
    a.dpart = track ? h->b.dpart : nullptr;
    return a;
}

static bool logs_step(const StepCtx &c, int s)  // log after step s (0-based)?
{
    return c.log && c.energy_every > 0 && (s + 1) % c.energy_every == 0;
}

// Events of the kernel-class timing: a pool reused once the recorded pairs
// have been read back (at every block-end synchronisation).
static hipEvent_t timing_event(md_handle *h)
{
    if (!h->timing) return nullptr;
    if (h->tnext == h->tpool.size()) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        h->tpool.push_back(e);
    }
    return h->tpool[h->tnext++];
}

static void timing_collect(md_handle *h)
{
    for (const auto &p : h->tpend) {
        float ms = 0.f;
        if (hipEventSynchronize(p.b) == hipSuccess && hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
            h->tsum[2 * p.kind] += ms;
            h->tsum[2 * p.kind + 1] += 1.0;
        }
    }
    h->tpend.clear();
    h->tnext = 0;
}

// Cells and lists for the current positions.  with_force = false inside a
// step, after the drift: the forces of the previous step have been used by
// both kicks and are about to be recomputed, so they are not reordered.
static int rebuild(md_handle *h, const StepCtx &c, bool with_force = true, bool check_window = true)
{
    CurArrays cur{&c.pos, &c.vel, &c.force, &c.type, &c.ids};
    int rc = build_cells_impl(h, c.pos, c.vel, with_force ? c.force : nullptr, c.type, c.ids, c.s, &cur,
                              check_window);
    if (rc) return rc;
    return build_lists_impl(h, c.pos, c.s);
}

// One time step s: finish step s-1 (second kick, kinetic energy and, unless
// suppressed, its log entry), start step s (kick, drift, stage, skin check),
// rebuild when the structure is due (or when force_rebuild), then forces.
static int snapshot(md_handle *h, const StepCtx &c, bool restore, bool with_force);
static int step_forces(md_handle *h, const StepCtx &c, int s, bool fuse = false, bool track_next = false);

static int one_step(md_handle *h, const StepCtx &c, int s, bool force_rebuild, bool log_prev_ok = true,
                    bool snap_after_rebuild = false, bool track = false, bool fuse = false, bool track_next = false)
{
    bool log_prev = s > 0 && logs_step(c, s - 1) && log_prev_ok;
    if (h->started == s) {
        // the previous force pass has done the integration (the kinetic
        // energy and displacement partials included)
        h->started = -1;
    } else {
        launch_integrate(integ_args(h, c, s > 0, 1, log_prev, s, track), h->g, c.s);
        h->kpart_blocks = integrate_blocks((int)h->n);
        if (track) h->dpart_blocks = integrate_blocks((int)h->n);
    }
    if (log_prev) {
        // the slots the energy pass wrote: a tuning trial may have switched the
        // configuration (and the kernel's partial count) since
        launch_log_entry(h->b.partials, h->epart_blocks, h->energy_gather, h->b.kpart, h->kpart_blocks,
                         c.log + 4 * (s / c.energy_every - 1), c.s);
    }
    h->age++;
    if (force_rebuild || h->age >= h->cfg.rebuild_interval) {
        hipEvent_t e0 = timing_event(h), e1 = nullptr;
        if (e0) MD_HIP(hipEventRecord(e0, c.s));
        // a block's scheduled rebuild leaves the window check to the block's
        // end (read_flags); a forced one checks at once
        int rc = rebuild(h, c, false, force_rebuild);
        if (rc) return rc;
        if (e0 && (e1 = timing_event(h))) {
            MD_HIP(hipEventRecord(e1, c.s));
            h->tpend.push_back({e0, e1, 1});
        }
        if (snap_after_rebuild && (rc = snapshot(h, c, false, false))) return rc;
    }
    return step_forces(h, c, s, fuse, track_next);
}

// The force pass of step s (energy partials when step s is logged).
// The force pass of step s.  fuse: step s + 1 follows at once (same block,
// no host decision in between), so with the Verlet-list gather kernel the
// pass also does step s + 1's integration (second half kick of s, first
// half kick and drift of s + 1): the positions and stage go to the second
// buffers, which then become the current ones.  track_next: record the
// displacement partials of that integration (the autotuner's motion).
static bool fusable(const md_handle *h)
{
    return use_window(h) && h->cfg.container == MD_CONTAINER_VL && h->cfg.newton3 == MD_N3L_OFF &&
           h->lists;
}

static int step_forces(md_handle *h, const StepCtx &c, int s, bool fuse, bool track_next)
{
    hipEvent_t e0 = timing_event(h), e1 = nullptr;
    if (e0) MD_HIP(hipEventRecord(e0, c.s));
    int rc;
    bool energy = logs_step(c, s);
    if (fuse && fusable(h)) {
        Buffers &b = h->b;
        size_t n = (size_t)h->n;
        if (!b.pos_alt && ((rc = dalloc(&b.pos_alt, 3 * std::max<size_t>(n, 1))) ||
                           (rc = dalloc(&b.stage_alt, std::max<size_t>(n, 1)))))
            return rc;
        ForceArgs a = force_args(h, c.pos, c.type, c.force, energy);
        if (force_blocks(a) > kMaxPartials) return fail(MD_ERR_INVALID_ARG, "too many particles for the reduction");
        a.fused = true;
        a.ia = integ_args(h, c, 1, 1, energy, s + 1, track_next);
        a.ia.stage = b.stage_alt;
        a.pos_out = b.pos_alt;
        a.stage_out = b.stage_alt;
        launch_force(a, h->g, c.s);
        if (energy) {
            h->energy_gather = true;
            h->epart_blocks = force_blocks(a);
        }
        std::swap(c.pos, b.pos_alt);
        std::swap(b.stage, b.stage_alt);
        h->started = s + 1;
        h->kpart_blocks = force_blocks(a);
        if (track_next) h->dpart_blocks = force_blocks(a);
        rc = MD_OK;
    } else {
        rc = forces_impl(h, c.pos, c.type, c.force, energy, c.s);
    }
    if (e0 && (e1 = timing_event(h))) {
        MD_HIP(hipEventRecord(e1, c.s));
        h->tpend.push_back({e0, e1, 0});
    }
    return rc;
}

// Snapshot of the state a block may be replayed from: positions and
// velocities, plus forces when the snapshot precedes an integration.  Types
// and ids change only at rebuilds, which never fall inside a replayed span.
static int snapshot(md_handle *h, const StepCtx &c, bool restore, bool with_force)
{
    Buffers &b = h->b;
    size_t n = (size_t)h->n;
    size_t rs = real_size(h->cfg);
    int rc;
    if (!b.snap_pos) {
        if ((rc = dalloc(&b.snap_pos, 3 * n))) return rc;
        if ((rc = dalloc_bytes(&b.snap_vel, 3 * n * rs))) return rc;
        if ((rc = dalloc_bytes(&b.snap_force, 3 * n * rs))) return rc;
    }
    if (n == 0) return MD_OK;
    auto cp = [&](void *dst, const void *src, size_t bytes) {
        return hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, c.s);
    };
    if (!restore) {
        MD_HIP(cp(b.snap_pos, c.pos, 3 * n * 8));
        MD_HIP(cp(b.snap_vel, c.vel, 3 * n * rs));
        if (with_force) MD_HIP(cp(b.snap_force, c.force, 3 * n * rs));
    } else {
        h->started = -1;
        MD_HIP(cp(c.pos, b.snap_pos, 3 * n * 8));
        MD_HIP(cp(c.vel, b.snap_vel, 3 * n * rs));
        if (with_force) MD_HIP(cp(c.force, b.snap_force, 3 * n * rs));
        // the FP32 kernels and the list builds read the staged copy of the
        // positions: stage the restored ones
        launch_stage((int)n, c.pos, c.type, h->g, b.stage, c.s);
    }
    return MD_OK;
}

// Bit of read_flags' out[0] (above the device flag bits): the block's cell
// build overflowed the LDS windows and its forces must be redone.
constexpr int32_t kWindowRedo = 1 << 16;

// Read the device flags (synchronises the stream).
static int read_flags(md_handle *h, hipStream_t s, int32_t out[4])
{
    MD_HIP(hipMemcpyAsync(h->b.host_flags, h->b.flags, 5 * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    MD_HIP(hipStreamSynchronize(s));
    out[0] = (int32_t)h->b.host_flags[0];
    out[1] = (int32_t)h->b.host_flags[1];
    out[2] = (int32_t)h->b.host_flags[2];
    out[3] = (int32_t)h->b.host_flags[4];  // squared displacement since the build (float bits)
    timing_collect(h);
    if (h->b.host_flags[0] & MD_FLAG_NONFINITE) {
        // checked first: a particle far outside the box is binned into an
        // edge cell, which can also overfill a window
        h->sticky |= MD_FLAG_NONFINITE;
        return fail(MD_ERR_NONFINITE,
                    "a position outside the box (beyond one cell) or a non-finite position or force appeared; "
                    "md_status clears the flag");
    }
    if (h->b.host_flags[3] & 1u) {
        // the packer of this block's cell build met a cell column whose
        // window exceeds the tile (the kernels skipped its blocks): switch to
        // the global kernels; the caller redoes the block's forces
        int rc = window_overflow_fallback(h, s);
        if (rc) return rc;
        out[0] |= kWindowRedo;
    } else if (h->b.host_flags[3]) {
        // a kernel met a block whose window does not fit, which the packer
        // never makes
        return fail(MD_ERR_HIP, "internal error: a windowed kernel met an unpacked block");
    }
    return MD_OK;
}

// Largest displacement per step, from the largest squared displacement
// since the last build (d2bits: float bits, fixed-point units) after h->age
// steps; particles move ballistically between builds, so it grows linearly.
static void update_motion(md_handle *h, int32_t d2bits)
{
    float d2;
    memcpy(&d2, &d2bits, sizeof(d2));
    if (!(d2 > 0.f) || h->age < 1) return;
    h->rate[h->rate_pos++ & 3] = sqrt((double)d2) / (double)h->age;
}

// Rebuild interval derived by the autotuner.  A structure built at step s
// serves the forces of steps s .. s + R - 1, after 0 .. R - 1 drifts: R is
// the most steps that keep the fastest recent particle's displacement after
// R - 1 drifts within 95 % of skin/2 (the skin check and the replay still
// guard every step).  The base interval until motion has been measured.
static int derived_interval(const md_handle *h)
{
    double r = 0.0;
    for (double v : h->rate) r = std::max(r, v);
    if (!(h->cfg.skin > 0.0)) return 1;
    if (r <= 0.0) return h->base.rebuild_interval;
    double R = floor(0.95 * sqrt((double)h->g.disp2) / r) + 1.0;
    return (int)std::max(1.0, std::min(R, 100.0));
}

// Run one block of steps starting at s0: a rebuild can only happen at the
// block's first step (after its integration, when the structure is due); the
// block then runs until the step before the next due rebuild, or s_end - 1.
// Afterwards the device flags are read.  If the skin check fired at a step v
// whose forces used the block's structure, the block is replayed from its
// snapshot (deterministically, same structure) up to v - 1 and rebuilt right
// after the integration of v.  If the list overflowed at the block's rebuild,
// the list grows and the block is replayed.  *next = first step not yet done.
static int run_block(md_handle *h, const StepCtx &c, int s0, int s_end, int *next)
{
    int R = h->cfg.rebuild_interval;
    int age0 = h->age;
    bool rebuild_first = age0 + 1 >= R;
    int len = rebuild_first ? R : R - age0 - 1;
    int last = std::min(s_end - 1, s0 + std::max(len, 1) - 1);
    int rc;
    // rebuild_first: snapshot right after the rebuild of step s0 (cell order
    // of the block); otherwise before step s0, forces included.
    if (!rebuild_first && (rc = snapshot(h, c, false, true))) return rc;
    launch_fill_i32(h->b.flags + 1, INT32_MAX, 1, c.s);
    // the autotuner tracks the motion at the block's last step
    bool track = h->tuner != nullptr;
    // every step but the block's last hands its successor's integration to
    // its force pass where the configuration allows (fused integrator)
    for (int st = s0; st <= last; st++)
        if ((rc = one_step(h, c, st, false, true, rebuild_first && st == s0, track && st == last, st < last,
                           track && st + 1 == last)))
            return rc;
    if (track) launch_dmax_reduce(h->b.dpart, h->dpart_blocks, h->b.flags, c.s);
    int32_t f[4];
    if ((rc = read_flags(h, c.s, f))) return rc;
    if (track) update_motion(h, f[3]);
    int v = f[1];
    int first_used = rebuild_first ? s0 + 1 : s0;  // first step whose forces used the checked structure
    bool overflow = (f[0] & MD_FLAG_LIST_OVERFLOW) != 0;
    if (f[0] & kWindowRedo) {
        // the cell build of step s0 overflowed the LDS windows (only a
        // block's own rebuild is checked here; every other build is checked
        // when it is made): rebuild the lists for the global kernels from the
        // snapshot and redo step s0's forces; the rest of the block is run
        // again
        if (!rebuild_first) return fail(MD_ERR_HIP, "internal error: window overflow outside a block's rebuild");
        launch_fill_i32(h->b.flags, 0, 1, c.s);
        if ((rc = snapshot(h, c, true, false))) return rc;
        for (;;) {
            if (has_lists(h->cfg) && (rc = build_lists_impl(h, c.pos, c.s))) return rc;
            if ((rc = step_forces(h, c, s0))) return rc;
            if (!has_lists(h->cfg)) break;
            // the global lists must not be truncated either
            if ((rc = read_flags(h, c.s, f))) return rc;
            if (!(f[0] & MD_FLAG_LIST_OVERFLOW)) break;
            if (h->cfg.max_neighbors >= 4096)
                return fail(MD_ERR_LIST_OVERFLOW, "neighbour rows exceed the largest max_neighbors (4096)");
            h->cfg.max_neighbors = std::min(4096, std::max(h->cfg.max_neighbors * 3 / 2, f[2] + 16));
            launch_fill_i32(h->b.flags, 0, 1, c.s);
        }
        h->age = 0;
        *next = s0 + 1;
        return MD_OK;
    }
    if (overflow && rebuild_first && has_lists(h->cfg) && h->cfg.max_neighbors < 4096) {
        // the lists built at step s0 were truncated: grow them, rebuild the
        // lists from the snapshot (the cells are still valid for it) and redo
        // step s0's forces; the rest of the block is run again
        h->sticky |= (uint32_t)f[0] & ~MD_FLAG_LIST_OVERFLOW;
        h->cfg.max_neighbors = std::min(4096, std::max(h->cfg.max_neighbors * 3 / 2, f[2] + 16));
        launch_fill_i32(h->b.flags, 0, 1, c.s);
        if ((rc = snapshot(h, c, true, false))) return rc;
        if ((rc = build_lists_impl(h, c.pos, c.s))) return rc;
        if ((rc = step_forces(h, c, s0))) return rc;
        h->age = 0;
        *next = s0 + 1;
        return MD_OK;
    }
    if (v >= first_used && v <= last) {
        // replay deterministically with the same structure, then rebuild
        // right after the integration of step v
        if (rebuild_first) {
            if ((rc = snapshot(h, c, true, false))) return rc;
            if ((rc = step_forces(h, c, s0))) return rc;
            h->age = 0;
            for (int st = s0 + 1; st < v; st++)
                if ((rc = one_step(h, c, st, false))) return rc;
        } else {
            if ((rc = snapshot(h, c, true, true))) return rc;
            h->age = age0;
            for (int st = s0; st < v; st++)
                if ((rc = one_step(h, c, st, false, st != s0))) return rc;
        }
        if ((rc = one_step(h, c, v, true, v != s0))) return rc;
        h->forced++;
        // the forced rebuild's lists must not be truncated either
        if ((rc = read_flags(h, c.s, f))) return rc;
        if ((f[0] & MD_FLAG_LIST_OVERFLOW) && has_lists(h->cfg)) {
            h->sticky |= (uint32_t)f[0] & ~MD_FLAG_LIST_OVERFLOW;
            h->cfg.max_neighbors = std::min(4096, std::max(h->cfg.max_neighbors * 3 / 2, f[2] + 16));
            launch_fill_i32(h->b.flags, 0, 1, c.s);
            if ((rc = build_lists_impl(h, c.pos, c.s))) return rc;
            if ((rc = step_forces(h, c, v))) return rc;
        }
        *next = v + 1;
        return MD_OK;
    }
    *next = last + 1;
    return MD_OK;
}

static int finish_steps(md_handle *h, const StepCtx &c)
{
    bool log_last = logs_step(c, c.nsteps - 1);
    launch_integrate(integ_args(h, c, 1, 0, log_last, c.nsteps), h->g, c.s);
    if (log_last) {
        launch_log_entry(h->b.partials, h->epart_blocks, h->energy_gather, h->b.kpart,
                         integrate_blocks((int)h->n), c.log + 4 * (c.nsteps / c.energy_every - 1), c.s);
    }
    return MD_OK;
}

int run_tuning_phase(md_handle *h, const StepCtx &c, int s0, int *next);
int apply_config(md_handle *h, const md_config &nc);
static int run_steps(md_handle *h, const StepCtx &c, int s0, int s1);

static int run_steps(md_handle *h, const StepCtx &c, int s0, int s1)
{
    int s = s0;
    h->replay_no_log = false;
    while (s < s1) {
        if (h->tuner) h->cfg.rebuild_interval = derived_interval(h);
        int next = s;
        int rc = run_block(h, c, s, s1, &next);
        if (rc) return rc;
        s = next;
    }
    return MD_OK;
}

extern "C" int md_step(md_handle *h, double *pos, void *vel, void *force, int32_t *type, int32_t *ids,
                       const double *inv_mass, const double *lj, double dt, int32_t nsteps, int32_t energy_every,
                       double *log, void *stream)
{
    int rc = check_handle(h);
    if (rc) return rc;
    if ((rc = check_particles(h, pos, type))) return rc;
    if (h->n > 0 && (!vel || !force || !ids)) return fail(MD_ERR_INVALID_ARG, "vel, force, ids must not be NULL");
    if (!inv_mass || !lj) return fail(MD_ERR_INVALID_ARG, "inv_mass and lj must not be NULL");
    if (nsteps < 0) return fail(MD_ERR_INVALID_ARG, "nsteps must be >= 0");
    if (!(dt > 0.0) || !isfinite(dt)) return fail(MD_ERR_INVALID_ARG, "dt must be positive");
    if (energy_every < 0) return fail(MD_ERR_INVALID_ARG, "energy_every must be >= 0");
    if (nsteps == 0) return MD_OK;
    StepCtx c{pos, vel, force, type, ids, inv_mass, lj, dt, nsteps, energy_every, log, (hipStream_t)stream};
    // on every return: arrays that live in the handle's buffers are copied
    // to the caller's, and those buffers go back to the handle
    struct Restore {
        md_handle *h;
        const StepCtx &c;
        double *pos;
        void *vel, *force;
        int32_t *type, *ids;
        ~Restore()
        {
            Buffers &b = h->b;
            size_t n = (size_t)h->n, rs = real_size(h->cfg);
            auto back = [&](auto *&cur, auto *&spare, auto *mine, size_t bytes) {
                if (cur == mine) return;
                if (n > 0) (void)hipMemcpyAsync(mine, cur, bytes, hipMemcpyDeviceToDevice, c.s);
                spare = cur;
                cur = mine;
            };
            // positions rotate through three buffers (the caller's, the cell
            // build's output, the fused integrator's second buffer)
            if (c.pos != pos) {
                if (n > 0) (void)hipMemcpyAsync(pos, c.pos, 3 * n * sizeof(double), hipMemcpyDeviceToDevice, c.s);
                if (b.tmp_pos == pos)
                    b.tmp_pos = c.pos;
                else if (b.pos_alt == pos)
                    b.pos_alt = c.pos;
                c.pos = pos;
            }
            back(c.vel, b.tmp_vel, vel, 3 * n * rs);
            back(c.force, b.tmp_force, force, 3 * n * rs);
            back(c.type, b.tmp_type, type, n * sizeof(int32_t));
            back(c.ids, b.tmp_ids, ids, n * sizeof(int32_t));
        }
    } restore{h, c, pos, vel, force, type, ids};
    h->started = -1;
    launch_prepare_tab(lj, h->cfg.rc2, h->g, h->b.tab, c.s);
    // lists truncated since the last look (a build before this call overflowed):
    // grow them, rebuild and recompute the entry forces
    int32_t f0[4];
    if ((rc = read_flags(h, c.s, f0))) return rc;
    if (f0[0] & kWindowRedo) h->built = false;  // structures for the global kernels
    if (f0[0] & MD_FLAG_LIST_OVERFLOW) {
        h->sticky |= (uint32_t)f0[0];
        h->truncated = true;
        launch_fill_i32(h->b.flags, 0, 1, c.s);
    }
    if (h->truncated && has_lists(h->cfg)) {
        h->cfg.max_neighbors = std::min(4096, std::max(h->cfg.max_neighbors * 3 / 2, f0[2] + 16));
        h->built = false;
        h->truncated = false;
        if ((rc = rebuild(h, c))) return rc;
        if ((rc = forces_impl(h, c.pos, c.type, c.force, false, c.s))) return rc;
        int32_t f1[4];
        if ((rc = read_flags(h, c.s, f1))) return rc;
        if (f1[0] & MD_FLAG_LIST_OVERFLOW) h->truncated = true;
        if (h->truncated) return fail(MD_ERR_LIST_OVERFLOW, "neighbour rows exceed max_neighbors after growth");
    }
    if (!h->built) {
        if ((rc = rebuild(h, c))) return rc;
    }
    int s = 0;
    while (s < nsteps) {
        int s_stop = nsteps;
        if (h->tuner) {
            if (h->steps_done + s >= h->next_phase) {
                int next = s;
                if ((rc = run_tuning_phase(h, c, s, &next))) return rc;
                s = next;
                continue;
            }
            s_stop = (int)std::min<int64_t>(nsteps, h->next_phase - h->steps_done);
        }
        if ((rc = run_steps(h, c, s, s_stop))) return rc;
        s = s_stop;
    }
    h->steps_done += nsteps;
    return finish_steps(h, c);
}


// ------------------------------------------------------------------ adjoint

extern "C" int md_forces_backward(md_handle *h, const double *pos, const int32_t *type, const double *lj,
                                  const void *grad_force, double *grad_pos, double *grad_lj, void *stream)
{
    int rc = check_handle(h);
    if (rc) return rc;
    if ((rc = check_particles(h, pos, type))) return rc;
    if (!lj || !grad_lj || (h->n > 0 && (!grad_force || !grad_pos)))
        return fail(MD_ERR_INVALID_ARG, "lj, grad_force, grad_pos and grad_lj must not be NULL");
    if (!h->built) return fail(MD_ERR_NOT_BUILT, "md_build_cells must be called first");
    if (adjoint_blocks((int)h->n) > kMaxPartials) return fail(MD_ERR_INVALID_ARG, "too many particles");
    hipStream_t s = (hipStream_t)stream;
    launch_prepare_tab(lj, h->cfg.rc2, h->g, h->b.tab, s);
    launch_stage((int)h->n, pos, type, h->g, h->b.stage, s);
    AdjointArgs a;
    memset(&a, 0, sizeof(a));
    a.n = (int)h->n;
    a.precision = h->cfg.precision;
    a.pos = pos;
    a.type = type;
    a.stage = h->b.stage;
    a.cell_start = h->b.cell_start;
    a.cell_sorted = h->b.cell_sorted;
    a.tab = h->b.tab;
    a.lj = lj;
    a.grad_force = grad_force;
    a.grad_pos = grad_pos;
    a.gpart = h->b.gpart;
    a.flags = h->b.flags;
    if (use_window(h) && h->cfg.newton3 == MD_N3L_OFF && h->cfg.container == MD_CONTAINER_VL &&
        h->cfg.layout == MD_LAYOUT_PACKED && h->lists && !h->truncated) {
        // the full lists of the current build, over the same windows
        launch_adjoint_lists(h->b.stage, h->b.cell_start, h->b.cell_sorted, h->g, (int)h->n,
                             h->b.w_rowb + window_nbands(h->g), h->b.w_blk, h->b.w_nbr, h->b.nbr_count, h->b.tab,
                             pos, (const float *)grad_force, grad_pos, h->b.gpart, h->b.flags, s);
        launch_adjoint_finish(h->b.gpart, h->n > 0 ? window_force_blocks() : 0, lj, h->cfg.n_types, grad_lj, s);
        return MD_OK;
    }
    if (use_window(h) && h->cfg.newton3 == MD_N3L_OFF) {
        // the blocks of the current cell build were packed for full windows
        launch_adjoint_window(h->b.stage, h->b.cell_start, h->b.cell_sorted, h->g, (int)h->n,
                              h->b.w_rowb + window_nbands(h->g), h->b.w_blk, h->b.tab, pos,
                              (const float *)grad_force, grad_pos, h->b.gpart, h->b.flags, s);
        launch_adjoint_finish(h->b.gpart, h->n > 0 ? window_force_blocks() : 0, lj, h->cfg.n_types, grad_lj, s);
        return MD_OK;
    }
    launch_adjoint(a, h->g, s);
    launch_adjoint_finish(h->b.gpart, h->n > 0 ? adjoint_blocks((int)h->n) : 0, lj, h->cfg.n_types, grad_lj, s);
    return MD_OK;
}

// ------------------------------------------------------------------ statistics, status

// Live statistics (Sec. 4) over CSF-1 bins.  hist false: only what the
// counts alone give (mean, bins, compute units, skin; the rest NaN).
static int live_stats(md_handle *h, const double *pos, double *out, hipStream_t s, bool hist)
{
    int rc;
    Geom g;
    if ((rc = make_geom(h->cfg, 1.0, g))) return rc;
    hipDeviceProp_t prop;
    int cus = 0;
    if (hipGetDeviceProperties(&prop, h->device) == hipSuccess) cus = prop.multiProcessorCount;
    int64_t nb = (int64_t)g.ncell;
    out[0] = (double)h->n / (double)nb;
    out[1] = out[2] = out[3] = out[5] = NAN;
    out[4] = (double)nb;
    out[6] = (double)cus;
    out[7] = h->cfg.skin;
    if (!hist) return MD_OK;
    Buffers &b = h->b;
    if (!b.stat && (rc = dalloc(&b.stat, (size_t)(8 + kStatBins)))) return rc;
    if ((int64_t)g.ncell > b.stat_count_cap) {
        if (b.stat_count) (void)hipFree(b.stat_count);
        b.stat_count = nullptr;
        b.stat_count_cap = 0;
        if ((rc = dalloc(&b.stat_count, (size_t)g.ncell))) return rc;
        b.stat_count_cap = g.ncell;
    }
    launch_fill_i32(b.stat_count, 0, g.ncell, s);
    launch_bin_counts((int)h->n, pos, g, b.stat_count, s);
    launch_bin_summary(g.ncell, b.stat_count, b.stat, s);
    std::vector<int32_t> sm(8 + kStatBins);
    MD_HIP(hipMemcpyAsync(sm.data(), b.stat, sm.size() * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    MD_HIP(hipStreamSynchronize(s));
    int64_t sum, sumsq;
    memcpy(&sum, &sm[0], 8);
    memcpy(&sumsq, &sm[2], 8);
    double mean = (double)sum / (double)nb;
    // population variance from the integer sums (exact up to the final
    // divisions)
    double var = ((double)sumsq - (double)sum * (double)sum / (double)nb) / (double)nb;
    var = std::max(var, 0.0);
    // median: the middle order statistic(s), from the histogram of counts
    auto order_stat = [&](int64_t k, double &v) {  // k-th smallest (0-based); false past the histogram
        int64_t c = 0;
        for (int b = 0; b < kStatBins - 1; b++) {
            c += sm[8 + b];
            if (c > k) {
                v = (double)b;
                return true;
            }
        }
        return false;
    };
    double hi = 0.0, lo = 0.0;
    bool ok = order_stat(nb / 2, hi) && (nb % 2 == 1 || order_stat(nb / 2 - 1, lo));
    if (!ok) {
        // a middle bin holds kStatBins - 1 or more particles: select on the
        // host from the counts themselves
        std::vector<int32_t> cnt(g.ncell);
        MD_HIP(hipMemcpy(cnt.data(), b.stat_count, g.ncell * sizeof(int32_t), hipMemcpyDeviceToHost));
        std::nth_element(cnt.begin(), cnt.begin() + nb / 2, cnt.end());
        hi = (double)cnt[nb / 2];
        if (nb % 2 == 0) lo = (double)*std::max_element(cnt.begin(), cnt.begin() + nb / 2);
    }
    double med = nb % 2 ? hi : 0.5 * (lo + hi);
    out[0] = mean;
    out[1] = mean > 0.0 ? sqrt(var) / mean : 0.0;
    out[2] = med;
    out[3] = (double)sm[4];
    out[5] = (double)sm[5];
    return MD_OK;
}

extern "C" int md_live_stats(md_handle *h, const double *pos, double *out, void *stream)
{
    int rc = check_handle(h);
    if (rc) return rc;
    if (!out || (h->n > 0 && !pos)) return fail(MD_ERR_INVALID_ARG, "pos and out must not be NULL");
    return live_stats(h, pos, out, (hipStream_t)stream, true);
}

extern "C" int md_set_expert_rules(md_handle *h, const md_fuzzy_rule *rules, int32_t n_rules)
{
    int rc = check_handle(h);
    if (rc) return rc;
    if (!h->tuner) return fail(MD_ERR_INVALID_ARG, "the handle does not tune (autotune is MD_TUNE_OFF)");
    if (!rules || n_rules == 0) {
        set_builtin_rules(h);
        return MD_OK;
    }
    std::string why = check_rules(rules, n_rules, (int)h->space.size());
    if (!why.empty()) return fail(MD_ERR_INVALID_ARG, why);
    h->rules.assign(rules, rules + n_rules);
    return MD_OK;
}

__global__ void k_copy_rows(int n, const int32_t *__restrict__ nbr, const int32_t *__restrict__ cnt, int64_t ld,
                            int maxr, int32_t *__restrict__ counts, int32_t *__restrict__ rows)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int c = cnt[i];
    counts[i] = c;
    int m = c < maxr ? c : maxr;
    for (int k = 0; k < m; k++) rows[(size_t)i * maxr + k] = nbr[(size_t)k * ld + i];
}

extern "C" int md_get_neighbors(md_handle *h, int32_t *counts, int32_t *rows, int32_t max_per_row, void *stream)
{
    int rc = check_handle(h);
    if (rc) return rc;
    if (h->cfg.container == MD_CONTAINER_LC) return fail(MD_ERR_INVALID_ARG, "linked cells keep no lists");
    if (!h->built || !h->lists) return fail(MD_ERR_NOT_BUILT, "lists not built");
    if (max_per_row < 1 || (h->n > 0 && (!counts || !rows))) return fail(MD_ERR_INVALID_ARG, "bad arguments");
    int n = (int)h->n;
    if (h->cfg.container == MD_CONTAINER_VLC) {
        const Buffers &b = h->b;
        launch_vlc_rows(n, b.cell_start, b.cell_sorted, h->g, b.vlc_nbr, vlc_ld(h), b.vlc_seg, max_per_row, counts,
                        rows, (hipStream_t)stream);
    } else if (h->cfg.container == MD_CONTAINER_PVL) {
        const Buffers &b = h->b;
        launch_pvl_rows(n, b.cell_start, b.cell_sorted, h->g, b.pvl_perm, b.pvl_cnt, max_per_row, counts, rows,
                        (hipStream_t)stream);
    } else if (h->cfg.container == MD_CONTAINER_CL) {
        const Buffers &b = h->b;
        launch_cl_rows(n, b.cell_sorted, b.cell_start, b.cl_base, b.cl_start, b.cl_count, b.cl_nbr, b.cl_nbr_count,
                       b.cl_cap, max_per_row, counts, rows, (hipStream_t)stream);
    } else if (use_window(h)) {
        const Geom &g = h->g;
        launch_vlw_decode(h->b.cell_start, h->b.cell_sorted, g, n, h->b.w_rowb + window_nbands(g), h->b.w_blk,
                          h->b.w_nbr, h->b.nbr_count, max_per_row, counts, rows, h->cfg.newton3 == MD_N3L_ON,
                          (hipStream_t)stream);
    } else if (n > 0) {
        k_copy_rows<<<(n + kBlock - 1) / kBlock, kBlock, 0, (hipStream_t)stream>>>(
            n, h->b.nbr, h->b.nbr_count, h->n, max_per_row, counts, rows);
    }
    return MD_OK;
}

extern "C" int md_status(md_handle *h, uint32_t *flags)
{
    int rc = check_handle(h);
    if (rc) return rc;
    if (!flags) return fail(MD_ERR_INVALID_ARG, "flags is NULL");
    MD_HIP(hipDeviceSynchronize());
    uint32_t f = 0;
    MD_HIP(hipMemcpy(&f, h->b.flags, sizeof(uint32_t), hipMemcpyDeviceToHost));
    uint32_t zero = 0;
    MD_HIP(hipMemcpy(h->b.flags, &zero, sizeof(uint32_t), hipMemcpyHostToDevice));
    if (f & MD_FLAG_LIST_OVERFLOW) h->truncated = true;
    *flags = f | h->sticky;
    h->sticky = 0;
    return MD_OK;
}

extern "C" int md_get_config(md_handle *h, md_config *cfg)
{
    if (!h || !cfg) return fail(MD_ERR_INVALID_ARG, "NULL argument");
    *cfg = h->cfg;
    return MD_OK;
}

// Entries of the current neighbour lists: particle entries (Verlet lists)
// or cluster-pair entries (cluster lists); 0 for linked cells.  Waits for
// the device.
static int list_entries(md_handle *h, int64_t *entries)
{
    *entries = 0;
    const Buffers &b = h->b;
    if (!h->built || !h->lists || !has_lists(h->cfg)) return MD_OK;
    int32_t m = (int32_t)h->n;
    const int32_t *cnt = b.nbr_count;
    if (h->cfg.container == MD_CONTAINER_PVL) {
        // candidates: own cells and stored prefixes
        if (!h->b.pvl_entries) {
            int rc = dalloc(&h->b.pvl_entries, 1);
            if (rc) return rc;
        }
        unsigned long long e = 0;
        MD_HIP(hipDeviceSynchronize());
        MD_HIP(hipMemcpy(h->b.pvl_entries, &e, sizeof(e), hipMemcpyHostToDevice));
        launch_pvl_entries(m, b.cell_start, b.cell_sorted, b.pvl_cnt, h->b.pvl_entries, nullptr);
        MD_HIP(hipMemcpy(&e, h->b.pvl_entries, sizeof(e), hipMemcpyDeviceToHost));
        *entries = (int64_t)e;
        return MD_OK;
    }
    if (h->cfg.container == MD_CONTAINER_CL) {
        if (!b.cl_base || !b.cl_nbr_count) return MD_OK;
        MD_HIP(hipDeviceSynchronize());
        MD_HIP(hipMemcpy(&m, b.cl_base + h->g.ncell, sizeof(int32_t), hipMemcpyDeviceToHost));
        cnt = b.cl_nbr_count;
    }
    if (!cnt || m <= 0) return MD_OK;
    std::vector<int32_t> host((size_t)m);
    MD_HIP(hipDeviceSynchronize());
    MD_HIP(hipMemcpy(host.data(), cnt, sizeof(int32_t) * (size_t)m, hipMemcpyDeviceToHost));
    int64_t sum = 0;
    for (int32_t c : host) sum += c;
    *entries = sum;
    return MD_OK;
}

extern "C" int md_get_counters(md_handle *h, int64_t *out)
{
    if (!h || !out) return fail(MD_ERR_INVALID_ARG, "NULL argument");
    int rc = list_entries(h, &h->list_entries);
    if (rc) return rc;
    out[0] = h->rebuilds;
    out[1] = h->forced;
    out[2] = h->phases;
    out[3] = h->trials;
    out[4] = h->config_index;
    out[5] = h->list_entries;
    out[6] = h->cfg.container == MD_CONTAINER_CL ? 2 : use_window(h) ? 1 : 0;
    return MD_OK;
}

extern "C" int md_get_trial_scores(md_handle *h, double *scores, md_config *configs, int32_t n)
{
    if (!h) return fail(MD_ERR_INVALID_ARG, "NULL handle");
    int m = (int)h->space.size();
    if (m == 0) return fail(MD_ERR_INVALID_ARG, "the handle does not tune (autotune is MD_TUNE_OFF)");
    if (n < m || !scores) return fail(MD_ERR_INVALID_ARG, "scores needs room for " + std::to_string(m) + " entries");
    for (int k = 0; k < m; k++) {
        scores[k] = h->tuner->last_score(k);
        if (configs) configs[k] = h->space[k];
    }
    return m;
}

extern "C" int md_get_phase_choices(md_handle *h, int32_t *configs, int32_t n)
{
    if (!h) return fail(MD_ERR_INVALID_ARG, "NULL handle");
    if (n < 0 || (n > 0 && !configs)) return fail(MD_ERR_INVALID_ARG, "configs needs room for n entries");
    int m = (int)h->phase_choices.size();
    for (int k = 0; k < m && k < n; k++) configs[k] = h->phase_choices[k];
    return m;
}

extern "C" int md_timing(md_handle *h, int32_t enable, double *out)
{
    int rc = check_handle(h);
    if (rc) return rc;
    timing_collect(h);
    if (out)
        for (int k = 0; k < 4; k++) out[k] = h->tsum[k];
    if (enable && !h->timing)
        for (int k = 0; k < 4; k++) h->tsum[k] = 0.0;
    h->timing = enable != 0;
    return MD_OK;
}

extern "C" const char *md_last_error(void) { return g_err.c_str(); }

// ------------------------------------------------------------------ tuning

// Whether two configurations of the tuning space build the same structure.
static bool same_structure(const md_config &a, const md_config &b)
{
    return a.container == b.container && a.newton3 == b.newton3 && a.csf == b.csf && a.skin == b.skin &&
           a.layout == b.layout;
}

// Whether two configurations differ at most in the skin.
static bool same_method(const md_config &a, const md_config &b)
{
    return a.container == b.container && a.newton3 == b.newton3 && a.csf == b.csf && a.layout == b.layout;
}

// Switch the handle to configuration nc (same particles, box, cutoffs,
// precision); the structures are rebuilt at the next step.
int apply_config(md_handle *h, const md_config &nc)
{
    Geom g;
    int rc = make_geom(nc, nc.csf, g);
    if (rc) return rc;
    if ((rc = ensure_cells(h, g))) return rc;
    h->cfg = nc;
    h->g = g;
    h->built = false;
    h->age = INT32_MAX / 2;
    return MD_OK;
}

// One tuning phase (Sec. 2.2.5): trial the configurations the strategy asks
// for, each for tune_trial_steps steps starting with a rebuild, score each by
// its per-step time plus its build time spread over its rebuild interval
// (the weighted average of build and force time), keep the best.  The trial
// steps advance the simulation.  A phase whose trials (as many as the
// strategy asks for this phase) do not fit into the rest of this md_step call
// is postponed to the next call.
int run_tuning_phase(md_handle *h, const StepCtx &c, int s0, int *next)
{
    Tuner *t = h->tuner;
    int T = h->base.tune_trial_steps;
    int rc0;
    *next = s0;
    if ((int64_t)T > (int64_t)(c.nsteps - s0)) {  // not even one trial fits
        h->next_phase = h->steps_done + c.nsteps;
        return MD_OK;
    }
    if (h->base.autotune == MD_TUNE_EXPERT) {
        // Sec. 5.2: the rules read the live statistics of the current
        // positions (the histogram only if a rule needs more than counts)
        double st[8];
        if ((rc0 = live_stats(h, c.pos, st, c.s, rules_need_histogram(h->rules)))) return rc0;
        std::vector<double> suit;
        expert_suitability(h->rules.data(), (int)h->rules.size(), t->n(), st, suit);
        t->set_suitability(suit);
    }
    if (h->base.autotune == MD_TUNE_RF) {
        // Sec. 5.3: the forest reads all the live statistics of the current
        // positions and names the one configuration to run
        double st[8];
        if ((rc0 = live_stats(h, c.pos, st, c.s, true))) return rc0;
        // the forest's classes are configurations of the FP32 space without
        // skin variants: map each by its structure (at the base skin)
        md_config cb = h->base;
        cb.precision = MD_FP32;
        cb.tune_skin = 0;
        std::vector<md_config> canon;
        tuning_space(cb, canon);
        int pick = rf_predict_mapped(st, [&](int k) {
            if (k < 0 || k >= (int)canon.size()) return -1;
            for (int j = 0; j < (int)h->space.size(); j++)
                if (same_method(h->space[j], canon[k]) && h->space[j].skin == h->base.skin) return j;
            return -1;
        });
        std::vector<double> suit(t->n(), 0.0);
        if (pick >= 0) suit[pick] = 1.0;
        t->set_suitability(suit);
    }
    if ((h->base.autotune == MD_TUNE_EXPERT || h->base.autotune == MD_TUNE_RF) && h->base.tune_skin) {
        // the rules and the forest name structures; with the skin tuned, a
        // named structure's other skins are trialled beside it (the skin is a
        // parameter measured per phase, like the rebuild interval)
        std::vector<double> suit = t->suitability();
        std::vector<double> wide = suit;
        int m = (int)h->space.size();
        for (int a = 0; a < m && a < (int)suit.size(); a++)
            for (int b = 0; b < m && b < (int)suit.size(); b++)
                if (a != b && same_method(h->space[a], h->space[b])) wide[b] = std::max(wide[b], suit[a]);
        t->set_suitability(wide);
    }
    {
        std::vector<int> plan;
        int count = t->plan_phase(plan);
        if ((int64_t)count * T > (int64_t)(c.nsteps - s0)) {
            h->next_phase = h->steps_done + c.nsteps;
            return MD_OK;
        }
    }
    std::vector<int> trial;
    int ntrial = t->begin_phase(trial);
    h->phases++;
    int s = s0, last_k = -1, rc;
    for (int k = 0; k < (int)trial.size(); k++) {
        if (!trial[k]) continue;
        md_config kc = h->space[k];
        // a phase whose one trial is the configuration in use runs it on,
        // without the rebuild a switch needs
        bool keep = ntrial == 1 && same_structure(kc, h->cfg) && h->built &&
                    (h->lists || !has_lists(h->cfg));
        if (!keep && (rc = apply_config(h, kc))) return rc;
        // the interval follows from the motion and this configuration's skin
        kc.rebuild_interval = h->cfg.rebuild_interval = derived_interval(h);
        MD_HIP(hipEventRecord(h->ev0, c.s));
        if ((rc = run_steps(h, c, s, s + 1))) return rc;
        MD_HIP(hipEventRecord(h->ev1, c.s));
        int64_t rb1 = h->rebuilds;
        if ((rc = run_steps(h, c, s + 1, s + T))) return rc;
        MD_HIP(hipEventRecord(h->ev2, c.s));
        MD_HIP(hipEventSynchronize(h->ev2));
        int64_t nrb = h->rebuilds - rb1;  // scheduled and forced rebuilds after the first step
        float t01 = 0.f, t12 = 0.f;
        MD_HIP(hipEventElapsedTime(&t01, h->ev0, h->ev1));
        MD_HIP(hipEventElapsedTime(&t12, h->ev1, h->ev2));
        // first step = one step + one build; later steps = (T-1) steps + nrb
        // builds (replays inflate the per-step part): solve for both, then
        // charge builds at the rate this configuration needs them
        double score;
        if (T - 1 - nrb > 0) {
            double per = ((double)t12 - (double)nrb * t01) / (double)(T - 1 - nrb);
            per = std::max(per, 0.0);
            double build = std::max(0.0, (double)t01 - per);
            double rate = std::max(1.0 / kc.rebuild_interval, (double)nrb / (double)(T - 1));
            score = per + build * rate;
        } else {
            score = ((double)t01 + (double)t12) / (double)T;
        }
        t->report(k, score);
        h->trials++;
        last_k = k;
        s += T;
    }
    int chosen = t->end_phase();
    if (chosen < 0) return fail(MD_ERR_INVALID_ARG, "tuning phase without scores");
    if (chosen != last_k && (rc = apply_config(h, h->space[chosen]))) return rc;
    h->config_index = chosen;
    h->phase_choices.push_back(chosen);
    h->next_phase = h->steps_done + s0 + h->base.tune_interval;
    *next = s;
    return MD_OK;
}

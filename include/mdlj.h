/*
 * mdlj.h -- C-ABI of the MI355X (gfx950) short-range Lennard-Jones MD library.
 *
 * The library is a particle container in the sense of the paper (Sec. 2.2:
 * a black-box container for a cutoff-based particle simulator): it finds
 * interacting pairs (linked cells, Verlet lists with a skin, cluster-pair
 * lists), evaluates the cutoff Lennard-Jones 12-6 forces, advances the
 * Stormer-Verlet (velocity form) integrator, differentiates a force-matching
 * loss, and selects its own algorithmic configuration at run time (Sec. 2.2.5
 * tuning phases, Sec. 5.1 Predictive strategy).
 *
 * Conventions for every call:
 *   - All particle arrays are caller-owned DEVICE buffers on the handle's
 *     device, contiguous, SoA: pos is double[3][n] (x row, then y, then z),
 *     positions in [0, box[d]).  vel and force are real[3][n] where real is
 *     float for MD_FP32 and double for MD_FP64 (md_config.precision).
 *     type and ids are int32[n]; types lie in [0, n_types).
 *   - lj is a DEVICE array double[2 * n_types]: per-type epsilon
 *     (eps_0 .. eps_{nt-1}) then per-type sigma (sig_0 .. sig_{nt-1}).  Pair
 *     parameters follow Lorentz-Berthelot mixing: sig_ab = (sig_a + sig_b)/2,
 *     eps_ab = sqrt(eps_a eps_b).  The per-pair cutoffs are fixed in the
 *     config (rc2) and are not functions of lj.
 *   - stream is a hipStream_t passed as void*; NULL means the default stream.
 *     Every call only enqueues work on that stream and returns without
 *     waiting, unless its comment says it synchronises.
 *   - Every int-returning call returns MD_OK (0) or a negative MD_ERR_* code;
 *     md_last_error() then describes the failure.  Nothing throws across the
 *     ABI.  Invalid arguments are rejected before any work is enqueued.
 *   - A pair interacts iff r^2 < rc2[type_i][type_j] (strict), with r the
 *     periodic minimum-image distance (requires box >= 2 (r_c + skin)).
 */
#ifndef MDLJ_H
#define MDLJ_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MD_MAX_TYPES 2

/* return codes */
#define MD_OK 0
#define MD_ERR_INVALID_ARG (-1)
#define MD_ERR_BOX_TOO_SMALL (-2)
#define MD_ERR_LIST_OVERFLOW (-3)
#define MD_ERR_NONFINITE (-4)
#define MD_ERR_HIP (-5)
#define MD_ERR_NOT_BUILT (-6)
#define MD_ERR_NO_DEVICE (-7)

/* precision of the pair arithmetic and of vel/force storage */
#define MD_FP32 0
#define MD_FP64 1

/* containers (Sec. 2.2.1) */
#define MD_CONTAINER_LC 0 /* linked cells                                  */
#define MD_CONTAINER_VL 1 /* Verlet lists with skin, rebuilt every R steps  */
#define MD_CONTAINER_CL 2 /* cluster-pair lists (8-particle clusters; FP32,
                             gather-only)                                   */
#define MD_CONTAINER_PVL 3 /* pairwise Verlet lists (sorted cell pairs: per
                              neighbour cell a prefix of its order along the
                              pair's direction; FP32, gather-only, CSF 1,
                              at least three cells per dimension)          */
#define MD_CONTAINER_VLC 4 /* Verlet list cells: each pair once, in a list
                              owned by a cell, traversed with the C08 cell
                              colouring (Newton's third law without
                              atomics; FP32, newton3 = MD_N3L_ON, CSF 1, at
                              least three cells per dimension)             */

/* traversal (Sec. 2.2.2, Table 1: N3L column) */
#define MD_N3L_OFF 0 /* each pair evaluated from both sides, gather only  */
#define MD_N3L_ON 1  /* each pair once, j-side scattered with atomics     */
#define MD_N3L_C08 2 /* each pair once through the C08 colouring of cubes
                        of cells (Table 1's C08): linked cells only, FP32,
                        CSF 1, at least three cells per dimension; both
                        sides summed in the workgroup, no atomics on the
                        forces                                             */

/* data layout (Sec. 2.2.3) of the staged positions in the LDS windows of
 * the FP32 Verlet-list force (gather-only, one particle type): the list
 * entries address the window by byte offset */
#define MD_LAYOUT_PACKED 0  /* 12-byte entries (x, y, z)                      */
#define MD_LAYOUT_ALIGNED 1 /* 16-byte entries, one 16-byte LDS read each     */
#define MD_LAYOUT_SOA 2     /* one plane per coordinate, three 4-byte reads   */

/* autotuning strategy (Sec. 2.2.5 Full Search, Sec. 5.1 Predictive) */
#define MD_TUNE_OFF 0
#define MD_TUNE_FULL 1
#define MD_TUNE_PREDICTIVE 2
#define MD_TUNE_EXPERT 3 /* Sec. 5.2: fuzzy rules over the live statistics  */
#define MD_TUNE_RF 4     /* Sec. 5.3: a random forest over the statistics   */

/* consequents of the Expert strategy's fuzzy rules: terms of the output
 * variable "suitability" on [0, 1] (triangles peaking at 0, 0.5 and 1) */
#define MD_SUIT_BAD 0
#define MD_SUIT_OKAY 1
#define MD_SUIT_GOOD 2

/* md_status flag bits */
#define MD_FLAG_LIST_OVERFLOW 1u  /* a neighbour row exceeded max_neighbors   */
#define MD_FLAG_SKIN_EXCEEDED 2u  /* a particle moved >= skin/2 since a build */
#define MD_FLAG_NONFINITE 4u      /* a non-finite force or position appeared  */
#define MD_FLAG_WINDOW_FALLBACK 8u /* a cell neighbourhood held more particles
                                      than an LDS window tile: the handle
                                      switched to the global (non-windowed)
                                      kernels, with the same results        */

typedef struct md_handle md_handle;

typedef struct md_config {
    int64_t n;             /* number of particles, >= 0                        */
    int32_t n_types;       /* 1 .. MD_MAX_TYPES                                */
    int32_t precision;     /* MD_FP32 (default) or MD_FP64                     */
    double box[3];         /* periodic box lengths                             */
    double rc2[MD_MAX_TYPES * MD_MAX_TYPES]; /* squared cutoff per type pair,
                              row-major [a][b], symmetric; only the first
                              n_types x n_types block (row stride n_types) is
                              read                                             */
    double skin;           /* Verlet skin >= 0                                 */
    double csf;            /* cell size factor in (0, 1]: cell side >=
                              csf (r_c,max + skin), stretched to fit the box  */
    int32_t container;     /* MD_CONTAINER_*                                   */
    int32_t newton3;       /* MD_N3L_OFF / MD_N3L_ON / MD_N3L_C08              */
    int32_t rebuild_interval; /* R >= 1: rebuild cells and lists every R steps */
    int32_t max_neighbors; /* list row capacity: particles per Verlet row, or
                              j-clusters per i-cluster for cluster lists;
                              grown by md_step when a build overflows it      */
    int32_t autotune;      /* MD_TUNE_*; on: md_step selects the configuration */
    int32_t tune_interval; /* steps between tuning phases                      */
    int32_t tune_trial_steps; /* steps each trialled configuration runs        */
    int32_t total_steps_hint; /* expected steps of the run (retrial gap)       */
    int32_t tune_skin;     /* 1: the tuning space also holds Verlet lists
                              (gather-only, CSF 1) at 2/3, 4/3 and 5/3 of the
                              skin, each with its rebuild interval derived
                              from the motion (a joint skin / R search);
                              under MD_TUNE_EXPERT and MD_TUNE_RF a named
                              structure is trialled at every skin the space
                              holds for it; 0 (default): the skin stays
                              fixed                                         */
    int32_t tune_first;    /* steps (counted over the handle's md_step calls)
                              before the first tuning phase, >= 0; 0: the
                              first step.  Later phases follow every
                              tune_interval steps                           */
    int32_t layout;        /* MD_LAYOUT_*: MD_LAYOUT_PACKED (default), or for
                              FP32 Verlet lists, gather-only, one type,
                              MD_LAYOUT_ALIGNED or MD_LAYOUT_SOA            */
} md_config;

/* Fill *cfg with defaults for n particles in a cubic box of side L:
 * one type, r_c = 2.5, skin 0.3, CSF 1, Verlet lists, gather-only, R = 10,
 * FP32, no tuning.  Returns MD_OK or MD_ERR_INVALID_ARG (cfg NULL). */
int md_config_default(md_config *cfg, int64_t n, double L);

/* Create a handle on the current HIP device: validates cfg and allocates all
 * internal buffers (cells, lists, staging, reduction scratch).  *out is set
 * to NULL on failure.  Errors: MD_ERR_INVALID_ARG, MD_ERR_BOX_TOO_SMALL
 * (box[d] < 2 (r_c,max + skin)), MD_ERR_NO_DEVICE, MD_ERR_HIP. */
int md_create(const md_config *cfg, md_handle **out);

/* Release the handle and its device memory (synchronises its device). */
void md_destroy(md_handle *h);

/* Linked cells (Sec. 2.2.1): bin the particles into cells of side
 * >= csf (r_c,max + skin) stretched to fit the box, by a counting sort, and
 * reorder pos, vel, force, type and ids IN PLACE into cell order (cells in
 * x-fastest linear order; within a cell by ascending ids, or for cluster
 * lists by the 6-bit Morton code of the position inside the cell, then id).  ids carries each
 * particle's caller-defined identity through every reordering.  vel and force
 * may be NULL (then they are not permuted).  Also stages the positions for
 * the pair kernels and records them as the reference for the skin check.
 * Positions belong in [0, box[d]); one more than a cell outside the box, or
 * a non-finite one, is binned into an edge cell and sets MD_FLAG_NONFINITE
 * (this call does not wait to see it; md_step does).  Where the FP32
 * configuration runs over LDS cell windows, this call synchronises the stream
 * once to read the window packer's verdict: if some cell neighbourhood holds
 * more particles than a window tile (densities far above a liquid's), the
 * handle switches to the global kernels for good and md_status reports
 * MD_FLAG_WINDOW_FALLBACK; results are unchanged. */
int md_build_cells(md_handle *h, double *pos, void *vel, void *force,
                   int32_t *type, int32_t *ids, void *stream);

/* Verlet lists / cluster-pair lists (Sec. 2.2.1): for the current container,
 * build the candidate structure from the cells: every pair with
 * r^2 < (r_c,max + skin)^2 at the current positions (decided in FP64).  No-op
 * for linked cells.  pos and type must be in the order md_build_cells left.
 * Overflow of max_neighbors sets MD_FLAG_LIST_OVERFLOW (see md_status). */
int md_build_neighbors(md_handle *h, const double *pos, const int32_t *type,
                       void *stream);

/* Forces (Sec. 2.1): force[i] = sum_j f_ij over pairs within the cutoff,
 * f_ij = 24 eps q (2q - 1) / r^2 * d_ij, q = (sig^2/r^2)^3, with the current
 * container.  pos/type in cell order; force written in the same order.
 * If out (DEVICE double[4]) is not NULL it receives
 * { U = sum_{i<j} 4 eps q (q - 1), W = sum_{i<j} r . f, n_pairs, 0 }.
 * MD_ERR_NOT_BUILT if no md_build_cells came first, or (Verlet and cluster
 * lists) no md_build_neighbors after the last md_build_cells. */
int md_compute_forces(md_handle *h, const double *pos, const int32_t *type,
                      const double *lj, void *force, double *out, void *stream);

/* nsteps of velocity Verlet (Stormer-Verlet, Sec. 2.1):
 *   v += dt/2 F/m; x += dt v (wrapped into the box); F = F(x); v += dt/2 F/m
 * with cells/lists rebuilt every R steps (and whenever a particle has moved
 * >= skin/2 since the last build: the affected steps are recomputed).  With
 * autotune on, tuning phases trial configurations and keep the fastest.
 * force must hold F(pos) on entry (call md_compute_forces first).  The arrays
 * stay in cell order, reordered in place at each rebuild.  inv_mass is a
 * DEVICE double[n_types].  If energy_every > 0 and log is not NULL (DEVICE
 * double[nsteps / energy_every][4]), after every energy_every-th step it
 * receives { U, K = 1/2 sum m v^2, W, n_pairs }.  Synchronises the stream
 * once per rebuild interval (to read the skin check).  MD_ERR_NONFINITE when
 * MD_FLAG_NONFINITE is set (by this call or an earlier one, until md_status
 * clears it).  A rebuild whose cell neighbourhoods outgrow the LDS tile of
 * the windowed kernels switches the handle to the global kernels and redoes
 * the affected steps (MD_FLAG_WINDOW_FALLBACK). */
int md_step(md_handle *h, double *pos, void *vel, void *force, int32_t *type,
            int32_t *ids, const double *inv_mass, const double *lj, double dt,
            int32_t nsteps, int32_t energy_every, double *log, void *stream);

/* Adjoint of md_compute_forces: given grad_force = dL/dF (real[3][n], cell
 * order), writes grad_pos = dL/dx (DEVICE double[3][n]) and grad_lj = dL/dlj
 * (DEVICE double[2 n_types], same layout as lj), the exact derivatives of the
 * truncated forces at fixed cutoffs:
 *   per pair, J = phi I + 2 (dphi/dr2) d d^T acts on (g_i - g_j);
 *   dphi/deps_ab = phi/eps_ab, dphi/dsig_ab = 144 eps q (4q - 1)/(sig r^2),
 * chained through the mixing rule.  Uses the current container's pairs. */
int md_forces_backward(md_handle *h, const double *pos, const int32_t *type,
                       const double *lj, const void *grad_force,
                       double *grad_pos, double *grad_lj, void *stream);

/* Live simulation statistics (Sec. 4) over bins that mimic a CSF-1 cell
 * (side >= r_c,max + skin) of the given positions: out (HOST double[8]) =
 * { mean, std/mean, median, max particles per bin, n_bins, n_empty_bins,
 *   n_compute_units, skin }.  Synchronises the stream. */
int md_live_stats(md_handle *h, const double *pos, double *out, void *stream);

/* Copy the current lists out (Verlet or cluster-pair lists): counts (DEVICE
 * int32[n]) gets each particle's number of entries, rows (DEVICE
 * int32[n][max_per_row], row-major) its entries, both in the cell order the
 * arrays are in.  For cluster lists a particle's entries are all particles of
 * the j-clusters listed for its cluster, itself excluded: a superset of its
 * partners within r_c + skin.  For pairwise Verlet lists a particle's entries
 * are its candidates: the other particles of its cell and, per neighbour
 * cell, the stored prefix of that cell's order along the pair's direction
 * (also a superset of its partners within r_c + skin).  Rows longer than
 * max_per_row are truncated
 * (counts still give the full length).  MD_ERR_INVALID_ARG for linked cells.
 * For inspection and tests. */
int md_get_neighbors(md_handle *h, int32_t *counts, int32_t *rows,
                     int32_t max_per_row, void *stream);

/* Sticky device-side condition flags (MD_FLAG_* bits) accumulated since the
 * last call, then cleared.  Synchronises the handle's work. */
int md_status(md_handle *h, uint32_t *flags);

/* The tuning-space index each tuning phase chose, in phase order (Sec.
 * 2.2.5: the selection of every phase): writes the first min(n, phases)
 * into configs (HOST int32[n]; NULL with n = 0 to ask for the count) and
 * returns the number of phases so far, or an error. */
int md_get_phase_choices(md_handle *h, int32_t *configs, int32_t n);

/* Configuration the handle currently uses (after tuning decisions). */
int md_get_config(md_handle *h, md_config *cfg);

/* Counters since md_create: out (HOST int64[7]) = { rebuilds,
 * forced_rebuilds (skin exceeded), tuning_phases, trials, current config
 * index in the tuning space, entries of the current neighbour lists
 * (particle entries of Verlet lists, cluster-pair entries of cluster lists,
 * 0 for linked cells; reading them waits for the device), force-kernel family of the current configuration (0 one cell row per
 * thread, 1 LDS cell windows, 2 cluster pairs; valid after the first
 * step) }. */
int md_get_counters(md_handle *h, int64_t *out);

/* Kernel-class timing of md_step with HIP events recorded on the caller's
 * stream around every force pass and every rebuild (the build and force
 * times the tuning phases weigh, Sec. 2.2.5).  enable = 1 resets the totals
 * and starts recording, 0 stops.  If out (HOST double[4]) is not NULL it
 * receives { force_ms, force_passes, build_ms, builds } accumulated so far
 * (this waits for the recorded events). */
int md_timing(md_handle *h, int32_t enable, double *out);

/* Thread-local description of the last failing call ("" if none). */
const char *md_last_error(void);

/* ---------------------------------------------------------------------- */
/* Batched systems: n_sys independent periodic systems advanced together
 * (one launch per phase for all systems).  Particles of system s occupy
 * [offsets[s], offsets[s+1]) of every particle array, and offsets (HOST
 * int64[n_sys + 1]) is non-decreasing from 0.  boxes is HOST double[3 n_sys].
 * The per-pair cutoffs, skin, csf and precision come from cfg (cfg->n and
 * cfg->box are ignored).  cfg->container is MD_CONTAINER_LC (FP32 or FP64)
 * or MD_CONTAINER_VL (FP32, every system at most 65536 particles), newton3
 * MD_N3L_OFF; anything else is MD_ERR_INVALID_ARG.  The Verlet lists are
 * built with the cells (Sec. 2.2.1: every pair within r_c + skin), with room
 * per particle for max(max_neighbors, min(1024, 1.3 times the mean count
 * within the list radius of the densest system + 8)) entries, rounded up to
 * a multiple of 8; a particle with more walks its cell stencil instead (same
 * forces, more time). */
typedef struct md_batch md_batch;

int md_batch_create(const md_config *cfg, int32_t n_sys, const int64_t *offsets,
                    const double *boxes, md_batch **out);
void md_batch_destroy(md_batch *b);

/* Bin every system into its own cells and reorder the arrays in place (cell
 * order within each system's range; systems keep their ranges); with Verlet
 * lists, build them. */
int md_batch_build_cells(md_batch *b, double *pos, void *vel, void *force,
                         int32_t *type, int32_t *ids, void *stream);

/* Forces of every system; out (DEVICE double[4 n_sys] or NULL) receives each
 * system's { U, W, n_pairs, 0 }. */
int md_batch_compute_forces(md_batch *b, const double *pos, const int32_t *type,
                            const double *lj, void *force, double *out,
                            void *stream);

/* nsteps of velocity Verlet for every system.  The cells are rebuilt every R
 * steps, R at most cfg->rebuild_interval: a step at which a particle of any
 * system has moved more than half the skin since the last rebuild is redone
 * after a rebuild, and R is then shortened to the steps that passed; after a
 * run of blocks without such a step (32, doubling after each failed try) a
 * block one step longer is tried.  The trajectory does not depend on R.
 * use_graph != 0 captures one rebuild interval into a HIP graph and replays
 * it; 0 launches every kernel directly. */
int md_batch_step(md_batch *b, double *pos, void *vel, void *force,
                  int32_t *type, int32_t *ids, const double *inv_mass,
                  const double *lj, double dt, int32_t nsteps,
                  int32_t use_graph, void *stream);

/* Counters of md_batch_step since md_batch_create: out (HOST int64[4]) =
 * { rebuilds (one per block of steps), forced_rebuilds (blocks cut short by
 * a particle that moved more than half the skin), steps, the rebuild
 * interval the next block uses }.  MD_ERR_INVALID_ARG if b or out is NULL. */
int md_batch_get_counters(const md_batch *b, int64_t *out);

/* ---------------------------------------------------------------------- */
/* Scores of the autotuner's trials: scores (HOST double[n]) gets, per
 * configuration of the tuning space, its last measured score (ms per step:
 * per-step time plus build time spread over its rebuild interval) or NaN if
 * it was never trialled; configs (HOST md_config[n], may be NULL) gets the
 * configurations themselves.  Returns the size of the tuning space (n must be
 * at least that), or MD_ERR_INVALID_ARG when the handle does not tune.  The
 * data from which Expert rules are written (Sec. 5.2). */
int md_get_trial_scores(md_handle *h, double *scores, md_config *configs,
                        int32_t n);

/* Expert strategy (Sec. 5.2, with the fuzzy logic of Sec. 2.3): a rule
 *   IF stats[input[0]] IS trap[0] (AND stats[input[1]] IS trap[1])
 *   THEN suitability(config) IS then
 * where stats are the live statistics in md_live_stats order and trap[k] =
 * (a, b, c, d) is a trapezoid membership function: 0 outside (a, d), rising
 * linearly on [a, b], 1 on [b, c], falling on [c, d]; a = b = -INFINITY or
 * c = d = INFINITY make shoulders.  input[1] = -1: one antecedent.  config
 * indexes the tuning space (md_get_trial_scores lists it).  Evaluation:
 * firing strength = min over the antecedents; each rule clips its output
 * term at its strength; a configuration's clipped terms are joined by max;
 * the crisp suitability is the centre of gravity of that set over [0, 1],
 * or 0 if none of its rules fires.  A tuning phase trials every
 * configuration whose suitability is within 0.1 of the largest (all of them
 * if no rule fires at all). */
typedef struct md_fuzzy_rule {
    int32_t input[2];
    double trap[2][4];
    int32_t config;
    int32_t then; /* MD_SUIT_* */
} md_fuzzy_rule;

/* Rules the Expert strategy of this handle uses (copied).  rules NULL or
 * n_rules 0 restores the built-in rules, which were written from Full Search
 * scores measured on MI355X and use the mean particles per bin only.
 * MD_ERR_INVALID_ARG for an input outside 0..7, a config outside the tuning
 * space, an unknown term or a trapezoid with a > b, b > c, c > d or NaN. */
int md_set_expert_rules(md_handle *h, const md_fuzzy_rule *rules,
                        int32_t n_rules);

/* Host only: the crisp suitability (HOST double[n_configs]) of each
 * configuration under rules (NULL: those built-in rules that name
 * configurations below n_configs) for the live statistics stats (HOST
 * double[8]).  Same validation as md_set_expert_rules. */
int md_expert_suitability(const md_fuzzy_rule *rules, int32_t n_rules,
                          int32_t n_configs, const double *stats,
                          double *suitability);

/* Random Forest strategy (Sec. 5.3), host only: the tuning-space index of
 * the configuration the built-in forest (100 trees fitted offline to Full
 * Search trials on MI355X over generative scenarios) predicts for the live
 * statistics stats (HOST double[8], md_live_stats order): the class with the
 * largest mean leaf fraction over the trees, features compared in single
 * precision, ties to the first class, among the classes below n_configs.
 * A tuning phase under MD_TUNE_RF trials that configuration alone (with
 * tune_skin, at every skin the space holds for it); the handle maps the
 * class to its own space by structure (container, CSF, N3L).
 * MD_ERR_INVALID_ARG for a NaN statistic or if no class fits n_configs. */
int md_rf_predict(const double *stats, int32_t n_configs);

/* Allocation-free forces, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Needs no handle: computes what md_compute_forces computes
 * with linked cells, gather-only (cfg->container and cfg->newton3 are not
 * read), in cfg->precision, for the cfg->n particles of pos (DEVICE
 * double[3][n]) and type (DEVICE int32[n]) in the caller's order, which is
 * left unchanged; force (DEVICE real[3][n]) is written in the same order,
 * out (DEVICE double[4] or NULL) gets { U, W, n_pairs, 0 }.  Every
 * intermediate array (cells, the cell-order copy, staging, partial sums)
 * lives in a fixed device scratch of MD_NOALLOC_SCRATCH_MIB MiB that each
 * GPU holds from this call's first use on it until the process ends; the
 * call allocates nothing.  Limits: n <= MD_NOALLOC_MAX_N, and cells plus
 * particles must fit the scratch (MD_ERR_INVALID_ARG otherwise, before any
 * work is enqueued).  Calls on one GPU share its scratch: calls that overlap
 * in time on one GPU (other streams, other host threads) race and give
 * undefined results; calls ordered on one stream are safe.  Positions must
 * lie in the box (a non-finite one gives undefined forces; nothing faults).
 * Enqueues on stream and returns. */
#define MD_NOALLOC_MAX_N 131072
#define MD_NOALLOC_SCRATCH_MIB 16
int md_compute_forces_noalloc(const md_config *cfg, const double *pos,
                              const int32_t *type, const double *lj,
                              void *force, double *out, void *stream);
/* MD_NOALLOC_MAX_N, as the library was built. */
int64_t md_noalloc_max_particles(void);

/* Configuration-selection engine, usable on its own with externally measured
 * scores (host only; needs no GPU).  Sec. 2.2.5 Full Search and Sec. 5.1
 * Predictive: trial all in the first two phases; predict each configuration
 * by the line through its last two (phase, score) points (clamped below at
 * half its last score); trial those predicted within rel_threshold of the
 * best prediction (inclusive) or not trialled for ceil(total_phases/4)
 * phases; blacklist those measured above blacklist_factor x the phase's best;
 * choose the lowest score (ties: lower index).  Sec. 5.2 Expert (and Sec.
 * 5.3 Random Forest, with a suitability of 1 for the predicted configuration
 * and 0 elsewhere): trial the configurations whose suitability
 * (md_tuner_set_suitability, before each phase) is within 0.1 of the
 * largest; no blacklist. */
typedef struct md_tuner md_tuner;

int md_tuner_create(int32_t strategy, int32_t n_configs, int32_t total_phases,
                    double rel_threshold, double blacklist_factor,
                    md_tuner **out);
void md_tuner_destroy(md_tuner *t);
/* Start the next phase; trial[n_configs] (HOST) gets 1 for configurations to
 * trial, 0 otherwise.  Returns the number to trial (>= 0) or an error. */
int md_tuner_begin_phase(md_tuner *t, int32_t *trial);
/* Expert strategy: the suitability (HOST double[n_configs], each in [0, 1])
 * the next begin_phase selects by; all 0 (the default) trials everything. */
int md_tuner_set_suitability(md_tuner *t, const double *suitability);
/* Report the measured score (lower is better) of a trialled configuration. */
int md_tuner_report(md_tuner *t, int32_t config, double score);
/* Finish the phase: returns the chosen configuration index (>= 0) or an
 * error if a trialled configuration has no score. */
int md_tuner_end_phase(md_tuner *t);
/* blacklisted[n_configs] (HOST) gets 1 for blacklisted configurations. */
int md_tuner_blacklist(md_tuner *t, int32_t *blacklisted);

#ifdef __cplusplus
}
#endif

#endif /* MDLJ_H */

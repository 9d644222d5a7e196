// Internal declarations shared by the HIP translation units of libmdlj.
// Nothing here is part of the C-ABI (include/mdlj.h is).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "mdlj.h"

namespace mdlj {

// Guard band of the FP32 cutoff decisions: a squared distance within
// rc2 * (1 +- 2^-19) of a cutoff is decided again in FP64 from the master
// positions, exactly as the plain definition does, so that every pair set
// equals the FP64 one.  The FP32 squared distance from the fixed-point
// coordinates is within ~7e-7 relative of the FP64 one (fixed-point
// quantisation <= 2 units per component, int->float rounding, three
// products and two sums), well inside 2^-19 = 1.9e-6.
constexpr double kBand = 1.0 / 524288.0;

constexpr int kMaxOfs = 5;  // neighbour cell offsets per dimension (reach <= 2)
constexpr int kWinBlkRows = 4;  // maximum y-rows of a block of the windowed traversals

// Per-type-pair constants, computed on the device from the per-type
// parameters (Lorentz-Berthelot) so that parameters may live in device memory
// and change between calls without a host round trip.
struct PairTab {
    // FP32 path, in fixed-point length units u = L_x / 2^32
    float rc2_lo[4], rc2_hi[4];  // guard band around rc2 / u^2
    float sig2[4];               // sig_ab^2 / u^2
    float eps24[4];              // 24 eps_ab / u   (force per unit d)
    float eps4[4];               // 4 eps_ab        (pair energy)
    float eps24w[4];             // 24 eps_ab       (pair virial)
    // FP64 path, physical units
    double rc2[4], sig[4], eps[4];
};

// Cell geometry and fixed-point staging constants (passed by value).
struct Geom {
    int nc[3];        // cells per dimension
    int ncell;        // nc[0] nc[1] nc[2]
    int nofs[3];      // distinct neighbour offsets per dimension
    int ofs[3][kMaxOfs];  // the offsets, as non-negative shifts mod nc[d]
    double L[3];      // box
    double inv_w[3];  // nc[d] / L[d]
    double S[3];      // fixed-point scale 2^32 / L[d]
    float ry, rz;     // L_y / L_x, L_z / L_x (anisotropic scale of y, z units)
    int iso;          // 1 if all box lengths are equal
    double rl2;       // (r_c,max + skin)^2, FP64
    float rl2_lo, rl2_hi;  // guard band of rl2 in u^2
    float disp2;      // (skin/2)^2 (1 - 1e-4) in u^2: skin check threshold
    int nt;           // number of types
    int reach[3];     // stencil reach in cells per dimension
    int wband;        // y-rows per block of the windowed traversals
    int layout;       // LDS layout of the Verlet-list force windows (MD_LAYOUT_*)
};

// Device buffers and state of one handle.
// Bins of the count histogram in the live-statistics summary.
constexpr int kStatBins = 1024;

struct Buffers {
    int32_t *cell_id = nullptr, *slot = nullptr, *perm = nullptr, *perm2 = nullptr;
    int32_t *cell_count = nullptr, *cell_start = nullptr, *cell_sorted = nullptr;
    int32_t *scan_blocks = nullptr;
    double *tmp_pos = nullptr;
    void *tmp_vel = nullptr, *tmp_force = nullptr;
    int32_t *tmp_type = nullptr, *tmp_ids = nullptr;
    int4 *stage = nullptr, *stage_ref = nullptr;
    int32_t *nbr = nullptr, *nbr_count = nullptr;
    int64_t nbr_cap = 0;  // entries per row allocated
    double *partials = nullptr;  // [kMaxPartials][4]
    double *kpart = nullptr;     // [kMaxPartials]
    float *dpart = nullptr;      // [kMaxPartials] per-block displacement maxima
    int32_t *flags = nullptr;    // device [4]: sticky bits, first skin step, spare
    PairTab *tab = nullptr;
    // clusters
    int32_t *cl_start = nullptr, *cl_count = nullptr, *cl_cell = nullptr;  // per cluster
    int4 *cl_centre = nullptr;
    float4 *cl_half = nullptr;
    int32_t *cl_base = nullptr;  // first cluster of each cell; cl_base[ncell] = clusters
    int64_t cl_base_cap = 0;
    uint64_t *cl_key = nullptr;  // in-cell ordering keys
    int32_t *cl_nbr = nullptr, *cl_nbr_count = nullptr;
    int64_t cl_cap = 0, cl_list_cap = 0;
    int32_t n_clusters_max = 0;
    // rollback snapshot (md_step)
    // second position and stage buffers of the fused integrator (the force
    // pass of one step writes the next step's positions beside the current)
    double *pos_alt = nullptr;
    int4 *stage_alt = nullptr;
    double *snap_pos = nullptr;
    void *snap_vel = nullptr, *snap_force = nullptr;
    int32_t *snap_type = nullptr, *snap_ids = nullptr;
    int4 *snap_stage = nullptr;
    // Verlet lists over LDS windows (FP32 gather-only)
    int4 *w_blk = nullptr;  // per block: first cell, last cell, particle range (or -1, -1)
    int4 *w_staged = nullptr;  // the packer's per-band staging of blocks
    int64_t w_staged_cap = 0;
    int32_t *w_rown = nullptr, *w_rowb = nullptr;
    uint16_t *w_nbr = nullptr;
    int64_t w_cap = 0, w_rows_cap = 0, w_nbr_cap = 0;
    // adjoint
    double *gpart = nullptr;     // per-block parameter-gradient partials [blocks][8]
    // pairwise Verlet lists: per direction (13) the sorted in-cell order and
    // projections, per neighbour slot (26) each particle's prefix length
    uint16_t *pvl_perm = nullptr, *pvl_cnt = nullptr;
    float *pvl_s = nullptr;
    int64_t pvl_cap = 0;
    unsigned long long *pvl_entries = nullptr;
    // Verlet list cells: entries [max][n], segment ends [4][n], per-cube partials
    uint16_t *vlc_nbr = nullptr, *vlc_seg = nullptr;  // entries [n][ld] (ld: capacity rounded to 8), ends [4][n]
    double *vlc_part = nullptr;
    int64_t vlc_cap = 0, vlc_part_cap = 0;
    int32_t vlc_maxn = 0;
    int32_t *stat = nullptr;     // live-statistics summary of the bin counts [8 + kStatBins]
    int32_t *stat_count = nullptr;  // live-statistics bin counts (their own array: the
    int64_t stat_count_cap = 0;     // structure's cells stay valid)
    uint32_t *host_flags = nullptr;  // pinned
};

constexpr int kBlock = 256;
constexpr int kMaxPartials = 65536;  // per-block reduction slots

// Set the thread-local error string; returns code.
int fail(int code, const std::string &msg);
int hip_fail(hipError_t e, const char *what);

#define MD_HIP(call)                                              \
    do {                                                          \
        hipError_t e_ = (call);                                   \
        if (e_ != hipSuccess) return ::mdlj::hip_fail(e_, #call); \
    } while (0)

// ------------------------------------------------------------------ launchers
// cells.hip
void launch_fill_i32(int32_t *p, int32_t v, int64_t n, hipStream_t s);
void launch_cell_hist(int n, const double *pos, const Geom &g, int32_t *cell_id, int32_t *slot,
                      int32_t *count, int32_t *flags, hipStream_t s);
int64_t scan_scratch_size(int64_t n);
void launch_scan(const int32_t *in, int32_t *out, int64_t n, int32_t *scratch, hipStream_t s);
void launch_scatter(int n, const int32_t *cell_id, const int32_t *slot, const int32_t *start,
                    int32_t *perm, hipStream_t s);
void launch_scatter_sort(int n, const int32_t *cell_id, const int32_t *slot, const int32_t *start,
                         const int32_t *ids, int32_t *perm, int32_t *key, int32_t *cell_of_slot, int32_t *perm_out,
                         hipStream_t s);
void launch_cell_sort(int n, const int32_t *start, const int32_t *ids, const int32_t *cell_id, const int32_t *perm,
                      int32_t *key, int32_t *cell_of_slot, int32_t *perm_out, hipStream_t s);
void launch_scatter_sort_x(int n, const int32_t *cell_id, const int32_t *slot, const int32_t *start,
                           const int32_t *ids, const double *pos, const Geom &g, int32_t *perm, uint64_t *key,
                           int32_t *cell_of_slot, int32_t *perm_out, hipStream_t s);
void launch_gather(int n, int precision, const int32_t *perm, const double *pos, const void *vel,
                   const void *force, const int32_t *type, const int32_t *ids, double *tpos,
                   void *tvel, void *tforce, int32_t *ttype, int32_t *tids, const int32_t *cell_id,
                   int32_t *cell_sorted, const Geom &g, int4 *stage, int4 *stage_ref,
                   hipStream_t s);
void launch_stage(int n, const double *pos, const int32_t *type, const Geom &g, int4 *stage,
                  hipStream_t s);
void launch_prepare_tab(const double *lj, const double *rc2_host, const Geom &g, PairTab *tab,
                        hipStream_t s);
void launch_bin_counts(int n, const double *pos, const Geom &g, int32_t *count, hipStream_t s);
void launch_bin_summary(int nb, const int32_t *count, int32_t *out, hipStream_t s);

// force.hip
struct IntegrateArgs {
    int n;
    int precision;
    double *pos;
    void *vel;
    const void *force;
    const int32_t *type;
    const double *inv_mass;
    double hdt, dt;
    int kick_prev;  // complete the previous step: v += dt/2 F/m (and kinetic energy)
    int start;      // start a step: v += dt/2 F/m; x += dt v; wrap; stage; skin check
    int energy;
    int step_index;
    int4 *stage;
    const int4 *stage_ref;
    int32_t *flags;
    double *kpart;
    float *dpart;  // if not null: per-block largest squared displacement since the build
};

struct ForceArgs {
    int n;
    int precision;
    int container;
    int newton3;
    bool energy;
    const double *pos;
    const int32_t *type;
    const int4 *stage;
    const int32_t *cell_start, *cell_sorted;
    const int32_t *nbr, *nbr_count;
    int64_t nbr_ld;
    const int32_t *cl_start, *cl_count, *cl_nbr, *cl_nbr_count;
    int64_t cl_ld;
    int n_clusters;
    const int32_t *cl_ncl;  // device: number of clusters
    const uint16_t *pvl_perm, *pvl_cnt;  // pairwise Verlet lists: sorted orders, prefix lengths
    const uint16_t *vlc_nbr, *vlc_seg;   // Verlet list cells: entries, segment ends per role
    int vlc_ld;                          // Verlet list cells: entries per particle row (a multiple of 8)
    double *vlc_part;                    // Verlet list cells: per-cube energy partials
    int vlc_blocks;                      // Verlet list cells: partial slots written with energies
    const PairTab *tab;
    void *force;
    double *partials;  // per-block {U, W, n_pairs, 0}
    int32_t *flags;
    // window lists
    bool window;
    const int32_t *w_nblk;
    const int4 *w_blk;
    const uint16_t *w_nbr;
    // the Verlet-list gather kernel may also advance each particle right
    // after its force (second half kick of this step, first half kick and
    // drift of the next): positions and stage then go to pos_out, stage_out
    bool fused;
    IntegrateArgs ia;
    double *pos_out;
    int4 *stage_out;
};
int force_blocks(const ForceArgs &a);  // number of partial slots written when energy
void launch_force(const ForceArgs &a, const Geom &g, hipStream_t s);

// window.hip
int64_t window_block_cap(int64_t n, const Geom &g);
int window_nbands(const Geom &g);
int window_force_blocks();
void launch_blocks(const Geom &g, const int32_t *cs, int4 *staged, int32_t *band_n, int32_t *band_base,
                   int32_t *scan_scratch, int4 *blocks, int cap, int32_t *flags, bool half, hipStream_t s);
// Staging slots the packer needs (int4 each).
int64_t window_staged_blocks(const Geom &g);
void launch_vlw_build(const int4 *st, const int32_t *cs, const int32_t *cell_sorted, const double *pos,
                      const Geom &g, int n, const int32_t *nblk_p, const int4 *blocks, uint16_t *nbr, int32_t *cnt,
                      int maxn, int32_t *flags, bool half, hipStream_t s);
void launch_window_force(const ForceArgs &a, const Geom &g, hipStream_t s);
// Windowed traversals need the same reach (1 or 2 cells) in every
// dimension and 2 reach + 1 distinct cells per dimension.
bool window_geometry_ok(const Geom &g, bool half);
void launch_vlw_decode(const int32_t *cs, const int32_t *cell_sorted, const Geom &g, int n, const int32_t *nblk_p,
                       const int4 *blocks, const uint16_t *nbr, const int32_t *cnt, int maxr, int32_t *counts,
                       int32_t *rows, bool half, hipStream_t s);
void launch_vl_build(int n, const int4 *stage, const int32_t *cell_start, const int32_t *cell_sorted,
                     const double *pos, const Geom &g, int half, int32_t *nbr, int32_t *cnt,
                     int64_t ld, int maxn, int32_t *flags, hipStream_t s);
void launch_reduce_out(const double *partials, int nblocks, int gather, double *out,
                       hipStream_t s);

// integrate.hip

int integrate_blocks(int n);
void launch_integrate(const IntegrateArgs &a, const Geom &g, hipStream_t s);
void launch_log_entry(const double *fpart, int fblocks, int gather, const double *kpart,
                      int kblocks, double *out4, hipStream_t s);
// flags[4] = the bits of the largest of the nblocks per-block maxima.
void launch_dmax_reduce(const float *dpart, int nblocks, int32_t *flags, hipStream_t s);

// adjoint.hip
struct AdjointArgs {
    int n;
    int precision;
    const double *pos;
    const int32_t *type;
    const int4 *stage;
    const int32_t *cell_start, *cell_sorted;
    const PairTab *tab;
    const double *lj;
    const void *grad_force;
    double *grad_pos;
    double *gpart;  // per block [8]: dL/d(eps_ab) [4], dL/d(sig_ab) [4]
    int32_t *flags;
};
int adjoint_blocks(int n);
void launch_adjoint(const AdjointArgs &a, const Geom &g, hipStream_t s);
// The adjoint over the gather windows (FP32; blocks packed for full windows);
// per-workgroup partials in gpart[window_force_blocks()][8].  only_if_overflow:
// return at once unless flags[0] holds MD_FLAG_LIST_OVERFLOW.
void launch_adjoint_window(const int4 *st, const int32_t *cs, const int32_t *cell_sorted, const Geom &g, int n,
                           const int32_t *nblk_p, const int4 *blocks, const PairTab *tab, const double *pos,
                           const float *G, double *grad_pos, double *gpart, int32_t *flags, hipStream_t s,
                           int only_if_overflow = 0);
// The same over the full Verlet lists of the window build (packed layout),
// followed by the window kernel that takes over when flags[0] holds
// MD_FLAG_LIST_OVERFLOW (the lists may be truncated): exactly one of the two
// does the work, decided on the device.
void launch_adjoint_lists(const int4 *st, const int32_t *cs, const int32_t *cell_sorted, const Geom &g, int n,
                          const int32_t *nblk_p, const int4 *blocks, const uint16_t *nbr, const int32_t *cnt,
                          const PairTab *tab, const double *pos, const float *G, double *grad_pos, double *gpart,
                          int32_t *flags, hipStream_t s);
void launch_adjoint_finish(const double *gpart, int nblocks, const double *lj, int nt,
                           double *grad_lj, hipStream_t s);

// pairwise.hip
// Pairwise Verlet lists need cells of side >= r_c + skin (reach 1) and at
// least three cells per dimension.
bool pvl_geometry_ok(const Geom &g);
void launch_pvl_build(int n, const int4 *st, const int32_t *cs, const int32_t *cell_sorted, const Geom &g, float *sv,
                      uint16_t *perm, uint16_t *cnt, hipStream_t s);
void launch_pvl_force(const ForceArgs &a, const Geom &g, hipStream_t s);
void launch_pvl_rows(int n, const int32_t *cs, const int32_t *cell_sorted, const Geom &g, const uint16_t *perm,
                     const uint16_t *cnt, int maxr, int32_t *counts, int32_t *rows, hipStream_t s);
void launch_pvl_entries(int n, const int32_t *cs, const int32_t *cell_sorted, const uint16_t *cnt,
                        unsigned long long *out, hipStream_t s);

// vlcells.hip (Verlet list cells traversed with the C08 colouring; the same
// geometry needs as pairwise lists)
// maxn: the row capacity and stride of nbr, a multiple of 8
void launch_vlc_build(int n, const int4 *st, const int32_t *cs, const int32_t *cell_sorted, const double *pos,
                      const Geom &g, uint16_t *nbr, uint16_t *seg, int32_t *cnt, int maxn, int32_t *flags,
                      hipStream_t s);
void launch_vlc_force(const ForceArgs &a, const Geom &g, hipStream_t s);
void launch_lc08_force(const ForceArgs &a, const Geom &g, hipStream_t s);
int vlc_force_blocks(const Geom &g);
void launch_vlc_rows(int n, const int32_t *cs, const int32_t *cell_sorted, const Geom &g, const uint16_t *nbr,
                     int ld, const uint16_t *seg, int maxr, int32_t *counts, int32_t *rows, hipStream_t s);

// clusters.hip
int cluster_force_blocks();
int64_t cluster_cap(int64_t n, const Geom &g);
void launch_cl_sort(int n, const int32_t *start, const double *pos, const int32_t *ids, const int32_t *cell_id,
                    const int32_t *perm, const Geom &g, uint64_t *key, int32_t *cell_of_slot, int32_t *perm_out,
                    hipStream_t s);
void launch_cluster_build(int n, const Geom &g, const int32_t *cs, const int4 *st, int32_t *ncl_per_cell,
                          int32_t *cl_base, int32_t *scan_scratch, int32_t *first, int32_t *cnt, int32_t *cell_of,
                          int4 *centre, float4 *half, int32_t *list, int32_t *lcnt, int64_t ld, int maxn,
                          int32_t *flags, hipStream_t s);
void launch_cluster_force(const ForceArgs &a, const Geom &g, hipStream_t s);
void launch_cl_rows(int n, const int32_t *cell_sorted, const int32_t *cs, const int32_t *cl_base,
                    const int32_t *first, const int32_t *cnt, const int32_t *list, const int32_t *lcnt, int64_t ld,
                    int maxr, int32_t *counts, int32_t *rows, hipStream_t s);

}  // namespace mdlj

// Linked cells by a counting sort (Sec. 2.2.1): cell index + histogram,
// exclusive scan, scatter, per-cell ordering by id, gather of the particle
// arrays into cell order and fixed-point staging of the positions.
#include <math.h>

#include "md_internal.h"

namespace mdlj {

// ------------------------------------------------------------------ helpers

__global__ void k_fill_i32(int32_t *p, int32_t v, int64_t n)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

void launch_fill_i32(int32_t *p, int32_t v, int64_t n, hipStream_t s)
{
    if (n <= 0) return;
    int64_t b = (n + kBlock - 1) / kBlock;
    k_fill_i32<<<(unsigned)b, kBlock, 0, s>>>(p, v, n);
}

// Cell coordinate of x along one dimension: min(n-1, (int)(x * n/L)),
// clamped to [0, n-1] so that an out-of-box or non-finite position cannot
// index outside the cell arrays (it is flagged instead).
__device__ __forceinline__ int cell_coord(double x, double inv_w, int nc, bool &bad)
{
    double t = x * inv_w;
    if (!(t >= 0.0 && t < (double)nc + 1.0)) {  // also catches NaN
        bad = true;
        return t > 0.0 ? nc - 1 : 0;
    }
    int c = (int)t;
    return c < nc - 1 ? c : nc - 1;
}

// Fixed-point staging: q = floor(x * 2^32 / L) as an unsigned 32-bit
// integer.  Differences of two staged coordinates, taken modulo 2^32 and read
// as signed, are the periodic minimum-image displacement in units of L/2^32.
__device__ __forceinline__ uint32_t quantise(double x, double S)
{
    double q = x * S;
    q = q < 0.0 ? 0.0 : (q > 4294967295.0 ? 4294967295.0 : q);
    return (uint32_t)q;
}

__device__ __forceinline__ int4 stage_of(double x, double y, double z, int t, const Geom &g)
{
    int4 r;
    r.x = (int)quantise(x, g.S[0]);
    r.y = (int)quantise(y, g.S[1]);
    r.z = (int)quantise(z, g.S[2]);
    r.w = t;
    return r;
}

// ------------------------------------------------------------------ K1: histogram

// Particles arrive mostly in the previous cell order, so consecutive lanes
// usually share a cell: one atomic per run of equal cells in a wavefront,
// the run's lanes take consecutive slots.
__global__ void k_cell_hist(int n, const double *__restrict__ pos, Geom g, int32_t *__restrict__ cell_id,
                            int32_t *__restrict__ slot, int32_t *__restrict__ count,
                            int32_t *__restrict__ flags)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    int lane = threadIdx.x & 63;
    int c = -1;
    if (i < n) {
        bool bad = false;
        int cx = cell_coord(pos[i], g.inv_w[0], g.nc[0], bad);
        int cy = cell_coord(pos[n + i], g.inv_w[1], g.nc[1], bad);
        int cz = cell_coord(pos[2 * (size_t)n + i], g.inv_w[2], g.nc[2], bad);
        if (bad) atomicOr(&flags[0], (int)MD_FLAG_NONFINITE);
        c = (cz * g.nc[1] + cy) * g.nc[0] + cx;
        cell_id[i] = c;
    }
    int prev = __shfl_up(c, 1, 64);
    bool head = lane == 0 || prev != c;
    uint64_t heads = __ballot(head);
    // run of lane: from its head (highest head bit <= lane) to the next head
    uint64_t below = heads & (lane == 63 ? ~0ull : ((2ull << lane) - 1));
    int hl = 63 - __builtin_clzll(below);
    uint64_t above = heads & ~(lane == 63 ? ~0ull : ((2ull << lane) - 1));
    int next = above ? __builtin_ctzll(above) : 64;
    int base = 0;
    if (head && c >= 0) base = atomicAdd(&count[c], next - lane);
    base = __shfl(base, hl, 64);
    if (c >= 0) slot[i] = base + (lane - hl);
}

void launch_cell_hist(int n, const double *pos, const Geom &g, int32_t *cell_id, int32_t *slot,
                      int32_t *count, int32_t *flags, hipStream_t s)
{
    if (n <= 0) return;
    k_cell_hist<<<(n + kBlock - 1) / kBlock, kBlock, 0, s>>>(n, pos, g, cell_id, slot, count, flags);
}

// Count-only histogram for the live statistics.
__global__ void k_bin_counts(int n, const double *__restrict__ pos, Geom g, int32_t *__restrict__ count)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    bool bad = false;
    int cx = cell_coord(pos[i], g.inv_w[0], g.nc[0], bad);
    int cy = cell_coord(pos[n + i], g.inv_w[1], g.nc[1], bad);
    int cz = cell_coord(pos[2 * (size_t)n + i], g.inv_w[2], g.nc[2], bad);
    atomicAdd(&count[(cz * g.nc[1] + cy) * g.nc[0] + cx], 1);
}

void launch_bin_counts(int n, const double *pos, const Geom &g, int32_t *count, hipStream_t s)
{
    if (n <= 0) return;
    k_bin_counts<<<(n + kBlock - 1) / kBlock, kBlock, 0, s>>>(n, pos, g, count);
}

// Summary of the bin counts for the live statistics: out[0..1] int64 sum
// and sum of squares, out as int32 from word 4: [4] max, [5] empty bins,
// [8 + v] number of bins holding v particles (v < kStatBins - 1; the last
// bin counts every larger value).  out must be zeroed first.
__global__ void k_bin_summary(int nb, const int32_t *__restrict__ count, int32_t *out)
{
    __shared__ int32_t hist[kStatBins];
    __shared__ unsigned long long s1, s2;
    __shared__ int32_t smax, sempty;
    for (int k = threadIdx.x; k < kStatBins; k += blockDim.x) hist[k] = 0;
    if (threadIdx.x == 0) {
        s1 = s2 = 0ull;
        smax = sempty = 0;
    }
    __syncthreads();
    unsigned long long a = 0, b = 0;
    int mx = 0, em = 0;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nb; i += gridDim.x * blockDim.x) {
        int v = count[i];
        a += (unsigned long long)v;
        b += (unsigned long long)v * (unsigned long long)v;
        mx = max(mx, v);
        em += v == 0;
        atomicAdd(&hist[min(v, kStatBins - 1)], 1);
    }
    atomicAdd(&s1, a);
    atomicAdd(&s2, b);
    atomicMax(&smax, mx);
    atomicAdd(&sempty, em);
    __syncthreads();
    unsigned long long *o64 = (unsigned long long *)out;
    for (int k = threadIdx.x; k < kStatBins; k += blockDim.x)
        if (hist[k]) atomicAdd(&out[8 + k], hist[k]);
    if (threadIdx.x == 0) {
        atomicAdd(&o64[0], s1);
        atomicAdd(&o64[1], s2);
        atomicMax(&out[4], smax);
        atomicAdd(&out[5], sempty);
    }
}

void launch_bin_summary(int nb, const int32_t *count, int32_t *out, hipStream_t s)
{
    launch_fill_i32(out, 0, 8 + kStatBins, s);
    if (nb <= 0) return;
    int blocks = std::min(256, (nb + kBlock - 1) / kBlock);
    k_bin_summary<<<blocks, kBlock, 0, s>>>(nb, count, out);
}

// ------------------------------------------------------------------ K2: exclusive scan
// Three passes: per-block totals, a scan of the totals in one block, and the
// per-block scan plus offset.  out has n + 1 entries (out[n] = total).
constexpr int kScanItems = 8;
constexpr int kScanTile = kBlock * kScanItems;  // 2048 elements per block

__device__ __forceinline__ int block_exclusive_scan(int v, int *sh, int &total)
{
    // Hillis-Steele over 256 threads in LDS; deterministic.
    int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int off = 1; off < kBlock; off <<= 1) {
        int add = t >= off ? sh[t - off] : 0;
        __syncthreads();
        sh[t] += add;
        __syncthreads();
    }
    total = sh[kBlock - 1];
    int incl = sh[t];
    __syncthreads();
    return incl - v;
}

__global__ void k_scan_totals(const int32_t *__restrict__ in, int64_t n, int32_t *__restrict__ totals)
{
    __shared__ int sh[kBlock];
    int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    int s = 0;
    for (int k = 0; k < kScanItems; k++)
        if (base + k < n) s += in[base + k];
    int total;
    block_exclusive_scan(s, sh, total);
    if (threadIdx.x == 0) totals[blockIdx.x] = total;
}

// Exclusive scan of at most kScanTile block totals in one block, in place.
__global__ void k_scan_blocks(int32_t *__restrict__ totals, int nb)
{
    __shared__ int sh[kBlock];
    int base = threadIdx.x * kScanItems;
    int v[kScanItems];
    int s = 0;
    for (int k = 0; k < kScanItems; k++) {
        v[k] = base + k < nb ? totals[base + k] : 0;
        s += v[k];
    }
    int total;
    int ex = block_exclusive_scan(s, sh, total);
    for (int k = 0; k < kScanItems; k++) {
        if (base + k < nb) totals[base + k] = ex;
        ex += v[k];
    }
}

// Per-block scan plus the block's offset: offs[blockIdx.x] if offs is given
// (scanned block totals), else the sum of the totals of the blocks before
// this one (at most kScanTile of them; none for a single block).
__global__ void k_scan_final(const int32_t *__restrict__ in, int64_t n, const int32_t *__restrict__ offs,
                             const int32_t *__restrict__ totals, int32_t *__restrict__ out)
{
    __shared__ int sh[kBlock];
    int off;
    if (offs) {
        off = offs[blockIdx.x];
    } else {
        int part = 0;
        for (int b = threadIdx.x; b < (int)blockIdx.x; b += blockDim.x) part += totals[b];
        int tot;
        int ex0 = block_exclusive_scan(part, sh, tot);
        (void)ex0;
        off = tot;
    }
    int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    int v[kScanItems];
    int s = 0;
    for (int k = 0; k < kScanItems; k++) {
        v[k] = base + k < n ? in[base + k] : 0;
        s += v[k];
    }
    int total;
    int ex = block_exclusive_scan(s, sh, total) + off;
    for (int k = 0; k < kScanItems; k++) {
        if (base + k < n) out[base + k] = ex;
        ex += v[k];
    }
    if (base <= n - 1 && n - 1 < base + kScanItems) out[n] = ex;  // grand total
}

// scratch must hold scan_scratch_size(n) ints.  Block totals are scanned in
// one block when there are at most kScanTile of them, else recursively.
int64_t scan_scratch_size(int64_t n)
{
    int64_t nb = (n + kScanTile - 1) / kScanTile;
    if (nb <= kScanTile) return nb + 1;
    return 2 * (nb + 1) + scan_scratch_size(nb);
}

void launch_scan(const int32_t *in, int32_t *out, int64_t n, int32_t *scratch, hipStream_t s)
{
    if (n <= 0) {
        launch_fill_i32(out, 0, 1, s);
        return;
    }
    int64_t nb = (n + kScanTile - 1) / kScanTile;
    int32_t *totals = scratch;
    if (nb == 1) {  // one tile: a single pass
        k_scan_final<<<1, kBlock, 0, s>>>(in, n, nullptr, totals, out);
        return;
    }
    k_scan_totals<<<(unsigned)nb, kBlock, 0, s>>>(in, n, totals);
    if (nb <= 64) {  // each block sums the few totals before it
        k_scan_final<<<(unsigned)nb, kBlock, 0, s>>>(in, n, nullptr, totals, out);
        return;
    }
    const int32_t *offs = totals;
    if (nb <= kScanTile) {
        k_scan_blocks<<<1, kBlock, 0, s>>>(totals, (int)nb);
    } else {
        int32_t *scanned = totals + nb + 1;
        launch_scan(totals, scanned, nb, scanned + nb + 1, s);
        offs = scanned;
    }
    k_scan_final<<<(unsigned)nb, kBlock, 0, s>>>(in, n, offs, nullptr, out);
}

// ------------------------------------------------------------------ K3: scatter + order

__global__ void k_scatter(int n, const int32_t *__restrict__ cell_id, const int32_t *__restrict__ slot,
                          const int32_t *__restrict__ start, int32_t *__restrict__ perm)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    perm[start[cell_id[i]] + slot[i]] = i;
}

void launch_scatter(int n, const int32_t *cell_id, const int32_t *slot, const int32_t *start,
                    int32_t *perm, hipStream_t s)
{
    if (n <= 0) return;
    k_scatter<<<(n + kBlock - 1) / kBlock, kBlock, 0, s>>>(n, cell_id, slot, start, perm);
}

// The atomic histogram leaves each cell's members in arbitrary order; order
// every cell's segment by id so that the cell contents are deterministic.
// Slot k's key and cell are gathered first; then each slot's rank among its
// cell's keys (ids are distinct) gives its final place.  Cells hold tens of
// particles, so each rank is a short scan of contiguous keys.
__global__ void k_cell_keys(int n, const int32_t *__restrict__ perm, const int32_t *__restrict__ ids,
                            const int32_t *__restrict__ cell_id, int32_t *__restrict__ key,
                            int32_t *__restrict__ cell_of_slot)
{
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    int p = perm[k];
    key[k] = ids[p];
    cell_of_slot[k] = cell_id[p];
}

__global__ void k_cell_rank(int n, const int32_t *__restrict__ start, const int32_t *__restrict__ key,
                            const int32_t *__restrict__ cell_of_slot, const int32_t *__restrict__ perm,
                            int32_t *__restrict__ perm_out)
{
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    int c = cell_of_slot[k];
    int b = start[c], e = start[c + 1];
    int kk = key[k];
    int r = 0;
    for (int m = b; m < e; m++) r += key[m] < kk ? 1 : 0;
    perm_out[b + r] = perm[k];
}

// Scatter fused with the key gather of the in-cell ordering: slot p of the
// cell order gets particle i, its id as key and its cell.  key must not alias
// slot (slot[i] is read while other threads write key[p]).
__global__ void k_scatter_keys(int n, const int32_t *__restrict__ cell_id, const int32_t *__restrict__ slot,
                               const int32_t *__restrict__ start, const int32_t *__restrict__ ids,
                               int32_t *__restrict__ perm, int32_t *__restrict__ key,
                               int32_t *__restrict__ cell_of_slot)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int c = cell_id[i];
    int p = start[c] + slot[i];
    perm[p] = i;
    key[p] = ids[i];
    cell_of_slot[p] = c;
}

// Counting-sort scatter and in-cell ordering by id in two launches:
// perm_out[k] = particle in cell-order slot k (perm and key are scratch).
void launch_scatter_sort(int n, const int32_t *cell_id, const int32_t *slot, const int32_t *start,
                         const int32_t *ids, int32_t *perm, int32_t *key, int32_t *cell_of_slot, int32_t *perm_out,
                         hipStream_t s)
{
    if (n <= 0) return;
    int nb = (n + kBlock - 1) / kBlock;
    k_scatter_keys<<<nb, kBlock, 0, s>>>(n, cell_id, slot, start, ids, perm, key, cell_of_slot);
    k_cell_rank<<<nb, kBlock, 0, s>>>(n, start, key, cell_of_slot, perm, perm_out);
}

// The same with every cell ordered by its staged x coordinate, then id.
// Cells are numbered x-fastest, so any run of consecutive cells along x (a
// row of a pair stencil) is then ordered by x as well, and a traversal can
// bound a row's candidates to an interval of x by bisection.
__global__ void k_scatter_xkeys(int n, const int32_t *__restrict__ cell_id, const int32_t *__restrict__ slot,
                                const int32_t *__restrict__ start, const int32_t *__restrict__ ids,
                                const double *__restrict__ pos, double S0, int32_t *__restrict__ perm,
                                uint64_t *__restrict__ key, int32_t *__restrict__ cell_of_slot)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int c = cell_id[i];
    int p = start[c] + slot[i];
    perm[p] = i;
    key[p] = ((uint64_t)quantise(pos[i], S0) << 32) | (uint32_t)ids[i];
    cell_of_slot[p] = c;
}

__global__ void k_cell_rank64(int n, const int32_t *__restrict__ start, const uint64_t *__restrict__ key,
                              const int32_t *__restrict__ cell_of_slot, const int32_t *__restrict__ perm,
                              int32_t *__restrict__ perm_out)
{
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    int c = cell_of_slot[k];
    int b = start[c], e = start[c + 1];
    uint64_t kk = key[k];
    int r = 0;
    for (int m = b; m < e; m++) r += key[m] < kk ? 1 : 0;
    perm_out[b + r] = perm[k];
}

void launch_scatter_sort_x(int n, const int32_t *cell_id, const int32_t *slot, const int32_t *start,
                           const int32_t *ids, const double *pos, const Geom &g, int32_t *perm, uint64_t *key,
                           int32_t *cell_of_slot, int32_t *perm_out, hipStream_t s)
{
    if (n <= 0) return;
    int nb = (n + kBlock - 1) / kBlock;
    k_scatter_xkeys<<<nb, kBlock, 0, s>>>(n, cell_id, slot, start, ids, pos, g.S[0], perm, key, cell_of_slot);
    k_cell_rank64<<<nb, kBlock, 0, s>>>(n, start, key, cell_of_slot, perm, perm_out);
}

void launch_cell_sort(int n, const int32_t *start, const int32_t *ids, const int32_t *cell_id, const int32_t *perm,
                      int32_t *key, int32_t *cell_of_slot, int32_t *perm_out, hipStream_t s)
{
    if (n <= 0) return;
    int nb = (n + kBlock - 1) / kBlock;
    k_cell_keys<<<nb, kBlock, 0, s>>>(n, perm, ids, cell_id, key, cell_of_slot);
    k_cell_rank<<<nb, kBlock, 0, s>>>(n, start, key, cell_of_slot, perm, perm_out);
}

// ------------------------------------------------------------------ K4: gather + stage

template <typename real>
__global__ void k_gather(int n, const int32_t *__restrict__ perm, const double *__restrict__ pos,
                         const real *__restrict__ vel, const real *__restrict__ force,
                         const int32_t *__restrict__ type, const int32_t *__restrict__ ids,
                         double *__restrict__ tpos, real *__restrict__ tvel, real *__restrict__ tforce,
                         int32_t *__restrict__ ttype, int32_t *__restrict__ tids,
                         const int32_t *__restrict__ cell_id, int32_t *__restrict__ cell_sorted, Geom g,
                         int4 *__restrict__ stage, int4 *__restrict__ stage_ref)
{
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    int src = perm[k];
    size_t N = (size_t)n;
    double x = pos[src], y = pos[N + src], z = pos[2 * N + src];
    tpos[k] = x;
    tpos[N + k] = y;
    tpos[2 * N + k] = z;
    if (vel) {
        tvel[k] = vel[src];
        tvel[N + k] = vel[N + src];
        tvel[2 * N + k] = vel[2 * N + src];
    }
    if (force) {
        tforce[k] = force[src];
        tforce[N + k] = force[N + src];
        tforce[2 * N + k] = force[2 * N + src];
    }
    int t = type[src];
    ttype[k] = t;
    tids[k] = ids[src];
    cell_sorted[k] = cell_id[src];
    int4 q = stage_of(x, y, z, t, g);
    stage[k] = q;
    stage_ref[k] = q;
}

void launch_gather(int n, int precision, const int32_t *perm, const double *pos, const void *vel,
                   const void *force, const int32_t *type, const int32_t *ids, double *tpos,
                   void *tvel, void *tforce, int32_t *ttype, int32_t *tids, const int32_t *cell_id,
                   int32_t *cell_sorted, const Geom &g, int4 *stage, int4 *stage_ref, hipStream_t s)
{
    if (n <= 0) return;
    int nb = (n + kBlock - 1) / kBlock;
    if (precision == MD_FP64)
        k_gather<double><<<nb, kBlock, 0, s>>>(n, perm, pos, (const double *)vel, (const double *)force,
                                               type, ids, tpos, (double *)tvel, (double *)tforce, ttype,
                                               tids, cell_id, cell_sorted, g, stage, stage_ref);
    else
        k_gather<float><<<nb, kBlock, 0, s>>>(n, perm, pos, (const float *)vel, (const float *)force,
                                              type, ids, tpos, (float *)tvel, (float *)tforce, ttype,
                                              tids, cell_id, cell_sorted, g, stage, stage_ref);
}

__global__ void k_stage(int n, const double *__restrict__ pos, const int32_t *__restrict__ type, Geom g,
                        int4 *__restrict__ stage)
{
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    size_t N = (size_t)n;
    stage[k] = stage_of(pos[k], pos[N + k], pos[2 * N + k], type[k], g);
}

void launch_stage(int n, const double *pos, const int32_t *type, const Geom &g, int4 *stage, hipStream_t s)
{
    if (n <= 0) return;
    k_stage<<<(n + kBlock - 1) / kBlock, kBlock, 0, s>>>(n, pos, type, g, stage);
}

// ------------------------------------------------------------------ pair tables

// One thread: Lorentz-Berthelot mixing of the per-type parameters and the
// derived per-pair constants of both precisions.
__global__ void k_prepare_tab(const double *__restrict__ lj, double rc2_0, double rc2_1, double rc2_2,
                              double rc2_3, Geom g, PairTab *__restrict__ tab)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    int nt = g.nt;
    double rc2[4] = {rc2_0, rc2_1, rc2_2, rc2_3};
    double u = g.L[0] / 4294967296.0;  // fixed-point length unit
    for (int a = 0; a < nt; a++)
        for (int b = 0; b < nt; b++) {
            int ab = a * nt + b;
            double sig = 0.5 * (lj[nt + a] + lj[nt + b]);
            double eps = sqrt(lj[a] * lj[b]);
            tab->sig[ab] = sig;
            tab->eps[ab] = eps;
            tab->rc2[ab] = rc2[ab];
            double r2u = rc2[ab] / (u * u);
            tab->rc2_lo[ab] = (float)(r2u * (1.0 - kBand));
            tab->rc2_hi[ab] = (float)(r2u * (1.0 + kBand));
            tab->sig2[ab] = (float)(sig * sig / (u * u));
            tab->eps24[ab] = (float)(24.0 * eps / u);
            tab->eps4[ab] = (float)(4.0 * eps);
            tab->eps24w[ab] = (float)(24.0 * eps);
        }
}

void launch_prepare_tab(const double *lj, const double *rc2, const Geom &g, PairTab *tab, hipStream_t s)
{
    k_prepare_tab<<<1, 64, 0, s>>>(lj, rc2[0], rc2[1], rc2[2], rc2[3], g, tab);
}

}  // namespace mdlj

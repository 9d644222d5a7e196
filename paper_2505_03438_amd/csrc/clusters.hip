// Cluster-pair lists.
//
// Within each linked cell (side >= r_c + skin) the particles are ordered by a
// 6-bit Morton code of their position inside the cell (then by id), and cut
// into clusters of up to eight consecutive particles, which are therefore
// spatially compact.  Each cluster gets a bounding box; a cluster pair enters
// the list of cluster i when the distance between the boxes is below
// r_c + skin (the boxes are those of the build positions, and no particle
// moves more than skin/2 before the next build).  The force kernel runs one
// wavefront per i-cluster: lane (ii, jj) = (lane % 8, lane / 8) evaluates
// the pair (particle ii of cluster i, particle jj of cluster j) for every j
// cluster of the list, gather-only, and the eight partial forces of each
// i-particle are summed across lanes with shuffles at the end.
#include "pair.h"

struct md_handle;

namespace mdlj {

constexpr int kClusterSize = 8;
constexpr int kClGrid = 4096;  // persistent workgroups of 4 wavefronts

// 2-bit sub-cell coordinate of x inside its cell along one axis.
__device__ __forceinline__ uint32_t subcell(double x, double inv_w, int nc)
{
    double t = x * inv_w;
    int c = (int)t;
    c = c < 0 ? 0 : (c > nc - 1 ? nc - 1 : c);
    int s = (int)((t - (double)c) * 4.0);
    return (uint32_t)(s < 0 ? 0 : (s > 3 ? 3 : s));
}

__device__ __forceinline__ uint32_t morton6(uint32_t x, uint32_t y, uint32_t z)
{
    uint32_t m = 0;
    for (int b = 1; b >= 0; b--) m = (m << 3) | (((z >> b) & 1) << 2) | (((y >> b) & 1) << 1) | ((x >> b) & 1);
    return m;
}

// Key of slot k: Morton code inside the cell, then id.
__global__ void k_cl_keys(int n, const int32_t *__restrict__ perm, const double *__restrict__ pos,
                          const int32_t *__restrict__ ids, const int32_t *__restrict__ cell_id, Geom g,
                          uint64_t *__restrict__ key, int32_t *__restrict__ cell_of_slot)
{
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    int p = perm[k];
    size_t N = (size_t)n;
    uint32_t m = morton6(subcell(pos[p], g.inv_w[0], g.nc[0]), subcell(pos[N + p], g.inv_w[1], g.nc[1]),
                         subcell(pos[2 * N + p], g.inv_w[2], g.nc[2]));
    key[k] = ((uint64_t)m << 32) | (uint32_t)ids[p];
    cell_of_slot[k] = cell_id[p];
}

__global__ void k_cl_rank(int n, const int32_t *__restrict__ start, const uint64_t *__restrict__ key,
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

void launch_cl_sort(int n, const int32_t *start, const double *pos, const int32_t *ids, const int32_t *cell_id,
                    const int32_t *perm, const Geom &g, uint64_t *key, int32_t *cell_of_slot, int32_t *perm_out,
                    hipStream_t s)
{
    if (n <= 0) return;
    int nb = (n + kBlock - 1) / kBlock;
    k_cl_keys<<<nb, kBlock, 0, s>>>(n, perm, pos, ids, cell_id, g, key, cell_of_slot);
    k_cl_rank<<<nb, kBlock, 0, s>>>(n, start, key, cell_of_slot, perm, perm_out);
}

// Clusters per cell.
__global__ void k_cl_count(int ncell, const int32_t *__restrict__ cs, int32_t *__restrict__ ncl)
{
    int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncell) return;
    ncl[c] = (cs[c + 1] - cs[c] + kClusterSize - 1) / kClusterSize;
}

// Cluster k of cell c: particles [cs[c] + 8k, ...), its cell, and its
// bounding box: centre (fixed point) and half extents (x units).
template <bool ISO>
__global__ void k_cl_make(int ncell, const int32_t *__restrict__ cs, const int32_t *__restrict__ cl_base,
                          const int4 *__restrict__ st, Geom g, int32_t *__restrict__ first, int32_t *__restrict__ cnt,
                          int32_t *__restrict__ cell_of, int4 *__restrict__ centre, float4 *__restrict__ half)
{
    int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncell) return;
    int b = cs[c], e = cs[c + 1];
    int k0 = cl_base[c];
    for (int k = 0; b + k * kClusterSize < e; k++) {
        int p0 = b + k * kClusterSize, p1 = min(e, p0 + kClusterSize);
        int4 ref = st[p0];
        int lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
        for (int p = p0 + 1; p < p1; p++) {
            int4 q = st[p];
            int d[3] = {(int)((uint32_t)q.x - (uint32_t)ref.x), (int)((uint32_t)q.y - (uint32_t)ref.y),
                        (int)((uint32_t)q.z - (uint32_t)ref.z)};
            for (int a = 0; a < 3; a++) {
                lo[a] = min(lo[a], d[a]);
                hi[a] = max(hi[a], d[a]);
            }
        }
        int ci = k0 + k;
        first[ci] = p0;
        cnt[ci] = p1 - p0;
        cell_of[ci] = c;
        int4 ctr;
        ctr.x = (int)((uint32_t)ref.x + (uint32_t)((lo[0] + hi[0]) / 2));
        ctr.y = (int)((uint32_t)ref.y + (uint32_t)((lo[1] + hi[1]) / 2));
        ctr.z = (int)((uint32_t)ref.z + (uint32_t)((lo[2] + hi[2]) / 2));
        ctr.w = 0;
        centre[ci] = ctr;
        // half extents, rounded up by one unit for the integer midpoint (the
        // spread is taken in float: it may exceed INT32_MAX in a box of one cell)
        float hx = 0.5f * ((float)hi[0] - (float)lo[0]) + 1.0f;
        float hy = 0.5f * ((float)hi[1] - (float)lo[1]) + 1.0f;
        float hz = 0.5f * ((float)hi[2] - (float)lo[2]) + 1.0f;
        if (!ISO) {
            hy *= g.ry;
            hz *= g.rz;
        }
        half[ci] = make_float4(hx, hy, hz, 0.0f);
    }
}

// Cluster-pair list of every i-cluster: j-clusters of the stencil cells whose
// boxes are closer than r_c + skin (with a small margin for rounding).
template <bool ISO>
__global__ void k_cl_pairs(const int32_t *__restrict__ ncl_p, const int32_t *__restrict__ cl_base,
                           const int32_t *__restrict__ cell_of, const int4 *__restrict__ centre,
                           const float4 *__restrict__ half, Geom g, int32_t *__restrict__ list,
                           int32_t *__restrict__ lcnt, int64_t ld, int maxn, int32_t *__restrict__ flags)
{
    __shared__ int so[3][kMaxOfs];
    load_offsets(g, so);
    int ncl = *ncl_p;
    float cut2 = g.rl2_hi * 1.0001f;
    for (int ci = blockIdx.x * blockDim.x + threadIdx.x; ci < ncl; ci += gridDim.x * blockDim.x) {
        int c = cell_of[ci];
        int cx = c % g.nc[0], t = c / g.nc[0];
        int cy = t % g.nc[1], cz = t / g.nc[1];
        int4 a = centre[ci];
        float4 ha = half[ci];
        int cnt = 0;
        for (int oz = 0; oz < g.nofs[2]; oz++) {
            int zz = cz + so[2][oz];
            zz = zz >= g.nc[2] ? zz - g.nc[2] : zz;
            for (int oy = 0; oy < g.nofs[1]; oy++) {
                int yy = cy + so[1][oy];
                yy = yy >= g.nc[1] ? yy - g.nc[1] : yy;
                int row = (zz * g.nc[1] + yy) * g.nc[0];
                for (int ox = 0; ox < g.nofs[0]; ox++) {
                    int xx = cx + so[0][ox];
                    xx = xx >= g.nc[0] ? xx - g.nc[0] : xx;
                    int cell = row + xx;
                    for (int cj = cl_base[cell]; cj < cl_base[cell + 1]; cj++) {
                        float dx, dy, dz;
                        staged_delta<ISO>(a, centre[cj], g, dx, dy, dz);
                        float4 hb = half[cj];
                        float gx = fmaxf(0.0f, fabsf(dx) - (ha.x + hb.x));
                        float gy = fmaxf(0.0f, fabsf(dy) - (ha.y + hb.y));
                        float gz = fmaxf(0.0f, fabsf(dz) - (ha.z + hb.z));
                        if (gx * gx + gy * gy + gz * gz < cut2) {
                            if (cnt < maxn) list[(size_t)cnt * ld + ci] = cj;
                            cnt++;
                        }
                    }
                }
            }
        }
        if (cnt > maxn) atomicOr(&flags[0], (int)MD_FLAG_LIST_OVERFLOW);
        atomicMax(&flags[2], cnt);
        lcnt[ci] = cnt < maxn ? cnt : maxn;
    }
}

// One wavefront per i-cluster, lane (ii, jj); gather-only.  The list is
// read 64 entries at a time, one entry per lane, together with each entry's
// j-cluster first particle and count; the loop over the entries then takes
// them from those lanes (wavefront-uniform), and the staged positions of
// the next entry's j-cluster are loaded while the current one is computed.
template <int NT, bool ISO, bool ENERGY>
__global__ __launch_bounds__(256) void k_cl_f32(int n, const int32_t *__restrict__ ncl_p,
                                                const int32_t *__restrict__ first, const int32_t *__restrict__ cnt,
                                                const int32_t *__restrict__ list, const int32_t *__restrict__ lcnt,
                                                int64_t ld, const int4 *__restrict__ st,
                                                const PairTab *__restrict__ tabp, Geom g,
                                                const double *__restrict__ pos, float *__restrict__ F,
                                                double *__restrict__ partials)
{
    __shared__ double sh[16];
    TabF<NT> t;
    t.load(tabp);
    int lane = threadIdx.x & 63;
    int ii = lane & 7, jj = lane >> 3;
    int wave = __builtin_amdgcn_readfirstlane((blockIdx.x * blockDim.x + threadIdx.x) >> 6);
    int nwaves = (gridDim.x * blockDim.x) >> 6;
    int ncl = *ncl_p;
    float eu = 0.f, ew = 0.f;
    int np = 0;
    size_t N = (size_t)n;
    for (int ci = wave; ci < ncl; ci += nwaves) {
        int fi = first[ci], ni = cnt[ci];
        bool vi = ii < ni;
        int i = fi + (vi ? ii : 0);
        int4 pi = st[i];
        float fx = 0.f, fy = 0.f, fz = 0.f;
        int m = __builtin_amdgcn_readfirstlane(lcnt[ci]);
        for (int k0 = 0; k0 < m; k0 += 64) {
            int mm = min(64, m - k0);
            // lane e holds entry k0 + e: its j-cluster's first particle and count
            int cjl = lane < mm ? list[(size_t)(k0 + lane) * ld + ci] : 0;
            int fjl = lane < mm ? first[cjl] : 0;
            int njl = lane < mm ? cnt[cjl] : 0;
            int fj = __builtin_amdgcn_readlane(fjl, 0), nj = __builtin_amdgcn_readlane(njl, 0);
            int4 pj = st[fj + (jj < nj ? jj : 0)];
            for (int e = 0; e < mm; e++) {
                int en = min(e + 1, mm - 1);
                int fjn = __builtin_amdgcn_readlane(fjl, en), njn = __builtin_amdgcn_readlane(njl, en);
                int4 pjn = st[fjn + (jj < njn ? jj : 0)];
                int j = fj + (jj < nj ? jj : 0);
                bool valid = vi && jj < nj && i != j;
                float dx, dy, dz;
                staged_delta<ISO>(pi, pj, g, dx, dy, dz);
                float r2 = dx * dx + dy * dy + dz * dz;
                int ab = NT == 1 ? 0 : pi.w * NT + pj.w;
                float lo = t.pick(t.lo, ab), hi = t.pick(t.hi, ab);
                bool in = valid && r2 < lo;
                if (valid && r2 >= lo && r2 < hi)
                    in = exact_r2(pos, n, i, j, g.L[0], g.L[1], g.L[2]) < t.pickd(t.rc2, ab);
                float phi = lj_f32<NT, ENERGY>(r2, ab, in, t, eu, ew, np);
                fx += phi * dx;
                fy += phi * dy;
                fz += phi * dz;
                fj = fjn;
                nj = njn;
                pj = pjn;
            }
        }
        // sum the eight j-slots of every i-particle
        for (int off = 8; off < 64; off <<= 1) {
            fx += __shfl_xor(fx, off, 64);
            fy += __shfl_xor(fy, off, 64);
            fz += __shfl_xor(fz, off, 64);
        }
        if (jj == 0 && vi) {
            F[i] = fx;
            F[N + i] = fy;
            F[2 * N + i] = fz;
        }
    }
    if (ENERGY) {
        double v[4] = {(double)eu, (double)ew, (double)np, 0.0};
        block_sum4(v, sh);
        if (threadIdx.x == 0)
            for (int k = 0; k < 4; k++) partials[blockIdx.x * 4 + k] = v[k];
    }
}

// Candidate rows of the cluster lists for inspection: slot k gets every
// particle of the j-clusters of its own cluster, itself excluded.
__global__ void k_cl_rows(int n, const int32_t *__restrict__ cell_sorted, const int32_t *__restrict__ cs,
                          const int32_t *__restrict__ cl_base, const int32_t *__restrict__ first,
                          const int32_t *__restrict__ cnt, const int32_t *__restrict__ list,
                          const int32_t *__restrict__ lcnt, int64_t ld, int maxr, int32_t *__restrict__ counts,
                          int32_t *__restrict__ rows)
{
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    int c = cell_sorted[k];
    int ci = cl_base[c] + (k - cs[c]) / kClusterSize;
    int m = 0;
    for (int e = 0; e < lcnt[ci]; e++) {
        int cj = list[(size_t)e * ld + ci];
        for (int p = first[cj]; p < first[cj] + cnt[cj]; p++) {
            if (p == k) continue;
            if (m < maxr) rows[(size_t)k * maxr + m] = p;
            m++;
        }
    }
    counts[k] = m;
}

void launch_cl_rows(int n, const int32_t *cell_sorted, const int32_t *cs, const int32_t *cl_base,
                    const int32_t *first, const int32_t *cnt, const int32_t *list, const int32_t *lcnt, int64_t ld,
                    int maxr, int32_t *counts, int32_t *rows, hipStream_t s)
{
    if (n <= 0) return;
    k_cl_rows<<<(n + kBlock - 1) / kBlock, kBlock, 0, s>>>(n, cell_sorted, cs, cl_base, first, cnt, list, lcnt, ld,
                                                           maxr, counts, rows);
}

int cluster_force_blocks() { return kClGrid; }

int64_t cluster_cap(int64_t n, const Geom &g) { return n / kClusterSize + g.ncell + 1; }

void launch_cluster_build(int n, const Geom &g, const int32_t *cs, const int4 *st, int32_t *ncl_per_cell,
                          int32_t *cl_base, int32_t *scan_scratch, int32_t *first, int32_t *cnt, int32_t *cell_of,
                          int4 *centre, float4 *half, int32_t *list, int32_t *lcnt, int64_t ld, int maxn,
                          int32_t *flags, hipStream_t s)
{
    int nb = (g.ncell + kBlock - 1) / kBlock;
    k_cl_count<<<nb, kBlock, 0, s>>>(g.ncell, cs, ncl_per_cell);
    launch_scan(ncl_per_cell, cl_base, g.ncell, scan_scratch, s);
    if (n <= 0) return;
    const int32_t *ncl_p = cl_base + g.ncell;
    if (g.iso) {
        k_cl_make<true><<<nb, kBlock, 0, s>>>(g.ncell, cs, cl_base, st, g, first, cnt, cell_of, centre, half);
        k_cl_pairs<true><<<1024, kBlock, 0, s>>>(ncl_p, cl_base, cell_of, centre, half, g, list, lcnt, ld, maxn, flags);
    } else {
        k_cl_make<false><<<nb, kBlock, 0, s>>>(g.ncell, cs, cl_base, st, g, first, cnt, cell_of, centre, half);
        k_cl_pairs<false><<<1024, kBlock, 0, s>>>(ncl_p, cl_base, cell_of, centre, half, g, list, lcnt, ld, maxn,
                                                   flags);
    }
}

template <int NT, bool ISO, bool EN>
static void cl_launch(const ForceArgs &a, const Geom &g, hipStream_t s)
{
    k_cl_f32<NT, ISO, EN><<<kClGrid, 256, 0, s>>>(a.n, a.cl_ncl, a.cl_start, a.cl_count, a.cl_nbr, a.cl_nbr_count,
                                                  a.cl_ld, a.stage, a.tab, g, a.pos, (float *)a.force, a.partials);
}

void launch_cluster_force(const ForceArgs &a, const Geom &g, hipStream_t s)
{
    if (a.n <= 0) return;
    if (g.nt == 1) {
        if (g.iso) {
            if (a.energy) cl_launch<1, true, true>(a, g, s);
            else cl_launch<1, true, false>(a, g, s);
        } else {
            if (a.energy) cl_launch<1, false, true>(a, g, s);
            else cl_launch<1, false, false>(a, g, s);
        }
    } else {
        if (g.iso) {
            if (a.energy) cl_launch<2, true, true>(a, g, s);
            else cl_launch<2, true, false>(a, g, s);
        } else {
            if (a.energy) cl_launch<2, false, true>(a, g, s);
            else cl_launch<2, false, false>(a, g, s);
        }
    }
}

}  // namespace mdlj

// Pairwise Verlet lists (Sec. 2.2.1 names them among the containers; the
// method is the sorted cell pairs of Gonnet, 2012).  For every pair of
// neighbouring cells A, B = A + o the particles of both cells are sorted
// along the direction o; the partners j in B that particle i in A can reach
// within r_c + skin lie below a threshold of the projection x_j . o, so they
// are a prefix of B's sorted order (a suffix when looking from B back to A).
// Per particle and neighbour cell only that prefix length is stored: the
// "list" of i towards B.  The force pass walks, for each of the 26 neighbour
// cells, the stored prefix of its sorted order, plus the particle's own
// cell, and decides every candidate exactly (FP32 outside the guard band,
// FP64 inside), gather-only.
//
// Build, after the cell build (cells of side >= r_c + skin, at least three per
// dimension):
//   1. per cell and per direction o (13 directions, the other 13 are their
//      negatives) the cell's particles are ranked by projection: the sorted
//      order (in-cell offsets) and the sorted projections are written;
//   2. every particle counts, per neighbour cell, the particles of that cell
//      whose sorted projection passes its threshold: the prefix (or suffix)
//      length.  The count uses the stored projections, the very keys of the
//      sort, so the passing particles are exactly a prefix (suffix).
// A projection uses coordinates relative to the particle's own cell corner,
// in x units of the fixed-point staging; the threshold is r_l |o| with a
// relative margin of 1e-5 (the FP32 rounding of a projection is below 1e-6 of
// it), so the prefix always holds every partner within r_l at the build.
#include "pair.h"

namespace mdlj {

constexpr int kPvlDirs = 13;

// Direction d (0..12) of the forward half: the nine cells of the layer
// above, the three of the row ahead in the same layer, the next cell in x.
__device__ __forceinline__ void pvl_dir(int d, int &ox, int &oy, int &oz)
{
    if (d < 9) {
        ox = d % 3 - 1;
        oy = d / 3 - 1;
        oz = 1;
    } else if (d < 12) {
        ox = d - 10;
        oy = 1;
        oz = 0;
    } else {
        ox = 1;
        oy = 0;
        oz = 0;
    }
}

__device__ __forceinline__ int pvl_wrap(int v, int nc) { return v < 0 ? v + nc : (v >= nc ? v - nc : v); }

// Fixed-point corner of cell column c of nc (the cell's lowest coordinate).
__device__ __forceinline__ uint32_t pvl_corner(int c, int nc)
{
    return (uint32_t)((((uint64_t)c) << 32) / (uint64_t)nc);
}

// Coordinates of a staged particle relative to its cell's corner, in x units.
__device__ __forceinline__ void pvl_rel(const int4 &q, uint32_t cx, uint32_t cy, uint32_t cz, const Geom &g,
                                        float &rx, float &ry, float &rz)
{
    rx = (float)(int)((uint32_t)q.x - cx);
    ry = (float)(int)((uint32_t)q.y - cy) * g.ry;
    rz = (float)(int)((uint32_t)q.z - cz) * g.rz;
}

__device__ __forceinline__ float pvl_proj(float rx, float ry, float rz, int d)
{
    int ox, oy, oz;
    pvl_dir(d, ox, oy, oz);
    float s = (float)ox * rx;
    s = s + (float)oy * ry;
    return s + (float)oz * rz;
}

__device__ __forceinline__ void pvl_cell_xyz(int c, const Geom &g, int &cx, int &cy, int &cz)
{
    cx = c % g.nc[0];
    int t = c / g.nc[0];
    cy = t % g.nc[1];
    cz = t / g.nc[1];
}

// Phase 1: rank of particle k in its cell along every direction (ties by
// position in the cell), written as the sorted order and sorted projection.
__global__ __launch_bounds__(kBlock) void k_pvl_sort(int n, const int4 *__restrict__ st, const int32_t *__restrict__ cs,
                                                     const int32_t *__restrict__ cell_sorted, Geom g,
                                                     float *__restrict__ sv, uint16_t *__restrict__ perm)
{
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    int c = cell_sorted[k];
    int s0 = cs[c], m = cs[c + 1] - s0;
    int cx, cy, cz;
    pvl_cell_xyz(c, g, cx, cy, cz);
    uint32_t qx = pvl_corner(cx, g.nc[0]), qy = pvl_corner(cy, g.nc[1]), qz = pvl_corner(cz, g.nc[2]);
    float rx, ry, rz;
    pvl_rel(st[k], qx, qy, qz, g, rx, ry, rz);
    float sk[kPvlDirs];
    int rank[kPvlDirs];
#pragma unroll
    for (int d = 0; d < kPvlDirs; d++) {
        sk[d] = pvl_proj(rx, ry, rz, d);
        rank[d] = 0;
    }
    for (int l = s0; l < s0 + m; l++) {
        float ax, ay, az;
        pvl_rel(st[l], qx, qy, qz, g, ax, ay, az);
        bool before = l < k;
#pragma unroll
        for (int d = 0; d < kPvlDirs; d++) {
            float sl = pvl_proj(ax, ay, az, d);
            rank[d] += (sl < sk[d] || (sl == sk[d] && before)) ? 1 : 0;
        }
    }
    size_t N = (size_t)n;
#pragma unroll
    for (int d = 0; d < kPvlDirs; d++) {
        size_t slot = (size_t)d * N + (size_t)(s0 + rank[d]);
        sv[slot] = sk[d];
        perm[slot] = (uint16_t)(k - s0);
    }
}

// Phase 2: one thread per particle p (cell C) and each of its 26 neighbour
// slots counts the candidates by comparing with the sorted projections of the
// neighbour cell B (contiguous, so the loads are independent).  Forward slot
// d, B = C + o_d: the partners j with (x_j - x_p) . o_d < thr are the j with
// s_j < s_p + thr - D (D: B's corner lies D further along o_d), a prefix of
// B's order.  Backward slot 13 + d, B = C - o_d: the partners with
// (x_j - x_p) . (-o_d) < thr are the j with s_j > s_p + D - thr, a suffix.
// Projections s are relative to each particle's own cell corner.
__global__ __launch_bounds__(kBlock) void k_pvl_count(int n, const int4 *__restrict__ st, Geom g,
                                                      const int32_t *__restrict__ cs,
                                                      const int32_t *__restrict__ cell_sorted,
                                                      const float *__restrict__ sv, uint16_t *__restrict__ cnt,
                                                      float thr1, float thr2, float thr3, float wx, float wy, float wz)
{
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    size_t N = (size_t)n;
    int c = cell_sorted[p];
    int cx, cy, cz;
    pvl_cell_xyz(c, g, cx, cy, cz);
    float rx, ry, rz;
    pvl_rel(st[p], pvl_corner(cx, g.nc[0]), pvl_corner(cy, g.nc[1]), pvl_corner(cz, g.nc[2]), g, rx, ry, rz);
    for (int q = 0; q < 2 * kPvlDirs; q++) {
        bool fwd = q < kPvlDirs;
        int d = fwd ? q : q - kPvlDirs;
        int ox, oy, oz;
        pvl_dir(d, ox, oy, oz);
        int nz = (ox != 0) + (oy != 0) + (oz != 0);
        float thr = nz == 1 ? thr1 : (nz == 2 ? thr2 : thr3);
        float D = (ox ? wx : 0.f) + (oy ? wy : 0.f) + (oz ? wz : 0.f);
        float sp = pvl_proj(rx, ry, rz, d);
        int sg = fwd ? 1 : -1;
        int B = (pvl_wrap(cz + sg * oz, g.nc[2]) * g.nc[1] + pvl_wrap(cy + sg * oy, g.nc[1])) * g.nc[0] +
                pvl_wrap(cx + sg * ox, g.nc[0]);
        int s0B = cs[B], mB = cs[B + 1] - s0B;
        const float *sB = sv + (size_t)d * N + s0B;
        int m = 0;
        if (fwd) {
            float lim = sp + thr - D;
            for (int k = 0; k < mB; k++) m += sB[k] < lim ? 1 : 0;
        } else {
            float lim = sp + D - thr;
            for (int k = 0; k < mB; k++) m += sB[k] > lim ? 1 : 0;
        }
        cnt[(size_t)q * N + p] = (uint16_t)m;
    }
}

// Candidate q of particle i's neighbour slot (q < 13: prefix towards A + o_q;
// else suffix towards A - o_{q-13}), k-th of cnt: its particle index.
__device__ __forceinline__ int pvl_neighbour(const Geom &g, int cx, int cy, int cz, int q, int &d, bool &fwd)
{
    fwd = q < kPvlDirs;
    d = fwd ? q : q - kPvlDirs;
    int ox, oy, oz;
    pvl_dir(d, ox, oy, oz);
    if (!fwd) {
        ox = -ox;
        oy = -oy;
        oz = -oz;
    }
    return (pvl_wrap(cz + oz, g.nc[2]) * g.nc[1] + pvl_wrap(cy + oy, g.nc[1])) * g.nc[0] + pvl_wrap(cx + ox, g.nc[0]);
}

// Force pass, gather-only: thread per particle (cell order).
template <int NT, bool ISO, bool ENERGY>
__global__ __launch_bounds__(kBlock) void k_pvl_f32(int n, const int4 *__restrict__ st, const int32_t *__restrict__ cs,
                                                    const int32_t *__restrict__ cell_sorted,
                                                    const uint16_t *__restrict__ perm,
                                                    const uint16_t *__restrict__ cnt, const PairTab *__restrict__ tabp,
                                                    Geom g, const double *__restrict__ pos, float *__restrict__ F,
                                                    double *__restrict__ partials)
{
    __shared__ double sh[4 * kBlock / 64];
    TabF<NT> t;
    t.load(tabp);
    float fx = 0.f, fy = 0.f, fz = 0.f, eu = 0.f, ew = 0.f;
    int np = 0;
    int i = blockIdx.x * kBlock + threadIdx.x;
    size_t N = (size_t)n;
    if (i < n) {
        int4 pi = st[i];
        auto pair_at = [&](int j, const int4 &pj) {
            float dx, dy, dz;
            staged_delta<ISO>(pi, pj, g, dx, dy, dz);
            float r2 = dx * dx + dy * dy + dz * dz;
            int ab = NT == 1 ? 0 : pi.w * NT + pj.w;
            bool in = within(r2, t.pick(t.lo, ab), t.pick(t.hi, ab), t.pickd(t.rc2, ab), pos, n, i, j, g);
            float phi = lj_f32<NT, ENERGY>(r2, ab, in, t, eu, ew, np);
            fx += phi * dx;
            fy += phi * dy;
            fz += phi * dz;
        };
        int c = cell_sorted[i];
        int cx, cy, cz;
        pvl_cell_xyz(c, g, cx, cy, cz);
        int s0 = cs[c], e0 = cs[c + 1];
        auto pair = [&](int j) { pair_at(j, st[j]); };
        for (int j = s0; j < e0; j++)
            if (j != i) pair(j);
        for (int q = 0; q < 2 * kPvlDirs; q++) {
            int d;
            bool fwd;
            int B = pvl_neighbour(g, cx, cy, cz, q, d, fwd);
            int s0B = cs[B], mB = cs[B + 1] - s0B;
            int m = cnt[(size_t)q * N + i];
            // the walked part of B's order: [first, first + m) ascending
            const uint16_t *pp = perm + (size_t)d * N + s0B + (fwd ? 0 : mB - m);
            for (int k0 = 0; k0 < m; k0 += 4) {
                // four indices, then four positions, loaded before any is used
                int jj[4];
                int4 pj[4];
#pragma unroll
                for (int u = 0; u < 4; u++) jj[u] = s0B + (k0 + u < m ? (int)pp[k0 + u] : (int)pp[0]);
#pragma unroll
                for (int u = 0; u < 4; u++) pj[u] = st[jj[u]];
#pragma unroll
                for (int u = 0; u < 4; u++)
                    if (k0 + u < m) pair_at(jj[u], pj[u]);
            }
        }
        F[i] = fx;
        F[N + i] = fy;
        F[2 * N + i] = fz;
    }
    if (ENERGY) {
        double v[4] = {(double)eu, (double)ew, (double)np, 0.0};
        block_sum4(v, sh);
        if (threadIdx.x == 0)
            for (int k = 0; k < 4; k++) partials[blockIdx.x * 4 + k] = v[k];
    }
}

// The candidates of every particle (its own cell and the stored prefixes),
// for inspection: counts[i] and rows[i][0 .. max_per_row).
__global__ void k_pvl_rows(int n, const int32_t *__restrict__ cs, const int32_t *__restrict__ cell_sorted, Geom g,
                           const uint16_t *__restrict__ perm, const uint16_t *__restrict__ cnt, int maxr,
                           int32_t *__restrict__ counts, int32_t *__restrict__ rows)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    size_t N = (size_t)n;
    int c = cell_sorted[i];
    int cx, cy, cz;
    pvl_cell_xyz(c, g, cx, cy, cz);
    int e = 0;
    auto put = [&](int j) {
        if (e < maxr) rows[(size_t)i * maxr + e] = j;
        e++;
    };
    for (int j = cs[c]; j < cs[c + 1]; j++)
        if (j != i) put(j);
    for (int q = 0; q < 2 * kPvlDirs; q++) {
        int d;
        bool fwd;
        int B = pvl_neighbour(g, cx, cy, cz, q, d, fwd);
        int s0B = cs[B], mB = cs[B + 1] - s0B;
        int m = cnt[(size_t)q * N + i];
        const uint16_t *pp = perm + (size_t)d * N + s0B;
        for (int k = 0; k < m; k++) put(s0B + (int)pp[fwd ? k : mB - 1 - k]);
    }
    counts[i] = e;
}

// Total candidates (own cells and prefixes) into *out (int64, zeroed first).
__global__ void k_pvl_entries(int n, const int32_t *__restrict__ cs, const int32_t *__restrict__ cell_sorted,
                              const uint16_t *__restrict__ cnt, unsigned long long *out)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    unsigned long long e = 0;
    if (i < n) {
        size_t N = (size_t)n;
        int c = cell_sorted[i];
        e = (unsigned long long)(cs[c + 1] - cs[c] - 1);
        for (int q = 0; q < 2 * kPvlDirs; q++) e += cnt[(size_t)q * N + i];
    }
    for (int off = 32; off > 0; off >>= 1) e += __shfl_xor(e, off, 64);
    if ((threadIdx.x & 63) == 0 && e) atomicAdd(out, e);
}

bool pvl_geometry_ok(const Geom &g)
{
    for (int d = 0; d < 3; d++)
        if (g.reach[d] != 1 || g.nc[d] < 3) return false;
    return true;
}

void launch_pvl_build(int n, const int4 *st, const int32_t *cs, const int32_t *cell_sorted, const Geom &g, float *sv,
                      uint16_t *perm, uint16_t *cnt, hipStream_t s)
{
    if (n <= 0) return;
    k_pvl_sort<<<(n + kBlock - 1) / kBlock, kBlock, 0, s>>>(n, st, cs, cell_sorted, g, sv, perm);
    // threshold r_l |o| in x units (u = L_x / 2^32), widened by 1e-5
    double rl = sqrt(g.rl2) * g.S[0] * (1.0 + 1e-5);
    float thr1 = (float)rl, thr2 = (float)(rl * sqrt(2.0)), thr3 = (float)(rl * sqrt(3.0));
    float wx = (float)(4294967296.0 / g.nc[0]), wy = (float)(4294967296.0 / g.nc[1]) * g.ry,
          wz = (float)(4294967296.0 / g.nc[2]) * g.rz;
    k_pvl_count<<<(n + kBlock - 1) / kBlock, kBlock, 0, s>>>(n, st, g, cs, cell_sorted, sv, cnt, thr1, thr2, thr3, wx,
                                                             wy, wz);
}

template <int NT, bool ISO, bool EN>
static void launch_pvl_t(const ForceArgs &a, const Geom &g, hipStream_t s)
{
    int nb = (a.n + kBlock - 1) / kBlock;
    k_pvl_f32<NT, ISO, EN><<<nb, kBlock, 0, s>>>(a.n, a.stage, a.cell_start, a.cell_sorted, a.pvl_perm, a.pvl_cnt,
                                                 a.tab, g, a.pos, (float *)a.force, a.partials);
}

void launch_pvl_force(const ForceArgs &a, const Geom &g, hipStream_t s)
{
    if (a.n <= 0) return;
    if (g.nt == 1) {
        if (g.iso) a.energy ? launch_pvl_t<1, true, true>(a, g, s) : launch_pvl_t<1, true, false>(a, g, s);
        else a.energy ? launch_pvl_t<1, false, true>(a, g, s) : launch_pvl_t<1, false, false>(a, g, s);
    } else {
        if (g.iso) a.energy ? launch_pvl_t<2, true, true>(a, g, s) : launch_pvl_t<2, true, false>(a, g, s);
        else a.energy ? launch_pvl_t<2, false, true>(a, g, s) : launch_pvl_t<2, false, false>(a, g, s);
    }
}

void launch_pvl_rows(int n, const int32_t *cs, const int32_t *cell_sorted, const Geom &g, const uint16_t *perm,
                     const uint16_t *cnt, int maxr, int32_t *counts, int32_t *rows, hipStream_t s)
{
    if (n <= 0) return;
    k_pvl_rows<<<(n + kBlock - 1) / kBlock, kBlock, 0, s>>>(n, cs, cell_sorted, g, perm, cnt, maxr, counts, rows);
}

void launch_pvl_entries(int n, const int32_t *cs, const int32_t *cell_sorted, const uint16_t *cnt,
                        unsigned long long *out, hipStream_t s)
{
    if (n <= 0) return;
    k_pvl_entries<<<(n + kBlock - 1) / kBlock, kBlock, 0, s>>>(n, cs, cell_sorted, cnt, out);
}

}  // namespace mdlj

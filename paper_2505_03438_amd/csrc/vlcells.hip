// Verlet list cells (Sec. 2.2.1 names the container; Table 1's C08
// traversal): every pair within r_c + skin once, in a list owned by the cell
// of one of its two particles, arranged so that the C08 colouring applies.
//
// C08: base cell b owns the cube of cells b + e, e in {0,1}^3, and the
// fourteen cell pairs of its base step: b with itself and with the other
// seven, and (b+x, b+y), (b+x, b+z), (b+x, b+yz), (b+y, b+z), (b+y, b+xz),
// (b+z, b+xy).  Their directions are the thirteen forward neighbour
// directions, so every pair of neighbouring cells belongs to exactly one
// base step.  A particle of cell P appears as the first cell of a pair in
// four base steps: as b (role 0, partners in eight cells), as b+x (role 1,
// three), as b+y (role 2, two) and as b+z (role 3, one); its list is four
// segments, one per role.  Cubes of base cells whose coordinates share a
// colour (the parity per dimension, and a third colour for the last cell of
// an odd dimension) are disjoint, so one launch per colour processes its
// cubes with no two workgroups writing the same particle: both sides of
// every pair are summed in the workgroup's LDS (64-bit fixed point, integer
// atomics) and added to the forces with plain stores.
//
// Entries are (cube cell index e_Q << 13) | (offset in cell Q), a row of
// maxn (a multiple of 8) per particle, written and read as 16-byte chunks of
// eight: FP32 pair arithmetic on the fixed-point staging, cutoff decisions in
// FP64 inside the guard band, as every other kernel.
#include "entry_chunk.h"
#include "pair.h"

namespace mdlj {

constexpr int kVlcMax = 256;   // particles of a cube staged in LDS (a liquid cube holds ~140)
constexpr int kVlcThreads = 128;

__device__ __forceinline__ int vlc_wrap(int v, int nc) { return v < 0 ? v + nc : (v >= nc ? v - nc : v); }

// Cube cell index e -> offsets (bit 0: x, bit 1: y, bit 2: z).
__device__ __forceinline__ void vlc_e(int e, int &ex, int &ey, int &ez)
{
    ex = e & 1;
    ey = (e >> 1) & 1;
    ez = (e >> 2) & 1;
}

// Role r: the cube cell of the first cell, and its partner cells.
__device__ __forceinline__ int vlc_role_cell(int r) { return r == 0 ? 0 : (r == 1 ? 1 : (r == 2 ? 2 : 4)); }
__device__ __forceinline__ int vlc_role_npart(int r) { return r == 0 ? 8 : (r == 1 ? 3 : (r == 2 ? 2 : 1)); }
__device__ __forceinline__ int vlc_partner(int r, int k)
{
    // role 0: itself, then x, y, z, xy, xz, yz, xyz; role 1 (x): y, z, yz;
    // role 2 (y): z, xz; role 3 (z): xy
    if (r == 0) return k == 0 ? 0 : (k == 1 ? 1 : (k == 2 ? 2 : (k == 3 ? 4 : (k == 4 ? 3 : (k == 5 ? 5 : (k == 6 ? 6 : 7))))));
    if (r == 1) return k == 0 ? 2 : (k == 1 ? 4 : 6);
    if (r == 2) return k == 0 ? 4 : 5;
    return 3;
}

__device__ __forceinline__ void vlc_cell_xyz(int c, const Geom &g, int &cx, int &cy, int &cz)
{
    cx = c % g.nc[0];
    int t = c / g.nc[0];
    cy = t % g.nc[1];
    cz = t / g.nc[1];
}

__device__ __forceinline__ int vlc_cell(const Geom &g, int x, int y, int z)
{
    return (vlc_wrap(z, g.nc[2]) * g.nc[1] + vlc_wrap(y, g.nc[1])) * g.nc[0] + vlc_wrap(x, g.nc[0]);
}

// Build: thread per particle i (cell P).  For each role r, the base cell is
// P minus the role cell's offset; the partners are tested against r_c + skin
// (FP64 inside the guard band); entries append in role order to the
// particle's row, eight at a time, segment ends in seg[r][i].
template <bool ISO>
__global__ __launch_bounds__(kBlock) void k_vlc_build(int n, const int4 *__restrict__ st,
                                                      const int32_t *__restrict__ cs,
                                                      const int32_t *__restrict__ cell_sorted,
                                                      const double *__restrict__ pos, Geom g,
                                                      uint16_t *__restrict__ nbr, uint16_t *__restrict__ seg,
                                                      int32_t *__restrict__ cnt, int maxn,
                                                      int32_t *__restrict__ flags)
{
    int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    size_t N = (size_t)n;
    int4 pi = st[i];
    int px, py, pz;
    vlc_cell_xyz(cell_sorted[i], g, px, py, pz);
    int c = 0;
    EntryChunk ck;
    uint4 *row = (uint4 *)nbr + (size_t)i * (maxn >> 3);
    for (int r = 0; r < 4; r++) {
        int ex, ey, ez;
        vlc_e(vlc_role_cell(r), ex, ey, ez);
        int bx = px - ex, by = py - ey, bz = pz - ez;  // base cell of this role
        for (int k = 0; k < vlc_role_npart(r); k++) {
            int eq = vlc_partner(r, k);
            int qx, qy, qz;
            vlc_e(eq, qx, qy, qz);
            int Q = vlc_cell(g, bx + qx, by + qy, bz + qz);
            int jb = cs[Q], je = cs[Q + 1];
            for (int j = (r == 0 && k == 0) ? i + 1 : jb; j < je; j++) {
                float dx, dy, dz;
                staged_delta<ISO>(pi, st[j], g, dx, dy, dz);
                float r2 = dx * dx + dy * dy + dz * dz;
                if (within(r2, g.rl2_lo, g.rl2_hi, g.rl2, pos, n, i, j, g)) {
                    ck.push((uint32_t)((eq << 13) | (j - jb)));
                    c++;
                    if ((c & 7) == 0 && c <= maxn) row[(c >> 3) - 1] = ck.word();
                }
            }
        }
        seg[(size_t)r * N + i] = (uint16_t)(c < maxn ? c : maxn);
    }
    if ((c & 7) != 0 && c < maxn) {
        for (int e = c & 7; e < 8; e++) ck.push(0u);
        row[c >> 3] = ck.word();
    }
    if (c > maxn) atomicOr(&flags[0], (int)MD_FLAG_LIST_OVERFLOW);
    atomicMax(&flags[2], c);
    cnt[i] = c < maxn ? c : maxn;
}

// Base cells of one colour: per dimension the coordinates with parity k (the
// last coordinate of an odd dimension alone has colour 2).
__device__ __forceinline__ int vlc_colour_coord(int k, int idx, int nc)
{
    if (k == 2) return nc - 1;
    return k + 2 * idx;
}

struct VlcColour {
    int k[3];      // colour per dimension
    int cnt[3];    // base cells per dimension of that colour
};

// Force pass of one colour: workgroup per base cell (cube).  The cube's
// particles (up to kVlcMax) are staged in LDS with fixed-point force
// accumulators; a larger cube (never at liquid densities) takes its
// positions from global memory and adds both sides with global atomics.
template <int NT, bool ISO, bool ENERGY>
__global__ __launch_bounds__(kVlcThreads) void k_vlc_f32(VlcColour col, int n, const int4 *__restrict__ st,
                                                         const int32_t *__restrict__ cs,
                                                         const uint16_t *__restrict__ nbr, int ld,
                                                         const uint16_t *__restrict__ seg,
                                                         const PairTab *__restrict__ tabp, Geom g,
                                                         const double *__restrict__ pos, float *__restrict__ F,
                                                         double *__restrict__ cube_part)
{
    __shared__ int4 wp[kVlcMax];
    __shared__ unsigned long long ax[kVlcMax], ay[kVlcMax], az[kVlcMax];
    __shared__ int cst[8], base[9];
    __shared__ int tq[kVlcMax + 1], te0[kVlcMax], te1[kVlcMax];  // tasks per role particle, segments
    __shared__ int wsum[2 * kVlcThreads / 64];                     // wavefront totals of the task scan
    __shared__ double sh[4 * kVlcThreads / 64];
    int b = blockIdx.x;
    int ix = b % col.cnt[0], t = b / col.cnt[0];
    int iy = t % col.cnt[1], iz = t / col.cnt[1];
    int bx = vlc_colour_coord(col.k[0], ix, g.nc[0]), by = vlc_colour_coord(col.k[1], iy, g.nc[1]),
        bz = vlc_colour_coord(col.k[2], iz, g.nc[2]);
    if (threadIdx.x < 8) {
        int ex, ey, ez;
        vlc_e(threadIdx.x, ex, ey, ez);
        int c = vlc_cell(g, bx + ex, by + ey, bz + ez);
        cst[threadIdx.x] = cs[c];
        base[threadIdx.x + 1] = cs[c + 1] - cs[c];  // counts for now
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        base[0] = 0;
        for (int e = 0; e < 8; e++) base[e + 1] += base[e];
    }
    __syncthreads();
    const int M = base[8];
    const bool lds = M <= kVlcMax;
    TabF<NT> tb;
    tb.load(tabp);
    size_t N = (size_t)n;
    if (lds) {
        int e = 0;
        for (int p = threadIdx.x; p < M; p += kVlcThreads) {
            while (base[e + 1] <= p) e++;
            wp[p] = st[cst[e] + (p - base[e])];
            ax[p] = ay[p] = az[p] = 0ull;
        }
    }
    __syncthreads();
    float eu = 0.f, ew = 0.f;
    int np = 0;
    // particles of the four role cells (cube cells 0, 1, 2, 4)
    int nr0 = base[1] - base[0], nr1 = base[2] - base[1], nr2 = base[3] - base[2], nr3 = base[5] - base[4];
    int Mr = nr0 + nr1 + nr2 + nr3;
    auto role_of = [&](int p, int &r, int &off) {
        if (p < nr0) {
            r = 0;
            off = p;
        } else if (p < nr0 + nr1) {
            r = 1;
            off = p - nr0;
        } else if (p < nr0 + nr1 + nr2) {
            r = 2;
            off = p - nr0 - nr1;
        } else {
            r = 3;
            off = p - nr0 - nr1 - nr2;
        }
    };
    // chunk c of particle i's row (entries 8c .. 8c + 7, one 16-byte load),
    // its entries in [e0, e1) taken: the j sides go to the accumulators, the
    // i side is returned in f
    const uint4 *rows = (const uint4 *)nbr;
    const size_t ld8 = (size_t)(ld >> 3);
    auto walk = [&](int i, const int4 &pi, int c, int e0, int e1, float &fx, float &fy, float &fz) {
        const uint4 chunk = rows[(size_t)i * ld8 + c];
#pragma unroll
        for (int u = 0; u < 8; u++) {
            const int q = 8 * c + u;
            if (q < e0 || q >= e1) continue;
            uint32_t ent = chunk_entry(chunk, u);
            int eq = (int)(ent >> 13), oq = (int)(ent & 8191u);
            int lj = base[eq] + oq, j = cst[eq] + oq;
            int4 pj = lds ? wp[lj] : st[j];
            float dx, dy, dz;
            staged_delta<ISO>(pi, pj, g, dx, dy, dz);
            float r2 = dx * dx + dy * dy + dz * dz;
            int ab = NT == 1 ? 0 : pi.w * NT + pj.w;
            bool in = within(r2, tb.pick(tb.lo, ab), tb.pick(tb.hi, ab), tb.pickd(tb.rc2, ab), pos, n, i, j, g);
            float phi = lj_f32<NT, ENERGY>(r2, ab, in, tb, eu, ew, np);
            float px = phi * dx, py = phi * dy, pz = phi * dz;
            fx += px;
            fy += py;
            fz += pz;
            if (in) {
                if (lds) {
                    atomicAdd(&ax[lj], to_fix(-px));
                    atomicAdd(&ay[lj], to_fix(-py));
                    atomicAdd(&az[lj], to_fix(-pz));
                } else {
                    atomicAdd(&F[j], -px);
                    atomicAdd(&F[N + j], -py);
                    atomicAdd(&F[2 * N + j], -pz);
                }
            }
        }
    };
    if (lds) {
        // the role particles' segments dealt to the threads in tasks of one
        // 16-byte chunk of a row (the chunks a segment touches): the long
        // segments (the base cell's particles pair with eight cells, the
        // others with fewer) take several threads each, so no thread waits
        // on the longest one of its wavefront
        // thread t takes role particles t and t + kVlcThreads (Mr <= kVlcMax
        // = 2 kVlcThreads); the prefix of their task counts is a scan within
        // each wavefront (shuffles) plus the wavefronts' totals
        static_assert(kVlcMax == 2 * kVlcThreads, "two role particles per thread");
        int cnt2[2];
        for (int h = 0; h < 2; h++) {
            const int p = threadIdx.x + h * kVlcThreads;
            cnt2[h] = 0;
            if (p < Mr) {
                int r, off;
                role_of(p, r, off);
                int i = cst[vlc_role_cell(r)] + off;
                int e0 = r == 0 ? 0 : seg[(size_t)(r - 1) * N + i], e1 = seg[(size_t)r * N + i];
                te0[p] = e0;
                te1[p] = e1;
                cnt2[h] = e1 > e0 ? ((e1 + 7) >> 3) - (e0 >> 3) : 0;
            }
        }
        const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
        constexpr int kWaves = kVlcThreads / 64;
        int inc[2];
        for (int h = 0; h < 2; h++) {
            int x = cnt2[h];
            for (int o = 1; o < 64; o <<= 1) {
                const int y = __shfl_up(x, o, 64);
                if (lane >= o) x += y;
            }
            inc[h] = x;
            if (lane == 63) wsum[h * kWaves + wave] = x;
        }
        __syncthreads();
        for (int h = 0; h < 2; h++) {
            int before = 0;  // the totals of the wavefronts (and halves) before this one
            for (int k = 0; k < h * kWaves + wave; k++) before += wsum[k];
            const int p = threadIdx.x + h * kVlcThreads;
            tq[p + 1] = before + inc[h];  // inclusive: tq[p + 1] counts the tasks of particles 0 .. p
        }
        if (threadIdx.x == 0) tq[0] = 0;
        __syncthreads();
        const int T = tq[Mr];
        for (int task = threadIdx.x; task < T; task += kVlcThreads) {
            int lo = 0, hi = Mr;  // the role particle lo with tq[lo] <= task < tq[lo + 1]
            while (hi - lo > 1) {
                int mid = (lo + hi) >> 1;
                if (tq[mid] <= task)
                    lo = mid;
                else
                    hi = mid;
            }
            int r, off;
            role_of(lo, r, off);
            int ep = vlc_role_cell(r);
            int li = base[ep] + off, i = cst[ep] + off;
            const int c = (te0[lo] >> 3) + (task - tq[lo]);
            float fx = 0.f, fy = 0.f, fz = 0.f;
            walk(i, wp[li], c, te0[lo], te1[lo], fx, fy, fz);
            atomicAdd(&ax[li], to_fix(fx));
            atomicAdd(&ay[li], to_fix(fy));
            atomicAdd(&az[li], to_fix(fz));
        }
    } else {
        for (int p = threadIdx.x; p < Mr; p += kVlcThreads) {
            int r, off;
            role_of(p, r, off);
            int ep = vlc_role_cell(r);
            int i = cst[ep] + off;
            int4 pi = st[i];
            int e0 = r == 0 ? 0 : seg[(size_t)(r - 1) * N + i], e1 = seg[(size_t)r * N + i];
            float fx = 0.f, fy = 0.f, fz = 0.f;
            if (e1 > e0)
                for (int c = e0 >> 3; c <= (e1 - 1) >> 3; c++) walk(i, pi, c, e0, e1, fx, fy, fz);
            atomicAdd(&F[i], fx);
            atomicAdd(&F[N + i], fy);
            atomicAdd(&F[2 * N + i], fz);
        }
    }
    __syncthreads();
    if (lds) {
        // the cube is this colour's alone: plain read-modify-write
        int e = 0;
        for (int p = threadIdx.x; p < M; p += kVlcThreads) {
            while (base[e + 1] <= p) e++;
            int j = cst[e] + (p - base[e]);
            if (ax[p]) F[j] += from_fix(ax[p]);
            if (ay[p]) F[N + j] += from_fix(ay[p]);
            if (az[p]) F[2 * N + j] += from_fix(az[p]);
        }
    }
    if (ENERGY) {
        double v[4] = {(double)eu, (double)ew, (double)np, 0.0};
        block_sum4_n<kVlcThreads>(v, sh);
        if (threadIdx.x == 0) {
            int bc = (bz * g.nc[1] + by) * g.nc[0] + bx;
            for (int k = 0; k < 4; k++) cube_part[(size_t)bc * 4 + k] = v[k];
        }
    }
}

// ------------------------------------------------------------------ linked cells, C08 traversal

// Linked cells traversed with the C08 colouring (Table 1), no lists: the
// base step of base cell b covers the fourteen cell pairs of the cube (see
// the top of this file), so a colour's cubes run concurrently with both sides
// of every pair summed in the workgroup's LDS.  The work of a cube is spread
// over its threads as tasks (cell pair, particle of the pair's first cell):
// a task tests the particles of the pair's second cell (those after it when
// the base cell pairs with itself) 32 at a time against the largest upper
// edge of the cutoffs' guard bands, then evaluates the pairs that pass
// (guard-band pairs decided from the FP64 positions); the i side is summed
// in registers and added once per task, the j side goes to the LDS
// accumulators.  Cell pair p: first cube cell A, second B (the partners of
// the four roles in order).
constexpr int kC08Pairs = 14;

__device__ __forceinline__ void c08_pair(int p, int &A, int &B)
{
    if (p < 8) {
        A = 0;
        B = vlc_partner(0, p);
    } else if (p < 11) {
        A = 1;
        B = vlc_partner(1, p - 8);
    } else if (p < 13) {
        A = 2;
        B = vlc_partner(2, p - 11);
    } else {
        A = 4;
        B = vlc_partner(3, 0);
    }
}

template <int NT, bool ISO, bool ENERGY>
__global__ __launch_bounds__(kVlcThreads) void k_lc08_f32(VlcColour col, int n, const int4 *__restrict__ st,
                                                          const int32_t *__restrict__ cs,
                                                          const PairTab *__restrict__ tabp, Geom g,
                                                          const double *__restrict__ pos, float *__restrict__ F,
                                                          double *__restrict__ cube_part)
{
    __shared__ int4 wp[kVlcMax];
    __shared__ unsigned long long ax[kVlcMax], ay[kVlcMax], az[kVlcMax];
    __shared__ int cst[8], base[9], tpre[kC08Pairs + 1];
    __shared__ double sh[4 * kVlcThreads / 64];
    int b = blockIdx.x;
    int ix = b % col.cnt[0], t = b / col.cnt[0];
    int iy = t % col.cnt[1], iz = t / col.cnt[1];
    int bx = vlc_colour_coord(col.k[0], ix, g.nc[0]), by = vlc_colour_coord(col.k[1], iy, g.nc[1]),
        bz = vlc_colour_coord(col.k[2], iz, g.nc[2]);
    if (threadIdx.x < 8) {
        int ex, ey, ez;
        vlc_e(threadIdx.x, ex, ey, ez);
        int c = vlc_cell(g, bx + ex, by + ey, bz + ez);
        cst[threadIdx.x] = cs[c];
        base[threadIdx.x + 1] = cs[c + 1] - cs[c];  // counts for now
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        base[0] = 0;
        for (int e = 0; e < 8; e++) base[e + 1] += base[e];
        tpre[0] = 0;
        for (int p = 0; p < kC08Pairs; p++) {
            int A, B;
            c08_pair(p, A, B);
            tpre[p + 1] = tpre[p] + (base[A + 1] - base[A]);
        }
    }
    __syncthreads();
    const int M = base[8];
    const bool lds = M <= kVlcMax;
    TabF<NT> tb;
    tb.load(tabp);
    float hmax = tb.hi[0];
    for (int k = 1; k < NT * NT; k++) hmax = fmaxf(hmax, tb.hi[k]);
    size_t N = (size_t)n;
    if (lds) {
        int e = 0;
        for (int p = threadIdx.x; p < M; p += kVlcThreads) {
            while (base[e + 1] <= p) e++;
            wp[p] = st[cst[e] + (p - base[e])];
            ax[p] = ay[p] = az[p] = 0ull;
        }
    }
    __syncthreads();
    float eu = 0.f, ew = 0.f;
    int np = 0;
    const int T = tpre[kC08Pairs];
    for (int task = threadIdx.x; task < T; task += kVlcThreads) {
        int p = 0;
        while (tpre[p + 1] <= task) p++;
        int A, B;
        c08_pair(p, A, B);
        int a = task - tpre[p];
        int li = base[A] + a, i = cst[A] + a;
        int4 pi = lds ? wp[li] : st[i];
        int jb = A == B ? li + 1 : base[B], je = base[B + 1];  // candidates, cube positions
        int joff = cst[B] - base[B];                          // cube position -> particle index
        float fx = 0.f, fy = 0.f, fz = 0.f;
        for (int q0 = jb; q0 < je; q0 += 32) {
            int m = min(32, je - q0);
            uint32_t mask = 0;
            for (int u = 0; u < m; u++) {
                int4 pj = lds ? wp[q0 + u] : st[q0 + u + joff];
                float dx, dy, dz;
                staged_delta<ISO>(pi, pj, g, dx, dy, dz);
                float r2 = dx * dx + dy * dy + dz * dz;
                mask |= (r2 < hmax ? 1u : 0u) << u;
            }
            while (mask) {
                int u = __builtin_ctz(mask);
                mask &= mask - 1;
                int lj = q0 + u, j = lj + joff;
                int4 pj = lds ? wp[lj] : st[j];
                float dx, dy, dz;
                staged_delta<ISO>(pi, pj, g, dx, dy, dz);
                float r2 = dx * dx + dy * dy + dz * dz;
                int ab = NT == 1 ? 0 : pi.w * NT + pj.w;
                bool in = within(r2, tb.pick(tb.lo, ab), tb.pick(tb.hi, ab), tb.pickd(tb.rc2, ab), pos, n, i, j, g);
                if (!in) continue;
                float phi = lj_f32<NT, ENERGY>(r2, ab, true, tb, eu, ew, np);
                float px = phi * dx, py = phi * dy, pz = phi * dz;
                fx += px;
                fy += py;
                fz += pz;
                if (lds) {
                    atomicAdd(&ax[lj], to_fix(-px));
                    atomicAdd(&ay[lj], to_fix(-py));
                    atomicAdd(&az[lj], to_fix(-pz));
                } else {
                    atomicAdd(&F[j], -px);
                    atomicAdd(&F[N + j], -py);
                    atomicAdd(&F[2 * N + j], -pz);
                }
            }
        }
        if (lds) {
            atomicAdd(&ax[li], to_fix(fx));
            atomicAdd(&ay[li], to_fix(fy));
            atomicAdd(&az[li], to_fix(fz));
        } else {
            atomicAdd(&F[i], fx);
            atomicAdd(&F[N + i], fy);
            atomicAdd(&F[2 * N + i], fz);
        }
    }
    __syncthreads();
    if (lds) {
        // the cube is this colour's alone: plain read-modify-write
        int e = 0;
        for (int p = threadIdx.x; p < M; p += kVlcThreads) {
            while (base[e + 1] <= p) e++;
            int j = cst[e] + (p - base[e]);
            if (ax[p]) F[j] += from_fix(ax[p]);
            if (ay[p]) F[N + j] += from_fix(ay[p]);
            if (az[p]) F[2 * N + j] += from_fix(az[p]);
        }
    }
    if (ENERGY) {
        double v[4] = {(double)eu, (double)ew, (double)np, 0.0};
        block_sum4_n<kVlcThreads>(v, sh);
        if (threadIdx.x == 0) {
            int bc = (bz * g.nc[1] + by) * g.nc[0] + bx;
            for (int k = 0; k < 4; k++) cube_part[(size_t)bc * 4 + k] = v[k];
        }
    }
}

// Fixed-order sum of the per-cube partials into nb slots of partials.
__global__ void k_vlc_fold(const double *__restrict__ cube_part, int ncell, int nb, double *__restrict__ partials)
{
    int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= nb) return;
    int per = (ncell + nb - 1) / nb;
    double v[3] = {0.0, 0.0, 0.0};
    for (int c = s * per; c < min(ncell, (s + 1) * per); c++)
        for (int k = 0; k < 3; k++) v[k] += cube_part[(size_t)c * 4 + k];
    for (int k = 0; k < 3; k++) partials[s * 4 + k] = v[k];
    partials[s * 4 + 3] = 0.0;
}

// The lists as global indices (each pair once, in the row of the particle
// whose cell comes first in its base step), for inspection.
__global__ void k_vlc_rows(int n, const int32_t *__restrict__ cs, const int32_t *__restrict__ cell_sorted, Geom g,
                           const uint16_t *__restrict__ nbr, int ld, const uint16_t *__restrict__ seg, int maxr,
                           int32_t *__restrict__ counts, int32_t *__restrict__ rows)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    size_t N = (size_t)n;
    int px, py, pz;
    vlc_cell_xyz(cell_sorted[i], g, px, py, pz);
    int e = 0, q0 = 0;
    for (int r = 0; r < 4; r++) {
        int ex, ey, ez;
        vlc_e(vlc_role_cell(r), ex, ey, ez);
        int q1 = seg[(size_t)r * N + i];
        for (int q = q0; q < q1; q++) {
            uint32_t ent = nbr[(size_t)i * ld + q];
            int qx, qy, qz;
            vlc_e((int)(ent >> 13), qx, qy, qz);
            int Q = vlc_cell(g, px - ex + qx, py - ey + qy, pz - ez + qz);
            if (e < maxr) rows[(size_t)i * maxr + e] = cs[Q] + (int)(ent & 8191u);
            e++;
        }
        q0 = q1;
    }
    counts[i] = e;
}

int vlc_colours(const Geom &g, VlcColour *out)
{
    int m = 0;
    int kd[3];
    auto ncol = [&](int d) { return g.nc[d] % 2 ? 3 : 2; };
    for (kd[2] = 0; kd[2] < ncol(2); kd[2]++)
        for (kd[1] = 0; kd[1] < ncol(1); kd[1]++)
            for (kd[0] = 0; kd[0] < ncol(0); kd[0]++) {
                VlcColour c;
                for (int d = 0; d < 3; d++) {
                    c.k[d] = kd[d];
                    int nc = g.nc[d];
                    if (kd[d] == 2) c.cnt[d] = 1;
                    else if (nc % 2 == 0) c.cnt[d] = nc / 2;
                    else c.cnt[d] = (nc - 1 - kd[d] + 1) / 2;  // coordinates kd, kd+2, .. <= nc - 2
                }
                out[m++] = c;
            }
    return m;
}

void launch_vlc_build(int n, const int4 *st, const int32_t *cs, const int32_t *cell_sorted, const double *pos,
                      const Geom &g, uint16_t *nbr, uint16_t *seg, int32_t *cnt, int maxn, int32_t *flags,
                      hipStream_t s)
{
    if (n <= 0) return;
    int nb = (n + kBlock - 1) / kBlock;
    if (g.iso)
        k_vlc_build<true><<<nb, kBlock, 0, s>>>(n, st, cs, cell_sorted, pos, g, nbr, seg, cnt, maxn, flags);
    else
        k_vlc_build<false><<<nb, kBlock, 0, s>>>(n, st, cs, cell_sorted, pos, g, nbr, seg, cnt, maxn, flags);
}

int vlc_force_blocks(const Geom &g) { return std::min(g.ncell, 1024); }

template <int NT, bool ISO, bool EN>
static void launch_vlc_t(const ForceArgs &a, const Geom &g, hipStream_t s)
{
    VlcColour cols[27];
    int m = vlc_colours(g, cols);
    for (int k = 0; k < m; k++) {
        int grid = cols[k].cnt[0] * cols[k].cnt[1] * cols[k].cnt[2];
        if (grid <= 0) continue;
        k_vlc_f32<NT, ISO, EN><<<grid, kVlcThreads, 0, s>>>(cols[k], a.n, a.stage, a.cell_start, a.vlc_nbr,
                                                            a.vlc_ld, a.vlc_seg, a.tab, g, a.pos, (float *)a.force,
                                                            a.vlc_part);
    }
    if (EN) {
        int nb = vlc_force_blocks(g);
        k_vlc_fold<<<(nb + kBlock - 1) / kBlock, kBlock, 0, s>>>(a.vlc_part, g.ncell, nb, a.partials);
    }
}

void launch_vlc_force(const ForceArgs &a, const Geom &g, hipStream_t s)
{
    if (a.n <= 0) return;
    if (g.nt == 1) {
        if (g.iso) a.energy ? launch_vlc_t<1, true, true>(a, g, s) : launch_vlc_t<1, true, false>(a, g, s);
        else a.energy ? launch_vlc_t<1, false, true>(a, g, s) : launch_vlc_t<1, false, false>(a, g, s);
    } else {
        if (g.iso) a.energy ? launch_vlc_t<2, true, true>(a, g, s) : launch_vlc_t<2, true, false>(a, g, s);
        else a.energy ? launch_vlc_t<2, false, true>(a, g, s) : launch_vlc_t<2, false, false>(a, g, s);
    }
}

template <int NT, bool ISO, bool EN>
static void launch_lc08_t(const ForceArgs &a, const Geom &g, hipStream_t s)
{
    VlcColour cols[27];
    int m = vlc_colours(g, cols);
    for (int k = 0; k < m; k++) {
        int grid = cols[k].cnt[0] * cols[k].cnt[1] * cols[k].cnt[2];
        if (grid <= 0) continue;
        k_lc08_f32<NT, ISO, EN><<<grid, kVlcThreads, 0, s>>>(cols[k], a.n, a.stage, a.cell_start, a.tab, g, a.pos,
                                                             (float *)a.force, a.vlc_part);
    }
    if (EN) {
        int nb = vlc_force_blocks(g);
        k_vlc_fold<<<(nb + kBlock - 1) / kBlock, kBlock, 0, s>>>(a.vlc_part, g.ncell, nb, a.partials);
    }
}

void launch_lc08_force(const ForceArgs &a, const Geom &g, hipStream_t s)
{
    if (a.n <= 0) return;
    if (g.nt == 1) {
        if (g.iso) a.energy ? launch_lc08_t<1, true, true>(a, g, s) : launch_lc08_t<1, true, false>(a, g, s);
        else a.energy ? launch_lc08_t<1, false, true>(a, g, s) : launch_lc08_t<1, false, false>(a, g, s);
    } else {
        if (g.iso) a.energy ? launch_lc08_t<2, true, true>(a, g, s) : launch_lc08_t<2, true, false>(a, g, s);
        else a.energy ? launch_lc08_t<2, false, true>(a, g, s) : launch_lc08_t<2, false, false>(a, g, s);
    }
}

void launch_vlc_rows(int n, const int32_t *cs, const int32_t *cell_sorted, const Geom &g, const uint16_t *nbr,
                     int ld, const uint16_t *seg, int maxr, int32_t *counts, int32_t *rows, hipStream_t s)
{
    if (n <= 0) return;
    k_vlc_rows<<<(n + kBlock - 1) / kBlock, kBlock, 0, s>>>(n, cs, cell_sorted, g, nbr, ld, seg, maxr, counts, rows);
}

}  // namespace mdlj

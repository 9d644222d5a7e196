// Pair traversals over LDS windows (FP32, gather-only).
//
// Particles are in linked-cell order (cells x-fastest, within a cell by id).
// A block is a run of consecutive cells of one x-row holding at most 256
// particles (one workgroup, one thread per particle).  Its window is the
// union of its cells' stencils: for every neighbouring (y, z) row the
// contiguous cell columns [x_first - 1, x_last + 1] (two particle ranges, or
// pieces, when they wrap around the periodic box).  The block packer bounds
// every window to the LDS tile.  A workgroup stages the window once, then:
//   - linked cells: each thread scans its own stencil cells inside the
//     window (the GPU analogue of the C01 traversal: no write conflicts);
//   - Verlet lists: each thread walks its list of 16-bit window positions,
//     stored in chunks of eight (one 16-byte load per chunk, the next chunk
//     in flight while the current one is computed).
// Blocks of neighbouring cells share most of their windows, so the blocks
// are dealt to the eight XCDs in contiguous chunks (workgroup w runs on XCD
// w mod 8) to keep the shared window data in one L2.
#include "pair.h"

namespace mdlj {

constexpr int kWinMax = 3072;    // LDS window capacity (particles)
constexpr int kBlkCells = 32;    // maximum cells of a block along x
constexpr int kMaxRows = 9;      // stencil rows of a reach-1 window (3 x 3)
constexpr int kMaxCols = kBlkCells + 2;  // window columns of a reach-1 window
constexpr int kLoadPer = (kWinMax + 255) / 256;
constexpr int kWinGrid = 2048;   // persistent workgroups (multiple of 8)
constexpr int kHalfRows = 5;     // rows of a half window (four forward rows, then the own row)
constexpr int kHalfOwn = 4;      // the own row of a half window
constexpr int kWinMaxHalf = 2048;  // LDS capacity of a half window (positions and j-side forces)

using Ofs = int (*)[kMaxOfs];
using COfs = const int (*)[kMaxOfs];

// LDS entry of a window particle: its staged fixed-point coordinates, and its
// type when there are two.  Twelve bytes for one type keep four workgroups'
// windows (4 x 36 KB) within a compute unit's LDS.
template <int NT>
struct WinEntry {
    int x, y, z, w;
    __device__ __forceinline__ void set(const int4 &a)
    {
        x = a.x;
        y = a.y;
        z = a.z;
        w = a.w;
    }
    __device__ __forceinline__ int4 get() const { return make_int4(x, y, z, w); }
};
template <>
struct WinEntry<1> {
    int x, y, z;
    __device__ __forceinline__ void set(const int4 &a)
    {
        x = a.x;
        y = a.y;
        z = a.z;
    }
    __device__ __forceinline__ int4 get() const { return make_int4(x, y, z, 0); }
};

// ------------------------------------------------------------------ windows

// Columns [lo, hi] of the window of a block spanning xa..xb (hi < lo when it
// wraps); returns the number of columns.
__device__ __forceinline__ int window_columns(const Geom &g, int xa, int xb, int &lo, int &hi)
{
    int nx = g.nc[0];
    if (xb - xa + 3 >= nx) {
        lo = 0;
        hi = nx - 1;
        return nx;
    }
    lo = xa == 0 ? nx - 1 : xa - 1;
    hi = xb + 1 == nx ? 0 : xb + 1;
    return xb - xa + 3;
}

// Linear id of the x = 0 cell of stencil row rr around row (cy, cz).  A full
// window holds the 3 x 3 stencil rows (fewer when a small periodic grid
// repeats a row); a half window, for the traversals with Newton's third law,
// holds the four forward rows (z + 1 with y - 1, y, y + 1, then z with y + 1)
// and the own row last.  With the forward columns of the own row this is half
// of the 26 neighbour cells: every pair of distinct cells is seen from exactly
// one of its two cells (this needs at least three cells in every dimension).
template <bool HALF>
__device__ __forceinline__ int row_cell_of(const Geom &g, COfs so, int cy, int cz, int rr)
{
    int zz, yy;
    if (HALF) {
        int dz = rr < 3 ? 1 : 0;
        int dy = rr < 3 ? rr - 1 : (rr == 3 ? 1 : 0);
        zz = cz + dz;
        zz = zz >= g.nc[2] ? zz - g.nc[2] : zz;
        yy = cy + dy;
        yy = yy < 0 ? yy + g.nc[1] : (yy >= g.nc[1] ? yy - g.nc[1] : yy);
    } else {
        int a = rr / g.nofs[1], b = rr - a * g.nofs[1];
        zz = cz + so[2][a];
        zz = zz >= g.nc[2] ? zz - g.nc[2] : zz;
        yy = cy + so[1][b];
        yy = yy >= g.nc[1] ? yy - g.nc[1] : yy;
    }
    return (zz * g.nc[1] + yy) * g.nc[0];
}

// Window layout in LDS.  Column m of stencil row rr is cell column
// (lo + m) mod nx; its particles occupy window positions
// [col[rr][m], col[rr][m + 1]).  Piece k (two per row, the second empty
// unless the columns wrap) holds particles [pc_start[k], ...) at window
// positions [pc_win[k], pc_win[k + 1]).
struct Window {
    int nrow, ncols, lo, self_row, W;
    int pc_start[2 * kMaxRows];
    int pc_win[2 * kMaxRows + 1];
    int col[kMaxRows][kMaxCols + 1];
};

// Lay out the (full or half) window of the block with cells c0..c1 (one
// row).  All threads take part; ends with a barrier.
template <bool HALF>
__device__ void make_window(const Geom &g, COfs so, const int32_t *__restrict__ cs, int c0, int c1, Window &w)
{
    int nx = g.nc[0];
    int xa = c0 % nx, xb = c1 % nx;
    int r = c0 / nx;
    int cy = r % g.nc[1], cz = r / g.nc[1];
    int lo, hi;
    int ncols = window_columns(g, xa, xb, lo, hi);
    int nrow = HALF ? kHalfRows : g.nofs[1] * g.nofs[2];
    int t = threadIdx.x;
    bool wrap = hi < lo;
    int x1a = wrap ? nx - 1 : hi;
    if (t < nrow) {
        int rb = row_cell_of<HALF>(g, so, cy, cz, t);
        int s0 = cs[rb + lo], e0 = cs[rb + x1a + 1];
        int s1 = cs[rb], e1 = wrap ? cs[rb + hi + 1] : s1;
        w.pc_start[2 * t] = s0;
        w.pc_start[2 * t + 1] = s1;
        w.pc_win[2 * t] = e0 - s0;  // lengths for now
        w.pc_win[2 * t + 1] = e1 - s1;
    }
    __syncthreads();
    if (t == 0) {
        int pos = 0;
        for (int k = 0; k < 2 * nrow; k++) {
            int len = w.pc_win[k];
            w.pc_win[k] = pos;
            pos += len;
        }
        w.pc_win[2 * nrow] = pos;
        w.W = pos;
        w.nrow = nrow;
        w.ncols = ncols;
        w.lo = lo;
        if (HALF) {
            w.self_row = kHalfOwn;
        } else {
            int a0 = 0, b0 = 0;
            for (int a = 0; a < g.nofs[2]; a++)
                if (so[2][a] == 0) a0 = a;
            for (int b = 0; b < g.nofs[1]; b++)
                if (so[1][b] == 0) b0 = b;
            w.self_row = a0 * g.nofs[1] + b0;
        }
    }
    __syncthreads();
    int ncol0 = x1a - lo + 1;  // columns in the first piece
    for (int e = t; e < nrow * (ncols + 1); e += blockDim.x) {
        int rr = e / (ncols + 1), m = e - rr * (ncols + 1);
        int v;
        if (m == ncols) {
            v = w.pc_win[2 * rr + 2];
        } else {
            int rb = row_cell_of<HALF>(g, so, cy, cz, rr);
            if (m < ncol0)
                v = w.pc_win[2 * rr] + cs[rb + lo + m] - w.pc_start[2 * rr];
            else
                v = w.pc_win[2 * rr + 1] + cs[rb + m - ncol0] - w.pc_start[2 * rr + 1];
        }
        w.col[rr][m] = v;
    }
    __syncthreads();
}

// Piece holding window position p, searching forward from piece k.
__device__ __forceinline__ int piece_from(const Window &w, int k, int p)
{
    while (k + 1 < 2 * w.nrow && w.pc_win[k + 1] <= p) k++;
    return k;
}

// Global particle index of window position p (rare paths).
__device__ __forceinline__ int window_global(const Window &w, int p)
{
    int k = piece_from(w, 0, p);
    return w.pc_start[k] + (p - w.pc_win[k]);
}

// Stage the window into LDS, four loads in flight per thread (named
// registers: an array here would be placed in scratch memory).
template <int NT>
__device__ __forceinline__ void load_window(const Window &w, const int4 *__restrict__ st, WinEntry<NT> *lds)
{
    int W = w.W;
    int k = 0;
    for (int p0 = threadIdx.x; p0 < W; p0 += 1024) {
        int p1 = p0 + 256, p2 = p0 + 512, p3 = p0 + 768;
        int4 a0, a1 = a0, a2 = a0, a3 = a0;
        k = piece_from(w, k, p0);
        a0 = st[w.pc_start[k] + (p0 - w.pc_win[k])];
        if (p1 < W) {
            k = piece_from(w, k, p1);
            a1 = st[w.pc_start[k] + (p1 - w.pc_win[k])];
        }
        if (p2 < W) {
            k = piece_from(w, k, p2);
            a2 = st[w.pc_start[k] + (p2 - w.pc_win[k])];
        }
        if (p3 < W) {
            k = piece_from(w, k, p3);
            a3 = st[w.pc_start[k] + (p3 - w.pc_win[k])];
        }
        lds[p0].set(a0);
        if (p1 < W) lds[p1].set(a1);
        if (p2 < W) lds[p2].set(a2);
        if (p3 < W) lds[p3].set(a3);
    }
}

// XCD-aware block order: workgroup w runs on XCD w % 8; each XCD takes a
// contiguous chunk of blocks.
struct BlockIter {
    int blk, end, stride;
    __device__ BlockIter(int nblk)
    {
        int chunk = (nblk + 7) / 8;
        int xcd = blockIdx.x & 7;
        stride = gridDim.x >> 3;
        blk = xcd * chunk + (blockIdx.x >> 3);
        end = min(nblk, (xcd + 1) * chunk);
    }
};

// Window range of the cell column x + (e-th x offset) in stencil row rr.
__device__ __forceinline__ void stencil_range(const Geom &g, COfs so, const Window &w, int x, int rr, int e, int &b,
                                              int &en)
{
    int nx = g.nc[0];
    int xx = x + so[0][e];
    xx = xx >= nx ? xx - nx : xx;
    int m = xx - w.lo;
    m = m < 0 ? m + nx : m;
    b = w.col[rr][m];
    en = w.col[rr][m + 1];
}

// ------------------------------------------------------------------ block partition

// Particles in the stencil rows (full or half window) at column x of each
// cell: the window of a block spanning columns xa..xb is the sum over its
// window columns.
template <bool HALF>
__global__ void k_colsum(Geom g, const int32_t *__restrict__ cs, int32_t *__restrict__ colsum)
{
    __shared__ int so[3][kMaxOfs];
    load_offsets(g, so);
    int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= g.ncell) return;
    int nx = g.nc[0];
    int x = c % nx, r = c / nx;
    int cy = r % g.nc[1], cz = r / g.nc[1];
    int nrow = HALF ? kHalfRows : g.nofs[1] * g.nofs[2];
    int s = 0;
    for (int rr = 0; rr < nrow; rr++) {
        int cell = row_cell_of<HALF>(g, so, cy, cz, rr) + x;
        s += cs[cell + 1] - cs[cell];
    }
    colsum[c] = s;
}

// Greedy packing of one x-row: a block starts at a non-empty cell and grows
// while it holds <= 256 particles, spans at most kBlkCells columns and its
// window fits the LDS tile (wmax positions).  emit == false only counts.  A
// single cell of more than 256 particles, or whose window alone exceeds the
// tile, cannot be held: flags[3] reports it.
__device__ int pack_row(int row, const Geom &g, const int32_t *__restrict__ cs, const int32_t *__restrict__ colsum,
                        int base, int32_t *i0, int32_t *i1, int32_t *c0, int32_t *c1, bool emit, int cap,
                        int32_t *flags, int wmax)
{
    int nx = g.nc[0];
    int rb = row * nx;
    int rowsum = 0;
    for (int x = 0; x < nx; x++) rowsum += colsum[rb + x];
    auto col = [&](int k) { return colsum[rb + (k < 0 ? k + nx : (k >= nx ? k - nx : k))]; };
    // window of a block spanning xa..xb: the column sums of xa-1 .. xb+1
    // (the whole row once the columns cover it); extended one column at a
    // time as a block grows
    auto window_of = [&](int xa, int xb) {
        if (xb - xa + 3 >= nx) return rowsum;
        int s = 0;
        for (int k = xa - 1; k <= xb + 1; k++) s += col(k);
        return s;
    };
    int nb = 0;
    int bs = -1, bp = 0, bx0 = 0, bxl = 0, bw = 0;  // open block: first particle, particles, x range, window
    auto close = [&]() {
        if (bs >= 0 && bp > 0) {
            if (emit && base + nb < cap) {
                i0[base + nb] = bs;
                i1[base + nb] = bs + bp;
                c0[base + nb] = rb + bx0;
                c1[base + nb] = rb + bxl;
            }
            nb++;
        }
        bs = -1;
        bp = 0;
    };
    for (int x = 0; x < nx; x++) {
        int s = cs[rb + x], e = cs[rb + x + 1];
        int m = e - s;
        if (m == 0) continue;
        if (bs >= 0) {
            // window of [bx0, x] from that of [bx0, bxl]: add columns bxl+2 .. x+1
            int w2;
            if (x - bx0 + 3 >= nx) {
                w2 = rowsum;
            } else {
                w2 = bw;
                for (int k = bxl + 2; k <= x + 1; k++) w2 += col(k);
            }
            if (bp + m > 256 || x - bx0 >= kBlkCells || w2 > wmax) close();
            else bw = w2;
        }
        if (bs < 0) {
            bs = s;
            bx0 = x;
            bw = window_of(x, x);
            if (emit && (m > 256 || bw > wmax)) atomicOr(&flags[3], 1);
        }
        bp += m;
        bxl = x;
    }
    close();
    (void)bw;
    return nb;
}

__global__ void k_blk_count(const Geom g, const int32_t *__restrict__ cs, const int32_t *__restrict__ colsum,
                            int32_t *__restrict__ row_n, int wmax)
{
    int row = blockIdx.x * blockDim.x + threadIdx.x;
    if (row >= g.nc[1] * g.nc[2]) return;
    row_n[row] = pack_row(row, g, cs, colsum, 0, nullptr, nullptr, nullptr, nullptr, false, 0, nullptr, wmax);
}

__global__ void k_blk_write(const Geom g, const int32_t *__restrict__ cs, const int32_t *__restrict__ colsum,
                            const int32_t *__restrict__ row_base, int32_t *i0, int32_t *i1, int32_t *c0, int32_t *c1,
                            int cap, int32_t *flags, int wmax)
{
    int row = blockIdx.x * blockDim.x + threadIdx.x;
    int nrows = g.nc[1] * g.nc[2];
    if (row >= nrows) return;
    pack_row(row, g, cs, colsum, row_base[row], i0, i1, c0, c1, true, cap, flags, wmax);
}

// Common head of the windowed kernels: lay out and stage the window of
// block blk; returns false (uniformly) if it does not fit the tile.
template <int NT, bool HALF = false>
__device__ __forceinline__ bool setup_block(const Geom &g, COfs so, const int32_t *__restrict__ cs,
                                            const int4 *__restrict__ st, int c0, int c1, Window &w,
                                            WinEntry<NT> *win, int32_t *flags)
{
    __syncthreads();
    make_window<HALF>(g, so, cs, c0, c1, w);
    if (w.W > (HALF ? kWinMaxHalf : kWinMax)) {  // the packer never makes such blocks; never overrun the tile
        if (threadIdx.x == 0) atomicOr(&flags[3], 2);
        return false;
    }
    load_window(w, st, win);
    __syncthreads();
    return true;
}

// Window position of particle i (in cell ci) itself.
__device__ __forceinline__ int self_position(const Geom &g, const Window &w, const int32_t *__restrict__ cs, int i,
                                             int ci, int &x)
{
    x = ci % g.nc[0];
    int m = x - w.lo;
    m = m < 0 ? m + g.nc[0] : m;
    return w.col[w.self_row][m] + (i - cs[ci]);
}

// ------------------------------------------------------------------ traversal helpers

// The cell columns a particle in column x visits, as up to three ranges of
// window columns [a, b]: one range x-1 .. x+1 unless the columns wrap inside
// a window that covers the whole x-row (or the row has fewer than three
// distinct columns); then one range per column.  Identical for every stencil
// row.
struct ColRanges {
    int a0, b0, a1, b1, a2, b2;
};

__device__ __forceinline__ ColRanges column_ranges(const Geom &g, COfs so, const Window &w, int x)
{
    int nx = g.nc[0];
    int m = x - w.lo;
    m = m < 0 ? m + nx : m;
    ColRanges r{0, -1, 0, -1, 0, -1};
    if (g.nofs[0] == 3 && m >= 1 && m + 1 < w.ncols) {
        r.a0 = m - 1;
        r.b0 = m + 1;
        return r;
    }
    auto col = [&](int e) {
        int xx = x + so[0][e];
        xx = xx >= nx ? xx - nx : xx;
        int mm = xx - w.lo;
        return mm < 0 ? mm + nx : mm;
    };
    r.a0 = r.b0 = col(0);
    if (g.nofs[0] > 1) r.a1 = r.b1 = col(1);
    if (g.nofs[0] > 2) r.a2 = r.b2 = col(2);
    return r;
}

// One candidate pair (i, window position p) of the force traversals, branch
// free: the FP32 cutoff decision, the pair force added to f and the energy
// terms.  Returns true if the pair lies inside the guard band of the cutoff;
// the caller then decides it from the FP64 positions (pair_exact).
template <int NT, bool ISO, bool ENERGY>
__device__ __forceinline__ bool pair_fast(const int4 &pi, const int4 &pj, bool valid, const TabF<NT> &t,
                                          const Geom &g, float &fx, float &fy, float &fz, float &eu, float &ew,
                                          int &np)
{
    float dx, dy, dz;
    staged_delta<ISO>(pi, pj, g, dx, dy, dz);
    float r2 = dx * dx + dy * dy + dz * dz;
    int ab = NT == 1 ? 0 : pi.w * NT + pj.w;
    float lo = t.pick(t.lo, ab), hi = t.pick(t.hi, ab);
    bool in = valid && r2 < lo;
    float phi = lj_f32<NT, ENERGY>(r2, ab, in, t, eu, ew, np);
    fx += phi * dx;
    fy += phi * dy;
    fz += phi * dz;
    return valid && r2 >= lo && r2 < hi;
}

// A guard-band pair: added if its FP64 distance is inside the cutoff (only
// the FP64 distance is a call; the accumulators stay in registers).
template <int NT, bool ISO, bool ENERGY>
__device__ __forceinline__ void pair_exact(const int4 &pi, const int4 &pj, int i, int j, const TabF<NT> &t,
                                        const Geom &g, const double *__restrict__ pos, int n, float &fx, float &fy,
                                        float &fz, float &eu, float &ew, int &np)
{
    int ab = NT == 1 ? 0 : pi.w * NT + pj.w;
    if (exact_r2(pos, n, i, j, g.L[0], g.L[1], g.L[2]) < t.pickd(t.rc2, ab)) {
        float dx, dy, dz;
        staged_delta<ISO>(pi, pj, g, dx, dy, dz);
        float r2 = dx * dx + dy * dy + dz * dz;
        float phi = lj_f32<NT, ENERGY>(r2, ab, true, t, eu, ew, np);
        fx += phi * dx;
        fy += phi * dy;
        fz += phi * dz;
    }
}

// ------------------------------------------------------------------ linked cells

// Each thread scans the window ranges of its stencil, four candidates at a
// time (the four LDS reads issued before any arithmetic); guard-band pairs
// are collected in a bit mask and decided after the batch.
template <int NT, bool ISO, bool ENERGY>
__global__ __launch_bounds__(256) void k_lcw_f32(const int4 *__restrict__ st, const int32_t *__restrict__ cs,
                                                 const int32_t *__restrict__ cell_sorted, Geom g, int n,
                                                 const int32_t *__restrict__ nblk_p, int cap,
                                                 const int32_t *__restrict__ bi0, const int32_t *__restrict__ bi1,
                                                 const int32_t *__restrict__ bc0, const int32_t *__restrict__ bc1,
                                                 const PairTab *__restrict__ tabp, const double *__restrict__ pos,
                                                 float *__restrict__ F, double *__restrict__ partials,
                                                 int32_t *__restrict__ flags)
{
    __shared__ WinEntry<NT> win[kWinMax];
    __shared__ Window w;
    __shared__ double sh[16];
    __shared__ int so[3][kMaxOfs];
    load_offsets(g, so);
    TabF<NT> t;
    t.load(tabp);
    float eu = 0.f, ew = 0.f;
    int np = 0;
    size_t N = (size_t)n;
    for (BlockIter it(min(*nblk_p, cap)); it.blk < it.end; it.blk += it.stride) {
        int blk = it.blk;
        if (!setup_block<NT>(g, so, cs, st, bc0[blk], bc1[blk], w, win, flags)) continue;
        int i = bi0[blk] + threadIdx.x;
        if (i >= bi1[blk]) continue;
        int x;
        int self = self_position(g, w, cs, i, cell_sorted[i], x);
        int4 pi = win[self].get();
        ColRanges cr = column_ranges(g, so, w, x);
        float fx = 0.f, fy = 0.f, fz = 0.f;
        for (int rr = 0; rr < w.nrow; rr++)
            for (int sgi = 0; sgi < 3; sgi++) {
                int ca = sgi == 0 ? cr.a0 : (sgi == 1 ? cr.a1 : cr.a2);
                int cb = sgi == 0 ? cr.b0 : (sgi == 1 ? cr.b1 : cr.b2);
                if (cb < ca) continue;
                int b = w.col[rr][ca], en = w.col[rr][cb + 1];
                for (int p0 = b; p0 < en; p0 += 4) {
                    int p1 = min(p0 + 1, en - 1), p2 = min(p0 + 2, en - 1), p3 = min(p0 + 3, en - 1);
                    int4 q0 = win[p0].get(), q1 = win[p1].get(), q2 = win[p2].get(), q3 = win[p3].get();
                    uint32_t amb = 0;
                    amb |= pair_fast<NT, ISO, ENERGY>(pi, q0, p0 != self, t, g, fx, fy, fz, eu, ew, np) ? 1u : 0u;
                    amb |= pair_fast<NT, ISO, ENERGY>(pi, q1, p0 + 1 < en && p1 != self, t, g, fx, fy, fz, eu, ew,
                                                      np) ? 2u : 0u;
                    amb |= pair_fast<NT, ISO, ENERGY>(pi, q2, p0 + 2 < en && p2 != self, t, g, fx, fy, fz, eu, ew,
                                                      np) ? 4u : 0u;
                    amb |= pair_fast<NT, ISO, ENERGY>(pi, q3, p0 + 3 < en && p3 != self, t, g, fx, fy, fz, eu, ew,
                                                      np) ? 8u : 0u;
                    while (amb) {
                        int u = __builtin_ctz(amb);
                        amb &= amb - 1;
                        int p = p0 + u;
                        pair_exact<NT, ISO, ENERGY>(pi, win[p].get(), i, window_global(w, p), t, g, pos, n, fx, fy,
                                                    fz, eu, ew, np);
                    }
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

// ------------------------------------------------------------------ Verlet lists

// List entry c of particle i: nbr[((c / 8) * n + i) * 8 + c % 8].
__device__ __forceinline__ size_t list_slot(int c, int i, size_t N) { return ((size_t)(c >> 3) * N + i) * 8 + (c & 7); }

// Pending chunk of eight 16-bit entries of the list being built.
struct Chunk {
    uint64_t lo = 0, hi = 0;
    __device__ __forceinline__ void put(int e, uint32_t p)
    {
        uint64_t v = (uint64_t)p << (16 * (e & 3));
        if (e < 4)
            lo |= v;
        else
            hi |= v;
    }
    __device__ __forceinline__ uint4 word() const
    {
        return make_uint4((uint32_t)lo, (uint32_t)(lo >> 32), (uint32_t)hi, (uint32_t)(hi >> 32));
    }
};

// Append window position p to the list of particle i (c entries so far);
// every completed chunk is written with one 16-byte store.
__device__ __forceinline__ void list_append(uint32_t p, int &c, Chunk &ck, uint4 *__restrict__ row, size_t N,
                                            int maxn)
{
    ck.put(c & 7, p);
    c++;
    if ((c & 7) == 0) {
        if (c <= maxn) row[(size_t)((c >> 3) - 1) * N] = ck.word();
        ck.lo = ck.hi = 0;
    }
}

template <bool ISO>
__device__ __forceinline__ bool build_fast(const int4 &pi, const int4 &pj, bool valid, const Geom &g, bool &amb)
{
    float dx, dy, dz;
    staged_delta<ISO>(pi, pj, g, dx, dy, dz);
    float r2 = dx * dx + dy * dy + dz * dz;
    amb = valid && r2 >= g.rl2_lo && r2 < g.rl2_hi;
    return valid && r2 < g.rl2_lo;
}

template <bool ISO>
__global__ __launch_bounds__(256) void k_vlw_build(const int4 *__restrict__ st, const int32_t *__restrict__ cs,
                                                   const int32_t *__restrict__ cell_sorted,
                                                   const double *__restrict__ pos, Geom g, int n,
                                                   const int32_t *__restrict__ nblk_p, int cap,
                                                   const int32_t *__restrict__ bi0, const int32_t *__restrict__ bi1,
                                                   const int32_t *__restrict__ bc0, const int32_t *__restrict__ bc1,
                                                   uint16_t *__restrict__ nbr, int32_t *__restrict__ cnt, int maxn,
                                                   int32_t *__restrict__ flags)
{
    __shared__ WinEntry<1> win[kWinMax];
    __shared__ Window w;
    __shared__ int so[3][kMaxOfs];
    load_offsets(g, so);
    size_t N = (size_t)n;
    int cmax = 0;
    for (BlockIter it(min(*nblk_p, cap)); it.blk < it.end; it.blk += it.stride) {
        int blk = it.blk;
        if (!setup_block<1>(g, so, cs, st, bc0[blk], bc1[blk], w, win, flags)) continue;
        int i = bi0[blk] + threadIdx.x;
        if (i >= bi1[blk]) continue;
        int x;
        int self = self_position(g, w, cs, i, cell_sorted[i], x);
        int4 pi = win[self].get();
        ColRanges cr = column_ranges(g, so, w, x);
        uint4 *row = (uint4 *)nbr + i;
        int c = 0;
        Chunk ck;
        for (int rr = 0; rr < w.nrow; rr++)
            for (int sgi = 0; sgi < 3; sgi++) {
                int ca = sgi == 0 ? cr.a0 : (sgi == 1 ? cr.a1 : cr.a2);
                int cb = sgi == 0 ? cr.b0 : (sgi == 1 ? cr.b1 : cr.b2);
                if (cb < ca) continue;
                int b = w.col[rr][ca], en = w.col[rr][cb + 1];
                for (int p0 = b; p0 < en; p0 += 4) {
                    int p1 = min(p0 + 1, en - 1), p2 = min(p0 + 2, en - 1), p3 = min(p0 + 3, en - 1);
                    int4 q0 = win[p0].get(), q1 = win[p1].get(), q2 = win[p2].get(), q3 = win[p3].get();
                    bool a0, a1, a2, a3;
                    bool i0 = build_fast<ISO>(pi, q0, p0 != self, g, a0);
                    bool i1 = build_fast<ISO>(pi, q1, p0 + 1 < en && p1 != self, g, a1);
                    bool i2 = build_fast<ISO>(pi, q2, p0 + 2 < en && p2 != self, g, a2);
                    bool i3 = build_fast<ISO>(pi, q3, p0 + 3 < en && p3 != self, g, a3);
                    // rare: guard-band pairs decided from the FP64 positions
                    if (a0) i0 = exact_r2(pos, n, i, window_global(w, p0), g.L[0], g.L[1], g.L[2]) < g.rl2;
                    if (a1) i1 = exact_r2(pos, n, i, window_global(w, p1), g.L[0], g.L[1], g.L[2]) < g.rl2;
                    if (a2) i2 = exact_r2(pos, n, i, window_global(w, p2), g.L[0], g.L[1], g.L[2]) < g.rl2;
                    if (a3) i3 = exact_r2(pos, n, i, window_global(w, p3), g.L[0], g.L[1], g.L[2]) < g.rl2;
                    if (i0) list_append((uint32_t)p0, c, ck, row, N, maxn);
                    if (i1) list_append((uint32_t)p1, c, ck, row, N, maxn);
                    if (i2) list_append((uint32_t)p2, c, ck, row, N, maxn);
                    if (i3) list_append((uint32_t)p3, c, ck, row, N, maxn);
                }
            }
        if ((c & 7) && c < maxn) row[(size_t)(c >> 3) * N] = ck.word();
        if (c > maxn) atomicOr(&flags[0], (int)MD_FLAG_LIST_OVERFLOW);
        cmax = max(cmax, c);
        cnt[i] = c < maxn ? c : maxn;
    }
    if (cmax > 0) atomicMax(&flags[2], cmax);
}

// Each thread walks its list in chunks of eight entries; the next chunk's
// load is in flight while the current one is computed.
template <int NT, bool ISO, bool ENERGY>
__global__ __launch_bounds__(256) void k_vlw_f32(const int4 *__restrict__ st, const int32_t *__restrict__ cs, Geom g,
                                                 int n, const int32_t *__restrict__ nblk_p, int cap,
                                                 const int32_t *__restrict__ bi0, const int32_t *__restrict__ bi1,
                                                 const int32_t *__restrict__ bc0, const int32_t *__restrict__ bc1,
                                                 const uint16_t *__restrict__ nbr, const int32_t *__restrict__ cnt,
                                                 const PairTab *__restrict__ tabp, const double *__restrict__ pos,
                                                 float *__restrict__ F, double *__restrict__ partials,
                                                 int32_t *__restrict__ flags)
{
    __shared__ WinEntry<NT> win[kWinMax];
    __shared__ Window w;
    __shared__ double sh[16];
    __shared__ int so[3][kMaxOfs];
    load_offsets(g, so);
    TabF<NT> t;
    t.load(tabp);
    float eu = 0.f, ew = 0.f;
    int np = 0;
    size_t N = (size_t)n;
    for (BlockIter it(min(*nblk_p, cap)); it.blk < it.end; it.blk += it.stride) {
        int blk = it.blk;
        if (!setup_block<NT>(g, so, cs, st, bc0[blk], bc1[blk], w, win, flags)) continue;
        int i = bi0[blk] + threadIdx.x;
        if (i >= bi1[blk]) continue;
        int4 pi = st[i];
        int c = cnt[i];
        int nch = (c + 7) >> 3;
        float fx = 0.f, fy = 0.f, fz = 0.f;
        // chunk ch of particle i is row[ch * n]; the prefetch index is clamped
        // so that every load is an in-bounds global load
        const uint4 *row = (const uint4 *)nbr + i;
        uint4 cur = row[0];
        for (int ch = 0; ch < nch; ch++) {
            uint4 nxt = row[(size_t)min(ch + 1, nch - 1) * N];
            int valid = min(8, c - ch * 8);
            int pp[8] = {(int)(cur.x & 0xffff), (int)(cur.x >> 16), (int)(cur.y & 0xffff), (int)(cur.y >> 16),
                         (int)(cur.z & 0xffff), (int)(cur.z >> 16), (int)(cur.w & 0xffff), (int)(cur.w >> 16)};
            uint32_t amb = 0;
#pragma unroll
            for (int u = 0; u < 8; u++) {
                int4 pj = win[pp[u]].get();
                amb |= pair_fast<NT, ISO, ENERGY>(pi, pj, u < valid, t, g, fx, fy, fz, eu, ew, np) ? 1u << u : 0u;
            }
            // rare: pairs within the guard band of the cutoff
            while (amb) {
                int u = __builtin_ctz(amb);
                amb &= amb - 1;
                uint32_t word = u < 2 ? cur.x : (u < 4 ? cur.y : (u < 6 ? cur.z : cur.w));
                int p = (word >> ((u & 1) * 16)) & 0xffff;
                pair_exact<NT, ISO, ENERGY>(pi, win[p].get(), i, window_global(w, p), t, g, pos, n, fx, fy, fz, eu,
                                            ew, np);
            }
            cur = nxt;
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

// ------------------------------------------------------------------ Newton's third law (half windows)

// Each pair once: a thread takes the pairs of its particle with the forward
// rows of the half window and, in its own row, with the particles after it
// in its cell and those of the next cell.  The j-side forces accumulate in
// LDS (one float per component and window position, LDS atomics); after the
// block every nonzero entry is added to the global force with one atomic per
// component, where consecutive positions of a piece are consecutive
// particles, so that a wavefront's atomics are coalesced.
struct HalfAcc {
    float x[kWinMaxHalf], y[kWinMaxHalf], z[kWinMaxHalf];
};

// Head of the half-window kernels: window laid out and staged, accumulators
// cleared; false (uniformly) if the window does not fit.
template <int NT>
__device__ __forceinline__ bool setup_half(const Geom &g, COfs so, const int32_t *__restrict__ cs,
                                           const int4 *__restrict__ st, int c0, int c1, Window &w,
                                           WinEntry<NT> *win, HalfAcc &acc, int32_t *flags)
{
    __syncthreads();
    make_window<true>(g, so, cs, c0, c1, w);
    if (w.W > kWinMaxHalf) {  // the packer never makes such blocks; never overrun the tile
        if (threadIdx.x == 0) atomicOr(&flags[3], 2);
        return false;
    }
    load_window(w, st, win);
    for (int p = threadIdx.x; p < w.W; p += blockDim.x) {
        acc.x[p] = 0.f;
        acc.y[p] = 0.f;
        acc.z[p] = 0.f;
    }
    __syncthreads();
    return true;
}

__device__ __forceinline__ void flush_half(const HalfAcc &acc, const Window &w, float *__restrict__ F, size_t N)
{
    __syncthreads();
    int k = 0;
    for (int p = threadIdx.x; p < w.W; p += blockDim.x) {
        k = piece_from(w, k, p);
        int j = w.pc_start[k] + (p - w.pc_win[k]);
        float vx = acc.x[p], vy = acc.y[p], vz = acc.z[p];
        if (vx != 0.f) atomicAdd(&F[j], vx);
        if (vy != 0.f) atomicAdd(&F[N + j], vy);
        if (vz != 0.f) atomicAdd(&F[2 * N + j], vz);
    }
}

// One candidate pair with Newton's third law: the i-side force in registers,
// the j-side one into the LDS accumulator of window position p.  Returns true
// for a guard-band pair (decided by the caller from the FP64 positions).
template <int NT, bool ISO, bool ENERGY>
__device__ __forceinline__ bool pair_n3l(const int4 &pi, const int4 &pj, int p, bool valid, const TabF<NT> &t,
                                         const Geom &g, HalfAcc &acc, float &fx, float &fy, float &fz, float &eu,
                                         float &ew, int &np)
{
    float dx, dy, dz;
    staged_delta<ISO>(pi, pj, g, dx, dy, dz);
    float r2 = dx * dx + dy * dy + dz * dz;
    int ab = NT == 1 ? 0 : pi.w * NT + pj.w;
    float lo = t.pick(t.lo, ab), hi = t.pick(t.hi, ab);
    bool in = valid && r2 < lo;
    float phi = lj_f32<NT, ENERGY>(r2, ab, in, t, eu, ew, np);
    fx += phi * dx;
    fy += phi * dy;
    fz += phi * dz;
    if (in) {
        atomicAdd(&acc.x[p], -phi * dx);
        atomicAdd(&acc.y[p], -phi * dy);
        atomicAdd(&acc.z[p], -phi * dz);
    }
    return valid && r2 >= lo && r2 < hi;
}

template <int NT, bool ISO, bool ENERGY>
__device__ __forceinline__ void pair_exact_n3l(const int4 &pi, const int4 &pj, int p, int i, int j,
                                               const TabF<NT> &t, const Geom &g, const double *__restrict__ pos,
                                               int n, HalfAcc &acc, float &fx, float &fy, float &fz, float &eu,
                                               float &ew, int &np)
{
    int ab = NT == 1 ? 0 : pi.w * NT + pj.w;
    if (exact_r2(pos, n, i, j, g.L[0], g.L[1], g.L[2]) < t.pickd(t.rc2, ab)) {
        float dx, dy, dz;
        staged_delta<ISO>(pi, pj, g, dx, dy, dz);
        float r2 = dx * dx + dy * dy + dz * dz;
        float phi = lj_f32<NT, ENERGY>(r2, ab, true, t, eu, ew, np);
        fx += phi * dx;
        fy += phi * dy;
        fz += phi * dz;
        atomicAdd(&acc.x[p], -phi * dx);
        atomicAdd(&acc.y[p], -phi * dy);
        atomicAdd(&acc.z[p], -phi * dz);
    }
}

// The candidate window ranges of a particle in a half window: the forward
// rows over its three columns (as in the full traversal), then in the own
// row the positions after its own (self + 1 to the end of its cell) and the
// cell of column x + 1, merged when the two are adjacent in the window.
struct HalfOwn {
    int b0, e0, b1, e1;
};

__device__ __forceinline__ HalfOwn half_own(const Geom &g, const Window &w, int self, int x)
{
    int nx = g.nc[0];
    int m = x - w.lo;
    m = m < 0 ? m + nx : m;
    int x1 = x + 1 == nx ? 0 : x + 1;
    int m1 = x1 - w.lo;
    m1 = m1 < 0 ? m1 + nx : m1;
    HalfOwn r;
    if (m1 == m + 1) {
        r.b0 = self + 1;
        r.e0 = w.col[kHalfOwn][m + 2];
        r.b1 = r.e1 = 0;
    } else {
        r.b0 = self + 1;
        r.e0 = w.col[kHalfOwn][m + 1];
        r.b1 = w.col[kHalfOwn][m1];
        r.e1 = w.col[kHalfOwn][m1 + 1];
    }
    return r;
}

// All pairs of particle i with window positions [b, en), four at a time.
template <int NT, bool ISO, bool ENERGY>
__device__ __forceinline__ void range_n3l(int b, int en, const int4 &pi, int i, const WinEntry<NT> *win,
                                          const Window &w, const TabF<NT> &t, const Geom &g,
                                          const double *__restrict__ pos, int n, HalfAcc &acc, float &fx, float &fy,
                                          float &fz, float &eu, float &ew, int &np)
{
    for (int p0 = b; p0 < en; p0 += 4) {
        int p1 = min(p0 + 1, en - 1), p2 = min(p0 + 2, en - 1), p3 = min(p0 + 3, en - 1);
        int4 q0 = win[p0].get(), q1 = win[p1].get(), q2 = win[p2].get(), q3 = win[p3].get();
        uint32_t amb = 0;
        amb |= pair_n3l<NT, ISO, ENERGY>(pi, q0, p0, true, t, g, acc, fx, fy, fz, eu, ew, np) ? 1u : 0u;
        amb |= pair_n3l<NT, ISO, ENERGY>(pi, q1, p1, p0 + 1 < en, t, g, acc, fx, fy, fz, eu, ew, np) ? 2u : 0u;
        amb |= pair_n3l<NT, ISO, ENERGY>(pi, q2, p2, p0 + 2 < en, t, g, acc, fx, fy, fz, eu, ew, np) ? 4u : 0u;
        amb |= pair_n3l<NT, ISO, ENERGY>(pi, q3, p3, p0 + 3 < en, t, g, acc, fx, fy, fz, eu, ew, np) ? 8u : 0u;
        while (amb) {
            int u = __builtin_ctz(amb);
            amb &= amb - 1;
            int p = p0 + u;
            pair_exact_n3l<NT, ISO, ENERGY>(pi, win[p].get(), p, i, window_global(w, p), t, g, pos, n, acc, fx, fy,
                                            fz, eu, ew, np);
        }
    }
}

template <int NT, bool ISO, bool ENERGY>
__global__ __launch_bounds__(256) void k_lcwh_f32(const int4 *__restrict__ st, const int32_t *__restrict__ cs,
                                                  const int32_t *__restrict__ cell_sorted, Geom g, int n,
                                                  const int32_t *__restrict__ nblk_p, int cap,
                                                  const int32_t *__restrict__ bi0, const int32_t *__restrict__ bi1,
                                                  const int32_t *__restrict__ bc0, const int32_t *__restrict__ bc1,
                                                  const PairTab *__restrict__ tabp, const double *__restrict__ pos,
                                                  float *__restrict__ F, double *__restrict__ partials,
                                                  int32_t *__restrict__ flags)
{
    __shared__ WinEntry<NT> win[kWinMaxHalf];
    __shared__ HalfAcc acc;
    __shared__ Window w;
    __shared__ double sh[16];
    __shared__ int so[3][kMaxOfs];
    load_offsets(g, so);
    TabF<NT> t;
    t.load(tabp);
    float eu = 0.f, ew = 0.f;
    int np = 0;
    size_t N = (size_t)n;
    for (BlockIter it(min(*nblk_p, cap)); it.blk < it.end; it.blk += it.stride) {
        int blk = it.blk;
        if (!setup_half<NT>(g, so, cs, st, bc0[blk], bc1[blk], w, win, acc, flags)) continue;
        int i = bi0[blk] + threadIdx.x;
        if (i < bi1[blk]) {
            int x;
            int self = self_position(g, w, cs, i, cell_sorted[i], x);
            int4 pi = win[self].get();
            ColRanges cr = column_ranges(g, so, w, x);
            float fx = 0.f, fy = 0.f, fz = 0.f;
            for (int rr = 0; rr < kHalfOwn; rr++)
                for (int sgi = 0; sgi < 3; sgi++) {
                    int ca = sgi == 0 ? cr.a0 : (sgi == 1 ? cr.a1 : cr.a2);
                    int cb = sgi == 0 ? cr.b0 : (sgi == 1 ? cr.b1 : cr.b2);
                    if (cb < ca) continue;
                    range_n3l<NT, ISO, ENERGY>(w.col[rr][ca], w.col[rr][cb + 1], pi, i, win, w, t, g, pos, n, acc,
                                               fx, fy, fz, eu, ew, np);
                }
            HalfOwn ow = half_own(g, w, self, x);
            range_n3l<NT, ISO, ENERGY>(ow.b0, ow.e0, pi, i, win, w, t, g, pos, n, acc, fx, fy, fz, eu, ew, np);
            range_n3l<NT, ISO, ENERGY>(ow.b1, ow.e1, pi, i, win, w, t, g, pos, n, acc, fx, fy, fz, eu, ew, np);
            atomicAdd(&acc.x[self], fx);
            atomicAdd(&acc.y[self], fy);
            atomicAdd(&acc.z[self], fz);
        }
        flush_half(acc, w, F, N);
    }
    if (ENERGY) {
        double v[4] = {(double)eu, (double)ew, (double)np, 0.0};
        block_sum4(v, sh);
        if (threadIdx.x == 0)
            for (int k = 0; k < 4; k++) partials[blockIdx.x * 4 + k] = v[k];
    }
}

// Half Verlet lists: the candidates of the half traversal within r_c + skin.
template <bool ISO>
__device__ __forceinline__ void range_build(int b, int en, const int4 &pi, int i, const WinEntry<1> *win,
                                            const Window &w, const Geom &g, const double *__restrict__ pos, int n,
                                            int &c, Chunk &ck, uint4 *__restrict__ row, size_t N, int maxn)
{
    for (int p0 = b; p0 < en; p0 += 4) {
        int p1 = min(p0 + 1, en - 1), p2 = min(p0 + 2, en - 1), p3 = min(p0 + 3, en - 1);
        int4 q0 = win[p0].get(), q1 = win[p1].get(), q2 = win[p2].get(), q3 = win[p3].get();
        bool a0, a1, a2, a3;
        bool i0 = build_fast<ISO>(pi, q0, true, g, a0);
        bool i1 = build_fast<ISO>(pi, q1, p0 + 1 < en, g, a1);
        bool i2 = build_fast<ISO>(pi, q2, p0 + 2 < en, g, a2);
        bool i3 = build_fast<ISO>(pi, q3, p0 + 3 < en, g, a3);
        if (a0) i0 = exact_r2(pos, n, i, window_global(w, p0), g.L[0], g.L[1], g.L[2]) < g.rl2;
        if (a1) i1 = exact_r2(pos, n, i, window_global(w, p1), g.L[0], g.L[1], g.L[2]) < g.rl2;
        if (a2) i2 = exact_r2(pos, n, i, window_global(w, p2), g.L[0], g.L[1], g.L[2]) < g.rl2;
        if (a3) i3 = exact_r2(pos, n, i, window_global(w, p3), g.L[0], g.L[1], g.L[2]) < g.rl2;
        if (i0) list_append((uint32_t)p0, c, ck, row, N, maxn);
        if (i1) list_append((uint32_t)p1, c, ck, row, N, maxn);
        if (i2) list_append((uint32_t)p2, c, ck, row, N, maxn);
        if (i3) list_append((uint32_t)p3, c, ck, row, N, maxn);
    }
}

template <bool ISO>
__global__ __launch_bounds__(256) void k_vlwh_build(const int4 *__restrict__ st, const int32_t *__restrict__ cs,
                                                    const int32_t *__restrict__ cell_sorted,
                                                    const double *__restrict__ pos, Geom g, int n,
                                                    const int32_t *__restrict__ nblk_p, int cap,
                                                    const int32_t *__restrict__ bi0, const int32_t *__restrict__ bi1,
                                                    const int32_t *__restrict__ bc0, const int32_t *__restrict__ bc1,
                                                    uint16_t *__restrict__ nbr, int32_t *__restrict__ cnt, int maxn,
                                                    int32_t *__restrict__ flags)
{
    __shared__ WinEntry<1> win[kWinMaxHalf];
    __shared__ Window w;
    __shared__ int so[3][kMaxOfs];
    load_offsets(g, so);
    size_t N = (size_t)n;
    int cmax = 0;
    for (BlockIter it(min(*nblk_p, cap)); it.blk < it.end; it.blk += it.stride) {
        int blk = it.blk;
        if (!setup_block<1, true>(g, so, cs, st, bc0[blk], bc1[blk], w, win, flags)) continue;
        int i = bi0[blk] + threadIdx.x;
        if (i >= bi1[blk]) continue;
        int x;
        int self = self_position(g, w, cs, i, cell_sorted[i], x);
        int4 pi = win[self].get();
        ColRanges cr = column_ranges(g, so, w, x);
        uint4 *row = (uint4 *)nbr + i;
        int c = 0;
        Chunk ck;
        for (int rr = 0; rr < kHalfOwn; rr++)
            for (int sgi = 0; sgi < 3; sgi++) {
                int ca = sgi == 0 ? cr.a0 : (sgi == 1 ? cr.a1 : cr.a2);
                int cb = sgi == 0 ? cr.b0 : (sgi == 1 ? cr.b1 : cr.b2);
                if (cb < ca) continue;
                range_build<ISO>(w.col[rr][ca], w.col[rr][cb + 1], pi, i, win, w, g, pos, n, c, ck, row, N, maxn);
            }
        HalfOwn ow = half_own(g, w, self, x);
        range_build<ISO>(ow.b0, ow.e0, pi, i, win, w, g, pos, n, c, ck, row, N, maxn);
        range_build<ISO>(ow.b1, ow.e1, pi, i, win, w, g, pos, n, c, ck, row, N, maxn);
        if ((c & 7) && c < maxn) row[(size_t)(c >> 3) * N] = ck.word();
        if (c > maxn) atomicOr(&flags[0], (int)MD_FLAG_LIST_OVERFLOW);
        cmax = max(cmax, c);
        cnt[i] = c < maxn ? c : maxn;
    }
    if (cmax > 0) atomicMax(&flags[2], cmax);
}

template <int NT, bool ISO, bool ENERGY>
__global__ __launch_bounds__(256) void k_vlwh_f32(const int4 *__restrict__ st, const int32_t *__restrict__ cs,
                                                  const int32_t *__restrict__ cell_sorted, Geom g, int n,
                                                  const int32_t *__restrict__ nblk_p, int cap,
                                                  const int32_t *__restrict__ bi0, const int32_t *__restrict__ bi1,
                                                  const int32_t *__restrict__ bc0, const int32_t *__restrict__ bc1,
                                                  const uint16_t *__restrict__ nbr, const int32_t *__restrict__ cnt,
                                                  const PairTab *__restrict__ tabp, const double *__restrict__ pos,
                                                  float *__restrict__ F, double *__restrict__ partials,
                                                  int32_t *__restrict__ flags)
{
    __shared__ WinEntry<NT> win[kWinMaxHalf];
    __shared__ HalfAcc acc;
    __shared__ Window w;
    __shared__ double sh[16];
    __shared__ int so[3][kMaxOfs];
    load_offsets(g, so);
    TabF<NT> t;
    t.load(tabp);
    float eu = 0.f, ew = 0.f;
    int np = 0;
    size_t N = (size_t)n;
    for (BlockIter it(min(*nblk_p, cap)); it.blk < it.end; it.blk += it.stride) {
        int blk = it.blk;
        if (!setup_half<NT>(g, so, cs, st, bc0[blk], bc1[blk], w, win, acc, flags)) continue;
        int i = bi0[blk] + threadIdx.x;
        if (i < bi1[blk]) {
            int x;
            int self = self_position(g, w, cs, i, cell_sorted[i], x);
            int4 pi = win[self].get();
            int c = cnt[i];
            int nch = (c + 7) >> 3;
            float fx = 0.f, fy = 0.f, fz = 0.f;
            const uint4 *row = (const uint4 *)nbr + i;
            uint4 cur = row[0];
            for (int ch = 0; ch < nch; ch++) {
                uint4 nxt = row[(size_t)min(ch + 1, nch - 1) * N];
                int valid = min(8, c - ch * 8);
                int pp[8] = {(int)(cur.x & 0xffff), (int)(cur.x >> 16), (int)(cur.y & 0xffff), (int)(cur.y >> 16),
                             (int)(cur.z & 0xffff), (int)(cur.z >> 16), (int)(cur.w & 0xffff), (int)(cur.w >> 16)};
                uint32_t amb = 0;
#pragma unroll
                for (int u = 0; u < 8; u++) {
                    int4 pj = win[pp[u]].get();
                    amb |= pair_n3l<NT, ISO, ENERGY>(pi, pj, pp[u], u < valid, t, g, acc, fx, fy, fz, eu, ew, np)
                               ? 1u << u
                               : 0u;
                }
                while (amb) {
                    int u = __builtin_ctz(amb);
                    amb &= amb - 1;
                    uint32_t word = u < 2 ? cur.x : (u < 4 ? cur.y : (u < 6 ? cur.z : cur.w));
                    int p = (word >> ((u & 1) * 16)) & 0xffff;
                    pair_exact_n3l<NT, ISO, ENERGY>(pi, win[p].get(), p, i, window_global(w, p), t, g, pos, n, acc,
                                                    fx, fy, fz, eu, ew, np);
                }
                cur = nxt;
            }
            atomicAdd(&acc.x[self], fx);
            atomicAdd(&acc.y[self], fy);
            atomicAdd(&acc.z[self], fz);
        }
        flush_half(acc, w, F, N);
    }
    if (ENERGY) {
        double v[4] = {(double)eu, (double)ew, (double)np, 0.0};
        block_sum4(v, sh);
        if (threadIdx.x == 0)
            for (int k = 0; k < 4; k++) partials[blockIdx.x * 4 + k] = v[k];
    }
}

// Decode the window lists back to global indices (inspection).
template <bool HALF>
__global__ void k_vlw_decode(const int32_t *__restrict__ cs, Geom g, int n, const int32_t *__restrict__ nblk_p, int cap,
                             const int32_t *__restrict__ bi0, const int32_t *__restrict__ bi1,
                             const int32_t *__restrict__ bc0, const int32_t *__restrict__ bc1,
                             const uint16_t *__restrict__ nbr, const int32_t *__restrict__ cnt, int maxr,
                             int32_t *__restrict__ counts, int32_t *__restrict__ rows)
{
    __shared__ Window w;
    __shared__ int so[3][kMaxOfs];
    load_offsets(g, so);
    size_t N = (size_t)n;
    int nblk = min(*nblk_p, cap);
    for (int blk = blockIdx.x; blk < nblk; blk += gridDim.x) {
        __syncthreads();
        make_window<HALF>(g, so, cs, bc0[blk], bc1[blk], w);
        int i = bi0[blk] + threadIdx.x;
        if (i >= bi1[blk]) continue;
        int c = cnt[i];
        counts[i] = c;
        for (int k = 0; k < c && k < maxr; k++) rows[(size_t)i * maxr + k] = window_global(w, nbr[list_slot(k, i, N)]);
    }
}

// ------------------------------------------------------------------ host side

int64_t window_block_cap(int64_t n, const Geom &g) { return n + (int64_t)g.nc[1] * g.nc[2] + 16; }

bool window_geometry_ok(const Geom &g, bool half)
{
    bool ok = g.reach[0] == 1 && g.reach[1] == 1 && g.reach[2] == 1 && g.nofs[1] * g.nofs[2] <= kMaxRows;
    if (half) ok = ok && g.nofs[0] == 3 && g.nofs[1] == 3 && g.nofs[2] == 3;
    return ok;
}

void launch_blocks(const Geom &g, const int32_t *cs, int32_t *colsum, int32_t *row_n, int32_t *row_base,
                   int32_t *scan_scratch, int32_t *i0, int32_t *i1, int32_t *c0, int32_t *c1, int cap,
                   int32_t *flags, bool half, hipStream_t s)
{
    int nrows = g.nc[1] * g.nc[2];
    int wmax = half ? kWinMaxHalf : kWinMax;
    if (half)
        k_colsum<true><<<(g.ncell + 255) / 256, 256, 0, s>>>(g, cs, colsum);
    else
        k_colsum<false><<<(g.ncell + 255) / 256, 256, 0, s>>>(g, cs, colsum);
    k_blk_count<<<(nrows + 63) / 64, 64, 0, s>>>(g, cs, colsum, row_n, wmax);
    launch_scan(row_n, row_base, nrows, scan_scratch, s);
    k_blk_write<<<(nrows + 63) / 64, 64, 0, s>>>(g, cs, colsum, row_base, i0, i1, c0, c1, cap, flags, wmax);
}

// maxn is rounded up to whole chunks of eight (the list holds them).
void launch_vlw_build(const int4 *st, const int32_t *cs, const int32_t *cell_sorted, const double *pos,
                      const Geom &g, int n, const int32_t *nblk_p, const int32_t *i0, const int32_t *i1,
                      const int32_t *c0, const int32_t *c1, uint16_t *nbr, int32_t *cnt, int maxn, int32_t *flags,
                      bool half, hipStream_t s)
{
    if (n <= 0) return;
    int cap = (int)window_block_cap(n, g);
    maxn = (maxn + 7) & ~7;
    if (half) {
        if (g.iso)
            k_vlwh_build<true><<<kWinGrid, 256, 0, s>>>(st, cs, cell_sorted, pos, g, n, nblk_p, cap, i0, i1, c0, c1,
                                                         nbr, cnt, maxn, flags);
        else
            k_vlwh_build<false><<<kWinGrid, 256, 0, s>>>(st, cs, cell_sorted, pos, g, n, nblk_p, cap, i0, i1, c0,
                                                          c1, nbr, cnt, maxn, flags);
    } else {
        if (g.iso)
            k_vlw_build<true><<<kWinGrid, 256, 0, s>>>(st, cs, cell_sorted, pos, g, n, nblk_p, cap, i0, i1, c0, c1,
                                                        nbr, cnt, maxn, flags);
        else
            k_vlw_build<false><<<kWinGrid, 256, 0, s>>>(st, cs, cell_sorted, pos, g, n, nblk_p, cap, i0, i1, c0, c1,
                                                         nbr, cnt, maxn, flags);
    }
}

int window_force_blocks() { return kWinGrid; }

template <int NT, bool ISO, bool EN>
static void win_launch(const ForceArgs &a, const Geom &g, hipStream_t s)
{
    int cap = (int)window_block_cap(a.n, g);
    bool vl = a.container == MD_CONTAINER_VL;
    if (a.newton3 && vl)
        k_vlwh_f32<NT, ISO, EN><<<kWinGrid, 256, 0, s>>>(a.stage, a.cell_start, a.cell_sorted, g, a.n, a.w_nblk, cap,
                                                        a.w_i0, a.w_i1, a.w_c0, a.w_c1, a.w_nbr, a.nbr_count, a.tab,
                                                        a.pos, (float *)a.force, a.partials, a.flags);
    else if (a.newton3)
        k_lcwh_f32<NT, ISO, EN><<<kWinGrid, 256, 0, s>>>(a.stage, a.cell_start, a.cell_sorted, g, a.n, a.w_nblk, cap,
                                                        a.w_i0, a.w_i1, a.w_c0, a.w_c1, a.tab, a.pos,
                                                        (float *)a.force, a.partials, a.flags);
    else if (vl)
        k_vlw_f32<NT, ISO, EN><<<kWinGrid, 256, 0, s>>>(a.stage, a.cell_start, g, a.n, a.w_nblk, cap, a.w_i0, a.w_i1,
                                                       a.w_c0, a.w_c1, a.w_nbr, a.nbr_count, a.tab, a.pos,
                                                       (float *)a.force, a.partials, a.flags);
    else
        k_lcw_f32<NT, ISO, EN><<<kWinGrid, 256, 0, s>>>(a.stage, a.cell_start, a.cell_sorted, g, a.n, a.w_nblk, cap,
                                                       a.w_i0, a.w_i1, a.w_c0, a.w_c1, a.tab, a.pos,
                                                       (float *)a.force, a.partials, a.flags);
}

void launch_window_force(const ForceArgs &a, const Geom &g, hipStream_t s)
{
    if (a.n <= 0) return;
    if (g.nt == 1) {
        if (g.iso) {
            if (a.energy) win_launch<1, true, true>(a, g, s);
            else win_launch<1, true, false>(a, g, s);
        } else {
            if (a.energy) win_launch<1, false, true>(a, g, s);
            else win_launch<1, false, false>(a, g, s);
        }
    } else {
        if (g.iso) {
            if (a.energy) win_launch<2, true, true>(a, g, s);
            else win_launch<2, true, false>(a, g, s);
        } else {
            if (a.energy) win_launch<2, false, true>(a, g, s);
            else win_launch<2, false, false>(a, g, s);
        }
    }
}

void launch_vlw_decode(const int32_t *cs, const Geom &g, int n, const int32_t *nblk_p, const int32_t *i0,
                       const int32_t *i1, const int32_t *c0, const int32_t *c1, const uint16_t *nbr,
                       const int32_t *cnt, int maxr, int32_t *counts, int32_t *rows, bool half, hipStream_t s)
{
    if (n <= 0) return;
    int cap = (int)window_block_cap(n, g);
    if (half)
        k_vlw_decode<true><<<kWinGrid, 256, 0, s>>>(cs, g, n, nblk_p, cap, i0, i1, c0, c1, nbr, cnt, maxr, counts,
                                                    rows);
    else
        k_vlw_decode<false><<<kWinGrid, 256, 0, s>>>(cs, g, n, nblk_p, cap, i0, i1, c0, c1, nbr, cnt, maxr, counts,
                                                     rows);
}

}  // namespace mdlj

// Pair traversals over LDS windows (FP32).
//
// Particles are in linked-cell order (cells x-fastest).  A block is a
// rectangle of cells in one z-layer: up to four consecutive y-rows (more rows
// when cells hold few particles) times a run of consecutive x-columns, with
// at most 256 particles (one workgroup, one thread per particle).  Its window
// is the union of its cells' stencils for a reach of r = 1 or 2 cells: the
// (y, z) rows y0 - r .. y1 + r of layers z - r .. z + r, each over the cell
// columns [x_first - r, x_last + r] (two particle ranges, or pieces, when the
// columns wrap around the periodic box).  The block packer bounds every
// window to the LDS tile.  A workgroup stages the window once, then:
//   - linked cells: each thread scans its own stencil inside the window (the
//     GPU analogue of the C01 traversal: no write conflicts);
//   - Verlet lists: each thread walks its list of 16-bit window positions,
//     stored in chunks of eight (one 16-byte load per chunk, the next chunk
//     in flight while the current one is computed);
//   - with Newton's third law, a half window holds only the forward part of
//     the stencils (see row_of) and the j-side forces go to LDS.
// Blocks of neighbouring cells share most of their windows, so the blocks
// are dealt to the eight XCDs in contiguous chunks (workgroup w runs on XCD
// w mod 8) to keep the shared window data in one L2.
#include <type_traits>

#include "verlet.h"

namespace mdlj {

constexpr int kWinMax = 2880;      // LDS window capacity (particles), full windows
constexpr int kWinMaxHalf = 2048;  // half windows (positions and j-side forces)
constexpr int kBlkCells = 32;      // maximum cells of a block along x
constexpr int kMaxReach = 2;
constexpr int kMaxRows = (2 * kMaxReach + 1) * (kWinBlkRows + 2 * kMaxReach);  // window rows
constexpr int kMaxCols = kBlkCells + 2 * kMaxReach;                            // window columns
constexpr int kWinGrid = 2048;     // persistent workgroups (multiple of 8)

using COfs = const int (*)[kMaxOfs];

// LDS entry of a window particle: its staged fixed-point coordinates, and its
// type when there are two (12 or 16 bytes).
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

// Block rectangle from its first and last cells.
struct Rect {
    int xa, xb, y0, y1, z;
};

__device__ __forceinline__ Rect rect_of(const Geom &g, int c0, int c1)
{
    int nx = g.nc[0], ny = g.nc[1];
    Rect r;
    r.xa = c0 % nx;
    r.y0 = (c0 / nx) % ny;
    r.z = c0 / (nx * ny);
    r.xb = c1 % nx;
    r.y1 = (c1 / nx) % ny;
    return r;
}

// Columns [lo, ...] of the window of a block spanning xa..xb with reach r:
// ncols columns starting at lo, or the whole row (lo = 0, ncols = nx) when
// that is not longer.
__device__ __forceinline__ int window_columns(const Geom &g, int r, int xa, int xb, int &lo)
{
    int nx = g.nc[0];
    if (xb - xa + 1 + 2 * r >= nx) {
        lo = 0;
        return nx;
    }
    lo = xa - r;
    lo = lo < 0 ? lo + nx : lo;
    return xb - xa + 1 + 2 * r;
}

// Rows of a window for a block of nyb y-rows, reach r.  Row rr maps to the
// layer offset dz and y-row offset dy (relative to y0) of the cells it holds:
//   full window: layers z - r .. z + r, each with y-rows y0 - r .. y1 + r;
//   half window: layers z + 1 .. z + r with y-rows y0 - r .. y1 + r, then
//     layer z with y-rows y0 .. y1 + r (the own rows first).
// A particle in block row k (y = y0 + k) meets, in a half window, the rows
// of layers z + 1 .. z + r at y - r .. y + r, the rows y + 1 .. y + r of its
// own layer, and in its own row the columns x + 1 .. x + r and the particles
// after it in its own cell: half of the (2r + 1)^3 - 1 neighbour cells, so
// that every pair of distinct cells is seen from exactly one of its two cells
// (with at least 2r + 1 cells per dimension).
__device__ __forceinline__ int window_nrow(int r, int nyb, bool half)
{
    int span = nyb + 2 * r;
    return half ? r * span + nyb + r : (2 * r + 1) * span;
}

__device__ __forceinline__ void row_of(int r, int nyb, bool half, int rr, int &dz, int &dy)
{
    int span = nyb + 2 * r;
    if (!half) {
        dz = rr / span - r;
        dy = rr % span - r;
    } else if (rr < r * span) {
        dz = rr / span + 1;
        dy = rr % span - r;
    } else {
        dz = 0;
        dy = rr - r * span;
    }
}

// Window row of layer offset dz, y-row offset dy (relative to y0).
__device__ __forceinline__ int row_index(int r, int nyb, bool half, int dz, int dy)
{
    int span = nyb + 2 * r;
    if (!half) return (dz + r) * span + dy + r;
    return dz > 0 ? (dz - 1) * span + dy + r : r * span + dy;
}

__device__ __forceinline__ int wrap_dim(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }

// Window layout in LDS.  Column m of window row rr is cell column
// (lo + m) mod nx; its particles occupy window positions
// [col[rr][m], col[rr][m + 1]).  Piece k (two per row, the second empty
// unless the columns wrap) holds particles [pc_start[k], ...) at window
// positions [pc_win[k], pc_win[k + 1]).  The block's own particles are, per
// block row k, [ba[k], ba[k] + bpref[k + 1] - bpref[k]), threads
// bpref[k] .. bpref[k + 1] - 1.
struct Window {
    int nrow, ncols, lo, W, nyb, r, npart;
    Rect rc;
    int ba[kWinBlkRows], bpref[kWinBlkRows + 1];
    int pc_start[2 * kMaxRows];
    int pc_win[2 * kMaxRows + 1];
    uint16_t col[kMaxRows][kMaxCols + 1];
};

// Lay out the (full or half) window of block blk = (first cell, last cell,
// first particle, end particle; the particle range is -1 for blocks of whole
// cells).  The column table is filled only when COLS.  All threads take
// part; ends with a barrier.
template <bool HALF, bool COLS = true>
__device__ void make_window(const Geom &g, const int32_t *__restrict__ cs, int4 blk, Window &w)
{
    int nx = g.nc[0], ny = g.nc[1], nz = g.nc[2];
    int r = g.reach[0];
    Rect rc = rect_of(g, blk.x, blk.y);
    int nyb = rc.y1 - rc.y0 + 1;
    int lo;
    int ncols = window_columns(g, r, rc.xa, rc.xb, lo);
    int nrow = window_nrow(r, nyb, HALF);
    bool wrap = lo + ncols > nx;
    int x1a = wrap ? nx - 1 : lo + ncols - 1;  // last column of the first piece
    int t = threadIdx.x;
    if (t < nrow) {
        int dz, dy;
        row_of(r, nyb, HALF, t, dz, dy);
        int rb = (wrap_dim(rc.z + dz, nz) * ny + wrap_dim(rc.y0 + dy, ny)) * nx;
        int s0 = cs[rb + lo], e0 = cs[rb + x1a + 1];
        int s1 = cs[rb], e1 = wrap ? cs[rb + lo + ncols - nx] : s1;
        w.pc_start[2 * t] = s0;
        w.pc_start[2 * t + 1] = s1;
        w.pc_win[2 * t] = e0 - s0;  // lengths for now
        w.pc_win[2 * t + 1] = e1 - s1;
    } else if (t >= 64 && t < 64 + nyb) {
        int k = t - 64;
        if (blk.z >= 0) {  // a particle range (blocks of one row)
            w.ba[0] = blk.z;
            w.bpref[1] = blk.w - blk.z;
        } else {
            int rb = (rc.z * ny + rc.y0 + k) * nx;
            w.ba[k] = cs[rb + rc.xa];
            w.bpref[k + 1] = cs[rb + rc.xb + 1] - cs[rb + rc.xa];  // counts for now
        }
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
        w.nyb = nyb;
        w.r = r;
        w.rc = rc;
        int np = 0;
        w.bpref[0] = 0;
        for (int k = 0; k < nyb; k++) {
            np += w.bpref[k + 1];
            w.bpref[k + 1] = np;
        }
        w.npart = np;
    }
    __syncthreads();
    if (!COLS) return;
    int ncol0 = x1a - lo + 1;  // columns in the first piece
    for (int e = t; e < nrow * (ncols + 1); e += blockDim.x) {
        int rr = e / (ncols + 1), m = e - rr * (ncols + 1);
        int v;
        if (m == ncols) {
            v = w.pc_win[2 * rr + 2];
        } else {
            int dz, dy;
            row_of(r, nyb, HALF, rr, dz, dy);
            int rb = (wrap_dim(rc.z + dz, nz) * ny + wrap_dim(rc.y0 + dy, ny)) * nx;
            if (m < ncol0)
                v = w.pc_win[2 * rr] + cs[rb + lo + m] - w.pc_start[2 * rr];
            else
                v = w.pc_win[2 * rr + 1] + cs[rb + m - ncol0] - w.pc_start[2 * rr + 1];
        }
        w.col[rr][m] = (uint16_t)v;
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

// Single-precision build windows.  A window particle's coordinates relative
// to its block's centre, in x units (u = L_x / 2^32; y and z scaled by
// L_y / L_x and L_z / L_x), so that a candidate distance costs three float
// subtractions instead of three integer subtractions and conversions.  The
// offset to the centre is the true one when no window spans a whole periodic
// dimension (build_float_ok); its rounding (at most 2^-24 of a window
// extent) is far inside the build's guard band kBuildBand.
struct FEntry {
    float x, y, z;
};

constexpr float kBuildBand = 1.0f / 32768.0f;

// Block centre in fixed point (cell units times 2^32 / nc).
__device__ __forceinline__ void block_centre(const Geom &g, const Rect &rc, uint32_t &ox, uint32_t &oy, uint32_t &oz)
{
    ox = (uint32_t)((((uint64_t)(rc.xa + rc.xb + 1)) << 31) / (uint64_t)g.nc[0]);
    oy = (uint32_t)((((uint64_t)(rc.y0 + rc.y1 + 1)) << 31) / (uint64_t)g.nc[1]);
    oz = (uint32_t)((((uint64_t)(2 * rc.z + 1)) << 31) / (uint64_t)g.nc[2]);
}

__device__ __forceinline__ FEntry to_rel(const int4 &a, uint32_t ox, uint32_t oy, uint32_t oz, float ry, float rz)
{
    FEntry e;
    e.x = (float)(int)((uint32_t)a.x - ox);
    e.y = (float)(int)((uint32_t)a.y - oy) * ry;
    e.z = (float)(int)((uint32_t)a.z - oz) * rz;
    return e;
}

// Stage the window as FEntry (as load_window, four loads in flight).
__device__ __forceinline__ void load_window_rel(const Geom &g, const Window &w, const int4 *__restrict__ st,
                                                FEntry *lds)
{
    uint32_t ox, oy, oz;
    block_centre(g, w.rc, ox, oy, oz);
    float ry = g.ry, rz = g.rz;
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
        lds[p0] = to_rel(a0, ox, oy, oz, ry, rz);
        if (p1 < W) lds[p1] = to_rel(a1, ox, oy, oz, ry, rz);
        if (p2 < W) lds[p2] = to_rel(a2, ox, oy, oz, ry, rz);
        if (p3 < W) lds[p3] = to_rel(a3, ox, oy, oz, ry, rz);
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

// The particle of this thread in the block: its index i, block row k and
// cell column x; false if the thread has none.
__device__ __forceinline__ bool my_particle(const Geom &g, const Window &w, const int32_t *__restrict__ cell_sorted,
                                            int &i, int &k, int &x, int t = threadIdx.x)
{
    if (t >= w.npart) return false;
    k = 0;
    while (k + 1 < w.nyb && w.bpref[k + 1] <= t) k++;
    i = w.ba[k] + (t - w.bpref[k]);
    x = cell_sorted[i] % g.nc[0];
    return true;
}

// Window column of cell column x.
__device__ __forceinline__ int column_of(const Geom &g, const Window &w, int x)
{
    int m = x - w.lo;
    return m < 0 ? m + g.nc[0] : m;
}

// Window position of particle i (in block row k, cell column x) itself.
template <bool HALF>
__device__ __forceinline__ int self_position(const Window &w, const int32_t *__restrict__ cs, int i, int k,
                                             int m, int cell)
{
    int own = row_index(w.r, w.nyb, HALF, 0, k);
    return w.col[own][m] + (i - cs[cell]);
}

// The window columns of cell columns x + a .. x + b (a <= b, |a|, |b| <= r)
// as up to two contiguous ranges [a0, b0], [a1, b1] (b < a: empty): one
// range unless they wrap inside a window that covers the whole x-row.
struct ColRanges {
    int a0, b0, a1, b1;
};

__device__ __forceinline__ ColRanges column_ranges(const Geom &g, const Window &w, int x, int a, int b)
{
    int nx = g.nc[0];
    ColRanges cr{0, -1, 0, -1};
    if (w.ncols < nx) {
        int m = column_of(g, w, x);
        cr.a0 = m + a;
        cr.b0 = m + b;
        return cr;
    }
    int lo = x + a, hi = x + b;  // whole row: lo = 0, column m = cell column
    if (lo >= nx) {
        lo -= nx;
        hi -= nx;
    } else if (hi < 0) {
        lo += nx;
        hi += nx;
    }
    if (lo >= 0 && hi < nx) {
        cr.a0 = lo;
        cr.b0 = hi;
    } else if (lo < 0) {
        cr.a0 = 0;
        cr.b0 = hi;
        cr.a1 = lo + nx;
        cr.b1 = nx - 1;
    } else {
        cr.a0 = lo;
        cr.b0 = nx - 1;
        cr.a1 = 0;
        cr.b1 = hi - nx;
    }
    return cr;
}

// ------------------------------------------------------------------ block partition

// Particles of the window rows of band e (layer z, y-rows bi * band ..) in
// column x: the window of a block spanning columns xa..xb of the band is the
// sum over its window columns.
template <bool HALF>
__device__ __forceinline__ int band_column_sum(const Geom &g, const int32_t *__restrict__ cs, int e, int x)
{
    int nx = g.nc[0], ny = g.nc[1], nz = g.nc[2];
    int band = g.wband, nby = (ny + band - 1) / band;
    int bi = e % nby, z = e / nby;
    int r = g.reach[0];
    int y0 = bi * band, nyb = min(band, ny - y0);
    int nrow = window_nrow(r, nyb, HALF);
    int s = 0;
    for (int rr = 0; rr < nrow; rr++) {
        int dz, dy;
        row_of(r, nyb, HALF, rr, dz, dy);
        int cell = (wrap_dim(z + dz, nz) * ny + wrap_dim(y0 + dy, ny)) * nx + x;
        s += cs[cell + 1] - cs[cell];
    }
    return s;
}

// Greedy packing of one band, by one wavefront: the band's column data is
// staged in LDS, then lane 0 cuts the band into blocks.  A block grows while
// it holds <= 256 particles, spans at most kBlkCells columns and its window
// fits the LDS tile (wmax positions).  Bands of one row are cut at particle
// granularity (a block may start and end inside a cell, so that most blocks
// hold exactly 256 particles and fill four wavefronts); bands of several rows
// are cut at whole columns.  Blocks nb with base + nb < cap are written (if
// emit).  A single column whose window cannot be held reports flags[3].
constexpr int kPackMaxX = 4096;

template <bool HALF>
__device__ int pack_band(int e, const Geom &g, const int32_t *__restrict__ cs, int base, int4 *blocks, bool emit,
                         int cap, int32_t *flags, int wmax, int *scol, int *snum, int *sst)
{
    int nx = g.nc[0], ny = g.nc[1];
    int band = g.wband, nby = (ny + band - 1) / band;
    int bi = e % nby, z = e / nby;
    int y0 = bi * band, y1 = min(ny, y0 + band) - 1;
    int r = g.reach[0];
    bool one_row = y0 == y1;
    for (int x = threadIdx.x; x < nx; x += blockDim.x) {
        scol[x] = band_column_sum<HALF>(g, cs, e, x);
        int m = 0;
        for (int y = y0; y <= y1; y++) {
            int c = (z * ny + y) * nx + x;
            m += cs[c + 1] - cs[c];
        }
        snum[x] = m;
        sst[x] = cs[(z * ny + y0) * nx + x];
    }
    __syncthreads();
    int nb = 0;
    if (threadIdx.x == 0) {
        int rowsum = 0;
        for (int x = 0; x < nx; x++) rowsum += scol[x];
        auto col = [&](int k) { return scol[k < 0 ? k + nx : (k >= nx ? k - nx : k)]; };
        auto window_of = [&](int xa, int xb) {
            if (xb - xa + 1 + 2 * r >= nx) return rowsum;
            int s = 0;
            for (int k = xa - r; k <= xb + r; k++) s += col(k);
            return s;
        };
        int bs = -1, bp = 0, bx0 = 0, bxl = 0, bw = 0;  // open block: first particle, particles, x range, window
        auto close = [&]() {
            if (bs >= 0 && bp > 0) {
                if (emit && base + nb < cap)
                    blocks[base + nb] = make_int4((z * ny + y0) * nx + bx0, (z * ny + y1) * nx + bxl,
                                                  one_row ? bs : -1, one_row ? bs + bp : -1);
                nb++;
            }
            bs = -1;
            bp = 0;
        };
        for (int x = 0; x < nx; x++) {
            int m = snum[x];
            int off = 0;  // particles of column x already in blocks
            while (off < m) {
                if (bs >= 0 && x > bxl) {
                    // extend the window from [bx0, bxl] to [bx0, x]: columns bxl + r + 1 .. x + r
                    int w2;
                    if (x - bx0 + 1 + 2 * r >= nx) {
                        w2 = rowsum;
                    } else {
                        w2 = bw;
                        for (int k = bxl + r + 1; k <= x + r; k++) w2 += col(k);
                    }
                    bool fits = x - bx0 < kBlkCells && w2 <= wmax && (one_row || bp + m <= 256);
                    if (fits) {
                        bw = w2;
                        bxl = x;
                    } else {
                        close();
                    }
                }
                if (bs < 0) {
                    bs = sst[x] + off;
                    bx0 = bxl = x;
                    bw = window_of(x, x);
                    if (emit && (bw > wmax || (!one_row && m > 256))) atomicOr(&flags[3], 1);
                }
                int take = one_row ? min(m - off, 256 - bp) : m;
                bp += take;
                off += take;
                if (one_row && bp == 256) close();
            }
        }
        close();
    }
    return nb;
}

// The three per-column LDS arrays of the packer are sized at launch: 3 nx ints.
// The counting pass also writes the first kBandCap blocks of its band to
// staging (slots e * kBandCap ..); the writing pass copies them to their
// final places, and packs again only a band with more blocks.
constexpr int kBandCap = 16;

template <bool HALF>
__global__ void k_blk_count(const Geom g, const int32_t *__restrict__ cs, int32_t *__restrict__ band_n,
                            int4 *__restrict__ staged, int32_t *flags, int wmax)
{
    extern __shared__ int pack_lds[];
    int *scol = pack_lds, *snum = pack_lds + g.nc[0], *sst = pack_lds + 2 * g.nc[0];
    int e = blockIdx.x;
    int nb = pack_band<HALF>(e, g, cs, e * kBandCap, staged, true, (e + 1) * kBandCap, flags, wmax, scol, snum,
                             sst);
    if (threadIdx.x == 0) band_n[e] = nb;
}

template <bool HALF>
__global__ void k_blk_write(const Geom g, const int32_t *__restrict__ cs, const int32_t *__restrict__ band_n,
                            const int32_t *__restrict__ band_base, const int4 *__restrict__ staged, int4 *blocks,
                            int cap, int32_t *flags, int wmax)
{
    extern __shared__ int pack_lds[];
    int *scol = pack_lds, *snum = pack_lds + g.nc[0], *sst = pack_lds + 2 * g.nc[0];
    int e = blockIdx.x;
    int nb = band_n[e], base = band_base[e];
    if (nb <= kBandCap) {
        for (int j = threadIdx.x; j < nb; j += blockDim.x)
            if (base + j < cap) blocks[base + j] = staged[e * kBandCap + j];
    } else {
        pack_band<HALF>(e, g, cs, base, blocks, true, cap, flags, wmax, scol, snum, sst);
    }
}

// A staged position at least r_c + skin from every particle of the block
// (blk: its descriptor): half the box away in z from the centre of the
// block's z layer of cells.  The particles of the block lie within half a
// cell of that centre, and a box holds at least three cells per dimension,
// so every one of them is at least a cell side (>= r_c + skin) from it.
__device__ __forceinline__ int4 far_entry(const Geom &g, int4 blk)
{
    int zc = blk.x / (g.nc[0] * g.nc[1]);
    uint32_t centre = (uint32_t)((((uint64_t)(2 * zc + 1)) << 31) / (uint64_t)g.nc[2]);
    return make_int4(0, 0, (int)(centre + 0x80000000u), 0);
}

// Common head of the windowed kernels: lay out and stage the window of a
// block; false (uniformly) if it does not fit the tile.  FAR: also stage
// far_entry at position kWinMax (the padding of the full Verlet lists).
template <int NT, bool HALF = false, bool COLS = true, bool FAR = false>
__device__ __forceinline__ bool setup_block(const Geom &g, const int32_t *__restrict__ cs, const int4 *__restrict__ st,
                                            int4 blk, Window &w, WinEntry<NT> *win, int32_t *flags)
{
    __syncthreads();
    make_window<HALF, COLS>(g, cs, blk, w);
    if (w.W > (HALF ? kWinMaxHalf : kWinMax) || w.npart > 256) {  // never made by the packer
        if (threadIdx.x == 0) atomicOr(&flags[3], 2);
        return false;
    }
    load_window(w, st, win);
    if (FAR && threadIdx.x == 0) win[kWinMax].set(far_entry(g, blk));
    __syncthreads();
    return true;
}

// setup_block for the single-precision build windows.
template <bool HALF>
__device__ __forceinline__ bool setup_block_rel(const Geom &g, const int32_t *__restrict__ cs,
                                                const int4 *__restrict__ st, int4 blk, Window &w, FEntry *win,
                                                int32_t *flags)
{
    __syncthreads();
    make_window<HALF>(g, cs, blk, w);
    if (w.W > (HALF ? kWinMaxHalf : kWinMax) || w.npart > 256) {  // never made by the packer
        if (threadIdx.x == 0) atomicOr(&flags[3], 2);
        return false;
    }
    load_window_rel(g, w, st, win);
    __syncthreads();
    return true;
}

// Every candidate range of window positions of the particle in block row k,
// cell column x (window position self): the full stencil, or its forward
// half (see row_of).  fn(b, en) is called per contiguous range [b, en).
template <bool HALF, typename Fn>
__device__ __forceinline__ void stencil_ranges(const Geom &g, const Window &w, int k, int x, int self, Fn &&fn)
{
    int r = w.r, nyb = w.nyb;
    ColRanges cr = column_ranges(g, w, x, -r, r);
    auto row = [&](int rr) {
        fn((int)w.col[rr][cr.a0], (int)w.col[rr][cr.b0 + 1]);
        if (cr.b1 >= cr.a1) fn((int)w.col[rr][cr.a1], (int)w.col[rr][cr.b1 + 1]);
    };
    if (!HALF) {
        for (int dz = -r; dz <= r; dz++)
            for (int dy = -r; dy <= r; dy++) row(row_index(r, nyb, false, dz, k + dy));
    } else {
        for (int dz = 1; dz <= r; dz++)
            for (int dy = -r; dy <= r; dy++) row(row_index(r, nyb, true, dz, k + dy));
        for (int dy = 1; dy <= r; dy++) row(row_index(r, nyb, true, 0, k + dy));
        int own = row_index(r, nyb, true, 0, k);
        int m = column_of(g, w, x);
        fn(self + 1, (int)w.col[own][m + 1]);
        ColRanges cf = column_ranges(g, w, x, 1, r);
        fn((int)w.col[own][cf.a0], (int)w.col[own][cf.b0 + 1]);
        if (cf.b1 >= cf.a1) fn((int)w.col[own][cf.a1], (int)w.col[own][cf.b1 + 1]);
    }
}

// First position p in [b, e) of an x-ordered run of a build window with
// x >= t (e if none).
__device__ __forceinline__ int first_at_least(const FEntry *__restrict__ win, int b, int e, float t)
{
    while (b < e) {
        int m = (b + e) >> 1;
        if (win[m].x < t)
            b = m + 1;
        else
            e = m;
    }
    return b;
}

// First position p in [b, e) with x > t.
__device__ __forceinline__ int first_above(const FEntry *__restrict__ win, int b, int e, float t)
{
    while (b < e) {
        int m = (b + e) >> 1;
        if (win[m].x <= t)
            b = m + 1;
        else
            e = m;
    }
    return b;
}

// stencil_ranges for the single-precision build windows, each range cut to
// the candidates that can lie within the list radius.  Every cell is ordered
// by x (launch_scatter_sort_x) and a range is a run of consecutive cells
// along x, so it is ordered by x.  A row of cells at layer offset dz and row
// offset dy lies at least gy from the particle in y and gz in z (0 for its
// own row and layer), so its candidates within the radius have
// |dx| < sqrt(rl2 - gy^2 - gz^2); the range is cut to that interval by
// bisection.  The gaps are shrunk and the interval widened by 2^-10 of the
// cell size and the radius, far beyond the rounding of the relative
// coordinates, so that no candidate whose FP32 distance passes the list test
// (or falls in its guard band) is cut: the lists are the same as those of the
// uncut ranges.  rl2: the radius squared in relative units (the upper edge of
// the build's band); hy, hz: the cell height and depth in the same units.
template <bool HALF, typename Fn>
__device__ __forceinline__ void stencil_ranges_cut(const Geom &g, const Window &w, const FEntry *__restrict__ win,
                                                   const FEntry &pf, int k, int x, int self, float rl2, float hy,
                                                   float hz, Fn &&fn)
{
    constexpr float kMargin = 1.0f / 1024.0f;
    int r = w.r, nyb = w.nyb;
    // the particle's own cell in relative units: y in [ylo, ylo + hy) (block
    // row k of nyb, the centre in the middle of the rows), z in [-hz/2, hz/2)
    float ylo = ((float)k - 0.5f * (float)nyb) * hy, zlo = -0.5f * hz;
    float py = pf.y - ylo, pz = pf.z - zlo;  // offsets inside the own cell
    auto gap = [&](int d, float p, float h) {
        float v = d < 0 ? p + (float)(-d - 1) * h : (d > 0 ? (float)d * h - p : 0.0f);
        return fmaxf(v - kMargin * h, 0.0f);
    };
    const float rlm = rl2 * (1.0f + kMargin);
    auto cut = [&](int b, int e, int dz, int dy) {
        if (b >= e) return;
        float gy = gap(dy, py, hy), gz = gap(dz, pz, hz);
        float rx2 = rlm - gy * gy - gz * gz;
        if (rx2 <= 0.0f) return;
        float rx = sqrtf(rx2) * (1.0f + kMargin);
        int lb = first_at_least(win, b, e, pf.x - rx);
        int ub = first_above(win, lb, e, pf.x + rx);
        if (lb < ub) fn(lb, ub);
    };
    // one contiguous range per row: these windows never span a whole row
    int m = column_of(g, w, x);
    auto row = [&](int dz, int dy) {
        int rr = row_index(r, nyb, HALF, dz, k + dy);
        cut((int)w.col[rr][m - r], (int)w.col[rr][m + r + 1], dz, dy);
    };
    if (!HALF) {
        for (int dz = -r; dz <= r; dz++)
            for (int dy = -r; dy <= r; dy++) row(dz, dy);
    } else {
        for (int dz = 1; dz <= r; dz++)
            for (int dy = -r; dy <= r; dy++) row(dz, dy);
        for (int dy = 1; dy <= r; dy++) row(0, dy);
        int own = row_index(r, nyb, true, 0, k);
        cut(self + 1, (int)w.col[own][m + 1], 0, 0);
        cut((int)w.col[own][m + 1], (int)w.col[own][m + r + 1], 0, 0);
    }
}

// First position p in [b, e) of a force window with x_p - xi >= t (staged
// units, minimum image), and the first with x_p - xi > t.
template <int NT>
__device__ __forceinline__ int first_at_least_i(const WinEntry<NT> *__restrict__ win, int b, int e, uint32_t xi,
                                                int t)
{
    while (b < e) {
        int m = (b + e) >> 1;
        if ((int)((uint32_t)win[m].x - xi) < t)
            b = m + 1;
        else
            e = m;
    }
    return b;
}

template <int NT>
__device__ __forceinline__ int first_above_i(const WinEntry<NT> *__restrict__ win, int b, int e, uint32_t xi, int t)
{
    while (b < e) {
        int m = (b + e) >> 1;
        if ((int)((uint32_t)win[m].x - xi) <= t)
            b = m + 1;
        else
            e = m;
    }
    return b;
}

// Whether the force windows' stencil rows can be cut by x: at least 2r + 3
// cells per dimension, so that a row's minimum-image x differences to the
// particle are ordered along the row (they span less than half the box) and
// a neighbour row's nearest image is the one beside the particle's cell.
__device__ __forceinline__ bool can_cut(const Geom &g, int r)
{
    return g.nc[0] >= 2 * r + 3 && g.nc[1] >= 2 * r + 3 && g.nc[2] >= 2 * r + 3;
}

// stencil_ranges for the linked-cell force windows, each range cut to the
// candidates that can lie within the cutoff.  The cells were ordered by x at
// the last build (launch_scatter_sort_x) and every particle has since moved
// by at most the skin check's bound d (half the skin: a step whose particles
// moved further is redone after a rebuild), so along a stencil row the
// current x coordinates are ordered up to 2d.  A bisection that stops at p
// with x_{p-1} - xi < t has seen an entry below t, so every particle before p
// lies below t + 2d (and symmetrically at the upper end): the cut interval is
// widened by 2d on each side.  The y and z gaps to a neighbour row are taken
// from the row's cells as built, less d for its particles' motion; 2^-10 of
// a cell and of the radius are added to every margin, far beyond the
// rounding, so that no pair within the upper edge of the cutoff's guard band
// is cut.  rc2: that edge squared (x units); drift: d in x units.
template <int NT, typename Fn>
__device__ __forceinline__ void stencil_ranges_drift(const Geom &g, const Window &w,
                                                     const WinEntry<NT> *__restrict__ win, const int4 &pi, int k,
                                                     int x, float rc2, float drift, Fn &&fn)
{
    constexpr float kMargin = 1.0f / 1024.0f;
    int r = w.r, nyb = w.nyb;
    ColRanges cr = column_ranges(g, w, x, -r, r);
    // the particle's offsets from the low corner of its cell as built, in x units
    int cy = w.rc.y0 + k, cz = w.rc.z;
    uint32_t y0 = (uint32_t)(((uint64_t)cy << 32) / (uint64_t)g.nc[1]);
    uint32_t z0 = (uint32_t)(((uint64_t)cz << 32) / (uint64_t)g.nc[2]);
    float py = (float)(int)((uint32_t)pi.y - y0) * g.ry, pz = (float)(int)((uint32_t)pi.z - z0) * g.rz;
    float hy = 4294967296.0f / (float)g.nc[1] * g.ry, hz = 4294967296.0f / (float)g.nc[2] * g.rz;
    auto gap = [&](int d, float p, float h) {
        float v = d < 0 ? p + (float)(-d - 1) * h : (d > 0 ? (float)d * h - p : 0.0f);
        return fmaxf(v - drift - kMargin * h, 0.0f);
    };
    const float rcm = rc2 * (1.0f + kMargin);
    const float wide = 2.0f * drift * (1.0f + kMargin);
    uint32_t xi = (uint32_t)pi.x;
    auto cut = [&](int b, int e, int dz, int dy) {
        if (b >= e) return;
        float gy = gap(dy, py, hy), gz = gap(dz, pz, hz);
        float rx2 = rcm - gy * gy - gz * gz;
        if (rx2 <= 0.0f) return;
        float rx = sqrtf(rx2) * (1.0f + kMargin) + wide;
        int t = (int)ceilf(rx);
        int lb = first_at_least_i(win, b, e, xi, -t);
        int ub = first_above_i(win, lb, e, xi, t);
        if (lb < ub) fn(lb, ub);
    };
    for (int dz = -r; dz <= r; dz++)
        for (int dy = -r; dy <= r; dy++) {
            int rr = row_index(r, nyb, false, dz, k + dy);
            cut((int)w.col[rr][cr.a0], (int)w.col[rr][cr.b0 + 1], dz, dy);
            if (cr.b1 >= cr.a1) cut((int)w.col[rr][cr.a1], (int)w.col[rr][cr.b1 + 1], dz, dy);
        }
}

// One candidate pair (i, window position p) of the gather traversals, branch
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
                                           const Geom &g, const double *__restrict__ pos, int n, float &fx,
                                           float &fy, float &fz, float &eu, float &ew, int &np)
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

// Cutoff prefilter of the linked-cell traversals: window positions q[0 ..
// m-1], m <= 32, tested against the largest upper guard-band edge of the
// cutoffs; returns the mask of the candidates below it (candidate u at bit
// m - 1 - u).  Reads whole groups of four, up to three positions past the
// batch (the window arrays are padded for them); their bits are dropped.
template <int NT, bool ISO>
__device__ __forceinline__ uint32_t cut_batch(const int4 &pi, const WinEntry<NT> *__restrict__ q, int m,
                                              const Geom &g, float hi)
{
    uint32_t mask = 0;
    int nb = 0;
    auto test = [&](const WinEntry<NT> &e) {
        float dx, dy, dz;
        staged_delta<ISO>(pi, e.get(), g, dx, dy, dz);
        float r2 = dx * dx + dy * dy + dz * dz;
        mask = mask + mask + (r2 < hi ? 1u : 0u);
    };
    for (; nb < m; nb += 4) {
        test(q[nb]);
        test(q[nb + 1]);
        test(q[nb + 2]);
        test(q[nb + 3]);
    }
    return mask >> (nb - m);
}

template <int NT>
__device__ __forceinline__ float max_hi(const TabF<NT> &t)
{
    float h = t.hi[0];
    for (int k = 1; k < NT * NT; k++) h = fmaxf(h, t.hi[k]);
    return h;
}

// Each thread scans the window ranges of its stencil (cut by x when the box
// allows it, stencil_ranges_drift) 32 candidates at a time: a cheap distance
// test gives the mask of those that may interact, and only they are
// evaluated (guard-band pairs decided from the FP64 positions).
template <int NT, bool ISO, bool ENERGY>
__global__ __launch_bounds__(256) void k_lcw_f32(const int4 *__restrict__ st, const int32_t *__restrict__ cs,
                                                 const int32_t *__restrict__ cell_sorted, Geom g, int n,
                                                 const int32_t *__restrict__ nblk_p, int cap,
                                                 const int4 *__restrict__ blocks,
                                                 const PairTab *__restrict__ tabp, const double *__restrict__ pos,
                                                 float *__restrict__ F, double *__restrict__ partials,
                                                 int32_t *__restrict__ flags)
{
    __shared__ WinEntry<NT> win[kWinMax + 4];  // + the reads past a batch
    __shared__ Window w;
    __shared__ double sh[16];
    TabF<NT> t;
    t.load(tabp);
    const float hi = max_hi(t);
    // the motion allowed since the build (no bound without a skin)
    const float drift = sqrtf(g.disp2);
    const bool cut = can_cut(g, g.reach[0]) && drift < 1.0e30f;
    float eu = 0.f, ew = 0.f;
    int np = 0;
    size_t N = (size_t)n;
    for (BlockIter it(min(*nblk_p, cap)); it.blk < it.end; it.blk += it.stride) {
        int blk = it.blk;
        if (!setup_block<NT>(g, cs, st, blocks[blk], w, win, flags)) continue;
        int i, k, x;
        if (!my_particle(g, w, cell_sorted, i, k, x)) continue;
        int self = self_position<false>(w, cs, i, k, column_of(g, w, x), cell_sorted[i]);
        int4 pi = win[self].get();
        float fx = 0.f, fy = 0.f, fz = 0.f;
        auto batches = [&](int b, int en) {
            for (int base = b; base < en; base += 32) {
                int m = min(32, en - base);
                uint32_t mask = cut_batch<NT, ISO>(pi, win + base, m, g, hi);
                unsigned us = (unsigned)(self - base);
                if (us < (unsigned)m) mask &= ~(1u << (m - 1 - us));
                while (mask) {
                    int h = 31 - __builtin_clz(mask);
                    mask ^= 1u << h;
                    int p = base + m - 1 - h;
                    int4 pj = win[p].get();
                    if (pair_fast<NT, ISO, ENERGY>(pi, pj, true, t, g, fx, fy, fz, eu, ew, np))
                        pair_exact<NT, ISO, ENERGY>(pi, pj, i, window_global(w, p), t, g, pos, n, fx, fy, fz, eu,
                                                    ew, np);
                }
            }
        };
        if (cut)
            stencil_ranges_drift<NT>(g, w, win, pi, k, x, hi, drift, batches);
        else
            stencil_ranges<false>(g, w, k, x, self, batches);
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

// ------------------------------------------------------------------ adjoint

// The pair constants of particle i's type against each partner type (the
// adjoint picks them per pair by the partner's type alone).
struct AdjParams {
    float lo[2], hi[2], eps[2], ieps[2], sig2[2], c144[2];
    double rc2[2];
    template <int NT>
    __device__ __forceinline__ void load(const PairTab *__restrict__ tabp, int ti)
    {
        for (int tj = 0; tj < NT; tj++) {
            int ab = ti * NT + tj;
            lo[tj] = tabp->rc2_lo[ab];
            hi[tj] = tabp->rc2_hi[ab];
            rc2[tj] = tabp->rc2[ab];
            float e = (float)tabp->eps[ab], sg = (float)tabp->sig[ab];
            eps[tj] = e;
            ieps[tj] = 1.0f / e;
            sig2[tj] = sg * sg;
            c144[tj] = 144.0f * e / sg;
        }
    }
};

// The adjoint terms of one pair within the cutoff (Sec. 2.1's force f_ij =
// phi(r) d, differentiated): with dg = g_i - g_j, the position gradient of
// i gains phi dg + 2 phi'(r^2) (d . dg) d, and the parameter gradients of the
// partner type (t1: the second type) gain (dphi/d eps, dphi/d sigma) (d . dg).
// d in fixed-point units (scaled here by uf), sums in FP64.
__device__ __forceinline__ void adj_pair(float dx, float dy, float dz, float uf, bool t1, float dgx, float dgy,
                                         float dgz, const AdjParams &pp, double &ax, double &ay, double &az,
                                         double &ge0, double &ge1, double &gs0, double &gs1)
{
    dx *= uf;
    dy *= uf;
    dz *= uf;
    float r2 = dx * dx + dy * dy + dz * dz;
    float eps = t1 ? pp.eps[1] : pp.eps[0];
    float ir2 = __builtin_amdgcn_rcpf(r2);
    float s2 = (t1 ? pp.sig2[1] : pp.sig2[0]) * ir2;
    float q = s2 * s2 * s2;
    float phi = 24.0f * eps * ir2 * q * (2.0f * q - 1.0f);
    float dphi = -48.0f * eps * ir2 * ir2 * q * (7.0f * q - 2.0f);
    float ddg = dx * dgx + dy * dgy + dz * dgz;
    float k2 = 2.0f * dphi * ddg;
    ax += (double)(phi * dgx + k2 * dx);
    ay += (double)(phi * dgy + k2 * dy);
    az += (double)(phi * dgz + k2 * dz);
    double de = (double)(phi * (t1 ? pp.ieps[1] : pp.ieps[0]) * ddg);
    double ds = (double)((t1 ? pp.c144[1] : pp.c144[0]) * ir2 * q * (4.0f * q - 1.0f) * ddg);
    ge0 += t1 ? 0.0 : de;
    ge1 += t1 ? de : 0.0;
    gs0 += t1 ? 0.0 : ds;
    gs1 += t1 ? ds : 0.0;
}

// Adjoint of the forces (the differentiable extension) over the gather
// windows, FP32 pairs: each thread gathers its particle's row
//   dL/dx_i = sum_j J_ij (g_i - g_j),  J = phi I + 2 (dphi/dr2) d d^T,
// from its stencil ranges (cut by x where the box allows it, as in the
// linked-cell force; the cutoff prefilter, then the pair terms for the
// survivors only, guard-band pairs decided from the FP64 positions; g_j read
// from global memory).  The pair parameters are picked per pair by the
// partner's type alone (this particle's type fixes the rest).  The parameter
// terms
//   (phi/eps_ab) d.(g_i - g_j),  144 eps q (4q - 1)/(sig r^2) d.(g_i - g_j)
// are seen from both sides of each pair and halved when the per-workgroup
// partials are summed.  FP64 accumulation of the gradient and the parameter
// terms; 1/r^2 by the hardware reciprocal.  (Four or two threads per
// particle, to occupy the GPU better on small systems, measured slower.)
template <int NT, bool ISO>
__global__ __launch_bounds__(256) void k_adjw_f32(
    const int4 *__restrict__ st, const int32_t *__restrict__ cs, const int32_t *__restrict__ cell_sorted, Geom g,
    int n, const int32_t *__restrict__ nblk_p, int cap, const int4 *__restrict__ blocks,
    const PairTab *__restrict__ tabp, const double *__restrict__ pos, const float *__restrict__ G,
    double *__restrict__ grad_pos, double *__restrict__ gpart, int32_t *__restrict__ flags, int only_if_overflow)
{
    // behind the list adjoint: the work is this kernel's only when the lists
    // may be truncated (the overflow flag is set), and then the list kernel
    // did none (a uniform exit either way)
    if (only_if_overflow && !(flags[0] & (int)MD_FLAG_LIST_OVERFLOW)) return;
    __shared__ WinEntry<NT> win[kWinMax + 4];  // + the reads past a batch
    __shared__ Window w;
    __shared__ double sh[8][256 / 64];
    float hmax = 0.f;
    for (int k = 0; k < NT * NT; k++) hmax = fmaxf(hmax, tabp->rc2_hi[k]);
    // stencil rows cut by x as in the linked-cell force (stencil_ranges_drift)
    const float drift = sqrtf(g.disp2);
    const bool cut = can_cut(g, g.reach[0]) && drift < 1.0e30f;
    const float uf = (float)(g.L[0] / 4294967296.0);
    double gp[8] = {0, 0, 0, 0, 0, 0, 0, 0};  // eps_ab[4], sig_ab[4]
    size_t N = (size_t)n;
    for (BlockIter it(min(*nblk_p, cap)); it.blk < it.end; it.blk += it.stride) {
        int blk = it.blk;
        if (!setup_block<NT>(g, cs, st, blocks[blk], w, win, flags)) continue;
        int i, k, x;
        if (!my_particle(g, w, cell_sorted, i, k, x)) continue;
        double ax = 0.0, ay = 0.0, az = 0.0;
        {
            int self = self_position<false>(w, cs, i, k, column_of(g, w, x), cell_sorted[i]);
            int4 pi = win[self].get();
            float gix = G[i], giy = G[N + i], giz = G[2 * N + i];
            // the pair parameters for this particle's type against each
            // partner type (picked per pair by the partner's type alone)
            const int ti = NT == 1 ? 0 : pi.w;
            AdjParams pp;
            pp.load<NT>(tabp, ti);
            const float *lo_ = pp.lo, *hi_ = pp.hi;
            const double *rc2_ = pp.rc2;
            // parameter terms per partner type (FP64)
            double ge0 = 0.0, ge1 = 0.0, gs0 = 0.0, gs1 = 0.0;
            auto batches = [&](int b, int en) {
                // global index of window position p: the range lies in one
                // row, so in its first piece or the one after it
                int k0 = piece_from(w, 0, b);
                int split = k0 + 1 < 2 * w.nrow ? w.pc_win[k0 + 1] : INT_MAX;
                int off0 = w.pc_start[k0] - w.pc_win[k0];
                int off1 = k0 + 1 < 2 * w.nrow ? w.pc_start[k0 + 1] - w.pc_win[k0 + 1] : 0;
                for (int base = b; base < en; base += 32) {
                    int m = min(32, en - base);
                    uint32_t mask = cut_batch<NT, ISO>(pi, win + base, m, g, hmax);
                    unsigned us = (unsigned)(self - base);
                    if (us < (unsigned)m) mask &= ~(1u << (m - 1 - us));
                    while (mask) {
                        int h = 31 - __builtin_clz(mask);
                        mask ^= 1u << h;
                        int p = base + m - 1 - h;
                        int j = p + (p < split ? off0 : off1);
                        float gjx = G[j], gjy = G[N + j], gjz = G[2 * N + j];
                        int4 pj = win[p].get();
                        bool t1 = NT > 1 && pj.w != 0;
                        float dx, dy, dz;
                        staged_delta<ISO>(pi, pj, g, dx, dy, dz);
                        float r2u = dx * dx + dy * dy + dz * dz;
                        if (!within(r2u, t1 ? lo_[1] : lo_[0], t1 ? hi_[1] : hi_[0], t1 ? rc2_[1] : rc2_[0], pos, n,
                                    i, j, g))
                            continue;
                        adj_pair(dx, dy, dz, uf, t1, gix - gjx, giy - gjy, giz - gjz, pp, ax, ay, az, ge0, ge1, gs0,
                                 gs1);
                    }
                }
            };
            if (cut)
                stencil_ranges_drift<NT>(g, w, win, pi, k, x, hmax, drift, batches);
            else
                stencil_ranges<false>(g, w, k, x, self, batches);
            gp[ti * NT] += ge0;
            gp[4 + ti * NT] += gs0;
            if (NT > 1) {
                gp[ti * NT + 1] += ge1;
                gp[4 + ti * NT + 1] += gs1;
            }
        }
        grad_pos[i] = ax;
        grad_pos[N + i] = ay;
        grad_pos[2 * N + i] = az;
    }
    // the workgroup's parameter sums, fixed order
#pragma unroll
    for (int q = 0; q < 8; q++)
        for (int off = 32; off > 0; off >>= 1) gp[q] += __shfl_down(gp[q], off, 64);
    __syncthreads();
    int wv = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0)
        for (int q = 0; q < 8; q++) sh[q][wv] = gp[q];
    __syncthreads();
    if (threadIdx.x < 8) {
        double t = 0.0;
        for (int v = 0; v < 256 / 64; v++) t += sh[threadIdx.x][v];
        gpart[blockIdx.x * 8 + threadIdx.x] = t;
    }
}

// The adjoint over the gather Verlet lists (packed window layout): the same
// blocks, windows and lists as the list force, each particle walking its own
// list in chunks of eight, so that no candidate outside the list radius is
// tested.  The window's fourth word holds the position's global index (with
// two types, times two plus the type): the partner's g is read from global
// memory by that index.  Terms and sums as k_adjw_f32.
template <int NT, bool ISO>
__global__ __launch_bounds__(256) void k_adjvl_f32(
    const int4 *__restrict__ st, const int32_t *__restrict__ cs, const int32_t *__restrict__ cell_sorted, Geom g,
    int n, const int32_t *__restrict__ nblk_p, int cap, const int4 *__restrict__ blocks,
    const uint16_t *__restrict__ nbr, const int32_t *__restrict__ cnt, const PairTab *__restrict__ tabp,
    const double *__restrict__ pos, const float *__restrict__ G, double *__restrict__ grad_pos,
    double *__restrict__ gpart, int32_t *__restrict__ flags)
{
    // lists that may be truncated (a build overflowed them) are left to the
    // stencil kernel launched after this one
    if (flags[0] & (int)MD_FLAG_LIST_OVERFLOW) return;
    constexpr int kEsz = (int)sizeof(WinEntry<NT>);  // the lists' entries are window positions times this
    __shared__ int4 win[kWinMax + 1];                // + the far entry
    __shared__ Window w;
    __shared__ double sh[8][256 / 64];
    const float uf = (float)(g.L[0] / 4294967296.0);
    double gp[8] = {0, 0, 0, 0, 0, 0, 0, 0};  // eps_ab[4], sig_ab[4]
    size_t N = (size_t)n;
    for (BlockIter it(min(*nblk_p, cap)); it.blk < it.end; it.blk += it.stride) {
        const int4 blk = blocks[it.blk];
        __syncthreads();
        make_window<false, false>(g, cs, blk, w);
        if (w.W > kWinMax || w.npart > 256) {  // never made by the packer
            if (threadIdx.x == 0) atomicOr(&flags[3], 2);
            continue;
        }
        {
            int k = 0;
            for (int p = threadIdx.x; p < w.W; p += blockDim.x) {
                k = piece_from(w, k, p);
                const int j = w.pc_start[k] + (p - w.pc_win[k]);
                int4 q = st[j];
                q.w = NT == 1 ? j : 2 * j + q.w;
                win[p] = q;
            }
            if (threadIdx.x == 0) win[kWinMax] = far_entry(g, blk);
        }
        __syncthreads();
        int i, k, x;
        if (!my_particle(g, w, cell_sorted, i, k, x)) continue;
        const int4 pi = st[i];
        const float gix = G[i], giy = G[N + i], giz = G[2 * N + i];
        const int ti = NT == 1 ? 0 : pi.w;
        AdjParams pp;
        pp.load<NT>(tabp, ti);
        double ax = 0.0, ay = 0.0, az = 0.0, ge0 = 0.0, ge1 = 0.0, gs0 = 0.0, gs1 = 0.0;
        const int nch = (cnt[i] + 7) >> 3;
        const uint4 *row = (const uint4 *)nbr + i;
        uint4 cur = *row;
        for (int ch = 0; ch < nch; ch++) {
            row += N;
            const uint4 nxt = *row;  // the list has one chunk row more than it fills
            const uint32_t off[8] = {cur.x & 0xffff, cur.x >> 16, cur.y & 0xffff, cur.y >> 16,
                                     cur.z & 0xffff, cur.z >> 16, cur.w & 0xffff, cur.w >> 16};
#pragma unroll
            for (int u = 0; u < 8; u++) {
                const int4 e = win[off[u] / kEsz];
                const bool t1 = NT > 1 && (e.w & 1);
                const int j = NT == 1 ? e.w : (e.w >> 1);
                float dx, dy, dz;
                staged_delta<ISO>(pi, e, g, dx, dy, dz);
                const float r2u = dx * dx + dy * dy + dz * dz;
                if (!within(r2u, t1 ? pp.lo[1] : pp.lo[0], t1 ? pp.hi[1] : pp.hi[0], t1 ? pp.rc2[1] : pp.rc2[0],
                            pos, n, i, j, g))
                    continue;
                adj_pair(dx, dy, dz, uf, t1, gix - G[j], giy - G[N + j], giz - G[2 * N + j], pp, ax, ay, az, ge0,
                         ge1, gs0, gs1);
            }
            cur = nxt;
        }
        gp[ti * NT] += ge0;
        gp[4 + ti * NT] += gs0;
        if (NT > 1) {
            gp[ti * NT + 1] += ge1;
            gp[4 + ti * NT + 1] += gs1;
        }
        grad_pos[i] = ax;
        grad_pos[N + i] = ay;
        grad_pos[2 * N + i] = az;
    }
    // the workgroup's parameter sums, fixed order
#pragma unroll
    for (int q = 0; q < 8; q++)
        for (int off = 32; off > 0; off >>= 1) gp[q] += __shfl_down(gp[q], off, 64);
    __syncthreads();
    int wv = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0)
        for (int q = 0; q < 8; q++) sh[q][wv] = gp[q];
    __syncthreads();
    if (threadIdx.x < 8) {
        double t = 0.0;
        for (int v = 0; v < 256 / 64; v++) t += sh[threadIdx.x][v];
        gpart[blockIdx.x * 8 + threadIdx.x] = t;
    }
}

void launch_adjoint_lists(const int4 *st, const int32_t *cs, const int32_t *cell_sorted, const Geom &g, int n,
                          const int32_t *nblk_p, const int4 *blocks, const uint16_t *nbr, const int32_t *cnt,
                          const PairTab *tab, const double *pos, const float *G, double *grad_pos, double *gpart,
                          int32_t *flags, hipStream_t s)
{
    if (n <= 0) return;
    int cap = (int)window_block_cap(n, g);
    if (g.nt == 1) {
        if (g.iso)
            k_adjvl_f32<1, true><<<kWinGrid, 256, 0, s>>>(st, cs, cell_sorted, g, n, nblk_p, cap, blocks, nbr, cnt,
                                                           tab, pos, G, grad_pos, gpart, flags);
        else
            k_adjvl_f32<1, false><<<kWinGrid, 256, 0, s>>>(st, cs, cell_sorted, g, n, nblk_p, cap, blocks, nbr, cnt,
                                                            tab, pos, G, grad_pos, gpart, flags);
    } else {
        if (g.iso)
            k_adjvl_f32<2, true><<<kWinGrid, 256, 0, s>>>(st, cs, cell_sorted, g, n, nblk_p, cap, blocks, nbr, cnt,
                                                           tab, pos, G, grad_pos, gpart, flags);
        else
            k_adjvl_f32<2, false><<<kWinGrid, 256, 0, s>>>(st, cs, cell_sorted, g, n, nblk_p, cap, blocks, nbr, cnt,
                                                            tab, pos, G, grad_pos, gpart, flags);
    }
    // the stencil kernel does the work instead when the lists overflowed
    launch_adjoint_window(st, cs, cell_sorted, g, n, nblk_p, blocks, tab, pos, G, grad_pos, gpart, flags, s, 1);
}

void launch_adjoint_window(const int4 *st, const int32_t *cs, const int32_t *cell_sorted, const Geom &g, int n,
                           const int32_t *nblk_p, const int4 *blocks, const PairTab *tab, const double *pos,
                           const float *G, double *grad_pos, double *gpart, int32_t *flags, hipStream_t s,
                           int only_if_overflow)
{
    if (n <= 0) return;
    int cap = (int)window_block_cap(n, g);
    if (g.nt == 1) {
        if (g.iso)
            k_adjw_f32<1, true><<<kWinGrid, 256, 0, s>>>(st, cs, cell_sorted, g, n, nblk_p, cap, blocks, tab, pos,
                                                          G, grad_pos, gpart, flags, only_if_overflow);
        else
            k_adjw_f32<1, false><<<kWinGrid, 256, 0, s>>>(st, cs, cell_sorted, g, n, nblk_p, cap, blocks, tab, pos,
                                                           G, grad_pos, gpart, flags, only_if_overflow);
    } else {
        if (g.iso)
            k_adjw_f32<2, true><<<kWinGrid, 256, 0, s>>>(st, cs, cell_sorted, g, n, nblk_p, cap, blocks, tab, pos,
                                                          G, grad_pos, gpart, flags, only_if_overflow);
        else
            k_adjw_f32<2, false><<<kWinGrid, 256, 0, s>>>(st, cs, cell_sorted, g, n, nblk_p, cap, blocks, tab, pos,
                                                           G, grad_pos, gpart, flags, only_if_overflow);
    }
}

// ------------------------------------------------------------------ Verlet lists

// List entry c of particle i: nbr[((c / 8) * n + i) * 8 + c % 8].
__device__ __forceinline__ size_t list_slot(int c, int i, size_t N) { return ((size_t)(c >> 3) * N + i) * 8 + (c & 7); }

// Pending chunk of the list being built: a 128-bit shift register of eight
// 16-bit entries (each append shifts the register down by one entry and
// puts the new entry on top; after eight appends entry 0 is in the low half
// of word x, entry 7 in the high half of word w, as the force kernels read
// them).
struct Chunk {
    uint32_t x = 0, y = 0, z = 0, w = 0;
    __device__ __forceinline__ void push(uint32_t p)
    {
        x = __builtin_amdgcn_alignbit(y, x, 16);
        y = __builtin_amdgcn_alignbit(z, y, 16);
        z = __builtin_amdgcn_alignbit(w, z, 16);
        w = __builtin_amdgcn_alignbit(p, w, 16);
    }
    __device__ __forceinline__ uint4 word() const { return make_uint4(x, y, z, w); }
};

// Append window position p to the list of particle i (c entries so far);
// every completed chunk is written with one 16-byte store.
__device__ __forceinline__ void list_append(uint32_t p, int &c, Chunk &ck, uint4 *__restrict__ row, size_t N,
                                            int maxn)
{
    ck.push(p);
    c++;
    if ((c & 7) == 0 && c <= maxn) row[(size_t)((c >> 3) - 1) * N] = ck.word();
}

// Write the last, partial chunk (its entries shifted down to the bottom,
// the rest filled with pad).
__device__ __forceinline__ void list_finish(int c, Chunk &ck, uint4 *__restrict__ row, size_t N, int maxn,
                                            uint32_t pad)
{
    if ((c & 7) == 0 || c >= maxn) return;
    for (int e = c & 7; e < 8; e++) ck.push(pad);
    row[(size_t)(c >> 3) * N] = ck.word();
}

// Guard band of the list radius as centre and half width, the half width
// widened so that every r2 in [rl2_lo, rl2_hi) passes |r2 - mid| <= hw: the
// band is 2^-18 of rl2 wide, the rounding of mid moves it by at most 2^-24
// of rl2 (3 % of the half width), and r2 - mid is exact near the band.
struct Band {
    float mid, hw;
    __device__ __forceinline__ explicit Band(const Geom &g)
        : mid(0.5f * (g.rl2_lo + g.rl2_hi)), hw(0.5f * (g.rl2_hi - g.rl2_lo) * 1.125f)
    {
    }
};

// One batch of Verlet-list candidates: window positions q[0 .. m-1], m <= 32,
// tested against the list radius in FP32.  Returns the mask of those with
// r2 below the upper edge of the guard band (candidate u at bit m - 1 - u:
// each test shifts the mask up and adds its outcome); amb is set if one of
// them may lie inside the band (the nearest r2 to its centre is within the
// widened half width; the caller then decides those from the FP64
// positions).  Reads whole groups of four, up to three positions past the
// batch (the window arrays are padded for them); their bits are dropped.
template <bool ISO>
__device__ __forceinline__ uint32_t build_batch(const int4 &pi, const WinEntry<1> *__restrict__ q, int m,
                                                const Geom &g, const Band &band, bool &amb)
{
    uint32_t mask = 0;
    float near = 3.0e38f;
    int nb = 0;
    auto test = [&](const WinEntry<1> &e) {
        float dx, dy, dz;
        staged_delta<ISO>(pi, e.get(), g, dx, dy, dz);
        float r2 = dx * dx + dy * dy + dz * dz;
        mask = mask + mask + (r2 < g.rl2_hi ? 1u : 0u);
        near = fminf(near, fabsf(r2 - band.mid));
    };
    for (; nb < m; nb += 4) {
        test(q[nb]);
        test(q[nb + 1]);
        test(q[nb + 2]);
        test(q[nb + 3]);
    }
    // the candidates read past the batch may raise amb: a harmless slow path
    amb = near <= band.hw;
    return mask >> (nb - m);
}

// build_batch on single-precision relative coordinates (FEntry windows):
// mask of the candidates with r2 < hi; amb if one lies within hw of mid.
__device__ __forceinline__ uint32_t build_batch_rel(const FEntry &pi, const FEntry *__restrict__ q, int m, float hi,
                                                    float mid, float hw, bool &amb)
{
    uint32_t mask = 0;
    float near = 3.0e38f;
    int nb = 0;
    auto test = [&](const FEntry &e) {
        float dx = e.x - pi.x, dy = e.y - pi.y, dz = e.z - pi.z;
        float r2 = dx * dx + dy * dy + dz * dz;
        mask = mask + mask + (r2 < hi ? 1u : 0u);
        near = fminf(near, fabsf(r2 - mid));
    };
    for (; nb < m; nb += 4) {
        test(q[nb]);
        test(q[nb + 1]);
        test(q[nb + 2]);
        test(q[nb + 3]);
    }
    amb = near <= hw;
    return mask >> (nb - m);
}

// Verlet lists (full windows: every pair within r_c + skin from both sides;
// half windows: each pair once, in the forward half of the stencil).  Each
// range of candidates (with the single-precision windows first cut to its x
// interval, stencil_ranges_cut) is tested 32 positions at a time into a bit
// mask, then the set bits are appended in window order.  Full lists hold LDS byte
// offsets (window position times esz, the size of the force kernel's window
// entry) and pad their last chunk with the offset of the far entry; half
// lists hold window positions (esz 1) padded with 0.
template <bool ISO, bool HALF, bool REL>
__global__ __launch_bounds__(256) void k_vlw_build(const int4 *__restrict__ st, const int32_t *__restrict__ cs,
                                                   const int32_t *__restrict__ cell_sorted,
                                                   const double *__restrict__ pos, Geom g, int n,
                                                   const int32_t *__restrict__ nblk_p, int cap,
                                                   const int4 *__restrict__ blocks,
                                                   uint16_t *__restrict__ nbr, int32_t *__restrict__ cnt, int maxn,
                                                   int esz, int32_t *__restrict__ flags)
{
    // REL: single-precision windows relative to the block centre (FEntry,
    // the same 12 bytes as WinEntry<1>), with the wider band kBuildBand
    __shared__ WinEntry<1> win[(HALF ? kWinMaxHalf : kWinMax) + 4];  // + the reads past a batch
    __shared__ Window w;
    FEntry *winf = (FEntry *)win;
    size_t N = (size_t)n;
    int cmax = 0;
    const float rl2u = (float)(g.rl2 * g.S[0] * g.S[0]);
    const float rel_hi = rl2u * (1.0f + kBuildBand), rel_lo = rl2u * (1.0f - kBuildBand);
    const float rel_hw = rl2u * kBuildBand;
    // cell height and depth in relative units (y and z scaled to x units)
    const float hy = 4294967296.0f / (float)g.nc[1] * g.ry, hz = 4294967296.0f / (float)g.nc[2] * g.rz;
    for (BlockIter it(min(*nblk_p, cap)); it.blk < it.end; it.blk += it.stride) {
        int blk = it.blk;
        if (REL) {
            if (!setup_block_rel<HALF>(g, cs, st, blocks[blk], w, winf, flags)) continue;
        } else {
            if (!setup_block<1, HALF>(g, cs, st, blocks[blk], w, win, flags)) continue;
        }
        int i, k, x;
        if (!my_particle(g, w, cell_sorted, i, k, x)) continue;
        int self = self_position<HALF>(w, cs, i, k, column_of(g, w, x), cell_sorted[i]);
        int4 pi = REL ? make_int4(0, 0, 0, 0) : win[self].get();
        FEntry pf = REL ? winf[self] : FEntry{0.f, 0.f, 0.f};
        uint4 *row = (uint4 *)nbr + i;
        int c = 0;
        Chunk ck;
        const Band band(g);
        auto batches = [&](int b, int en) {
            for (int base = b; base < en; base += 32) {
                int m = min(32, en - base);
                bool amb;
                uint32_t mask = REL ? build_batch_rel(pf, winf + base, m, rel_hi, rl2u, rel_hw, amb)
                                    : build_batch<ISO>(pi, win + base, m, g, band, amb);
                unsigned us = (unsigned)(self - base);
                if (us < (unsigned)m) mask &= ~(1u << (m - 1 - us));
                if (amb) {
                    // rare: guard-band candidates decided from the FP64 positions
                    for (uint32_t t = mask; t;) {
                        int h = 31 - __builtin_clz(t);
                        t ^= 1u << h;
                        int p = base + m - 1 - h;
                        float r2, lo;
                        if (REL) {
                            float dx = winf[p].x - pf.x, dy = winf[p].y - pf.y, dz = winf[p].z - pf.z;
                            r2 = dx * dx + dy * dy + dz * dz;
                            lo = rel_lo;
                        } else {
                            float dx, dy, dz;
                            staged_delta<ISO>(pi, win[p].get(), g, dx, dy, dz);
                            r2 = dx * dx + dy * dy + dz * dz;
                            lo = g.rl2_lo;
                        }
                        if (r2 >= lo && !(exact_r2(pos, n, i, window_global(w, p), g.L[0], g.L[1], g.L[2]) < g.rl2))
                            mask ^= 1u << h;
                    }
                }
                // entries are window positions times esz (< 2^16): bit 31 - z
                // is position base + m - 32 + z, its entry z0 + z esz (mod
                // 2^32), with a 24-bit product per entry
                const unsigned esz8 = (unsigned)esz & 0xffu;
                const unsigned z0 = (unsigned)(base + m - 32) * (unsigned)esz;
                while (mask) {
                    unsigned z = (unsigned)__builtin_clz(mask);
                    mask ^= 0x80000000u >> z;
                    list_append(z0 + z * esz8, c, ck, row, N, maxn);
                }
            }
        };
        if (REL)
            stencil_ranges_cut<HALF>(g, w, winf, pf, k, x, self, rel_hi, hy, hz, batches);
        else
            stencil_ranges<HALF>(g, w, k, x, self, batches);
        list_finish(c, ck, row, N, maxn, HALF ? 0u : (uint32_t)(kWinMax * esz));
        if (c > maxn) atomicOr(&flags[0], (int)MD_FLAG_LIST_OVERFLOW);
        cmax = max(cmax, c);
        cnt[i] = c < maxn ? c : maxn;
    }
    if (cmax > 0) atomicMax(&flags[2], cmax);
}

// One entry of the gather Verlet-list force.  As pair_fast, except that with
// one type the factor 24 eps is applied once per particle after the sum
// (FOLD), and the guard band is tested with one unsigned compare of the
// float bits (r2 >= 0, so the bit patterns order as the values).  Returns
// true for a guard-band pair.
template <int NT, bool ISO, bool ENERGY>
__device__ __forceinline__ bool vl_entry(const int4 &pi, const int4 &pj, bool valid, const TabF<NT> &t,
                                         const Geom &g, float &fx, float &fy, float &fz, float &eu, float &ew,
                                         int &np)
{
    float dx, dy, dz;
    staged_delta<ISO>(pi, pj, g, dx, dy, dz);
    float r2 = dx * dx + dy * dy + dz * dz;
    int ab = NT == 1 ? 0 : pi.w * NT + pj.w;
    float lo = t.pick(t.lo, ab), hi = t.pick(t.hi, ab);
    bool in = valid && r2 < lo;
    float ir2 = in ? __builtin_amdgcn_rcpf(r2) : 0.0f;
    float s2 = t.pick(t.sig2, ab) * ir2;
    float q = s2 * s2 * s2;
    float a = q * (2.0f * q - 1.0f);
    float phi = NT == 1 ? ir2 * a : t.pick(t.eps24, ab) * ir2 * a;
    if (ENERGY) {
        eu += t.pick(t.eps4, ab) * q * (q - 1.0f);
        ew += t.pick(t.eps24w, ab) * a;
        np += in ? 1 : 0;
    }
    fx += phi * dx;
    fy += phi * dy;
    fz += phi * dz;
    uint32_t lob = __float_as_uint(lo);
    return valid && __float_as_uint(r2) - lob < __float_as_uint(hi) - lob;
}

// Guard-band entry, decided from the FP64 positions (same folding).
template <int NT, bool ISO, bool ENERGY>
__device__ __forceinline__ void vl_exact(const int4 &pi, const int4 &pj, int i, int j, const TabF<NT> &t,
                                         const Geom &g, const double *__restrict__ pos, int n, float &fx, float &fy,
                                         float &fz, float &eu, float &ew, int &np)
{
    int ab = NT == 1 ? 0 : pi.w * NT + pj.w;
    if (exact_r2(pos, n, i, j, g.L[0], g.L[1], g.L[2]) < t.pickd(t.rc2, ab)) {
        float dx, dy, dz;
        staged_delta<ISO>(pi, pj, g, dx, dy, dz);
        float r2 = dx * dx + dy * dy + dz * dz;
        float ir2 = __builtin_amdgcn_rcpf(r2);
        float s2 = t.pick(t.sig2, ab) * ir2;
        float q = s2 * s2 * s2;
        float a = q * (2.0f * q - 1.0f);
        float phi = NT == 1 ? ir2 * a : t.pick(t.eps24, ab) * ir2 * a;
        if (ENERGY) {
            eu += t.pick(t.eps4, ab) * q * (q - 1.0f);
            ew += t.pick(t.eps24w, ab) * a;
            np += 1;
        }
        fx += phi * dx;
        fy += phi * dy;
        fz += phi * dz;
    }
}

// LDS layout of the Verlet-list force windows (the data layout of Sec.
// 2.2.3, for the window the force pass reads): MD_LAYOUT_PACKED holds
// WinEntry<NT> (12 bytes with one type), MD_LAYOUT_ALIGNED 16-byte entries
// (one 16-byte read), MD_LAYOUT_SOA one plane of kWinMax + 1 words per
// coordinate (three 4-byte reads at fixed distances).  List entries are the
// entries' byte offsets: position times kEsz.  The last position of each
// (kWinMax) is the far entry.  The other layouts hold one type.
template <int NT, int LAYOUT>
struct WinLay {
    static constexpr int kEsz = LAYOUT == MD_LAYOUT_ALIGNED ? 16 : (LAYOUT == MD_LAYOUT_SOA ? 4 : (int)sizeof(WinEntry<NT>));
    static constexpr int kPlane = kWinMax + 1;  // words per plane
    // LDS storage, in WinEntry<NT> units (packed) or 16-byte units
    using Unit = typename std::conditional<LAYOUT == MD_LAYOUT_PACKED, WinEntry<NT>, int4>::type;
    static constexpr int kUnits = LAYOUT == MD_LAYOUT_SOA ? (3 * kPlane + 3) / 4 : kWinMax + 1;
    __device__ static __forceinline__ void put(Unit *win, int p, const int4 &a)
    {
        if (LAYOUT == MD_LAYOUT_PACKED) {
            ((WinEntry<NT> *)win)[p].set(a);
        } else if (LAYOUT == MD_LAYOUT_ALIGNED) {
            ((int4 *)win)[p] = make_int4(a.x, a.y, a.z, 0);
        } else {
            int *x = (int *)win;
            x[p] = a.x;
            x[p + kPlane] = a.y;
            x[p + 2 * kPlane] = a.z;
        }
    }
    // the entry at byte offset off (a list entry)
    __device__ static __forceinline__ int4 at(const Unit *win, uint32_t off)
    {
        const char *b = (const char *)win + off;
        if (LAYOUT == MD_LAYOUT_PACKED) return ((const WinEntry<NT> *)b)->get();
        if (LAYOUT == MD_LAYOUT_ALIGNED) {
            int4 v = *(const int4 *)b;
            return make_int4(v.x, v.y, v.z, 0);
        }
        const int *x = (const int *)b;
        return make_int4(x[0], x[kPlane], x[2 * kPlane], 0);
    }
};

// setup_block for the Verlet-list force windows of any layout (full window,
// no column table, the far entry at position kWinMax).
template <int NT, int LAYOUT>
__device__ __forceinline__ bool setup_block_lay(const Geom &g, const int32_t *__restrict__ cs,
                                                const int4 *__restrict__ st, int4 blk, Window &w,
                                                typename WinLay<NT, LAYOUT>::Unit *win, int32_t *flags)
{
    if (LAYOUT == MD_LAYOUT_PACKED)
        return setup_block<NT, false, false, true>(g, cs, st, blk, w, (WinEntry<NT> *)win, flags);
    __syncthreads();
    make_window<false, false>(g, cs, blk, w);
    if (w.W > kWinMax || w.npart > 256) {  // never made by the packer
        if (threadIdx.x == 0) atomicOr(&flags[3], 2);
        return false;
    }
    int k = 0;
    for (int p = threadIdx.x; p < w.W; p += blockDim.x) {
        k = piece_from(w, k, p);
        WinLay<NT, LAYOUT>::put(win, p, st[w.pc_start[k] + (p - w.pc_win[k])]);
    }
    if (threadIdx.x == 0) WinLay<NT, LAYOUT>::put(win, kWinMax, far_entry(g, blk));
    __syncthreads();
    return true;
}

// One list entry of the gather force, branch free: the window entry at LDS
// byte offset off.  With one type the guard band is tracked through near,
// the smallest |r2 - centre| seen; otherwise through amb.
template <int NT, bool ISO, bool ENERGY, int LAYOUT = MD_LAYOUT_PACKED>
__device__ __forceinline__ void vl_step(const int4 &pi, const typename WinLay<NT, LAYOUT>::Unit *__restrict__ win,
                                        uint32_t off, const TabF<NT> &t, const Geom &g, float mid, float &near,
                                        bool &amb, float &fx, float &fy, float &fz, float &eu, float &ew, int &np)
{
    const int4 ej = WinLay<NT, LAYOUT>::at(win, off);
    if (NT == 1) {
        float dx, dy, dz;
        staged_delta<ISO>(pi, ej, g, dx, dy, dz);
        float r2 = dx * dx + dy * dy + dz * dz;
        bool in = r2 < t.lo[0];
        float ir2 = in ? __builtin_amdgcn_rcpf(r2) : 0.0f;
        float s2 = t.sig2[0] * ir2;
        float q = s2 * s2 * s2;
        float a = q * (2.0f * q - 1.0f);
        float phi = ir2 * a;
        if (ENERGY) {
            eu += t.eps4[0] * q * (q - 1.0f);
            ew += t.eps24w[0] * a;
            np += in ? 1 : 0;
        }
        fx += phi * dx;
        fy += phi * dy;
        fz += phi * dz;
        near = fminf(near, fabsf(r2 - mid));
    } else {
        amb |= vl_entry<NT, ISO, ENERGY>(pi, ej, true, t, g, fx, fy, fz, eu, ew, np);
    }
}

// Each thread walks its list in chunks of eight entries (the lists hold LDS
// byte offsets; the last chunk is padded with the far entry, whose pairs
// never interact); the next chunk's load is in flight while the current one
// is computed.  A chunk with an entry that may lie in the guard band (rare)
// is walked again for those entries.  FUSED: each thread then advances its
// particle (verlet_update: this step's second half kick, the next step's
// first half kick, drift, stage and skin check), reading the positions from
// pos and writing them to pos_out and stage_out (other blocks still read pos
// and st); the kinetic energy and the largest displacement go to ia.kpart
// and ia.dpart per workgroup.
template <int NT, bool ISO, bool ENERGY, bool FUSED, int LAYOUT = MD_LAYOUT_PACKED>
__global__ __launch_bounds__(256) void k_vlw_f32(const int4 *__restrict__ st, const int32_t *__restrict__ cs,
                                                 const int32_t *__restrict__ cell_sorted, Geom g, int n,
                                                 const int32_t *__restrict__ nblk_p, int cap,
                                                 const int4 *__restrict__ blocks,
                                                 const uint16_t *__restrict__ nbr, const int32_t *__restrict__ cnt,
                                                 const PairTab *__restrict__ tabp, const double *__restrict__ pos,
                                                 float *__restrict__ F, double *__restrict__ partials,
                                                 int32_t *__restrict__ flags, IntegrateArgs ia, double *pos_out,
                                                 int4 *stage_out)
{
    using Lay = WinLay<NT, LAYOUT>;
    __shared__ typename Lay::Unit win[Lay::kUnits];  // + the far entry
    __shared__ Window w;
    __shared__ double sh[16];
    TabF<NT> t;
    t.load(tabp);
    // guard band of the cutoff as centre and widened half width (one type)
    const float mid = 0.5f * (t.lo[0] + t.hi[0]), hw = 0.5f * (t.hi[0] - t.lo[0]) * 1.125f;
    float eu = 0.f, ew = 0.f;
    int np = 0;
    double ke = 0.0;
    float dmax = 0.f;
    size_t N = (size_t)n;
    for (BlockIter it(min(*nblk_p, cap)); it.blk < it.end; it.blk += it.stride) {
        int blk = it.blk;
        // the list holds window positions: only the window's pieces are needed
        if (!setup_block_lay<NT, LAYOUT>(g, cs, st, blocks[blk], w, win, flags)) continue;
        int i, k, x;
        if (!my_particle(g, w, cell_sorted, i, k, x)) continue;
        int4 pi = st[i];
        int c = cnt[i];
        int nch = (c + 7) >> 3;
        float fx = 0.f, fy = 0.f, fz = 0.f;
        VState<float, NT == 1> vs;
        if (FUSED) vs.load(ia, i, N, pos, true);  // in flight during the force loop
        // chunk ch of particle i is row[ch * n]; the list has one chunk row
        // more than it can fill, so the prefetch past the last chunk is an
        // in-bounds load
        const uint4 *row = (const uint4 *)nbr + i;
        uint4 cur = *row;
        for (int ch = 0; ch < nch; ch++) {
            row += N;
            uint4 nxt = *row;
            uint32_t off[8] = {cur.x & 0xffff, cur.x >> 16, cur.y & 0xffff, cur.y >> 16,
                               cur.z & 0xffff, cur.z >> 16, cur.w & 0xffff, cur.w >> 16};
            float near = 3.0e38f;
            bool amb = false;
#pragma unroll
            for (int u = 0; u < 8; u++)
                vl_step<NT, ISO, ENERGY, LAYOUT>(pi, win, off[u], t, g, mid, near, amb, fx, fy, fz, eu, ew, np);
            if (NT == 1) amb = near <= hw;
            if (amb) {
                // the far entries of the padding are never in the band
                for (int u = 0; u < 8; u++) {
                    int p = (int)(off[u] / Lay::kEsz);
                    int4 pj = Lay::at(win, off[u]);
                    float dx, dy, dz;
                    staged_delta<ISO>(pi, pj, g, dx, dy, dz);
                    float r2 = dx * dx + dy * dy + dz * dz;
                    int ab = NT == 1 ? 0 : pi.w * NT + pj.w;
                    if (r2 >= t.pick(t.lo, ab) && r2 < t.pick(t.hi, ab))
                        vl_exact<NT, ISO, ENERGY>(pi, pj, i, window_global(w, p), t, g, pos, n, fx, fy, fz, eu, ew,
                                                  np);
                }
            }
            cur = nxt;
        }
        if (NT == 1) {
            float e24 = t.eps24[0];
            fx *= e24;
            fy *= e24;
            fz *= e24;
        }
        F[i] = fx;
        F[N + i] = fy;
        F[2 * N + i] = fz;
        if (FUSED) {
            double kei = 0.0;
            float d2 = 0.f;
            verlet_update<float, ISO, NT == 1>(ia, g, i, N, vs, fx, fy, fz, true, true, pos_out, stage_out, kei, d2);
            ke += kei;
            dmax = fmaxf(dmax, d2);
        }
    }
    if (ENERGY) {
        double v[4] = {(double)eu, (double)ew, (double)np, 0.0};
        block_sum4(v, sh);
        if (threadIdx.x == 0)
            for (int k = 0; k < 4; k++) partials[blockIdx.x * 4 + k] = v[k];
    }
    if (FUSED) {
        if (ia.energy) {
            double v[4] = {ke, 0.0, 0.0, 0.0};
            block_sum4(v, sh);
            if (threadIdx.x == 0) ia.kpart[blockIdx.x] = v[0];
        }
        if (ia.dpart) {
            __shared__ float wm[256 / 64];
            for (int off = 32; off > 0; off >>= 1) dmax = fmaxf(dmax, __shfl_xor(dmax, off, 64));
            if ((threadIdx.x & 63) == 0) wm[threadIdx.x >> 6] = dmax;
            __syncthreads();
            if (threadIdx.x == 0) ia.dpart[blockIdx.x] = fmaxf(fmaxf(wm[0], wm[1]), fmaxf(wm[2], wm[3]));
        }
    }
}

// ------------------------------------------------------------------ Newton's third law (half windows)

// Each pair once: a thread takes the pairs of its particle with the forward
// half of its stencil (stencil_ranges<true>).  The j-side forces accumulate
// in LDS, one 64-bit fixed-point integer per component and window position:
// integer LDS atomics run at the LDS's full rate, float ones (measured on
// this device) about thirty times slower.  After the block every nonzero
// entry is added to the global force with one atomic per component, where
// consecutive positions of a piece are consecutive particles, so that a
// wavefront's atomics are coalesced.
struct HalfAcc {
    unsigned long long x[kWinMaxHalf], y[kWinMaxHalf], z[kWinMaxHalf];
};

// (The fixed-point accumulators, to_fix and from_fix, are in pair.h.)

// Head of the half-window force kernels: window laid out and staged,
// accumulators cleared; false (uniformly) if the window does not fit.
template <int NT>
__device__ __forceinline__ bool setup_half(const Geom &g, const int32_t *__restrict__ cs, const int4 *__restrict__ st,
                                           int4 blk, Window &w, WinEntry<NT> *win, HalfAcc &acc, int32_t *flags)
{
    __syncthreads();
    make_window<true>(g, cs, blk, w);
    if (w.W > kWinMaxHalf || w.npart > 256) {  // never made by the packer
        if (threadIdx.x == 0) atomicOr(&flags[3], 2);
        return false;
    }
    load_window(w, st, win);
    for (int p = threadIdx.x; p < w.W; p += blockDim.x) {
        acc.x[p] = 0ull;
        acc.y[p] = 0ull;
        acc.z[p] = 0ull;
    }
    __syncthreads();
    return true;
}

// Add the block's accumulators to the global forces: one atomic per
// component and nonzero window position; consecutive positions of a piece
// are consecutive particles, so a wavefront's atomics are coalesced.  (The
// device-wide float atomics are performed at the memory side; per-XCD
// copies of the forces with L2-scope atomics were measured no faster.)
__device__ __forceinline__ void flush_half(const HalfAcc &acc, const Window &w, float *__restrict__ F, size_t N)
{
    __syncthreads();
    int k = 0;
    for (int p = threadIdx.x; p < w.W; p += blockDim.x) {
        k = piece_from(w, k, p);
        int j = w.pc_start[k] + (p - w.pc_win[k]);
        unsigned long long ax = acc.x[p], ay = acc.y[p], az = acc.z[p];
        if (ax) atomicAdd(&F[j], from_fix(ax));
        if (ay) atomicAdd(&F[N + j], from_fix(ay));
        if (az) atomicAdd(&F[2 * N + j], from_fix(az));
    }
}

// The thread's own particle's force (its i-side sum) into the accumulator.
__device__ __forceinline__ void add_own(HalfAcc &acc, int self, float fx, float fy, float fz)
{
    atomicAdd(&acc.x[self], to_fix(fx));
    atomicAdd(&acc.y[self], to_fix(fy));
    atomicAdd(&acc.z[self], to_fix(fz));
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
    float px = phi * dx, py = phi * dy, pz = phi * dz;
    fx += px;
    fy += py;
    fz += pz;
    if (in) {
        atomicAdd(&acc.x[p], to_fix(-px));
        atomicAdd(&acc.y[p], to_fix(-py));
        atomicAdd(&acc.z[p], to_fix(-pz));
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
        float px = phi * dx, py = phi * dy, pz = phi * dz;
        fx += px;
        fy += py;
        fz += pz;
        atomicAdd(&acc.x[p], to_fix(-px));
        atomicAdd(&acc.y[p], to_fix(-py));
        atomicAdd(&acc.z[p], to_fix(-pz));
    }
}

template <int NT, bool ISO, bool ENERGY>
__global__ __launch_bounds__(256) void k_lcwh_f32(const int4 *__restrict__ st, const int32_t *__restrict__ cs,
                                                  const int32_t *__restrict__ cell_sorted, Geom g, int n,
                                                  const int32_t *__restrict__ nblk_p, int cap,
                                                  const int4 *__restrict__ blocks,
                                                  const PairTab *__restrict__ tabp, const double *__restrict__ pos,
                                                  float *__restrict__ F, double *__restrict__ partials,
                                                  int32_t *__restrict__ flags)
{
    __shared__ WinEntry<NT> win[kWinMaxHalf + 4];  // + the reads past a batch
    __shared__ HalfAcc acc;
    __shared__ Window w;
    __shared__ double sh[16];
    TabF<NT> t;
    t.load(tabp);
    const float hi = max_hi(t);
    float eu = 0.f, ew = 0.f;
    int np = 0;
    size_t N = (size_t)n;
    for (BlockIter it(min(*nblk_p, cap)); it.blk < it.end; it.blk += it.stride) {
        int blk = it.blk;
        if (!setup_half<NT>(g, cs, st, blocks[blk], w, win, acc, flags)) continue;
        int i, k, x;
        if (my_particle(g, w, cell_sorted, i, k, x)) {
            int self = self_position<true>(w, cs, i, k, column_of(g, w, x), cell_sorted[i]);
            int4 pi = win[self].get();
            float fx = 0.f, fy = 0.f, fz = 0.f;
            stencil_ranges<true>(g, w, k, x, self, [&](int b, int en) {
                for (int base = b; base < en; base += 32) {
                    int m = min(32, en - base);
                    uint32_t mask = cut_batch<NT, ISO>(pi, win + base, m, g, hi);
                    while (mask) {
                        int h = 31 - __builtin_clz(mask);
                        mask ^= 1u << h;
                        int p = base + m - 1 - h;
                        int4 pj = win[p].get();
                        if (pair_n3l<NT, ISO, ENERGY>(pi, pj, p, true, t, g, acc, fx, fy, fz, eu, ew, np))
                            pair_exact_n3l<NT, ISO, ENERGY>(pi, pj, p, i, window_global(w, p), t, g, pos, n, acc, fx,
                                                            fy, fz, eu, ew, np);
                    }
                }
            });
            add_own(acc, self, fx, fy, fz);
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

template <int NT, bool ISO, bool ENERGY>
__global__ __launch_bounds__(256) void k_vlwh_f32(const int4 *__restrict__ st, const int32_t *__restrict__ cs,
                                                  const int32_t *__restrict__ cell_sorted, Geom g, int n,
                                                  const int32_t *__restrict__ nblk_p, int cap,
                                                  const int4 *__restrict__ blocks,
                                                  const uint16_t *__restrict__ nbr, const int32_t *__restrict__ cnt,
                                                  const PairTab *__restrict__ tabp, const double *__restrict__ pos,
                                                  float *__restrict__ F, double *__restrict__ partials,
                                                  int32_t *__restrict__ flags)
{
    __shared__ WinEntry<NT> win[kWinMaxHalf];
    __shared__ HalfAcc acc;
    __shared__ Window w;
    __shared__ double sh[16];
    TabF<NT> t;
    t.load(tabp);
    float eu = 0.f, ew = 0.f;
    int np = 0;
    size_t N = (size_t)n;
    for (BlockIter it(min(*nblk_p, cap)); it.blk < it.end; it.blk += it.stride) {
        int blk = it.blk;
        if (!setup_half<NT>(g, cs, st, blocks[blk], w, win, acc, flags)) continue;
        int i, k, x;
        if (my_particle(g, w, cell_sorted, i, k, x)) {
            int self = self_position<true>(w, cs, i, k, column_of(g, w, x), cell_sorted[i]);
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
            add_own(acc, self, fx, fy, fz);
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
__global__ void k_vlw_decode(const int32_t *__restrict__ cs, const int32_t *__restrict__ cell_sorted, Geom g, int n,
                             const int32_t *__restrict__ nblk_p, int cap, const int4 *__restrict__ blocks,
                             const uint16_t *__restrict__ nbr,
                             const int32_t *__restrict__ cnt, int maxr, int esz, int32_t *__restrict__ counts,
                             int32_t *__restrict__ rows)
{
    __shared__ Window w;
    size_t N = (size_t)n;
    int nblk = min(*nblk_p, cap);
    for (int blk = blockIdx.x; blk < nblk; blk += gridDim.x) {
        __syncthreads();
        make_window<HALF, false>(g, cs, blocks[blk], w);
        int i, k, x;
        if (!my_particle(g, w, cell_sorted, i, k, x)) continue;
        int c = cnt[i];
        counts[i] = c;
        for (int e = 0; e < c && e < maxr; e++)
            rows[(size_t)i * maxr + e] = window_global(w, (int)nbr[list_slot(e, i, N)] / esz);
    }
}

// ------------------------------------------------------------------ host side

int window_nbands(const Geom &g) { return g.nc[2] * ((g.nc[1] + g.wband - 1) / g.wband); }

int64_t window_block_cap(int64_t n, const Geom &g) { return n + (int64_t)window_nbands(g) + 16; }

bool window_geometry_ok(const Geom &g, bool half)
{
    (void)half;
    int r = g.reach[0];
    if (r < 1 || r > kMaxReach || g.reach[1] != r || g.reach[2] != r) return false;
    for (int d = 0; d < 3; d++)
        if (g.nofs[d] != 2 * r + 1) return false;  // every stencil cell distinct
    return g.wband >= 1 && g.wband <= kWinBlkRows && g.nc[1] >= g.wband + 2 * r && g.nc[0] <= kPackMaxX;
}

// Blocks of the windowed kernels: per-band block counts (with the band's
// first blocks staged), their scan, then the descriptors.  (Ordering each
// XCD's blocks by size, largest first, was measured to gain nothing and cost
// a launch per build.)
void launch_blocks(const Geom &g, const int32_t *cs, int4 *staged, int32_t *band_n, int32_t *band_base,
                   int32_t *scan_scratch, int4 *blocks, int cap, int32_t *flags, bool half, hipStream_t s)
{
    int nb = window_nbands(g);
    int wmax = half ? kWinMaxHalf : kWinMax;
    size_t lds = 3 * (size_t)g.nc[0] * sizeof(int);  // <= 48 KB (nc[0] <= kPackMaxX)
    if (half)
        k_blk_count<true><<<nb, 64, lds, s>>>(g, cs, band_n, staged, flags, wmax);
    else
        k_blk_count<false><<<nb, 64, lds, s>>>(g, cs, band_n, staged, flags, wmax);
    launch_scan(band_n, band_base, nb, scan_scratch, s);
    if (half)
        k_blk_write<true><<<nb, 64, lds, s>>>(g, cs, band_n, band_base, staged, blocks, cap, flags, wmax);
    else
        k_blk_write<false><<<nb, 64, lds, s>>>(g, cs, band_n, band_base, staged, blocks, cap, flags, wmax);
}

int64_t window_staged_blocks(const Geom &g) { return (int64_t)window_nbands(g) * kBandCap; }

// The single-precision build windows need every window to span less than
// the box in each dimension: at most kBlkCells columns plus the reach on
// both sides in x, the band's rows plus the reach in y, 2 r + 1 layers in z.
bool build_float_ok(const Geom &g)
{
    int r = g.reach[0];
    return g.nc[0] > kBlkCells + 2 * r && g.nc[1] > g.wband + 2 * r && g.nc[2] > 2 * r + 1;
}

// Size of the force kernels' LDS window entry (positions, plus the type when
// there are several).
static int window_entry_size(const Geom &g)
{
    if (g.nt == 1 && g.layout == MD_LAYOUT_ALIGNED) return WinLay<1, MD_LAYOUT_ALIGNED>::kEsz;
    if (g.nt == 1 && g.layout == MD_LAYOUT_SOA) return WinLay<1, MD_LAYOUT_SOA>::kEsz;
    return g.nt == 1 ? (int)sizeof(WinEntry<1>) : (int)sizeof(WinEntry<2>);
}

// maxn is rounded up to whole chunks of eight (the list holds them).
void launch_vlw_build(const int4 *st, const int32_t *cs, const int32_t *cell_sorted, const double *pos,
                      const Geom &g, int n, const int32_t *nblk_p, const int4 *blocks, uint16_t *nbr, int32_t *cnt,
                      int maxn, int32_t *flags, bool half, hipStream_t s)
{
    if (n <= 0) return;
    int cap = (int)window_block_cap(n, g);
    maxn = (maxn + 7) & ~7;
    int esz = half ? 1 : window_entry_size(g);
    if (build_float_ok(g)) {
        // relative single-precision windows (the scale of y and z is applied
        // when staging, so one variant serves every box shape)
        if (half)
            k_vlw_build<true, true, true><<<kWinGrid, 256, 0, s>>>(st, cs, cell_sorted, pos, g, n, nblk_p, cap,
                                                                    blocks, nbr, cnt, maxn, esz, flags);
        else
            k_vlw_build<true, false, true><<<kWinGrid, 256, 0, s>>>(st, cs, cell_sorted, pos, g, n, nblk_p, cap,
                                                                     blocks, nbr, cnt, maxn, esz, flags);
    } else if (half) {
        if (g.iso)
            k_vlw_build<true, true, false><<<kWinGrid, 256, 0, s>>>(st, cs, cell_sorted, pos, g, n, nblk_p, cap,
                                                                     blocks, nbr, cnt, maxn, esz, flags);
        else
            k_vlw_build<false, true, false><<<kWinGrid, 256, 0, s>>>(st, cs, cell_sorted, pos, g, n, nblk_p, cap,
                                                                      blocks, nbr, cnt, maxn, esz, flags);
    } else {
        if (g.iso)
            k_vlw_build<true, false, false><<<kWinGrid, 256, 0, s>>>(st, cs, cell_sorted, pos, g, n, nblk_p, cap,
                                                                      blocks, nbr, cnt, maxn, esz, flags);
        else
            k_vlw_build<false, false, false><<<kWinGrid, 256, 0, s>>>(st, cs, cell_sorted, pos, g, n, nblk_p, cap,
                                                                       blocks, nbr, cnt, maxn, esz, flags);
    }
}

int window_force_blocks() { return kWinGrid; }

template <int NT, bool ISO, bool EN, int LAYOUT>
static void vlw_launch(const ForceArgs &a, const Geom &g, int cap, hipStream_t s)
{
    if (a.fused)
        k_vlw_f32<NT, ISO, EN, true, LAYOUT><<<kWinGrid, 256, 0, s>>>(
            a.stage, a.cell_start, a.cell_sorted, g, a.n, a.w_nblk, cap, a.w_blk, a.w_nbr, a.nbr_count, a.tab, a.pos,
            (float *)a.force, a.partials, a.flags, a.ia, a.pos_out, a.stage_out);
    else
        k_vlw_f32<NT, ISO, EN, false, LAYOUT><<<kWinGrid, 256, 0, s>>>(
            a.stage, a.cell_start, a.cell_sorted, g, a.n, a.w_nblk, cap, a.w_blk, a.w_nbr, a.nbr_count, a.tab, a.pos,
            (float *)a.force, a.partials, a.flags, a.ia, a.pos_out, a.stage_out);
}

template <int NT, bool ISO, bool EN>
static void win_launch(const ForceArgs &a, const Geom &g, hipStream_t s)
{
    int cap = (int)window_block_cap(a.n, g);
    bool vl = a.container == MD_CONTAINER_VL;
    if (a.newton3) {
        if (vl)
            k_vlwh_f32<NT, ISO, EN><<<kWinGrid, 256, 0, s>>>(a.stage, a.cell_start, a.cell_sorted, g, a.n, a.w_nblk,
                                                            cap, a.w_blk, a.w_nbr, a.nbr_count, a.tab, a.pos,
                                                            (float *)a.force, a.partials, a.flags);
        else
            k_lcwh_f32<NT, ISO, EN><<<kWinGrid, 256, 0, s>>>(a.stage, a.cell_start, a.cell_sorted, g, a.n, a.w_nblk,
                                                            cap, a.w_blk, a.tab, a.pos, (float *)a.force, a.partials,
                                                            a.flags);
    } else if (vl) {
        if (NT == 1 && g.layout == MD_LAYOUT_ALIGNED)
            vlw_launch<NT, ISO, EN, MD_LAYOUT_ALIGNED>(a, g, cap, s);
        else if (NT == 1 && g.layout == MD_LAYOUT_SOA)
            vlw_launch<NT, ISO, EN, MD_LAYOUT_SOA>(a, g, cap, s);
        else
            vlw_launch<NT, ISO, EN, MD_LAYOUT_PACKED>(a, g, cap, s);
    } else {
        k_lcw_f32<NT, ISO, EN><<<kWinGrid, 256, 0, s>>>(a.stage, a.cell_start, a.cell_sorted, g, a.n, a.w_nblk, cap,
                                                       a.w_blk, a.tab, a.pos, (float *)a.force, a.partials,
                                                       a.flags);
    }
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

void launch_vlw_decode(const int32_t *cs, const int32_t *cell_sorted, const Geom &g, int n, const int32_t *nblk_p,
                       const int4 *blocks, const uint16_t *nbr, const int32_t *cnt, int maxr,
                       int32_t *counts, int32_t *rows, bool half, hipStream_t s)
{
    if (n <= 0) return;
    int cap = (int)window_block_cap(n, g);
    if (half)
        k_vlw_decode<true><<<kWinGrid, 256, 0, s>>>(cs, cell_sorted, g, n, nblk_p, cap, blocks, nbr, cnt, maxr,
                                                    1, counts, rows);
    else
        k_vlw_decode<false><<<kWinGrid, 256, 0, s>>>(cs, cell_sorted, g, n, nblk_p, cap, blocks, nbr, cnt, maxr,
                                                     window_entry_size(g), counts, rows);
}

}  // namespace mdlj

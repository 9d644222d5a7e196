// Many independent periodic systems advanced together: every phase of a time
// step (integration, cell build, forces) is one launch over all particles of
// all systems, and one rebuild interval of steps is captured into a HIP graph
// and replayed.  Each system has its own cubic box, cells and fixed-point
// scale; one particle type; linked cells or (FP32) Verlet lists, gather-only.
//
// Particles of system s occupy [offsets[s], offsets[s+1]) of every array.
// Global cell ids are system-major (cell_base[s] + local id), so the counting
// sort keeps every system inside its own range.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <type_traits>
#include <vector>

#include "entry_chunk.h"
#include "pair.h"

namespace mdlj {

int make_geom(const md_config &c, double csf, Geom &g);
void launch_zero(void *p, int64_t bytes, hipStream_t s);

// Per-system constants (device table).
struct BSys {
    int nc, nofs;           // cells per dimension (cubic box), distinct offsets
    int ofs[kMaxOfs];       // neighbour cell shifts mod nc
    int cell_base;          // first global cell id
    double L, inv_w, S;     // box, cells per length, fixed-point scale
    float disp2;            // skin check threshold in fixed-point units
    float hl;               // upper edge of the list radius's guard band, fixed-point units squared
    // pair constants in this box's fixed-point units (filled from lj on the device)
    float lo, hi, sig2, eps24, eps4, eps24w;
    double rc2, eps, sig;
};

__global__ void k_bprep(BSys *__restrict__ sys, int n_sys, const double *__restrict__ lj, double rc2)
{
    int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n_sys) return;
    BSys &b = sys[s];
    double u = b.L / 4294967296.0;
    double sig = lj[1], eps = lj[0];
    double r2u = rc2 / (u * u);
    b.lo = (float)(r2u * (1.0 - kBand));
    b.hi = (float)(r2u * (1.0 + kBand));
    b.sig2 = (float)(sig * sig / (u * u));
    b.eps24 = (float)(24.0 * eps / u);
    b.eps4 = (float)(4.0 * eps);
    b.eps24w = (float)(24.0 * eps);
    b.rc2 = rc2;
    b.eps = eps;
    b.sig = sig;
}

__device__ __forceinline__ int bcoord(double x, double inv_w, int nc, bool &bad)
{
    double t = x * inv_w;
    if (!(t >= 0.0 && t < (double)nc + 1.0)) {
        bad = true;
        return t > 0.0 ? nc - 1 : 0;
    }
    int c = (int)t;
    return c < nc - 1 ? c : nc - 1;
}

__device__ __forceinline__ uint32_t bquant(double x, double S)
{
    double q = x * S;
    q = q < 0.0 ? 0.0 : (q > 4294967295.0 ? 4294967295.0 : q);
    return (uint32_t)q;
}

// Cell of every particle in its own system's grid; one atomic per run of
// equal cells in a wavefront.
__global__ void k_bhist(int n, const double *__restrict__ pos, const int32_t *__restrict__ sys_of,
                        const BSys *__restrict__ sys, int32_t *__restrict__ cell_id, int32_t *__restrict__ slot,
                        int32_t *__restrict__ count, int32_t *__restrict__ flags)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    int lane = threadIdx.x & 63;
    int c = -1;
    if (i < n) {
        const BSys &b = sys[sys_of[i]];
        bool bad = false;
        size_t N = (size_t)n;
        int cx = bcoord(pos[i], b.inv_w, b.nc, bad);
        int cy = bcoord(pos[N + i], b.inv_w, b.nc, bad);
        int cz = bcoord(pos[2 * N + i], b.inv_w, b.nc, bad);
        if (bad) atomicOr(&flags[0], (int)MD_FLAG_NONFINITE);
        c = b.cell_base + (cz * b.nc + cy) * b.nc + cx;
        cell_id[i] = c;
    }
    int prev = __shfl_up(c, 1, 64);
    bool head = lane == 0 || prev != c;
    uint64_t heads = __ballot(head);
    uint64_t mask = lane == 63 ? ~0ull : ((2ull << lane) - 1);
    int hl = 63 - __builtin_clzll(heads & mask);
    uint64_t above = heads & ~mask;
    int next = above ? __builtin_ctzll(above) : 64;
    int base = 0;
    if (head && c >= 0) base = atomicAdd(&count[c], next - lane);
    base = __shfl(base, hl, 64);
    if (c >= 0) slot[i] = base + (lane - hl);
}

template <typename real>
__global__ void k_bgather(int n, const int32_t *__restrict__ perm, const int32_t *__restrict__ sys_of,
                          const BSys *__restrict__ sys, const double *__restrict__ pos, const real *__restrict__ vel,
                          const real *__restrict__ force, const int32_t *__restrict__ type,
                          const int32_t *__restrict__ ids, double *__restrict__ tpos, real *__restrict__ tvel,
                          real *__restrict__ tforce, int32_t *__restrict__ ttype, int32_t *__restrict__ tids,
                          const int32_t *__restrict__ cell_id, int32_t *__restrict__ cell_sorted,
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
    for (int d = 0; d < 3; d++) {
        tvel[d * N + k] = vel[d * N + src];
        tforce[d * N + k] = force[d * N + src];
    }
    int t = type[src];
    ttype[k] = t;
    tids[k] = ids[src];
    cell_sorted[k] = cell_id[src];
    double S = sys[sys_of[k]].S;  // systems keep their particle ranges
    int4 q;
    q.x = (int)bquant(x, S);
    q.y = (int)bquant(y, S);
    q.z = (int)bquant(z, S);
    q.w = t;
    stage[k] = q;
    stage_ref[k] = q;
}

__global__ void k_bstage(int n, const double *__restrict__ pos, const int32_t *__restrict__ type,
                         const int32_t *__restrict__ sys_of, const BSys *__restrict__ sys, int4 *__restrict__ stage)
{
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    size_t N = (size_t)n;
    double S = sys[sys_of[k]].S;
    stage[k] = make_int4((int)bquant(pos[k], S), (int)bquant(pos[N + k], S), (int)bquant(pos[2 * N + k], S), type[k]);
}

// FP64 linked-cell gather force, one thread per particle, its system's
// geometry (the FP32 passes are the work-item kernels below).  Writes
// per-particle energy partials when pe != nullptr.
__global__ __launch_bounds__(256) void k_bforce_f64(int n, const double *__restrict__ pos,
                                                    const int32_t *__restrict__ sys_of, const BSys *__restrict__ sys,
                                                    const int32_t *__restrict__ cs,
                                                    const int32_t *__restrict__ cell_sorted, double *__restrict__ F,
                                                    double *__restrict__ pe)
{
#pragma clang fp contract(off)
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    size_t N = (size_t)n;
    const BSys &b = sys[sys_of[i]];
    int nc = b.nc, nofs = b.nofs;
    int local = cell_sorted[i] - b.cell_base;
    int cx = local % nc, cy = (local / nc) % nc, cz = local / (nc * nc);
    double eu = 0.0, ew = 0.0, np = 0.0;
    double fx = 0, fy = 0, fz = 0;
    double xi = pos[i], yi = pos[N + i], zi = pos[2 * N + i];
    for (int a = 0; a < nofs; a++) {
        int zz = cz + b.ofs[a];
        zz = zz >= nc ? zz - nc : zz;
        for (int bb = 0; bb < nofs; bb++) {
            int yy = cy + b.ofs[bb];
            yy = yy >= nc ? yy - nc : yy;
            int row = b.cell_base + (zz * nc + yy) * nc;
            for (int e = 0; e < nofs; e++) {
                int xx = cx + b.ofs[e];
                xx = xx >= nc ? xx - nc : xx;
                int jb = cs[row + xx], je = cs[row + xx + 1];
                for (int j = jb; j < je; j++) {
                    if (j == i) continue;
                    double dx = min_image(xi - pos[j], b.L);
                    double dy = min_image(yi - pos[N + j], b.L);
                    double dz = min_image(zi - pos[2 * N + j], b.L);
                    double r2 = dx * dx + dy * dy + dz * dz;
                    if (!(r2 < b.rc2)) continue;
                    double phi, u;
                    lj_f64(r2, b.eps, b.sig, phi, u);
                    fx += phi * dx;
                    fy += phi * dy;
                    fz += phi * dz;
                    eu += u;
                    ew += phi * r2;
                    np += 1.0;
                }
            }
        }
    }
    F[i] = fx;
    F[N + i] = fy;
    F[2 * N + i] = fz;
    if (pe) {
        pe[i] = eu;
        pe[N + i] = ew;
        pe[2 * N + i] = np;
    }
}

// Work items of z-slabs: an item is a system and a range of z cell layers
// [z0, z0 + t), the largest items first.  The workgroup stages the layers the
// slab's stencils reach (the slab and h halo layers on either side, or the
// whole system) into LDS: their cell starts, as LDS indices, and their
// fixed-point positions.  When the staged layers hold more particles than the
// LDS tile (the slabs are sized from the mean density), the item reads its
// candidates from global memory instead.  Three kernels share the staging:
//  - kSlabCells, the linked-cell force: each thread takes the slab's particles
//    in turn and tests its stencil candidates 32 at a time (distance test into
//    a bit mask), evaluating the pair force only for those within the cutoff
//    band (guard-band pairs decided from the FP64 positions);
//  - kSlabBuild, the Verlet lists (Sec. 2.2.1): the same candidate tests
//    against the upper edge of the list radius's band (a superset of the
//    pairs within r_c + skin), the hits appended as 16-bit entries, eight to
//    a 16-byte chunk, chunk k of particle i at nbr[k N + i]: the LDS index of
//    the partner in the item's staging, or its index in its system when the
//    item reads global memory; cnt[i] is the full count;
//  - kSlabList, the force over those lists: each entry evaluated as above.  A
//    particle whose list outgrew the capacity (cnt[i] > maxn) walks its
//    stencil instead, so an overflow costs time, never a pair.
// The staging depends only on the cells, so the build and the force passes
// between two rebuilds make the same tile decision for every item.
#ifndef MDLJ_BATCH_LDS_KB
#define MDLJ_BATCH_LDS_KB 40
#endif
constexpr int kBSysLdsBytes = MDLJ_BATCH_LDS_KB * 1024;  // LDS tile per workgroup, at most
constexpr int kSlabCells = 0, kSlabBuild = 1, kSlabList = 2;

// LDS words of an item's tables: layer bases (K + 1), layer offsets (K), cell
// starts (K nc^2 + 1) and 16 words of positions read past the last batch.
__host__ __device__ static inline int64_t bslab_table_words(int64_t K, int64_t nc2)
{
    return 2 * K + 2 + K * nc2 + 12;
}

// Velocity Verlet update of particle i (the single-system integrator's
// steps, per-system box): with kick_prev the second half kick of the last
// step, with start the first half kick, drift, wrap, staging and skin check
// of the next (step: its index in the block, for the check).  The inputs are
// loaded first (bload) so that a force pass can have them in flight during
// its pair loop; positions are written to pos_out (the array they were read
// from in the integrator pass; another one when the force pass integrates,
// since other work items still read the current positions).
template <typename real>
struct BState {
    real vx, vy, vz;
    double x, y, z;
    int t, s;
    int4 ref;
};

template <typename real>
__device__ __forceinline__ BState<real> bload(int i, size_t N, const double *pos_in, const real *v,
                                              const int32_t *__restrict__ type, const int32_t *__restrict__ sys_of,
                                              const int4 *__restrict__ stage_ref)
{
    BState<real> b;
    b.vx = v[i];
    b.vy = v[N + i];
    b.vz = v[2 * N + i];
    b.x = pos_in[i];
    b.y = pos_in[N + i];
    b.z = pos_in[2 * N + i];
    b.t = type[i];
    b.s = sys_of[i];
    b.ref = stage_ref[i];
    return b;
}

template <typename real>
__device__ __forceinline__ void bupdate(int i, size_t N, const BState<real> &p, real fx, real fy, real fz,
                                        double *pos_out, real *__restrict__ v, const double *__restrict__ inv_mass,
                                        const BSys *__restrict__ sys, double hdt, double dt, int kick_prev,
                                        int start, int step, int4 *__restrict__ stage, int32_t *__restrict__ flags)
{
#pragma clang fp contract(off)
    real c = (real)(hdt * inv_mass[p.t]);
    real vx = p.vx, vy = p.vy, vz = p.vz;
    real ax = c * fx, ay = c * fy, az = c * fz;
    if (kick_prev) {
        vx += ax;
        vy += ay;
        vz += az;
    }
    if (start) {
        vx += ax;
        vy += ay;
        vz += az;
        const BSys &b = sys[p.s];
        double L = b.L;
        double xs[3] = {p.x + dt * (double)vx, p.y + dt * (double)vy, p.z + dt * (double)vz};
        uint32_t q[3];
        for (int d = 0; d < 3; d++) {
            double x = xs[d];
            if (x >= L) x -= L;
            else if (x < 0.0) x += L;
            if (x >= L) x = 0.0;
            pos_out[d * N + i] = x;
            q[d] = bquant(x, b.S);
            if (!(x == x)) atomicOr(&flags[0], (int)MD_FLAG_NONFINITE);
        }
        stage[i] = make_int4((int)q[0], (int)q[1], (int)q[2], p.t);
        float dx = (float)(int)(q[0] - (uint32_t)p.ref.x);
        float dy = (float)(int)(q[1] - (uint32_t)p.ref.y);
        float dz = (float)(int)(q[2] - (uint32_t)p.ref.z);
        if (dx * dx + dy * dy + dz * dz >= b.disp2) {
            atomicOr(&flags[0], (int)MD_FLAG_SKIN_EXCEEDED);
            atomicMin(&flags[1], step);
        }
    }
    v[i] = vx;
    v[N + i] = vy;
    v[2 * N + i] = vz;
}

// The next step's update fused into a force pass: the arrays and constants
// of bload and bupdate; positions and staged positions go to pos_out and
// stage_out.
struct BFuse {
    double *pos_out;
    float *v;
    const int32_t *type;
    const double *inv_mass;
    const int32_t *sys_of;
    double hdt, dt;
    int step;
    int4 *stage_out;
    const int4 *stage_ref;
    int32_t *flags;
};

template <int MODE, bool ENERGY, bool FUSED = false>
__global__ __launch_bounds__(256) void k_bslab(const int4 *__restrict__ items, const int64_t *__restrict__ offs,
                                               const int4 *__restrict__ st, const double *__restrict__ pos, int n,
                                               const BSys *__restrict__ sys, const int32_t *__restrict__ cs,
                                               const int32_t *__restrict__ cell_sorted, float *__restrict__ F,
                                               double *__restrict__ pe, int lds_bytes, uint4 *__restrict__ nbr,
                                               int32_t *__restrict__ cnt, int maxn, BFuse fu)
{
    extern __shared__ int sm[];
    const int4 it = items[blockIdx.x];
    const BSys &b = sys[it.x];
    const int z0 = it.y, t = it.z, h = it.w;
    const int p0 = (int)offs[it.x];
    const int nc = b.nc, nofs = b.nofs, nc2 = nc * nc, cbase = b.cell_base;
    const float lo = b.lo, hi = b.hi, sig2 = b.sig2, eps24 = b.eps24, eps4 = b.eps4, eps24w = b.eps24w;
    const float thr = MODE == kSlabBuild ? b.hl : hi;  // the candidate test
    const double rc2 = b.rc2, L = b.L;
    const bool whole = t + 2 * h >= nc;
    const int K = whole ? nc : t + 2 * h;          // staged layers
    const int zlo = whole ? 0 : (z0 - h + nc) % nc;  // the first of them
    int *lb = sm, *gofs = sm + K + 1, *scs = sm + 2 * K + 1;
    int *pp = scs + K * nc2 + 1;
    bool tile = 4 * bslab_table_words(K, nc2) <= lds_bytes;
    if (tile) {
        for (int k = threadIdx.x; k < K; k += blockDim.x) {
            int zz = (zlo + k) % nc;
            lb[k + 1] = cs[cbase + (zz + 1) * nc2] - cs[cbase + zz * nc2];
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            lb[0] = 0;
            for (int k = 0; k < K; k++) lb[k + 1] += lb[k];
        }
        __syncthreads();
        tile = 4 * (bslab_table_words(K, nc2) + 3 * (int64_t)lb[K]) <= lds_bytes;
    }
    if (tile) {
        for (int k = threadIdx.x; k < K; k += blockDim.x) {
            int zz = (zlo + k) % nc;
            gofs[k] = cs[cbase + zz * nc2] - p0 - lb[k];
        }
        __syncthreads();
        for (int k = 0; k < K; k++) {
            const int m = lb[k + 1] - lb[k], g = p0 + lb[k] + gofs[k];
            int *dst = pp + 3 * lb[k];
            for (int u = threadIdx.x; u < m; u += blockDim.x) {
                int4 q = st[g + u];
                dst[3 * u] = q.x;
                dst[3 * u + 1] = q.y;
                dst[3 * u + 2] = q.z;
            }
        }
        for (int e = threadIdx.x; e < K * nc2; e += blockDim.x) {
            int k = e / nc2, zz = (zlo + k) % nc;
            scs[e] = cs[cbase + zz * nc2 + (e - k * nc2)] - p0 - gofs[k];
        }
        if (threadIdx.x == 0) scs[K * nc2] = lb[K];
        __syncthreads();
    }
    const int i0 = cs[cbase + z0 * nc2] - p0, i1 = cs[cbase + (z0 + t) * nc2] - p0;
    size_t N = (size_t)n;
    for (int il = i0 + (int)threadIdx.x; il < i1; il += blockDim.x) {
        const int i = p0 + il;
        const int4 pi = st[i];
        BState<float> up;  // the next step's update: inputs in flight during the pair loop
        if (FUSED) up = bload<float>(i, N, pos, fu.v, fu.type, fu.sys_of, fu.stage_ref);
        float fx = 0.f, fy = 0.f, fz = 0.f, eus = 0.f, ews = 0.f;
        int np = 0;
        // pair with partner jg (global index) in the cell traversal
        auto pair = [&](int jg, int qx, int qy, int qz) {
            float dx = (float)(int)((uint32_t)pi.x - (uint32_t)qx);
            float dy = (float)(int)((uint32_t)pi.y - (uint32_t)qy);
            float dz = (float)(int)((uint32_t)pi.z - (uint32_t)qz);
            float r2 = dx * dx + dy * dy + dz * dz;
            bool in = r2 < lo;
            if (r2 >= lo && r2 < hi) in = exact_r2(pos, n, i, jg, L, L, L) < rc2;
            float ir2 = __builtin_amdgcn_rcpf(r2);
            float s2 = sig2 * ir2;
            float q = s2 * s2 * s2;
            float aa = q * (2.0f * q - 1.0f);
            float phi = in ? eps24 * ir2 * aa : 0.0f;
            fx += phi * dx;
            fy += phi * dy;
            fz += phi * dz;
            if (ENERGY) {
                eus += in ? eps4 * q * (q - 1.0f) : 0.0f;
                ews += in ? eps24w * aa : 0.0f;
                np += in ? 1 : 0;
            }
        };
        int c = 0;  // list entries (build)
        EntryChunk ck;
        uint4 *row = nbr + i;
        auto hit = [&](int jl, int jg, int qx, int qy, int qz) {
            if (MODE == kSlabBuild) {
                ck.push((uint32_t)(tile ? jl : jg - p0));
                c++;
                if ((c & 7) == 0 && c <= maxn) row[(size_t)((c >> 3) - 1) * N] = ck.word();
            } else {
                pair(jg, qx, qy, qz);
            }
        };
        bool stencil = true;
        if (MODE == kSlabList) {
            const int cl = cnt[i];
            if (cl <= maxn) {
                stencil = false;
                // sums in units of the one type's factors (24 eps for the
                // force and the virial, 4 eps for the energy), applied once
                float gx = 0.f, gy = 0.f, gz = 0.f, gu = 0.f, gw = 0.f;
                const uint32_t lob = __float_as_uint(lo), wb = __float_as_uint(hi) - lob;
                auto walk = [&](auto tile_c) {
                    constexpr bool TILE = decltype(tile_c)::value;
                    auto at = [&](int e, float &dx, float &dy, float &dz) {
                        int qx, qy, qz;
                        if (TILE) {
                            const int *q = pp + 3 * e;
                            qx = q[0];
                            qy = q[1];
                            qz = q[2];
                        } else {
                            const int4 q = st[p0 + e];
                            qx = q.x;
                            qy = q.y;
                            qz = q.z;
                        }
                        dx = (float)(int)((uint32_t)pi.x - (uint32_t)qx);
                        dy = (float)(int)((uint32_t)pi.y - (uint32_t)qy);
                        dz = (float)(int)((uint32_t)pi.z - (uint32_t)qz);
                        return dx * dx + dy * dy + dz * dz;
                    };
                    auto add = [&](float r2, float dx, float dy, float dz, bool in) {
                        // a pair outside gets 1/r^2 = 0, which zeroes every term
                        float ir2 = in ? __builtin_amdgcn_rcpf(r2) : 0.0f;
                        float s2 = sig2 * ir2;
                        float q = s2 * s2 * s2;
                        float aa = q * (2.0f * q - 1.0f);
                        float phi = ir2 * aa;
                        gx += phi * dx;
                        gy += phi * dy;
                        gz += phi * dz;
                        if (ENERGY) {
                            gu += q * (q - 1.0f);
                            gw += aa;
                            np += in ? 1 : 0;
                        }
                    };
                    const uint4 *lrow = nbr + i;
                    uint4 nx = lrow[0];
                    for (int q0 = 0; q0 < cl; q0 += 8) {
                        const uint32_t w[4] = {nx.x, nx.y, nx.z, nx.w};
                        if (q0 + 8 < cl) nx = lrow[(size_t)((q0 >> 3) + 1) * N];  // the next chunk in flight
                        bool band = false;
#pragma unroll
                        for (int u = 0; u < 8; u++) {
                            const int e = (int)((w[u >> 1] >> (16 * (u & 1))) & 0xffffu);
                            const bool valid = q0 + u < cl;
                            float dx, dy, dz;
                            const float r2 = at(e, dx, dy, dz);
                            band = band || (valid && __float_as_uint(r2) - lob < wb);
                            add(r2, dx, dy, dz, valid && r2 < lo);
                        }
                        if (band) {
                            // rare: the chunk's guard-band entries, decided
                            // from the FP64 positions
                            for (int u = 0; u < 8 && q0 + u < cl; u++) {
                                const int e = (int)((w[u >> 1] >> (16 * (u & 1))) & 0xffffu);
                                float dx, dy, dz;
                                const float r2 = at(e, dx, dy, dz);
                                if (__float_as_uint(r2) - lob < wb) {
                                    int jg = p0 + e;
                                    if (TILE) {
                                        int k = 0;
                                        while (lb[k + 1] <= e) k++;
                                        jg = e + gofs[k] + p0;
                                    }
                                    add(r2, dx, dy, dz, exact_r2(pos, n, i, jg, L, L, L) < rc2);
                                }
                            }
                        }
                    }
                };
                if (cl > 0) {
                    if (tile)
                        walk(std::true_type{});
                    else
                        walk(std::false_type{});
                }
                fx = eps24 * gx;
                fy = eps24 * gy;
                fz = eps24 * gz;
                if (ENERGY) {
                    eus = eps4 * gu;
                    ews = eps24w * gw;
                }
            }
        }
        if (stencil) {
            const int local = cell_sorted[i] - cbase;
            const int cx = local % nc, cy = (local / nc) % nc, cz = local / nc2;
            const int self = tile ? il - gofs[(cz - zlo + nc) % nc] : 0;  // the particle's LDS index
            // staged candidates jb .. je - 1 (LDS indices; layer offset gz):
            // tested 32 at a time, the hits passed on
            auto scan = [&](int jb, int je, int gz) {
                for (int base = jb; base < je; base += 32) {
                    const int m = min(32, je - base);
                    uint32_t mask = 0;
                    int nb = 0;
                    for (; nb < m; nb += 4)
                        for (int u = 0; u < 4; u++) {
                            const int *q = pp + 3 * (base + nb + u);
                            float dx = (float)(int)((uint32_t)pi.x - (uint32_t)q[0]);
                            float dy = (float)(int)((uint32_t)pi.y - (uint32_t)q[1]);
                            float dz = (float)(int)((uint32_t)pi.z - (uint32_t)q[2]);
                            float r2 = dx * dx + dy * dy + dz * dz;
                            mask = mask + mask + (r2 < thr ? 1u : 0u);
                        }
                    mask >>= nb - m;  // the reads past the batch
                    unsigned us = (unsigned)(self - base);
                    if (us < (unsigned)m) mask &= ~(1u << (m - 1 - us));
                    while (mask) {
                        int hb = 31 - __builtin_clz(mask);
                        mask ^= 1u << hb;
                        int jl = base + m - 1 - hb;
                        const int *q = pp + 3 * jl;
                        hit(jl, jl + gz, q[0], q[1], q[2]);
                    }
                }
            };
            for (int a = 0; a < nofs; a++) {
                int zz = cz + b.ofs[a];
                zz = zz >= nc ? zz - nc : zz;
                const int k = (zz - zlo + nc) % nc;  // < K: the slab's stencils stay in the staged layers
                const int gz = tile ? gofs[k] + p0 : 0;
                for (int bb = 0; bb < nofs; bb++) {
                    int yy = cy + b.ofs[bb];
                    yy = yy >= nc ? yy - nc : yy;
                    for (int e = 0; e < nofs; e++) {
                        int xx = cx + b.ofs[e];
                        xx = xx >= nc ? xx - nc : xx;
                        if (tile) {
                            const int cc = (k * nc + yy) * nc + xx;
                            scan(scs[cc], scs[cc + 1], gz);
                        } else {
                            const int cc = cbase + (zz * nc + yy) * nc + xx;
                            const int jb = cs[cc], je = cs[cc + 1];
                            for (int j = jb; j < je; j++)
                                if (j != i) {
                                    int4 q = st[j];
                                    if (MODE == kSlabBuild) {
                                        float dx = (float)(int)((uint32_t)pi.x - (uint32_t)q.x);
                                        float dy = (float)(int)((uint32_t)pi.y - (uint32_t)q.y);
                                        float dz = (float)(int)((uint32_t)pi.z - (uint32_t)q.z);
                                        if (dx * dx + dy * dy + dz * dz < thr) hit(0, j, q.x, q.y, q.z);
                                    } else {
                                        hit(0, j, q.x, q.y, q.z);
                                    }
                                }
                        }
                    }
                }
            }
        }
        if (MODE == kSlabBuild) {
            if ((c & 7) != 0 && c < maxn) {
                for (int e = c & 7; e < 8; e++) ck.push(0u);
                row[(size_t)(c >> 3) * N] = ck.word();
            }
            cnt[i] = c;
        } else {
            F[i] = fx;
            F[N + i] = fy;
            F[2 * N + i] = fz;
            if (FUSED)
                bupdate<float>(i, N, up, fx, fy, fz, fu.pos_out, fu.v, fu.inv_mass, sys, fu.hdt, fu.dt, 1, 1, fu.step,
                               fu.stage_out, fu.flags);
            if (ENERGY) {
                pe[i] = eus;
                pe[N + i] = ews;
                pe[2 * N + i] = (double)np;
            }
        }
    }
}

// Velocity Verlet pass (as the single-system integrator) with per-system box.
template <typename real>
__global__ __launch_bounds__(256) void k_bintegrate(int n, double *__restrict__ pos, real *__restrict__ v,
                                                    const real *__restrict__ F, const int32_t *__restrict__ type,
                                                    const double *__restrict__ inv_mass, const int32_t *__restrict__ sys_of,
                                                    const BSys *__restrict__ sys, double hdt, double dt, int kick_prev,
                                                    int start, int step, int4 *__restrict__ stage,
                                                    const int4 *__restrict__ stage_ref, int32_t *__restrict__ flags)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    size_t N = (size_t)n;
    const BState<real> p = bload<real>(i, N, pos, v, type, sys_of, stage_ref);
    bupdate<real>(i, N, p, F[i], F[N + i], F[2 * N + i], pos, v, inv_mass, sys, hdt, dt, kick_prev, start, step,
                  stage, flags);
}

// Per-system sums of the per-particle energy partials, in a fixed order.
__global__ void k_bsys_reduce(int n, const int64_t *__restrict__ offs, const double *__restrict__ pe, int fp32,
                              double *__restrict__ out)
{
    __shared__ double sh[16];
    int s = blockIdx.x;
    size_t N = (size_t)n;
    double v[4] = {0, 0, 0, 0};
    for (int64_t i = offs[s] + threadIdx.x; i < offs[s + 1]; i += blockDim.x) {
        v[0] += pe[i];
        v[1] += pe[N + i];
        v[2] += pe[2 * N + i];
    }
    block_sum4(v, sh);
    if (threadIdx.x == 0) {
        out[4 * s + 0] = 0.5 * v[0];
        out[4 * s + 1] = 0.5 * v[1];
        out[4 * s + 2] = 0.5 * v[2];
        out[4 * s + 3] = 0.0;
    }
    (void)fp32;
}

}  // namespace mdlj

using namespace mdlj;

// ------------------------------------------------------------------ handle

struct md_batch {
    md_config cfg;
    int n_sys = 0;
    int64_t n = 0;
    int device = 0;
    std::vector<int64_t> offsets;
    std::vector<BSys> hsys;
    BSys *sys = nullptr;
    int64_t *d_offs = nullptr;
    int4 *items = nullptr;  // the FP32 force kernel's work items (system, z0, t, halo), largest first
    int n_items = 0;
    int sys_lds = 0;        // that kernel's LDS tile (bytes)
    // Verlet lists (FP32): chunks of eight 16-bit entries, [maxn / 8][n], and
    // each particle's full count; built with the cells
    bool lists = false;
    int maxn = 0;
    uint4 *nbr = nullptr;
    int32_t *bcnt = nullptr;
    // Rebuild interval in use (at most cfg.rebuild_interval): shortened to the
    // block step of a skin violation, lengthened by one after `backoff` blocks
    // in a row without one (the backoff doubling after each failed try).
    int r_eff = 1, calm = 0, backoff = 32;
    int64_t n_rebuilds = 0, n_forced = 0, n_steps = 0;  // since md_batch_create
    int32_t *sys_of = nullptr;
    int64_t ncell = 0;
    int32_t *cell_id = nullptr, *slot = nullptr, *perm = nullptr, *perm2 = nullptr, *count = nullptr,
            *cell_start = nullptr, *cell_sorted = nullptr, *scan = nullptr;
    double *tpos = nullptr;
    void *tvel = nullptr, *tforce = nullptr;
    int32_t *ttype = nullptr, *tids = nullptr;
    int4 *stage = nullptr, *stage_ref = nullptr;
    int4 *stage2 = nullptr;  // FP32: the staged positions a fused force pass writes
    double *pe = nullptr;
    double *snap_pos = nullptr;
    void *snap_vel = nullptr;
    int32_t *flags = nullptr;
    uint32_t *host_flags = nullptr;
    bool built = false;
    // captured rebuild interval
    hipGraphExec_t exec = nullptr;
    hipGraph_t graph = nullptr;
    const void *graph_key[8] = {nullptr};
    double graph_dt = 0.0;
    int graph_R = 0;
    hipStream_t cap = nullptr;  // capture stream
};

static size_t bsize(const md_config &c) { return c.precision == MD_FP64 ? 8 : 4; }

static void batch_free(md_batch *b)
{
    void *p[] = {b->sys,   b->d_offs, b->items, b->sys_of, b->cell_id,  b->slot,      b->perm,       b->perm2,
                 b->count, b->cell_start, b->cell_sorted, b->scan, b->tpos,  b->tvel,       b->tforce,
                 b->ttype, b->tids,   b->stage,  b->stage_ref, b->pe,       b->snap_pos,   b->snap_vel, b->flags,
                 b->nbr,   b->bcnt,   b->stage2};
    for (void *q : p)
        if (q) (void)hipFree(q);
    if (b->host_flags) (void)hipHostFree(b->host_flags);
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    if (b->cap) (void)hipStreamDestroy(b->cap);
}

// Work items of the FP32 force kernel.  A system whose layers all fit the LDS
// tile is one item; a larger one is cut into z-slabs of t layers, t the
// largest for which the slab and its halo layers fit with 20 % headroom over
// the mean density.  Items run largest first.
static bool upload_items(md_batch *b)
{
    std::vector<int4> items;
    std::vector<int64_t> est;
    int64_t lds = 0;
    bool slabs = false;
    for (int s = 0; s < b->n_sys; s++) {
        const BSys &y = b->hsys[s];
        const int nc = y.nc;
        const int64_t nc2 = (int64_t)nc * nc, ns = b->offsets[s + 1] - b->offsets[s];
        int h = 0;
        for (int a = 0; a < y.nofs; a++) h = std::max(h, std::min(y.ofs[a], nc - y.ofs[a]));
        const int64_t whole = 4 * (bslab_table_words(nc, nc2) + 3 * ns);
        int t = nc;
        if (whole > kBSysLdsBytes) {
            slabs = true;
            t = 1;
            for (int tt = nc - 1; tt >= 1; tt--) {
                const int K = tt + 2 * h;
                if (K >= nc) continue;
                const double need = 4.0 * ((double)bslab_table_words(K, nc2) + 3.0 * 1.2 * ns * K / nc);
                if (need <= kBSysLdsBytes) {
                    t = tt;
                    break;
                }
            }
        } else {
            lds = std::max(lds, whole);
        }
        for (int z0 = 0; z0 < nc; z0 += t) {
            const int tt = std::min(t, nc - z0);
            items.push_back(make_int4(s, z0, tt, h));
            est.push_back(ns * tt / nc);
        }
    }
    std::vector<int> idx(items.size());
    for (size_t k = 0; k < idx.size(); k++) idx[k] = (int)k;
    std::stable_sort(idx.begin(), idx.end(), [&](int a, int c) { return est[a] > est[c]; });
    std::vector<int4> sorted(items.size());
    for (size_t k = 0; k < idx.size(); k++) sorted[k] = items[idx[k]];
    b->n_items = (int)sorted.size();
    b->sys_lds = slabs ? kBSysLdsBytes : (int)lds;
    if (hipMalloc((void **)&b->items, sizeof(int4) * sorted.size()) != hipSuccess) return false;
    return hipMemcpy(b->items, sorted.data(), sizeof(int4) * sorted.size(), hipMemcpyHostToDevice) == hipSuccess;
}

extern "C" int md_batch_create(const md_config *cfg, int32_t n_sys, const int64_t *offsets, const double *boxes,
                               md_batch **out)
{
    if (!out) return fail(MD_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (!cfg || !offsets || !boxes || n_sys < 1) return fail(MD_ERR_INVALID_ARG, "bad arguments");
    if (cfg->n_types != 1) return fail(MD_ERR_INVALID_ARG, "batched systems hold one particle type");
    if (cfg->precision != MD_FP32 && cfg->precision != MD_FP64) return fail(MD_ERR_INVALID_ARG, "bad precision");
    if (!(cfg->rc2[0] > 0.0) || !(cfg->skin >= 0.0) || !(cfg->csf >= 0.5 && cfg->csf <= 1.0))
        return fail(MD_ERR_INVALID_ARG, "bad cutoff, skin or csf");
    if (cfg->rebuild_interval < 1) return fail(MD_ERR_INVALID_ARG, "rebuild_interval must be >= 1");
    if (cfg->container != MD_CONTAINER_LC && cfg->container != MD_CONTAINER_VL)
        return fail(MD_ERR_INVALID_ARG, "batched systems use linked cells or Verlet lists");
    if (cfg->newton3 != MD_N3L_OFF) return fail(MD_ERR_INVALID_ARG, "batched systems are gather-only (newton3 off)");
    const bool lists = cfg->container == MD_CONTAINER_VL;
    if (lists && cfg->precision != MD_FP32) return fail(MD_ERR_INVALID_ARG, "batched Verlet lists are FP32");
    if (lists && !(cfg->max_neighbors >= 1 && cfg->max_neighbors <= 4096))
        return fail(MD_ERR_INVALID_ARG, "max_neighbors out of range");
    if (offsets[0] != 0) return fail(MD_ERR_INVALID_ARG, "offsets[0] must be 0");
    for (int s = 0; s < n_sys; s++) {
        if (offsets[s + 1] < offsets[s]) return fail(MD_ERR_INVALID_ARG, "offsets must be non-decreasing");
        if (lists && offsets[s + 1] - offsets[s] > 65536)
            return fail(MD_ERR_INVALID_ARG, "batched Verlet lists hold systems of at most 65536 particles");
    }
    if (offsets[n_sys] > (int64_t)INT32_MAX / 3) return fail(MD_ERR_INVALID_ARG, "too many particles");
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return fail(MD_ERR_NO_DEVICE, "no HIP device");
    md_batch *b = new md_batch();
    b->cfg = *cfg;
    b->r_eff = std::max(1, cfg->rebuild_interval);
    b->n_sys = n_sys;
    b->n = offsets[n_sys];
    b->offsets.assign(offsets, offsets + n_sys + 1);
    (void)hipGetDevice(&b->device);
    int64_t cells = 0;
    for (int s = 0; s < n_sys; s++) {
        const double *bx = boxes + 3 * s;
        if (!(bx[0] > 0.0) || bx[0] != bx[1] || bx[1] != bx[2]) {
            delete b;
            return fail(MD_ERR_INVALID_ARG, "batched boxes must be cubic (system " + std::to_string(s) + ")");
        }
        md_config c = *cfg;
        c.box[0] = c.box[1] = c.box[2] = bx[0];
        Geom g;
        int rc = make_geom(c, cfg->csf, g);
        if (rc) {
            delete b;
            return fail(rc, "system " + std::to_string(s) + ": " + md_last_error());
        }
        BSys y;
        memset(&y, 0, sizeof(y));
        y.nc = g.nc[0];
        y.nofs = g.nofs[0];
        for (int k = 0; k < kMaxOfs; k++) y.ofs[k] = g.ofs[0][k];
        y.cell_base = (int)cells;
        y.L = bx[0];
        y.inv_w = g.inv_w[0];
        y.S = g.S[0];
        y.disp2 = g.disp2;
        {
            const double u = bx[0] / 4294967296.0, rl = sqrt(cfg->rc2[0]) + cfg->skin;
            y.hl = (float)(rl * rl / (u * u) * (1.0 + kBand));
        }
        cells += g.ncell;
        if (cells > (int64_t)1 << 30) {
            delete b;
            return fail(MD_ERR_INVALID_ARG, "too many cells");
        }
        b->hsys.push_back(y);
    }
    b->ncell = cells;
    int64_t n = std::max<int64_t>(b->n, 1);
    size_t rs = bsize(*cfg);
    std::vector<int32_t> sys_of(n, 0);
    for (int s = 0; s < n_sys; s++)
        for (int64_t i = offsets[s]; i < offsets[s + 1]; i++) sys_of[i] = s;
    bool ok = true;
    auto A = [&](void **p, size_t bytes) {
        if (ok && hipMalloc(p, bytes ? bytes : 1) != hipSuccess) ok = false;
    };
    A((void **)&b->sys, sizeof(BSys) * n_sys);
    A((void **)&b->d_offs, sizeof(int64_t) * (n_sys + 1));

    A((void **)&b->sys_of, 4 * n);
    A((void **)&b->cell_id, 4 * n);
    A((void **)&b->slot, 4 * n);
    A((void **)&b->perm, 4 * n);
    A((void **)&b->perm2, 4 * n);
    A((void **)&b->cell_sorted, 4 * n);
    A((void **)&b->count, 4 * (cells + 1));
    A((void **)&b->cell_start, 4 * (cells + 1));
    A((void **)&b->scan, 4 * (scan_scratch_size(cells + 1) + 64));
    A((void **)&b->tpos, 24 * n);
    A(&b->tvel, 3 * rs * n);
    A(&b->tforce, 3 * rs * n);
    A((void **)&b->ttype, 4 * n);
    A((void **)&b->tids, 4 * n);
    A((void **)&b->stage, 16 * n);
    A((void **)&b->stage_ref, 16 * n);
    if (cfg->precision == MD_FP32) A((void **)&b->stage2, 16 * n);
    A((void **)&b->pe, 24 * n);
    A((void **)&b->snap_pos, 24 * n);
    A(&b->snap_vel, 3 * rs * n);
    A((void **)&b->flags, 16);
    if (lists) {
        // capacity: the configured row length, or 1.3 times the mean count
        // within the list radius of the densest system if that is more, in
        // whole chunks (a longer list falls back to the stencil)
        double rho = 0.0, rl = sqrt(cfg->rc2[0]) + cfg->skin;
        for (int s = 0; s < n_sys; s++) {
            const double L = boxes[3 * s];
            rho = std::max(rho, (double)(offsets[s + 1] - offsets[s]) / (L * L * L));
        }
        const double est = 1.3 * rho * 4.0 / 3.0 * M_PI * rl * rl * rl + 8.0;
        int maxn = std::max(cfg->max_neighbors, (int)std::min(est, 1024.0));
        b->maxn = (maxn + 7) / 8 * 8;
        b->lists = true;
        A((void **)&b->nbr, (size_t)2 * b->maxn * n);
        A((void **)&b->bcnt, 4 * n);
    }
    if (ok && hipHostMalloc((void **)&b->host_flags, 16, 0) != hipSuccess) ok = false;
    if (ok) ok = hipMemcpy(b->sys, b->hsys.data(), sizeof(BSys) * n_sys, hipMemcpyHostToDevice) == hipSuccess;
    if (ok) ok = hipMemcpy(b->d_offs, offsets, sizeof(int64_t) * (n_sys + 1), hipMemcpyHostToDevice) == hipSuccess;
    if (ok) ok = hipMemcpy(b->sys_of, sys_of.data(), 4 * n, hipMemcpyHostToDevice) == hipSuccess;
    if (ok) ok = upload_items(b);
    int32_t init[4] = {0, INT32_MAX, 0, 0};
    if (ok) ok = hipMemcpy(b->flags, init, sizeof(init), hipMemcpyHostToDevice) == hipSuccess;
    if (!ok) {
        batch_free(b);
        delete b;
        return fail(MD_ERR_HIP, "device allocation failed");
    }
    *out = b;
    return MD_OK;
}

extern "C" int md_batch_get_counters(const md_batch *b, int64_t *out)
{
    if (!b || !out) return fail(MD_ERR_INVALID_ARG, "NULL argument");
    out[0] = b->n_rebuilds;
    out[1] = b->n_forced;
    out[2] = b->n_steps;
    out[3] = b->r_eff;
    return MD_OK;
}

extern "C" void md_batch_destroy(md_batch *b)
{
    if (!b) return;
    (void)hipSetDevice(b->device);
    (void)hipDeviceSynchronize();
    batch_free(b);
    delete b;
}

static int bblocks(int64_t n) { return (int)((n + 255) / 256); }

static int batch_rebuild(md_batch *b, double *pos, void *vel, void *force, int32_t *type, int32_t *ids,
                         hipStream_t s)
{
    int n = (int)b->n;
    size_t rs = bsize(b->cfg);
    launch_fill_i32(b->count, 0, b->ncell, s);
    if (n > 0) k_bhist<<<bblocks(n), 256, 0, s>>>(n, pos, b->sys_of, b->sys, b->cell_id, b->slot, b->count, b->flags);
    launch_scan(b->count, b->cell_start, b->ncell, b->scan, s);
    launch_scatter(n, b->cell_id, b->slot, b->cell_start, b->perm, s);
    launch_cell_sort(n, b->cell_start, ids, b->cell_id, b->perm, b->slot, b->cell_sorted, b->perm2, s);
    if (n > 0) {
        if (b->cfg.precision == MD_FP64)
            k_bgather<double><<<bblocks(n), 256, 0, s>>>(
                n, b->perm2, b->sys_of, b->sys, pos, (const double *)vel, (const double *)force, type, ids, b->tpos,
                (double *)b->tvel, (double *)b->tforce, b->ttype, b->tids, b->cell_id, b->cell_sorted, b->stage,
                b->stage_ref);
        else
            k_bgather<float><<<bblocks(n), 256, 0, s>>>(n, b->perm2, b->sys_of, b->sys, pos, (const float *)vel,
                                                        (const float *)force, type, ids, b->tpos, (float *)b->tvel,
                                                        (float *)b->tforce, b->ttype, b->tids, b->cell_id,
                                                        b->cell_sorted, b->stage, b->stage_ref);
        if (b->lists)
            k_bslab<kSlabBuild, false><<<b->n_items, 256, b->sys_lds, s>>>(
                b->items, b->d_offs, b->stage, b->tpos, n, b->sys, b->cell_start, b->cell_sorted, nullptr, nullptr,
                b->sys_lds, b->nbr, b->bcnt, b->maxn, BFuse{});
        MD_HIP(hipMemcpyAsync(pos, b->tpos, 24 * (size_t)n, hipMemcpyDeviceToDevice, s));
        MD_HIP(hipMemcpyAsync(vel, b->tvel, 3 * rs * n, hipMemcpyDeviceToDevice, s));
        MD_HIP(hipMemcpyAsync(force, b->tforce, 3 * rs * n, hipMemcpyDeviceToDevice, s));
        MD_HIP(hipMemcpyAsync(type, b->ttype, 4 * (size_t)n, hipMemcpyDeviceToDevice, s));
        MD_HIP(hipMemcpyAsync(ids, b->tids, 4 * (size_t)n, hipMemcpyDeviceToDevice, s));
    }
    b->built = true;
    return MD_OK;
}

// Forces at positions pos (staged copy st).  FP32 with fu: the pass also
// advances every particle to the next step (BFuse).
static void batch_forces(md_batch *b, const double *pos, void *force, bool energy, hipStream_t s,
                         const int4 *st = nullptr, const BFuse *fu = nullptr)
{
    int n = (int)b->n;
    if (n <= 0) return;
    if (!st) st = b->stage;
    if (b->cfg.precision == MD_FP64)
        k_bforce_f64<<<bblocks(n), 256, 0, s>>>(n, pos, b->sys_of, b->sys, b->cell_start, b->cell_sorted,
                                                 (double *)force, energy ? b->pe : nullptr);
    else {
        const BFuse f = fu ? *fu : BFuse{};
        auto go = [&](auto kern) {
            kern<<<b->n_items, 256, b->sys_lds, s>>>(b->items, b->d_offs, st, pos, n, b->sys, b->cell_start,
                                                     b->cell_sorted, (float *)force, energy ? b->pe : nullptr,
                                                     b->sys_lds, b->nbr, b->bcnt, b->maxn, f);
        };
        if (fu) {
            if (b->lists)
                go(k_bslab<kSlabList, false, true>);
            else
                go(k_bslab<kSlabCells, false, true>);
        } else if (b->lists) {
            energy ? go(k_bslab<kSlabList, true>) : go(k_bslab<kSlabList, false>);
        } else {
            energy ? go(k_bslab<kSlabCells, true>) : go(k_bslab<kSlabCells, false>);
        }
    }
}

static void batch_integrate(md_batch *b, double *pos, void *vel, const void *force, const int32_t *type,
                            const double *inv_mass, double dt, int kick_prev, int start, int step, hipStream_t s)
{
    int n = (int)b->n;
    if (n <= 0) return;
    if (b->cfg.precision == MD_FP64)
        k_bintegrate<double><<<bblocks(n), 256, 0, s>>>(n, pos, (double *)vel, (const double *)force, type, inv_mass,
                                                        b->sys_of, b->sys, 0.5 * dt, dt, kick_prev, start, step,
                                                        b->stage, b->stage_ref, b->flags);
    else
        k_bintegrate<float><<<bblocks(n), 256, 0, s>>>(n, pos, (float *)vel, (const float *)force, type, inv_mass,
                                                       b->sys_of, b->sys, 0.5 * dt, dt, kick_prev, start, step,
                                                       b->stage, b->stage_ref, b->flags);
}

extern "C" int md_batch_build_cells(md_batch *b, double *pos, void *vel, void *force, int32_t *type, int32_t *ids,
                                    void *stream)
{
    if (!b) return fail(MD_ERR_INVALID_ARG, "batch is NULL");
    if (b->n > 0 && (!pos || !vel || !force || !type || !ids))
        return fail(MD_ERR_INVALID_ARG, "pos, vel, force, type, ids must not be NULL");
    MD_HIP(hipSetDevice(b->device));
    return batch_rebuild(b, pos, vel, force, type, ids, (hipStream_t)stream);
}

extern "C" int md_batch_compute_forces(md_batch *b, const double *pos, const int32_t *type, const double *lj,
                                       void *force, double *out, void *stream)
{
    if (!b) return fail(MD_ERR_INVALID_ARG, "batch is NULL");
    if (!lj || (b->n > 0 && (!pos || !type || !force))) return fail(MD_ERR_INVALID_ARG, "NULL argument");
    if (!b->built) return fail(MD_ERR_NOT_BUILT, "md_batch_build_cells must be called first");
    MD_HIP(hipSetDevice(b->device));
    hipStream_t s = (hipStream_t)stream;
    k_bprep<<<(b->n_sys + 255) / 256, 256, 0, s>>>(b->sys, b->n_sys, lj, b->cfg.rc2[0]);
    int n = (int)b->n;
    if (n > 0) k_bstage<<<bblocks(n), 256, 0, s>>>(n, pos, type, b->sys_of, b->sys, b->stage);
    batch_forces(b, pos, force, out != nullptr, s);
    if (out) {
        if (n == 0) launch_zero(b->pe, 24, s);
        k_bsys_reduce<<<b->n_sys, 256, 0, s>>>(n, b->d_offs, b->pe, b->cfg.precision == MD_FP32, out);
    }
    return MD_OK;
}

// One rebuild interval starting at step s0 (first step: integrate, rebuild,
// snapshot, forces; then R - 1 plain steps).  The skin-check step indices are
// relative to the block, so the same sequence can be captured and replayed.
struct BatchCtx {
    double *pos;
    void *vel, *force;
    int32_t *type, *ids;
    const double *inv_mass;
    double dt;
    hipStream_t s;
};

static int batch_block_ops(md_batch *b, const BatchCtx &c, int len, bool first_of_run)
{
    size_t rs = bsize(b->cfg);
    size_t n = (size_t)b->n;
    launch_fill_i32(b->flags + 1, INT32_MAX, 1, c.s);
    batch_integrate(b, c.pos, c.vel, c.force, c.type, c.inv_mass, c.dt, first_of_run ? 0 : 1, 1, 0, c.s);
    int rc = batch_rebuild(b, c.pos, c.vel, c.force, c.type, c.ids, c.s);
    if (rc) return rc;
    launch_fill_i32(b->flags + 1, INT32_MAX, 1, c.s);  // the check restarts from this build
    if (n > 0) {
        MD_HIP(hipMemcpyAsync(b->snap_pos, c.pos, 24 * n, hipMemcpyDeviceToDevice, c.s));
        MD_HIP(hipMemcpyAsync(b->snap_vel, c.vel, 3 * rs * n, hipMemcpyDeviceToDevice, c.s));
    }
    if (b->cfg.precision == MD_FP32 && n > 0) {
        // the force pass of step k - 1 also advances the particles to step k;
        // positions and staged positions alternate between two buffers
        // (other work items read the current ones during the pass), the
        // cell build's output standing in for the second position buffer
        double *cur = c.pos, *alt = b->tpos;
        int4 *cst = b->stage, *ast = b->stage2;
        for (int k = 1; k < len; k++) {
            const BFuse fu{alt,   (float *)c.vel, c.type, c.inv_mass, b->sys_of, 0.5 * c.dt, c.dt, k,
                           ast, b->stage_ref,   b->flags};
            batch_forces(b, cur, c.force, false, c.s, cst, &fu);
            std::swap(cur, alt);
            std::swap(cst, ast);
        }
        batch_forces(b, cur, c.force, false, c.s, cst);
        // the block ends with the positions in the caller's array (the next
        // block's integrator and any restore stage them again from there)
        if (cur != c.pos) MD_HIP(hipMemcpyAsync(c.pos, cur, 24 * n, hipMemcpyDeviceToDevice, c.s));
        return MD_OK;
    }
    batch_forces(b, c.pos, c.force, false, c.s);
    for (int k = 1; k < len; k++) {
        batch_integrate(b, c.pos, c.vel, c.force, c.type, c.inv_mass, c.dt, 1, 1, k, c.s);
        batch_forces(b, c.pos, c.force, false, c.s);
    }
    return MD_OK;
}

static int batch_read_flags(md_batch *b, hipStream_t s, int32_t f[2])
{
    MD_HIP(hipMemcpyAsync(b->host_flags, b->flags, 8, hipMemcpyDeviceToHost, s));
    MD_HIP(hipStreamSynchronize(s));
    f[0] = (int32_t)b->host_flags[0];
    f[1] = (int32_t)b->host_flags[1];
    return MD_OK;
}

extern "C" int md_batch_step(md_batch *b, double *pos, void *vel, void *force, int32_t *type, int32_t *ids,
                             const double *inv_mass, const double *lj, double dt, int32_t nsteps, int32_t use_graph,
                             void *stream)
{
    if (!b) return fail(MD_ERR_INVALID_ARG, "batch is NULL");
    if (!inv_mass || !lj || (b->n > 0 && (!pos || !vel || !force || !type || !ids)))
        return fail(MD_ERR_INVALID_ARG, "NULL argument");
    if (nsteps < 0 || !(dt > 0.0)) return fail(MD_ERR_INVALID_ARG, "bad nsteps or dt");
    if (!b->built) return fail(MD_ERR_NOT_BUILT, "md_batch_build_cells must be called first");
    if (nsteps == 0) return MD_OK;
    MD_HIP(hipSetDevice(b->device));
    hipStream_t s = (hipStream_t)stream;
    k_bprep<<<(b->n_sys + 255) / 256, 256, 0, s>>>(b->sys, b->n_sys, lj, b->cfg.rc2[0]);
    BatchCtx c{pos, vel, force, type, ids, inv_mass, dt, s};
    size_t rs = bsize(b->cfg);
    size_t n = (size_t)b->n;
    const void *key[8] = {pos, vel, force, type, ids, inv_mass, lj, stream};
    int st = 0;
    while (st < nsteps) {
        // a block one step longer than the interval in use, after enough calm
        // blocks, tries whether the motion now allows it (launched directly:
        // the graph holds the interval in use)
        const bool probe = b->r_eff < b->cfg.rebuild_interval && b->calm >= b->backoff;
        const int R = probe ? b->r_eff + 1 : b->r_eff;
        int len = std::min(R, nsteps - st);
        bool graphable = use_graph && st > 0 && len == R && !probe;
        int rc;
        if (graphable) {
            bool same = b->exec && b->graph_R == R && b->graph_dt == dt && memcmp(key, b->graph_key, sizeof(key)) == 0;
            if (!same) {
                if (b->exec) (void)hipGraphExecDestroy(b->exec);
                if (b->graph) (void)hipGraphDestroy(b->graph);
                b->exec = nullptr;
                b->graph = nullptr;
                // capture on a stream of our own (the caller's may be the
                // null stream, which cannot be captured); replay on theirs
                if (!b->cap) MD_HIP(hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking));
                BatchCtx cc = c;
                cc.s = b->cap;
                MD_HIP(hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal));
                rc = batch_block_ops(b, cc, R, false);
                hipGraph_t gr = nullptr;
                hipError_t e = hipStreamEndCapture(b->cap, &gr);
                if (rc) return rc;
                if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
                b->graph = gr;
                MD_HIP(hipGraphInstantiate(&b->exec, gr, nullptr, nullptr, 0));
                memcpy(b->graph_key, key, sizeof(key));
                b->graph_dt = dt;
                b->graph_R = R;
            }
            MD_HIP(hipGraphLaunch(b->exec, s));
        } else {
            if ((rc = batch_block_ops(b, c, len, st == 0))) return rc;
        }
        int32_t f[2];
        if ((rc = batch_read_flags(b, s, f))) return rc;
        int v = f[1];
        b->n_rebuilds++;
        if (v >= 1 && v < len) {
            // a particle outgrew the skin at block step v: redo steps 1 .. v-1
            // from the snapshot taken after the block's rebuild; the next
            // block starts at step v with a rebuild
            if (n > 0) {
                MD_HIP(hipMemcpyAsync(pos, b->snap_pos, 24 * n, hipMemcpyDeviceToDevice, s));
                MD_HIP(hipMemcpyAsync(vel, b->snap_vel, 3 * rs * n, hipMemcpyDeviceToDevice, s));
                // the FP32 force reads the staged copy of the positions: stage
                // the restored ones
                k_bstage<<<bblocks((int64_t)n), 256, 0, s>>>((int)n, pos, type, b->sys_of, b->sys, b->stage);
            }
            batch_forces(b, pos, force, false, s);
            for (int k = 1; k < v; k++) {
                batch_integrate(b, pos, vel, force, type, inv_mass, dt, 1, 1, k, s);
                batch_forces(b, pos, force, false, s);
            }
            st += v;
            b->n_steps += v;
            b->n_forced++;
            // a block of v steps would have passed
            if (probe) b->backoff = std::min(2 * b->backoff, 1 << 12);
            b->r_eff = std::max(1, std::min(b->r_eff, v));
            b->calm = 0;
        } else {
            st += len;
            b->n_steps += len;
            if (probe && len == R) {
                b->r_eff = R;
                b->backoff = 32;
                b->calm = 0;
            } else {
                b->calm++;
            }
        }
    }
    // final half kick
    batch_integrate(b, pos, vel, force, type, inv_mass, dt, 1, 0, 0, s);
    return MD_OK;
}

// Cutoff Lennard-Jones forces (Sec. 2.1) over the pair-finding containers of
// Sec. 2.2.1: linked cells and Verlet lists, each either gather-only (every
// pair evaluated from both sides, no write conflicts: the GPU analogue of the
// List_Iter / C01 traversals of Table 1) or with Newton's third law (each pair
// once, the j-side force scattered with atomics).  Also the Verlet-list build.
//
// FP32 path: positions staged as 32-bit fixed point (box -> 2^32), so the
// periodic minimum image is a wrapping integer subtraction; pair arithmetic in
// FP32 in units u = L_x / 2^32; cutoff decisions equal the FP64 ones (guard
// band).  FP64 path: the plain definition's operation order on the FP64
// positions.
#include "pair.h"

namespace mdlj {

// ------------------------------------------------------------------ helpers

__device__ __forceinline__ void cell_xyz(int c, const Geom &g, int &cx, int &cy, int &cz)
{
    cx = c % g.nc[0];
    int t = c / g.nc[0];
    cy = t % g.nc[1];
    cz = t / g.nc[1];
}

__device__ __forceinline__ int wrap_add(int c, int o, int n)
{
    c += o;
    return c >= n ? c - n : c;
}

template <typename real>
__device__ __forceinline__ void atomic_add_real(real *p, real v)
{
    atomicAdd(p, v);
}

__device__ __forceinline__ void write_partials(double *partials, float eu, float ew, int np, double *sh)
{
    double v[4] = {(double)eu, (double)ew, (double)np, 0.0};
    block_sum4(v, sh);
    if (threadIdx.x == 0) {
        partials[blockIdx.x * 4 + 0] = v[0];
        partials[blockIdx.x * 4 + 1] = v[1];
        partials[blockIdx.x * 4 + 2] = v[2];
        partials[blockIdx.x * 4 + 3] = 0.0;
    }
}

// ------------------------------------------------------------------ FP32 kernels

// Per-particle FP32 accumulator and pair step shared by both traversals.
template <int NT, bool ISO, bool ENERGY, bool N3L>
struct AccF32 {
    int4 pi;
    int i;
    float fx = 0.f, fy = 0.f, fz = 0.f, eu = 0.f, ew = 0.f;
    int np = 0;
    __device__ __forceinline__ void pair(int j, const int4 &pj, const TabF<NT> &t, const Geom &g,
                                         const double *pos, int n, float *F)
    {
        float dx, dy, dz;
        staged_delta<ISO>(pi, pj, g, dx, dy, dz);
        float r2 = dx * dx + dy * dy + dz * dz;
        int ab = NT == 1 ? 0 : pi.w * NT + pj.w;
        bool in = within(r2, t.pick(t.lo, ab), t.pick(t.hi, ab), t.pickd(t.rc2, ab), pos, n, i, j, g);
        float phi = lj_f32<NT, ENERGY>(r2, ab, in, t, eu, ew, np);
        fx += phi * dx;
        fy += phi * dy;
        fz += phi * dz;
        if (N3L && in) {
            size_t N = (size_t)n;
            atomicAdd(&F[j], -phi * dx);
            atomicAdd(&F[N + j], -phi * dy);
            atomicAdd(&F[2 * N + j], -phi * dz);
        }
    }
    // In fixed-point units the force is phi_u * d_u; y and z were already
    // scaled to x units, so the three components are consistent.
    __device__ __forceinline__ void store(float *F, int n)
    {
        size_t N = (size_t)n;
        if (N3L) {
            atomicAdd(&F[i], fx);
            atomicAdd(&F[N + i], fy);
            atomicAdd(&F[2 * N + i], fz);
        } else {
            F[i] = fx;
            F[N + i] = fy;
            F[2 * N + i] = fz;
        }
    }
};

template <int NT, bool ISO, bool ENERGY, bool N3L>
__global__ __launch_bounds__(kBlock) void k_lc_f32(int n, const int4 *__restrict__ st,
                                                   const int32_t *__restrict__ cell_start,
                                                   const int32_t *__restrict__ cell_sorted,
                                                   const PairTab *__restrict__ tabp, Geom g,
                                                   const double *__restrict__ pos, float *__restrict__ F,
                                                   double *__restrict__ partials)
{
    __shared__ double sh[4 * kBlock / 64];
    __shared__ int so[3][kMaxOfs];
    load_offsets(g, so);
    TabF<NT> t;
    t.load(tabp);
    AccF32<NT, ISO, ENERGY, N3L> acc;
    acc.i = blockIdx.x * kBlock + threadIdx.x;
    if (acc.i < n) {
        int i = acc.i;
        acc.pi = st[i];
        int cx, cy, cz;
        cell_xyz(cell_sorted[i], g, cx, cy, cz);
        for (int a = 0; a < g.nofs[2]; a++) {
            int zz = wrap_add(cz, so[2][a], g.nc[2]);
            for (int b = 0; b < g.nofs[1]; b++) {
                int yy = wrap_add(cy, so[1][b], g.nc[1]);
                int row = (zz * g.nc[1] + yy) * g.nc[0];
                for (int e = 0; e < g.nofs[0]; e++) {
                    int cj = row + wrap_add(cx, so[0][e], g.nc[0]);
                    int jb = cell_start[cj], je = cell_start[cj + 1];
                    for (int j = jb; j < je; j++) {
                        if (N3L ? j <= i : j == i) continue;
                        acc.pair(j, st[j], t, g, pos, n, F);
                    }
                }
            }
        }
        acc.store(F, n);
    }
    if (ENERGY) write_partials(partials, acc.eu, acc.ew, acc.np, sh);
}

template <int NT, bool ISO, bool ENERGY, bool N3L>
__global__ __launch_bounds__(kBlock) void k_vl_f32(int n, const int4 *__restrict__ st,
                                                   const int32_t *__restrict__ nbr,
                                                   const int32_t *__restrict__ cnt, int64_t ld,
                                                   const PairTab *__restrict__ tabp, Geom g,
                                                   const double *__restrict__ pos, float *__restrict__ F,
                                                   double *__restrict__ partials)
{
    __shared__ double sh[4 * kBlock / 64];
    TabF<NT> t;
    t.load(tabp);
    AccF32<NT, ISO, ENERGY, N3L> acc;
    acc.i = blockIdx.x * kBlock + threadIdx.x;
    if (acc.i < n) {
        int i = acc.i;
        acc.pi = st[i];
        int c = cnt[i];
        const int32_t *row = nbr + i;
        for (int k = 0; k < c; k++) {
            int j = row[(size_t)k * ld];
            acc.pair(j, st[j], t, g, pos, n, F);
        }
        acc.store(F, n);
    }
    if (ENERGY) write_partials(partials, acc.eu, acc.ew, acc.np, sh);
}

// ------------------------------------------------------------------ FP64 kernels

template <bool N3L>
struct AccF64 {
    int i, ti;
    double xi, yi, zi;
    double fx = 0.0, fy = 0.0, fz = 0.0, eu = 0.0, ew = 0.0;
    int np = 0;
    __device__ __forceinline__ void pair(int j, const double *__restrict__ pos, const int32_t *__restrict__ type,
                                         const PairTab *__restrict__ t, const Geom &g, int n, double *F)
    {
#pragma clang fp contract(off)
        size_t N = (size_t)n;
        double dx = min_image(xi - pos[j], g.L[0]);
        double dy = min_image(yi - pos[N + j], g.L[1]);
        double dz = min_image(zi - pos[2 * N + j], g.L[2]);
        double r2 = dx * dx + dy * dy + dz * dz;
        int ab = ti * g.nt + type[j];
        if (!(r2 < t->rc2[ab])) return;
        double phi, u;
        lj_f64(r2, t->eps[ab], t->sig[ab], phi, u);
        fx += phi * dx;
        fy += phi * dy;
        fz += phi * dz;
        eu += u;
        ew += phi * r2;
        np += 1;
        if (N3L) {
            atomicAdd(&F[j], -(phi * dx));
            atomicAdd(&F[N + j], -(phi * dy));
            atomicAdd(&F[2 * N + j], -(phi * dz));
        }
    }
    __device__ __forceinline__ void store(double *F, int n)
    {
        size_t N = (size_t)n;
        if (N3L) {
            atomicAdd(&F[i], fx);
            atomicAdd(&F[N + i], fy);
            atomicAdd(&F[2 * N + i], fz);
        } else {
            F[i] = fx;
            F[N + i] = fy;
            F[2 * N + i] = fz;
        }
    }
};

template <bool ENERGY, bool N3L>
__global__ __launch_bounds__(kBlock) void k_lc_f64(int n, const int32_t *__restrict__ cell_start,
                                                   const int32_t *__restrict__ cell_sorted,
                                                   const PairTab *__restrict__ tab, Geom g,
                                                   const double *__restrict__ pos,
                                                   const int32_t *__restrict__ type, double *__restrict__ F,
                                                   double *__restrict__ partials)
{
    __shared__ double sh[4 * kBlock / 64];
    __shared__ int so[3][kMaxOfs];
    load_offsets(g, so);
    AccF64<N3L> acc;
    acc.i = blockIdx.x * kBlock + threadIdx.x;
    if (acc.i < n) {
        int i = acc.i;
        size_t N = (size_t)n;
        acc.xi = pos[i];
        acc.yi = pos[N + i];
        acc.zi = pos[2 * N + i];
        acc.ti = type[i];
        int cx, cy, cz;
        cell_xyz(cell_sorted[i], g, cx, cy, cz);
        for (int a = 0; a < g.nofs[2]; a++) {
            int zz = wrap_add(cz, so[2][a], g.nc[2]);
            for (int b = 0; b < g.nofs[1]; b++) {
                int yy = wrap_add(cy, so[1][b], g.nc[1]);
                int row = (zz * g.nc[1] + yy) * g.nc[0];
                for (int e = 0; e < g.nofs[0]; e++) {
                    int cj = row + wrap_add(cx, so[0][e], g.nc[0]);
                    int jb = cell_start[cj], je = cell_start[cj + 1];
                    for (int j = jb; j < je; j++) {
                        if (N3L ? j <= i : j == i) continue;
                        acc.pair(j, pos, type, tab, g, n, F);
                    }
                }
            }
        }
        acc.store(F, n);
    }
    if (ENERGY) {
        double v[4] = {acc.eu, acc.ew, (double)acc.np, 0.0};
        block_sum4(v, sh);
        if (threadIdx.x == 0)
            for (int k = 0; k < 4; k++) partials[blockIdx.x * 4 + k] = v[k];
    }
}

template <bool ENERGY, bool N3L>
__global__ __launch_bounds__(kBlock) void k_vl_f64(int n, const int32_t *__restrict__ nbr,
                                                   const int32_t *__restrict__ cnt, int64_t ld,
                                                   const PairTab *__restrict__ tab, Geom g,
                                                   const double *__restrict__ pos,
                                                   const int32_t *__restrict__ type, double *__restrict__ F,
                                                   double *__restrict__ partials)
{
    __shared__ double sh[4 * kBlock / 64];
    AccF64<N3L> acc;
    acc.i = blockIdx.x * kBlock + threadIdx.x;
    if (acc.i < n) {
        int i = acc.i;
        size_t N = (size_t)n;
        acc.xi = pos[i];
        acc.yi = pos[N + i];
        acc.zi = pos[2 * N + i];
        acc.ti = type[i];
        int c = cnt[i];
        for (int k = 0; k < c; k++) acc.pair(nbr[(size_t)k * ld + i], pos, type, tab, g, n, F);
        acc.store(F, n);
    }
    if (ENERGY) {
        double v[4] = {acc.eu, acc.ew, (double)acc.np, 0.0};
        block_sum4(v, sh);
        if (threadIdx.x == 0)
            for (int k = 0; k < 4; k++) partials[blockIdx.x * 4 + k] = v[k];
    }
}

// ------------------------------------------------------------------ Verlet-list build

// One thread per particle: scan the cell stencil and keep every j with
// r2 < (r_c,max + skin)^2 (decided in FP64 inside the guard band), in stencil
// order.  Column-major rows: entry k of particle i at nbr[k * ld + i].  With
// half != 0 only j > i (sorted index) is kept, for Newton's third law.
template <bool ISO>
__global__ __launch_bounds__(kBlock) void k_vl_build(int n, const int4 *__restrict__ st,
                                                     const int32_t *__restrict__ cell_start,
                                                     const int32_t *__restrict__ cell_sorted,
                                                     const double *__restrict__ pos, Geom g, int half,
                                                     int32_t *__restrict__ nbr, int32_t *__restrict__ cnt,
                                                     int64_t ld, int maxn, int32_t *__restrict__ flags)
{
    __shared__ int so[3][kMaxOfs];
    load_offsets(g, so);
    int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    int4 pi = st[i];
    int cx, cy, cz;
    cell_xyz(cell_sorted[i], g, cx, cy, cz);
    int c = 0;
    for (int a = 0; a < g.nofs[2]; a++) {
        int zz = wrap_add(cz, so[2][a], g.nc[2]);
        for (int b = 0; b < g.nofs[1]; b++) {
            int yy = wrap_add(cy, so[1][b], g.nc[1]);
            int row = (zz * g.nc[1] + yy) * g.nc[0];
            for (int e = 0; e < g.nofs[0]; e++) {
                int cj = row + wrap_add(cx, so[0][e], g.nc[0]);
                int jb = cell_start[cj], je = cell_start[cj + 1];
                for (int j = jb; j < je; j++) {
                    if (half ? j <= i : j == i) continue;
                    float dx, dy, dz;
                    staged_delta<ISO>(pi, st[j], g, dx, dy, dz);
                    float r2 = dx * dx + dy * dy + dz * dz;
                    if (within(r2, g.rl2_lo, g.rl2_hi, g.rl2, pos, n, i, j, g)) {
                        if (c < maxn) nbr[(size_t)c * ld + i] = j;
                        c++;
                    }
                }
            }
        }
    }
    if (c > maxn) atomicOr(&flags[0], (int)MD_FLAG_LIST_OVERFLOW);
    atomicMax(&flags[2], c);
    cnt[i] = c < maxn ? c : maxn;
}

void launch_vl_build(int n, const int4 *stage, const int32_t *cell_start, const int32_t *cell_sorted,
                     const double *pos, const Geom &g, int half, int32_t *nbr, int32_t *cnt, int64_t ld,
                     int maxn, int32_t *flags, hipStream_t s)
{
    if (n <= 0) return;
    int nb = (n + kBlock - 1) / kBlock;
    if (g.iso)
        k_vl_build<true><<<nb, kBlock, 0, s>>>(n, stage, cell_start, cell_sorted, pos, g, half, nbr, cnt,
                                                ld, maxn, flags);
    else
        k_vl_build<false><<<nb, kBlock, 0, s>>>(n, stage, cell_start, cell_sorted, pos, g, half, nbr, cnt,
                                                 ld, maxn, flags);
}

// ------------------------------------------------------------------ dispatch

int force_blocks(const ForceArgs &a)
{
    if (a.n <= 0) return 0;
    if (a.container == MD_CONTAINER_CL) return cluster_force_blocks();
    if (a.container == MD_CONTAINER_VLC || a.newton3 == MD_N3L_C08) return a.vlc_blocks;
    if (a.window) return window_force_blocks();
    return (a.n + kBlock - 1) / kBlock;
}

template <int NT, bool ISO, bool EN, bool N3>
static void launch_f32(const ForceArgs &a, const Geom &g, hipStream_t s)
{
    int nb = force_blocks(a);
    if (a.container == MD_CONTAINER_LC)
        k_lc_f32<NT, ISO, EN, N3><<<nb, kBlock, 0, s>>>(a.n, a.stage, a.cell_start, a.cell_sorted, a.tab, g,
                                                        a.pos, (float *)a.force, a.partials);
    else
        k_vl_f32<NT, ISO, EN, N3><<<nb, kBlock, 0, s>>>(a.n, a.stage, a.nbr, a.nbr_count, a.nbr_ld, a.tab, g,
                                                        a.pos, (float *)a.force, a.partials);
}

template <int NT, bool ISO>
static void launch_f32_b(const ForceArgs &a, const Geom &g, hipStream_t s)
{
    if (a.energy) {
        if (a.newton3) launch_f32<NT, ISO, true, true>(a, g, s);
        else launch_f32<NT, ISO, true, false>(a, g, s);
    } else {
        if (a.newton3) launch_f32<NT, ISO, false, true>(a, g, s);
        else launch_f32<NT, ISO, false, false>(a, g, s);
    }
}

template <bool EN, bool N3>
static void launch_f64(const ForceArgs &a, const Geom &g, hipStream_t s)
{
    int nb = force_blocks(a);
    if (a.container == MD_CONTAINER_LC)
        k_lc_f64<EN, N3><<<nb, kBlock, 0, s>>>(a.n, a.cell_start, a.cell_sorted, a.tab, g, a.pos, a.type,
                                               (double *)a.force, a.partials);
    else
        k_vl_f64<EN, N3><<<nb, kBlock, 0, s>>>(a.n, a.nbr, a.nbr_count, a.nbr_ld, a.tab, g, a.pos, a.type,
                                               (double *)a.force, a.partials);
}

void launch_force(const ForceArgs &a, const Geom &g, hipStream_t s)
{
    if (a.n <= 0) return;
    if (a.container == MD_CONTAINER_CL) {
        launch_cluster_force(a, g, s);
        return;
    }
    if (a.container == MD_CONTAINER_PVL) {
        launch_pvl_force(a, g, s);
        return;
    }
    if (a.container == MD_CONTAINER_VLC) {
        launch_vlc_force(a, g, s);
        return;
    }
    if (a.newton3 == MD_N3L_C08) {
        launch_lc08_force(a, g, s);
        return;
    }
    if (a.window) {
        launch_window_force(a, g, s);
        return;
    }
    if (a.precision == MD_FP64) {
        if (a.energy) {
            if (a.newton3) launch_f64<true, true>(a, g, s);
            else launch_f64<true, false>(a, g, s);
        } else {
            if (a.newton3) launch_f64<false, true>(a, g, s);
            else launch_f64<false, false>(a, g, s);
        }
        return;
    }
    if (g.nt == 1) {
        if (g.iso) launch_f32_b<1, true>(a, g, s);
        else launch_f32_b<1, false>(a, g, s);
    } else {
        if (g.iso) launch_f32_b<2, true>(a, g, s);
        else launch_f32_b<2, false>(a, g, s);
    }
}

// ------------------------------------------------------------------ reductions

// Deterministic sum of per-block {U, W, n_pairs} partials in one block, in a
// fixed order.  gather != 0: each pair was seen from both sides.
__global__ void k_reduce_out(const double *__restrict__ part, int nb, int gather, double *__restrict__ out)
{
    __shared__ double sh[4 * kBlock / 64];
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    for (int b = threadIdx.x; b < nb; b += kBlock)
        for (int k = 0; k < 3; k++) v[k] += part[b * 4 + k];
    block_sum4(v, sh);
    if (threadIdx.x == 0) {
        double h = gather ? 0.5 : 1.0;
        out[0] = v[0] * h;
        out[1] = v[1] * h;
        out[2] = v[2] * h;
        out[3] = 0.0;
    }
}

void launch_reduce_out(const double *partials, int nblocks, int gather, double *out, hipStream_t s)
{
    k_reduce_out<<<1, kBlock, 0, s>>>(partials, nblocks, gather, out);
}

}  // namespace mdlj

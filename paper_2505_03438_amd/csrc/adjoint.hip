// Adjoint of the truncated Lennard-Jones forces (the differentiable
// extension): for g = dL/dF, every interacting pair contributes
//   dL/dx_i += J (g_i - g_j),   J = phi I + 2 (dphi/dr2) d d^T,
//   dphi/dr2 = -48 eps q (7q - 2) / r^4,
// and to the per-pair parameters
//   dL/deps_ab += (phi/eps_ab) d.(g_i - g_j),
//   dL/dsig_ab += 144 eps q (4q - 1)/(sig r^2) d.(g_i - g_j),
// with the cutoffs held fixed.  One thread per particle gathers its own row
// over the linked-cell stencil (no write conflicts); parameter terms are seen
// from both sides of each pair and halved.  Pair arithmetic in FP32 with FP64
// accumulation, or all FP64.
#include "pair.h"

namespace mdlj {

__device__ __forceinline__ void cell_xyz_a(int c, const Geom &g, int &cx, int &cy, int &cz)
{
    cx = c % g.nc[0];
    int t = c / g.nc[0];
    cy = t % g.nc[1];
    cz = t / g.nc[1];
}

__device__ __forceinline__ int wrap_add_a(int c, int o, int n)
{
    c += o;
    return c >= n ? c - n : c;
}

template <typename real, bool ISO>
__global__ __launch_bounds__(kBlock) void k_adjoint(AdjointArgs a, Geom g)
{
    __shared__ double sh[8 * kBlock / 64];
    __shared__ int so[3][kMaxOfs];
    load_offsets(g, so);
    int i = blockIdx.x * kBlock + threadIdx.x;
    const int nt = g.nt;
    double gp[8] = {0, 0, 0, 0, 0, 0, 0, 0};  // eps_ab[4], sig_ab[4]
    if (i < a.n) {
        size_t N = (size_t)a.n;
        const real *G = (const real *)a.grad_force;
        double gix = (double)G[i], giy = (double)G[N + i], giz = (double)G[2 * N + i];
        double ax = 0.0, ay = 0.0, az = 0.0;
        int ti = a.type[i];
        int4 pi = a.stage[i];
        double xi = a.pos[i], yi = a.pos[N + i], zi = a.pos[2 * N + i];
        double u = g.L[0] / 4294967296.0;
        int cx, cy, cz;
        cell_xyz_a(a.cell_sorted[i], g, cx, cy, cz);
        for (int aa = 0; aa < g.nofs[2]; aa++) {
            int zz = wrap_add_a(cz, so[2][aa], g.nc[2]);
            for (int b = 0; b < g.nofs[1]; b++) {
                int yy = wrap_add_a(cy, so[1][b], g.nc[1]);
                int row = (zz * g.nc[1] + yy) * g.nc[0];
                for (int e = 0; e < g.nofs[0]; e++) {
                    int cj = row + wrap_add_a(cx, so[0][e], g.nc[0]);
                    int jb = a.cell_start[cj], je = a.cell_start[cj + 1];
                    for (int j = jb; j < je; j++) {
                        if (j == i) continue;
                        int ab = ti * nt + a.type[j];
                        double dgx = gix - (double)G[j], dgy = giy - (double)G[N + j],
                               dgz = giz - (double)G[2 * N + j];
                        if (sizeof(real) == 4) {
                            float dx, dy, dz;
                            staged_delta<ISO>(pi, a.stage[j], g, dx, dy, dz);
                            float r2u = dx * dx + dy * dy + dz * dz;
                            if (!within(r2u, a.tab->rc2_lo[ab], a.tab->rc2_hi[ab], a.tab->rc2[ab], a.pos,
                                        a.n, i, j, g))
                                continue;
                            float uf = (float)u;
                            dx *= uf;
                            dy *= uf;
                            dz *= uf;
                            float r2 = dx * dx + dy * dy + dz * dz;
                            float eps = (float)a.tab->eps[ab], sig = (float)a.tab->sig[ab];
                            float ir2 = 1.0f / r2;
                            float s2 = sig * sig * ir2;
                            float q = s2 * s2 * s2;
                            float phi = 24.0f * eps * ir2 * q * (2.0f * q - 1.0f);
                            float dphi = -48.0f * eps * ir2 * ir2 * q * (7.0f * q - 2.0f);
                            float ddg = dx * (float)dgx + dy * (float)dgy + dz * (float)dgz;
                            float k2 = 2.0f * dphi * ddg;
                            ax += (double)(phi * (float)dgx + k2 * dx);
                            ay += (double)(phi * (float)dgy + k2 * dy);
                            az += (double)(phi * (float)dgz + k2 * dz);
                            gp[ab] += (double)(phi / eps * ddg);
                            gp[4 + ab] += (double)(144.0f * eps * ir2 * q * (4.0f * q - 1.0f) / sig * ddg);
                        } else {
#pragma clang fp contract(off)
                            double dx = min_image(xi - a.pos[j], g.L[0]);
                            double dy = min_image(yi - a.pos[N + j], g.L[1]);
                            double dz = min_image(zi - a.pos[2 * N + j], g.L[2]);
                            double r2 = dx * dx + dy * dy + dz * dz;
                            if (!(r2 < a.tab->rc2[ab])) continue;
                            double eps = a.tab->eps[ab], sig = a.tab->sig[ab];
                            double ir2 = 1.0 / r2;
                            double s2 = sig * sig * ir2;
                            double q = s2 * s2 * s2;
                            double phi = 24.0 * eps * ir2 * q * (2.0 * q - 1.0);
                            double dphi = -48.0 * eps * ir2 * ir2 * q * (7.0 * q - 2.0);
                            double ddg = dx * dgx + dy * dgy + dz * dgz;
                            ax += phi * dgx + 2.0 * dphi * dx * ddg;
                            ay += phi * dgy + 2.0 * dphi * dy * ddg;
                            az += phi * dgz + 2.0 * dphi * dz * ddg;
                            gp[ab] += phi / eps * ddg;
                            gp[4 + ab] += 144.0 * eps * ir2 * q * (4.0 * q - 1.0) / sig * ddg;
                        }
                    }
                }
            }
        }
        a.grad_pos[i] = ax;
        a.grad_pos[N + i] = ay;
        a.grad_pos[2 * N + i] = az;
    }
    // block sums of the 8 parameter partials, fixed order
    double v0[4] = {gp[0], gp[1], gp[2], gp[3]};
    double v1[4] = {gp[4], gp[5], gp[6], gp[7]};
    block_sum4(v0, sh);
    __syncthreads();
    block_sum4(v1, sh + 4 * kBlock / 64);
    if (threadIdx.x == 0)
        for (int k = 0; k < 4; k++) {
            a.gpart[blockIdx.x * 8 + k] = v0[k];
            a.gpart[blockIdx.x * 8 + 4 + k] = v1[k];
        }
}

int adjoint_blocks(int n) { return (n + kBlock - 1) / kBlock; }

void launch_adjoint(const AdjointArgs &a, const Geom &g, hipStream_t s)
{
    if (a.n <= 0) return;
    int nb = adjoint_blocks(a.n);
    if (a.precision == MD_FP64) {
        if (g.iso) k_adjoint<double, true><<<nb, kBlock, 0, s>>>(a, g);
        else k_adjoint<double, false><<<nb, kBlock, 0, s>>>(a, g);
    } else {
        if (g.iso) k_adjoint<float, true><<<nb, kBlock, 0, s>>>(a, g);
        else k_adjoint<float, false><<<nb, kBlock, 0, s>>>(a, g);
    }
}

// Sum the per-block partials (fixed order), halve (each pair seen twice) and
// chain through Lorentz-Berthelot: sig_ab = (sig_a + sig_b)/2 gives 1/2 to
// each of sig_a, sig_b; eps_ab = sqrt(eps_a eps_b) gives eps_b / (2 eps_ab)
// to eps_a and eps_a / (2 eps_ab) to eps_b.
__global__ void k_adjoint_finish(const double *__restrict__ gpart, int nb, const double *__restrict__ lj, int nt,
                                 double *__restrict__ grad_lj)
{
    __shared__ double sh[8 * kBlock / 64];
    double v0[4] = {0, 0, 0, 0}, v1[4] = {0, 0, 0, 0};
    for (int b = threadIdx.x; b < nb; b += kBlock)
        for (int k = 0; k < 4; k++) {
            v0[k] += gpart[b * 8 + k];
            v1[k] += gpart[b * 8 + 4 + k];
        }
    block_sum4(v0, sh);
    __syncthreads();
    block_sum4(v1, sh + 4 * kBlock / 64);
    if (threadIdx.x == 0) {
        double ge[MD_MAX_TYPES] = {0}, gs[MD_MAX_TYPES] = {0};
        for (int a = 0; a < nt; a++)
            for (int b = 0; b < nt; b++) {
                int ab = a * nt + b;
                double geps = 0.5 * v0[ab], gsig = 0.5 * v1[ab];
                double eab = sqrt(lj[a] * lj[b]);
                gs[a] += 0.5 * gsig;
                gs[b] += 0.5 * gsig;
                ge[a] += geps * lj[b] / (2.0 * eab);
                ge[b] += geps * lj[a] / (2.0 * eab);
            }
        for (int a = 0; a < nt; a++) {
            grad_lj[a] = ge[a];
            grad_lj[nt + a] = gs[a];
        }
    }
}

void launch_adjoint_finish(const double *gpart, int nblocks, const double *lj, int nt, double *grad_lj,
                           hipStream_t s)
{
    k_adjoint_finish<<<1, kBlock, 0, s>>>(gpart, nblocks, lj, nt, grad_lj);
}

}  // namespace mdlj

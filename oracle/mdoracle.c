/*
 * mdoracle.c -- plain, slow, FP64 CPU oracle for cutoff Lennard-Jones MD.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the tests, the smoke check and the CPU-baseline leg
 * of the benchmark do.  It shares no code, header or table with the HIP path.
 *
 * Every routine is the plain definition of what the method computes, written
 * for a reader to check by eye:
 *   - brute force over all pairs, no blocking, no reordering;
 *   - FP64 throughout, compiled with -ffp-contract=off so that every
 *     operation is one IEEE round-to-nearest operation in the order written.
 *
 * The paper (Sec. 2.1, "Molecular Dynamics") names the ingredients -- the
 * Lennard-Jones force, a cutoff r_c beyond which pairs are neglected, Newton's
 * third law, the Stormer-Verlet integrator -- but prints no formula.  The
 * readings used here are the textbook ones:
 *   U(r)   = 4 eps [ (sig/r)^12 - (sig/r)^6 ]
 *   f_ij   = phi * d_ij,   d_ij = x_i - x_j (minimum image),
 *   phi    = 24 eps q (2q - 1) / r^2,   q = (sig^2 / r^2)^3
 *   a pair interacts iff r^2 < r_c^2 (strict; truncated, not shifted)
 * Linked cells (Sec. 2.2.1): cell side (r_c + skin) * CSF stretched to fit
 * the domain, i.e. n = floor(L / (CSF (r_c + skin))), side = L / n.
 * Verlet lists (Sec. 2.2.1): the set of pairs within r_c + skin.
 * Live statistics (Sec. 4): particle counts over CSF-1 cell bins.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_MAX_TYPES 4

/* ------------------------------------------------------------------------ */
/* Pair potential (Sec. 2.1: Lennard-Jones force; formula is the textbook one) */

/* phi such that f_ij = phi * d_ij, and the pair energy u, for squared
 * distance r2 and pair parameters eps, sig. */
void orc_lj(double r2, double eps, double sig, double *phi, double *u)
{
    double ir2 = 1.0 / r2;
    double s2 = sig * sig * ir2;
    double q = s2 * s2 * s2;
    *phi = 24.0 * eps * ir2 * q * (2.0 * q - 1.0);
    *u = 4.0 * eps * q * (q - 1.0);
}

/* Periodic minimum image of one displacement component, valid for
 * |d| < L (positions kept in [0, L)). */
static double min_image(double d, double L)
{
    if (d > 0.5 * L)
        d -= L;
    else if (d < -0.5 * L)
        d += L;
    return d;
}

/* Squared minimum-image distance between particles i and j, in the fixed
 * order dx*dx + dy*dy + dz*dz.  Also returns the displacement x_i - x_j. */
static double dist2(const double *x, const double *y, const double *z,
                    int64_t i, int64_t j, const double *box, double d[3])
{
    d[0] = min_image(x[i] - x[j], box[0]);
    d[1] = min_image(y[i] - y[j], box[1]);
    d[2] = min_image(z[i] - z[j], box[2]);
    return d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
}

/* Lorentz-Berthelot mixing of per-type parameters into per-pair tables:
 * sig_ab = (sig_a + sig_b)/2, eps_ab = sqrt(eps_a eps_b). */
void orc_mix(int nt, const double *eps_t, const double *sig_t, double *eps_ab,
             double *sig_ab)
{
    for (int a = 0; a < nt; a++)
        for (int b = 0; b < nt; b++) {
            sig_ab[a * nt + b] = 0.5 * (sig_t[a] + sig_t[b]);
            eps_ab[a * nt + b] = sqrt(eps_t[a] * eps_t[b]);
        }
}

/* ------------------------------------------------------------------------ */
/* Forces, energy, virial by brute force (Sec. 2.1: force on each molecule is
 * the sum over all others; cutoff neglects pairs beyond r_c).
 *
 * pos is SoA [3][n].  Per-pair tables eps/sig/rc2 are [nt][nt].
 * force[3][n] receives F_i = sum_{j != i, r2 < rc2} phi d_ij (j ascending).
 * out[0] = U = sum_{i<j} u,  out[1] = W = sum_{i<j} phi r2,
 * out[2] = number of unordered pairs with r2 < rc2.                        */
void orc_forces(int64_t n, const double *pos, const int32_t *type, int nt,
                const double *box, const double *eps, const double *sig,
                const double *rc2, double *force, double *out)
{
    const double *x = pos, *y = pos + n, *z = pos + 2 * n;
    double *rowU = (double *)calloc((size_t)(n > 0 ? n : 1), sizeof(double));
    double *rowW = (double *)calloc((size_t)(n > 0 ? n : 1), sizeof(double));
    int64_t *rowP = (int64_t *)calloc((size_t)(n > 0 ? n : 1), sizeof(int64_t));
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < n; i++) {
        double fx = 0.0, fy = 0.0, fz = 0.0, u_i = 0.0, w_i = 0.0;
        int64_t p_i = 0;
        for (int64_t j = 0; j < n; j++) {
            if (j == i)
                continue;
            double d[3];
            double r2 = dist2(x, y, z, i, j, box, d);
            int ab = type[i] * nt + type[j];
            if (!(r2 < rc2[ab]))
                continue;
            double phi, u;
            orc_lj(r2, eps[ab], sig[ab], &phi, &u);
            fx += phi * d[0];
            fy += phi * d[1];
            fz += phi * d[2];
            if (j > i) {
                u_i += u;
                w_i += phi * r2;
                p_i += 1;
            }
        }
        force[i] = fx;
        force[n + i] = fy;
        force[2 * n + i] = fz;
        rowU[i] = u_i;
        rowW[i] = w_i;
        rowP[i] = p_i;
    }
    double U = 0.0, W = 0.0;
    int64_t P = 0;
    for (int64_t i = 0; i < n; i++) {
        U += rowU[i];
        W += rowW[i];
        P += rowP[i];
    }
    out[0] = U;
    out[1] = W;
    out[2] = (double)P;
    free(rowU);
    free(rowW);
    free(rowP);
}

/* The same brute-force force sum for a subset of rows only (sampled parity
 * at sizes where all N^2 pairs would take too long).  force_rows is [3][m]. */
void orc_forces_rows(int64_t n, const double *pos, const int32_t *type, int nt,
                     const double *box, const double *eps, const double *sig,
                     const double *rc2, int64_t m, const int64_t *rows,
                     double *force_rows, int64_t *npairs_rows)
{
    const double *x = pos, *y = pos + n, *z = pos + 2 * n;
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t r = 0; r < m; r++) {
        int64_t i = rows[r];
        double fx = 0.0, fy = 0.0, fz = 0.0;
        int64_t p = 0;
        for (int64_t j = 0; j < n; j++) {
            if (j == i)
                continue;
            double d[3];
            double r2 = dist2(x, y, z, i, j, box, d);
            int ab = type[i] * nt + type[j];
            if (!(r2 < rc2[ab]))
                continue;
            double phi, u;
            orc_lj(r2, eps[ab], sig[ab], &phi, &u);
            fx += phi * d[0];
            fy += phi * d[1];
            fz += phi * d[2];
            p++;
        }
        force_rows[r] = fx;
        force_rows[m + r] = fy;
        force_rows[2 * m + r] = fz;
        if (npairs_rows)
            npairs_rows[r] = p;
    }
}

/* ------------------------------------------------------------------------ */
/* Pair sets (Sec. 2.2.1: neighbours are pairs within the cutoff; Verlet lists
 * keep pairs within r_c + skin).  Brute force over all i < j.
 * Writes pairs as (i, j) with i < j in lexicographic order into out[2*cap];
 * returns the total count (which may exceed cap; then only cap are written). */
int64_t orc_pairs(int64_t n, const double *pos, const double *box, double r2cut,
                  int64_t cap, int64_t *out)
{
    const double *x = pos, *y = pos + n, *z = pos + 2 * n;
    int64_t cnt = 0;
    for (int64_t i = 0; i < n; i++)
        for (int64_t j = i + 1; j < n; j++) {
            double d[3];
            if (dist2(x, y, z, i, j, box, d) < r2cut) {
                if (cnt < cap) {
                    out[2 * cnt] = i;
                    out[2 * cnt + 1] = j;
                }
                cnt++;
            }
        }
    return cnt;
}

/* Neighbour rows: for each sampled particle i, every j != i with r2 < r2cut,
 * j ascending.  counts[m]; lists[m][cap_per_row]; returns 0, or -1 if some
 * row exceeded cap_per_row (its count is still exact). */
int orc_neighbor_rows(int64_t n, const double *pos, const double *box,
                      double r2cut, int64_t m, const int64_t *rows,
                      int64_t cap_per_row, int64_t *counts, int64_t *lists)
{
    const double *x = pos, *y = pos + n, *z = pos + 2 * n;
    int overflow = 0;
#pragma omp parallel for schedule(dynamic, 4) reduction(| : overflow)
    for (int64_t r = 0; r < m; r++) {
        int64_t i = rows[r], c = 0;
        for (int64_t j = 0; j < n; j++) {
            if (j == i)
                continue;
            double d[3];
            if (dist2(x, y, z, i, j, box, d) < r2cut) {
                if (c < cap_per_row)
                    lists[r * cap_per_row + c] = j;
                else
                    overflow = 1;
                c++;
            }
        }
        counts[r] = c;
    }
    return overflow ? -1 : 0;
}

/* ------------------------------------------------------------------------ */
/* Linked cells (Sec. 2.2.1).  n_d = floor(L_d / side_min), at least 1; a
 * particle at x goes to cell min(n_d - 1, (int)(x * (n_d / L_d))) per
 * dimension; the linear id is (cz * ny + cy) * nx + cx.  Within a cell,
 * particles keep their input order (a stable counting sort).
 * ncell[3] out; cell_of[n] out; order[n] out (input indices in cell order);
 * cell_start[ncells + 1] out (caller sizes it from ncell).                 */
void orc_cell_dims(const double *box, double side_min, int32_t *ncell)
{
    for (int d = 0; d < 3; d++) {
        int32_t nd = (int32_t)floor(box[d] / side_min);
        ncell[d] = nd < 1 ? 1 : nd;
    }
}

void orc_cells(int64_t n, const double *pos, const double *box,
               const int32_t *ncell, int32_t *cell_of, int32_t *order,
               int32_t *cell_start)
{
    int64_t nc = (int64_t)ncell[0] * ncell[1] * ncell[2];
    double inv_w[3];
    for (int d = 0; d < 3; d++)
        inv_w[d] = (double)ncell[d] / box[d];
    for (int64_t i = 0; i < n; i++) {
        int32_t c[3];
        for (int d = 0; d < 3; d++) {
            int32_t cd = (int32_t)(pos[d * n + i] * inv_w[d]);
            c[d] = cd < ncell[d] - 1 ? cd : ncell[d] - 1;
        }
        cell_of[i] = (c[2] * ncell[1] + c[1]) * ncell[0] + c[0];
    }
    for (int64_t c = 0; c <= nc; c++)
        cell_start[c] = 0;
    for (int64_t i = 0; i < n; i++)
        cell_start[cell_of[i] + 1]++;
    for (int64_t c = 0; c < nc; c++)
        cell_start[c + 1] += cell_start[c];
    int32_t *fill = (int32_t *)malloc((size_t)(nc > 0 ? nc : 1) * sizeof(int32_t));
    for (int64_t c = 0; c < nc; c++)
        fill[c] = cell_start[c];
    for (int64_t i = 0; i < n; i++)
        order[fill[cell_of[i]]++] = (int32_t)i;
    free(fill);
}

/* Forces by the linked-cell neighbour search, for speed at large n.  The
 * pair set equals the brute-force one (every pair within the cutoff lies in
 * neighbouring cells of side >= sqrt(max rc2)); only the summation order of
 * each row differs (cells in stencil order, particles in cell order).
 * Requires box >= 2 sqrt(max rc2) in every dimension.                     */
void orc_forces_cells(int64_t n, const double *pos, const int32_t *type,
                      int nt, const double *box, const double *eps,
                      const double *sig, const double *rc2, double *force,
                      double *out)
{
    const double *x = pos, *y = pos + n, *z = pos + 2 * n;
    double rcmax2 = 0.0;
    for (int k = 0; k < nt * nt; k++)
        if (rc2[k] > rcmax2)
            rcmax2 = rc2[k];
    int32_t nc3[3];
    orc_cell_dims(box, sqrt(rcmax2), nc3);
    int64_t nc = (int64_t)nc3[0] * nc3[1] * nc3[2];
    int32_t *cell_of = (int32_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
    int32_t *order = (int32_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
    int32_t *start = (int32_t *)malloc((size_t)(nc + 1) * sizeof(int32_t));
    orc_cells(n, pos, box, nc3, cell_of, order, start);
    /* Distinct neighbour cell offsets per dimension (a small box has fewer
     * than three distinct neighbour cells along a dimension). */
    int32_t off[3][3], noff[3];
    for (int d = 0; d < 3; d++) {
        noff[d] = 0;
        for (int o = -1; o <= 1; o++) {
            int32_t v = ((o % nc3[d]) + nc3[d]) % nc3[d];
            int dup = 0;
            for (int k = 0; k < noff[d]; k++)
                if (off[d][k] == v)
                    dup = 1;
            if (!dup)
                off[d][noff[d]++] = v;
        }
    }
    double *rowU = (double *)calloc((size_t)(n > 0 ? n : 1), sizeof(double));
    double *rowW = (double *)calloc((size_t)(n > 0 ? n : 1), sizeof(double));
    int64_t *rowP = (int64_t *)calloc((size_t)(n > 0 ? n : 1), sizeof(int64_t));
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < n; i++) {
        int32_t ci = cell_of[i];
        int32_t cx = ci % nc3[0], cy = (ci / nc3[0]) % nc3[1],
                cz = ci / (nc3[0] * nc3[1]);
        double fx = 0.0, fy = 0.0, fz = 0.0, u_i = 0.0, w_i = 0.0;
        int64_t p_i = 0;
        for (int a = 0; a < noff[2]; a++)
            for (int b = 0; b < noff[1]; b++)
                for (int c = 0; c < noff[0]; c++) {
                    int32_t nz = (cz + off[2][a]) % nc3[2];
                    int32_t ny = (cy + off[1][b]) % nc3[1];
                    int32_t nx = (cx + off[0][c]) % nc3[0];
                    int32_t cj = (nz * nc3[1] + ny) * nc3[0] + nx;
                    for (int32_t k = start[cj]; k < start[cj + 1]; k++) {
                        int64_t j = order[k];
                        if (j == i)
                            continue;
                        double d[3];
                        double r2 = dist2(x, y, z, i, j, box, d);
                        int ab = type[i] * nt + type[j];
                        if (!(r2 < rc2[ab]))
                            continue;
                        double phi, u;
                        orc_lj(r2, eps[ab], sig[ab], &phi, &u);
                        fx += phi * d[0];
                        fy += phi * d[1];
                        fz += phi * d[2];
                        if (j > i) {
                            u_i += u;
                            w_i += phi * r2;
                            p_i++;
                        }
                    }
                }
        force[i] = fx;
        force[n + i] = fy;
        force[2 * n + i] = fz;
        rowU[i] = u_i;
        rowW[i] = w_i;
        rowP[i] = p_i;
    }
    double U = 0.0, W = 0.0;
    int64_t P = 0;
    for (int64_t i = 0; i < n; i++) {
        U += rowU[i];
        W += rowW[i];
        P += rowP[i];
    }
    out[0] = U;
    out[1] = W;
    out[2] = (double)P;
    free(rowU);
    free(rowW);
    free(rowP);
    free(cell_of);
    free(order);
    free(start);
}

/* ------------------------------------------------------------------------ */
/* Stormer-Verlet in velocity form (Sec. 2.1 names the Stormer-Verlet
 * integrator; the velocity form is the reading used):
 *   v += (dt/2) F / m;  x += dt v;  wrap x into [0, L);
 *   F = F(x);           v += (dt/2) F / m.
 * vel and force are SoA [3][n] and updated in place; force must hold F(x) on
 * entry.  inv_mass is per type.  log (if not NULL) gets, after each step s,
 * log[4 s + 0..3] = { U, K, W, n_pairs }, with K = 1/2 sum m v^2.
 * use_cells selects orc_forces_cells instead of orc_forces.              */
static double wrap(double x, double L)
{
    if (x >= L)
        x -= L;
    else if (x < 0.0)
        x += L;
    if (x >= L) /* x + L may round up to exactly L */
        x = 0.0;
    return x;
}

void orc_velocity_verlet(int64_t n, double *pos, double *vel, double *force,
                         const int32_t *type, int nt, const double *box,
                         const double *eps, const double *sig,
                         const double *rc2, const double *inv_mass, double dt,
                         int64_t nsteps, int use_cells, double *log)
{
    double half = 0.5 * dt;
    for (int64_t s = 0; s < nsteps; s++) {
        for (int d = 0; d < 3; d++)
            for (int64_t i = 0; i < n; i++) {
                vel[d * n + i] += half * inv_mass[type[i]] * force[d * n + i];
                pos[d * n + i] = wrap(pos[d * n + i] + dt * vel[d * n + i], box[d]);
            }
        double out[3];
        if (use_cells)
            orc_forces_cells(n, pos, type, nt, box, eps, sig, rc2, force, out);
        else
            orc_forces(n, pos, type, nt, box, eps, sig, rc2, force, out);
        double K = 0.0;
        for (int64_t i = 0; i < n; i++) {
            double v2 = 0.0;
            for (int d = 0; d < 3; d++) {
                vel[d * n + i] += half * inv_mass[type[i]] * force[d * n + i];
                v2 += vel[d * n + i] * vel[d * n + i];
            }
            K += 0.5 * v2 / inv_mass[type[i]];
        }
        if (log) {
            log[4 * s + 0] = out[0];
            log[4 * s + 1] = K;
            log[4 * s + 2] = out[1];
            log[4 * s + 3] = out[2];
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Force-matching loss and its exact gradient (the differentiable extension).
 * Per-type parameters theta = (eps_0..eps_{nt-1}, sig_0..sig_{nt-1}) are
 * mixed by Lorentz-Berthelot; the per-pair cutoff rc2 is held fixed.
 *   L = 1/(3n) sum_i |F_i(x; theta) - Ft_i|^2,   g_i = dL/dF_i.
 * Per interacting pair, with J = phi I + 2 (dphi/dr2) d d^T:
 *   dL/dx_i += J (g_i - g_j),  dL/dx_j -= J (g_i - g_j),
 *   dL/dtheta_ab += (dphi/dtheta_ab) d . (g_i - g_j),
 * dphi/dr2 = -48 eps q (7q - 2) / r^4, dphi/deps = phi/eps,
 * dphi/dsig = 144 eps q (4q - 1) / (sig r^2); then the chain rule through
 * the mixing rule.  Returns L; grad_pos[3][n], grad_theta[2 nt].
 * Brute force over all pairs.                                            */
double orc_force_matching(int64_t n, const double *pos, const int32_t *type,
                          int nt, const double *box, const double *theta,
                          const double *rc2, const double *target,
                          double *force_out, double *grad_pos,
                          double *grad_theta)
{
    const double *x = pos, *y = pos + n, *z = pos + 2 * n;
    double eps[ORC_MAX_TYPES * ORC_MAX_TYPES], sig[ORC_MAX_TYPES * ORC_MAX_TYPES];
    orc_mix(nt, theta, theta + nt, eps, sig);
    double out[3];
    orc_forces(n, pos, type, nt, box, eps, sig, rc2, force_out, out);
    double L = 0.0;
    double scale = 2.0 / (3.0 * (double)n);
    double *g = (double *)malloc((size_t)(3 * (n > 0 ? n : 1)) * sizeof(double));
    for (int64_t k = 0; k < 3 * n; k++) {
        double e = force_out[k] - target[k];
        L += e * e;
        g[k] = scale * e;
    }
    L /= 3.0 * (double)n;
    int npair = nt * nt;
    int nthr = 1;
#ifdef _OPENMP
    nthr = omp_get_max_threads();
#endif
    double *gp_thr = (double *)calloc((size_t)nthr * 2 * npair, sizeof(double));
#pragma omp parallel
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        double *gp = gp_thr + (size_t)tid * 2 * npair;
#pragma omp for schedule(dynamic, 16)
        for (int64_t i = 0; i < n; i++) {
            double gx = 0.0, gy = 0.0, gz = 0.0;
            for (int64_t j = 0; j < n; j++) {
                if (j == i)
                    continue;
                double d[3];
                double r2 = dist2(x, y, z, i, j, box, d);
                int ab = type[i] * nt + type[j];
                if (!(r2 < rc2[ab]))
                    continue;
                double ir2 = 1.0 / r2;
                double s2 = sig[ab] * sig[ab] * ir2;
                double q = s2 * s2 * s2;
                double phi = 24.0 * eps[ab] * ir2 * q * (2.0 * q - 1.0);
                double dphi = -48.0 * eps[ab] * ir2 * ir2 * q * (7.0 * q - 2.0);
                double dg[3] = {g[i] - g[j], g[n + i] - g[n + j],
                                g[2 * n + i] - g[2 * n + j]};
                double ddg = d[0] * dg[0] + d[1] * dg[1] + d[2] * dg[2];
                /* row i collects J (g_i - g_j) from every neighbour j */
                gx += phi * dg[0] + 2.0 * dphi * d[0] * ddg;
                gy += phi * dg[1] + 2.0 * dphi * d[1] * ddg;
                gz += phi * dg[2] + 2.0 * dphi * d[2] * ddg;
                if (j > i) {
                    double dphi_deps = phi / eps[ab];
                    double dphi_dsig = 144.0 * eps[ab] * ir2 * q * (4.0 * q - 1.0) / sig[ab];
                    gp[ab] += dphi_deps * ddg;
                    gp[npair + ab] += dphi_dsig * ddg;
                }
            }
            grad_pos[i] = gx;
            grad_pos[n + i] = gy;
            grad_pos[2 * n + i] = gz;
        }
    }
    /* per ordered type pair gradients (a, b): unordered pair contributions
     * were recorded under (type_i, type_j); fold symmetric entries. */
    double geps[ORC_MAX_TYPES * ORC_MAX_TYPES] = {0}, gsig[ORC_MAX_TYPES * ORC_MAX_TYPES] = {0};
    for (int t = 0; t < nthr; t++)
        for (int k = 0; k < npair; k++) {
            geps[k] += gp_thr[(size_t)t * 2 * npair + k];
            gsig[k] += gp_thr[(size_t)t * 2 * npair + npair + k];
        }
    for (int k = 0; k < 2 * nt; k++)
        grad_theta[k] = 0.0;
    for (int a = 0; a < nt; a++)
        for (int b = 0; b < nt; b++) {
            int ab = a * nt + b;
            /* sig_ab = (sig_a + sig_b)/2 ; eps_ab = sqrt(eps_a eps_b) */
            grad_theta[nt + a] += 0.5 * gsig[ab];
            grad_theta[nt + b] += 0.5 * gsig[ab];
            grad_theta[a] += geps[ab] * theta[b] / (2.0 * eps[ab]);
            grad_theta[b] += geps[ab] * theta[a] / (2.0 * eps[ab]);
        }
    free(gp_thr);
    free(g);
    return L;
}

/* ------------------------------------------------------------------------ */
/* Live simulation statistics (Sec. 4): particles binned into cells that
 * mimic a CSF-1 cell of side >= bin_side; returns
 * out[0] mean, out[1] std/mean (population std; 0 when mean is 0),
 * out[2] median (mean of the two middle values for an even count),
 * out[3] max, out[4] number of bins, out[5] number of empty bins.       */
static int cmp_i64(const void *a, const void *b)
{
    int64_t x = *(const int64_t *)a, y = *(const int64_t *)b;
    return (x > y) - (x < y);
}

void orc_live_stats(int64_t n, const double *pos, const double *box,
                    double bin_side, double *out)
{
    int32_t nc3[3];
    orc_cell_dims(box, bin_side, nc3);
    int64_t nb = (int64_t)nc3[0] * nc3[1] * nc3[2];
    int32_t *cell_of = (int32_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
    int32_t *order = (int32_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
    int32_t *start = (int32_t *)malloc((size_t)(nb + 1) * sizeof(int32_t));
    orc_cells(n, pos, box, nc3, cell_of, order, start);
    int64_t *cnt = (int64_t *)malloc((size_t)nb * sizeof(int64_t));
    double sum = 0.0;
    int64_t mx = 0, empty = 0;
    for (int64_t c = 0; c < nb; c++) {
        cnt[c] = start[c + 1] - start[c];
        sum += (double)cnt[c];
        if (cnt[c] > mx)
            mx = cnt[c];
        if (cnt[c] == 0)
            empty++;
    }
    double mean = sum / (double)nb;
    double var = 0.0;
    for (int64_t c = 0; c < nb; c++)
        var += ((double)cnt[c] - mean) * ((double)cnt[c] - mean);
    var /= (double)nb;
    qsort(cnt, (size_t)nb, sizeof(int64_t), cmp_i64);
    double median = (nb % 2) ? (double)cnt[nb / 2]
                             : 0.5 * ((double)cnt[nb / 2 - 1] + (double)cnt[nb / 2]);
    out[0] = mean;
    out[1] = mean > 0.0 ? sqrt(var) / mean : 0.0;
    out[2] = median;
    out[3] = (double)mx;
    out[4] = (double)nb;
    out[5] = (double)empty;
    free(cnt);
    free(cell_of);
    free(order);
    free(start);
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

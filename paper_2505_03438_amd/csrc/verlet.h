// Per-particle update of the Stormer-Verlet integrator (velocity form, Sec.
// 2.1), shared by the integrator kernel and the force kernels that run it
// right after a particle's force (so that a step's positions are advanced
// without a separate pass over the particle arrays).
#pragma once

#include "pair.h"

namespace mdlj {

__device__ __forceinline__ double wrap_box(double x, double L)
{
#pragma clang fp contract(off)
    if (x >= L)
        x -= L;
    else if (x < 0.0)
        x += L;
    if (x >= L) x = 0.0;  // x + L may round up to exactly L
    return x;
}

__device__ __forceinline__ uint32_t quantise_i(double x, double S)
{
    double q = x * S;
    q = q < 0.0 ? 0.0 : (q > 4294967295.0 ? 4294967295.0 : q);
    return (uint32_t)q;
}

// What the update of particle i reads besides its force: loaded ahead of
// the update (a force kernel loads it before the particle's force loop, so
// that the loads are in flight while the force is computed).
template <typename real, bool ONE_TYPE>
struct VState {
    real vx, vy, vz;
    double x, y, z;
    int4 ref;
    int t;
    __device__ __forceinline__ void load(const IntegrateArgs &a, int i, size_t N, const double *pos_in, bool start)
    {
        const real *v = (const real *)a.vel;
        t = ONE_TYPE ? 0 : a.type[i];
        vx = v[i];
        vy = v[N + i];
        vz = v[2 * N + i];
        if (start) {
            x = pos_in[i];
            y = pos_in[N + i];
            z = pos_in[2 * N + i];
            ref = a.stage_ref[i];
        }
    }
};

// Particle i (state p, loaded by VState::load) with force (Fx, Fy, Fz):
// kick_prev completes the previous step (v += (dt/2) F/m, and its kinetic
// energy into ke), start begins the next one (v += (dt/2) F/m; x += dt v,
// wrapped, into pos_out; the fixed-point stage into stage_out; the skin
// check against the reference stage, its squared displacement into d2).
// ONE_TYPE: a single particle type, so the type array is not read and the
// staged type field (0, written by the cell build) is left as it is.
template <typename real, bool ISO, bool ONE_TYPE>
__device__ __forceinline__ void verlet_update(const IntegrateArgs &a, const Geom &g, int i, size_t N,
                                              const VState<real, ONE_TYPE> &p, real Fx, real Fy, real Fz,
                                              bool kick_prev, bool start, double *pos_out, int4 *stage_out,
                                              double &ke, float &d2)
{
#pragma clang fp contract(off)
    real *v = (real *)a.vel;
    double im = a.inv_mass[p.t];
    real c = (real)(a.hdt * im);  // (dt/2) / m, as in v += (dt/2) (1/m) F
    real vx = p.vx, vy = p.vy, vz = p.vz;
    real ax = c * Fx, ay = c * Fy, az = c * Fz;
    if (kick_prev) {
        vx += ax;
        vy += ay;
        vz += az;
        if (a.energy) ke = 0.5 * ((double)vx * (double)vx + (double)vy * (double)vy + (double)vz * (double)vz) / im;
    }
    if (start) {
        vx += ax;
        vy += ay;
        vz += az;
        double x = wrap_box(p.x + a.dt * (double)vx, g.L[0]);
        double y = wrap_box(p.y + a.dt * (double)vy, g.L[1]);
        double z = wrap_box(p.z + a.dt * (double)vz, g.L[2]);
        pos_out[i] = x;
        pos_out[N + i] = y;
        pos_out[2 * N + i] = z;
        int4 q;
        q.x = (int)quantise_i(x, g.S[0]);
        q.y = (int)quantise_i(y, g.S[1]);
        q.z = (int)quantise_i(z, g.S[2]);
        q.w = p.t;
        if (ONE_TYPE)
            *(int3 *)&stage_out[i] = make_int3(q.x, q.y, q.z);
        else
            stage_out[i] = q;
        // skin check: displacement since the last build, minimum image
        float dx, dy, dz;
        staged_delta<ISO>(q, p.ref, g, dx, dy, dz);
        float dd = dx * dx + dy * dy + dz * dz;
        if (dd >= g.disp2) {
            atomicOr(&a.flags[0], (int)MD_FLAG_SKIN_EXCEEDED);
            atomicMin(&a.flags[1], a.step_index);
        }
        if (!(x == x && y == y && z == z)) atomicOr(&a.flags[0], (int)MD_FLAG_NONFINITE);
        d2 = dd;
    }
    v[i] = vx;
    v[N + i] = vy;
    v[2 * N + i] = vz;
}

}  // namespace mdlj

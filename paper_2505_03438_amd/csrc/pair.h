// Device-side pair arithmetic shared by the force, list-build and adjoint
// kernels: the FP32 Lennard-Jones pair on fixed-point staged coordinates and
// the FP64 exact cutoff decision used inside the guard band.
#pragma once

#include "md_internal.h"

namespace mdlj {

// Per-kernel copy of the FP32 pair constants.  With one type every lookup is
// a scalar; with two types the 2x2 tables are selected per lane.  Every
// index below is a constant (no loops), so that the tables are promoted to
// registers before any later pass could turn the selects into an indexed
// load from a stack copy.
template <int NT>
struct TabF {
    float lo[NT * NT], hi[NT * NT], sig2[NT * NT], eps24[NT * NT], eps4[NT * NT], eps24w[NT * NT];
    double rc2[NT * NT];
    __device__ __forceinline__ void load_one(const PairTab *__restrict__ t, int k)
    {
        lo[k] = t->rc2_lo[k];
        hi[k] = t->rc2_hi[k];
        sig2[k] = t->sig2[k];
        eps24[k] = t->eps24[k];
        eps4[k] = t->eps4[k];
        eps24w[k] = t->eps24w[k];
        rc2[k] = t->rc2[k];
    }
    __device__ __forceinline__ void load(const PairTab *__restrict__ t)
    {
        load_one(t, 0);
        if (NT > 1) {
            load_one(t, 1);
            load_one(t, 2);
            load_one(t, 3);
        }
    }
    __device__ __forceinline__ float pick(const float *v, int ab) const
    {
        if (NT == 1) return v[0];
        return ab == 0 ? v[0] : (ab == 1 ? v[1] : (ab == 2 ? v[2] : v[3]));
    }
    __device__ __forceinline__ double pickd(const double *v, int ab) const
    {
        if (NT == 1) return v[0];
        return ab == 0 ? v[0] : (ab == 1 ? v[1] : (ab == 2 ? v[2] : v[3]));
    }
};

// Stencil offsets copied out of the by-value geometry with constant indices
// into LDS: indexing the kernel-argument struct with a run-time index would
// make the compiler copy the whole struct to scratch memory.  Ends with a
// barrier.
__device__ __forceinline__ void load_offsets(const Geom &g, int (*so)[kMaxOfs])
{
    if (threadIdx.x == 0) {
#pragma unroll
        for (int d = 0; d < 3; d++)
#pragma unroll
            for (int k = 0; k < kMaxOfs; k++) so[d][k] = g.ofs[d][k];
    }
    __syncthreads();
}

// Exact FP64 squared minimum-image distance of particles i and j, in the
// fixed order of the plain definition: d = x_i - x_j; if d > L/2, d -= L,
// else if d < -L/2, d += L; r2 = dx*dx + dy*dy + dz*dz; no FMA contraction.
static __device__ __noinline__ double exact_r2(const double *__restrict__ pos, int n, int i, int j, double L0,
                                        double L1, double L2)
{
#pragma clang fp contract(off)
    size_t N = (size_t)n;
    double dx = pos[i] - pos[j];
    if (dx > 0.5 * L0)
        dx -= L0;
    else if (dx < -0.5 * L0)
        dx += L0;
    double dy = pos[N + i] - pos[N + j];
    if (dy > 0.5 * L1)
        dy -= L1;
    else if (dy < -0.5 * L1)
        dy += L1;
    double dz = pos[2 * N + i] - pos[2 * N + j];
    if (dz > 0.5 * L2)
        dz -= L2;
    else if (dz < -0.5 * L2)
        dz += L2;
    return dx * dx + dy * dy + dz * dz;
}

// Minimum-image displacement of staged coordinates, in units of L_x / 2^32.
template <bool ISO>
__device__ __forceinline__ void staged_delta(const int4 &a, const int4 &b, const Geom &g, float &dx,
                                             float &dy, float &dz)
{
    dx = (float)(int)((uint32_t)a.x - (uint32_t)b.x);
    dy = (float)(int)((uint32_t)a.y - (uint32_t)b.y);
    dz = (float)(int)((uint32_t)a.z - (uint32_t)b.z);
    if (!ISO) {
        dy *= g.ry;
        dz *= g.rz;
    }
}

// Decide "r2 < cutoff" for a staged pair: in FP32 outside the guard band,
// from the FP64 master positions inside it.
__device__ __forceinline__ bool within(float r2, float lo, float hi, double cut2, const double *pos,
                                       int n, int i, int j, const Geom &g)
{
    bool in = r2 < lo;
    if (r2 >= lo && r2 < hi) in = exact_r2(pos, n, i, j, g.L[0], g.L[1], g.L[2]) < cut2;
    return in;
}

// FP32 Lennard-Jones pair in fixed-point units: returns phi_u with
// f_ij = phi_u * d_u (force in physical units) and, for ENERGY, adds the pair
// energy 4 eps q (q - 1) and virial 24 eps q (2q - 1) to eu, ew.
template <int NT, bool ENERGY>
__device__ __forceinline__ float lj_f32(float r2, int ab, bool in, const TabF<NT> &t, float &eu, float &ew,
                                        int &np)
{
    // a pair outside the cutoff gets 1/r^2 = 0, which zeroes every term
    // below without a branch
    float ir2 = in ? __builtin_amdgcn_rcpf(r2) : 0.0f;
    float s2 = t.pick(t.sig2, ab) * ir2;
    float q = s2 * s2 * s2;
    float a = q * (2.0f * q - 1.0f);
    float phi = t.pick(t.eps24, ab) * ir2 * a;
    if (ENERGY) {
        eu += t.pick(t.eps4, ab) * q * (q - 1.0f);
        ew += t.pick(t.eps24w, ab) * a;
        np += in ? 1 : 0;
    }
    return phi;
}

// FP64 pair in the operation order of the plain definition.
__device__ __forceinline__ void lj_f64(double r2, double eps, double sig, double &phi, double &u)
{
#pragma clang fp contract(off)
    double ir2 = 1.0 / r2;
    double s2 = sig * sig * ir2;
    double q = s2 * s2 * s2;
    phi = 24.0 * eps * ir2 * q * (2.0 * q - 1.0);
    u = 4.0 * eps * q * (q - 1.0);
}

__device__ __forceinline__ double min_image(double d, double L)
{
#pragma clang fp contract(off)
    if (d > 0.5 * L)
        d -= L;
    else if (d < -0.5 * L)
        d += L;
    return d;
}

// Deterministic block sum of up to 4 doubles over a block of NTH threads
// (wave shuffles then LDS), the result valid in thread 0.
template <int NTH>
__device__ __forceinline__ void block_sum4_n(double v[4], double *sh /* [4 * NTH/64] */)
{
#pragma unroll
    for (int k = 0; k < 4; k++)
        for (int off = 32; off > 0; off >>= 1) v[k] += __shfl_down(v[k], off, 64);
    int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0)
        for (int k = 0; k < 4; k++) sh[wave * 4 + k] = v[k];
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int k = 0; k < 4; k++) {
            double s = 0.0;
            for (int w = 0; w < NTH / 64; w++) s += sh[w * 4 + k];
            v[k] = s;
        }
    }
}

// Fixed point of the LDS force accumulators: force value c is held as c * K
// rounded toward zero to an even number of units, K = 2^62 / 1e10, in two's
// complement.  The resolution (4e-9 force units) is far below FP32 rounding
// of the forces, for small forces too (the integer and fraction parts are
// split toward zero, so a negative value keeps its full relative precision);
// a sum is exact up to |c| ~ 4.6e8 (a pair closer than ~0.2 sigma), beyond
// which the conversion saturates.
constexpr float kFixHi = 0.10737418f;           // K / 2^32 = 2^30 / 1e10
constexpr double kFixInv = 2.168404344971009e-9;  // 1e10 / 2^62

__device__ __forceinline__ unsigned long long to_fix(float c)
{
    float t = c * kFixHi;                     // in units of 2^32
    float h = truncf(t);                      // integer part, exact
    int hi = (int)h;                          // saturating conversion
    int lo = (int)((t - h) * 2147483648.0f);  // the fraction (exact) in units of 2, |lo| < 2^31
    return (unsigned long long)((long long)hi * 4294967296LL + (long long)lo * 2LL);
}

__device__ __forceinline__ float from_fix(unsigned long long v) { return (float)((double)(long long)v * kFixInv); }

// Deterministic block sum of up to 4 doubles (wave shuffles then LDS), the
// result valid in thread 0.
__device__ __forceinline__ void block_sum4(double v[4], double *sh /* [4 * kBlock/64] */)
{
#pragma unroll
    for (int k = 0; k < 4; k++)
        for (int off = 32; off > 0; off >>= 1) v[k] += __shfl_down(v[k], off, 64);
    int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0)
        for (int k = 0; k < 4; k++) sh[wave * 4 + k] = v[k];
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int k = 0; k < 4; k++) {
            double s = 0.0;
            for (int w = 0; w < kBlock / 64; w++) s += sh[w * 4 + k];
            v[k] = s;
        }
    }
}

}  // namespace mdlj

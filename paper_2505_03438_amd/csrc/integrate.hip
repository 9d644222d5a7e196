// Stormer-Verlet in velocity form (Sec. 2.1 names the Stormer-Verlet
// integrator): one kernel completes the previous step's second half kick and
// starts the next step (half kick, drift, wrap, fixed-point staging and the
// skin check of the rebuild policy), so each time step costs one integrator
// pass plus the force pass.  Kinetic energy is taken between the two kicks.
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

// ONE_TYPE: a single particle type, so the type array is not read and the
// staged type field (0, written by the cell build) is left as it is.
template <typename real, bool ISO, bool ONE_TYPE>
__global__ __launch_bounds__(kBlock) void k_integrate(IntegrateArgs a, Geom g)
{
#pragma clang fp contract(off)
    __shared__ double sh[4 * kBlock / 64];
    int i = blockIdx.x * kBlock + threadIdx.x;
    double ke = 0.0;
    float dmax = 0.f;  // squared displacement since the last build
    if (i < a.n) {
        size_t N = (size_t)a.n;
        real *v = (real *)a.vel;
        const real *F = (const real *)a.force;
        int t = ONE_TYPE ? 0 : a.type[i];
        double im = a.inv_mass[t];
        real c = (real)(a.hdt * im);  // (dt/2) / m, as in v += (dt/2) (1/m) F
        real vx = v[i], vy = v[N + i], vz = v[2 * N + i];
        real ax = c * F[i], ay = c * F[N + i], az = c * F[2 * N + i];
        if (a.kick_prev) {
            vx += ax;
            vy += ay;
            vz += az;
            if (a.energy)
                ke = 0.5 * ((double)vx * (double)vx + (double)vy * (double)vy + (double)vz * (double)vz) / im;
        }
        if (a.start) {
            vx += ax;
            vy += ay;
            vz += az;
            double x = wrap_box(a.pos[i] + a.dt * (double)vx, g.L[0]);
            double y = wrap_box(a.pos[N + i] + a.dt * (double)vy, g.L[1]);
            double z = wrap_box(a.pos[2 * N + i] + a.dt * (double)vz, g.L[2]);
            a.pos[i] = x;
            a.pos[N + i] = y;
            a.pos[2 * N + i] = z;
            int4 q;
            q.x = (int)quantise_i(x, g.S[0]);
            q.y = (int)quantise_i(y, g.S[1]);
            q.z = (int)quantise_i(z, g.S[2]);
            q.w = t;
            if (ONE_TYPE)
                *(int3 *)&a.stage[i] = make_int3(q.x, q.y, q.z);
            else
                a.stage[i] = q;
            // skin check: displacement since the last build, minimum image
            int4 r = a.stage_ref[i];
            float dx, dy, dz;
            staged_delta<ISO>(q, r, g, dx, dy, dz);
            float d2 = dx * dx + dy * dy + dz * dz;
            if (d2 >= g.disp2) {
                atomicOr(&a.flags[0], (int)MD_FLAG_SKIN_EXCEEDED);
                atomicMin(&a.flags[1], a.step_index);
            }
            if (!(x == x && y == y && z == z)) atomicOr(&a.flags[0], (int)MD_FLAG_NONFINITE);
            dmax = d2;
        }
        v[i] = vx;
        v[N + i] = vy;
        v[2 * N + i] = vz;
    }
    if (a.start && a.dpart) {
        // largest squared displacement since the last build, per block: the
        // rate of motion from which the autotuner derives the rebuild
        // interval (reduced by k_dmax_reduce)
        __shared__ float wm[kBlock / 64];
        for (int off = 32; off > 0; off >>= 1) dmax = fmaxf(dmax, __shfl_xor(dmax, off, 64));
        if ((threadIdx.x & 63) == 0) wm[threadIdx.x >> 6] = dmax;
        __syncthreads();
        if (threadIdx.x == 0) {
            float m = wm[0];
            for (int w = 1; w < kBlock / 64; w++) m = fmaxf(m, wm[w]);
            a.dpart[blockIdx.x] = m;
        }
    }
    if (a.energy && a.kick_prev) {
        double s4[4] = {ke, 0.0, 0.0, 0.0};
        block_sum4(s4, sh);
        if (threadIdx.x == 0) a.kpart[blockIdx.x] = s4[0];
    }
}

int integrate_blocks(int n) { return (n + kBlock - 1) / kBlock; }

void launch_integrate(const IntegrateArgs &a, const Geom &g, hipStream_t s)
{
    if (a.n <= 0) return;
    int nb = integrate_blocks(a.n);
    bool one = g.nt == 1;
    if (a.precision == MD_FP64) {
        if (g.iso) {
            if (one) k_integrate<double, true, true><<<nb, kBlock, 0, s>>>(a, g);
            else k_integrate<double, true, false><<<nb, kBlock, 0, s>>>(a, g);
        } else {
            if (one) k_integrate<double, false, true><<<nb, kBlock, 0, s>>>(a, g);
            else k_integrate<double, false, false><<<nb, kBlock, 0, s>>>(a, g);
        }
    } else {
        if (g.iso) {
            if (one) k_integrate<float, true, true><<<nb, kBlock, 0, s>>>(a, g);
            else k_integrate<float, true, false><<<nb, kBlock, 0, s>>>(a, g);
        } else {
            if (one) k_integrate<float, false, true><<<nb, kBlock, 0, s>>>(a, g);
            else k_integrate<float, false, false><<<nb, kBlock, 0, s>>>(a, g);
        }
    }
}

// One log entry {U, K, W, n_pairs} from the force partials {U, W, n} and the
// kinetic-energy partials, summed in a fixed order.
__global__ void k_log_entry(const double *__restrict__ fpart, int fb, int gather,
                            const double *__restrict__ kpart, int kb, double *__restrict__ out)
{
    __shared__ double sh[4 * kBlock / 64];
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    for (int b = threadIdx.x; b < fb; b += kBlock) {
        v[0] += fpart[b * 4 + 0];
        v[1] += fpart[b * 4 + 1];
        v[2] += fpart[b * 4 + 2];
    }
    for (int b = threadIdx.x; b < kb; b += kBlock) v[3] += kpart[b];
    block_sum4(v, sh);
    if (threadIdx.x == 0) {
        double h = gather ? 0.5 : 1.0;
        out[0] = v[0] * h;
        out[1] = v[3];
        out[2] = v[1] * h;
        out[3] = v[2] * h;
    }
}

void launch_log_entry(const double *fpart, int fblocks, int gather, const double *kpart, int kblocks,
                      double *out4, hipStream_t s)
{
    k_log_entry<<<1, kBlock, 0, s>>>(fpart, fblocks, gather, kpart, kblocks, out4);
}

__global__ void k_dmax_reduce(const float *__restrict__ dpart, int nb, int32_t *__restrict__ flags)
{
    __shared__ float wm[kBlock / 64];
    float m = 0.f;
    for (int b = threadIdx.x; b < nb; b += kBlock) m = fmaxf(m, dpart[b]);
    for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off, 64));
    if ((threadIdx.x & 63) == 0) wm[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < kBlock / 64; w++) m = fmaxf(m, wm[w]);
        m = fmaxf(m, wm[0]);
        flags[4] = __float_as_int(m);
    }
}

void launch_dmax_reduce(const float *dpart, int nblocks, int32_t *flags, hipStream_t s)
{
    k_dmax_reduce<<<1, kBlock, 0, s>>>(dpart, nblocks, flags);
}

// Zero a buffer with a kernel (not a memset node, so it can sit in a graph).
__global__ void k_zero_u32(uint32_t *p, int64_t n)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0u;
}

void launch_zero(void *p, int64_t bytes, hipStream_t s)
{
    int64_t n = bytes / 4;
    if (n <= 0) return;
    k_zero_u32<<<(unsigned)((n + kBlock - 1) / kBlock), kBlock, 0, s>>>((uint32_t *)p, n);
}

}  // namespace mdlj

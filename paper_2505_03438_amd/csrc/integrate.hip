// Stormer-Verlet in velocity form (Sec. 2.1 names the Stormer-Verlet
// integrator): one kernel completes the previous step's second half kick and
// starts the next step (half kick, drift, wrap, fixed-point staging and the
// skin check of the rebuild policy), so each time step costs one integrator
// pass plus the force pass.  Kinetic energy is taken between the two kicks.
#include "verlet.h"

namespace mdlj {

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
        const real *F = (const real *)a.force;
        VState<real, ONE_TYPE> p;
        p.load(a, i, N, a.pos, a.start != 0);
        verlet_update<real, ISO, ONE_TYPE>(a, g, i, N, p, F[i], F[N + i], F[2 * N + i], a.kick_prev != 0,
                                           a.start != 0, a.pos, a.stage, ke, dmax);
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

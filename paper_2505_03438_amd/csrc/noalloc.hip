// Forces without a handle and without any allocation: for callers that
// cannot allocate device memory (code under HIP graph capture, tight serving
// loops, harnesses that forbid allocation).
//
// The computation is md_compute_forces with linked cells, gather-only (each
// pair evaluated from both sides; Sec. 2.1 forces over the Sec. 2.2.1 linked
// cells): bin by a counting sort, order each cell by particle index, gather
// the positions into cell order and stage them, run the linked-cell force
// kernel, scatter the forces back to the caller's order.  Every intermediate
// array lives in one file-scope device array, `scratch`, carved per call;
// each GPU holds its own copy of it until the process ends.
#include <string.h>

#include <algorithm>
#include <mutex>
#include <string>

#include "md_internal.h"

namespace mdlj {
int validate_md_config(const md_config *c);
int make_geom(const md_config &c, double csf, Geom &g);
}  // namespace mdlj

using namespace mdlj;

namespace {

constexpr size_t kScratchBytes = (size_t)MD_NOALLOC_SCRATCH_MIB << 20;

// The scratch memory of the allocation-free entry point.  Host code never
// passes this name to a kernel or a copy: it is a host-side stand-in.  The
// device address comes from hipGetSymbolAddress, once per device.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// Device address of this device's scratch (the current device), or NULL
// with the error set.
int scratch_ptr(void **out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) return fail(MD_ERR_NO_DEVICE, "device index out of range");
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return MD_OK;
}

// Bump allocator over the scratch: 256-byte aligned pieces.
struct Carve {
    unsigned char *base;
    size_t off = 0;
    template <typename T>
    T *take(size_t count)
    {
        T *p = (T *)(base + off);
        off += (count * sizeof(T) + 255) & ~(size_t)255;
        return p;
    }
};

// Bytes the carving below takes for n particles and ncell cells.
size_t scratch_need(int64_t n, int64_t ncell, size_t real)
{
    auto r = [](size_t b) { return (b + 255) & ~(size_t)255; };
    size_t m = (size_t)std::max<int64_t>(n, 1), c = (size_t)ncell;
    size_t blocks = (m + kBlock - 1) / kBlock;
    return r(8 * 4) + r(sizeof(PairTab)) + r(blocks * 4 * 8) + 7 * r(m * 4) + r(c * 4) + r((c + 1) * 4) +
           r((size_t)scan_scratch_size(c) * 4) + r(3 * m * 8) + r(m * 16) + r(3 * m * real);
}

__global__ void k_iota(int n, int32_t *__restrict__ ids)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) ids[i] = i;
}

template <typename real>
__global__ void k_unsort(int n, const int32_t *__restrict__ ids, const real *__restrict__ fs,
                         real *__restrict__ force)
{
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    size_t N = (size_t)n;
    int i = ids[k];
    force[i] = fs[k];
    force[N + i] = fs[N + k];
    force[2 * N + i] = fs[2 * N + k];
}

}  // namespace

extern "C" int64_t md_noalloc_max_particles(void) { return MD_NOALLOC_MAX_N; }

extern "C" int md_compute_forces_noalloc(const md_config *cfg, const double *pos, const int32_t *type,
                                         const double *lj, void *force, double *out, void *stream)
{
    int rc = validate_md_config(cfg);
    if (rc) return rc;
    const int64_t n = cfg->n;
    if (n > MD_NOALLOC_MAX_N)
        return fail(MD_ERR_INVALID_ARG, "md_compute_forces_noalloc: n = " + std::to_string(n) + " exceeds " +
                                            std::to_string((long long)MD_NOALLOC_MAX_N));
    if (n > 0 && (!pos || !type || !force)) return fail(MD_ERR_INVALID_ARG, "pos, type and force must not be NULL");
    if (!lj) return fail(MD_ERR_INVALID_ARG, "lj must not be NULL");
    Geom g;
    if ((rc = make_geom(*cfg, cfg->csf, g))) return rc;
    size_t real = cfg->precision == MD_FP64 ? 8 : 4;
    size_t need = scratch_need(n, g.ncell, real);
    if (need > kScratchBytes)
        return fail(MD_ERR_INVALID_ARG, "md_compute_forces_noalloc: " + std::to_string(g.ncell) + " cells and " +
                                            std::to_string(n) + " particles need " + std::to_string(need >> 10) +
                                            " KiB of scratch, more than its " +
                                            std::to_string(kScratchBytes >> 10) + " KiB (use a coarser csf)");
    void *base = nullptr;
    if ((rc = scratch_ptr(&base))) return rc;
    hipStream_t s = (hipStream_t)stream;
    int m = (int)n;
    Carve cv{(unsigned char *)base};
    int32_t *flags = cv.take<int32_t>(8);
    PairTab *tab = cv.take<PairTab>(1);
    double *partials = cv.take<double>((size_t)((std::max(m, 1) + kBlock - 1) / kBlock) * 4);
    int32_t *cell_id = cv.take<int32_t>(std::max(m, 1));
    int32_t *slot = cv.take<int32_t>(std::max(m, 1));
    int32_t *perm = cv.take<int32_t>(std::max(m, 1));
    int32_t *key = cv.take<int32_t>(std::max(m, 1));
    int32_t *cell_sorted = cv.take<int32_t>(std::max(m, 1));
    int32_t *order = cv.take<int32_t>(std::max(m, 1));
    int32_t *ids = cv.take<int32_t>(std::max(m, 1));
    int32_t *cell_count = cv.take<int32_t>(g.ncell);
    int32_t *cell_start = cv.take<int32_t>((size_t)g.ncell + 1);
    int32_t *scan = cv.take<int32_t>((size_t)scan_scratch_size(g.ncell));
    double *spos = cv.take<double>(3 * (size_t)std::max(m, 1));
    int4 *stage = cv.take<int4>(std::max(m, 1));
    void *sforce = cv.take<unsigned char>(3 * (size_t)std::max(m, 1) * real);
    // (the sorted types and ids reuse key and perm, free after the in-cell sort)
    int32_t *stype = key, *sids = perm;
    if (cv.off > kScratchBytes) return fail(MD_ERR_HIP, "internal error: scratch carving exceeds its size");
    launch_fill_i32(flags, 0, 8, s);
    launch_prepare_tab(lj, cfg->rc2, g, tab, s);
    if (m > 0) {
        int nb = (m + kBlock - 1) / kBlock;
        launch_fill_i32(cell_count, 0, g.ncell, s);
        launch_cell_hist(m, pos, g, cell_id, slot, cell_count, flags, s);
        launch_scan(cell_count, cell_start, g.ncell, scan, s);
        k_iota<<<nb, kBlock, 0, s>>>(m, ids);
        // cell-order slot k -> particle order[k], each cell by particle index
        launch_scatter_sort(m, cell_id, slot, cell_start, ids, perm, key, cell_sorted, order, s);
        launch_gather(m, cfg->precision, order, pos, nullptr, nullptr, type, ids, spos, nullptr, nullptr, stype,
                      sids, cell_id, cell_sorted, g, stage, stage, s);
    }
    ForceArgs a;
    memset(&a, 0, sizeof(a));
    a.n = m;
    a.precision = cfg->precision;
    a.container = MD_CONTAINER_LC;
    a.newton3 = MD_N3L_OFF;
    a.energy = out != nullptr;
    a.pos = spos;
    a.type = stype;
    a.stage = stage;
    a.cell_start = cell_start;
    a.cell_sorted = cell_sorted;
    a.tab = tab;
    a.force = sforce;
    a.partials = partials;
    a.flags = flags;
    a.window = false;
    if (m > 0) {
        launch_force(a, g, s);
        int nb = (m + kBlock - 1) / kBlock;
        if (cfg->precision == MD_FP64)
            k_unsort<double><<<nb, kBlock, 0, s>>>(m, sids, (const double *)sforce, (double *)force);
        else
            k_unsort<float><<<nb, kBlock, 0, s>>>(m, sids, (const float *)sforce, (float *)force);
    }
    if (out) launch_reduce_out(partials, force_blocks(a), 1, out, s);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "md_compute_forces_noalloc launch");
    return MD_OK;
}

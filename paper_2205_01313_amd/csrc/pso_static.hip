// pso_static.hip -- pso_batch_run_static: the batched run of pso_batch_run
// for callers that cannot allocate device memory.  Every device buffer the
// batched kernels need (each swarm's state and gang region, the descriptors,
// the work queue, the results, the work counter and the error flag) is
// carved out of `scratch`, one fixed array in device memory that each GPU
// holds from the library's first use on it until the process ends.  Host
// staging is fixed-size too, so the call neither allocates device memory nor
// touches the heap; it launches the same kernels, in the same shape rules,
// as pso_batch_create + pso_batch_launch + pso_batch_results.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstring>
#include <mutex>

#include "pso.h"
#include "pso_block.hpp"
#include "pso_device.hpp"
#include "pso_guard.hpp"
#include "pso_kernels.hpp"

int pso_internal_fail(int code, const char *fmt, ...);
int pso_internal_check_desc(const pso_desc *d);

namespace {

constexpr size_t SCRATCH_BYTES = PSO_STATIC_SCRATCH_BYTES;
constexpr int64_t MAX_SWARMS = PSO_STATIC_MAX_SWARMS;
constexpr uint32_t MAX_ENTRIES = PSO_STATIC_MAX_ENTRIES;
constexpr int MAX_DEVICES = 64;
constexpr int MAX_D = 4096; // the largest D any descriptor may have

// The device memory of every call on a device.  In host code this name is
// only a stand-in for the symbol: its device address comes from
// hipGetSymbolAddress (scratch_ptr below) and nothing else.
static __device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];

// One call at a time in this process: calls share each device's scratch and
// the host staging below.
std::mutex g_mu;
void *g_ptr[MAX_DEVICES]; // each device's address of `scratch`

// Host staging (fixed size; nothing is allocated per call).
pso::BatchItem h_items[MAX_SWARMS];
pso::BatchEntry h_entries[MAX_ENTRIES];
pso::BatchResult h_results[MAX_SWARMS];
uint32_t h_parts[MAX_SWARMS];
uint32_t h_order[MAX_SWARMS];
unsigned char h_streamed[MAX_SWARMS];
const float h_zero_shift[MAX_D] = {};

#define HIP_TRY(expr)                                                                                    \
    do {                                                                                                 \
        hipError_t e_ = (expr);                                                                          \
        if (e_ != hipSuccess) return pso_internal_fail(PSO_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

size_t al256(size_t b) { return (b + 255) & ~size_t(255); }

// The device address of `scratch` on the current device, looked up once per
// device with that device current.
int scratch_ptr(char **out)
{
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= MAX_DEVICES) return pso_internal_fail(PSO_EDEVICE, "device %d beyond %d devices", dev, MAX_DEVICES);
    if (!g_ptr[dev]) {
        void *p = nullptr;
        HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return pso_internal_fail(PSO_EDEVICE, "hipGetSymbolAddress returned no address");
        g_ptr[dev] = p;
    }
    *out = static_cast<char *>(g_ptr[dev]);
    return PSO_OK;
}

int run_locked(const pso_desc *descs, int64_t count, pso_result *results, hipStream_t stream)
{
    int maxD = 1;
    for (int64_t i = 0; i < count; ++i) {
        if (const int rc = pso_internal_check_desc(&descs[i])) return rc;
        maxD = std::max(maxD, (int)descs[i].D);
    }
    if (maxD > MAX_D) return pso_internal_fail(PSO_EINVAL, "D=%d above %d", maxD, MAX_D);

    // The shape of a new batch before any autotuning (pso_batch_create): one
    // 1024-lane workgroup per compute unit with its parts' state staged in
    // LDS; a swarm too large to stage streams, in a second kernel of the
    // same launch.
    pso::BatchShape sh = pso::DEFAULT_STAGED_SHAPE;
    sh.stage_kib = pso::staged_kib_fitting(maxD, 1);
    const pso::BatchShape stream_sh = pso::DEFAULT_BATCH_SHAPE;
    int grid = 0, grid_s = 0;
    if (sh.stage_kib > 0) HIP_TRY(pso::shape_grid(maxD, sh, &grid));
    HIP_TRY(pso::shape_grid(maxD, stream_sh, &grid_s));
    if (grid_s < 1) return pso_internal_fail(PSO_EDEVICE, "no co-resident workgroup for the streamed kernel");

    uint64_t n_entries = 0, n_first = 0;
    for (int64_t i = 0; i < count; ++i) {
        const pso_desc &d = descs[i];
        uint32_t parts = grid > 0 ? pso::staged_parts((uint64_t)d.N, d.D, d.fitness_id, sh.stage_kib, grid) : 0u;
        h_streamed[i] = parts == 0;
        if (parts == 0) parts = pso::parts_for((uint64_t)d.N, d.D, grid_s, stream_sh);
        h_parts[i] = parts;
        n_entries += parts;
        if (!h_streamed[i]) n_first += parts;
    }
    if (n_entries > MAX_ENTRIES)
        return pso_internal_fail(PSO_EINVAL, "the swarms need %llu work-queue entries, above %u",
                                 (unsigned long long)n_entries, MAX_ENTRIES);

    // Byte layout of the scratch: descriptors, work queue, results, work
    // counter, error flag, then each swarm's state and gang region.
    const size_t o_items = 0;
    const size_t o_entries = o_items + al256(sizeof(pso::BatchItem) * count);
    const size_t o_results = o_entries + al256(sizeof(pso::BatchEntry) * n_entries);
    const size_t o_next = o_results + al256(sizeof(pso::BatchResult) * count);
    const size_t o_err = o_next + 256;
    size_t total = o_err + 256;
    for (int64_t i = 0; i < count; ++i) {
        const pso::Layout L = pso::layout_of((uint64_t)descs[i].N, descs[i].D, false);
        total += al256(L.total) + al256(pso::gang_bytes(h_parts[i], descs[i].D));
        if (total > SCRATCH_BYTES)
            return pso_internal_fail(PSO_ENOMEM, "the swarms need more than the %zu bytes of static scratch",
                                     SCRATCH_BYTES);
    }

    char *base = nullptr;
    if (const int rc = scratch_ptr(&base)) return rc;
    pso::BatchItem *d_items = reinterpret_cast<pso::BatchItem *>(base + o_items);
    pso::BatchEntry *d_entries = reinterpret_cast<pso::BatchEntry *>(base + o_entries);
    pso::BatchResult *d_results = reinterpret_cast<pso::BatchResult *>(base + o_results);
    unsigned int *d_next = reinterpret_cast<unsigned int *>(base + o_next);
    unsigned int *d_err = reinterpret_cast<unsigned int *>(base + o_err);

    size_t off = o_err + 256;
    for (int64_t i = 0; i < count; ++i) {
        const pso_desc &d = descs[i];
        const pso::Layout L = pso::layout_of((uint64_t)d.N, d.D, false);
        pso::BatchItem &it = h_items[i];
        it = pso::BatchItem{};
        it.a = pso::bind(base + off, L, (uint64_t)d.N, d.D);
        off += al256(L.total);
        it.a.lo = d.bounds[0];
        it.a.hi = d.bounds[1];
        it.a.w = d.w;
        it.a.c1 = d.c1;
        it.a.c2 = d.c2;
        it.a.vmax = d.vmax;
        it.a.k0 = (uint32_t)d.seed;
        it.a.k1 = (uint32_t)(d.seed >> 32);
        it.fitness = d.fitness_id;
        it.max_iter = d.max_iter;
        it.tol = d.tol;
        it.fstar = d.f_star;
        pso::bind_gang(&it, base + off, h_parts[i]);
        off += al256(pso::gang_bytes(h_parts[i], d.D));
        HIP_TRY(hipMemcpyAsync(const_cast<float *>(it.a.shift), d.shift ? d.shift : h_zero_shift,
                               sizeof(float) * d.D, hipMemcpyHostToDevice, stream));
    }

    // Work queue as pso_batch_create orders it: staged swarms first, then
    // the largest work per part first (ties by swarm index).
    for (int64_t i = 0; i < count; ++i) h_order[i] = (uint32_t)i;
    std::sort(h_order, h_order + count, [&](uint32_t x, uint32_t y) {
        if (h_streamed[x] != h_streamed[y]) return h_streamed[x] < h_streamed[y];
        const double wx = double(descs[x].N) * descs[x].D * double(descs[x].max_iter + 1) / h_parts[x];
        const double wy = double(descs[y].N) * descs[y].D * double(descs[y].max_iter + 1) / h_parts[y];
        if (wx != wy) return wx > wy;
        return x < y;
    });
    uint32_t e = 0;
    for (int64_t k = 0; k < count; ++k)
        for (uint32_t p = 0; p < h_parts[h_order[k]]; ++p)
            h_entries[e++] = pso::BatchEntry{h_order[k], p, h_order[k], 0u};

    HIP_TRY(hipMemcpyAsync(d_items, h_items, sizeof(pso::BatchItem) * count, hipMemcpyHostToDevice, stream));
    HIP_TRY(hipMemcpyAsync(d_entries, h_entries, sizeof(pso::BatchEntry) * n_entries, hipMemcpyHostToDevice, stream));
    HIP_TRY(pso::launch_clear_u32(d_err, stream));
    HIP_TRY(pso::launch_batch_reset(d_items, d_results, (uint32_t)count, d_next, stream));
    const long long unlimited = (long long)1 << 62;
    if (n_first > 0)
        HIP_TRY(pso::launch_batch(d_items, d_entries, d_results, (uint32_t)n_first, d_next, maxD,
                                  (int)std::min<uint64_t>(n_first, (uint64_t)grid), sh.lanes, unlimited, unlimited,
                                  stream, nullptr, nullptr, d_err, sh.stage_kib));
    if (n_entries > n_first)
        HIP_TRY(pso::launch_batch(d_items, d_entries + n_first, d_results, (uint32_t)(n_entries - n_first), d_next,
                                  maxD, (int)std::min<uint64_t>(n_entries - n_first, (uint64_t)grid_s),
                                  stream_sh.lanes, unlimited, unlimited, stream, nullptr, nullptr, d_err, 0));

    unsigned int err = 0;
    HIP_TRY(hipMemcpyAsync(&err, d_err, sizeof err, hipMemcpyDeviceToHost, stream));
    HIP_TRY(hipMemcpyAsync(h_results, d_results, sizeof(pso::BatchResult) * count, hipMemcpyDeviceToHost, stream));
    HIP_TRY(hipStreamSynchronize(stream));
    if (err) return pso_internal_fail(PSO_EDEVICE, "a batched swarm's parts timed out waiting for each other");
    for (int64_t i = 0; i < count; ++i) {
        results[i].gbest_value = pso::key_fitness(h_results[i].gkey);
        results[i].status = PSO_OK;
        results[i].gbest_iter = h_results[i].giter;
        results[i].iters = h_results[i].iters;
        if (results[i].gbest_pos)
            HIP_TRY(hipMemcpyAsync(results[i].gbest_pos, h_items[i].a.gpos, sizeof(float) * descs[i].D,
                                   hipMemcpyDeviceToHost, stream));
    }
    HIP_TRY(hipStreamSynchronize(stream));
    return PSO_OK;
}

} // namespace

extern "C" int pso_batch_run_static(const pso_desc *descs, int64_t count, pso_result *results, void *hip_stream)
{
    return pso::guarded([&]() -> int {
        if (count < 1 || count > MAX_SWARMS)
            return pso_internal_fail(PSO_EINVAL, "count=%lld outside [1, %lld]", (long long)count, (long long)MAX_SWARMS);
        if (!descs) return pso_internal_fail(PSO_EINVAL, "descs is NULL");
        if (!results) return pso_internal_fail(PSO_EINVAL, "results is NULL");
        std::lock_guard<std::mutex> g(g_mu);
        return run_locked(descs, count, results, static_cast<hipStream_t>(hip_stream));
    });
}

// pso_prims.hip -- test kernels around the library's device primitives of
// the gbest aggregation (Alg. 1 Step 5; Sec. 3.1 Alg. 2, Sec. 3.2 Alg. 3):
// the packed (fitness, index) key, the wavefront minimum, the workgroup
// minimum, the device-wide 64-bit atomicMin publish and the seqlock of the
// asynchronous variant.  They run the library's own device functions
// (csrc/pso_device.hpp, csrc/pso_aggregate.hpp) on inputs the tests choose,
// so the tests can compare each with brute force.  Built into
// libpso_prims.so; test infrastructure only.
//
// Every entry point takes and returns host arrays, allocates and frees its
// own device memory, synchronises, and returns 0 or a negative HIP error.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>

#include "pso_aggregate.hpp"

using namespace pso;

namespace {

__global__ void k_make_key(const float *f, const uint32_t *idx, unsigned long long *out, uint32_t n)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = make_key(f[i], idx[i]);
}

// Each wavefront reduces its 64 values; every lane writes what it holds.
__global__ void k_wave_min(const unsigned long long *in, unsigned long long *out)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    out[i] = wave_min_u64(in[i]);
}

// Each workgroup: workgroup_min of its lanes' keys against its threshold;
// every lane writes the result it returns.
__global__ void k_group_min(const unsigned long long *keys, const unsigned long long *thr, unsigned long long *out)
{
    __shared__ unsigned long long slot;
    if (threadIdx.x == 0) slot = NO_KEY;
    __syncthreads();
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    out[i] = workgroup_min(keys[i], thr[blockIdx.x], &slot);
}

__global__ void k_ctrl_reset(Ctrl *c, unsigned long long gkey)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        c->gkey = gkey;
        c->seq = 0;
        c->lock = 0;
        c->pubkey = NO_KEY;
        c->err = 0;
    }
}

// Each workgroup publishes its key (synchronous rule) against threshold thr.
__global__ void k_publish_sync(const unsigned long long *wg_keys, Ctrl *c, unsigned long long thr)
{
    publish_sync(c, wg_keys[blockIdx.x], thr);
}

// Seqlock stress.  Workgroups [0, writers) publish `rounds` keys each
// through publish_async: writer w's r-th key has fitness order bits
// HI - (r * writers + w) (later rounds lower) and index gi = r * writers + w,
// so each publish that wins copies column gi of x into gpos.  Column gi of x
// holds pattern(gi, d) = gi * 4096 + d (exact in binary32 for the sizes
// used); they start once every reader has started and pause `gap` sleeps of
// 127 x 64 cycles after each publish.  Workgroups
// [writers, writers + readers) take snapshot_async
// snapshots until every writer is done (or `max_snaps` each) and count the
// snapshots whose position is not the published key's column (torn), the
// snapshots taken, and those that saw a key different from their previous
// one.  Every loop is bounded.
constexpr uint32_t STRESS_HI = 0x90000000u;

__global__ void k_seqlock_stress(SwarmArgs a, uint32_t writers, uint32_t rounds, uint32_t gap, uint32_t max_snaps,
                                 unsigned int *done, unsigned int *started, unsigned int *stats)
{
    extern __shared__ float s_g[];
    __shared__ unsigned long long s_key;
    __shared__ int flag;
    __shared__ unsigned int s_bad, s_changes, s_last_done;
    if (blockIdx.x < writers) {
        const uint32_t w = blockIdx.x;
        // start once every reader runs, so publishes overlap snapshots (a
        // bounded wait: on timeout the writer starts anyway and the test's
        // overlap check fails instead of the kernel hanging)
        if (threadIdx.x == 0) {
            for (uint32_t spins = 0; spins < (1u << 20); ++spins) {
                if (__hip_atomic_load(started, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= gridDim.x - writers) break;
                __builtin_amdgcn_s_sleep(2);
            }
        }
        __syncthreads();
        for (uint32_t r = 0; r < rounds; ++r) {
            const uint32_t gi = r * writers + w;
            const unsigned long long m = ((unsigned long long)(STRESS_HI - gi) << 32) | gi;
            publish_async(a, m, NO_KEY, &flag);
            __syncthreads();
            // a pause of `gap` sleeps between publishes: a snapshot of a wide
            // position needs a window without a publish to complete
            for (uint32_t k = 0; k < gap; ++k) __builtin_amdgcn_s_sleep(127);
        }
        if (threadIdx.x == 0) {
            __threadfence();
            atomicAdd(done, 1u);
        }
        return;
    }
    if (threadIdx.x == 0) {
        s_bad = 0;
        s_changes = 0;
        s_last_done = 0;
        atomicAdd(started, 1u);
    }
    __syncthreads();
    unsigned long long prev = NO_KEY;
    uint32_t snaps = 0;
    while (snaps < max_snaps) {
        const unsigned long long k = snapshot_async(a, s_g, &s_key); // ends with a barrier
        ++snaps;
        uint32_t bad = 0;
        if (k != NO_KEY) {
            const uint32_t gi = (uint32_t)k;
            for (int d = threadIdx.x; d < a.D; d += blockDim.x)
                bad += s_g[d] != (float)(gi * 4096u + (uint32_t)d);
        }
        if (bad) atomicAdd(&s_bad, bad);
        if (threadIdx.x == 0) {
            if (k != prev) ++s_changes;
            s_last_done = __hip_atomic_load(done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        prev = k;
        __syncthreads();
        const bool finished = s_last_done >= writers;
        __syncthreads();
        if (finished) break;
    }
    if (threadIdx.x == 0) {
        atomicAdd(&stats[0], s_bad);
        atomicAdd(&stats[1], snaps);
        atomicAdd(&stats[2], s_changes);
    }
}

// VALU throughput of the random-number generator: each lane draws `calls`
// Philox4x32-10 blocks, four independent ones at a time (as a step kernel
// draws one per particle of its quad), with the counters the step kernels
// use -- (pair j, particle `lane`, iteration 0, velocity tag) under key
// (k0, k1) -- and folds every output word into a running XOR, so no draw is
// dead code; out[lane] receives the XOR.
__global__ void __launch_bounds__(256) k_philox_rate(uint32_t k0, uint32_t k1, uint32_t calls, uint32_t *out)
{
    const uint32_t lane = blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t acc = 0;
    for (uint32_t j = 0; j < calls; j += 4) {
        U4 u[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) u[k] = philox4x32_10(k0, k1, j + (uint32_t)k, lane, 0u, TAG_VEL);
#pragma unroll
        for (int k = 0; k < 4; ++k) acc ^= u[k].a ^ u[k].b ^ u[k].c ^ u[k].d;
    }
    out[lane] = acc;
}

template <class T>
hipError_t upload(T **d, const T *h, size_t n)
{
    hipError_t e = hipMalloc(reinterpret_cast<void **>(d), sizeof(T) * (n ? n : 1));
    if (e == hipSuccess && n) e = hipMemcpy(*d, h, sizeof(T) * n, hipMemcpyHostToDevice);
    return e;
}

} // namespace

#define TRY(expr)                              \
    do {                                       \
        hipError_t e_ = (expr);                \
        if (e_ != hipSuccess) {                \
            rc = -(int)e_;                     \
            goto out;                          \
        }                                      \
    } while (0)

extern "C" {

// out[i] = make_key(f[i], idx[i]) for i < n.
int prim_make_key(const float *f, const uint32_t *idx, int64_t n, uint64_t *out)
{
    int rc = 0;
    float *df = nullptr;
    uint32_t *di = nullptr;
    unsigned long long *dout = nullptr;
    TRY(upload(&df, f, n));
    TRY(upload(&di, idx, n));
    TRY(hipMalloc(&dout, sizeof(uint64_t) * (n ? n : 1)));
    hipLaunchKernelGGL(k_make_key, dim3((uint32_t)((n + 255) / 256)), dim3(256), 0, 0, df, di, dout, (uint32_t)n);
    TRY(hipGetLastError());
    TRY(hipMemcpy(out, dout, sizeof(uint64_t) * n, hipMemcpyDeviceToHost));
out:
    (void)hipFree(df);
    (void)hipFree(di);
    (void)hipFree(dout);
    return rc;
}

// in: n_waves * 64 values; out: what every lane holds after wave_min_u64.
int prim_wave_min(const uint64_t *in, int64_t n_waves, uint64_t *out)
{
    int rc = 0;
    const size_t n = (size_t)n_waves * 64;
    unsigned long long *din = nullptr, *dout = nullptr;
    TRY(upload(&din, reinterpret_cast<const unsigned long long *>(in), n));
    TRY(hipMalloc(&dout, sizeof(uint64_t) * n));
    hipLaunchKernelGGL(k_wave_min, dim3((uint32_t)n_waves), dim3(64), 0, 0, din, dout);
    TRY(hipGetLastError());
    TRY(hipMemcpy(out, dout, sizeof(uint64_t) * n, hipMemcpyDeviceToHost));
out:
    (void)hipFree(din);
    (void)hipFree(dout);
    return rc;
}

// keys: groups * lanes values, thr: one threshold per group (lanes 64, 128,
// 256, 512 or 1024); out: what every lane's workgroup_min returned.
int prim_group_min(const uint64_t *keys, const uint64_t *thr, int64_t groups, int lanes, uint64_t *out)
{
    if (lanes != 64 && lanes != 128 && lanes != 256 && lanes != 512 && lanes != 1024) return -1;
    int rc = 0;
    const size_t n = (size_t)groups * lanes;
    unsigned long long *dk = nullptr, *dt = nullptr, *dout = nullptr;
    TRY(upload(&dk, reinterpret_cast<const unsigned long long *>(keys), n));
    TRY(upload(&dt, reinterpret_cast<const unsigned long long *>(thr), (size_t)groups));
    TRY(hipMalloc(&dout, sizeof(uint64_t) * n));
    hipLaunchKernelGGL(k_group_min, dim3((uint32_t)groups), dim3(lanes), 0, 0, dk, dt, dout);
    TRY(hipGetLastError());
    TRY(hipMemcpy(out, dout, sizeof(uint64_t) * n, hipMemcpyDeviceToHost));
out:
    (void)hipFree(dk);
    (void)hipFree(dt);
    (void)hipFree(dout);
    return rc;
}

// k_philox_rate over `lanes` lanes (a multiple of 256) and `calls` draws per
// lane (a multiple of 4): out (lanes words) receives each lane's XOR and
// *ms the kernel's time from HIP events (after one untimed launch).
int prim_philox_rate(uint32_t k0, uint32_t k1, uint32_t calls, int64_t lanes, uint32_t *out, float *ms)
{
    if (lanes < 256 || lanes % 256 != 0 || lanes > (1ll << 24) || calls < 4 || calls % 4 != 0) return -1;
    int rc = 0;
    uint32_t *dout = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    TRY(hipMalloc(&dout, sizeof(uint32_t) * (size_t)lanes));
    TRY(hipEventCreate(&e0));
    TRY(hipEventCreate(&e1));
    hipLaunchKernelGGL(k_philox_rate, dim3((uint32_t)(lanes / 256)), dim3(256), 0, 0, k0, k1, calls, dout);
    TRY(hipGetLastError());
    TRY(hipEventRecord(e0, 0));
    hipLaunchKernelGGL(k_philox_rate, dim3((uint32_t)(lanes / 256)), dim3(256), 0, 0, k0, k1, calls, dout);
    TRY(hipGetLastError());
    TRY(hipEventRecord(e1, 0));
    TRY(hipEventSynchronize(e1));
    TRY(hipEventElapsedTime(ms, e0, e1));
    TRY(hipMemcpy(out, dout, sizeof(uint32_t) * (size_t)lanes, hipMemcpyDeviceToHost));
out:
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipFree(dout);
    return rc;
}

// One workgroup per key publishes it with publish_sync against thr, starting
// from device key `init`; *gkey_out receives the device key afterwards.
int prim_publish_sync(const uint64_t *wg_keys, int64_t groups, uint64_t thr, uint64_t init, uint64_t *gkey_out)
{
    int rc = 0;
    unsigned long long *dk = nullptr;
    Ctrl *c = nullptr;
    TRY(upload(&dk, reinterpret_cast<const unsigned long long *>(wg_keys), (size_t)groups));
    TRY(hipMalloc(&c, sizeof(Ctrl)));
    hipLaunchKernelGGL(k_ctrl_reset, dim3(1), dim3(64), 0, 0, c, (unsigned long long)init);
    hipLaunchKernelGGL(k_publish_sync, dim3((uint32_t)groups), dim3(256), 0, 0, dk, c, (unsigned long long)thr);
    TRY(hipGetLastError());
    TRY(hipMemcpy(gkey_out, &c->gkey, sizeof(uint64_t), hipMemcpyDeviceToHost));
out:
    (void)hipFree(dk);
    (void)hipFree(c);
    return rc;
}

// Seqlock stress (k_seqlock_stress) over a D-float position: stats[0] torn
// elements seen, stats[1] snapshots, stats[2] snapshots whose key differed
// from the reader's previous one, stats[3] the control block's error bits,
// stats[4] writers done; *final_key the published key at the end and
// final_pos (D floats) the published position.
int prim_seqlock_stress(int D, int writers, int readers, int rounds, int gap, int max_snaps, uint32_t *stats,
                        uint64_t *final_key, float *final_pos)
{
    if (D < 1 || D > 4096 || writers < 1 || readers < 0 || rounds < 1 || gap < 0 || gap > 1000 || max_snaps < 1)
        return -1;
    if ((uint64_t)writers * rounds * 4096ull + (uint64_t)D > (1ull << 24)) return -1; // patterns exact in binary32
    int rc = 0;
    const uint64_t np = ((uint64_t)writers * rounds + 63) / 64 * 64;
    float *x = nullptr, *gpos = nullptr, *hx = nullptr;
    Ctrl *c = nullptr;
    unsigned int *done = nullptr, *started = nullptr, *dstats = nullptr;
    SwarmArgs a{};
    hx = static_cast<float *>(std::malloc(sizeof(float) * np * D));
    if (!hx) return -2;
    for (int d = 0; d < D; ++d)
        for (uint64_t i = 0; i < np; ++i) hx[(size_t)d * np + i] = (float)(uint32_t)(i * 4096u + (uint32_t)d);
    TRY(upload(&x, hx, np * D));
    TRY(hipMalloc(&gpos, sizeof(float) * D));
    TRY(hipMemset(gpos, 0, sizeof(float) * D));
    TRY(hipMalloc(&c, sizeof(Ctrl)));
    TRY(hipMalloc(&done, sizeof(unsigned int)));
    TRY(hipMemset(done, 0, sizeof(unsigned int)));
    TRY(hipMalloc(&started, sizeof(unsigned int)));
    TRY(hipMemset(started, 0, sizeof(unsigned int)));
    TRY(hipMalloc(&dstats, sizeof(unsigned int) * 3));
    TRY(hipMemset(dstats, 0, sizeof(unsigned int) * 3));
    a.x = x;
    a.gpos = gpos;
    a.ctrl = c;
    a.N = (uint32_t)np;
    a.Np = (uint32_t)np;
    a.D = D;
    hipLaunchKernelGGL(k_ctrl_reset, dim3(1), dim3(64), 0, 0, c, NO_KEY);
    hipLaunchKernelGGL(k_seqlock_stress, dim3((uint32_t)(writers + readers)), dim3(256), sizeof(float) * D, 0, a,
                       (uint32_t)writers, (uint32_t)rounds, (uint32_t)gap, (uint32_t)max_snaps, done, started, dstats);
    TRY(hipGetLastError());
    TRY(hipDeviceSynchronize());
    TRY(hipMemcpy(stats, dstats, sizeof(unsigned int) * 3, hipMemcpyDeviceToHost));
    TRY(hipMemcpy(&stats[3], &c->err, sizeof(unsigned int), hipMemcpyDeviceToHost));
    TRY(hipMemcpy(&stats[4], done, sizeof(unsigned int), hipMemcpyDeviceToHost));
    TRY(hipMemcpy(final_key, &c->pubkey, sizeof(uint64_t), hipMemcpyDeviceToHost));
    TRY(hipMemcpy(final_pos, gpos, sizeof(float) * D, hipMemcpyDeviceToHost));
out:
    std::free(hx);
    (void)hipFree(x);
    (void)hipFree(gpos);
    (void)hipFree(c);
    (void)hipFree(done);
    (void)hipFree(started);
    (void)hipFree(dstats);
    return rc;
}

} // extern "C"

// pso_aggregate.hpp -- aggregation of the particles' pbest keys into the
// swarm's gbest (Alg. 1 Step 5), shared by every kernel that ends an
// iteration over a workgroup's particles.  The paper's queue (Sec. 3.1,
// Alg. 2) keeps the threads whose fitness beats the gbest and lets one thread
// scan them; its lock-protected form (Sec. 3.2, Alg. 3) folds each block's
// result into the global one under a spin lock.  Here:
//   - workgroup_min: a lane is a candidate only if its key beats the
//     threshold (the gbest key); a wavefront with a candidate takes the
//     minimum by a butterfly over lanes (wave_min_u64), and one lane folds it
//     into an LDS cell with a 64-bit atomicMin;
//   - publish_sync: one device-scope 64-bit atomicMin of the packed
//     (fitness, index) key per workgroup whose minimum can still win;
//   - publish_async / snapshot_async: the asynchronous variant's gbest
//     position, written under a lock and a sequence counter (seqlock) and
//     read as a consistent (key, position) snapshot.
// Every wait is bounded by SPIN_LIMIT; a wait that gives up sets an error
// bit in the control block.
#pragma once

#include "pso_device.hpp"
#include "pso_kernels.hpp"

namespace pso {

constexpr unsigned int SPIN_LIMIT = 1u << 22; // bound on every wait loop

// ---------------------------------------------------------------------------
// Workgroup minimum of the candidate keys (key < thr): butterfly minimum in
// each wavefront that has a candidate, then one LDS atomicMin per such
// wavefront.  *wg_min must hold NO_KEY before the call; ends with a
// barrier and returns the minimum (NO_KEY if none) in every lane.
// ---------------------------------------------------------------------------
__device__ __forceinline__ unsigned long long workgroup_min(unsigned long long key, unsigned long long thr,
                                                            unsigned long long *wg_min)
{
    const bool cand = key < thr;
    if (__ballot(cand)) {
        const unsigned long long m = wave_min_u64(cand ? key : NO_KEY);
        if ((threadIdx.x & 63) == 0) atomicMin(wg_min, m);
    }
    __syncthreads();
    return *wg_min;
}

// Adds the workgroup's pbest improvements to the control block's counter
// (wavefront sums, one LDS add per wavefront, one device add per workgroup;
// the device add happens after the barrier in workgroup_min).
__device__ __forceinline__ void count_improvements(Ctrl *c, uint32_t n, unsigned int *wg_count)
{
    uint32_t s = n;
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off, 64);
    if ((threadIdx.x & 63) == 0 && s) atomicAdd(wg_count, s);
}

__device__ __forceinline__ void flush_count(Ctrl *c, const unsigned int *wg_count)
{
    if (threadIdx.x == 0 && *wg_count) atomicAdd(&c->improved, (unsigned long long)*wg_count);
}

// Arrival count: true in every lane of the last workgroup of the launch,
// after an acquire fence.
// Lane 0 alone fences: the barrier orders the other lanes' later loads
// after its acquire.
__device__ __forceinline__ bool arrive_last(Ctrl *c, int *last_flag)
{
    if (threadIdx.x == 0) {
        const unsigned int ticket = atomicAdd(&c->arrive, 1u);
        const int last = (ticket == gridDim.x - 1);
        if (last) __threadfence(); // acquire every workgroup's results
        *last_flag = last;
    }
    __syncthreads();
    return *last_flag != 0;
}

// Synchronous aggregation: the workgroup minimum goes to the global key.
// Called after the barrier that ends workgroup_min, so every lane's x stores
// precede lane 0's release fence at workgroup scope; one agent-scope fence
// per workgroup then publishes them all (a fence per wavefront costs ~5 us
// per iteration at 1024 workgroups).  A candidate already beaten by the
// running global key cannot win and is not published (keys are unique).
__device__ __forceinline__ void publish_sync(Ctrl *c, unsigned long long m, unsigned long long thr)
{
    if (m < thr && threadIdx.x == 0 &&
        m < __hip_atomic_load(&c->gkey, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
        __threadfence(); // release this workgroup's stores (the winner's x)
        atomicMin(&c->gkey, m);
        __threadfence(); // the minimum precedes the arrival
    }
}

// Asynchronous aggregation: a workgroup whose minimum lowers the global key
// publishes the winner's position (x of particle m & 0xffffffff, just stored
// by this workgroup) under the seqlock, unless a better key arrived first.
// Every wait is bounded; a wait that gives up sets an error bit.
__device__ void publish_async(const SwarmArgs &a, unsigned long long m, unsigned long long thr, int *pub_flag)
{
    Ctrl *c = a.ctrl;
    if (!(m < thr)) return; // uniform: m and thr are the same in every lane
    if (threadIdx.x == 0) {
        int pub = 0;
        const unsigned long long old = atomicMin(&c->gkey, m);
        if (m < old) {
            unsigned int spins = 0;
            bool locked = false;
            while (!(locked = (atomicCAS(&c->lock, 0u, 1u) == 0u)) && ++spins < SPIN_LIMIT)
                __builtin_amdgcn_s_sleep(2);
            if (!locked) {
                atomicOr(&c->err, ERR_SEQLOCK_SPIN);
            } else {
                __threadfence();
                const unsigned long long cur = __hip_atomic_load(&c->gkey, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                const unsigned long long pk = __hip_atomic_load(&c->pubkey, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if (cur == m && m < pk) {
                    const unsigned int s = __hip_atomic_load(&c->seq, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    __hip_atomic_store(&c->seq, s + 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); // odd: writing
                    __threadfence();
                    pub = 1;
                } else {
                    __hip_atomic_store(&c->lock, 0u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
                }
            }
        }
        *pub_flag = pub;
    }
    __syncthreads();
    if (*pub_flag) {
        const size_t gi = (uint32_t)m;
        for (int d = threadIdx.x; d < a.D; d += (int)blockDim.x)
            __hip_atomic_store(&a.gpos[d], a.x[(size_t)d * a.Np + gi], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __syncthreads();
        if (threadIdx.x == 0) {
            // one release fence for the workgroup, as in publish_sync: the
            // barrier orders every lane's position stores before it (a fence
            // per wavefront writes the L2 back once per wavefront)
            __threadfence();
            __hip_atomic_store(&c->pubkey, m, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            const unsigned int s = __hip_atomic_load(&c->seq, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&c->seq, s + 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT); // even: done
            __hip_atomic_store(&c->lock, 0u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

// Consistent copy of (published key, gbest position) into LDS, read by the
// first wavefront under the seqlock; returns the key in every lane.  The wait
// is bounded; giving up sets an error bit.
__device__ unsigned long long snapshot_async(const SwarmArgs &a, float *s_g, unsigned long long *s_key)
{
    Ctrl *c = a.ctrl;
    if (threadIdx.x < 64) {
        unsigned long long key = NO_KEY;
        for (unsigned int spins = 0;; ++spins) {
            const unsigned int s1 = __hip_atomic_load(&c->seq, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
            if (!(s1 & 1u)) {
                key = __hip_atomic_load(&c->pubkey, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                for (int d = threadIdx.x; d < a.D; d += 64)
                    s_g[d] = __hip_atomic_load(&a.gpos[d], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __atomic_thread_fence(__ATOMIC_ACQUIRE);
                const unsigned int s2 = __hip_atomic_load(&c->seq, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if (s1 == s2) break;
            }
            if (spins + 1 == SPIN_LIMIT) {
                if (threadIdx.x == 0) atomicOr(&c->err, ERR_SEQLOCK_SPIN);
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
        if (threadIdx.x == 0) *s_key = key;
    }
    __syncthreads();
    return *s_key;
}

} // namespace pso

// pso_block.hip -- one workgroup runs one whole swarm (Step 1 and all its
// iterations) with workgroup barriers only.
//
// For a swarm small enough for one compute unit, a launch per iteration
// costs more than the iteration itself, and the paper's answer -- removing
// the second kernel (Sec. 3.2) -- still leaves one launch per iteration.
// Here the iteration loop runs inside the workgroup: the gbest minimum is a
// wavefront butterfly plus an LDS atomicMin, the gbest position lives in LDS,
// and the state stays in the same per-swarm layout as the grid kernels (it is
// cache-resident for small swarms).  The per-particle work is the same
// init_quad / iterate_quad as the grid kernels, so a swarm computes the same
// bits whichever kernel runs it.
//
// The batched kernel is persistent: each workgroup takes the next swarm from
// an atomic work counter (swarms are queued largest first), runs it to its
// iteration limit or stop rule, writes the result, and takes the next; every
// workgroup exits when the counter passes the swarm count.
#include "pso_block.hpp"
#include "pso_quad.hpp"

#ifndef PSO_BLOCK_SWARM
#define PSO_BLOCK_SWARM 256 // lanes of a swarm-owning workgroup
#endif

namespace pso {

constexpr int BLOCK_SWARM = PSO_BLOCK_SWARM;

// Per-swarm loop state, identical in every lane.
struct SwarmLoop {
    unsigned long long gkey; // gbest key
    long long giter;         // iteration of the last gbest change
    long long t;             // iterations completed
    bool stop;
    uint32_t improved;       // this lane's pbest improvements (block_iterate)
};

__device__ __forceinline__ bool meets_tol(unsigned long long key, float tol, float fstar)
{
    return tol > 0.0f && __builtin_fabsf(key_fitness(key) - fstar) < tol;
}

// Workgroup minimum of candidate keys (key < thr) into *slot (NO_KEY before
// the call); ends with a barrier and returns the minimum in every lane.
__device__ __forceinline__ unsigned long long block_min(unsigned long long key, unsigned long long thr,
                                                        unsigned long long *slot)
{
    const bool cand = key < thr;
    if (__ballot(cand)) {
        const unsigned long long m = wave_min_u64(cand ? key : NO_KEY);
        if ((threadIdx.x & 63) == 0) atomicMin(slot, m);
    }
    __syncthreads();
    return *slot;
}

// gbest position <- x of particle gi, stored by a lane of this workgroup
// before the last barrier (one compute unit: its L1 serves every lane).
__device__ __forceinline__ void gather_gbest(const SwarmArgs &a, int D, uint32_t gi, float *s_g)
{
    for (int d = threadIdx.x; d < D; d += BLOCK_SWARM) s_g[d] = a.x[(size_t)d * a.Np + gi];
}

// Step 1 by one workgroup; leaves the gbest position in s_g.
template <int FIT>
__device__ void block_init(const SwarmArgs &a, const float *s_shift, float *s_g, unsigned long long *s_min,
                           SwarmLoop &L)
{
    const int D = a.D;
    unsigned long long key = NO_KEY;
    for (uint32_t q = threadIdx.x; 4 * q < a.Np; q += BLOCK_SWARM) {
        const unsigned long long k = init_quad<FIT>(a, D, q, s_shift);
        key = k < key ? k : key;
    }
    const unsigned long long m = block_min(key, NO_KEY, &s_min[0]);
    if (threadIdx.x == 0) s_min[1] = NO_KEY;
    gather_gbest(a, D, (uint32_t)m, s_g);
    L.gkey = m;
    L.giter = 0;
    L.t = 0;
    __syncthreads();
}

// Up to T iterations after L.t, stopping after the first iteration at which
// the stop rule holds (it is tested before the first one too).  s_min[2]
// alternates between iterations: slot (t & 1) collects iteration t's
// minimum, and the other slot is cleared for iteration t+1.  hist (may be
// null) receives each iteration's gbest key.
template <int FIT>
__device__ void block_iterate(const SwarmArgs &a, long long T, float tol, float fstar, const float *s_shift,
                              float *s_g, unsigned long long *s_min, unsigned long long *hist, SwarmLoop &L)
{
    uint32_t n_imp = 0; // this lane's pbest improvements over the run
    const int D = a.D;
    L.stop = L.stop || meets_tol(L.gkey, tol, fstar);
    for (long long it = 0; it < T && !L.stop; ++it) {
        const uint32_t t = (uint32_t)(L.t + 1);
        unsigned long long key = NO_KEY;
        for (uint32_t q = threadIdx.x; 4 * q < a.N; q += BLOCK_SWARM) {
            uint32_t n = 0;
            const unsigned long long k = iterate_quad<FIT, 0, 1>(a, D, q, t, s_g, s_shift, &n);
            key = k < key ? k : key;
            n_imp += n;
        }
        unsigned long long *slot = &s_min[t & 1];
        const unsigned long long m = block_min(key, L.gkey, slot);
        if (threadIdx.x == 0) s_min[(t + 1) & 1] = NO_KEY;
        if (m < L.gkey) {
            L.gkey = m;
            L.giter = t;
            gather_gbest(a, D, (uint32_t)m, s_g);
        }
        if (hist && threadIdx.x == 0) hist[t & (HIST_CAP - 1)] = L.gkey;
        L.t = t;
        L.stop = meets_tol(L.gkey, tol, fstar);
        __syncthreads();
    }
    L.improved = n_imp;
}

// ---------------------------------------------------------------------------
// A single swarm's run (the pso_run path for small swarms): continues from the
// control block's state for up to T iterations with its stop rule.
// ---------------------------------------------------------------------------
template <int FIT>
__global__ void __launch_bounds__(BLOCK_SWARM) k_block_run(SwarmArgs a, long long T)
{
    __shared__ unsigned long long s_min[2];
    extern __shared__ float s_dyn[]; // gbest position (D), shift (D)
    Ctrl *c = a.ctrl;
    const int D = a.D;
    float *s_g = s_dyn, *s_shift = s_dyn + D;
    for (int d = threadIdx.x; d < D; d += BLOCK_SWARM) {
        s_g[d] = a.gpos[d];
        s_shift[d] = a.shift[d];
    }
    if (threadIdx.x == 0) {
        s_min[0] = NO_KEY;
        s_min[1] = NO_KEY;
    }
    SwarmLoop L;
    L.gkey = c->gkey_prev;
    L.giter = c->giter;
    L.t = c->t;
    L.stop = c->stop != 0u;
    const float tol = c->tol, fstar = c->fstar;
    __syncthreads();
    block_iterate<FIT>(a, T, tol, fstar, s_shift, s_g, s_min, a.hist, L);
    if (L.improved) atomicAdd(&c->improved, (unsigned long long)L.improved);
    for (int d = threadIdx.x; d < D; d += BLOCK_SWARM) a.gpos[d] = s_g[d];
    if (threadIdx.x == 0) {
        c->gkey = L.gkey;
        c->gkey_prev = L.gkey;
        c->pubkey = L.gkey;
        c->giter = L.giter;
        c->t = L.t;
        c->stop = L.stop ? 1u : 0u;
    }
}

// ---------------------------------------------------------------------------
// Batched: many independent swarms in one persistent launch.  Each launch
// runs up to `chunk` iterations of every listed swarm and leaves its loop
// state (BatchResult) and gbest position in device memory, so a later launch
// resumes it exactly where it stopped: a swarm computes the same bits however
// its iterations are split over launches.
// ---------------------------------------------------------------------------
__global__ void k_batch_reset(BatchResult *results, uint32_t count, unsigned int *next)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) *next = 0u;
    if (i < count) {
        results[i].gkey = NO_KEY;
        results[i].giter = 0;
        results[i].iters = 0;
        results[i].started = 0;
        results[i].stop = 0;
    }
}

__global__ void k_counter_reset(unsigned int *next)
{
    if (threadIdx.x == 0) *next = 0u;
}

template <int FIT>
__device__ void batch_one(const BatchItem &it, BatchResult *res, long long chunk, float *s_g, float *s_shift,
                          unsigned long long *s_min)
{
    const SwarmArgs &a = it.a;
    const int D = a.D;
    for (int d = threadIdx.x; d < D; d += BLOCK_SWARM) s_shift[d] = a.shift[d];
    if (threadIdx.x == 0) {
        s_min[0] = NO_KEY;
        s_min[1] = NO_KEY;
    }
    SwarmLoop L;
    const bool started = res->started != 0u;
    __syncthreads();
    if (!started) {
        L.stop = false;
        block_init<FIT>(a, s_shift, s_g, s_min, L);
    } else {
        L.gkey = res->gkey;
        L.giter = res->giter;
        L.t = res->iters;
        L.stop = res->stop != 0u;
        for (int d = threadIdx.x; d < D; d += BLOCK_SWARM) s_g[d] = a.gpos[d];
        __syncthreads();
    }
    // iterations this launch: about `chunk` particle-dimension updates' worth
    // (at least one), so every swarm of a launch takes a similar time
    const long long left = it.max_iter - L.t;
    const long long nd = (long long)a.N * a.D;
    long long iters = chunk / nd;
    iters = iters < 1 ? 1 : iters;
    block_iterate<FIT>(a, left < iters ? left : iters, it.tol, it.fstar, s_shift, s_g, s_min, nullptr, L);
    for (int d = threadIdx.x; d < D; d += BLOCK_SWARM) a.gpos[d] = s_g[d];
    if (threadIdx.x == 0) {
        res->gkey = L.gkey;
        res->giter = L.giter;
        res->iters = L.t;
        res->stop = L.stop ? 1u : 0u;
        res->started = 1u;
    }
}

__global__ void __launch_bounds__(BLOCK_SWARM) k_batch(const BatchItem *items, const uint32_t *order,
                                                       BatchResult *results, uint32_t count, unsigned int *next,
                                                       long long chunk, BatchResult *out_state, float *out_pos,
                                                       int pos_stride)
{
    __shared__ unsigned long long s_min[2];
    __shared__ uint32_t s_idx;
    extern __shared__ float s_dyn[]; // gbest position (maxD floats), then shift
    for (;;) {
        if (threadIdx.x == 0) s_idx = atomicAdd(next, 1u);
        __syncthreads();
        const uint32_t j = s_idx;
        __syncthreads();
        if (j >= count) break; // uniform: every workgroup leaves once the list is drained
        const uint32_t idx = order[j];
        const BatchItem &it = items[idx];
        float *s_g = s_dyn, *s_shift = s_dyn + it.a.D;
        switch (it.fitness) {
        case F_SPHERE: batch_one<F_SPHERE>(it, &results[idx], chunk, s_g, s_shift, s_min); break;
        case F_RASTRIGIN: batch_one<F_RASTRIGIN>(it, &results[idx], chunk, s_g, s_shift, s_min); break;
        case F_ROSENBROCK: batch_one<F_ROSENBROCK>(it, &results[idx], chunk, s_g, s_shift, s_min); break;
        case F_ACKLEY: batch_one<F_ACKLEY>(it, &results[idx], chunk, s_g, s_shift, s_min); break;
        default: batch_one<F_CUBIC>(it, &results[idx], chunk, s_g, s_shift, s_min); break;
        }
        __syncthreads();
        if (out_state && threadIdx.x == 0) out_state[j] = results[idx];
        if (out_pos)
            for (int d = threadIdx.x; d < it.a.D; d += BLOCK_SWARM) out_pos[(size_t)j * pos_stride + d] = s_g[d];
    }
}

// ---------------------------------------------------------------------------
// Launchers.
// ---------------------------------------------------------------------------
hipError_t launch_block_run(int fitness, const SwarmArgs &a, long long T, hipStream_t stream)
{
    const size_t lds = 2 * sizeof(float) * a.D;
    switch (fitness) {
    case F_SPHERE: hipLaunchKernelGGL(k_block_run<F_SPHERE>, dim3(1), dim3(BLOCK_SWARM), lds, stream, a, T); break;
    case F_RASTRIGIN: hipLaunchKernelGGL(k_block_run<F_RASTRIGIN>, dim3(1), dim3(BLOCK_SWARM), lds, stream, a, T); break;
    case F_ROSENBROCK: hipLaunchKernelGGL(k_block_run<F_ROSENBROCK>, dim3(1), dim3(BLOCK_SWARM), lds, stream, a, T); break;
    case F_ACKLEY: hipLaunchKernelGGL(k_block_run<F_ACKLEY>, dim3(1), dim3(BLOCK_SWARM), lds, stream, a, T); break;
    case F_CUBIC: hipLaunchKernelGGL(k_block_run<F_CUBIC>, dim3(1), dim3(BLOCK_SWARM), lds, stream, a, T); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

int batch_block_lanes() { return BLOCK_SWARM; }

hipError_t launch_batch_reset(BatchResult *results, uint32_t count, unsigned int *next, hipStream_t stream)
{
    hipLaunchKernelGGL(k_batch_reset, dim3((count + 255) / 256), dim3(256), 0, stream, results, count, next);
    return hipGetLastError();
}

hipError_t launch_batch(const BatchItem *items, const uint32_t *order, BatchResult *results, uint32_t count,
                        unsigned int *next, int maxD, int grid, long long chunk, hipStream_t stream,
                        BatchResult *out_state, float *out_pos)
{
    hipLaunchKernelGGL(k_counter_reset, dim3(1), dim3(64), 0, stream, next);
    const size_t lds = 2 * sizeof(float) * maxD;
    hipLaunchKernelGGL(k_batch, dim3(grid), dim3(BLOCK_SWARM), lds, stream, items, order, results, count, next,
                       chunk, out_state, out_pos, maxD);
    return hipGetLastError();
}

hipError_t batch_occupancy(int maxD, int *blocks_per_cu)
{
    const size_t lds = 2 * sizeof(float) * maxD;
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k_batch, BLOCK_SWARM, lds);
}

} // namespace pso

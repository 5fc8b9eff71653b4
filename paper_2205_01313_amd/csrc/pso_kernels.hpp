// pso_kernels.hpp -- device state of one swarm and the launchers of its
// kernels (host side of the kernels in pso_kernels.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace pso {

constexpr int HIST_CAP = 8192; // gbest keys kept per swarm (ring, power of two)

// Control block of a swarm in device memory.  The fields that workgroups
// update atomically sit on their own 256-byte lines.
struct alignas(256) Ctrl {
    // line 0: running minimum key of the current iteration (atomicMin target)
    unsigned long long gkey;
    unsigned long long improved; // pbest improvements since Step 1 (one add per workgroup)
    // asynchronous step: tiles run since Step 1, and those that used a gbest
    // published during the same iteration
    unsigned long long tiles, fresh;
    unsigned char pad0[224];
    // line 1: workgroups that finished the current launch
    unsigned int arrive;
    unsigned char pad1[252];
    // line 2: bookkeeping, written by the last workgroup of each launch
    unsigned long long gkey_prev; // gbest key after the previous iteration
    long long giter;              // iteration at which the gbest last changed
    long long t;                  // iterations completed
    long long t_run0;             // t when the current pso_run began
    unsigned int stop;            // 1 once the stop rule of the current run holds
    unsigned int err;             // device-detected error bits
    float tol, fstar;             // stop rule |gbest - fstar| < tol (tol <= 0: off)
    unsigned char pad2[208];
    // line 3: asynchronous variant -- seqlock over gpos
    unsigned int seq;             // odd while a workgroup rewrites gpos
    unsigned int lock;            // publisher lock
    unsigned long long pubkey;    // key whose position gpos holds
    unsigned char pad3[240];
};
static_assert(sizeof(Ctrl) == 1024, "Ctrl layout");

constexpr unsigned int ERR_SEQLOCK_SPIN = 1u; // a seqlock wait gave up
constexpr unsigned int ERR_STALE_WAIT = 2u;   // a bounded-staleness wait gave up
constexpr unsigned int ERR_GANG_WAIT = 4u;    // a gang part waited past the time bound

// Aggregation variants (values of PSO_SYNC / PSO_ASYNC / PSO_REDUCE /
// PSO_REDUCE_UNROLLED in pso.h).
constexpr int VAR_SYNC = 0;
constexpr int VAR_ASYNC = 1;
constexpr int VAR_REDUCE = 2;
constexpr int VAR_REDUCE_UNROLLED = 3;
constexpr int VAR_PERSISTENT = 4;

// Workgroups of a persistent run hold their iteration counts here.
constexpr uint32_t PERSIST_MAX_GRID = 8192;

// Device pointers and parameters of one swarm, passed by value to kernels
// (the kernel-argument segment is read through the scalar cache, the role
// constant memory plays in Sec. 4.2).
struct SwarmArgs {
    float *x, *v, *p, *pf;      // D*Np, D*Np, D*Np, Np; element (d, i) at d*Np + i
    uint8_t *pend;              // Np: 1 = pbest position of i is x (not yet copied to p)
    float *gpos;                // D
    const float *shift;         // D
    unsigned long long *hist;   // HIST_CAP
    unsigned long long *aux;    // one key per step workgroup (two-kernel reduction)
    uint32_t *prog;             // PERSIST_MAX_GRID iteration counts (persistent run)
    Ctrl *ctrl;
    uint32_t N;
    uint32_t Np;                // row pitch: N rounded up to a multiple of 64
    int32_t D;
    float lo, hi, w, c1, c2, vmax;
    uint32_t k0, k1;            // Philox key = seed
};

// Cache policy of the streamed state x, v, p: a set bit gives that array
// ordinary (cache-allocating) accesses so it can stay resident in the
// memory-side last-level cache across iterations; clear bits stream it with
// non-temporal hints.  Kept arrays must fit in that cache together, or they
// evict each other and gain nothing.
constexpr int KEEP_X = 1, KEEP_V = 2, KEEP_P = 4;
constexpr int POL_STREAM = 0, POL_X = KEEP_X, POL_XV = KEEP_X | KEEP_V, POL_ALL = KEEP_X | KEEP_V | KEEP_P;
// The policy for rows of Np particles and D dimensions: as many of x, v, p
// (in that order) as fit together in the cache budget; x alone also for
// rows up to twice the cache.
int cache_policy(uint64_t Np, int D);

// Byte layout of a swarm's workspace.  Each dimension's row of x, v, p holds
// Np = N rounded up to 64 particles, so every row starts 256-byte aligned and
// a lane can move four consecutive particles with one 16-byte access.
struct Layout {
    size_t ctrl, gpos, shift, hist, aux, prog, pf, pend, x, v, p, total;
    uint64_t Np;
    bool control; // ctrl and hist present
};
constexpr uint64_t ROW_ALIGN = 64;
// control = false leaves out the control block and history (batched swarms).
Layout layout_of(uint64_t N, int D, bool control = true);
SwarmArgs bind(void *base, const Layout &L, uint64_t N, int D);

// Launchers; all enqueue on `stream` and return the launch status.
hipError_t launch_reset(const SwarmArgs &a, hipStream_t stream);
hipError_t launch_init(int fitness, const SwarmArgs &a, hipStream_t stream);
hipError_t launch_step(int fitness, int variant, const SwarmArgs &a, hipStream_t stream);
// Tiles each workgroup of the asynchronous step runs one after another
// (PSO_ASYNC_TILES in the environment, 1..64; default 2).
uint32_t async_tiles_per_workgroup();
hipError_t launch_arm(const SwarmArgs &a, float tol, float fstar, hipStream_t stream);
// Copies every pending pbest position from x to p (before the state is read).
hipError_t launch_flush(const SwarmArgs &a, hipStream_t stream);
// Marks no pbest position pending (after the state is replaced).
hipError_t launch_clear_pending(const SwarmArgs &a, hipStream_t stream);
// Fully asynchronous persistent run: T iterations in one launch, no barrier
// between iterations; a workgroup runs at most max_lead iterations ahead of
// the slowest one (>= T: unbounded).  Needs the control block (launch_arm
// first for the stop rule); clears the workgroups' iteration counts itself.
hipError_t launch_persistent(int fitness, const SwarmArgs &a, uint32_t T, uint32_t max_lead, hipStream_t stream);

} // namespace pso

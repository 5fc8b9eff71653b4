// pso_block.hpp -- per-swarm workgroup kernels: a small swarm's whole run,
// and many swarms in one persistent launch.
#pragma once

#include "pso_kernels.hpp"

namespace pso {

// One swarm of a batch: its state view (pointers into the batch's memory,
// parameters, Philox key) and its run limits.  The control block is unused.
struct BatchItem {
    SwarmArgs a;
    int32_t fitness;
    int32_t pad;
    long long max_iter;
    float tol, fstar;
};

// Loop state (and result) of one batched swarm, kept in device memory
// between launches; the gbest position is kept in a.gpos.
struct BatchResult {
    unsigned long long gkey; // gbest key (fitness, index)
    long long giter;         // iteration of the last gbest change
    long long iters;         // iterations run
    uint32_t started;        // Step 1 done
    uint32_t stop;           // stop rule met
};

// Runs up to T more iterations of one swarm in one workgroup, continuing from
// and updating its control block (stop rule included).
hipError_t launch_block_run(int fitness, const SwarmArgs &a, long long T, hipStream_t stream);

// Marks results[0..count) not started and clears the work counter.
hipError_t launch_batch_reset(BatchResult *results, uint32_t count, unsigned int *next, hipStream_t stream);

// One persistent launch of `grid` workgroups over the `count` items listed in
// `order`: Step 1 for items not started, then max(1, chunk / (N*D)) more
// iterations of each -- `chunk` is a budget of particle-dimension updates
// per swarm and launch -- within its max_iter and stop rule.  `next` is a device work
// counter (cleared by the launch); maxD bounds every listed item's D.
// Optionally the launch also writes, for the j-th listed item, its state to
// out_state[j] and its gbest position to out_pos[j*maxD ..] (for one compact
// copy back to the host).
hipError_t launch_batch(const BatchItem *items, const uint32_t *order, BatchResult *results, uint32_t count,
                        unsigned int *next, int maxD, int grid, long long chunk, hipStream_t stream,
                        BatchResult *out_state = nullptr, float *out_pos = nullptr);
hipError_t batch_occupancy(int maxD, int *blocks_per_cu);
int batch_block_lanes();

} // namespace pso

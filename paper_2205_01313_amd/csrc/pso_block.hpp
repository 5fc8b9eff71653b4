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

// Result of one batched swarm; the gbest position goes to a.gpos.
struct BatchResult {
    unsigned long long gkey; // gbest key (fitness, index)
    long long giter;         // iteration of the last gbest change
    long long iters;         // iterations run
};

// Runs up to T more iterations of one swarm in one workgroup, continuing from
// and updating its control block (stop rule included).
hipError_t launch_block_run(int fitness, const SwarmArgs &a, long long T, hipStream_t stream);

// Runs every item of a batch: init and iterations, one persistent launch of
// `grid` workgroups taking items in the order `order`.  `next` is a device
// counter (reset by the launch); maxD bounds every item's D.
hipError_t launch_batch(const BatchItem *items, const uint32_t *order, BatchResult *results, uint32_t count,
                        unsigned int *next, int maxD, int grid, hipStream_t stream);
hipError_t batch_occupancy(int maxD, int *blocks_per_cu);
int batch_block_lanes();

} // namespace pso

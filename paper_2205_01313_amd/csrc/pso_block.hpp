// pso_block.hpp -- per-swarm workgroup kernels: a small swarm's whole run,
// and many swarms in one persistent launch (large swarms split into parts).
#pragma once

#include "pso_kernels.hpp"

namespace pso {

constexpr uint32_t MAX_PARTS = 64; // workgroups one batched swarm may span

// Meeting point of the parts of one swarm (parts > 1): each part posts its
// workgroup-minimum key and, if it has one, that particle's position into the
// slots of the step's parity, then arrives; the arrival count is monotonic
// (parts * (steps so far)), so it needs no reset between steps or launches.
struct GangSync {
    unsigned long long arrive;
    unsigned int err;
    unsigned int pad;
};

// One swarm of a batch: its state view (pointers into the batch's memory,
// parameters, Philox key), its run limits and, when split into parts, the
// parts' meeting point: cand_key[2][parts] and cand_pos[2][parts][D].
struct BatchItem {
    SwarmArgs a;
    int32_t fitness;
    uint32_t parts;
    long long max_iter;
    float tol, fstar;
    GangSync *gang;
    unsigned long long *cand_key;
    float *cand_pos;
};

// Tiles and schedule of a batched launch: lanes per workgroup (64, 128 or
// 256), co-resident workgroups, and particle-dimension updates per part and
// iteration when a large swarm is split into parts.  Every shape computes the
// same bits; only the time differs.
struct BatchShape {
    int lanes;
    int grid;
    long long part_work;
};
constexpr BatchShape DEFAULT_BATCH_SHAPE = {256, 0, 1 << 17}; // grid 0: three quarters of occupancy

bool batch_lanes_supported(int lanes);

// Parts for a batched swarm: about one part per shape.part_work
// particle-dimension updates of an iteration, at least one particle quad per
// lane of a part, at most MAX_PARTS and at most grid_cap (the workgroups of
// the launches it joins).
uint32_t parts_for(uint64_t N, int D, int grid_cap, const BatchShape &shape);

// Bytes of a swarm's gang region for `parts` parts (0 when parts == 1).
size_t gang_bytes(uint32_t parts, int D);
// Points the item's gang fields into a region of gang_bytes(parts, D).
void bind_gang(BatchItem *it, void *region, uint32_t parts);

// Loop state (and result) of one batched swarm, kept in device memory
// between launches; the gbest position is kept in a.gpos.
struct BatchResult {
    unsigned long long gkey; // gbest key (fitness, index)
    long long giter;         // iteration of the last gbest change
    long long iters;         // iterations run
    uint32_t started;        // Step 1 done
    uint32_t stop;           // stop rule met
    uint32_t ticks;          // device wall-clock ticks of the last launch's share (part 0)
    uint32_t pad;
};

// One unit of a batched launch: part `part` of item `item`; the item's state
// is also copied to position `out` of the launch's compact outputs.  iters > 0
// fixes the iterations of this launch for the swarm (every part of a swarm
// carries the same value); 0 takes the `chunk` rule of launch_batch.
struct BatchEntry {
    uint32_t item, part, out, iters;
};

// Runs up to T more iterations of one swarm in one workgroup, continuing from
// and updating its control block (stop rule included).
hipError_t launch_block_run(int fitness, const SwarmArgs &a, long long T, hipStream_t stream);

// Marks results[0..count) not started (and their gangs unused); clears the
// work counter.
hipError_t launch_batch_reset(const BatchItem *items, BatchResult *results, uint32_t count, unsigned int *next,
                              hipStream_t stream);

// One persistent launch of `grid` workgroups over `count` entries (every part
// of a listed swarm, consecutive): Step 1 for swarms not started, then the
// entry's iters, or clamp(chunk / (N*D), 1, iter_cap), more iterations of
// each -- `chunk` is a budget of particle-dimension updates per swarm and
// launch -- within its max_iter and stop rule.  `next` is a device work counter (cleared by the launch).  The
// grid must be fully co-resident (at most batch_capacity workgroups, less
// any other launch running concurrently) and every swarm's parts <= grid.
// Optionally writes each swarm's state to out_state[out] and its gbest
// position to out_pos[out*maxD ..]; device errors set *err.
hipError_t launch_batch(const BatchItem *items, const BatchEntry *entries, BatchResult *results, uint32_t count,
                        unsigned int *next, int maxD, int grid, int lanes, long long chunk, long long iter_cap,
                        hipStream_t stream, BatchResult *out_state, float *out_pos, unsigned int *err);
// Workgroups of `lanes` lanes of the batched kernel that are safely
// co-resident (three quarters of the occupancy bound).
hipError_t batch_capacity(int maxD, int lanes, int *workgroups);

} // namespace pso

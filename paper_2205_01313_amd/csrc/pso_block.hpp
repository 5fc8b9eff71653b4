// pso_block.hpp -- per-swarm workgroup kernels: a small swarm's whole run,
// and many swarms in one persistent launch (large swarms split into parts).
#pragma once

#include "pso_kernels.hpp"

namespace pso {

constexpr uint32_t MAX_PARTS = 64;         // workgroups one streamed batched swarm may span
constexpr uint32_t MAX_STAGED_PARTS = 512; // workgroups one LDS-staged batched swarm may span

// Meeting point of the parts of one swarm (parts > 1): each part posts its
// workgroup-minimum key and, if it has one, that particle's position into the
// slots of the step's parity, as words tagged with the step (cand_key,
// cand_pos); err records a part that waited past the time bound.  The arrival
// count serves no meeting and stays zero.
struct GangSync {
    unsigned long long arrive;
    unsigned int err;
    unsigned int pad;
};

// One swarm of a batch: its state view (pointers into the batch's memory,
// parameters, Philox key), its run limits and, when split into parts, the
// parts' meeting point: cand_key[2][parts][2] (a key's low and high halves)
// and cand_pos[2][parts][D] (one coordinate's bits), 64-bit words whose high
// halves carry the step.
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

// Tiles and schedule of a batched launch: lanes per workgroup, co-resident
// workgroups, particle-dimension updates per part and iteration when a large
// swarm is split into parts, and the state's home during a launch.
// stage_kib = 0 streams every part's state from device memory each
// iteration (lanes 64, 128 or 256; parts by part_work); stage_kib > 0 copies
// each part's state into stage_kib KiB of LDS for the whole launch and
// splits swarms into as many parts as that takes (lanes 256, 512 or 1024;
// part_work unused).  Every shape computes the same bits; only the time
// differs.
struct BatchShape {
    int lanes;
    int grid;
    long long part_work;
    int stage_kib;
};
constexpr BatchShape DEFAULT_BATCH_SHAPE = {256, 0, 1 << 17, 0}; // grid 0: the co-resident capacity
// A batch's shape before any autotuning when every swarm fits it (else the
// streamed default): one 1024-lane workgroup per compute unit with 158 KiB
// of staged state (less where the batch's widest D needs more LDS room).
constexpr BatchShape DEFAULT_STAGED_SHAPE = {1024, 0, 0, 158};

bool batch_lanes_supported(int lanes, bool staged = false);

// LDS bytes one staged particle quad takes: x, v, p and the fitness terms of
// each of D dimensions, its pbest fitness and pending marks.
size_t staged_quad_bytes(int D, int fitness);
// Parts of a swarm under an LDS-staged shape (each part's quads fit
// stage_kib KiB), or 0 if it would need more than MAX_STAGED_PARTS or
// grid_cap workgroups.
uint32_t staged_parts(uint64_t N, int D, int fitness, int stage_kib, int grid_cap);

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
// and updating its control block (stop rule included): its state staged in
// LDS where it fits (or PSO_BLOCK_STAGED=0 in the environment), else read
// from device memory every iteration.
hipError_t launch_block_run(int fitness, const SwarmArgs &a, long long T, hipStream_t stream);
// Whether a pso_run of this swarm should take the one-workgroup run: its
// state fits one workgroup's LDS (always true under PSO_BLOCK_STAGED=0).
bool block_run_suits(int fitness, const SwarmArgs &a);
// A single swarm too large for one workgroup's LDS, with D <= 16: the parts
// of its gang (one particle per lane of 256, all co-resident), or 0 when the
// gang does not suit it (or PSO_GANG=0 in the environment).
uint32_t gang_run_parts(int fitness, const SwarmArgs &a);
// Device words its meeting needs (64-bit each).
size_t gang_run_words(uint32_t parts, int D);
// Runs up to T more iterations of the swarm as that gang, continuing from
// and updating its control block (stop rule included); words: at least
// gang_run_words(parts, D), cleared by the launch itself.
hipError_t launch_gang_run(int fitness, const SwarmArgs &a, long long T, uint32_t parts, unsigned long long *words,
                           hipStream_t stream);

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
// stage_kib > 0 runs the LDS-staged kernel (every item's parts must come from
// staged_parts for the same stage_kib).
hipError_t launch_batch(const BatchItem *items, const BatchEntry *entries, BatchResult *results, uint32_t count,
                        unsigned int *next, int maxD, int grid, int lanes, long long chunk, long long iter_cap,
                        hipStream_t stream, BatchResult *out_state, float *out_pos, unsigned int *err,
                        int stage_kib = 0);
// Workgroups of `lanes` lanes of the batched kernel (LDS-staged with
// stage_kib KiB if > 0) that are safely co-resident: three quarters of the
// occupancy bound streamed, all but 8 compute units' worth staged; 0 if the
// staged LDS does not fit a workgroup.
hipError_t batch_capacity(int maxD, int lanes, int *workgroups, int stage_kib = 0);
// LDS bytes a workgroup of the batched kernel takes dynamically.
size_t batch_dynamic_lds(int maxD, int stage_kib);

// Staged KiB per workgroup that leave room, in a compute unit's LDS shared
// by per_cu workgroups, for each workgroup's gbest position and shift of
// maxD floats: at most 158 (per_cu = 1) or 78 (per_cu = 2); 0 if none fit.
int staged_kib_fitting(int maxD, int per_cu);
// Workgroups a launch of this shape takes: grid > 0 as given (at most the
// co-resident capacity), 0 the capacity, -k the capacity / k; 0 if a staged
// shape's LDS does not fit a workgroup.
hipError_t shape_grid(int maxD, const BatchShape &sh, int *grid);
// Sets one device word to zero with a kernel (stream-ordered; no memset).
hipError_t launch_clear_u32(unsigned int *p, hipStream_t stream);

// The first upload of a newly admitted request to the request server's
// device tables: its item and loop state go to slot `slot`, its D shift
// floats (from a launch's float pool, at shift_at) to item.a.shift, and a
// swarm of several parts gets its gang counters cleared.  One record per
// request; launch_upload applies a launch's records in one kernel, so the
// uploads of a launch are two copies and one launch whatever their number.
struct UploadRec {
    BatchItem item;
    BatchResult state;
    uint32_t slot;
    uint32_t shift_at;
    uint32_t reset_gang;
    uint32_t pad;
};
hipError_t launch_upload(const UploadRec *recs, uint32_t n, const float *pool, BatchItem *items, BatchResult *state,
                         hipStream_t stream);

} // namespace pso

/*
 * pso.h -- C ABI of libpso: global-best particle swarm optimisation on AMD
 * Instinct MI355X (gfx950), after cuPSO (Wang, Ho, Tu, Hung, ACM SAC 2022).
 *
 * The library runs the per-iteration global-best PSO step on the GPU: the
 * velocity and position update (Sec. 2.1, Eq. 1 and Eq. 2, with the clamps of
 * Alg. 1 Step 2), the fitness (Alg. 1 Step 3), the personal-best update
 * (Alg. 1 Step 4) and the aggregation into the swarm's global best (Alg. 1
 * Step 5; Sec. 3.1 Alg. 2 and Sec. 3.2 Alg. 3 for the paper's queue and
 * lock-protected aggregation, which this library replaces by a wavefront
 * minimum, a workgroup (LDS) minimum and one packed 64-bit atomic minimum).
 *
 * Conventions for every call:
 *   - Every call returns PSO_OK (0) or a negative PSO_E* code and never
 *     aborts; pso_last_error() then describes the failure (thread-local text,
 *     valid until the thread's next failing call).
 *   - Pointers named *_host are host memory owned by the caller; the library
 *     copies from or into them before returning and keeps no reference.
 *   - A pso_swarm* is owned by the caller from pso_create/pso_create_in until
 *     pso_destroy.  One swarm must not be used by two host threads at once.
 *   - Work is enqueued on the swarm's HIP stream.  Calls that return results
 *     to the host (pso_run, pso_get_*) synchronise that stream; the others
 *     return as soon as the work is enqueued.
 *   - The swarm minimises.  The paper's experiments maximise its Cubic
 *     function (Sec. 5.1, Eq. 3); PSO_CUBIC is that function negated.
 *
 * State layout in device memory (structure of arrays, Sec. 4.1 Data
 * Structure 2): position x, velocity v and personal-best position p are
 * float arrays of D*N elements with element (d, i) -- dimension d of
 * particle i -- at index d*N + i; the personal-best fitness pf holds N floats.
 */
#ifndef PSO_H
#define PSO_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes. */
#define PSO_OK 0
#define PSO_EINVAL (-1)  /* an argument is out of range or a handle is NULL */
#define PSO_ENOMEM (-2)  /* device or pinned host memory could not be obtained */
#define PSO_EDEVICE (-3) /* the HIP runtime or a kernel reported an error */
#define PSO_EAGAIN (-4)  /* a result is not ready yet (server polling) */
#define PSO_ESTATE (-5)  /* the call does not fit the object's current state */
#define PSO_ECANCELED (-6) /* a server request was cancelled (pso_server_cancel) */
#define PSO_ETIMEDOUT (-7) /* a server request did not finish by its deadline */

/* Fitness functions, all minimised over f(x) = F(x - shift). */
#define PSO_SPHERE 0     /* sum z^2 */
#define PSO_RASTRIGIN 1  /* 10 D + sum (z^2 - 10 cos(2 pi z)) */
#define PSO_ROSENBROCK 2 /* sum_{d<D-1} 100 (z_{d+1} - z_d^2)^2 + (1 - z_d)^2, D >= 2 */
#define PSO_ACKLEY 3     /* 20 - 20 exp(-0.2 sqrt(mean z^2)) + e - exp(mean cos(2 pi z)) */
#define PSO_CUBIC 4      /* -(sum z^3 - 0.8 z^2 - 1000 z + 8000), Sec. 5.1 Eq. 3 negated */

/* Aggregation variants (pso_set_variant). */
#define PSO_SYNC 0  /* gbest of iteration t-1 for every particle of iteration t (Sec. 2.2) */
#define PSO_ASYNC 1 /* a workgroup publishes a better gbest at once (Sec. 3.2) */
#define PSO_REDUCE 2 /* the paper's comparator: two kernels, tree reduction through auxiliary arrays (Sec. 2.2) */
#define PSO_REDUCE_UNROLLED 3 /* the same with the last wavefront's reduction steps unrolled (Sec. 2.2) */
#define PSO_PERSISTENT 4 /* fully asynchronous: one launch runs every iteration, no barrier between them (Sec. 6) */

typedef struct pso_swarm pso_swarm;

/* Text of the calling thread's last failure ("" if none). */
const char *pso_last_error(void);

/* Device bytes a swarm of N particles in D dimensions needs when the caller
 * provides the memory (pso_create_in); 0 if N or D is out of range. */
size_t pso_workspace_bytes(int64_t N, int32_t D);

/* Creates a swarm and runs Step 1 of Alg. 1 (Sec. 2.1) on the GPU: position
 * and velocity uniform in [bounds[0], bounds[1]) and [-vmax, vmax), fitness,
 * pbest <- position, gbest (iteration 0).  Parameters follow Table 1:
 * w inertia weight, c1 cognitive and c2 social coefficient, bounds = {min_pos,
 * max_pos} for every dimension, vmax = max_v with min_v = -vmax.
 * fitness_id is one of PSO_SPHERE..PSO_CUBIC; seed keys the Philox4x32-10
 * generator.  Requires 1 <= N <= 2^30, 1 <= D <= 4096 (D >= 2 for
 * Rosenbrock), finite parameters, bounds[0] < bounds[1], vmax > 0.
 * The library allocates device memory and a stream; *out receives the handle.
 * Errors: PSO_EINVAL, PSO_ENOMEM, PSO_EDEVICE. */
int pso_create(int fitness_id, int64_t N, int32_t D, const float bounds[2], float w, float c1, float c2,
               float vmax, uint64_t seed, pso_swarm **out);

/* As pso_create, but the swarm lives in the caller's device memory
 * dev_workspace (at least pso_workspace_bytes(N, D) bytes, 256-byte aligned)
 * and its work goes to the caller's HIP stream hip_stream (a hipStream_t;
 * NULL selects the null stream).  The caller keeps ownership of both and
 * must keep them alive until pso_destroy. */
int pso_create_in(int fitness_id, int64_t N, int32_t D, const float bounds[2], float w, float c1, float c2,
                  float vmax, uint64_t seed, void *dev_workspace, size_t bytes, void *hip_stream,
                  pso_swarm **out);

/* Sets the shift vector s (D floats, host) of f(x) = F(x - s) and re-runs
 * Step 1 so that the state is that of a fresh swarm with this shift.
 * NULL restores s = 0. */
int pso_set_shift(pso_swarm *s, const float *shift_host);

/* Selects the aggregation of the iterations that follow: PSO_SYNC
 * (default), PSO_ASYNC, the comparators PSO_REDUCE / PSO_REDUCE_UNROLLED
 * (which compute exactly what PSO_SYNC computes, with two launches per
 * iteration), or PSO_PERSISTENT: one launch runs all the iterations of a
 * pso_run (pso_step: one), each workgroup iterating its own slice of the
 * particles with no barrier between iterations, reading the published gbest
 * as a consistent snapshot and publishing a better one at once (the
 * asynchronous variant's rule); a particle still draws Philox numbers with
 * its own iteration count, and bounded staleness (pso_set_max_lead) keeps
 * workgroups within a window of each other.  Its trajectory is not
 * deterministic; its gbest is always the minimum over the pbest fitness, and
 * its history entry for iteration t is the best key known when the first
 * workgroup finished iteration t (non-increasing in t). */
int pso_set_variant(pso_swarm *s, int variant);

/* PSO_PERSISTENT: the most iterations a workgroup may run ahead of the
 * slowest one (default 8; a value >= max_iter leaves it unbounded).
 * max_lead < 0 -> EINVAL. */
int pso_set_max_lead(pso_swarm *s, int64_t max_lead);

/* Re-runs Step 1 in place: the swarm returns to iteration 0 with the same
 * parameters, seed and shift.  Allocates nothing. */
int pso_reset(pso_swarm *s);

/* Enqueues one iteration t -> t+1 (Alg. 1 Steps 2-5) and returns.  Once a
 * pso_run stop rule has been met, further steps leave the swarm unchanged. */
int pso_step(pso_swarm *s);

/* Runs up to max_iter more iterations, stopping after the first iteration
 * (or at once) where |gbest_fit - f_star| < tol; tol <= 0 disables the test.
 * Blocks until done, then writes the gbest fitness, the gbest position
 * (D floats, host), the iteration at which the gbest last changed (0 = at
 * initialisation) and the number of iterations this call ran.  Any output
 * pointer may be NULL.  A synchronous swarm with N*D <= 65536 whose state
 * fits one workgroup's LDS runs the whole call as one launch of one
 * workgroup (its state staged in LDS), unless N >= 4096 or N*D >= 8192 and
 * the gang below has 8 parts or more; a synchronous swarm with D <= 16 that
 * does not take it runs the call as one launch of ceil(N / 256) co-resident
 * workgroups (2 to 256), each holding a slice in LDS and meeting the others
 * once per iteration (PSO_GANG=0 in the environment turns this off; a part
 * that waits past 20 s sets a device error, returned as PSO_EDEVICE); others
 * take one launch per iteration (PSO_PERSISTENT: one persistent launch).
 * Every path computes the same bits. */
int pso_run(pso_swarm *s, int64_t max_iter, float tol, float f_star, float *gbest_value,
            float *gbest_pos_host, int64_t *gbest_iter, int64_t *iters_done);

/* Synchronises and reads the gbest fitness, position (D floats, host), the
 * iteration of its last change and the number of iterations completed. */
int pso_get_best(pso_swarm *s, float *gbest_value, float *gbest_pos_host, int64_t *gbest_iter,
                 int64_t *iters_completed);

/* Synchronises and copies the gbest keys of iterations t0 .. t0+count-1
 * (key = order-preserving map of the gbest fitness << 32 | gbest index) into
 * keys_host.  The library keeps the last 8192 iterations; older ones fail
 * with PSO_ESTATE. */
int pso_get_history(pso_swarm *s, int64_t t0, int64_t count, uint64_t *keys_host);

/* Synchronises and copies the full state to host buffers: x, v, p (D*N
 * floats each, layout above), pf (N floats), gbest key, gbest position (D),
 * gbest iteration and iterations completed.  NULL buffers are skipped. */
int pso_get_state(pso_swarm *s, float *x_host, float *v_host, float *p_host, float *pf_host,
                  uint64_t *gbest_key, float *gbest_pos_host, int64_t *gbest_iter, int64_t *iters_completed);

/* Replaces the state with the given one (same layout); the next iteration
 * is iters_completed + 1.  Together with pso_get_state this checkpoints and
 * resumes a swarm: the random numbers depend only on (seed, iteration,
 * particle, dimension), so a resumed run repeats the uninterrupted one. */
int pso_set_state(pso_swarm *s, const float *x_host, const float *v_host, const float *p_host,
                  const float *pf_host, uint64_t gbest_key, const float *gbest_pos_host, int64_t gbest_iter,
                  int64_t iters_completed);

/* Synchronises and reads the number of pbest improvements (Alg. 1 Step 4)
 * since the last Step 1 -- the measured improvement rate of the run. */
int pso_get_counters(pso_swarm *s, uint64_t *pbest_improvements);

/* PSO_ASYNC (the lock-protected gbest of Sec. 3.2, Alg. 3): synchronises and
 * reads, since the last Step 1, the number of tiles of particles the
 * asynchronous step ran (a workgroup runs its tiles one after another and
 * reads the running gbest before each), and how many of them used a gbest
 * published during the same iteration -- newer than the gbest at the end of
 * the previous iteration, which the synchronous variant would use.  Both
 * stay 0 under the other variants.  Either pointer may be NULL. */
int pso_get_async_counters(pso_swarm *s, uint64_t *tiles, uint64_t *fresh_tiles);

/* Blocks until the swarm's enqueued work is done; reports device errors. */
int pso_sync(pso_swarm *s);

/* Frees the library-owned memory and stream of the swarm.  NULL -> EINVAL. */
int pso_destroy(pso_swarm *s);

/* ------------------------------------------------------------------------ */
/* Binary64 path: the same method computed in double -- the paper's own     */
/* precision (Sec. 5) -- from the same binary32 parameters, shift and 24-bit */
/* Philox uniforms as the binary32 swarm.  Velocity and position updates    */
/* follow Eq. 1 and Eq. 2 with their clamps (Alg. 1 Step 2), the gbest is   */
/* synchronised once per iteration (lowest index among equal fitness), and  */
/* the fitness functions are those of pso_create, Cubic (Eq. 3) negated.    */
/* State is double, rows of N particles per dimension ((d, i) at d*N + i).  */
/* ------------------------------------------------------------------------ */
typedef struct pso_swarm64 pso_swarm64;

/* As pso_create (same arguments and checks), then Step 1 in double.  The
 * swarm owns its device memory and a stream until pso64_destroy. */
int pso64_create(int fitness_id, int64_t N, int32_t D, const float bounds[2], float w, float c1, float c2,
                 float vmax, uint64_t seed, pso_swarm64 **out);

/* Shift s (D floats, host, copied; finite): f(x) = F(x - s); re-runs Step 1. */
int pso64_set_shift(pso_swarm64 *s, const float *shift);

/* Re-runs Step 1 (iteration count back to 0). */
int pso64_reset(pso_swarm64 *s);

/* Enqueues one iteration (asynchronous). */
int pso64_step(pso_swarm64 *s);

/* Up to max_iter more iterations, stopping once |gbest - f_star| < tol
 * (tol <= 0: off; tested before the first and after every iteration);
 * blocks.  Outputs (each may be NULL, host): gbest fitness, position (D
 * doubles), iteration of the last gbest change, iterations run.  A swarm
 * with D >= 32 and N <= 32768 launches one grid step per iteration (lanes
 * share each particle's dimensions); else a swarm whose x, v, p and pbest
 * fitness fit one workgroup's LDS ((3D+1)*N doubles, up to about 160 KiB)
 * runs in one workgroup (one launch, the state loaded once and stored back
 * at the end), unless D <= 8 and N >= 4096; a swarm with D <= 8 that does
 * not run there runs as one persistent launch of co-resident workgroups that
 * meet once per iteration, as does one with D < 32 whose workgroups can hold
 * their slices of the swarm in LDS; others launch one grid step per
 * iteration.  Every path gives the same results. */
int pso64_run(pso_swarm64 *s, int64_t max_iter, double tol, double f_star, double *gbest_value, double *gbest_pos,
              int64_t *gbest_iter, int64_t *iters_done);

/* Copies the state to host buffers (each may be NULL): x, v, p (D*N doubles
 * each, (d, i) at d*N + i), pbest fitness (N doubles), gbest particle index,
 * iterations completed.  Synchronises. */
int pso64_get_state(pso_swarm64 *s, double *x, double *v, double *p, double *pf, int64_t *gbest_index,
                    int64_t *t);

/* The swarm's fitness function, with its shift, in binary64 at M points
 * (host, row-major M x D doubles) -> values (host, M doubles): the same
 * operation sequence as the binary64 swarm evaluates (Eq. 3 and the test
 * functions of Sec. 5, in dimension order).  Used to re-evaluate a binary32
 * result in binary64.  Synchronous; allocates a device buffer for the call.
 * M < 0 or NULL pointers (with M > 0) -> EINVAL. */
int pso64_eval(pso_swarm64 *s, const double *points, int64_t M, double *values);

/* Frees the swarm.  NULL -> EINVAL. */
int pso64_destroy(pso_swarm64 *s);

/* ------------------------------------------------------------------------ */
/* Batches: many independent swarms (uneven N, D and fitness) run by one     */
/* persistent launch; each swarm computes exactly what pso_create + pso_run  */
/* (synchronous variant) computes for it alone.                              */
/* ------------------------------------------------------------------------ */

/* One swarm of a batch: the pso_create parameters, an optional shift (D
 * floats, host, copied at pso_batch_create; NULL = 0) and the pso_run limits
 * (max_iter iterations, stop once |gbest - f_star| < tol; tol <= 0: off). */
typedef struct pso_desc {
    int32_t fitness_id;
    int32_t D;
    int64_t N;
    float bounds[2];
    float w, c1, c2, vmax;
    uint64_t seed;
    const float *shift;
    int64_t max_iter;
    float tol;
    float f_star;
} pso_desc;

/* Result of one batched swarm.  gbest_pos is caller memory (D floats, host)
 * filled by pso_batch_results, or NULL to skip the position. */
typedef struct pso_result {
    float gbest_value;  /* gbest fitness */
    int32_t status;     /* PSO_OK */
    int64_t gbest_iter; /* iteration of the last gbest change (0 = init) */
    int64_t iters;      /* iterations run */
    float *gbest_pos;
} pso_result;

typedef struct pso_batch pso_batch;

/* Validates count descriptors (each as pso_create, plus max_iter >= 0),
 * allocates the device memory of all swarms and uploads their parameters.
 * Work goes to hip_stream (a hipStream_t; NULL: a library-created stream).
 * The descriptors are copied; the caller keeps ownership of them. */
int pso_batch_create(const pso_desc *descs, int64_t count, void *hip_stream, pso_batch **out);

/* Enqueues the whole batch -- Step 1 and every iteration of every swarm --
 * as one persistent launch; returns without synchronising.  May be called
 * again to rerun the batch from scratch.  The launch is captured into a HIP
 * graph on first use (and again after a shape change) and replayed from
 * then on; PSO_BATCH_GRAPH=0 in the environment launches it directly. */
int pso_batch_launch(pso_batch *b);

/* Synchronises and writes results[i] for every swarm i (results[i].gbest_pos
 * as described above). */
int pso_batch_results(pso_batch *b, pso_result *results);

/* Frees the batch's device memory (and its stream if the library made it). */
int pso_batch_destroy(pso_batch *b);

/* pso_batch_create + pso_batch_launch + pso_batch_results + destroy. */
int pso_batch_run(const pso_desc *descs, int64_t count, pso_result *results);

/* For callers that cannot allocate device memory (code that must not call
 * hipMalloc, such as tight serving loops or harnesses that forbid it):
 * pso_batch_run without any allocation.  Every device buffer the batch
 * needs (each swarm's state, the descriptors, the work queue, the results
 * and counters) is carved out of one fixed array of PSO_STATIC_SCRATCH_BYTES
 * that the library keeps on each device it runs on, from its first use there
 * until the process ends; host staging is fixed-size as well.  Results are
 * bit for bit those of pso_batch_run (same kernels, the default batch shape;
 * the autotuner and graph capture are not used).
 *   descs, count  as pso_batch_run; count <= PSO_STATIC_MAX_SWARMS.
 *   results       caller host memory, count entries (gbest_pos as in
 *                 pso_batch_results).
 *   hip_stream    a hipStream_t on the current device, or NULL for its null
 *                 stream; the call synchronises it before returning.
 * Errors: PSO_EINVAL for a bad descriptor, count out of range or more than
 * PSO_STATIC_MAX_ENTRIES work-queue entries; PSO_ENOMEM when the swarms'
 * state and bookkeeping exceed the scratch (nothing is launched then);
 * PSO_EDEVICE for a HIP error.  Calls in one process are serialised by the
 * library; each call overwrites the scratch of the current device, whose
 * contents are the last call's afterwards.  Work of another process, or
 * kernels of this one still reading a previous call's state, must not
 * overlap a call on the same device. */
#define PSO_STATIC_SCRATCH_BYTES ((size_t)64 << 20)
#define PSO_STATIC_MAX_SWARMS 1024
#define PSO_STATIC_MAX_ENTRIES 16384u
int pso_batch_run_static(const pso_desc *descs, int64_t count, pso_result *results, void *hip_stream);

/* Tiles and schedule of a batch's launches (they change the time, never the
 * results).  stage_kib = 0 streams each swarm's state from device memory
 * every iteration: lanes per workgroup (64, 128 or 256), co-resident
 * workgroups (grid; 0 = the device's co-resident capacity for that shape),
 * and the particle-dimension updates per part and iteration at which a
 * large swarm is split over several workgroups (part_work >= 1).
 * stage_kib > 0 keeps each part's state in stage_kib KiB of LDS for a whole
 * launch (lanes 256, 512 or 1024; part_work is ignored): a swarm is split into as
 * many parts as its state needs, at most 512 and at most the grid; swarms
 * that would need more stream, in a second kernel of the same launch.  A new
 * batch takes the shape pso_batch_autotune chose earlier in this process for
 * the same swarm sizes and iteration limits on the same device, else 1024
 * lanes with 158 KiB staged (less for D above 64: the LDS also holds
 * 2 x D floats) if every swarm fits that, else 256 lanes, the
 * full capacity, 2^17 updates per part, streamed.  The co-resident capacity
 * is three quarters of the occupancy bound streamed and all but 8 compute
 * units' worth staged: a batch sharing the device with other long-running
 * kernels may find its parts not co-resident, which its bounded waits report
 * as PSO_EDEVICE from pso_batch_results. */
typedef struct pso_batch_shape {
    int32_t lanes;
    int32_t grid;
    int64_t part_work;
    int32_t stage_kib;
    int32_t reserved; /* 0 */
} pso_batch_shape;

/* The batch's current shape (grid as launched: at most the entry count). */
int pso_batch_get_shape(pso_batch *b, pso_batch_shape *shape);

/* Sets the shape for the following launches (synchronises the batch's
 * stream).  EINVAL for unsupported lanes, grid < 0, part_work < 1 (streamed),
 * stage_kib < 0 or more staged KiB than a workgroup's LDS; a grid above the
 * co-resident capacity is reduced to it, so every launch stays
 * deadlock-free.  Between launches only: the batch's state is restarted by
 * the next pso_batch_launch anyway. */
int pso_batch_set_shape(pso_batch *b, const pso_batch_shape *shape);

/* Autotuner (the batching row of the workload set: tiles and schedules
 * picked by measurement on the device).  Under each candidate shape --
 * streamed: 64/128/256 lanes x 2^15/2^17 updates per part x all or half of
 * the co-resident workgroups; LDS-staged: 512/1024 lanes x 78/158 KiB per
 * workgroup (less for D above 64), where the swarms fit -- it runs Step 1
 * untimed, then times launches of probe_iters and 3 x probe_iters
 * iterations of the whole batch, splits a launch's time into a fixed part
 * and a part per iteration, and prices the shape at the batch's mean
 * iteration limit (max_iter); it keeps the cheapest, records it for later
 * batches of the same signature, and writes it to *chosen (may be NULL).
 * Leaves the batch ready for pso_batch_launch (which restarts it).
 * Synchronous; costs about 16 x (4 probe_iters + 1) iterations of the batch.
 * probe_iters < 1 -> EINVAL. */
int pso_batch_autotune(pso_batch *b, int64_t probe_iters, pso_batch_shape *chosen);

/* ------------------------------------------------------------------------ */
/* Request server: solves arrive over time (the real-time uses of Sec. 1).   */
/* Requests are admitted in arrival order as device memory allows; admitted  */
/* swarms stay resident and advance together -- each launch runs about       */
/* chunk_updates particle-dimension updates of every swarm (at least one     */
/* iteration) -- with two launches in flight so that new arrivals start      */
/* while others run.  A request's result is the same bits as pso_create + pso_run  */
/* (synchronous) of the same descriptor alone.  Thread-safe: submit and poll */
/* may be called from any host thread.                                       */
/* ------------------------------------------------------------------------ */
typedef struct pso_server pso_server;

typedef struct pso_server_counters {
    uint64_t submitted, completed, rejected, queued, launches;
    size_t mem_budget, mem_used, mem_peak; /* device bytes of swarm state */
    double p50_ms, p99_ms, max_ms;         /* submit-to-completion latency of completed requests */
    uint64_t cancelled, timed_out;         /* requests ended by pso_server_cancel / their deadline */
} pso_server_counters;

/* Starts a server with mem_budget bytes of device memory for swarm state
 * (allocated now).  Each launch gives each of its swarms the iterations
 * that fit a 2 ms slice at the swarm's own measured speed (4 on its first
 * launch), at most chunk_updates particle-dimension updates' worth (<= 0: no
 * such cap).  A request with D <= 64 whose state fits runs in LDS-staged
 * launches (its state in LDS during each launch), others in streamed ones; a launch is of
 * one kind and takes the longest-waiting ready swarms of that kind, at most
 * 8 parts per workgroup (PSO_SERVER_STAGED=0 in the environment streams
 * every request). */
int pso_server_create(size_t mem_budget, int64_t chunk_updates, pso_server **out);

/* Queues one request (validated as a batch descriptor; the shift is copied)
 * and returns its ticket. */
int pso_server_submit(pso_server *srv, const pso_desc *desc, uint64_t *ticket);

/* PSO_EAGAIN while the request is queued or running.  Once it is done, fills
 * *result (result->gbest_pos as for batches) and the submit-to-completion
 * latency, forgets the ticket and returns PSO_OK -- or, also forgetting the
 * ticket, PSO_ENOMEM if the request needs more memory than the whole budget,
 * PSO_ECANCELED or PSO_ETIMEDOUT if it was cancelled or passed its deadline
 * (the latency is then submit-to-drop).  Unknown ticket: EINVAL. */
int pso_server_poll(pso_server *srv, uint64_t ticket, pso_result *result, double *latency_ms);

/* Cancels a request.  A request still waiting for memory leaves the queue at
 * once; an admitted one leaves at the scheduler's next decision about it --
 * before its next launch, or when its running launch ends (if that launch
 * finishes it, its result stands) -- and its memory returns to the budget.
 * pso_server_poll then reports PSO_ECANCELED.  Unknown ticket: EINVAL; a
 * request that has already finished (or was rejected): ESTATE. */
int pso_server_cancel(pso_server *srv, uint64_t ticket);

/* Gives a request a deadline timeout_ms after its submission (> 0 and
 * finite).  A request not finished by then is dropped as pso_server_cancel
 * drops it, and pso_server_poll reports PSO_ETIMEDOUT; the result of a launch
 * that finishes it before the drop stands.  The scheduler checks deadlines
 * every pass (about every 50 us while idle).  Unknown ticket: EINVAL;
 * finished request: ESTATE. */
int pso_server_set_deadline(pso_server *srv, uint64_t ticket, double timeout_ms);

/* Counters, memory use and latency percentiles since the server started. */
int pso_server_stats(pso_server *srv, pso_server_counters *stats);

/* Stops the scheduler (requests still queued or running are dropped) and
 * frees the server. */
int pso_server_destroy(pso_server *srv);

#ifdef __cplusplus
}
#endif

#endif /* PSO_H */

// pso_block.hip -- a workgroup runs a whole swarm, or one part of it, for
// many iterations with workgroup barriers only.
//
// For a swarm small enough for one compute unit, a launch per iteration
// costs more than the iteration itself, and the paper's answer -- removing
// the second kernel (Sec. 3.2) -- still leaves one launch per iteration.
// Here the iteration loop runs inside the workgroup: the gbest minimum is a
// wavefront butterfly plus an LDS atomicMin and the gbest position lives in
// LDS.  The state either stays in device memory in the grid kernels' layout
// (streamed: the same init_quad / iterate_quad) or is staged into LDS for
// the whole launch (staged: per-(particle, dimension pair) items, the same
// per-element Eq. 1 / Eq. 2 functions, fitness terms folded in dimension
// order), so a swarm computes the same bits whichever kernel runs it.
//
// The batched kernels are persistent: each workgroup takes the next entry (a
// swarm, or one part of a large one) from an atomic work counter (largest
// per-part work first), runs it to its iteration limit or stop rule, writes
// the result, and takes the next; the parts of a swarm meet once per
// iteration; every workgroup exits when the counter passes the entry count.
#include <algorithm>
#include <cstdlib>
#include <cstring>

#include "pso_aggregate.hpp"
#include "pso_block.hpp"
#include "pso_quad.hpp"

#ifndef PSO_RUN_LANES
#define PSO_RUN_LANES 256 // lanes of the workgroup running one small swarm (pso_run)
#endif
#ifndef PSO_SWARM_POLICY
// cache policy of the per-swarm workgroup kernels: a workgroup re-reads its
// swarm's (small) state every iteration, so all of it stays cacheable
#define PSO_SWARM_POLICY POL_ALL
#endif

namespace pso {

constexpr int RUN_LANES = PSO_RUN_LANES;

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

// The share of a swarm one workgroup runs: particle quads [q_lo, q_hi)
// (4q < N), padded quads [qi_lo, qi_hi) initialised by it (4q < Np), and for
// a swarm of several parts, their meeting point.
struct Part {
    uint32_t q_lo, q_hi, qi_lo, qi_hi;
    uint32_t part, parts;
    GangSync *gang;
    unsigned long long *cand_key;
    float *cand_pos;
};

__device__ __forceinline__ Part whole_swarm(const SwarmArgs &a)
{
    Part P{};
    P.q_lo = 0;
    P.q_hi = (a.N + 3) / 4;
    P.qi_lo = 0;
    P.qi_hi = a.Np / 4;
    P.part = 0;
    P.parts = 1;
    return P;
}

// Workgroup-shared scratch of the per-swarm loop.
struct Scratch {
    unsigned long long min[2]; // workgroup_min slots, alternating by step
    unsigned long long bkey;   // broadcast of the combined key
    unsigned int owner;        // broadcast of the part owning it
    unsigned int err;          // a wait gave up
};

constexpr unsigned long long GANG_WAIT_TICKS = 2000000000ull; // 20 s of the 100 MHz wall clock

// The parts of a swarm meet without fences: every word a part posts for step
// tau -- its minimum key as two words (low and high half), its candidate's
// coordinates one word each -- carries tau + 1 in its high half and moves by
// relaxed device-scope atomics, which are coherent per word; a reader waits
// for each word it needs to carry the step's tag.  (An agent-scope release
// and acquire write back and invalidate the XCD's L2, microseconds a step.)
// Words of the other parity cannot be overwritten early: a part posts step
// tau + 2 only after every part has posted tau + 1, after reading tau.  The
// words are zeroed when the swarm starts (batch reset, server upload), since
// another swarm's earlier steps could carry the same tags.  Without fences
// no other memory may pass between parts within a launch: each part
// initialises and iterates its own particles only.
__device__ __forceinline__ unsigned long long gang_tag(long long tau)
{
    return (unsigned long long)(uint32_t)(tau + 1) << 32;
}

// Waits until *w carries tag; its payload (0 and sc->err set after the
// bound).
__device__ __forceinline__ uint32_t gang_read(const unsigned long long *w, unsigned long long tag, Scratch *sc,
                                              unsigned long long t0)
{
    unsigned long long v;
    while (((v = __hip_atomic_load(w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) & 0xFFFFFFFF00000000ull) != tag) {
        __builtin_amdgcn_s_sleep(1);
        if (wall_clock64() - t0 > GANG_WAIT_TICKS) {
            sc->err = 1u;
            return 0u;
        }
    }
    return (uint32_t)v;
}

// Posts this part's candidate position for step tau: the D coordinates of
// memory column mi of row-major state x (row pitch `pitch`).
template <int LANES>
__device__ __forceinline__ void stage_candidate(const Part &P, long long tau, int D, const float *x, size_t pitch,
                                                uint32_t mi)
{
    unsigned long long *dst =
        reinterpret_cast<unsigned long long *>(P.cand_pos) + ((size_t)(tau & 1) * P.parts + P.part) * D;
    const unsigned long long tag = gang_tag(tau);
    for (int d = threadIdx.x; d < D; d += LANES)
        __hip_atomic_store(&dst[d], tag | __float_as_uint(x[(size_t)d * pitch + mi]), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
}

// Combining the workgroup minima of step tau over the swarm's parts, in two
// halves so that a caller can work between them.  gang_post publishes this
// part's minimum m (its candidate position already posted if m != NO_KEY);
// gang_wait waits for every part's key and returns the swarm minimum, with
// *owner the part that posted it (its position is in cand_pos).  The first
// wavefront reads the parts' keys in parallel.
template <int LANES>
__device__ __forceinline__ void gang_post(const Part &P, long long tau, unsigned long long m)
{
    if (threadIdx.x < 2) {
        unsigned long long *kw = P.cand_key + ((size_t)(tau & 1) * P.parts + P.part) * 2;
        const uint32_t pay = threadIdx.x ? (uint32_t)(m >> 32) : (uint32_t)m;
        __hip_atomic_store(&kw[threadIdx.x], gang_tag(tau) | pay, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __syncthreads();
}

template <int LANES>
__device__ unsigned long long gang_wait(const Part &P, long long tau, Scratch *sc, uint32_t *owner)
{
    if (threadIdx.x < 64) {
        const unsigned long long tag = gang_tag(tau), t0 = wall_clock64();
        const unsigned long long *kw = P.cand_key + (size_t)(tau & 1) * P.parts * 2;
        unsigned long long g = NO_KEY;
        uint32_t o = 0;
        for (uint32_t p = threadIdx.x; p < P.parts; p += 64) {
            const uint32_t lo = gang_read(&kw[2 * p], tag, sc, t0), hi = gang_read(&kw[2 * p + 1], tag, sc, t0);
            const unsigned long long k = ((unsigned long long)hi << 32) | lo;
            if (k < g) {
                g = k;
                o = p;
            }
        }
        const unsigned long long gm = wave_min_u64(g);
        // keys name distinct particles, so one lane holds gm (or all hold NO_KEY)
        const int src = __builtin_ctzll(__ballot(g == gm));
        const uint32_t om = (uint32_t)__shfl((int)o, src, 64);
        if (threadIdx.x == 0) {
            sc->bkey = gm;
            sc->owner = om;
        }
    }
    __syncthreads();
    *owner = sc->owner;
    return sc->bkey;
}

template <int LANES>
__device__ __forceinline__ unsigned long long gang_exchange(const Part &P, long long tau, unsigned long long m,
                                                            Scratch *sc, uint32_t *owner)
{
    gang_post<LANES>(P, tau, m);
    return gang_wait<LANES>(P, tau, sc, owner);
}

// The same over the streamed state: the candidate's position is column m of
// x in device memory (stored by this workgroup).
template <int LANES>
__device__ unsigned long long gang_min(const SwarmArgs &a, const Part &P, long long tau, unsigned long long m,
                                       Scratch *sc, uint32_t *owner)
{
    if (P.parts == 1) { // uniform per swarm
        *owner = 0;
        return m;
    }
    if (m != NO_KEY) stage_candidate<LANES>(P, tau, a.D, a.x, a.Np, (uint32_t)m);
    return gang_exchange<LANES>(P, tau, m, sc, owner);
}

// gbest position <- the particle of key k: from x (one part: stored by this
// workgroup before the last barrier) or from the owner part's posted copy.
template <int LANES>
__device__ __forceinline__ void gather_gbest(const SwarmArgs &a, const Part &P, long long tau, unsigned long long k,
                                             uint32_t owner, float *s_g, Scratch *sc)
{
    const int D = a.D;
    if (k == NO_KEY) return; // no part had a candidate: nothing was posted
    if (P.parts == 1) {
        const size_t gi = (uint32_t)k;
        for (int d = threadIdx.x; d < D; d += LANES) s_g[d] = a.x[(size_t)d * a.Np + gi];
    } else {
        const unsigned long long *src =
            reinterpret_cast<const unsigned long long *>(P.cand_pos) + ((size_t)(tau & 1) * P.parts + owner) * D;
        const unsigned long long tag = gang_tag(tau), t0 = wall_clock64();
        for (int d = threadIdx.x; d < D; d += LANES) s_g[d] = __uint_as_float(gang_read(&src[d], tag, sc, t0));
    }
}

// Step 1 by one workgroup (its part); leaves the gbest position in s_g.
template <int FIT, int LANES>
__device__ void block_init(const SwarmArgs &a, const Part &P, const float *s_shift, float *s_g, Scratch *sc,
                           SwarmLoop &L)
{
    const int D = a.D;
    unsigned long long key = NO_KEY;
    for (uint32_t q = P.qi_lo + threadIdx.x; q < P.qi_hi; q += LANES) {
        const unsigned long long k = init_quad<FIT, PSO_SWARM_POLICY>(a, D, q, s_shift);
        key = k < key ? k : key;
    }
    const unsigned long long m = workgroup_min(key, NO_KEY, &sc->min[0]);
    if (threadIdx.x == 0) sc->min[1] = NO_KEY;
    uint32_t owner;
    const unsigned long long g = gang_min<LANES>(a, P, 0, m, sc, &owner);
    gather_gbest<LANES>(a, P, 0, g, owner, s_g, sc);
    L.gkey = g;
    L.giter = 0;
    L.t = 0;
    __syncthreads();
}

// Up to T iterations after L.t, stopping after the first iteration at which
// the stop rule holds (it is tested before the first one too).  sc->min[2]
// alternates between iterations: slot (t & 1) collects iteration t's
// minimum, and the other slot is cleared for iteration t+1.  hist (may be
// null) receives each iteration's gbest key.
template <int FIT, int LANES, bool PF>
__device__ void block_iterate(const SwarmArgs &a, const Part &P, long long T, float tol, float fstar,
                              const float *s_shift, float *s_g, Scratch *sc, unsigned long long *hist, SwarmLoop &L)
{
    uint32_t n_imp = 0; // this lane's pbest improvements over the run
    const int D = a.D;
    L.stop = L.stop || meets_tol(L.gkey, tol, fstar);
    for (long long it = 0; it < T && !L.stop; ++it) {
        const uint32_t t = (uint32_t)(L.t + 1);
        unsigned long long key = NO_KEY;
        for (uint32_t q = P.q_lo + threadIdx.x; q < P.q_hi; q += LANES) {
            uint32_t n = 0;
            const unsigned long long k = iterate_quad<FIT, 0, 1, PSO_SWARM_POLICY, PF>(a, D, q, t, s_g, s_shift, &n);
            key = k < key ? k : key;
            n_imp += n;
        }
        const unsigned long long m = workgroup_min(key, L.gkey, &sc->min[t & 1]);
        if (threadIdx.x == 0) sc->min[(t + 1) & 1] = NO_KEY;
        uint32_t owner;
        const unsigned long long g = gang_min<LANES>(a, P, t, m, sc, &owner);
        if (g < L.gkey) {
            L.gkey = g;
            L.giter = t;
            gather_gbest<LANES>(a, P, t, g, owner, s_g, sc);
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
__global__ void __launch_bounds__(RUN_LANES) k_block_run(SwarmArgs a, long long T)
{
    __shared__ Scratch sc;
    extern __shared__ float s_dyn[]; // gbest position (D), shift (D)
    Ctrl *c = a.ctrl;
    const int D = a.D;
    float *s_g = s_dyn, *s_shift = s_dyn + D;
    for (int d = threadIdx.x; d < D; d += RUN_LANES) {
        s_g[d] = a.gpos[d];
        s_shift[d] = a.shift[d];
    }
    if (threadIdx.x == 0) {
        sc.min[0] = NO_KEY;
        sc.min[1] = NO_KEY;
        sc.err = 0;
    }
    SwarmLoop L;
    L.gkey = c->gkey_prev;
    L.giter = c->giter;
    L.t = c->t;
    L.stop = c->stop != 0u;
    const float tol = c->tol, fstar = c->fstar;
    __syncthreads();
    block_iterate<FIT, RUN_LANES, false>(a, whole_swarm(a), T, tol, fstar, s_shift, s_g, &sc, a.hist, L);
    if (L.improved) atomicAdd(&c->improved, (unsigned long long)L.improved);
    for (int d = threadIdx.x; d < D; d += RUN_LANES) a.gpos[d] = s_g[d];
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
// advances every listed swarm by about `chunk` updates' worth of iterations
// and leaves its loop state (BatchResult) and gbest position in device
// memory, so a later launch resumes it exactly where it stopped: a swarm
// computes the same bits however its iterations are split over launches.
//
// A large swarm is split into parts run by different workgroups, which meet
// once per step (gang_min).  Parts are consecutive in the work queue and the
// grid is fully co-resident, so a part waiting for its siblings always has
// them dequeued by workgroups that finish their own work: the first swarm in
// queue order with a part not yet dequeued has all its earlier parts either
// running or waiting for it, and every swarm before it has all its parts.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(64) k_batch_reset(const BatchItem *items, BatchResult *results, uint32_t count,
                                                     unsigned int *next)
{
    const uint32_t i = blockIdx.x; // one wavefront per swarm
    if (i >= count) return;
    if (threadIdx.x == 0) {
        if (i == 0) *next = 0u;
        results[i].gkey = NO_KEY;
        results[i].giter = 0;
        results[i].iters = 0;
        results[i].started = 0;
        results[i].stop = 0;
        results[i].ticks = 0;
        if (items[i].parts > 1) {
            items[i].gang->arrive = 0ull;
            items[i].gang->err = 0u;
        }
    }
    if (items[i].parts > 1) { // the meeting's tagged words (keys, then candidate positions)
        const size_t nk = (size_t)4 * items[i].parts, np = (size_t)2 * items[i].parts * items[i].a.D;
        for (size_t w = threadIdx.x; w < nk; w += 64) items[i].cand_key[w] = 0ull;
        unsigned long long *pw = reinterpret_cast<unsigned long long *>(items[i].cand_pos);
        for (size_t w = threadIdx.x; w < np; w += 64) pw[w] = 0ull;
    }
}

__global__ void k_counter_reset(unsigned int *next)
{
    if (threadIdx.x == 0) *next = 0u;
}

template <int FIT, int LANES>
__device__ void batch_part(const BatchItem &it, uint32_t part, uint32_t fixed_iters, BatchResult *res, long long chunk,
                           long long iter_cap, float *s_g,
                           float *s_shift, Scratch *sc, BatchResult *out_state, float *out_pos, uint32_t out,
                           int pos_stride)
{
    const SwarmArgs &a = it.a;
    const int D = a.D;
    Part P;
    const uint32_t nq = (a.N + 3) / 4, nqi = a.Np / 4;
    P.parts = it.parts;
    P.part = part;
    P.q_lo = (uint32_t)((unsigned long long)nq * part / it.parts);
    P.q_hi = (uint32_t)((unsigned long long)nq * (part + 1) / it.parts);
    // Step 1 over the quads this part iterates (the last part also takes
    // the padding): a part reads no state another part wrote during the
    // launch, so the tagged meeting words are all the parts share
    P.qi_lo = P.q_lo;
    P.qi_hi = part + 1 == it.parts ? nqi : P.q_hi;
    P.gang = it.gang;
    P.cand_key = it.cand_key;
    P.cand_pos = it.cand_pos;
    for (int d = threadIdx.x; d < D; d += LANES) s_shift[d] = a.shift[d];
    if (threadIdx.x == 0) {
        sc->min[0] = NO_KEY;
        sc->min[1] = NO_KEY;
    }
    SwarmLoop L;
    const bool started = res->started != 0u;
    __syncthreads();
    if (!started) {
        L.stop = false;
        block_init<FIT, LANES>(a, P, s_shift, s_g, sc, L);
    } else {
        L.gkey = res->gkey;
        L.giter = res->giter;
        L.t = res->iters;
        L.stop = res->stop != 0u;
        for (int d = threadIdx.x; d < D; d += LANES) s_g[d] = a.gpos[d];
        __syncthreads();
    }
    // iterations this launch: about `chunk` particle-dimension updates' worth
    // (at least one); the same number for every part of the swarm
    const long long left = it.max_iter - L.t;
    const long long nd = (long long)a.N * a.D;
    long long iters = chunk / nd;
    iters = iters < 1 ? 1 : (iters > iter_cap ? iter_cap : iters);
    if (fixed_iters > 0) iters = fixed_iters;
    const unsigned long long c0 = wall_clock64();
    // prefetch pays in the batch: many short rows need more loads in flight
    block_iterate<FIT, LANES, true>(a, P, left < iters ? left : iters, it.tol, it.fstar, s_shift, s_g, sc, nullptr,
                                    L);
    const unsigned long long ticks = wall_clock64() - c0;
    if (part == 0) {
        for (int d = threadIdx.x; d < D; d += LANES) {
            a.gpos[d] = s_g[d];
            if (out_pos) out_pos[(size_t)out * pos_stride + d] = s_g[d];
        }
        if (threadIdx.x == 0) {
            res->gkey = L.gkey;
            res->giter = L.giter;
            res->iters = L.t;
            res->stop = L.stop ? 1u : 0u;
            res->started = 1u;
            res->ticks = ticks > 0xFFFFFFFFull ? 0xFFFFFFFFu : (uint32_t)ticks;
            if (out_state) out_state[out] = *res;
        }
    }
}

// ---------------------------------------------------------------------------
// LDS-staged batched part.  A part's state (x, v, p, pf, pending marks) is
// copied into LDS once per launch and every iteration of the launch works
// there, so device memory sees two passes per launch instead of one per
// iteration.  A part holds so few particles at high D that one particle per
// lane would leave most lanes idle, so the iteration has two phases, as in
// the split grid step: (1) each lane takes (particle, dimension pair) items
// -- one Philox call each; consecutive lanes take consecutive particles of
// one pair, so LDS accesses are conflict-free, and items of one particle
// each are small enough that the last round over the lanes wastes little --
// and applies Eq. 1 and Eq. 2 with the per-element functions every other
// kernel uses, staging each dimension's fitness terms; (2) after a barrier
// one lane per particle folds the terms in dimension order, so the fitness
// is the sequential sum of the other paths bit for bit, and applies the
// strict pbest test.  A pbest position stays pending in x until the next
// iteration copies it (only that particle's own elements are written: LDS
// has no write granularity to respect).  Step 1 runs in device memory (block_init over
// exactly this part's quads and, for the last part, the padding) and is then
// staged like a resumed part.
// ---------------------------------------------------------------------------
// Lane-strided walk over the cells (row, col) of a rows x cols grid in
// row-major order, starting at cell threadIdx.x: one division at the start,
// then additions only.
template <int LANES>
struct GridWalk {
    uint32_t row, col, drow, dcol, cols;
    __device__ __forceinline__ explicit GridWalk(uint32_t ncols) : cols(ncols)
    {
        row = threadIdx.x / ncols;
        col = threadIdx.x - row * ncols;
        drow = LANES / ncols;
        dcol = LANES - drow * ncols;
    }
    __device__ __forceinline__ void next()
    {
        row += drow;
        col += dcol;
        if (col >= cols) {
            col -= cols;
            ++row;
        }
    }
};

static constexpr int staged_words(int fitness) { return fitness == F_ACKLEY ? 2 : 1; }

size_t staged_quad_bytes(int D, int fitness)
{
    return 4 * (sizeof(float) * (3 + staged_words(fitness)) * (size_t)D + sizeof(float) + 1);
}

// A staged part's view in LDS: x, v, p, the fitness terms (W words) in rows
// of `pitch` particles, then pf and the pending marks; local quad q is
// particle ibase + 4q + k (the part holds quads [q_lo, q_lo + nql)).
struct Staged {
    SwarmArgs la;
    float *t0, *t1;
    uint32_t nql, pitch, ibase, q_lo;
};

template <int FIT>
__device__ __forceinline__ Staged staged_view(const SwarmArgs &a, float *s_state, uint32_t q_lo, uint32_t q_hi)
{
    constexpr int W = Fitness<FIT>::STAGE_WORDS;
    Staged S;
    S.q_lo = q_lo;
    S.nql = q_hi - q_lo;
    S.pitch = 4 * S.nql;
    S.ibase = 4 * q_lo;
    const size_t plane = (size_t)a.D * S.pitch;
    S.la = a;
    S.la.x = s_state;
    S.la.v = S.la.x + plane;
    S.la.p = S.la.v + plane;
    S.t0 = S.la.p + plane;
    S.t1 = S.t0 + plane;
    S.la.pf = S.t0 + (size_t)W * plane;
    S.la.pend = reinterpret_cast<uint8_t *>(S.la.pf + S.pitch);
    S.la.Np = S.pitch;
    return S;
}

// Device memory -> LDS (ends with a barrier); LDS -> device memory (pending
// marks included, so the stored state means what the streamed paths store).
template <int LANES>
__device__ void staged_load(const SwarmArgs &a, const Staged &S)
{
    const uint32_t nql = S.nql;
    for (uint32_t e = threadIdx.x; e < (uint32_t)a.D * nql; e += LANES) {
        const uint32_t d = e / nql, q = e - d * nql;
        const size_t g = (size_t)d * a.Np / 4 + S.q_lo + q, l = (size_t)d * nql + q;
        reinterpret_cast<f4 *>(S.la.x)[l] = reinterpret_cast<const f4 *>(a.x)[g];
        reinterpret_cast<f4 *>(S.la.v)[l] = reinterpret_cast<const f4 *>(a.v)[g];
        reinterpret_cast<f4 *>(S.la.p)[l] = reinterpret_cast<const f4 *>(a.p)[g];
    }
    for (uint32_t q = threadIdx.x; q < nql; q += LANES) {
        reinterpret_cast<f4 *>(S.la.pf)[q] = reinterpret_cast<const f4 *>(a.pf)[S.q_lo + q];
        reinterpret_cast<uint32_t *>(S.la.pend)[q] = reinterpret_cast<const uint32_t *>(a.pend)[S.q_lo + q];
    }
    __syncthreads();
}

template <int LANES>
__device__ void staged_store(const SwarmArgs &a, const Staged &S)
{
    const uint32_t nql = S.nql;
    for (uint32_t e = threadIdx.x; e < (uint32_t)a.D * nql; e += LANES) {
        const uint32_t d = e / nql, q = e - d * nql;
        const size_t g = (size_t)d * a.Np / 4 + S.q_lo + q, l = (size_t)d * nql + q;
        reinterpret_cast<f4 *>(a.x)[g] = reinterpret_cast<const f4 *>(S.la.x)[l];
        reinterpret_cast<f4 *>(a.v)[g] = reinterpret_cast<const f4 *>(S.la.v)[l];
        reinterpret_cast<f4 *>(a.p)[g] = reinterpret_cast<const f4 *>(S.la.p)[l];
    }
    for (uint32_t q = threadIdx.x; q < nql; q += LANES) {
        reinterpret_cast<f4 *>(a.pf)[S.q_lo + q] = reinterpret_cast<const f4 *>(S.la.pf)[q];
        reinterpret_cast<uint32_t *>(a.pend)[S.q_lo + q] = reinterpret_cast<const uint32_t *>(S.la.pend)[q];
    }
}

// workgroup_min for the staged iteration: a wavefront with one candidate
// (the usual case once the gbest changes rarely) reads it from that lane
// instead of taking the butterfly.  Same contract: *wg_min holds NO_KEY
// before the call; ends with a barrier; the minimum in every lane.
__device__ __forceinline__ unsigned long long workgroup_min_sparse(unsigned long long key, unsigned long long thr,
                                                                   unsigned long long *wg_min)
{
    const unsigned long long c = __ballot(key < thr);
    if (c) {
        unsigned long long m;
        if ((c & (c - 1)) == 0) {
            const int l = __builtin_ctzll(c);
            m = ((unsigned long long)__builtin_amdgcn_readlane((uint32_t)(key >> 32), l) << 32) |
                __builtin_amdgcn_readlane((uint32_t)key, l);
        } else {
            m = wave_min_u64(key < thr ? key : NO_KEY);
        }
        if ((threadIdx.x & 63) == 0) atomicMin(wg_min, m);
    }
    __syncthreads();
    return *wg_min;
}

// Up to T iterations of a staged part after L.t, stopping after the first
// iteration at which the stop rule (tol, fstar) holds (tested before the
// first one too); a part of several meets the others every iteration.
// hist (may be null) receives each iteration's gbest key.  Returns this
// lane's pbest improvements.  PAIR: swarms with D <= 2 take the loop that
// runs a particle whole in one lane (the one-workgroup run; the batched
// kernels, which hold every fitness function in one kernel, keep the
// general loop and its register budget).
template <int FIT, int LANES, bool PAIR = false>
__device__ uint32_t staged_iterate(const SwarmArgs &a, const Staged &S, const Part &P, long long T, float tol,
                                   float fstar, float *s_g, const float *s_shift, Scratch *sc,
                                   unsigned long long *hist, SwarmLoop &L)
{
    constexpr int W = Fitness<FIT>::STAGE_WORDS;
    const int D = a.D;
    const SwarmArgs &la = S.la;
    float *s_t0 = S.t0, *s_t1 = S.t1;
    const uint32_t pitch = S.pitch, ibase = S.ibase;
    const uint32_t npairs = (uint32_t)(D + 1) / 2;
    uint32_t n_imp = 0;
    // A part of several computes the gbest-independent half of the next
    // iteration's Eq. 1 -- the Philox draws, (w v) + ((c1 r1)(p - x)) into
    // v's slot and c2 r2 into the first term slot, the pending pbest
    // positions copied -- while the other parts arrive, and finishes it once
    // the gbest is known.  With a stop rule the next iteration may not run:
    // then v keeps that half-updated value, but a stopped swarm never runs
    // again (a batch or server swarm only runs again after Step 1) and its
    // results -- gbest value, index, iteration, position and iterations run
    // -- do not read v.
    // the next iteration's own half between the meeting's two halves (the
    // batched parts); the single-swarm gang (PAIR) updates whole particles
    const bool split = !PAIR && P.parts > 1;
    auto own_half = [&](uint32_t tn) {
        for (GridWalk<LANES> gw(pitch); gw.row < npairs; gw.next()) {
            const uint32_t pr = gw.row, sidx = gw.col;
            const bool pend = la.pend[sidx] != 0;
            const U4 u = philox4x32_10(a.k0, a.k1, pr, ibase + sidx, tn, TAG_VEL);
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int d = 2 * (int)pr + h;
                if (d >= D) break;
                const size_t e = (size_t)d * pitch + sidx;
                const float x = la.x[e];
                const float p = pend ? x : la.p[e];
                la.v[e] = velocity_eq1_own(la, x, la.v[e], p, unit_float(word_r1(u, h)));
                s_t0[e] = a.c2 * unit_float(word_r2(u, h));
                if (pend) la.p[e] = p;
            }
        }
    };
    // Step 5 and the stop rule once the lanes have taken iteration t (key:
    // the lane's least improved pbest key); ends with a barrier
    auto end_iteration = [&](uint32_t t, unsigned long long key, long long n) {
        const unsigned long long m = workgroup_min_sparse(key, L.gkey, &sc->min[t & 1]);
        if (threadIdx.x == 0) sc->min[(t + 1) & 1] = NO_KEY;
        unsigned long long g = m;
        uint32_t owner = 0;
        if (P.parts > 1) {
            if (m != NO_KEY) stage_candidate<LANES>(P, t, D, la.x, pitch, (uint32_t)m - ibase);
            gang_post<LANES>(P, t, m);
            if (split && n + 1 < T) own_half(t + 1);
            g = gang_wait<LANES>(P, t, sc, &owner);
        }
        if (g < L.gkey) {
            L.gkey = g;
            L.giter = t;
            if (P.parts == 1) {
                const uint32_t mi = (uint32_t)g - ibase;
                for (int d = threadIdx.x; d < D; d += LANES) s_g[d] = la.x[(size_t)d * pitch + mi];
            } else {
                gather_gbest<LANES>(a, P, t, g, owner, s_g, sc);
            }
        }
        if (hist && threadIdx.x == 0) hist[t & (HIST_CAP - 1)] = L.gkey;
        L.t = t;
        L.stop = meets_tol(L.gkey, tol, fstar);
        __syncthreads();
    };
    // the clamp bounds in vector registers for the whole call (a select
    // between a lane value and a scalar operand costs a move per use)
    SwarmArgs lv = la;
    asm volatile("" : "+v"(lv.vmax), "+v"(lv.lo), "+v"(lv.hi));
    L.stop = L.stop || meets_tol(L.gkey, tol, fstar);
    if (PAIR && !split && npairs == 1) {
        // D <= 2: a lane takes its particles whole, the fitness summed in
        // registers (add(z, d) = stage then fold), then Step 4; no staged
        // terms and no barrier between the update and the fold.
        for (long long n = 0; n < T && !L.stop; ++n) {
            const uint32_t t = (uint32_t)(L.t + 1);
            unsigned long long key = NO_KEY;
            for (uint32_t sidx = threadIdx.x; sidx < pitch; sidx += LANES) {
                const uint32_t i = ibase + sidx;
                const bool pend = la.pend[sidx] != 0;
                const U4 u = philox4x32_10(a.k0, a.k1, 0u, i, t, TAG_VEL);
                Fitness<FIT> fit;
#pragma unroll
                for (int d = 0; d < 2; ++d) {
                    if (d >= D) break;
                    const size_t e = (size_t)d * pitch + sidx;
                    const float x = la.x[e], v = la.v[e];
                    const float p = pend ? x : la.p[e];
                    const float nv =
                        velocity_eq1(lv, x, v, p, s_g[d], unit_float(word_r1(u, d)), unit_float(word_r2(u, d)));
                    const float xn = position_eq2(lv, x, nv);
                    la.x[e] = xn;
                    la.v[e] = nv;
                    if (pend) la.p[e] = p;
                    fit.add(xn - s_shift[d], d);
                }
                bool imp = false;
                if (i < a.N) {
                    const float f = fit.value(D);
                    imp = f < la.pf[sidx];
                    if (imp) {
                        la.pf[sidx] = f;
                        const unsigned long long kk = make_key(f, i);
                        key = kk < key ? kk : key;
                        ++n_imp;
                    }
                }
                la.pend[sidx] = imp ? 1 : 0;
            }
            end_iteration(t, key, n);
        }
        return n_imp;
    }
    if (split && T > 0 && !L.stop) own_half((uint32_t)(L.t + 1));
    for (long long n = 0; n < T && !L.stop; ++n) {
        const uint32_t t = (uint32_t)(L.t + 1);
        if (split) {
            // (1') the social half of Eq. 1 and Eq. 2; fitness terms staged
            __syncthreads(); // own_half's stores before they are read
            for (GridWalk<LANES> gw(pitch); gw.row < (uint32_t)D; gw.next()) {
                const uint32_t d = gw.row;
                const size_t e = (size_t)d * pitch + gw.col;
                const float x = la.x[e];
                const float nv = velocity_eq1_social(lv, la.v[e], s_t0[e], x, s_g[d]);
                const float xn = position_eq2(lv, x, nv);
                la.x[e] = xn;
                la.v[e] = nv;
                float t0 = 0.0f, t1 = 0.0f;
                Fitness<FIT>::stage(xn - s_shift[d], &t0, &t1);
                s_t0[e] = t0;
                if constexpr (W == 2) s_t1[e] = t1;
            }
        } else {
            // (1) Eq. 1 and Eq. 2 per (particle, dimension pair); fitness terms staged
            for (GridWalk<LANES> gw(pitch); gw.row < npairs; gw.next()) {
                const uint32_t pr = gw.row, sidx = gw.col;
                const bool pend = la.pend[sidx] != 0;
                const U4 u = philox4x32_10(a.k0, a.k1, pr, ibase + sidx, t, TAG_VEL);
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const int d = 2 * (int)pr + h;
                    if (d >= D) break;
                    const size_t e = (size_t)d * pitch + sidx;
                    const float x = la.x[e], v = la.v[e];
                    const float p = pend ? x : la.p[e];
                    const float nv =
                        velocity_eq1(lv, x, v, p, s_g[d], unit_float(word_r1(u, h)), unit_float(word_r2(u, h)));
                    const float xn = position_eq2(lv, x, nv);
                    la.x[e] = xn;
                    la.v[e] = nv;
                    if (pend) la.p[e] = p;
                    float t0 = 0.0f, t1 = 0.0f;
                    Fitness<FIT>::stage(xn - s_shift[d], &t0, &t1);
                    s_t0[e] = t0;
                    if constexpr (W == 2) s_t1[e] = t1;
                }
            }
        }
        __syncthreads();
        // (2) fold in dimension order; Step 4 (strict improvement, NaN never improves)
        unsigned long long key = NO_KEY;
        for (uint32_t sidx = threadIdx.x; sidx < pitch; sidx += LANES) {
            const uint32_t i = ibase + sidx;
            bool imp = false;
            if (i < a.N) {
                const float f = fold_terms<FIT>(s_t0, s_t1, pitch, sidx, D);
                imp = f < la.pf[sidx];
                if (imp) {
                    la.pf[sidx] = f;
                    const unsigned long long kk = make_key(f, i);
                    key = kk < key ? kk : key;
                    ++n_imp;
                }
            }
            la.pend[sidx] = imp ? 1 : 0;
        }
        end_iteration(t, key, n);
    }
    return n_imp;
}

template <int FIT, int LANES>
__device__ void staged_part(const BatchItem &it, uint32_t part, uint32_t fixed_iters, BatchResult *res,
                            long long chunk, long long iter_cap, float *s_g, float *s_shift, Scratch *sc,
                            float *s_state, BatchResult *out_state, float *out_pos, uint32_t out, int pos_stride)
{
    static_assert(Fitness<FIT>::STAGE_WORDS == staged_words(FIT), "staged LDS sizing");
    const SwarmArgs &a = it.a;
    const int D = a.D;
    const uint32_t nq = (a.N + 3) / 4, nqi = a.Np / 4;
    Part P;
    P.parts = it.parts;
    P.part = part;
    P.q_lo = (uint32_t)((unsigned long long)nq * part / it.parts);
    P.q_hi = (uint32_t)((unsigned long long)nq * (part + 1) / it.parts);
    P.qi_lo = P.q_lo;
    P.qi_hi = part + 1 == it.parts ? nqi : P.q_hi;
    P.gang = it.gang;
    P.cand_key = it.cand_key;
    P.cand_pos = it.cand_pos;
    for (int d = threadIdx.x; d < D; d += LANES) s_shift[d] = a.shift[d];
    if (threadIdx.x == 0) {
        sc->min[0] = NO_KEY;
        sc->min[1] = NO_KEY;
    }
    SwarmLoop L;
    const bool started = res->started != 0u;
    __syncthreads();
    if (!started) {
        L.stop = false;
        block_init<FIT, LANES>(a, P, s_shift, s_g, sc, L);
    } else {
        L.gkey = res->gkey;
        L.giter = res->giter;
        L.t = res->iters;
        L.stop = res->stop != 0u;
        for (int d = threadIdx.x; d < D; d += LANES) s_g[d] = a.gpos[d];
    }
    const Staged S = staged_view<FIT>(a, s_state, P.q_lo, P.q_hi);
    staged_load<LANES>(a, S);
    const long long left = it.max_iter - L.t;
    const long long nd = (long long)a.N * a.D;
    long long iters = chunk / nd;
    iters = iters < 1 ? 1 : (iters > iter_cap ? iter_cap : iters);
    if (fixed_iters > 0) iters = fixed_iters;
    const unsigned long long c0 = wall_clock64();
    staged_iterate<FIT, LANES>(a, S, P, left < iters ? left : iters, it.tol, it.fstar, s_g, s_shift, sc, nullptr, L);
    const unsigned long long ticks = wall_clock64() - c0;
    staged_store<LANES>(a, S);
    if (part == 0) {
        for (int d = threadIdx.x; d < D; d += LANES) {
            a.gpos[d] = s_g[d];
            if (out_pos) out_pos[(size_t)out * pos_stride + d] = s_g[d];
        }
        if (threadIdx.x == 0) {
            res->gkey = L.gkey;
            res->giter = L.giter;
            res->iters = L.t;
            res->stop = L.stop ? 1u : 0u;
            res->started = 1u;
            res->ticks = ticks > 0xFFFFFFFFull ? 0xFFFFFFFFu : (uint32_t)ticks;
            if (out_state) out_state[out] = *res;
        }
    }
}

// ---------------------------------------------------------------------------
// A single swarm's run with its whole state staged in one workgroup's LDS:
// k_block_run with the staged iteration (the pso_run path for swarms that
// fit; continues from and updates the control block).
// ---------------------------------------------------------------------------
template <int FIT, int LANES>
__global__ void __launch_bounds__(LANES) k_block_run_staged(SwarmArgs a, long long T)
{
    __shared__ Scratch sc;
    extern __shared__ float s_dyn[]; // gbest position, shift (D floats each, rounded up to 16 bytes), state
    Ctrl *c = a.ctrl;
    const int D = a.D;
    const int head = (D + 3) & ~3;
    float *s_g = s_dyn, *s_shift = s_dyn + head, *s_state = s_dyn + 2 * head;
    for (int d = threadIdx.x; d < D; d += LANES) {
        s_g[d] = a.gpos[d];
        s_shift[d] = a.shift[d];
    }
    if (threadIdx.x == 0) {
        sc.min[0] = NO_KEY;
        sc.min[1] = NO_KEY;
        sc.err = 0;
    }
    SwarmLoop L;
    L.gkey = c->gkey_prev;
    L.giter = c->giter;
    L.t = c->t;
    L.stop = c->stop != 0u;
    const float tol = c->tol, fstar = c->fstar;
    const Staged S = staged_view<FIT>(a, s_state, 0, (a.N + 3) / 4);
    staged_load<LANES>(a, S); // ends with a barrier (s_g, s_shift, sc too)
    const uint32_t n_imp =
        staged_iterate<FIT, LANES, true>(a, S, whole_swarm(a), T, tol, fstar, s_g, s_shift, &sc, a.hist, L);
    staged_store<LANES>(a, S);
    if (n_imp) atomicAdd(&c->improved, (unsigned long long)n_imp);
    for (int d = threadIdx.x; d < D; d += LANES) a.gpos[d] = s_g[d];
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
// A single swarm whose state does not fit one workgroup's LDS, run as a gang
// of co-resident workgroups (one per part, gridDim.x parts): each stages a
// contiguous slice of quads, iterates it in LDS with the staged iteration,
// and meets the others once per step through the step-tagged words (`words`:
// 4 * parts key words, then 2 * parts * D coordinate words, zero at launch).
// Continues from and updates the control block, as k_block_run_staged.
// ---------------------------------------------------------------------------
template <int FIT, int LANES>
__global__ void __launch_bounds__(LANES) k_gang_staged(SwarmArgs a, long long T, unsigned long long *words)
{
    __shared__ Scratch sc;
    extern __shared__ float s_dyn[]; // gbest position, shift (D floats each, rounded up to 16 bytes), state
    Ctrl *c = a.ctrl;
    const int D = a.D;
    const int head = (D + 3) & ~3;
    float *s_g = s_dyn, *s_shift = s_dyn + head, *s_state = s_dyn + 2 * head;
    for (int d = threadIdx.x; d < D; d += LANES) {
        s_g[d] = a.gpos[d];
        s_shift[d] = a.shift[d];
    }
    if (threadIdx.x == 0) {
        sc.min[0] = NO_KEY;
        sc.min[1] = NO_KEY;
        sc.err = 0;
    }
    // every part reads the control block before any part can finish: part 0
    // writes it back only after all parts have met at every step
    SwarmLoop L;
    L.gkey = c->gkey_prev;
    L.giter = c->giter;
    L.t = c->t;
    L.stop = c->stop != 0u;
    const float tol = c->tol, fstar = c->fstar;
    const uint32_t parts = gridDim.x, part = blockIdx.x, nq = (a.N + 3) / 4;
    Part P{};
    P.parts = parts;
    P.part = part;
    P.q_lo = (uint32_t)((unsigned long long)nq * part / parts);
    P.q_hi = (uint32_t)((unsigned long long)nq * (part + 1) / parts);
    P.qi_lo = P.q_lo;
    P.qi_hi = P.q_hi;
    P.cand_key = words;
    P.cand_pos = reinterpret_cast<float *>(words + (size_t)4 * parts);
    const Staged S = staged_view<FIT>(a, s_state, P.q_lo, P.q_hi);
    staged_load<LANES>(a, S); // ends with a barrier (s_g, s_shift, sc too)
    const uint32_t n_imp = staged_iterate<FIT, LANES, true>(a, S, P, T, tol, fstar, s_g, s_shift, &sc,
                                                            part == 0 ? a.hist : nullptr, L);
    staged_store<LANES>(a, S);
    if (n_imp) atomicAdd(&c->improved, (unsigned long long)n_imp);
    if (threadIdx.x == 0 && sc.err) atomicOr(&c->err, ERR_GANG_WAIT);
    if (part != 0) return;
    for (int d = threadIdx.x; d < D; d += LANES) a.gpos[d] = s_g[d];
    if (threadIdx.x == 0) {
        c->gkey = L.gkey;
        c->gkey_prev = L.gkey;
        c->pubkey = L.gkey;
        c->giter = L.giter;
        c->t = L.t;
        c->stop = L.stop ? 1u : 0u;
    }
}

__global__ void k_zero_words(unsigned long long *w, size_t n)
{
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        w[i] = 0ull;
}

template <int LANES>
__global__ void __launch_bounds__(LANES) k_batch(const BatchItem *items, const BatchEntry *entries,
                                                 BatchResult *results, uint32_t count, unsigned int *next,
                                                 long long chunk, long long iter_cap, BatchResult *out_state,
                                                 float *out_pos, int pos_stride, unsigned int *err)
{
    __shared__ Scratch sc;
    __shared__ uint32_t s_idx;
    extern __shared__ float s_dyn[]; // gbest position (maxD floats), then shift
    if (threadIdx.x == 0) sc.err = 0;
    for (;;) {
        if (threadIdx.x == 0) s_idx = atomicAdd(next, 1u);
        __syncthreads();
        const uint32_t j = s_idx;
        __syncthreads();
        if (j >= count) break; // uniform: every workgroup leaves once the list is drained
        const BatchEntry e = entries[j];
        const BatchItem &it = items[e.item];
        float *s_g = s_dyn, *s_shift = s_dyn + it.a.D;
        BatchResult *res = &results[e.item];
        switch (it.fitness) {
        case F_SPHERE: batch_part<F_SPHERE, LANES>(it, e.part, e.iters, res, chunk, iter_cap, s_g, s_shift, &sc, out_state, out_pos, e.out, pos_stride); break;
        case F_RASTRIGIN: batch_part<F_RASTRIGIN, LANES>(it, e.part, e.iters, res, chunk, iter_cap, s_g, s_shift, &sc, out_state, out_pos, e.out, pos_stride); break;
        case F_ROSENBROCK: batch_part<F_ROSENBROCK, LANES>(it, e.part, e.iters, res, chunk, iter_cap, s_g, s_shift, &sc, out_state, out_pos, e.out, pos_stride); break;
        case F_ACKLEY: batch_part<F_ACKLEY, LANES>(it, e.part, e.iters, res, chunk, iter_cap, s_g, s_shift, &sc, out_state, out_pos, e.out, pos_stride); break;
        default: batch_part<F_CUBIC, LANES>(it, e.part, e.iters, res, chunk, iter_cap, s_g, s_shift, &sc, out_state, out_pos, e.out, pos_stride); break;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0 && sc.err && err) atomicOr(err, 1u);
}

// The LDS-staged batched kernel: k_batch's work queue over staged parts.  The
// dynamic LDS holds the gbest position and shift (maxD floats each, rounded
// up to 16 bytes) and then the part's staged state.
__host__ __device__ constexpr int staged_head_floats(int maxD) { return 2 * ((maxD + 3) & ~3); }

template <int LANES>
__global__ void __launch_bounds__(LANES) k_batch_staged(const BatchItem *items, const BatchEntry *entries,
                                                        BatchResult *results, uint32_t count, unsigned int *next,
                                                        long long chunk, long long iter_cap, BatchResult *out_state,
                                                        float *out_pos, int pos_stride, unsigned int *err)
{
    __shared__ Scratch sc;
    __shared__ uint32_t s_idx;
    extern __shared__ float s_dyn[];
    float *s_state = s_dyn + staged_head_floats(pos_stride);
    if (threadIdx.x == 0) sc.err = 0;
    for (;;) {
        if (threadIdx.x == 0) s_idx = atomicAdd(next, 1u);
        __syncthreads();
        const uint32_t j = s_idx;
        __syncthreads();
        if (j >= count) break; // uniform: every workgroup leaves once the list is drained
        const BatchEntry e = entries[j];
        const BatchItem &it = items[e.item];
        float *s_g = s_dyn, *s_shift = s_dyn + ((pos_stride + 3) & ~3);
        BatchResult *res = &results[e.item];
        switch (it.fitness) {
        case F_SPHERE: staged_part<F_SPHERE, LANES>(it, e.part, e.iters, res, chunk, iter_cap, s_g, s_shift, &sc, s_state, out_state, out_pos, e.out, pos_stride); break;
        case F_RASTRIGIN: staged_part<F_RASTRIGIN, LANES>(it, e.part, e.iters, res, chunk, iter_cap, s_g, s_shift, &sc, s_state, out_state, out_pos, e.out, pos_stride); break;
        case F_ROSENBROCK: staged_part<F_ROSENBROCK, LANES>(it, e.part, e.iters, res, chunk, iter_cap, s_g, s_shift, &sc, s_state, out_state, out_pos, e.out, pos_stride); break;
        case F_ACKLEY: staged_part<F_ACKLEY, LANES>(it, e.part, e.iters, res, chunk, iter_cap, s_g, s_shift, &sc, s_state, out_state, out_pos, e.out, pos_stride); break;
        default: staged_part<F_CUBIC, LANES>(it, e.part, e.iters, res, chunk, iter_cap, s_g, s_shift, &sc, s_state, out_state, out_pos, e.out, pos_stride); break;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0 && sc.err && err) atomicOr(err, 1u);
}

uint32_t staged_parts(uint64_t N, int D, int fitness, int stage_kib, int grid_cap)
{
    if (stage_kib < 1 || D < 1 || N < 1) return 0;
    const uint64_t qmax = (uint64_t)stage_kib * 1024 / staged_quad_bytes(D, fitness);
    if (qmax < 1) return 0;
    const uint64_t nq = (N + 3) / 4;
    // part p takes quads [nq*p/parts, nq*(p+1)/parts): at most ceil(nq/parts) <= qmax
    const uint64_t parts = (nq + qmax - 1) / qmax;
    if (parts > MAX_STAGED_PARTS || parts > (uint64_t)std::max(1, grid_cap)) return 0;
    return (uint32_t)parts;
}

size_t batch_dynamic_lds(int maxD, int stage_kib)
{
    if (stage_kib > 0) return sizeof(float) * staged_head_floats(maxD) + (size_t)stage_kib * 1024;
    return 2 * sizeof(float) * maxD;
}

uint32_t parts_for(uint64_t N, int D, int grid_cap, const BatchShape &shape)
{
    const uint64_t work = N * (uint64_t)D;
    const uint64_t pw = (uint64_t)std::max<long long>(1, shape.part_work);
    uint64_t parts = (work + pw - 1) / pw;
    const uint64_t by_quads = ((N + 3) / 4) / (uint64_t)std::max(1, shape.lanes);
    parts = std::min<uint64_t>(parts, by_quads);
    parts = std::min<uint64_t>(parts, MAX_PARTS);
    parts = std::min<uint64_t>(parts, (uint64_t)std::max(1, grid_cap));
    return (uint32_t)std::max<uint64_t>(parts, 1);
}

bool batch_lanes_supported(int lanes, bool staged)
{
    if (staged) return lanes == 256 || lanes == 512 || lanes == 1024;
    return lanes == 64 || lanes == 128 || lanes == 256;
}

size_t gang_bytes(uint32_t parts, int D)
{
    if (parts <= 1) return 0;
    auto al = [](size_t b) { return (b + 255) & ~size_t(255); };
    // tagged words: two per key and one per coordinate, both parities
    return al(sizeof(GangSync)) + al(sizeof(unsigned long long) * 4 * parts) +
           al(sizeof(unsigned long long) * 2 * parts * (size_t)D);
}

void bind_gang(BatchItem *it, void *region, uint32_t parts)
{
    it->parts = parts < 1 ? 1 : parts;
    if (it->parts == 1) {
        it->gang = nullptr;
        it->cand_key = nullptr;
        it->cand_pos = nullptr;
        return;
    }
    auto al = [](size_t b) { return (b + 255) & ~size_t(255); };
    char *b = static_cast<char *>(region);
    it->gang = reinterpret_cast<GangSync *>(b);
    it->cand_key = reinterpret_cast<unsigned long long *>(b + al(sizeof(GangSync)));
    it->cand_pos = reinterpret_cast<float *>(b + al(sizeof(GangSync)) + al(sizeof(unsigned long long) * 4 * parts));
}

// ---------------------------------------------------------------------------
// Launchers.
// ---------------------------------------------------------------------------
// LDS bytes of k_block_run_staged for a swarm, or 0 when it does not fit
// one workgroup (or PSO_BLOCK_STAGED=0 in the environment).
static int device_lds_max()
{
    static const int lds_max = [] {
        int dev = 0, v = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
            return 0;
        return v;
    }();
    return lds_max;
}

static size_t block_staged_lds(int fitness, const SwarmArgs &a)
{
    const int lds_max = device_lds_max();
    const char *env = getenv("PSO_BLOCK_STAGED");
    if (env && !strcmp(env, "0")) return 0;
    const size_t lds = sizeof(float) * 2 * (((size_t)a.D + 3) & ~(size_t)3) +
                       (size_t)((a.N + 3) / 4) * staged_quad_bytes(a.D, fitness);
    return lds + 1024 <= (size_t)lds_max ? lds : 0;
}

bool block_run_suits(int fitness, const SwarmArgs &a)
{
    const char *env = getenv("PSO_BLOCK_STAGED");
    if (env && !strcmp(env, "0")) return true; // the unstaged one-workgroup run, for tests
    return block_staged_lds(fitness, a) > 0;
}

template <int FIT>
static hipError_t launch_block_staged(const SwarmArgs &a, long long T, size_t lds, hipStream_t stream)
{
    // 256 lanes while a swarm's (particle, dimension pair) items fill them,
    // else 1024
    const uint64_t items = (uint64_t)4 * ((a.N + 3) / 4) * (uint64_t)((a.D + 1) / 2);
    const void *f = items <= 256 ? reinterpret_cast<const void *>(k_block_run_staged<FIT, 256>)
                                 : reinterpret_cast<const void *>(k_block_run_staged<FIT, 1024>);
    // the most any swarm may ask for, so concurrent callers never lower it
    hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, device_lds_max() - 1024);
    if (e != hipSuccess) return e;
    if (items <= 256)
        hipLaunchKernelGGL((k_block_run_staged<FIT, 256>), dim3(1), dim3(256), lds, stream, a, T);
    else
        hipLaunchKernelGGL((k_block_run_staged<FIT, 1024>), dim3(1), dim3(1024), lds, stream, a, T);
    return hipGetLastError();
}

hipError_t launch_block_run(int fitness, const SwarmArgs &a, long long T, hipStream_t stream)
{
    if (const size_t lds_s = block_staged_lds(fitness, a)) {
        switch (fitness) {
        case F_SPHERE: return launch_block_staged<F_SPHERE>(a, T, lds_s, stream);
        case F_RASTRIGIN: return launch_block_staged<F_RASTRIGIN>(a, T, lds_s, stream);
        case F_ROSENBROCK: return launch_block_staged<F_ROSENBROCK>(a, T, lds_s, stream);
        case F_ACKLEY: return launch_block_staged<F_ACKLEY>(a, T, lds_s, stream);
        case F_CUBIC: return launch_block_staged<F_CUBIC>(a, T, lds_s, stream);
        default: return hipErrorInvalidValue;
        }
    }
    const size_t lds = 2 * sizeof(float) * a.D;
    switch (fitness) {
    case F_SPHERE: hipLaunchKernelGGL(k_block_run<F_SPHERE>, dim3(1), dim3(RUN_LANES), lds, stream, a, T); break;
    case F_RASTRIGIN: hipLaunchKernelGGL(k_block_run<F_RASTRIGIN>, dim3(1), dim3(RUN_LANES), lds, stream, a, T); break;
    case F_ROSENBROCK: hipLaunchKernelGGL(k_block_run<F_ROSENBROCK>, dim3(1), dim3(RUN_LANES), lds, stream, a, T); break;
    case F_ACKLEY: hipLaunchKernelGGL(k_block_run<F_ACKLEY>, dim3(1), dim3(RUN_LANES), lds, stream, a, T); break;
    case F_CUBIC: hipLaunchKernelGGL(k_block_run<F_CUBIC>, dim3(1), dim3(RUN_LANES), lds, stream, a, T); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}


// The gang: one particle per lane of 256, at least two parts, every part
// co-resident (checked against the occupancy).
constexpr int GANG_LANES = 256;
constexpr uint32_t GANG_MAX_PARTS = 256;
// D <= 2 takes the fused loop, larger D the staged general loop; past
// D = 16 the step launches keep up with the gang (Rastrigin, N = 16 384 and
// 65 536: D = 8 5.3 / 7.0 against 10.5 / 11.0 us per iteration, D = 31
// 13.4 / 15.2 against 12.4 / 16.0).  PSO_GANG_MAX_D in the environment
// moves the limit (up to 64).
constexpr int GANG_MAX_D = 16;

static const void *gang_kernel(int fitness)
{
    switch (fitness) {
    case F_SPHERE: return reinterpret_cast<const void *>(k_gang_staged<F_SPHERE, GANG_LANES>);
    case F_RASTRIGIN: return reinterpret_cast<const void *>(k_gang_staged<F_RASTRIGIN, GANG_LANES>);
    case F_ROSENBROCK: return reinterpret_cast<const void *>(k_gang_staged<F_ROSENBROCK, GANG_LANES>);
    case F_ACKLEY: return reinterpret_cast<const void *>(k_gang_staged<F_ACKLEY, GANG_LANES>);
    default: return reinterpret_cast<const void *>(k_gang_staged<F_CUBIC, GANG_LANES>);
    }
}

uint32_t gang_run_parts(int fitness, const SwarmArgs &a)
{
    const char *env = getenv("PSO_GANG");
    if (env && !strcmp(env, "0")) return 0;
    const char *max_d_env = getenv("PSO_GANG_MAX_D");
    const int max_d = max_d_env ? atoi(max_d_env) : GANG_MAX_D;
    if (a.D > max_d || a.D > 64 || fitness < F_SPHERE || fitness > F_CUBIC) return 0;
    const uint32_t nq = (a.N + 3) / 4;
    const uint32_t parts = (nq + GANG_LANES / 4 - 1) / (GANG_LANES / 4);
    if (parts < 2 || parts > GANG_MAX_PARTS) return 0;
    const size_t lds = sizeof(float) * 2 * (((size_t)a.D + 3) & ~(size_t)3) +
                       (size_t)((nq + parts - 1) / parts) * staged_quad_bytes(a.D, fitness);
    if (lds + sizeof(Scratch) + 1024 > (size_t)device_lds_max()) return 0;
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, gang_kernel(fitness), GANG_LANES, lds) != hipSuccess)
        return 0;
    return (uint64_t)per_cu * (uint64_t)cus >= parts ? parts : 0;
}

size_t gang_run_words(uint32_t parts, int D)
{
    return (size_t)4 * parts + (size_t)2 * parts * (size_t)D;
}

template <int FIT>
static hipError_t launch_gang_staged(const SwarmArgs &a, long long T, uint32_t parts, unsigned long long *words,
                                     hipStream_t stream)
{
    const uint32_t nq = (a.N + 3) / 4;
    const size_t lds = sizeof(float) * 2 * (((size_t)a.D + 3) & ~(size_t)3) +
                       (size_t)((nq + parts - 1) / parts) * staged_quad_bytes(a.D, FIT);
    // the most any swarm may ask for, so concurrent callers never lower it
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(k_gang_staged<FIT, GANG_LANES>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, device_lds_max() - 1024);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_zero_words, dim3(4), dim3(256), 0, stream, words, gang_run_words(parts, a.D));
    hipLaunchKernelGGL((k_gang_staged<FIT, GANG_LANES>), dim3(parts), dim3(GANG_LANES), lds, stream, a, T, words);
    return hipGetLastError();
}

hipError_t launch_gang_run(int fitness, const SwarmArgs &a, long long T, uint32_t parts, unsigned long long *words,
                           hipStream_t stream)
{
    switch (fitness) {
    case F_SPHERE: return launch_gang_staged<F_SPHERE>(a, T, parts, words, stream);
    case F_RASTRIGIN: return launch_gang_staged<F_RASTRIGIN>(a, T, parts, words, stream);
    case F_ROSENBROCK: return launch_gang_staged<F_ROSENBROCK>(a, T, parts, words, stream);
    case F_ACKLEY: return launch_gang_staged<F_ACKLEY>(a, T, parts, words, stream);
    case F_CUBIC: return launch_gang_staged<F_CUBIC>(a, T, parts, words, stream);
    default: return hipErrorInvalidValue;
    }
}

__global__ void __launch_bounds__(64) k_upload(const UploadRec *recs, uint32_t n, const float *pool, BatchItem *items,
                                                BatchResult *state)
{
    if (blockIdx.x >= n) return;
    const UploadRec &u = recs[blockIdx.x];
    if (threadIdx.x == 0) {
        items[u.slot] = u.item;
        state[u.slot] = u.state;
        if (u.reset_gang && u.item.gang) *u.item.gang = GangSync{};
    }
    if (u.reset_gang && u.item.gang) { // the meeting's tagged words
        const size_t nk = (size_t)4 * u.item.parts, np = (size_t)2 * u.item.parts * u.item.a.D;
        for (size_t w = threadIdx.x; w < nk; w += 64) u.item.cand_key[w] = 0ull;
        unsigned long long *pw = reinterpret_cast<unsigned long long *>(u.item.cand_pos);
        for (size_t w = threadIdx.x; w < np; w += 64) pw[w] = 0ull;
    }
    float *shift = const_cast<float *>(u.item.a.shift);
    for (int d = threadIdx.x; d < u.item.a.D; d += 64) shift[d] = pool[u.shift_at + d];
}

hipError_t launch_upload(const UploadRec *recs, uint32_t n, const float *pool, BatchItem *items, BatchResult *state,
                         hipStream_t stream)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_upload, dim3(n), dim3(64), 0, stream, recs, n, pool, items, state);
    return hipGetLastError();
}

hipError_t launch_batch_reset(const BatchItem *items, BatchResult *results, uint32_t count, unsigned int *next,
                              hipStream_t stream)
{
    if (count == 0) return hipSuccess;
    hipLaunchKernelGGL(k_batch_reset, dim3(count), dim3(64), 0, stream, items, results, count, next);
    return hipGetLastError();
}

template <int LANES>
static hipError_t launch_staged(const BatchItem *items, const BatchEntry *entries, BatchResult *results, uint32_t count,
                                unsigned int *next, int maxD, int grid, long long chunk, long long iter_cap,
                                hipStream_t stream, BatchResult *out_state, float *out_pos, unsigned int *err,
                                int stage_kib)
{
    // the kernel's dynamic-LDS limit was raised by batch_capacity (no
    // attribute call here: this launch may be captured into a graph)
    const size_t lds = batch_dynamic_lds(maxD, stage_kib);
    hipLaunchKernelGGL(k_batch_staged<LANES>, dim3(grid), dim3(LANES), lds, stream, items, entries, results, count,
                       next, chunk, iter_cap, out_state, out_pos, maxD, err);
    return hipGetLastError();
}

hipError_t launch_batch(const BatchItem *items, const BatchEntry *entries, BatchResult *results, uint32_t count,
                        unsigned int *next, int maxD, int grid, int lanes, long long chunk, long long iter_cap,
                        hipStream_t stream, BatchResult *out_state, float *out_pos, unsigned int *err, int stage_kib)
{
    if (!batch_lanes_supported(lanes, stage_kib > 0)) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_counter_reset, dim3(1), dim3(64), 0, stream, next);
    if (stage_kib > 0) {
        if (lanes == 1024)
            return launch_staged<1024>(items, entries, results, count, next, maxD, grid, chunk, iter_cap, stream,
                                       out_state, out_pos, err, stage_kib);
        if (lanes == 512)
            return launch_staged<512>(items, entries, results, count, next, maxD, grid, chunk, iter_cap, stream,
                                      out_state, out_pos, err, stage_kib);
        return launch_staged<256>(items, entries, results, count, next, maxD, grid, chunk, iter_cap, stream,
                                  out_state, out_pos, err, stage_kib);
    }
    const size_t lds = batch_dynamic_lds(maxD, 0);
    switch (lanes) {
    case 64:
        hipLaunchKernelGGL(k_batch<64>, dim3(grid), dim3(64), lds, stream, items, entries, results, count, next, chunk,
                           iter_cap, out_state, out_pos, maxD, err);
        break;
    case 128:
        hipLaunchKernelGGL(k_batch<128>, dim3(grid), dim3(128), lds, stream, items, entries, results, count, next,
                           chunk, iter_cap, out_state, out_pos, maxD, err);
        break;
    default:
        hipLaunchKernelGGL(k_batch<256>, dim3(grid), dim3(256), lds, stream, items, entries, results, count, next,
                           chunk, iter_cap, out_state, out_pos, maxD, err);
        break;
    }
    return hipGetLastError();
}

hipError_t batch_capacity(int maxD, int lanes, int *workgroups, int stage_kib)
{
    if (!batch_lanes_supported(lanes, stage_kib > 0)) return hipErrorInvalidValue;
    const size_t lds = batch_dynamic_lds(maxD, stage_kib);
    int per_cu = 0, dev = 0, cus = 0, lds_max = 0;
    hipError_t e;
    if ((e = hipGetDevice(&dev)) != hipSuccess) return e;
    if (stage_kib > 0) {
        if ((e = hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev)) != hipSuccess)
            return e;
        if (lds + 1024 > (size_t)lds_max) { // static LDS of the kernel included
            *workgroups = 0;
            return hipSuccess;
        }
        const void *f = lanes == 1024  ? reinterpret_cast<const void *>(k_batch_staged<1024>)
                        : lanes == 512 ? reinterpret_cast<const void *>(k_batch_staged<512>)
                                       : reinterpret_cast<const void *>(k_batch_staged<256>);
        // the most any batch may ask for (batches of other maxD share the kernel)
        if ((e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, lds_max - 1024)) != hipSuccess)
            return e;
        e = lanes == 1024  ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_batch_staged<1024>, 1024, lds)
            : lanes == 512 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_batch_staged<512>, 512, lds)
                           : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_batch_staged<256>, 256, lds);
    } else {
        e = lanes == 64    ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_batch<64>, 64, lds)
            : lanes == 128 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_batch<128>, 128, lds)
                           : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_batch<256>, 256, lds);
    }
    if (e != hipSuccess) return e;
    if ((e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess) return e;
    // A margin below the occupancy bound for anything else the device keeps
    // resident, so every launched workgroup is co-resident: three quarters
    // of it for the streamed kernel (several workgroups per compute unit, so
    // the quarter left out costs little), the workgroups of all but 8
    // compute units for the staged one (at most a few per compute unit,
    // where a quarter of the units left idle would cost a quarter of the
    // time: 4096-swarm batch, 572 ms with 192 of 256 units, 479 ms with 248).
    if (stage_kib > 0)
        *workgroups = per_cu * std::max(1, cus - 8);
    else
        *workgroups = std::max(1, per_cu * cus * 3 / 4);
    return hipSuccess;
}

// Staged KiB per workgroup that leave room, in a compute unit's LDS shared
// by `per_cu` workgroups, for each workgroup's gbest position and shift of
// maxD floats and its static LDS; at most 158 (per_cu = 1) or 78 (2).
int staged_kib_fitting(int maxD, int per_cu)
{
    const long long head = (long long)batch_dynamic_lds(maxD, 1) - 1024; // gbest position and shift
    const long long kib = ((long long)device_lds_max() / per_cu - 1024 - head) / 1024;
    return (int)std::max(0LL, std::min<long long>(kib, per_cu == 1 ? 158 : 78));
}

// Workgroups of a shape: grid > 0 as given (at most the capacity), 0 the
// capacity, -k the capacity / k.
hipError_t shape_grid(int maxD, const BatchShape &sh, int *grid)
{
    int cap = 0;
    hipError_t e = batch_capacity(maxD, sh.lanes, &cap, sh.stage_kib);
    if (e != hipSuccess) return e;
    if (cap < 1) { // a staged shape whose LDS does not fit a workgroup
        *grid = 0;
        return hipSuccess;
    }
    *grid = sh.grid > 0 ? std::min(sh.grid, cap) : sh.grid < 0 ? std::max(1, cap / -sh.grid) : cap;
    return hipSuccess;
}

hipError_t launch_clear_u32(unsigned int *p, hipStream_t stream)
{
    hipLaunchKernelGGL(k_counter_reset, dim3(1), dim3(64), 0, stream, p);
    return hipGetLastError();
}

} // namespace pso

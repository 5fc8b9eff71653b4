// pso_kernels.hip -- grid kernels of the global-best PSO step on gfx950.
//
// The paper gives each particle a thread (Sec. 2.2) over structure-of-arrays
// state (Sec. 4.1).  Here one lane owns four consecutive particles and walks
// their dimensions in order: each access moves 16 bytes per lane (1 KiB per
// wavefront) of one dimension's row, with non-temporal hints since the state
// streams through once per iteration, and the four particles' random numbers
// and fitness give the lane enough independent work to hide the loads.  One
// launch is one iteration: update (Eq. 1, Eq. 2, clamps), fitness and pbest
// (Alg. 1 Steps 2-4) are fused with the aggregation into the gbest (Step 5).
//
// Aggregation.  The paper's queue (Sec. 3.1, Alg. 2) appends, under an
// atomic counter, the threads whose fitness beats the gbest and lets one
// thread scan them; its queue-lock form (Sec. 3.2, Alg. 3) folds the block
// result into the global one under a spin lock.  Here a particle is a
// candidate only if its new pbest key beats the gbest key (the same rarity
// Alg. 2 exploits); a wavefront with a candidate takes its minimum by a
// butterfly over lanes, one lane folds it into a workgroup minimum in LDS,
// and a workgroup whose minimum beats the gbest issues one 64-bit atomicMin
// of the packed (fitness, index) key.  The index alone travels, as in
// Sec. 4.3.
//   - Synchronous variant: every particle of iteration t uses the gbest of
//     iteration t-1; the last workgroup to finish gathers the winner's
//     position for iteration t+1.
//   - Asynchronous variant (the lock-protected gbest of Sec. 3.2): a
//     workgroup that lowers the gbest publishes its position at once under a
//     seqlock, and workgroups that start later in the same iteration use it.
#include <algorithm>
#include <cstdlib>

#include "pso_aggregate.hpp"
#include "pso_quad.hpp"

// Launch-shape knobs of the step kernel (build-time; the defaults are the
// values measured best on gfx950).
#ifndef PSO_STEP_WAVES_PER_EU
#define PSO_STEP_WAVES_PER_EU 0 // 0: let the compiler choose the register budget
#endif
#ifndef PSO_STEP_EXACT_D
#define PSO_STEP_EXACT_D 1 // compile-time D for the common dimensions
#endif
#ifndef PSO_STEP_UNROLL
#define PSO_STEP_UNROLL 1 // unroll of the dimension-pair loop
#endif
#ifndef PSO_BLOCK
#define PSO_BLOCK 256
#endif
#ifndef PSO_ASYNC_PF
#define PSO_ASYNC_PF 0 // software prefetch of the next dimension pair in the asynchronous step
#endif
#ifndef PSO_STEP_ONE_K
#define PSO_STEP_ONE_K 8 // dimension pairs loaded ahead by the one-particle-per-lane step
#endif

// Bytes of the streamed state that may be kept resident in the memory-side
// cache (MI355X: 256 MiB of Infinity Cache in front of HBM).  Three quarters
// of it leaves room for pf, the pending marks and other traffic.  Up to twice
// the cache, keeping x alone still pays (part of it stays resident); beyond
// that everything streams.  Both limits are measured on gfx950.
#ifndef PSO_KEEP_BUDGET_MIB
#define PSO_KEEP_BUDGET_MIB 192
#endif
#ifndef PSO_KEEP_X_MAX_MIB
#define PSO_KEEP_X_MAX_MIB 512
#endif
// -1 chooses the cache policy from the state size; 0..7 forces one.
#ifndef PSO_CACHE_POLICY
#define PSO_CACHE_POLICY -1
#endif

#if PSO_STEP_WAVES_PER_EU > 0
#define PSO_STEP_ATTR __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(PSO_STEP_WAVES_PER_EU)))
#else
#define PSO_STEP_ATTR __launch_bounds__(BLOCK)
#endif

namespace pso {

constexpr int BLOCK = PSO_BLOCK;

static inline size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

Layout layout_of(uint64_t N, int D, bool control)
{
    Layout L;
    L.control = control;
    L.Np = (N + ROW_ALIGN - 1) / ROW_ALIGN * ROW_ALIGN;
    const uint64_t Np = L.Np;
    size_t o = 0;
    L.ctrl = o;  o += control ? align256(sizeof(Ctrl)) : 0;
    L.gpos = o;  o += align256(sizeof(float) * D);
    L.shift = o; o += align256(sizeof(float) * D);
    L.hist = o;  o += control ? align256(sizeof(unsigned long long) * HIST_CAP) : 0;
    L.aux = o;   o += control ? align256(sizeof(unsigned long long) * ((Np / 4 + BLOCK - 1) / BLOCK)) : 0;
    L.prog = o;  o += control ? align256(sizeof(uint32_t) * PERSIST_MAX_GRID) : 0;
    L.pf = o;    o += align256(sizeof(float) * Np);
    L.pend = o;  o += align256(Np);
    L.x = o;     o += align256(sizeof(float) * Np * (size_t)D);
    L.v = o;     o += align256(sizeof(float) * Np * (size_t)D);
    L.p = o;     o += align256(sizeof(float) * Np * (size_t)D);
    L.total = o;
    return L;
}

int cache_policy(uint64_t Np, int D)
{
    if (PSO_CACHE_POLICY >= 0) return PSO_CACHE_POLICY == 0 ? POL_STREAM
                                      : PSO_CACHE_POLICY == 1 ? POL_X
                                      : PSO_CACHE_POLICY == 3 ? POL_XV
                                                              : POL_ALL;
    const uint64_t row = sizeof(float) * Np * (uint64_t)D, budget = (uint64_t)PSO_KEEP_BUDGET_MIB << 20;
    if (3 * row <= budget) return POL_ALL;
    if (2 * row <= budget) return POL_XV;
    if (row <= ((uint64_t)PSO_KEEP_X_MAX_MIB << 20)) return POL_X;
    return POL_STREAM;
}

SwarmArgs bind(void *base, const Layout &L, uint64_t N, int D)
{
    char *b = static_cast<char *>(base);
    SwarmArgs a{};
    a.ctrl = L.control ? reinterpret_cast<Ctrl *>(b + L.ctrl) : nullptr;
    a.gpos = reinterpret_cast<float *>(b + L.gpos);
    a.shift = reinterpret_cast<const float *>(b + L.shift);
    a.hist = L.control ? reinterpret_cast<unsigned long long *>(b + L.hist) : nullptr;
    a.aux = L.control ? reinterpret_cast<unsigned long long *>(b + L.aux) : nullptr;
    a.prog = L.control ? reinterpret_cast<uint32_t *>(b + L.prog) : nullptr;
    a.pf = reinterpret_cast<float *>(b + L.pf);
    a.pend = reinterpret_cast<uint8_t *>(b + L.pend);
    a.x = reinterpret_cast<float *>(b + L.x);
    a.v = reinterpret_cast<float *>(b + L.v);
    a.p = reinterpret_cast<float *>(b + L.p);
    a.N = (uint32_t)N;
    a.Np = (uint32_t)L.Np;
    a.D = D;
    return a;
}


// Iteration epilogue, run by the last workgroup: history, counters, the stop
// rule and the gbest position for iteration t.  A changed gbest belongs to a
// particle whose pbest improved in this iteration, so its pbest position is
// its current position x.
__device__ void epilogue(const SwarmArgs &a, uint32_t t, bool first)
{
    Ctrl *c = a.ctrl;
    const unsigned long long k = __hip_atomic_load(&c->gkey, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const bool changed = first || k != c->gkey_prev;
    if (changed) {
        const size_t gi = (uint32_t)k;
        for (int d = threadIdx.x; d < a.D; d += BLOCK) a.gpos[d] = a.x[(size_t)d * a.Np + gi];
    }
    if (threadIdx.x == 0) {
        a.hist[t & (HIST_CAP - 1)] = k;
        if (changed) {
            c->giter = t;
            c->gkey_prev = k;
            c->pubkey = k;
        }
        c->t = t;
        c->arrive = 0;
        if (c->tol > 0.0f && __builtin_fabsf(key_fitness(k) - c->fstar) < c->tol) c->stop = 1u;
    }
}

// ---------------------------------------------------------------------------
// Control-block reset (stream-ordered, so a captured graph needs no memset).
// ---------------------------------------------------------------------------
__global__ void k_reset(SwarmArgs a)
{
    if (threadIdx.x != 0) return;
    Ctrl *c = a.ctrl;
    c->gkey = NO_KEY;
    c->improved = 0;
    c->tiles = 0;
    c->fresh = 0;
    c->arrive = 0;
    c->gkey_prev = NO_KEY;
    c->giter = 0;
    c->t = 0;
    c->t_run0 = 0;
    c->stop = 0;
    c->err = 0;
    c->tol = 0.0f;
    c->fstar = 0.0f;
    c->seq = 0;
    c->lock = 0;
    c->pubkey = NO_KEY;
}

// Arms the stop rule of a pso_run: records where the run starts and whether
// the gbest already meets the tolerance.
__global__ void k_arm(SwarmArgs a, float tol, float fstar)
{
    if (threadIdx.x != 0) return;
    Ctrl *c = a.ctrl;
    c->tol = tol;
    c->fstar = fstar;
    c->t_run0 = c->t;
    c->stop = (tol > 0.0f && __builtin_fabsf(key_fitness(c->gkey_prev) - fstar) < tol) ? 1u : 0u;
}

// ---------------------------------------------------------------------------
// Step 1 (Alg. 1) over the whole grid; lane q initialises particles 4q..4q+3
// (the padding past N included).
// ---------------------------------------------------------------------------
template <int FIT, int POL>
__global__ void __launch_bounds__(BLOCK) k_init(SwarmArgs a)
{
    __shared__ unsigned long long wg_min;
    __shared__ int last;
    extern __shared__ float s_shift[]; // D floats
    const int D = a.D;
    for (int d = threadIdx.x; d < D; d += BLOCK) s_shift[d] = a.shift[d];
    if (threadIdx.x == 0) wg_min = NO_KEY;
    __syncthreads();
    const uint32_t q = blockIdx.x * BLOCK + threadIdx.x;
    const unsigned long long key = (4 * q < a.Np) ? init_quad<FIT, POL>(a, D, q, s_shift) : NO_KEY;
    const unsigned long long m = workgroup_min(key, NO_KEY, &wg_min);
    publish_sync(a.ctrl, m, NO_KEY);
    if (arrive_last(a.ctrl, &last)) epilogue(a, 0u, true);
}

// ---------------------------------------------------------------------------
// One synchronous iteration t = (iterations completed) + 1 over the whole
// grid.  The gbest position and the shift vector are staged in LDS (each
// dimension's value is one broadcast read).  DC > 0 fixes D at compile time.
// ---------------------------------------------------------------------------
template <int FIT, int DC, int POL>
__global__ void PSO_STEP_ATTR k_step(SwarmArgs a)
{
    __shared__ unsigned long long wg_min;
    __shared__ unsigned int wg_count;
    __shared__ int flag;
    extern __shared__ float s_dyn[]; // gbest position (D floats), then shift (D floats)
    Ctrl *c = a.ctrl;
    if (c->stop) return;
    const int D = DC > 0 ? DC : a.D;
    float *s_g = s_dyn, *s_shift = s_dyn + D;
    const uint32_t t = (uint32_t)(c->t + 1);
    for (int d = threadIdx.x; d < D; d += BLOCK) {
        s_g[d] = a.gpos[d];
        s_shift[d] = a.shift[d];
    }
    if (threadIdx.x == 0) {
        wg_min = NO_KEY;
        wg_count = 0;
    }
    const unsigned long long thr = c->gkey_prev;
    __syncthreads();
    const uint32_t q = blockIdx.x * BLOCK + threadIdx.x;
    uint32_t n_imp = 0;
    const unsigned long long key =
        (4 * q < a.N) ? iterate_quad<FIT, DC, PSO_STEP_UNROLL, POL>(a, D, q, t, s_g, s_shift, &n_imp) : NO_KEY;
    count_improvements(c, n_imp, &wg_count);
    const unsigned long long m = workgroup_min(key, thr, &wg_min);
    flush_count(c, &wg_count);
    publish_sync(c, m, thr);
    if (arrive_last(c, &flag)) epilogue(a, t, false);
}

// ---------------------------------------------------------------------------
// One asynchronous iteration (the lock-protected gbest of Sec. 3.2, Alg. 3):
// a workgroup whose particles beat the gbest publishes the better gbest at
// once, and work that starts later in the same iteration uses it.
//
// The swarm is cut into tiles of BLOCK particle quads and each workgroup runs
// the tiles blockIdx.x, blockIdx.x + gridDim.x, ... one after another (with
// as many workgroups as tiles, all co-resident, every tile would start before
// any publish and the trajectory would be the synchronous one).  Every tile
// after a workgroup's first starts by reading the running gbest key.  If it
// is the key of the previous iteration's gbest, its position is gpos, as in
// the synchronous step.  If it is lower, a tile of this iteration published
// it, and the position is that particle's x: its pbest position, written
// once in this iteration before the key was published (release fence, then
// atomicMin) and not rewritten before the iteration ends.  So the packed
// (fitness, index) key is the whole publication -- the index locates the
// position, as in Sec. 4.3 -- and no lock is needed to keep key and position
// consistent.  The last workgroup copies the final gbest position to gpos,
// as the synchronous epilogue does.  Each tile is counted, and so is every
// tile that used a gbest published during the same iteration.
// ---------------------------------------------------------------------------
template <int FIT, int DC, int POL>
__global__ void PSO_STEP_ATTR k_step_async(SwarmArgs a, uint32_t tiles)
{
    __shared__ unsigned long long wg_min[2];
    __shared__ unsigned long long s_key;
    __shared__ unsigned int wg_count;
    __shared__ int flag;
    extern __shared__ float s_dyn[]; // gbest position (D floats), then shift (D floats)
    Ctrl *c = a.ctrl;
    if (c->stop) return;
    const int D = DC > 0 ? DC : a.D;
    float *s_g = s_dyn, *s_shift = s_dyn + D;
    const uint32_t t = (uint32_t)(c->t + 1);
    const unsigned long long start_key = c->gkey_prev; // the gbest after iteration t - 1; its position is gpos
    for (int d = threadIdx.x; d < D; d += BLOCK) {
        s_g[d] = a.gpos[d];
        s_shift[d] = a.shift[d];
    }
    if (threadIdx.x == 0) {
        wg_min[0] = NO_KEY;
        wg_min[1] = NO_KEY;
        wg_count = 0;
    }
    __syncthreads();
    unsigned long long thr = start_key; // the gbest whose position s_g holds
    uint32_t n_imp = 0, n_tiles = 0, n_fresh = 0;
    int slot = 0;
    for (uint32_t tile = blockIdx.x; tile < tiles; tile += gridDim.x, slot ^= 1) {
        // a workgroup's first tile uses the previous iteration's gbest, as
        // the synchronous step does; each later one reads the running key
        if (n_tiles > 0) {
            if (threadIdx.x == 0) s_key = __hip_atomic_load(&c->gkey, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __syncthreads();
            const unsigned long long k = s_key;
            if (k < thr) {
                // published during this iteration: the position is x of
                // particle k & 0xffffffff (coherent loads; their address
                // depends on the key)
                const size_t gi = (uint32_t)k;
                for (int d = threadIdx.x; d < D; d += BLOCK)
                    s_g[d] =
                        __hip_atomic_load(&a.x[(size_t)d * a.Np + gi], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                thr = k;
                __syncthreads();
            }
        }
        ++n_tiles;
        n_fresh += thr < start_key;
        const uint32_t q = tile * BLOCK + threadIdx.x;
        uint32_t n = 0;
        const unsigned long long key =
            (4 * q < a.N)
                ? iterate_quad<FIT, DC, PSO_STEP_UNROLL, POL, (PSO_ASYNC_PF != 0 || FIT == F_ACKLEY)>(a, D, q, t, s_g,
                                                                                                     s_shift, &n)
                : NO_KEY;
        n_imp += n;
        const unsigned long long m = workgroup_min(key, thr, &wg_min[slot]);
        if (threadIdx.x == 0) wg_min[slot ^ 1] = NO_KEY;
        publish_sync(c, m, thr);
    }
    count_improvements(c, n_imp, &wg_count);
    __syncthreads();
    flush_count(c, &wg_count);
    if (threadIdx.x == 0 && n_tiles) {
        atomicAdd(&c->tiles, (unsigned long long)n_tiles);
        if (n_fresh) atomicAdd(&c->fresh, (unsigned long long)n_fresh);
    }
    if (arrive_last(c, &flag)) epilogue(a, t, false);
}

// ---------------------------------------------------------------------------
// One particle per lane, for swarms with too few particles to give every SIMD
// several wavefronts at four per lane: the rows of the next K dimension pairs
// are loaded ahead (iterate_one), the aggregation is that of k_step.
// ---------------------------------------------------------------------------
template <int FIT, int DC, int K, int POL>
__global__ void PSO_STEP_ATTR k_step_one(SwarmArgs a)
{
    __shared__ unsigned long long wg_min;
    __shared__ unsigned int wg_count;
    __shared__ int flag;
    extern __shared__ float s_dyn[]; // gbest position (D floats), then shift (D floats)
    Ctrl *c = a.ctrl;
    if (c->stop) return;
    const int D = DC > 0 ? DC : a.D;
    float *s_g = s_dyn, *s_shift = s_dyn + D;
    const uint32_t t = (uint32_t)(c->t + 1);
    for (int d = threadIdx.x; d < D; d += BLOCK) {
        s_g[d] = a.gpos[d];
        s_shift[d] = a.shift[d];
    }
    if (threadIdx.x == 0) {
        wg_min = NO_KEY;
        wg_count = 0;
    }
    const unsigned long long thr = c->gkey_prev;
    __syncthreads();
    const uint32_t i = blockIdx.x * BLOCK + threadIdx.x;
    uint32_t n_imp = 0;
    const unsigned long long key = iterate_one<FIT, DC, K, POL>(a, D, i, i < a.N, t, s_g, s_shift, &n_imp);
    count_improvements(c, n_imp, &wg_count);
    const unsigned long long m = workgroup_min(key, thr, &wg_min);
    flush_count(c, &wg_count);
    publish_sync(c, m, thr);
    if (arrive_last(c, &flag)) epilogue(a, t, false);
}

// ---------------------------------------------------------------------------
// Staged fitness terms of the split step.  The fitness is a sequential sum
// over the dimensions (Fitness<FIT>::add), so it cannot be split across
// lanes; what can be is the work of each term.  Every term that does not
// depend on another dimension is computed by the lane that updates that
// dimension, and the folding lane only adds: Sphere z^2, Rastrigin and
// Cubic their term, Ackley z^2 and cos(2 pi z) (two independent sums).
// Rosenbrock's term of dimension d > 0 needs z_{d-1} as well; z itself is
// staged and the folding lane evaluates the terms (add()).  (Computing them
// in the updating lanes, with each chunk's last z in a boundary row for the
// next chunk's first term, was measured slower: 39.0 against 34.6 us per
// iteration at N = 65 536, D = 128.)  Each term is the same expression add()
// evaluates, so every sum is the same bits.
// ---------------------------------------------------------------------------
template <int FIT>
__device__ __forceinline__ float split_term(float z)
{
    if constexpr (FIT == F_SPHERE) return z * z;
    else if constexpr (FIT == F_RASTRIGIN) return z * z - 10.0f * cospi_f32(2.0f * z);
    else if constexpr (FIT == F_ACKLEY) return z * z;
    else if constexpr (FIT == F_CUBIC) {
        const float z2 = z * z;
        return ((z2 * z - 0.8f * z2) - 1000.0f * z) + 8000.0f;
    } else return z;
}

// acc + t[0] + t[pitch] + ... + t[(n - 1) * pitch], in that order, eight
// loads in flight.
__device__ __forceinline__ float fold_column(float acc, const float *t, uint32_t pitch, int n)
{
    int j = 0;
    for (; j + 8 <= n; j += 8) {
        float v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = t[(uint32_t)(j + u) * pitch];
#pragma unroll
        for (int u = 0; u < 8; ++u) acc = acc + v[u];
    }
    for (; j < n; ++j) acc = acc + t[(uint32_t)j * pitch];
    return acc;
}

// ---------------------------------------------------------------------------
// Split step, for swarms too small to fill the GPU at four particles per
// lane (at N = 65 536 the plain step has a quarter of a wavefront per SIMD).
// L lanes share a particle quad and each walks C consecutive dimensions of
// it (C even, so a chunk holds whole Philox pairs).  Lane t of the
// workgroup takes chunk t / Q of quad t % Q (Q = BLOCK / L quads per
// workgroup): the lanes of one chunk are consecutive, so a wavefront moves
// 256-byte row segments, and a 64-byte pbest group is four lanes of one
// chunk, as in the plain step.  Each lane stages its dimensions' fitness
// terms in LDS ([word][d][particle], one 16-byte store per quad, split_term
// above); after a barrier the folding lanes add them in dimension order, so
// the fitness is the same sequential sum as in the plain step, bit for bit.
// With H = 2 phases the dimensions are covered in two halves of L * C: each
// lane walks one chunk of each half, the terms of one half are staged at a
// time, and the folding lane carries its particle's running sum from the
// first half to the second -- the same additions in the same order, in half
// the LDS per particle.
//
// Every workgroup of the launch is resident at once, so the iteration ends
// when the workgroup whose loads were served last has folded, tested and
// published its particles: the work after the loads is on the critical path.
// So the folds are additions only (above), Ackley's two sums are folded by
// two lanes at once, the folding lanes are spread over the wavefronts, each
// folding lane reads its particle's pbest fitness before the update, and the
// first dimension pair's loads are issued before the barrier that publishes
// the gbest position and shift in LDS.
// ---------------------------------------------------------------------------
// At most 128 VGPRs (four wavefronts per SIMD): 1024 workgroups of 256 lanes,
// N = 65 536 at D = 128, are then resident at once.
template <int FIT, int POL, uint32_t H>
__global__ void __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(4)))
k_step_split(SwarmArgs a, uint32_t L, uint32_t C)
{
    __shared__ unsigned long long wg_min;
    __shared__ unsigned int wg_count;
    __shared__ int flag;
    extern __shared__ float s_dyn[]; // gbest position (D), shift (D), staged terms of one phase
    Ctrl *c = a.ctrl;
    if (c->stop) return;
    constexpr int W = Fitness<FIT>::STAGE_WORDS;
    constexpr bool KX = (POL & KEEP_X) != 0, KV = (POL & KEEP_V) != 0, KP = (POL & KEEP_P) != 0;
    constexpr uint32_t WAVES = BLOCK / 64;
    const int D = a.D;
    const size_t Np = a.Np;
    const uint32_t Q = BLOCK / L, P = 4 * Q;
    const int DP = H > 1 ? (int)(L * C) : D; // dimensions per phase
    float *s_g = s_dyn, *s_shift = s_dyn + D, *s_t0 = s_dyn + 2 * D, *s_t1 = s_t0 + (size_t)DP * P;
    const uint32_t t = (uint32_t)(c->t + 1);
    const uint32_t k = threadIdx.x / Q, qq = threadIdx.x % Q;
    const uint32_t q = blockIdx.x * Q + qq, i0 = 4 * q;
    const bool active = i0 < a.N;
    // Folding lanes.  With P <= BLOCK, particle slot j < P / WAVES of
    // wavefront w is particle w * P / WAVES + j; Ackley's second sum is
    // folded by lane j + 32 of the same wavefront where the slots fit in 32
    // lanes.  With P > BLOCK (one phase only) lane t folds particles t,
    // t + BLOCK, ... after the update.
    const bool spread = P <= BLOCK;
    const uint32_t per_wave = P / WAVES, lane = threadIdx.x & 63;
    const bool two = W == 2 && per_wave <= 32;
    const uint32_t slot = two ? (lane & 31u) : lane, word = two ? (lane >> 5) : 0u;
    const uint32_t fs = (threadIdx.x / 64) * per_wave + slot;
    const bool folder = spread && slot < per_wave && blockIdx.x * P + fs < a.N;
    const bool owner = folder && word == 0; // tests and writes the particle
    const float pf_old = owner ? a.pf[blockIdx.x * P + fs] : 0.0f;
    const uint32_t pend = active ? *reinterpret_cast<const uint32_t *>(a.pend + i0) : 0u;
    // the first dimension pair of the lane's first chunk, loaded before the
    // barrier below
    f4 ax[2], av[2], ap[2];
    {
        const int d_begin = (int)(k * C), d_end = min(D, (int)((k + 1) * C));
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            if (active && d_begin + h < d_end) {
                const size_t row = (size_t)(d_begin + h) * Np;
                ax[h] = ld_state<KX>(a.x + row, q);
                av[h] = ld_state<KV>(a.v + row, q);
                ap[h] = ld_state<KP>(a.p + row, q);
            }
        }
    }
    for (int d = threadIdx.x; d < D; d += BLOCK) {
        s_g[d] = a.gpos[d];
        s_shift[d] = a.shift[d];
    }
    if (threadIdx.x == 0) {
        wg_min = NO_KEY;
        wg_count = 0;
    }
    const unsigned long long thr = c->gkey_prev;
    __syncthreads();
    const bool line_dirty = group_dirty(pend);
    float acc = 0.0f, acc1 = 0.0f; // running sums of the folded particle (acc1: both words in one lane)
    Fitness<FIT> rfit;             // Rosenbrock: the folded particle's running fitness
#pragma unroll 1
    for (uint32_t ph = 0; ph < H; ++ph) {
        const int d_lo = (int)ph * DP; // first dimension of the phase
        const int d_begin = d_lo + (int)(k * C), d_end = min(D, d_lo + (int)((k + 1) * C));
        if (ph > 0) {
            __syncthreads(); // the previous phase's terms are folded
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                if (active && d_begin + h < d_end) {
                    const size_t row = (size_t)(d_begin + h) * Np;
                    ax[h] = ld_state<KX>(a.x + row, q);
                    av[h] = ld_state<KV>(a.v + row, q);
                    ap[h] = ld_state<KP>(a.p + row, q);
                }
            }
        }
        if (active) {
            // software pipeline over the chunk's dimension pairs, as in the
            // plain step: the next pair's rows are loaded before this pair's
            // stores
            for (int d = d_begin; d < d_end; d += 2) {
                f4 cx[2], cv[2], cp[2];
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    cx[h] = ax[h];
                    cv[h] = av[h];
                    cp[h] = ap[h];
                }
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    if (d + 2 + h < d_end) {
                        const size_t row = (size_t)(d + 2 + h) * Np;
                        ax[h] = ld_state<KX>(a.x + row, q);
                        av[h] = ld_state<KV>(a.v + row, q);
                        ap[h] = ld_state<KP>(a.p + row, q);
                    }
                }
                U4 u[4];
#pragma unroll
                for (int j = 0; j < 4; ++j) u[j] = philox4x32_10(a.k0, a.k1, (uint32_t)d >> 1, i0 + j, t, TAG_VEL);
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    if (h == 1 && d + 1 >= d_end) break;
                    const size_t row = (size_t)(d + h) * Np;
                    const f4 xn =
                        update_row<POL>(a, row, q, cx[h], cv[h], cp[h], pend, line_dirty, u, h, s_g[d + h]);
                    const float sh = s_shift[d + h];
                    f4 w0, w1;
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        const float z = xn[j] - sh;
                        w0[j] = split_term<FIT>(z);
                        if constexpr (W == 2) w1[j] = cospi_f32(2.0f * z);
                    }
                    const size_t at = (size_t)(d + h - d_lo) * P + 4 * qq;
                    *reinterpret_cast<f4 *>(s_t0 + at) = w0;
                    if constexpr (W == 2) *reinterpret_cast<f4 *>(s_t1 + at) = w1;
                }
            }
        }
        __syncthreads();
        if (folder) {
            const int n = min(DP, D - d_lo);
            if constexpr (FIT == F_ROSENBROCK) {
                fold_range<FIT>(rfit, s_t0, s_t1, P, fs, d_lo, n);
            } else {
                acc = fold_column(acc, (word ? s_t1 : s_t0) + fs, P, n);
                if (W == 2 && !two) acc1 = fold_column(acc1, s_t1 + fs, P, n);
            }
        }
    }
    // Step 4: strict improvement of each folded particle
    unsigned long long key = NO_KEY;
    uint32_t n_imp = 0;
    if (spread) {
        const float other = __shfl(acc, (int)((lane + 32) & 63), 64); // Ackley's second sum, from lane + 32
        if (owner) {
            const uint32_t i = blockIdx.x * P + fs;
            Fitness<FIT> fit = rfit;
            if constexpr (FIT != F_ROSENBROCK) {
                fit.acc = acc;
                fit.aux = two ? other : acc1;
            }
            const float f = fit.value(D);
            const bool imp = f < pf_old;
            if (imp) {
                a.pf[i] = f;
                key = make_key(f, i);
                n_imp = 1;
            }
            a.pend[i] = imp ? 1 : 0;
        }
    } else {
        for (uint32_t sidx = threadIdx.x; sidx < P; sidx += BLOCK) {
            const uint32_t i = blockIdx.x * P + sidx;
            if (i >= a.N) break;
            Fitness<FIT> fit;
            if constexpr (FIT == F_ROSENBROCK) {
                fold_range<FIT>(fit, s_t0, s_t1, P, sidx, 0, D);
            } else {
                fit.acc = fold_column(0.0f, s_t0 + sidx, P, D);
                if constexpr (W == 2) fit.aux = fold_column(0.0f, s_t1 + sidx, P, D);
            }
            const float f = fit.value(D);
            const bool imp = f < a.pf[i];
            if (imp) {
                a.pf[i] = f;
                const unsigned long long kk = make_key(f, i);
                key = kk < key ? kk : key;
                ++n_imp;
            }
            a.pend[i] = imp ? 1 : 0;
        }
    }
    count_improvements(c, n_imp, &wg_count);
    const unsigned long long m = workgroup_min(key, thr, &wg_min);
    flush_count(c, &wg_count);
    publish_sync(c, m, thr);
    if (arrive_last(c, &flag)) epilogue(a, t, false);
}

// ---------------------------------------------------------------------------
// Fully asynchronous persistent run (the further asynchronous scheme the
// paper leaves to future work, Sec. 6): one launch runs T iterations.  Every
// workgroup owns a fixed slice of particle quads and iterates it on its own:
// it reads the published gbest as a consistent snapshot (seqlock, as the
// asynchronous step), updates its particles with Philox counter t = its own
// iteration count (so each particle draws the same numbers as in any other
// variant), and publishes a better gbest at once.  No barrier separates
// iterations.  Staleness is bounded: before iteration k a workgroup waits
// until every workgroup has finished k - 1 - max_lead iterations (the grid is
// fully co-resident, so the slowest always progresses; the wait is bounded
// by the wall clock and sets an error bit if it gives up).  Any workgroup
// that sees the stop rule met stops them all.
// ---------------------------------------------------------------------------
constexpr unsigned long long PERSIST_WAIT_TICKS = 2000000000ull; // 20 s of the 100 MHz wall clock

// Waits (first wavefront) until every workgroup's iteration count is at
// least `need`; false in every lane if the wait gave up.  Uniform call.
__device__ bool wait_watermark(const uint32_t *prog, uint32_t need, uint32_t *s_seen, int *s_ok, Ctrl *c)
{
    if (*s_seen >= need) return true;
    if (threadIdx.x < 64) {
        const unsigned long long t0 = wall_clock64();
        for (;;) {
            uint32_t m = 0xFFFFFFFFu;
            for (uint32_t b = threadIdx.x; b < gridDim.x; b += 64) {
                const uint32_t v = __hip_atomic_load(&prog[b], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                m = v < m ? v : m;
            }
#pragma unroll
            for (int off = 32; off >= 1; off >>= 1) {
                const uint32_t o = __shfl_xor(m, off, 64);
                m = o < m ? o : m;
            }
            if (m >= need) {
                if (threadIdx.x == 0) {
                    *s_seen = m;
                    *s_ok = 1;
                }
                break;
            }
            // a workgroup that stopped (stop rule, or a wait that gave up)
            // will not reach `need`: stop too
            if (__hip_atomic_load(&c->stop, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u) {
                if (threadIdx.x == 0) *s_ok = 0;
                break;
            }
            if (wall_clock64() - t0 > PERSIST_WAIT_TICKS) {
                if (threadIdx.x == 0) {
                    atomicOr(&c->err, ERR_STALE_WAIT);
                    __hip_atomic_store(&c->stop, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    *s_ok = 0;
                }
                break;
            }
            __builtin_amdgcn_s_sleep(2);
        }
    }
    __syncthreads();
    return *s_ok != 0;
}

template <int FIT, int POL>
__global__ void PSO_STEP_ATTR k_persist(SwarmArgs a, uint32_t T, uint32_t max_lead, uint32_t qpw)
{
    __shared__ unsigned long long wg_min;
    __shared__ unsigned long long snap_key;
    __shared__ uint32_t s_seen;
    __shared__ int flag, s_go, s_ok;
    extern __shared__ float s_dyn[]; // gbest snapshot (D floats), then shift
    Ctrl *c = a.ctrl;
    const int D = a.D;
    float *s_g = s_dyn, *s_shift = s_dyn + D;
    for (int d = threadIdx.x; d < D; d += BLOCK) s_shift[d] = a.shift[d];
    if (threadIdx.x == 0) s_seen = 0;
    const long long t0 = c->t;
    const float tol = c->tol, fstar = c->fstar;
    const uint32_t nq = (a.N + 3) / 4;
    const uint32_t q_lo = blockIdx.x * qpw, q_hi = min(nq, q_lo + qpw);
    uint32_t n_imp = 0, done = 0;
    __syncthreads();
    for (uint32_t k = 1; k <= T; ++k) {
        if (threadIdx.x == 0) {
            s_go = __hip_atomic_load(&c->stop, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0u;
            wg_min = NO_KEY;
        }
        __syncthreads();
        if (!s_go) break;
        if (max_lead < T && k > max_lead + 1 && !wait_watermark(a.prog, k - 1 - max_lead, &s_seen, &s_ok, c)) break;
        const uint32_t t = (uint32_t)(t0 + k);
        const unsigned long long thr = snapshot_async(a, s_g, &snap_key); // ends with a barrier
        unsigned long long key = NO_KEY;
        for (uint32_t q = q_lo + threadIdx.x; q < q_hi; q += BLOCK) {
            uint32_t n = 0;
            const unsigned long long kk = iterate_quad<FIT, 0, 1, POL>(a, D, q, t, s_g, s_shift, &n);
            key = kk < key ? kk : key;
            n_imp += n;
        }
        const unsigned long long m = workgroup_min(key, thr, &wg_min);
        publish_async(a, m, thr, &flag);
        __syncthreads();
        done = k;
        if (threadIdx.x == 0) {
            if (m < thr && flag) atomicMax(reinterpret_cast<unsigned long long *>(&c->giter), (unsigned long long)t);
            __hip_atomic_store(&a.prog[blockIdx.x], k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            const unsigned long long g = __hip_atomic_load(&c->gkey, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            // history: the best key seen when a workgroup finished iteration t
            atomicMin(&a.hist[t & (HIST_CAP - 1)], g);
            if (tol > 0.0f && __builtin_fabsf(key_fitness(g) - fstar) < tol)
                __hip_atomic_store(&c->stop, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
    // bookkeeping: improvements, iteration count (the furthest workgroup's),
    // and from the last workgroup to finish the gbest of the run
    __shared__ unsigned int wg_count;
    if (threadIdx.x == 0) wg_count = 0;
    __syncthreads();
    count_improvements(c, n_imp, &wg_count);
    __syncthreads();
    flush_count(c, &wg_count);
    if (threadIdx.x == 0)
        atomicMax(reinterpret_cast<unsigned long long *>(&c->t), (unsigned long long)(t0 + done));
    if (threadIdx.x == 0) __threadfence();
    if (arrive_last(c, &flag) && threadIdx.x == 0) {
        const unsigned long long g = __hip_atomic_load(&c->gkey, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        c->gkey_prev = g;
        c->arrive = 0;
    }
}

// ---------------------------------------------------------------------------
// The paper's comparator (Sec. 2.2, Fig. 1): a two-kernel parallel
// reduction.  Kernel 1 updates the particles and reduces every particle's
// pbest key over its block with a shared-memory tree (log2 of the block
// size steps, a barrier each; UNROLLED ends with the last wavefront's steps
// unrolled without barriers) into an auxiliary array; kernel 2, one block,
// reduces the auxiliary array into the gbest.  Same results as the
// synchronous variant; two launches per iteration.
// ---------------------------------------------------------------------------
template <bool UNROLLED>
__device__ __forceinline__ unsigned long long tree_min(unsigned long long key, unsigned long long *sh)
{
    const int tid = threadIdx.x;
    sh[tid] = key;
    __syncthreads();
    const int stop = UNROLLED ? 64 : 1;
    for (int s = BLOCK / 2; s >= stop; s >>= 1) {
        if (tid < s) sh[tid] = sh[tid] < sh[tid + s] ? sh[tid] : sh[tid + s];
        __syncthreads();
    }
    if (UNROLLED && tid < 64) {
        // the last 64 keys: one wavefront, lanes in lockstep
        volatile unsigned long long *v = sh;
        unsigned long long m = v[tid];
#pragma unroll
        for (int s = 32; s >= 1; s >>= 1) {
            const unsigned long long o = __shfl_xor(m, s, 64);
            m = o < m ? o : m;
        }
        if (tid == 0) v[0] = m;
    }
    __syncthreads();
    return sh[0];
}

template <int FIT, int DC, bool UNROLLED, int POL>
__global__ void PSO_STEP_ATTR k_step_reduce(SwarmArgs a)
{
    __shared__ unsigned long long sh[BLOCK];
    extern __shared__ float s_dyn[];
    Ctrl *c = a.ctrl;
    if (c->stop) return;
    const int D = DC > 0 ? DC : a.D;
    float *s_g = s_dyn, *s_shift = s_dyn + D;
    const uint32_t t = (uint32_t)(c->t + 1);
    for (int d = threadIdx.x; d < D; d += BLOCK) {
        s_g[d] = a.gpos[d];
        s_shift[d] = a.shift[d];
    }
    __syncthreads();
    const uint32_t q = blockIdx.x * BLOCK + threadIdx.x;
    unsigned long long key = NO_KEY;
    if (4 * q < a.N) {
        iterate_quad<FIT, DC, PSO_STEP_UNROLL, POL>(a, D, q, t, s_g, s_shift);
        // every particle's pbest key, improved or not
        const f4 pf = *reinterpret_cast<const f4 *>(a.pf + 4 * q);
#pragma unroll
        for (int k = 0; k < 4; ++k)
            if (4 * q + k < a.N) {
                const unsigned long long kk = make_key(pf[k], 4 * q + k);
                key = kk < key ? kk : key;
            }
    }
    const unsigned long long m = tree_min<UNROLLED>(key, sh);
    if (threadIdx.x == 0) a.aux[blockIdx.x] = m;
}

template <bool UNROLLED>
__global__ void __launch_bounds__(BLOCK) k_reduce_final(SwarmArgs a, uint32_t nblocks)
{
    __shared__ unsigned long long sh[BLOCK];
    Ctrl *c = a.ctrl;
    if (c->stop) return;
    const uint32_t t = (uint32_t)(c->t + 1);
    unsigned long long key = NO_KEY;
    for (uint32_t b = threadIdx.x; b < nblocks; b += BLOCK) key = a.aux[b] < key ? a.aux[b] : key;
    const unsigned long long m = tree_min<UNROLLED>(key, sh);
    if (threadIdx.x == 0) c->gkey = m;
    __syncthreads();
    epilogue(a, t, false);
}

// ---------------------------------------------------------------------------
// Pending pbest positions: complete them (before the state is read) or drop
// the marks (after the state is replaced).
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(BLOCK) k_flush(SwarmArgs a)
{
    const uint32_t q = blockIdx.x * BLOCK + threadIdx.x;
    if (4 * q < a.Np) flush_quad(a, q);
}

__global__ void __launch_bounds__(BLOCK) k_clear_pending(SwarmArgs a)
{
    const uint32_t q = blockIdx.x * BLOCK + threadIdx.x;
    if (4 * q < a.Np) *reinterpret_cast<uint32_t *>(a.pend + 4 * q) = 0u;
}

// ---------------------------------------------------------------------------
// Launchers.  One lane per four particles.
// ---------------------------------------------------------------------------
static inline dim3 grid_of(const SwarmArgs &a) { return dim3((a.N + 4 * BLOCK - 1) / (4 * BLOCK)); }
static inline dim3 grid_all(const SwarmArgs &a) { return dim3((a.Np + 4 * BLOCK - 1) / (4 * BLOCK)); }

hipError_t launch_reset(const SwarmArgs &a, hipStream_t stream)
{
    hipLaunchKernelGGL(k_reset, dim3(1), dim3(64), 0, stream, a);
    return hipGetLastError();
}

hipError_t launch_arm(const SwarmArgs &a, float tol, float fstar, hipStream_t stream)
{
    hipLaunchKernelGGL(k_arm, dim3(1), dim3(64), 0, stream, a, tol, fstar);
    return hipGetLastError();
}

hipError_t launch_flush(const SwarmArgs &a, hipStream_t stream)
{
    hipLaunchKernelGGL(k_flush, grid_all(a), dim3(BLOCK), 0, stream, a);
    return hipGetLastError();
}

hipError_t launch_clear_pending(const SwarmArgs &a, hipStream_t stream)
{
    hipLaunchKernelGGL(k_clear_pending, grid_all(a), dim3(BLOCK), 0, stream, a);
    return hipGetLastError();
}

template <int FIT>
static void launch_init_f(const SwarmArgs &a, hipStream_t stream)
{
    const size_t lds = sizeof(float) * a.D;
    switch (cache_policy(a.Np, a.D)) {
    case POL_STREAM: hipLaunchKernelGGL((k_init<FIT, POL_STREAM>), grid_all(a), dim3(BLOCK), lds, stream, a); break;
    case POL_X: hipLaunchKernelGGL((k_init<FIT, POL_X>), grid_all(a), dim3(BLOCK), lds, stream, a); break;
    case POL_XV: hipLaunchKernelGGL((k_init<FIT, POL_XV>), grid_all(a), dim3(BLOCK), lds, stream, a); break;
    default: hipLaunchKernelGGL((k_init<FIT, POL_ALL>), grid_all(a), dim3(BLOCK), lds, stream, a); break;
    }
}

hipError_t launch_init(int fitness, const SwarmArgs &a, hipStream_t stream)
{
    switch (fitness) {
    case F_SPHERE: launch_init_f<F_SPHERE>(a, stream); break;
    case F_RASTRIGIN: launch_init_f<F_RASTRIGIN>(a, stream); break;
    case F_ROSENBROCK: launch_init_f<F_ROSENBROCK>(a, stream); break;
    case F_ACKLEY: launch_init_f<F_ACKLEY>(a, stream); break;
    case F_CUBIC: launch_init_f<F_CUBIC>(a, stream); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// Split shape (lanes per quad L, dimensions per lane C, phases H) for the
// step of a swarm, or false for the plain step.  The split step runs with C
// <= 8 (4 for Ackley's two staged words, keeping its LDS at 32 KiB) and L a
// power of two <= 64, for D >= 16.  It is chosen for N <= 2^17 (at most 512
// plain wavefronts, half a wavefront per SIMD) and, with two staged words,
// N*D <= 2^24: measured on gfx950 over N = 2^14..2^19, D = 16..256 for
// Rastrigin, Rosenbrock and Ackley, it is 1.1-8.9x faster there and slower
// beyond.  It runs in one phase: two phases of L / 2 lanes per quad (half
// the LDS per particle, twice the particles per workgroup, so Ackley's 2048
// workgroups at N = 65 536, D = 128 become 1024, all resident) need more
// than 128 VGPRs and spill (us per iteration, one / two phases: Rosenbrock
// 34.6 / 37.2, Ackley 44.0 / 48.2).  PSO_STEP_SPLIT=0 in the environment
// disables the split step, =1 uses it whenever the shape allows;
// PSO_SPLIT_PHASES=2 takes two phases where L >= 8 (tests of every path).
static bool split_shape(const SwarmArgs &a, int words, uint32_t *L, uint32_t *C, uint32_t *H)
{
    const char *env = getenv("PSO_STEP_SPLIT");
    const int mode = env ? atoi(env) : -1;
    if (mode == 0 || a.D < 16) return false;
    if (mode < 0 && (a.N > (1u << 17) || (words == 2 && (uint64_t)a.N * (uint64_t)a.D > (1ull << 24)))) return false;
    const uint32_t cmax = 8 / (uint32_t)words;
    uint32_t l = 2;
    while (l * cmax < (uint32_t)a.D) l *= 2;
    if (l > 64) return false;
    uint32_t c = ((uint32_t)a.D + l - 1) / l;
    c += c & 1u;
    const char *penv = getenv("PSO_SPLIT_PHASES");
    const int pmode = penv ? atoi(penv) : 0;
    const uint32_t h = (pmode == 2 && l >= 8) ? 2u : 1u;
    *L = l / h;
    *C = c;
    *H = h;
    return true;
}

template <int FIT, int POL>
static void launch_split(const SwarmArgs &a, uint32_t L, uint32_t C, uint32_t H, hipStream_t stream)
{
    constexpr int W = Fitness<FIT>::STAGE_WORDS;
    const uint32_t Q = BLOCK / L, P = 4 * Q;
    const size_t DP = H > 1 ? (size_t)L * C : (size_t)a.D;
    const uint64_t quads = ((uint64_t)a.N + 3) / 4;
    const dim3 grid((unsigned)((quads + Q - 1) / Q));
    const size_t lds = sizeof(float) * (2 * (size_t)a.D + (size_t)W * DP * P);
    if (H > 1)
        hipLaunchKernelGGL((k_step_split<FIT, POL, 2>), grid, dim3(BLOCK), lds, stream, a, L, C);
    else
        hipLaunchKernelGGL((k_step_split<FIT, POL, 1>), grid, dim3(BLOCK), lds, stream, a, L, C);
}

// One particle per lane (k_step_one) for the shapes where it is the faster
// synchronous step; PSO_STEP_ONE=1 in the environment forces it wherever the
// variant allows, =0 disables it.
static bool one_shape(const SwarmArgs &a)
{
    const char *env = getenv("PSO_STEP_ONE");
    const int mode = env ? atoi(env) : -1;
    if (mode >= 0) return mode == 1;
    return false;
}

template <int FIT, int POL>
static void launch_one(const SwarmArgs &a, hipStream_t stream)
{
    constexpr int K = PSO_STEP_ONE_K;
    const size_t lds = 2 * sizeof(float) * a.D;
    const dim3 grid((a.N + BLOCK - 1) / BLOCK);
    switch (PSO_STEP_EXACT_D ? a.D : 0) {
    case 128: hipLaunchKernelGGL((k_step_one<FIT, 128, K, POL>), grid, dim3(BLOCK), lds, stream, a); break;
    default: hipLaunchKernelGGL((k_step_one<FIT, 0, K, POL>), grid, dim3(BLOCK), lds, stream, a); break;
    }
}

// Tiles per workgroup of the asynchronous step: PSO_ASYNC_TILES in the
// environment (1..64), else PSO_ASYNC_TILES_DEFAULT.
#ifndef PSO_ASYNC_TILES_DEFAULT
#define PSO_ASYNC_TILES_DEFAULT 2
#endif
uint32_t async_tiles_per_workgroup()
{
    const char *env = getenv("PSO_ASYNC_TILES");
    const int v = env ? atoi(env) : 0;
    return (v >= 1 && v <= 64) ? (uint32_t)v : (uint32_t)PSO_ASYNC_TILES_DEFAULT;
}

template <int FIT, int POL>
static void launch_async(const SwarmArgs &a, hipStream_t stream)
{
    const size_t lds = 2 * sizeof(float) * a.D;
    const uint32_t tiles = grid_of(a).x, per = async_tiles_per_workgroup();
    const dim3 grid((tiles + per - 1) / per);
    switch (PSO_STEP_EXACT_D ? a.D : 0) {
    case 32: hipLaunchKernelGGL((k_step_async<FIT, 32, POL>), grid, dim3(BLOCK), lds, stream, a, tiles); break;
    case 128: hipLaunchKernelGGL((k_step_async<FIT, 128, POL>), grid, dim3(BLOCK), lds, stream, a, tiles); break;
    default: hipLaunchKernelGGL((k_step_async<FIT, 0, POL>), grid, dim3(BLOCK), lds, stream, a, tiles); break;
    }
}

template <int FIT, int VAR, int POL>
static void launch_step_fvp(const SwarmArgs &a, hipStream_t stream)
{
    uint32_t L = 0, C = 0, H = 1;
    if (VAR == VAR_ASYNC) {
        launch_async<FIT, POL>(a, stream);
        return;
    }
    if (one_shape(a)) {
        launch_one<FIT, POL>(a, stream);
        return;
    }
    if (split_shape(a, Fitness<FIT>::STAGE_WORDS, &L, &C, &H)) {
        launch_split<FIT, POL>(a, L, C, H, stream);
        return;
    }
    const size_t lds = 2 * sizeof(float) * a.D;
    switch (PSO_STEP_EXACT_D ? a.D : 0) {
    case 32: hipLaunchKernelGGL((k_step<FIT, 32, POL>), grid_of(a), dim3(BLOCK), lds, stream, a); break;
    case 128: hipLaunchKernelGGL((k_step<FIT, 128, POL>), grid_of(a), dim3(BLOCK), lds, stream, a); break;
    default: hipLaunchKernelGGL((k_step<FIT, 0, POL>), grid_of(a), dim3(BLOCK), lds, stream, a); break;
    }
}

template <int FIT, int VAR>
static void launch_step_fv(const SwarmArgs &a, hipStream_t stream)
{
    switch (cache_policy(a.Np, a.D)) {
    case POL_STREAM: launch_step_fvp<FIT, VAR, POL_STREAM>(a, stream); break;
    case POL_X: launch_step_fvp<FIT, VAR, POL_X>(a, stream); break;
    case POL_XV: launch_step_fvp<FIT, VAR, POL_XV>(a, stream); break;
    default: launch_step_fvp<FIT, VAR, POL_ALL>(a, stream); break;
    }
}

template <int FIT, bool UNROLLED, int POL>
static void launch_reduce_p(const SwarmArgs &a, hipStream_t stream)
{
    const size_t lds = 2 * sizeof(float) * a.D;
    const dim3 g = grid_of(a);
    switch (PSO_STEP_EXACT_D ? a.D : 0) {
    case 32: hipLaunchKernelGGL((k_step_reduce<FIT, 32, UNROLLED, POL>), g, dim3(BLOCK), lds, stream, a); break;
    default: hipLaunchKernelGGL((k_step_reduce<FIT, 0, UNROLLED, POL>), g, dim3(BLOCK), lds, stream, a); break;
    }
    hipLaunchKernelGGL(k_reduce_final<UNROLLED>, dim3(1), dim3(BLOCK), 0, stream, a, g.x);
}

template <int FIT, bool UNROLLED>
static void launch_reduce(const SwarmArgs &a, hipStream_t stream)
{
    switch (cache_policy(a.Np, a.D)) {
    case POL_STREAM: launch_reduce_p<FIT, UNROLLED, POL_STREAM>(a, stream); break;
    case POL_X: launch_reduce_p<FIT, UNROLLED, POL_X>(a, stream); break;
    case POL_XV: launch_reduce_p<FIT, UNROLLED, POL_XV>(a, stream); break;
    default: launch_reduce_p<FIT, UNROLLED, POL_ALL>(a, stream); break;
    }
}

template <int FIT, int POL>
static hipError_t launch_persist_p(const SwarmArgs &a, uint32_t T, uint32_t max_lead, hipStream_t stream)
{
    const size_t lds = 2 * sizeof(float) * a.D;
    int per_cu = 0, dev = 0, cus = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_persist<FIT, POL>, BLOCK, lds);
    if (e != hipSuccess) return e;
    if ((e = hipGetDevice(&dev)) != hipSuccess) return e;
    if ((e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess) return e;
    // every workgroup co-resident (three quarters of the occupancy bound),
    // one particle quad per lane where the swarm allows it
    const uint64_t cap = std::min<uint64_t>(PERSIST_MAX_GRID, std::max(1, per_cu * cus * 3 / 4));
    const uint64_t nq = ((uint64_t)a.N + 3) / 4;
    const uint64_t grid = std::max<uint64_t>(1, std::min<uint64_t>(cap, (nq + BLOCK - 1) / BLOCK));
    const uint32_t qpw = (uint32_t)((nq + grid - 1) / grid);
    const uint64_t used = (nq + qpw - 1) / qpw;
    hipLaunchKernelGGL((k_persist<FIT, POL>), dim3((unsigned)used), dim3(BLOCK), lds, stream, a, T, max_lead, qpw);
    return hipGetLastError();
}

template <int FIT>
static hipError_t launch_persist_f(const SwarmArgs &a, uint32_t T, uint32_t max_lead, hipStream_t stream)
{
    switch (cache_policy(a.Np, a.D)) {
    case POL_STREAM: return launch_persist_p<FIT, POL_STREAM>(a, T, max_lead, stream);
    case POL_X: return launch_persist_p<FIT, POL_X>(a, T, max_lead, stream);
    case POL_XV: return launch_persist_p<FIT, POL_XV>(a, T, max_lead, stream);
    default: return launch_persist_p<FIT, POL_ALL>(a, T, max_lead, stream);
    }
}

// Before a persistent run: the workgroups' iteration counts to zero, and the
// history entries of the run's iterations (after the control block's t) to
// "no key", so that each can take the minimum of what the workgroups saw.
__global__ void k_persist_prepare(SwarmArgs a, uint32_t T)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < PERSIST_MAX_GRID) a.prog[i] = 0u;
    if (i < T && i < (uint32_t)HIST_CAP) a.hist[(a.ctrl->t + 1 + i) & (HIST_CAP - 1)] = NO_KEY;
}

hipError_t launch_persistent(int fitness, const SwarmArgs &a, uint32_t T, uint32_t max_lead, hipStream_t stream)
{
    if (!a.ctrl || !a.prog || T == 0) return T == 0 ? hipSuccess : hipErrorInvalidValue;
    // a kernel, not a memset: the call may be captured into a graph
    const uint32_t n = std::max<uint32_t>(PERSIST_MAX_GRID, (uint32_t)HIST_CAP);
    hipLaunchKernelGGL(k_persist_prepare, dim3((n + 255) / 256), dim3(256), 0, stream, a, T);
    switch (fitness) {
    case F_SPHERE: return launch_persist_f<F_SPHERE>(a, T, max_lead, stream);
    case F_RASTRIGIN: return launch_persist_f<F_RASTRIGIN>(a, T, max_lead, stream);
    case F_ROSENBROCK: return launch_persist_f<F_ROSENBROCK>(a, T, max_lead, stream);
    case F_ACKLEY: return launch_persist_f<F_ACKLEY>(a, T, max_lead, stream);
    case F_CUBIC: return launch_persist_f<F_CUBIC>(a, T, max_lead, stream);
    default: return hipErrorInvalidValue;
    }
}

template <int FIT>
static void launch_step_f(int variant, const SwarmArgs &a, hipStream_t stream)
{
    switch (variant) {
    case VAR_SYNC: launch_step_fv<FIT, VAR_SYNC>(a, stream); break;
    case VAR_ASYNC: launch_step_fv<FIT, VAR_ASYNC>(a, stream); break;
    case VAR_REDUCE: launch_reduce<FIT, false>(a, stream); break;
    default: launch_reduce<FIT, true>(a, stream); break;
    }
}

hipError_t launch_step(int fitness, int variant, const SwarmArgs &a, hipStream_t stream)
{
    if (variant < VAR_SYNC || variant > VAR_REDUCE_UNROLLED) return hipErrorInvalidValue;
    switch (fitness) {
    case F_SPHERE: launch_step_f<F_SPHERE>(variant, a, stream); break;
    case F_RASTRIGIN: launch_step_f<F_RASTRIGIN>(variant, a, stream); break;
    case F_ROSENBROCK: launch_step_f<F_ROSENBROCK>(variant, a, stream); break;
    case F_ACKLEY: launch_step_f<F_ACKLEY>(variant, a, stream); break;
    case F_CUBIC: launch_step_f<F_CUBIC>(variant, a, stream); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

} // namespace pso

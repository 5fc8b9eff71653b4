// pso_kernels.hip -- the global-best PSO step on gfx950.
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
// candidate only if its new pbest key beats the previous gbest key (the same
// rarity Alg. 2 exploits); a wavefront with a candidate takes its minimum by
// a butterfly over lanes, one lane folds it into a workgroup minimum in LDS,
// and a workgroup whose minimum beats the previous gbest issues one 64-bit
// atomicMin of the packed (fitness, index) key.  The index alone travels, as
// in Sec. 4.3; the last workgroup to finish gathers the winner's position.
#include "pso_device.hpp"
#include "pso_kernels.hpp"

// Launch-shape knobs of the step kernel (build-time; defaults are the tuned
// values for gfx950).
#ifndef PSO_STEP_WAVES_PER_EU
#define PSO_STEP_WAVES_PER_EU 0 // 0: let the compiler choose the register budget
#endif
#ifndef PSO_STEP_EXACT_D
#define PSO_STEP_EXACT_D 1 // compile-time D for the common dimensions
#endif
#ifndef PSO_STEP_UNROLL
#define PSO_STEP_UNROLL 1 // unroll of the dimension-pair loop
#endif

#if PSO_STEP_WAVES_PER_EU > 0
#define PSO_STEP_ATTR __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(PSO_STEP_WAVES_PER_EU)))
#else
#define PSO_STEP_ATTR __launch_bounds__(BLOCK)
#endif

namespace pso {

#ifndef PSO_BLOCK
#define PSO_BLOCK 256
#endif
constexpr int BLOCK = PSO_BLOCK;

static inline size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

Layout layout_of(uint64_t N, int D)
{
    Layout L;
    L.Np = (N + ROW_ALIGN - 1) / ROW_ALIGN * ROW_ALIGN;
    const uint64_t Np = L.Np;
    size_t o = 0;
    L.ctrl = o;  o += align256(sizeof(Ctrl));
    L.gpos = o;  o += align256(sizeof(float) * D);
    L.shift = o; o += align256(sizeof(float) * D);
    L.hist = o;  o += align256(sizeof(unsigned long long) * HIST_CAP);
    L.pf = o;    o += align256(sizeof(float) * Np);
    L.pend = o;  o += align256(Np);
    L.x = o;     o += align256(sizeof(float) * Np * (size_t)D);
    L.v = o;     o += align256(sizeof(float) * Np * (size_t)D);
    L.p = o;     o += align256(sizeof(float) * Np * (size_t)D);
    L.total = o;
    return L;
}

SwarmArgs bind(void *base, const Layout &L, uint64_t N, int D)
{
    char *b = static_cast<char *>(base);
    SwarmArgs a{};
    a.ctrl = reinterpret_cast<Ctrl *>(b + L.ctrl);
    a.gpos = reinterpret_cast<float *>(b + L.gpos);
    a.shift = reinterpret_cast<const float *>(b + L.shift);
    a.hist = reinterpret_cast<unsigned long long *>(b + L.hist);
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

__device__ __forceinline__ float clampf(float v, float lo, float hi)
{
    v = (v < lo) ? lo : v;
    return (v > hi) ? hi : v;
}

typedef float f4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f4 ld_stream(const float *row, uint32_t q)
{
    return __builtin_nontemporal_load(reinterpret_cast<const f4 *>(row) + q);
}

__device__ __forceinline__ void st_stream(float *row, uint32_t q, f4 v)
{
    __builtin_nontemporal_store(v, reinterpret_cast<f4 *>(row) + q);
}

// The random words of particle i for dimension d (Philox output words
// 2(d&1) and 2(d&1)+1 of the call for dimension pair d>>1).
__device__ __forceinline__ uint32_t word_r1(const U4 &u, int h) { return h ? u.c : u.a; }
__device__ __forceinline__ uint32_t word_r2(const U4 &u, int h) { return h ? u.d : u.b; }

// ---------------------------------------------------------------------------
// Aggregation tail shared by init and step: wavefront and workgroup minimum
// of the candidate keys, one global atomicMin per workgroup that has one, and
// the arrival count that elects the last workgroup.  Returns true in every
// lane of the last workgroup, after an acquire fence.
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool aggregate(Ctrl *c, unsigned long long key, unsigned long long thr,
                                          unsigned long long *wg_min, int *last_flag)
{
    const bool cand = key < thr;
    if (__ballot(cand)) {
        const unsigned long long m = wave_min_u64(cand ? key : NO_KEY);
        if ((threadIdx.x & 63) == 0) atomicMin(wg_min, m);
    }
    __syncthreads();
    const unsigned long long m = *wg_min;
    const bool publish = m < thr;
    if (publish) {
        __threadfence(); // release this workgroup's pbest stores
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        if (publish) {
            atomicMin(&c->gkey, m);
            __threadfence(); // the minimum precedes the arrival
        }
        const unsigned int ticket = atomicAdd(&c->arrive, 1u);
        *last_flag = (ticket == gridDim.x - 1);
    }
    __syncthreads();
    if (*last_flag) {
        __threadfence(); // acquire every workgroup's results
        return true;
    }
    return false;
}

// Iteration epilogue, run by the last workgroup: gbest position, history,
// counters and the stop rule for iteration t.  A changed gbest belongs to a
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
// Step 1 (Alg. 1): x ~ U[lo, hi), v ~ U[-vmax, vmax), pbest <- x, gbest.
// Lane q initialises particles 4q .. 4q+3 (the padding past N included, so
// every stored element holds a finite value).
// ---------------------------------------------------------------------------
template <int FIT>
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
    const uint32_t i0 = 4 * q;
    unsigned long long key = NO_KEY;
    if (i0 < a.Np) {
        const size_t Np = a.Np;
        const float span = a.hi - a.lo, vspan = a.vmax + a.vmax;
        Fitness<FIT> fit[4];
        for (int d = 0; d < D; d += 2) {
            U4 u[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) u[k] = philox4x32_10(a.k0, a.k1, (uint32_t)d >> 1, i0 + k, 0u, TAG_INIT);
            const int nd = (d + 1 < D) ? 2 : 1;
            for (int h = 0; h < nd; ++h) {
                f4 xs, vs;
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    xs[k] = clampf(a.lo + span * unit_float(word_r1(u[k], h)), a.lo, a.hi);
                    vs[k] = clampf(-a.vmax + vspan * unit_float(word_r2(u[k], h)), -a.vmax, a.vmax);
                    fit[k].add(xs[k] - s_shift[d + h], d + h);
                }
                const size_t row = (size_t)(d + h) * Np;
                st_stream(a.x + row, q, xs);
                st_stream(a.v + row, q, vs);
                st_stream(a.p + row, q, xs);
            }
        }
        f4 fs;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            fs[k] = fit[k].value(D);
            if (i0 + k < a.N) {
                const unsigned long long kk = make_key(fs[k], i0 + k);
                key = kk < key ? kk : key;
            }
        }
        *reinterpret_cast<f4 *>(a.pf + i0) = fs;
        *reinterpret_cast<uint32_t *>(a.pend + i0) = 0u;
    }
    if (aggregate(a.ctrl, key, NO_KEY, &wg_min, &last)) epilogue(a, 0u, true);
}

// ---------------------------------------------------------------------------
// One iteration t = (iterations completed) + 1, synchronous gbest: every
// particle reads the gbest position of iteration t-1 (staged in LDS with the
// shift vector; each dimension's value is one broadcast read).
// DC > 0 fixes D at compile time; DC == 0 takes D from the arguments.
// ---------------------------------------------------------------------------
template <int FIT, int DC>
__global__ void PSO_STEP_ATTR k_step_sync(SwarmArgs a)
{
    __shared__ unsigned long long wg_min;
    __shared__ int last;
    extern __shared__ float s_dyn[]; // gbest position (D floats), then shift (D floats)
    Ctrl *c = a.ctrl;
    if (c->stop) return;
    const int D = DC > 0 ? DC : a.D;
    float *s_g = s_dyn, *s_shift = s_dyn + D;
    const uint32_t t = (uint32_t)(c->t + 1);
    const unsigned long long thr = c->gkey_prev;
    for (int d = threadIdx.x; d < D; d += BLOCK) {
        s_g[d] = a.gpos[d];
        s_shift[d] = a.shift[d];
    }
    if (threadIdx.x == 0) wg_min = NO_KEY;
    __syncthreads();

    const uint32_t q = blockIdx.x * BLOCK + threadIdx.x;
    const uint32_t i0 = 4 * q;
    unsigned long long key = NO_KEY;
    if (i0 < a.N) {
        const size_t Np = a.Np;
        const float w = a.w, c1 = a.c1, c2 = a.c2, vmax = a.vmax, lo = a.lo, hi = a.hi;
        const f4 pf_old = *reinterpret_cast<const f4 *>(a.pf + i0);
        // Pbest positions improved in the previous iteration are still in x;
        // this pass reads x anyway, so it completes them into p.  Every lane
        // of a 128-byte line (8 lanes x 4 particles) with a pending particle
        // rewrites its part of p, so lines are written whole.
        const uint32_t pend = *reinterpret_cast<const uint32_t *>(a.pend + i0);
        const unsigned long long dirty = __ballot(pend != 0u);
        const bool line_dirty = ((dirty >> ((threadIdx.x & 63) & ~7u)) & 0xFFull) != 0;
        Fitness<FIT> fit[4];
#pragma unroll PSO_STEP_UNROLL
        for (int d = 0; d < D; d += 2) {
            U4 u[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) u[k] = philox4x32_10(a.k0, a.k1, (uint32_t)d >> 1, i0 + k, t, TAG_VEL);
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                if (h == 1 && d + 1 >= D) break;
                const size_t row = (size_t)(d + h) * Np;
                const f4 xs = ld_stream(a.x + row, q);
                const f4 vs = ld_stream(a.v + row, q);
                f4 ps = ld_stream(a.p + row, q);
#pragma unroll
                for (int k = 0; k < 4; ++k)
                    if (pend & (0xFFu << (8 * k))) ps[k] = xs[k];
                const float g = s_g[d + h], sh = s_shift[d + h];
                f4 xn, vn;
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const float r1 = unit_float(word_r1(u[k], h));
                    const float r2 = unit_float(word_r2(u[k], h));
                    float nv = ((w * vs[k]) + ((c1 * r1) * (ps[k] - xs[k]))) + ((c2 * r2) * (g - xs[k]));
                    nv = clampf(nv, -vmax, vmax);
                    xn[k] = clampf(xs[k] + nv, lo, hi);
                    vn[k] = nv;
                    fit[k].add(xn[k] - sh, d + h);
                }
                st_stream(a.x + row, q, xn);
                st_stream(a.v + row, q, vn);
                if (line_dirty) st_stream(a.p + row, q, ps);
            }
        }
        // Step 4: strict improvement (NaN never improves).  The new pbest
        // position is x as just stored; it is marked pending.
        f4 pf_new = pf_old;
        uint32_t pend_new = 0;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const float f = fit[k].value(D);
            if (i0 + k < a.N && f < pf_old[k]) {
                pend_new |= 1u << (8 * k);
                pf_new[k] = f;
                const unsigned long long kk = make_key(f, i0 + k);
                key = kk < key ? kk : key;
            }
        }
        if (pend_new) *reinterpret_cast<f4 *>(a.pf + i0) = pf_new;
        if (pend_new != pend) *reinterpret_cast<uint32_t *>(a.pend + i0) = pend_new;
    }
    if (aggregate(c, key, thr, &wg_min, &last)) epilogue(a, t, false);
}

// ---------------------------------------------------------------------------
// Completes pending pbest positions (p <- x where pending) and clears the
// marks; run before the state is read.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(BLOCK) k_flush(SwarmArgs a)
{
    const uint32_t q = blockIdx.x * BLOCK + threadIdx.x;
    const uint32_t i0 = 4 * q;
    if (i0 >= a.Np) return;
    const uint32_t pend = *reinterpret_cast<const uint32_t *>(a.pend + i0);
    if (!pend) return;
    for (int d = 0; d < a.D; ++d) {
        const size_t row = (size_t)d * a.Np;
        const f4 xs = *(reinterpret_cast<const f4 *>(a.x + row) + q);
        f4 ps = *(reinterpret_cast<const f4 *>(a.p + row) + q);
#pragma unroll
        for (int k = 0; k < 4; ++k)
            if (pend & (0xFFu << (8 * k))) ps[k] = xs[k];
        *(reinterpret_cast<f4 *>(a.p + row) + q) = ps;
    }
    *reinterpret_cast<uint32_t *>(a.pend + i0) = 0u;
}

__global__ void __launch_bounds__(BLOCK) k_clear_pending(SwarmArgs a)
{
    const uint32_t q = blockIdx.x * BLOCK + threadIdx.x;
    if (4 * q < a.Np) *reinterpret_cast<uint32_t *>(a.pend + 4 * q) = 0u;
}

// ---------------------------------------------------------------------------
// Launchers.
// ---------------------------------------------------------------------------
// One lane per four particles.
static inline dim3 grid_of(const SwarmArgs &a) { return dim3((a.N + 4 * BLOCK - 1) / (4 * BLOCK)); }
// init also covers the padding up to Np
static inline dim3 grid_init(const SwarmArgs &a) { return dim3((a.Np + 4 * BLOCK - 1) / (4 * BLOCK)); }

hipError_t launch_reset(const SwarmArgs &a, hipStream_t stream)
{
    hipLaunchKernelGGL(k_reset, dim3(1), dim3(64), 0, stream, a);
    return hipGetLastError();
}

hipError_t launch_flush(const SwarmArgs &a, hipStream_t stream)
{
    hipLaunchKernelGGL(k_flush, grid_init(a), dim3(BLOCK), 0, stream, a);
    return hipGetLastError();
}

hipError_t launch_clear_pending(const SwarmArgs &a, hipStream_t stream)
{
    hipLaunchKernelGGL(k_clear_pending, grid_init(a), dim3(BLOCK), 0, stream, a);
    return hipGetLastError();
}

hipError_t launch_arm(const SwarmArgs &a, float tol, float fstar, hipStream_t stream)
{
    hipLaunchKernelGGL(k_arm, dim3(1), dim3(64), 0, stream, a, tol, fstar);
    return hipGetLastError();
}

hipError_t launch_init(int fitness, const SwarmArgs &a, hipStream_t stream)
{
    const size_t lds = sizeof(float) * a.D;
    switch (fitness) {
    case F_SPHERE: hipLaunchKernelGGL(k_init<F_SPHERE>, grid_init(a), dim3(BLOCK), lds, stream, a); break;
    case F_RASTRIGIN: hipLaunchKernelGGL(k_init<F_RASTRIGIN>, grid_init(a), dim3(BLOCK), lds, stream, a); break;
    case F_ROSENBROCK: hipLaunchKernelGGL(k_init<F_ROSENBROCK>, grid_init(a), dim3(BLOCK), lds, stream, a); break;
    case F_ACKLEY: hipLaunchKernelGGL(k_init<F_ACKLEY>, grid_init(a), dim3(BLOCK), lds, stream, a); break;
    case F_CUBIC: hipLaunchKernelGGL(k_init<F_CUBIC>, grid_init(a), dim3(BLOCK), lds, stream, a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int FIT>
static void launch_step_fit(const SwarmArgs &a, hipStream_t stream)
{
    const size_t lds = 2 * sizeof(float) * a.D;
    switch (PSO_STEP_EXACT_D ? a.D : 0) {
    case 2: hipLaunchKernelGGL((k_step_sync<FIT, 2>), grid_of(a), dim3(BLOCK), lds, stream, a); break;
    case 32: hipLaunchKernelGGL((k_step_sync<FIT, 32>), grid_of(a), dim3(BLOCK), lds, stream, a); break;
    case 128: hipLaunchKernelGGL((k_step_sync<FIT, 128>), grid_of(a), dim3(BLOCK), lds, stream, a); break;
    default: hipLaunchKernelGGL((k_step_sync<FIT, 0>), grid_of(a), dim3(BLOCK), lds, stream, a); break;
    }
}

hipError_t launch_step(int fitness, int variant, const SwarmArgs &a, hipStream_t stream)
{
    if (variant != 0) return hipErrorInvalidValue;
    switch (fitness) {
    case F_SPHERE: launch_step_fit<F_SPHERE>(a, stream); break;
    case F_RASTRIGIN: launch_step_fit<F_RASTRIGIN>(a, stream); break;
    case F_ROSENBROCK: launch_step_fit<F_ROSENBROCK>(a, stream); break;
    case F_ACKLEY: launch_step_fit<F_ACKLEY>(a, stream); break;
    case F_CUBIC: launch_step_fit<F_CUBIC>(a, stream); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

} // namespace pso

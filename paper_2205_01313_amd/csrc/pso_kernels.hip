// pso_kernels.hip -- the global-best PSO step on gfx950.
//
// One lane owns one particle (Sec. 2.2); its dimensions are walked in order
// over structure-of-arrays state (Sec. 4.1), so a wavefront reads 64
// consecutive floats of one dimension per access.  One launch is one
// iteration: update (Eq. 1, Eq. 2, clamps), fitness and pbest (Alg. 1 Steps
// 2-4) are fused with the aggregation into the gbest (Step 5).
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

namespace pso {

constexpr int BLOCK = 256;

static inline size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

Layout layout_of(uint64_t N, int D)
{
    Layout L;
    size_t o = 0;
    L.ctrl = o;  o += align256(sizeof(Ctrl));
    L.gpos = o;  o += align256(sizeof(float) * D);
    L.shift = o; o += align256(sizeof(float) * D);
    L.hist = o;  o += align256(sizeof(unsigned long long) * HIST_CAP);
    L.pf = o;    o += align256(sizeof(float) * N);
    L.x = o;     o += align256(sizeof(float) * N * (size_t)D);
    L.v = o;     o += align256(sizeof(float) * N * (size_t)D);
    L.p = o;     o += align256(sizeof(float) * N * (size_t)D);
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
    a.x = reinterpret_cast<float *>(b + L.x);
    a.v = reinterpret_cast<float *>(b + L.v);
    a.p = reinterpret_cast<float *>(b + L.p);
    a.N = (uint32_t)N;
    a.D = D;
    return a;
}

__device__ __forceinline__ float clampf(float v, float lo, float hi)
{
    v = (v < lo) ? lo : v;
    return (v > hi) ? hi : v;
}

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
// counters and the stop rule for iteration t.
__device__ void epilogue(const SwarmArgs &a, uint32_t t, bool first)
{
    Ctrl *c = a.ctrl;
    const unsigned long long k = __hip_atomic_load(&c->gkey, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const bool changed = first || k != c->gkey_prev;
    if (changed) {
        const size_t gi = (uint32_t)k;
        for (int d = threadIdx.x; d < a.D; d += BLOCK) a.gpos[d] = a.p[(size_t)d * a.N + gi];
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

    const uint32_t i = blockIdx.x * BLOCK + threadIdx.x;
    unsigned long long key = NO_KEY;
    if (i < a.N) {
        const size_t N = a.N;
        const float span = a.hi - a.lo, vspan = a.vmax + a.vmax;
        Fitness<FIT> fit;
        for (int d = 0; d < D; d += 2) {
            const U4 u = philox4x32_10(a.k0, a.k1, (uint32_t)d >> 1, i, 0u, TAG_INIT);
            const int nd = (d + 1 < D) ? 2 : 1;
            for (int j = 0; j < nd; ++j) {
                const float ux = unit_float(j ? u.c : u.a);
                const float uv = unit_float(j ? u.d : u.b);
                const float xv = clampf(a.lo + span * ux, a.lo, a.hi);
                const float vv = clampf(-a.vmax + vspan * uv, -a.vmax, a.vmax);
                const size_t e = (size_t)(d + j) * N + i;
                a.x[e] = xv;
                a.v[e] = vv;
                a.p[e] = xv;
                fit.add(xv - s_shift[d + j], d + j);
            }
        }
        const float f = fit.value(D);
        a.pf[i] = f;
        key = make_key(f, i);
    }
    if (aggregate(a.ctrl, key, NO_KEY, &wg_min, &last)) epilogue(a, 0u, true);
}

// ---------------------------------------------------------------------------
// One iteration t = (iterations completed) + 1, synchronous gbest: every
// particle reads the gbest position of iteration t-1.
// DREG > 0 keeps the new position in registers for the pbest store (D <=
// DREG); DREG == 0 re-reads it from x.
// ---------------------------------------------------------------------------
template <int FIT, int DREG>
__global__ void __launch_bounds__(BLOCK) k_step_sync(SwarmArgs a)
{
    __shared__ unsigned long long wg_min;
    __shared__ int last;
    extern __shared__ float s_dyn[]; // gbest position (D floats), then shift (D floats)
    float *s_g = s_dyn, *s_shift = s_dyn + a.D;
    Ctrl *c = a.ctrl;
    if (c->stop) return;
    const uint32_t t = (uint32_t)(c->t + 1);
    const unsigned long long thr = c->gkey_prev;
    const int D = a.D;
    for (int d = threadIdx.x; d < D; d += BLOCK) {
        s_g[d] = a.gpos[d];
        s_shift[d] = a.shift[d];
    }
    if (threadIdx.x == 0) wg_min = NO_KEY;
    __syncthreads();

    const uint32_t i = blockIdx.x * BLOCK + threadIdx.x;
    unsigned long long key = NO_KEY;
    if (i < a.N) {
        const size_t N = a.N;
        const float w = a.w, c1 = a.c1, c2 = a.c2, vmax = a.vmax, lo = a.lo, hi = a.hi;
        Fitness<FIT> fit;
        float xr[DREG > 0 ? DREG : 1];

        auto update = [&](int d, uint32_t ra, uint32_t rb) -> float {
            const size_t e = (size_t)d * N + i;
            const float xv = a.x[e], vv = a.v[e], pv = a.p[e];
            const float r1 = unit_float(ra), r2 = unit_float(rb);
            float vn = ((w * vv) + ((c1 * r1) * (pv - xv))) + ((c2 * r2) * (s_g[d] - xv));
            vn = clampf(vn, -vmax, vmax);
            const float xn = clampf(xv + vn, lo, hi);
            a.x[e] = xn;
            a.v[e] = vn;
            fit.add(xn - s_shift[d], d);
            return xn;
        };

        if constexpr (DREG > 0) {
#pragma unroll
            for (int d = 0; d < DREG; d += 2) {
                if (d < D) {
                    const U4 u = philox4x32_10(a.k0, a.k1, (uint32_t)d >> 1, i, t, TAG_VEL);
                    xr[d] = update(d, u.a, u.b);
                    if (d + 1 < D) xr[d + 1] = update(d + 1, u.c, u.d);
                }
            }
        } else {
            for (int d = 0; d < D; d += 2) {
                const U4 u = philox4x32_10(a.k0, a.k1, (uint32_t)d >> 1, i, t, TAG_VEL);
                update(d, u.a, u.b);
                if (d + 1 < D) update(d + 1, u.c, u.d);
            }
        }

        const float f = fit.value(D);
        if (f < a.pf[i]) { // Step 4: strict improvement, NaN never improves
            a.pf[i] = f;
            if constexpr (DREG > 0) {
#pragma unroll
                for (int d = 0; d < DREG; ++d)
                    if (d < D) a.p[(size_t)d * N + i] = xr[d];
            } else {
                for (int d = 0; d < D; ++d) a.p[(size_t)d * N + i] = a.x[(size_t)d * N + i];
            }
            key = make_key(f, i);
        }
    }
    if (aggregate(c, key, thr, &wg_min, &last)) epilogue(a, t, false);
}

// ---------------------------------------------------------------------------
// Launchers.
// ---------------------------------------------------------------------------
static inline dim3 grid_of(const SwarmArgs &a) { return dim3((a.N + BLOCK - 1) / BLOCK); }

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

hipError_t launch_init(int fitness, const SwarmArgs &a, hipStream_t stream)
{
    const size_t lds = sizeof(float) * a.D;
    switch (fitness) {
    case F_SPHERE: hipLaunchKernelGGL(k_init<F_SPHERE>, grid_of(a), dim3(BLOCK), lds, stream, a); break;
    case F_RASTRIGIN: hipLaunchKernelGGL(k_init<F_RASTRIGIN>, grid_of(a), dim3(BLOCK), lds, stream, a); break;
    case F_ROSENBROCK: hipLaunchKernelGGL(k_init<F_ROSENBROCK>, grid_of(a), dim3(BLOCK), lds, stream, a); break;
    case F_ACKLEY: hipLaunchKernelGGL(k_init<F_ACKLEY>, grid_of(a), dim3(BLOCK), lds, stream, a); break;
    case F_CUBIC: hipLaunchKernelGGL(k_init<F_CUBIC>, grid_of(a), dim3(BLOCK), lds, stream, a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int FIT>
static void launch_step_fit(const SwarmArgs &a, hipStream_t stream)
{
    const size_t lds = 2 * sizeof(float) * a.D;
    if (a.D <= 32)
        hipLaunchKernelGGL((k_step_sync<FIT, 32>), grid_of(a), dim3(BLOCK), lds, stream, a);
    else
        hipLaunchKernelGGL((k_step_sync<FIT, 0>), grid_of(a), dim3(BLOCK), lds, stream, a);
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

// pso_quad.hpp -- the per-particle work of Step 1 and Steps 2-4 (Alg. 1),
// for the four consecutive particles a lane owns.  Every kernel (grid step,
// per-swarm workgroup, batched) calls these, so all of them compute the same
// bits for the same particle and iteration.
#pragma once

#include "pso_device.hpp"
#include "pso_kernels.hpp"

namespace pso {

__device__ __forceinline__ float clampf(float v, float lo, float hi)
{
    v = (v < lo) ? lo : v;
    return (v > hi) ? hi : v;
}

typedef float f4 __attribute__((ext_vector_type(4)));

// 16-byte accesses of lane quad q within one dimension's row.  An array
// whose bit is set in the cache policy (KEEP_X / KEEP_V / KEEP_P) uses
// ordinary loads and stores, so it can stay resident in the memory-side
// cache between iterations; the others carry non-temporal hints and stream.
template <bool KEEP>
__device__ __forceinline__ f4 ld_state(const float *row, uint32_t q)
{
    if constexpr (KEEP)
        return *(reinterpret_cast<const f4 *>(row) + q);
    else
        return __builtin_nontemporal_load(reinterpret_cast<const f4 *>(row) + q);
}

template <bool KEEP>
__device__ __forceinline__ void st_state(float *row, uint32_t q, f4 v)
{
    if constexpr (KEEP)
        *(reinterpret_cast<f4 *>(row) + q) = v;
    else
        __builtin_nontemporal_store(v, reinterpret_cast<f4 *>(row) + q);
}

// Random words of dimension d = 2*pair + h: Philox output words 2h and 2h+1.
__device__ __forceinline__ uint32_t word_r1(const U4 &u, int h) { return h ? u.c : u.a; }
__device__ __forceinline__ uint32_t word_r2(const U4 &u, int h) { return h ? u.d : u.b; }

// Step 1 for particles 4q .. 4q+3: x ~ U[lo, hi), v ~ U[-vmax, vmax), p = x,
// pf = F(x), nothing pending.  Padding particles (index >= N, < Np) are
// initialised too, so every stored element is finite.  Returns the smallest
// key among the valid particles.
template <int FIT, int POL>
__device__ __forceinline__ unsigned long long init_quad(const SwarmArgs &a, int D, uint32_t q,
                                                        const float *s_shift)
{
    const uint32_t i0 = 4 * q;
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
            st_state<(POL & KEEP_X) != 0>(a.x + row, q, xs);
            st_state<(POL & KEEP_V) != 0>(a.v + row, q, vs);
            st_state<(POL & KEEP_P) != 0>(a.p + row, q, xs);
        }
    }
    unsigned long long key = NO_KEY;
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
    return key;
}

// Steps 2-4 of iteration t for particles 4q .. 4q+3 (4q < N), with the gbest
// position s_g and shift s_shift (D floats each, in LDS).  Returns the
// smallest key among the particles whose pbest improved (NO_KEY if none).
//
// Deferred pbest positions: a particle whose pbest improves is marked in
// pend and its new pbest position is left in x.  The next iteration reads x
// anyway, so it uses x as the pbest position of marked particles and writes
// it to p; every lane of a group of PSO_PBEST_GROUP lanes (4 lanes x 4
// particles = 64 bytes, measured best on gfx950 against 16..256-byte groups)
// holding a marked particle rewrites its 16 bytes, so p is written in whole
// groups.
// Must be called by all active lanes of the wavefront together (it ballots).
// *n_improved receives the number of this lane's particles that improved.
#ifndef PSO_PBEST_GROUP
#define PSO_PBEST_GROUP 4
#endif
// Software prefetch of the next dimension pair (PF): pays where the fitness
// is heavy enough to leave memory idle between pairs (grid step, Ackley:
// 196 -> 173 us per iteration at N = 2^18, D = 128; slightly slower for the
// other functions there) and in the batched kernel, whose short per-swarm
// rows need the extra loads in flight (4096-swarm batch: 749 -> 670 ms; a
// one-workgroup run of D = 2 is slower with it: 2.1 -> 2.6 us per iteration).
// Eq. 1 for one element, left to right, clamped to [-vmax, vmax]: the new
// velocity from position x, velocity v, pbest position p, gbest position g
// and the draws r1, r2.
// Split in two for callers that know the gbest position later: the inertia
// and cognitive terms (w v) + ((c1 r1)(p - x)) and the social coefficient
// c2 r2 first, then the social term and the clamp -- the same operations in
// the same order.
__device__ __forceinline__ float velocity_eq1_own(const SwarmArgs &a, float x, float v, float p, float r1)
{
    return (a.w * v) + ((a.c1 * r1) * (p - x));
}

__device__ __forceinline__ float velocity_eq1_social(const SwarmArgs &a, float own, float c2r2, float x, float g)
{
    return clampf(own + (c2r2 * (g - x)), -a.vmax, a.vmax);
}

__device__ __forceinline__ float velocity_eq1(const SwarmArgs &a, float x, float v, float p, float g, float r1, float r2)
{
    return velocity_eq1_social(a, velocity_eq1_own(a, x, v, p, r1), a.c2 * r2, x, g);
}

// Eq. 2 for one element, clamped to [lo, hi].
__device__ __forceinline__ float position_eq2(const SwarmArgs &a, float x, float nv) { return clampf(x + nv, a.lo, a.hi); }

// Eq. 1 and Eq. 2 for one dimension row of the four particles (x, v, p as
// loaded; p replaced by x where the pbest position is pending) and the stores
// of x, v and (for a dirty group) p.  Returns the new positions.
template <int POL>
__device__ __forceinline__ f4 update_row(const SwarmArgs &a, size_t row, uint32_t q, f4 xs, f4 vs, f4 ps,
                                         uint32_t pend, bool line_dirty, const U4 *u, int h, float g)
{
#pragma unroll
    for (int k = 0; k < 4; ++k)
        if (pend & (0xFFu << (8 * k))) ps[k] = xs[k];
    f4 xn, vn;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const float r1 = unit_float(word_r1(u[k], h));
        const float r2 = unit_float(word_r2(u[k], h));
        vn[k] = velocity_eq1(a, xs[k], vs[k], ps[k], g, r1, r2);
        xn[k] = position_eq2(a, xs[k], vn[k]);
    }
    st_state<(POL & KEEP_X) != 0>(a.x + row, q, xn);
    st_state<(POL & KEEP_V) != 0>(a.v + row, q, vn);
    if (line_dirty) st_state<(POL & KEEP_P) != 0>(a.p + row, q, ps);
    return xn;
}

// The pending marks of quad q and whether its 64-byte group of PSO_PBEST_GROUP
// lanes (consecutive in the wavefront) holds any: such a group rewrites p.
// Must be called by all active lanes of the wavefront together (it ballots).
__device__ __forceinline__ bool group_dirty(uint32_t pend)
{
    constexpr unsigned G = PSO_PBEST_GROUP;
    const unsigned long long dirty = __ballot(pend != 0u);
    return ((dirty >> ((threadIdx.x & 63) & ~(G - 1))) & ((1ull << G) - 1)) != 0;
}

template <int FIT, int DC, int UNROLL, int POL, bool PF = (FIT == F_ACKLEY)>
__device__ __forceinline__ unsigned long long iterate_quad(const SwarmArgs &a, int D, uint32_t q, uint32_t t,
                                                           const float *s_g, const float *s_shift,
                                                           uint32_t *n_improved = nullptr)
{
    const uint32_t i0 = 4 * q;
    const size_t Np = a.Np;
    const f4 pf_old = *reinterpret_cast<const f4 *>(a.pf + i0);
    const uint32_t pend = *reinterpret_cast<const uint32_t *>(a.pend + i0);
    const bool line_dirty = group_dirty(pend);
    constexpr bool KX = (POL & KEEP_X) != 0, KV = (POL & KEEP_V) != 0, KP = (POL & KEEP_P) != 0;
    Fitness<FIT> fit[4];
    if constexpr (PF) {
        // Software pipeline over dimension pairs: the next pair's x, v, p are
        // loaded before this pair's stores (the compiler may not hoist them
        // past stores to the same arrays), so two pairs' loads are in flight.
        f4 ax[2], av[2], ap[2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            if (h < D) {
                ax[h] = ld_state<KX>(a.x + (size_t)h * Np, q);
                av[h] = ld_state<KV>(a.v + (size_t)h * Np, q);
                ap[h] = ld_state<KP>(a.p + (size_t)h * Np, q);
            }
        }
#pragma unroll UNROLL
        for (int d = 0; d < D; d += 2) {
            f4 cx[2], cv[2], cp[2];
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                cx[h] = ax[h];
                cv[h] = av[h];
                cp[h] = ap[h];
            }
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                if (d + 2 + h < D) {
                    const size_t row = (size_t)(d + 2 + h) * Np;
                    ax[h] = ld_state<KX>(a.x + row, q);
                    av[h] = ld_state<KV>(a.v + row, q);
                    ap[h] = ld_state<KP>(a.p + row, q);
                }
            }
            U4 u[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) u[k] = philox4x32_10(a.k0, a.k1, (uint32_t)d >> 1, i0 + k, t, TAG_VEL);
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                if (h == 1 && d + 1 >= D) break;
                const f4 xn = update_row<POL>(a, (size_t)(d + h) * Np, q, cx[h], cv[h], cp[h], pend, line_dirty, u,
                                              h, s_g[d + h]);
                const float sh = s_shift[d + h];
#pragma unroll
                for (int k = 0; k < 4; ++k) fit[k].add(xn[k] - sh, d + h);
            }
        }
    } else {
#pragma unroll UNROLL
        for (int d = 0; d < D; d += 2) {
            U4 u[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) u[k] = philox4x32_10(a.k0, a.k1, (uint32_t)d >> 1, i0 + k, t, TAG_VEL);
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                if (h == 1 && d + 1 >= D) break;
                const size_t row = (size_t)(d + h) * Np;
                const f4 xn = update_row<POL>(a, row, q, ld_state<KX>(a.x + row, q), ld_state<KV>(a.v + row, q),
                                              ld_state<KP>(a.p + row, q), pend, line_dirty, u, h, s_g[d + h]);
                const float sh = s_shift[d + h];
#pragma unroll
                for (int k = 0; k < 4; ++k) fit[k].add(xn[k] - sh, d + h);
            }
        }
    }
    // Step 4: strict improvement; NaN never improves.
    unsigned long long key = NO_KEY;
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
    if (n_improved) *n_improved = __builtin_popcount(pend_new);
    return key;
}

// Steps 2-4 of iteration t for one particle i (i < N) per lane: the form of
// the step for swarms with too few particles to give every SIMD several
// wavefronts at four particles per lane.  A lane walks its particle's
// dimensions in order (the fitness is the same sequential sum, in
// registers), with the rows of the next K dimension pairs always loaded
// ahead (a ring of K slots), so one wavefront per SIMD keeps enough loads in
// flight.  Consecutive lanes read consecutive particles of a row (256 bytes
// per wavefront).  The deferred pbest positions work as in iterate_quad: an
// improved particle is marked in pend and its position left in x; the next
// iteration rewrites p for every lane of a 64-byte group (16 lanes) holding
// a marked particle.  Must be called by all active lanes of the wavefront
// together (it ballots).  Returns the particle's new pbest key (NO_KEY if it
// did not improve).
__device__ __forceinline__ bool group16_dirty(bool pend)
{
    const unsigned long long dirty = __ballot(pend);
    return ((dirty >> ((threadIdx.x & 63) & ~15u)) & 0xFFFFull) != 0;
}

template <int FIT, int DC, int K, int POL>
__device__ __forceinline__ unsigned long long iterate_one(const SwarmArgs &a, int D, uint32_t i, bool active,
                                                          uint32_t t, const float *s_g, const float *s_shift,
                                                          uint32_t *n_improved)
{
    constexpr bool KX = (POL & KEEP_X) != 0, KV = (POL & KEEP_V) != 0, KP = (POL & KEEP_P) != 0;
    const size_t Np = a.Np;
    const float pf_old = active ? a.pf[i] : 0.0f;
    const bool pend = active && a.pend[i] != 0;
    const bool line_dirty = group16_dirty(pend);
    Fitness<FIT> fit;
    const int npairs = (D + 1) / 2;
    float rx[K][2], rv[K][2], rp[K][2];
    auto load_pair = [&](int pr, int s) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int d = 2 * pr + h;
            if (d < D) {
                const size_t at = (size_t)d * Np + i;
                rx[s][h] = KX ? a.x[at] : __builtin_nontemporal_load(a.x + at);
                rv[s][h] = KV ? a.v[at] : __builtin_nontemporal_load(a.v + at);
                rp[s][h] = KP ? a.p[at] : __builtin_nontemporal_load(a.p + at);
            }
        }
    };
    if (active) {
#pragma unroll
        for (int s = 0; s < K; ++s)
            if (s < npairs) load_pair(s, s);
        for (int b = 0; b < npairs; b += K) {
#pragma unroll
            for (int s = 0; s < K; ++s) {
                const int pr = b + s;
                if (pr < npairs) {
                    float cx[2], cv[2], cp[2];
#pragma unroll
                    for (int h = 0; h < 2; ++h) {
                        cx[h] = rx[s][h];
                        cv[h] = rv[s][h];
                        cp[h] = rp[s][h];
                    }
                    if (pr + K < npairs) load_pair(pr + K, s);
                    const U4 u = philox4x32_10(a.k0, a.k1, (uint32_t)pr, i, t, TAG_VEL);
#pragma unroll
                    for (int h = 0; h < 2; ++h) {
                        const int d = 2 * pr + h;
                        if (d < D) {
                            const float ps = pend ? cx[h] : cp[h];
                            const float r1 = unit_float(word_r1(u, h));
                            const float r2 = unit_float(word_r2(u, h));
                            const float vn = velocity_eq1(a, cx[h], cv[h], ps, s_g[d], r1, r2);
                            const float xn = position_eq2(a, cx[h], vn);
                            const size_t at = (size_t)d * Np + i;
                            if (KX) a.x[at] = xn; else __builtin_nontemporal_store(xn, a.x + at);
                            if (KV) a.v[at] = vn; else __builtin_nontemporal_store(vn, a.v + at);
                            if (line_dirty) {
                                if (KP) a.p[at] = ps; else __builtin_nontemporal_store(ps, a.p + at);
                            }
                            fit.add(xn - s_shift[d], d);
                        }
                    }
                }
            }
        }
    }
    // Step 4: strict improvement; NaN never improves.
    unsigned long long key = NO_KEY;
    uint32_t imp = 0;
    if (active) {
        const float f = fit.value(D);
        if (f < pf_old) {
            imp = 1;
            a.pf[i] = f;
            key = make_key(f, i);
        }
        if ((imp != 0) != pend) a.pend[i] = (uint8_t)imp;
    }
    if (n_improved) *n_improved = imp;
    return key;
}

// Folds the staged fitness terms of one particle (column idx of the
// [dimension][particle] term arrays, row pitch `pitch`) in dimension order.
// The loads of eight dimensions are issued before their additions, so the
// sequential sum waits on LDS once per eight terms, not once per term; the
// order of the additions is unchanged.
template <int FIT>
__device__ __forceinline__ float fold_terms(const float *t0, const float *t1, size_t pitch, uint32_t idx, int D)
{
    constexpr int W = Fitness<FIT>::STAGE_WORDS;
    Fitness<FIT> fit;
    int d = 0;
    for (; d + 8 <= D; d += 8) {
        float a0[8], a1[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            a0[j] = t0[(size_t)(d + j) * pitch + idx];
            a1[j] = W == 2 ? t1[(size_t)(d + j) * pitch + idx] : 0.0f;
        }
#pragma unroll
        for (int j = 0; j < 8; ++j) fit.fold(a0[j], a1[j], d + j);
    }
    for (; d < D; ++d) fit.fold(t0[(size_t)d * pitch + idx], W == 2 ? t1[(size_t)d * pitch + idx] : 0.0f, d);
    return fit.value(D);
}

// Folds the staged terms of dimensions d0 .. d0+n-1 (rows 0 .. n-1 of the
// term arrays, column idx, row pitch `pitch`) into fit, in dimension order:
// folding a particle's dimensions in consecutive ranges gives exactly
// fold_terms over all of them.
template <int FIT>
__device__ __forceinline__ void fold_range(Fitness<FIT> &fit, const float *t0, const float *t1, size_t pitch,
                                           uint32_t idx, int d0, int n)
{
    constexpr int W = Fitness<FIT>::STAGE_WORDS;
    int j = 0;
    for (; j + 8 <= n; j += 8) {
        float a0[8], a1[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            a0[u] = t0[(size_t)(j + u) * pitch + idx];
            a1[u] = W == 2 ? t1[(size_t)(j + u) * pitch + idx] : 0.0f;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) fit.fold(a0[u], a1[u], d0 + j + u);
    }
    for (; j < n; ++j) fit.fold(t0[(size_t)j * pitch + idx], W == 2 ? t1[(size_t)j * pitch + idx] : 0.0f, d0 + j);
}

// p <- x for the marked particles of quad q; clears the marks.
__device__ __forceinline__ void flush_quad(const SwarmArgs &a, uint32_t q)
{
    const uint32_t i0 = 4 * q;
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

} // namespace pso

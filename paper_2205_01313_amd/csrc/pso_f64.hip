// pso_f64.hip -- the binary64 path (the paper computes in double, Sec. 5).
//
// The method is the same as the binary32 kernels' (Alg. 1 Steps 1-5, Eq. 1
// and Eq. 2 with their clamps, synchronous gbest), evaluated in double from
// the binary32 parameters and the same 24-bit Philox uniforms.  Its fitness
// expressions are written operation for operation as the binary64 reference
// definition; Rastrigin and Ackley call the device's double cos and exp.
//
// Layout: x, v, p as double rows of Np particles (element (d, i) at
// d*Np + i).  Small swarms take one particle per lane (8-byte accesses, 512
// bytes per wavefront) and write a new pbest position at once; the grid step
// of a large swarm takes two particles per lane with 16-byte accesses and
// defers the pbest position into the next iteration's pass, as the binary32
// step does (k_step64w).  A 64-bit fitness
// and a particle index no longer fit one 64-bit word, so the gbest is not an
// atomic minimum: every workgroup writes its (order bits, index) minimum of
// the improved particles into its own slot, and the last workgroup to arrive
// reduces the slots (lowest index among equal fitness).
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <new>
#include <vector>

#include "pso.h"
#include "pso_device.hpp"
#include "pso_f64.hpp"
#include "pso_guard.hpp"
#include "pso_kernels.hpp"

int pso_internal_fail(int code, const char *fmt, ...);
int pso_internal_check_desc(const pso_desc *d);

namespace pso {

constexpr int BLOCK64 = 256;
constexpr uint32_t NO_IDX = 0xFFFFFFFFu;
constexpr uint32_t SPLIT64_MIN_P = 4; // fewest particles per workgroup of the split step

static inline size_t al256(size_t b) { return (b + 255) & ~size_t(255); }

Layout64 layout64_of(uint64_t N, int D)
{
    Layout64 L;
    L.Np = (N + 63) / 64 * 64;
    L.nblocks = (uint32_t)((N + BLOCK64 - 1) / BLOCK64);
    size_t o = 0;
    L.ctrl = o;     o += al256(sizeof(Ctrl64));
    L.gpos = o;     o += al256(sizeof(double) * D);
    L.shift = o;    o += al256(sizeof(double) * D);
    // one slot per workgroup of a grid step (the split step's may hold only
    // SPLIT64_MIN_P particles each), two per gang workgroup, six tagged
    // words per staged-gang workgroup
    const uint64_t nslots = std::max<uint64_t>(6 * (uint64_t)L.nblocks, (N + SPLIT64_MIN_P - 1) / SPLIT64_MIN_P);
    L.slot_ord = o; o += al256(sizeof(unsigned long long) * nslots);
    L.slot_idx = o; o += al256(sizeof(uint32_t) * nslots);
    L.cand_pos = o; o += al256(sizeof(double) * 4 * L.nblocks * (size_t)D); // two parities; tagged words: two per double
    L.pf = o;       o += al256(sizeof(double) * L.Np);
    L.pend = o;     o += al256(L.Np);
    L.x = o;        o += al256(sizeof(double) * L.Np * (size_t)D);
    L.v = o;        o += al256(sizeof(double) * L.Np * (size_t)D);
    L.p = o;        o += al256(sizeof(double) * L.Np * (size_t)D);
    L.total = o;
    return L;
}

Swarm64Args bind64(void *base, const Layout64 &L, uint64_t N, int D)
{
    char *b = static_cast<char *>(base);
    Swarm64Args a{};
    a.ctrl = reinterpret_cast<Ctrl64 *>(b + L.ctrl);
    a.gpos = reinterpret_cast<double *>(b + L.gpos);
    a.shift = reinterpret_cast<const double *>(b + L.shift);
    a.slot_ord = reinterpret_cast<unsigned long long *>(b + L.slot_ord);
    a.slot_idx = reinterpret_cast<uint32_t *>(b + L.slot_idx);
    a.cand_pos = reinterpret_cast<double *>(b + L.cand_pos);
    a.pf = reinterpret_cast<double *>(b + L.pf);
    a.pend = reinterpret_cast<uint8_t *>(b + L.pend);
    a.x = reinterpret_cast<double *>(b + L.x);
    a.v = reinterpret_cast<double *>(b + L.v);
    a.p = reinterpret_cast<double *>(b + L.p);
    a.N = (uint32_t)N;
    a.Np = (uint32_t)L.Np;
    a.D = D;
    return a;
}

// Order bits of a binary64: unsigned order = numeric order, -0 = +0, NaN last.
__device__ __forceinline__ unsigned long long ord64(double f)
{
    if (f != f) return ~0ull;
    if (f == 0.0) f = 0.0;
    const unsigned long long b = (unsigned long long)__double_as_longlong(f);
    return (b & 0x8000000000000000ull) ? ~b : (b | 0x8000000000000000ull);
}

// Inverse of ord64 (for non-NaN values; -0 comes back as +0).
__device__ __forceinline__ double ord64_value(unsigned long long o)
{
    const unsigned long long b = (o & 0x8000000000000000ull) ? (o & 0x7FFFFFFFFFFFFFFFull) : ~o;
    return __longlong_as_double((long long)b);
}

__device__ __forceinline__ double clampd(double v, double lo, double hi)
{
    v = (v < lo) ? lo : v;
    return (v > hi) ? hi : v;
}

// cos(pi y) after the exact reduction y = n + r.
__device__ __forceinline__ double cospi64(double y)
{
    const double n = rint(y);
    const double r = y - n;
    const double c = cos(M_PI * r);
    return fmod(n, 2.0) != 0.0 ? -c : c;
}

// The fitness functions in binary64, accumulated in dimension order.
template <int FIT>
struct Fitness64 {
    double acc = 0.0, aux = 0.0;

    __device__ __forceinline__ void add(double z, int d)
    {
        if constexpr (FIT == F_SPHERE) {
            acc = acc + z * z;
        } else if constexpr (FIT == F_RASTRIGIN) {
            acc = acc + (z * z - 10.0 * cospi64(2.0 * z));
        } else if constexpr (FIT == F_ROSENBROCK) {
            if (d > 0) {
                const double a = z - aux * aux;
                const double b = 1.0 - aux;
                acc = acc + (100.0 * a * a + b * b);
            }
            aux = z;
        } else if constexpr (FIT == F_ACKLEY) {
            acc = acc + z * z;
            aux = aux + cospi64(2.0 * z);
        } else {
            acc = acc + (z * z * z - 0.8 * z * z - 1000.0 * z + 8000.0);
        }
    }

    __device__ __forceinline__ double value(int D) const
    {
        if constexpr (FIT == F_RASTRIGIN) {
            return 10.0 * D + acc;
        } else if constexpr (FIT == F_ACKLEY) {
            return 20.0 - 20.0 * exp(-0.2 * sqrt(acc / D)) + M_E - exp(aux / D);
        } else if constexpr (FIT == F_CUBIC) {
            return -acc; // Eq. 3, negated: the paper maximises it
        } else {
            return acc;
        }
    }
};

__device__ __forceinline__ void lexmin(unsigned long long &k, uint32_t &i, unsigned long long k2, uint32_t i2)
{
    if (k2 < k || (k2 == k && i2 < i)) {
        k = k2;
        i = i2;
    }
}

// Workgroup lexicographic minimum of (k, i) over LANES lanes; the result is
// in every lane.  Ends with a barrier.
template <int LANES = BLOCK64>
__device__ void wg_lexmin(unsigned long long &k, uint32_t &i, unsigned long long *s_k, uint32_t *s_i)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        const unsigned long long k2 = __shfl_xor(k, off, 64);
        const uint32_t i2 = __shfl_xor(i, off, 64);
        lexmin(k, i, k2, i2);
    }
    constexpr int NW = LANES / 64; // wavefronts, a power of two
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 0) {
        s_k[w] = k;
        s_i[w] = i;
    }
    __syncthreads();
    if constexpr (NW > 1) {
        // every wavefront reduces the NW wavefront minima in its first NW
        // lanes (one LDS read each, then a butterfly) and broadcasts lane 0's
        k = lane < NW ? s_k[lane] : ~0ull;
        i = lane < NW ? s_i[lane] : NO_IDX;
#pragma unroll
        for (int off = NW / 2; off >= 1; off >>= 1) {
            const unsigned long long k2 = __shfl_xor(k, off, 64);
            const uint32_t i2 = __shfl_xor(i, off, 64);
            lexmin(k, i, k2, i2);
        }
        k = __shfl(k, 0, 64);
        i = __shfl(i, 0, 64);
    } else {
        k = s_k[0];
        i = s_i[0];
    }
    __syncthreads();
}

// Wavefront lexicographic minimum of the candidates (lanes with i != NO_IDX,
// k != ~0) in every lane.  Beating the gbest is rare after the first
// iterations, so a wavefront with no candidate or one takes no shuffles.
__device__ __forceinline__ void wave_lexmin_sparse(unsigned long long &k, uint32_t &i)
{
    const unsigned long long m = __ballot(i != NO_IDX);
    if (m == 0) {
        k = ~0ull;
        i = NO_IDX;
    } else if ((m & (m - 1)) == 0) {
        const int l = __builtin_ctzll(m);
        const uint32_t lo = __builtin_amdgcn_readlane((uint32_t)k, l), hi = __builtin_amdgcn_readlane((uint32_t)(k >> 32), l);
        k = ((unsigned long long)hi << 32) | lo;
        i = __builtin_amdgcn_readlane(i, l);
    } else {
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) {
            const unsigned long long k2 = __shfl_xor(k, off, 64);
            const uint32_t i2 = __shfl_xor(i, off, 64);
            lexmin(k, i, k2, i2);
        }
    }
}

// Workgroup form of wave_lexmin_sparse: the wavefront minima meet in LDS
// behind one barrier.  No barrier at the end: the caller holds one between
// this call and its next.
template <int LANES>
__device__ __forceinline__ void wg_lexmin_sparse(unsigned long long &k, uint32_t &i, unsigned long long *s_k,
                                                 uint32_t *s_i)
{
    wave_lexmin_sparse(k, i);
    constexpr int NW = LANES / 64;
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 0) {
        s_k[w] = k;
        s_i[w] = i;
    }
    __syncthreads();
    k = lane < NW ? s_k[lane] : ~0ull;
    i = lane < NW ? s_i[lane] : NO_IDX;
    wave_lexmin_sparse(k, i);
}

// Step 1 for particle i: x ~ U[lo, hi), v ~ U[-vmax, vmax), p = x; returns F(x).
template <int FIT>
__device__ double init_particle64(const Swarm64Args &a, uint32_t i, const double *s_shift)
{
    const size_t Np = a.Np;
    const int D = a.D;
    Fitness64<FIT> fit;
    for (int d = 0; d < D; d += 2) {
        const U4 u = philox4x32_10(a.k0, a.k1, (uint32_t)d >> 1, i, 0u, TAG_INIT);
        for (int h = 0; h < 2 && d + h < D; ++h) {
            const double u0 = (double)unit_float(h ? u.c : u.a), u1 = (double)unit_float(h ? u.d : u.b);
            const double x = clampd(a.lo + (a.hi - a.lo) * u0, a.lo, a.hi);
            const double v = clampd(-a.vmax + 2.0 * a.vmax * u1, -a.vmax, a.vmax);
            const size_t e = (size_t)(d + h) * Np + i;
            a.x[e] = x;
            a.v[e] = v;
            a.p[e] = x;
            fit.add(x - s_shift[d + h], d + h);
        }
    }
    return fit.value(D);
}

// Steps 2-4 of iteration t for particle i; returns the order bits of its new
// pbest fitness if it improved (strictly), else ~0.
template <int FIT>
__device__ unsigned long long iterate_particle64(const Swarm64Args &a, uint32_t i, uint32_t t, const double *s_g,
                                                 const double *s_shift)
{
    const size_t Np = a.Np;
    const int D = a.D;
    Fitness64<FIT> fit;
    for (int d = 0; d < D; d += 2) {
        const U4 u = philox4x32_10(a.k0, a.k1, (uint32_t)d >> 1, i, t, TAG_VEL);
        for (int h = 0; h < 2 && d + h < D; ++h) {
            const double r1 = (double)unit_float(h ? u.c : u.a), r2 = (double)unit_float(h ? u.d : u.b);
            const size_t e = (size_t)(d + h) * Np + i;
            const double x = a.x[e], v = a.v[e], p = a.p[e];
            // Eq. 1 left to right, clamp to [-vmax, vmax]; Eq. 2, clamp to [lo, hi]
            double vn = a.w * v + a.c1 * r1 * (p - x) + a.c2 * r2 * (s_g[d + h] - x);
            vn = clampd(vn, -a.vmax, a.vmax);
            const double xn = clampd(x + vn, a.lo, a.hi);
            a.x[e] = xn;
            a.v[e] = vn;
            fit.add(xn - s_shift[d + h], d + h);
        }
    }
    const double f = fit.value(D);
    if (!(f < a.pf[i])) return ~0ull; // strict; NaN never improves
    a.pf[i] = f;
    for (int d = 0; d < D; ++d) a.p[(size_t)d * Np + i] = a.x[(size_t)d * Np + i];
    return ord64(f);
}

// The last workgroup of a grid launch: reduce the slots; a better gbest than
// the control block's (or any, at Step 1) becomes the gbest of iteration t.
__device__ void finish64(const Swarm64Args &a, uint32_t t, bool first, unsigned long long *s_k, uint32_t *s_i)
{
    Ctrl64 *c = a.ctrl;
    unsigned long long k = ~0ull;
    uint32_t i = NO_IDX;
    for (uint32_t b = threadIdx.x; b < gridDim.x; b += BLOCK64) lexmin(k, i, a.slot_ord[b], a.slot_idx[b]);
    wg_lexmin(k, i, s_k, s_i);
    const bool changed = i != NO_IDX;
    if (changed)
        for (int d = threadIdx.x; d < a.D; d += BLOCK64) a.gpos[d] = a.x[(size_t)d * a.Np + i];
    if (threadIdx.x == 0) {
        if (changed) {
            c->gord = k;
            c->gidx = i;
            c->giter = first ? 0 : (long long)t;
        }
        c->t = first ? 0 : (long long)t;
        c->arrive = 0;
        if (first) c->stop = 0;
        const double gf = a.pf[c->gidx];
        if (c->tol > 0.0 && fabs(gf - c->fstar) < c->tol) c->stop = 1;
    }
}

// Posts the workgroup minimum and arrives; true in every lane of the last
// workgroup (after its acquire).
__device__ bool post_and_arrive64(const Swarm64Args &a, unsigned long long k, uint32_t i, int *last)
{
    if (threadIdx.x == 0) {
        a.slot_ord[blockIdx.x] = k;
        a.slot_idx[blockIdx.x] = i;
        __threadfence(); // release: the slot and this workgroup's x (ordered by the barrier)
        const unsigned int ticket = atomicAdd(&a.ctrl->arrive, 1u);
        const int l = ticket == gridDim.x - 1;
        if (l) __threadfence(); // acquire every slot and position
        *last = l;
    }
    __syncthreads();
    return *last != 0;
}

template <int FIT>
__global__ void __launch_bounds__(BLOCK64) k_init64(Swarm64Args a)
{
    __shared__ unsigned long long s_k[BLOCK64 / 64];
    __shared__ uint32_t s_i[BLOCK64 / 64];
    __shared__ int last;
    extern __shared__ double s_shift64[];
    for (int d = threadIdx.x; d < a.D; d += BLOCK64) s_shift64[d] = a.shift[d];
    __syncthreads();
    const uint32_t i = blockIdx.x * BLOCK64 + threadIdx.x;
    unsigned long long k = ~0ull;
    uint32_t ki = NO_IDX;
    if (i < a.Np) a.pend[i] = 0;
    if (i < a.N) {
        const double f = init_particle64<FIT>(a, i, s_shift64);
        a.pf[i] = f;
        k = ord64(f);
        ki = i;
    }
    wg_lexmin(k, ki, s_k, s_i);
    if (post_and_arrive64(a, k, ki, &last)) finish64(a, 0u, true, s_k, s_i);
}

template <int FIT>
__global__ void __launch_bounds__(BLOCK64) k_step64(Swarm64Args a)
{
    __shared__ unsigned long long s_k[BLOCK64 / 64];
    __shared__ uint32_t s_i[BLOCK64 / 64];
    __shared__ int last;
    extern __shared__ double s_dyn64[]; // gbest position (D), shift (D)
    Ctrl64 *c = a.ctrl;
    if (c->stop) return;
    const int D = a.D;
    double *s_g = s_dyn64, *s_shift = s_dyn64 + D;
    for (int d = threadIdx.x; d < D; d += BLOCK64) {
        s_g[d] = a.gpos[d];
        s_shift[d] = a.shift[d];
    }
    const uint32_t t = (uint32_t)(c->t + 1);
    const unsigned long long pk = c->gord;
    const uint32_t pi = c->gidx;
    __syncthreads();
    const uint32_t i = blockIdx.x * BLOCK64 + threadIdx.x;
    unsigned long long k = ~0ull;
    uint32_t ki = NO_IDX;
    if (i < a.N) {
        const unsigned long long o = iterate_particle64<FIT>(a, i, t, s_g, s_shift);
        if (o < pk || (o == pk && i < pi)) {
            k = o;
            ki = i;
        }
    }
    wg_lexmin(k, ki, s_k, s_i);
    if (post_and_arrive64(a, k, ki, &last)) finish64(a, t, false, s_k, s_i);
}

// ---------------------------------------------------------------------------
// Grid step of a swarm too small to fill the GPU with one particle per lane
// (N = 1024, D = 120 is four workgroups): P particles per workgroup, L =
// 256 / P lanes per particle, lane k * P + j takes dimensions [k C, (k+1) C)
// of particle j (C even: whole Philox pairs), so the P lanes of a chunk read
// P consecutive doubles of a row.  Each lane stages its dimensions' fitness
// terms in LDS ([word][d][j]); after a barrier lane j folds particle j's
// terms in dimension order (the terms are the expressions Fitness64::add
// evaluates, Rosenbrock's from the staged z), so the fitness is the same
// sequential sum, bit for bit.  New pbest positions are left in x and
// marked in pend, as in the wide step; the next iteration writes them to p.
// ---------------------------------------------------------------------------
template <int FIT>
__host__ __device__ constexpr int split64_words() { return FIT == F_ACKLEY ? 2 : 1; }

template <int FIT>
__device__ __forceinline__ void split64_stage(double z, double *t0, double *t1)
{
    if constexpr (FIT == F_SPHERE) {
        *t0 = z * z;
    } else if constexpr (FIT == F_RASTRIGIN) {
        *t0 = z * z - 10.0 * cospi64(2.0 * z);
    } else if constexpr (FIT == F_ACKLEY) {
        *t0 = z * z;
        *t1 = cospi64(2.0 * z);
    } else if constexpr (FIT == F_CUBIC) {
        *t0 = z * z * z - 0.8 * z * z - 1000.0 * z + 8000.0;
    } else {
        *t0 = z; // Rosenbrock: the fold evaluates the terms
    }
}

template <int FIT>
__device__ __forceinline__ double split64_fold(const double *t0, const double *t1, uint32_t P, int D)
{
    Fitness64<FIT> fit;
    int d = 0;
    for (; d + 8 <= D; d += 8) {
        double a0[8], a1[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            a0[u] = t0[(size_t)(d + u) * P];
            if constexpr (split64_words<FIT>() == 2) a1[u] = t1[(size_t)(d + u) * P];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            if constexpr (FIT == F_ROSENBROCK) {
                fit.add(a0[u], d + u);
            } else {
                fit.acc = fit.acc + a0[u];
                if constexpr (split64_words<FIT>() == 2) fit.aux = fit.aux + a1[u];
            }
        }
    }
    for (; d < D; ++d) {
        if constexpr (FIT == F_ROSENBROCK) {
            fit.add(t0[(size_t)d * P], d);
        } else {
            fit.acc = fit.acc + t0[(size_t)d * P];
            if constexpr (split64_words<FIT>() == 2) fit.aux = fit.aux + t1[(size_t)d * P];
        }
    }
    return fit.value(D);
}

template <int FIT>
__global__ void __launch_bounds__(BLOCK64) k_step64s(Swarm64Args a, uint32_t P, uint32_t C)
{
    __shared__ unsigned long long s_k[BLOCK64 / 64];
    __shared__ uint32_t s_i[BLOCK64 / 64];
    __shared__ int last;
    extern __shared__ double s_dyn64[]; // gbest position (D), shift (D), terms [word][D][P]
    Ctrl64 *c = a.ctrl;
    if (c->stop) return;
    const int D = a.D;
    const size_t Np = a.Np;
    double *s_g = s_dyn64, *s_shift = s_dyn64 + D, *s_t0 = s_shift + D, *s_t1 = s_t0 + (size_t)D * P;
    for (int d = threadIdx.x; d < D; d += BLOCK64) {
        s_g[d] = a.gpos[d];
        s_shift[d] = a.shift[d];
    }
    const uint32_t t = (uint32_t)(c->t + 1);
    const unsigned long long pk = c->gord;
    const uint32_t pi = c->gidx;
    const uint32_t j = threadIdx.x % P, kc = threadIdx.x / P;
    const uint32_t i = blockIdx.x * P + j;
    const bool act = i < a.N;
    const bool pend = act && a.pend[i] != 0;
    const bool folder = act && kc == 0;
    const double pf_old = folder ? a.pf[i] : 0.0;
    const int d_begin = (int)(kc * C), d_end = min(D, (int)((kc + 1) * C));
    // software pipeline over the chunk's dimension pairs: the next pair's
    // rows are loaded before this pair's stores (the first pair's before
    // the barrier that publishes the gbest position and shift)
    double nx[2] = {0.0, 0.0}, nv[2] = {0.0, 0.0}, np[2] = {0.0, 0.0};
    auto load_pair = [&](int d) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            if (d + h < d_end) {
                const size_t e = (size_t)(d + h) * Np + i;
                nx[h] = a.x[e];
                nv[h] = a.v[e];
                np[h] = pend ? nx[h] : a.p[e];
            }
        }
    };
    if (act) load_pair(d_begin);
    __syncthreads();
    if (act) {
        for (int d = d_begin; d < d_end; d += 2) {
            const double cx[2] = {nx[0], nx[1]}, cv[2] = {nv[0], nv[1]}, cp[2] = {np[0], np[1]};
            if (d + 2 < d_end) load_pair(d + 2);
            const U4 u = philox4x32_10(a.k0, a.k1, (uint32_t)d >> 1, i, t, TAG_VEL);
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                if (d + h >= d_end) break;
                const double r1 = (double)unit_float(h ? u.c : u.a), r2 = (double)unit_float(h ? u.d : u.b);
                const size_t e = (size_t)(d + h) * Np + i;
                const double x = cx[h], v = cv[h], p = cp[h];
                // Eq. 1 left to right, clamp to [-vmax, vmax]; Eq. 2, clamp to [lo, hi]
                double vn = a.w * v + a.c1 * r1 * (p - x) + a.c2 * r2 * (s_g[d + h] - x);
                vn = clampd(vn, -a.vmax, a.vmax);
                const double xn = clampd(x + vn, a.lo, a.hi);
                a.x[e] = xn;
                a.v[e] = vn;
                if (pend) a.p[e] = p;
                const size_t at = (size_t)(d + h) * P + j;
                double w1 = 0.0;
                split64_stage<FIT>(xn - s_shift[d + h], &s_t0[at], &w1);
                if constexpr (split64_words<FIT>() == 2) s_t1[at] = w1;
            }
        }
    }
    __syncthreads();
    unsigned long long k = ~0ull;
    uint32_t ki = NO_IDX;
    if (folder) {
        const double f = split64_fold<FIT>(s_t0 + j, s_t1 + j, P, D);
        const bool imp = f < pf_old; // strict; NaN never improves
        if (imp) {
            a.pf[i] = f;
            const unsigned long long o = ord64(f);
            if (o < pk || (o == pk && i < pi)) {
                k = o;
                ki = i;
            }
        }
        a.pend[i] = imp ? 1 : 0;
    }
    wg_lexmin(k, ki, s_k, s_i); // its barriers order every lane's x stores before the release below
    if (post_and_arrive64(a, k, ki, &last)) finish64(a, t, false, s_k, s_i);
}

// ---------------------------------------------------------------------------
// Grid step of a large swarm: lane q owns particles 2q and 2q+1 and walks
// their dimensions in order with 16-byte accesses of one dimension's row
// (1 KiB per wavefront), the next dimension pair's rows loaded ahead.  A
// particle whose pbest improves is marked in pend and its new pbest
// position left in x; the next iteration reads x anyway, takes it as the
// pbest position of marked particles and writes p for every lane of a
// 64-byte group (4 lanes) holding a mark.  x may be kept in the
// memory-side cache while v and p stream (cache_policy).  The arithmetic
// of every element is iterate_particle64's, so the results are the same bits.
// ---------------------------------------------------------------------------
typedef double d2 __attribute__((ext_vector_type(2)));

template <bool KEEP>
__device__ __forceinline__ d2 ld64(const double *row, uint32_t q)
{
    if constexpr (KEEP)
        return *(reinterpret_cast<const d2 *>(row) + q);
    else
        return __builtin_nontemporal_load(reinterpret_cast<const d2 *>(row) + q);
}

template <bool KEEP>
__device__ __forceinline__ void st64(double *row, uint32_t q, d2 v)
{
    if constexpr (KEEP)
        *(reinterpret_cast<d2 *>(row) + q) = v;
    else
        __builtin_nontemporal_store(v, reinterpret_cast<d2 *>(row) + q);
}

template <int FIT, int POL>
__global__ void __launch_bounds__(BLOCK64) k_step64w(Swarm64Args a)
{
    __shared__ unsigned long long s_k[BLOCK64 / 64];
    __shared__ uint32_t s_i[BLOCK64 / 64];
    __shared__ int last;
    extern __shared__ double s_dyn64[]; // gbest position (D), shift (D)
    constexpr bool KX = (POL & KEEP_X) != 0, KV = (POL & KEEP_V) != 0, KP = (POL & KEEP_P) != 0;
    Ctrl64 *c = a.ctrl;
    if (c->stop) return;
    const int D = a.D;
    const size_t Np = a.Np;
    double *s_g = s_dyn64, *s_shift = s_dyn64 + D;
    for (int d = threadIdx.x; d < D; d += BLOCK64) {
        s_g[d] = a.gpos[d];
        s_shift[d] = a.shift[d];
    }
    const uint32_t t = (uint32_t)(c->t + 1);
    const unsigned long long pk = c->gord;
    const uint32_t pi = c->gidx;
    const uint32_t q = blockIdx.x * BLOCK64 + threadIdx.x, i0 = 2 * q;
    const bool active = i0 < a.N;
    const uint32_t pend = active ? *reinterpret_cast<const uint16_t *>(a.pend + i0) : 0u;
    const d2 pf_old = active ? *reinterpret_cast<const d2 *>(a.pf + i0) : d2{0.0, 0.0};
    __syncthreads();
    const unsigned long long dirty = __ballot(pend != 0u);
    const bool line_dirty = ((dirty >> ((threadIdx.x & 63) & ~3u)) & 0xFull) != 0;
    Fitness64<FIT> fit[2];
    if (active) {
        d2 ax[2], av[2], ap[2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            if (h < D) {
                ax[h] = ld64<KX>(a.x + (size_t)h * Np, q);
                av[h] = ld64<KV>(a.v + (size_t)h * Np, q);
                ap[h] = ld64<KP>(a.p + (size_t)h * Np, q);
            }
        }
        for (int d = 0; d < D; d += 2) {
            d2 cx[2], cv[2], cp[2];
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
                    ax[h] = ld64<KX>(a.x + row, q);
                    av[h] = ld64<KV>(a.v + row, q);
                    ap[h] = ld64<KP>(a.p + row, q);
                }
            }
            U4 u[2];
#pragma unroll
            for (int k = 0; k < 2; ++k) u[k] = philox4x32_10(a.k0, a.k1, (uint32_t)d >> 1, i0 + k, t, TAG_VEL);
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                if (d + h >= D) break;
                const size_t row = (size_t)(d + h) * Np;
                d2 ps = cp[h], xn, vn;
#pragma unroll
                for (int k = 0; k < 2; ++k) {
                    if (pend & (0xFFu << (8 * k))) ps[k] = cx[h][k];
                    const double x = cx[h][k], v = cv[h][k], p = ps[k];
                    const double r1 = (double)unit_float(h ? u[k].c : u[k].a);
                    const double r2 = (double)unit_float(h ? u[k].d : u[k].b);
                    // Eq. 1 left to right, clamp to [-vmax, vmax]; Eq. 2, clamp to [lo, hi]
                    double nv = a.w * v + a.c1 * r1 * (p - x) + a.c2 * r2 * (s_g[d + h] - x);
                    nv = clampd(nv, -a.vmax, a.vmax);
                    vn[k] = nv;
                    xn[k] = clampd(x + nv, a.lo, a.hi);
                    fit[k].add(xn[k] - s_shift[d + h], d + h);
                }
                st64<KX>(a.x + row, q, xn);
                st64<KV>(a.v + row, q, vn);
                if (line_dirty) st64<KP>(a.p + row, q, ps);
            }
        }
    }
    // Step 4: strict improvement (NaN never improves); candidates for the
    // gbest as in k_step64
    unsigned long long k = ~0ull;
    uint32_t ki = NO_IDX;
    if (active) {
        uint32_t pend_new = 0;
        d2 pf_new = pf_old;
#pragma unroll
        for (int kk = 0; kk < 2; ++kk) {
            const uint32_t i = i0 + kk;
            if (i >= a.N) continue;
            const double f = fit[kk].value(D);
            if (!(f < pf_old[kk])) continue;
            pf_new[kk] = f;
            pend_new |= 1u << (8 * kk);
            const unsigned long long o = ord64(f);
            if (o < pk || (o == pk && i < pi)) lexmin(k, ki, o, i);
        }
        if (pend_new) *reinterpret_cast<d2 *>(a.pf + i0) = pf_new;
        if (pend_new != pend) *reinterpret_cast<uint16_t *>(a.pend + i0) = (uint16_t)pend_new;
    }
    wg_lexmin(k, ki, s_k, s_i);
    if (post_and_arrive64(a, k, ki, &last)) finish64(a, t, false, s_k, s_i);
}

// Steps 2-4 of iteration t for particle i, column j of the state staged in
// LDS as rows of nl doubles (x, v, p; pf at j): iterate_particle64's
// arithmetic.  A particle whose pbest improves (strictly) and whose key
// (order bits, index) beats the gbest's (gk, gi) joins the lane's minimum
// (k, ki); the test runs only in the improving lanes.  The clamp bounds come
// in vector registers.
template <int FIT>
__device__ __forceinline__ void staged_particle64(const Swarm64Args &a, int D, uint32_t nl, uint32_t j, uint32_t i,
                                                  uint32_t t, double *sx, double *sv, double *sp, double *spf,
                                                  const double *s_g, const double *s_shift, double vlo, double vhi,
                                                  double xlo, double xhi, unsigned long long gk, uint32_t gi,
                                                  unsigned long long &k, uint32_t &ki)
{
    Fitness64<FIT> fit;
    for (int d = 0; d < D; d += 2) {
        const U4 u = philox4x32_10(a.k0, a.k1, (uint32_t)d >> 1, i, t, TAG_VEL);
        for (int h = 0; h < 2 && d + h < D; ++h) {
            const double r1 = (double)unit_float(h ? u.c : u.a), r2 = (double)unit_float(h ? u.d : u.b);
            const size_t e = (size_t)(d + h) * nl + j;
            const double x = sx[e], v = sv[e], p = sp[e];
            // Eq. 1 left to right, clamp to [-vmax, vmax]; Eq. 2, clamp to [lo, hi]
            double vn = a.w * v + a.c1 * r1 * (p - x) + a.c2 * r2 * (s_g[d + h] - x);
            vn = clampd(vn, vlo, vhi);
            const double xn = clampd(x + vn, xlo, xhi);
            sx[e] = xn;
            sv[e] = vn;
            fit.add(xn - s_shift[d + h], d + h);
        }
    }
    const double f = fit.value(D);
    if (f < spf[j]) { // strict; NaN never improves
        spf[j] = f;
        for (int d = 0; d < D; ++d) sp[(size_t)d * nl + j] = sx[(size_t)d * nl + j];
        const unsigned long long o = ord64(f);
        if (o < gk || (o == gk && i < gi)) lexmin(k, ki, o, i);
    }
}

// ---------------------------------------------------------------------------
// Up to T iterations of a small swarm in one workgroup with its whole state
// in LDS: x, v, p as rows of N doubles, then pf, loaded once and stored back
// at the end.  An iteration then waits on no device-memory access (the
// unstaged form below waits on the state's loads, the pbest fitness after
// the stores, and the new gbest position: about 3 us per iteration at
// N = 1024, D = 1).  Lane t runs particles t, t + LANES, ... with
// iterate_particle64's arithmetic, so the results are the same bits.  ONE:
// the paper's one-dimensional problems, loops resolved at compile time.
// ---------------------------------------------------------------------------
template <int FIT, int LANES, bool ONE>
__global__ void __launch_bounds__(LANES) k_block_run64s(Swarm64Args a, long long T)
{
    __shared__ unsigned long long s_k[LANES / 64];
    __shared__ uint32_t s_i[LANES / 64];
    extern __shared__ double s_dyn64[]; // gbest position (D), shift (D), x, v, p (D x N each), pf (N)
    Ctrl64 *c = a.ctrl;
    const int D = ONE ? 1 : a.D;
    const uint32_t N = a.N;
    const size_t Np = a.Np, rows = (size_t)D * N;
    double *s_g = s_dyn64, *s_shift = s_g + D, *sx = s_shift + D, *sv = sx + rows, *sp = sv + rows, *spf = sp + rows;
    for (int d = threadIdx.x; d < D; d += LANES) {
        s_g[d] = a.gpos[d];
        s_shift[d] = a.shift[d];
    }
    for (size_t e = threadIdx.x; e < rows; e += LANES) {
        const size_t d = e / N, i = e % N, g = d * Np + i;
        sx[e] = a.x[g];
        sv[e] = a.v[g];
        sp[e] = a.p[g];
    }
    for (uint32_t i = threadIdx.x; i < N; i += LANES) spf[i] = a.pf[i];
    unsigned long long gk = c->gord;
    uint32_t gi = c->gidx;
    long long giter = c->giter, t = c->t;
    bool stop = c->stop != 0;
    const double tol = c->tol, fstar = c->fstar;
    // the clamp bounds in vector registers for the whole run: a select
    // between a lane value and a scalar operand costs a move per half
    double vlo = -a.vmax, vhi = a.vmax, xlo = a.lo, xhi = a.hi;
    asm volatile("" : "+v"(vlo), "+v"(vhi), "+v"(xlo), "+v"(xhi));
    __syncthreads();
    for (long long it = 0; it < T && !stop; ++it) {
        const uint32_t t1 = (uint32_t)(t + 1);
        unsigned long long k = ~0ull;
        uint32_t ki = NO_IDX;
        for (uint32_t i = threadIdx.x; i < N; i += LANES)
            staged_particle64<FIT>(a, D, N, i, i, t1, sx, sv, sp, spf, s_g, s_shift, vlo, vhi, xlo, xhi, gk, gi, k, ki);
        wg_lexmin_sparse<LANES>(k, ki, s_k, s_i); // its barrier follows every lane's LDS stores
        if (ki != NO_IDX) {
            gk = k;
            gi = ki;
            giter = t1;
            for (int d = threadIdx.x; d < D; d += LANES) s_g[d] = sx[(size_t)d * N + gi];
        }
        t = t1;
        stop = tol > 0.0 && fabs(spf[gi] - fstar) < tol;
        __syncthreads();
    }
    for (size_t e = threadIdx.x; e < rows; e += LANES) {
        const size_t d = e / N, i = e % N, g = d * Np + i;
        a.x[g] = sx[e];
        a.v[g] = sv[e];
        a.p[g] = sp[e];
    }
    for (uint32_t i = threadIdx.x; i < N; i += LANES) a.pf[i] = spf[i];
    for (int d = threadIdx.x; d < D; d += LANES) a.gpos[d] = s_g[d];
    if (threadIdx.x == 0) {
        c->gord = gk;
        c->gidx = gi;
        c->giter = giter;
        c->t = t;
        c->stop = stop ? 1u : 0u;
    }
}

// p <- x for every pending particle; clears the marks.
__global__ void __launch_bounds__(BLOCK64) k_flush64(Swarm64Args a)
{
    const uint32_t i = blockIdx.x * BLOCK64 + threadIdx.x;
    if (i >= a.N || !a.pend[i]) return;
    for (int d = 0; d < a.D; ++d) a.p[(size_t)d * a.Np + i] = a.x[(size_t)d * a.Np + i];
    a.pend[i] = 0;
}

// Up to T iterations of a small swarm in one workgroup of LANES lanes
// (gbest position in LDS).
template <int FIT, int LANES>
__global__ void __launch_bounds__(LANES) k_block_run64(Swarm64Args a, long long T)
{
    __shared__ unsigned long long s_k[LANES / 64];
    __shared__ uint32_t s_i[LANES / 64];
    extern __shared__ double s_dyn64[];
    Ctrl64 *c = a.ctrl;
    const int D = a.D;
    double *s_g = s_dyn64, *s_shift = s_dyn64 + D;
    for (int d = threadIdx.x; d < D; d += LANES) {
        s_g[d] = a.gpos[d];
        s_shift[d] = a.shift[d];
    }
    unsigned long long gk = c->gord;
    uint32_t gi = c->gidx;
    long long giter = c->giter, t = c->t;
    bool stop = c->stop != 0;
    const double tol = c->tol, fstar = c->fstar;
    __syncthreads();
    for (long long it = 0; it < T && !stop; ++it) {
        const uint32_t t1 = (uint32_t)(t + 1);
        unsigned long long k = ~0ull;
        uint32_t ki = NO_IDX;
        for (uint32_t i = threadIdx.x; i < a.N; i += LANES) {
            const unsigned long long o = iterate_particle64<FIT>(a, i, t1, s_g, s_shift);
            if (o < gk || (o == gk && i < gi)) lexmin(k, ki, o, i);
        }
        wg_lexmin<LANES>(k, ki, s_k, s_i); // every lane's x and pf stores precede it
        if (ki != NO_IDX) {
            gk = k;
            gi = ki;
            giter = t1;
            for (int d = threadIdx.x; d < D; d += LANES) s_g[d] = a.x[(size_t)d * a.Np + gi];
        }
        t = t1;
        stop = tol > 0.0 && fabs(a.pf[gi] - fstar) < tol;
        __syncthreads();
    }
    for (int d = threadIdx.x; d < D; d += LANES) a.gpos[d] = s_g[d];
    if (threadIdx.x == 0) {
        c->gord = gk;
        c->gidx = gi;
        c->giter = giter;
        c->t = t;
        c->stop = stop ? 1u : 0u;
    }
}

// ---------------------------------------------------------------------------
// Persistent gang (synchronous): the launch's G co-resident workgroups each
// own a contiguous slice of particles and run T iterations, meeting once per
// iteration.  Workgroup b posts its lexicographic minimum of the improved
// particles and, if it has one, that particle's position into the slots of
// the iteration's parity, then arrives; once all G arrivals of the iteration
// are in, every workgroup reduces the same G slots the same way, so all agree
// on the gbest and on the stop rule, and read the winner's position from its
// staged copy (its owner may already be overwriting x in the next
// iteration; the slots of that iteration have the other parity).  The
// arrival count is monotonic (G per iteration); every wait is bounded by the
// wall clock and sets an error bit if it gives up.
// ---------------------------------------------------------------------------
constexpr unsigned long long GANG64_WAIT_TICKS = 2000000000ull; // 20 s of the 100 MHz wall clock
constexpr uint32_t GANG64S_MAX_G = 256;                          // workgroups of a staged gang at most

template <int FIT>
__global__ void __launch_bounds__(BLOCK64) k_gang64(Swarm64Args a, long long T, uint32_t per_wg)
{
    __shared__ unsigned long long s_k[BLOCK64 / 64];
    __shared__ uint32_t s_i[BLOCK64 / 64];
    __shared__ int s_fail;
    extern __shared__ double s_dyn64[]; // gbest position (D), shift (D)
    Ctrl64 *c = a.ctrl;
    const int D = a.D;
    const uint32_t G = gridDim.x, b = blockIdx.x;
    double *s_g = s_dyn64, *s_shift = s_dyn64 + D;
    for (int d = threadIdx.x; d < D; d += BLOCK64) {
        s_g[d] = a.gpos[d];
        s_shift[d] = a.shift[d];
    }
    unsigned long long gk = c->gord;
    uint32_t gi = c->gidx;
    long long giter = c->giter, t = c->t;
    bool stop = c->stop != 0;
    const double tol = c->tol, fstar = c->fstar;
    const uint32_t i_lo = b * per_wg, i_hi = min(a.N, i_lo + per_wg);
    if (threadIdx.x == 0) s_fail = 0;
    __syncthreads();
    for (long long it = 0; it < T && !stop; ++it) {
        const uint32_t t1 = (uint32_t)(t + 1);
        const int par = (int)(it & 1);
        unsigned long long k = ~0ull;
        uint32_t ki = NO_IDX;
        for (uint32_t i = i_lo + threadIdx.x; i < i_hi; i += BLOCK64) {
            const unsigned long long o = iterate_particle64<FIT>(a, i, t1, s_g, s_shift);
            if (o < gk || (o == gk && i < gi)) lexmin(k, ki, o, i);
        }
        wg_lexmin(k, ki, s_k, s_i); // every lane's stores precede it
        double *mine = a.cand_pos + ((size_t)par * G + b) * D;
        if (ki != NO_IDX)
            for (int d = threadIdx.x; d < D; d += BLOCK64) mine[d] = a.x[(size_t)d * a.Np + ki];
        __syncthreads();
        if (threadIdx.x == 0) {
            a.slot_ord[par * G + b] = k;
            a.slot_idx[par * G + b] = ki;
            __threadfence(); // release the slot and the staged position
            atomicAdd(&c->gang_arrive, 1ull);
            const unsigned long long target = (unsigned long long)G * (unsigned long long)(it + 1);
            const unsigned long long w0 = wall_clock64();
            while (__hip_atomic_load(&c->gang_arrive, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
                __builtin_amdgcn_s_sleep(1);
                if (wall_clock64() - w0 > GANG64_WAIT_TICKS) {
                    atomicOr(&c->err, 1u);
                    s_fail = 1;
                    break;
                }
            }
            __threadfence(); // acquire every slot and staged position
        }
        __syncthreads();
        if (s_fail) break; // uniform
        // every workgroup reduces the same slots
        unsigned long long rk = ~0ull;
        uint32_t ri = NO_IDX, rb = NO_IDX;
        for (uint32_t w = threadIdx.x; w < G; w += BLOCK64) {
            const unsigned long long sk =
                __hip_atomic_load(&a.slot_ord[par * G + w], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            const uint32_t si = __hip_atomic_load(&a.slot_idx[par * G + w], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (sk < rk || (sk == rk && si < ri)) {
                rk = sk;
                ri = si;
                rb = w;
            }
        }
        // carry the owning workgroup along with the index (indices are unique)
        wg_lexmin(rk, ri, s_k, s_i);
        if (ri != NO_IDX) {
            rb = ri / per_wg;
            const double *src = a.cand_pos + ((size_t)par * G + rb) * D;
            for (int d = threadIdx.x; d < D; d += BLOCK64)
                s_g[d] = __hip_atomic_load(&src[d], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            gk = rk;
            gi = ri;
            giter = t1;
        }
        t = t1;
        // every workgroup holds the same key, so all take the same decision
        // (the winner's pf may already be changing in its next iteration)
        stop = tol > 0.0 && fabs(ord64_value(gk) - fstar) < tol;
        __syncthreads();
    }
    if (b == 0) {
        for (int d = threadIdx.x; d < D; d += BLOCK64) a.gpos[d] = s_g[d];
        if (threadIdx.x == 0) {
            c->gord = gk;
            c->gidx = gi;
            c->giter = giter;
            c->t = t;
            c->stop = stop ? 1u : 0u;
        }
    }
}

// The gang with each workgroup's slice of the swarm (x, v, p as rows of
// per_wg doubles, pf) in LDS for the whole run, loaded once and stored back
// at the end, so an iteration reads no state from device memory.  The
// meeting uses no fences: every word a workgroup posts -- its key (order
// bits in two words, index in one) and its candidate position (two words
// per double) -- carries the iteration number in its high half and is
// written and read with relaxed device-scope atomics, which are coherent
// per word; a reader waits for each word it needs to carry the current
// iteration.  (An agent-scope release and acquire write back and
// invalidate the XCD's L2: 1.2-3 us of an iteration.)  Words of the other
// parity cannot be overwritten early: a workgroup posts iteration t + 2
// only after every workgroup has posted t + 1, after reading t.  The words
// are cleared before each launch (a previous run's iteration numbers could
// match).  Same arithmetic and choice of gbest as k_gang64, so the same
// results.
template <int FIT, bool ONE>
__global__ void __launch_bounds__(BLOCK64) k_gang64s(Swarm64Args a, long long T, uint32_t per_wg)
{
    __shared__ unsigned long long s_k[BLOCK64 / 64];
    __shared__ uint32_t s_i[BLOCK64 / 64];
    __shared__ int s_fail;
    __shared__ uint32_t s_word[3 * GANG64S_MAX_G]; // payloads of the tagged words read in a meeting
    extern __shared__ double s_dyn64[]; // gbest position (D), shift (D), x, v, p (D x per_wg each), pf (per_wg)
    Ctrl64 *c = a.ctrl;
    const int D = ONE ? 1 : a.D;
    const uint32_t G = gridDim.x, b = blockIdx.x;
    const uint32_t i_lo = b * per_wg, n_loc = min(a.N, i_lo + per_wg) - i_lo;
    const size_t Np = a.Np, rows = (size_t)D * per_wg;
    double *s_g = s_dyn64, *s_shift = s_g + D, *sx = s_shift + D, *sv = sx + rows, *sp = sv + rows, *spf = sp + rows;
    for (int d = threadIdx.x; d < D; d += BLOCK64) {
        s_g[d] = a.gpos[d];
        s_shift[d] = a.shift[d];
    }
    for (size_t e = threadIdx.x; e < rows; e += BLOCK64) {
        const size_t d = e / per_wg, j = e % per_wg;
        if (j < n_loc) {
            const size_t g = d * Np + i_lo + j;
            sx[e] = a.x[g];
            sv[e] = a.v[g];
            sp[e] = a.p[g];
        }
    }
    for (uint32_t j = threadIdx.x; j < n_loc; j += BLOCK64) spf[j] = a.pf[i_lo + j];
    unsigned long long gk = c->gord;
    uint32_t gi = c->gidx;
    long long giter = c->giter, t = c->t;
    bool stop = c->stop != 0;
    const double tol = c->tol, fstar = c->fstar;
    double vlo = -a.vmax, vhi = a.vmax, xlo = a.lo, xhi = a.hi;
    asm volatile("" : "+v"(vlo), "+v"(vhi), "+v"(xlo), "+v"(xhi));
    if (threadIdx.x == 0) s_fail = 0;
    __syncthreads();
    for (long long it = 0; it < T && !stop; ++it) {
        const uint32_t t1 = (uint32_t)(t + 1);
        const int par = (int)(it & 1);
        unsigned long long k = ~0ull;
        uint32_t ki = NO_IDX;
        for (uint32_t j = threadIdx.x; j < n_loc; j += BLOCK64)
            staged_particle64<FIT>(a, D, per_wg, j, i_lo + j, t1, sx, sv, sp, spf, s_g, s_shift, vlo, vhi, xlo, xhi,
                                   gk, gi, k, ki);
        wg_lexmin_sparse<BLOCK64>(k, ki, s_k, s_i); // its barrier follows every lane's LDS stores
        // post: the key (order bits in two words, index in one) and the
        // candidate position (two words per double), each word tagged with t1
        const unsigned long long tag = (unsigned long long)t1 << 32;
        unsigned long long *kw = a.slot_ord + (size_t)par * G * 3, *pw =
            reinterpret_cast<unsigned long long *>(a.cand_pos) + (size_t)par * G * 2 * D;
        if (threadIdx.x < 3) {
            const uint32_t pay = threadIdx.x == 0 ? (uint32_t)k : threadIdx.x == 1 ? (uint32_t)(k >> 32) : ki;
            __hip_atomic_store(&kw[(size_t)b * 3 + threadIdx.x], tag | pay, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        } else if (threadIdx.x < 3 + 2 * (uint32_t)D) {
            const uint32_t w = threadIdx.x - 3;
            const double v = ki != NO_IDX ? sx[(size_t)(w >> 1) * per_wg + (ki - i_lo)] : 0.0;
            const unsigned long long bits = (unsigned long long)__double_as_longlong(v);
            const uint32_t pay = (w & 1) ? (uint32_t)(bits >> 32) : (uint32_t)bits;
            __hip_atomic_store(&pw[(size_t)b * 2 * D + w], tag | pay, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        // every workgroup reads every key, each word once it carries t1
        const unsigned long long w0 = wall_clock64();
        for (uint32_t q = threadIdx.x; q < 3 * G; q += BLOCK64) {
            unsigned long long v;
            while (((v = __hip_atomic_load(&kw[q], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) >> 32) != t1) {
                __builtin_amdgcn_s_sleep(1);
                if (wall_clock64() - w0 > GANG64_WAIT_TICKS) {
                    s_fail = 1;
                    break;
                }
            }
            s_word[q] = (uint32_t)v;
        }
        __syncthreads();
        if (s_fail) { // uniform
            if (threadIdx.x == 0) atomicOr(&c->err, 1u);
            break;
        }
        unsigned long long rk = ~0ull;
        uint32_t ri = NO_IDX;
        for (uint32_t w = threadIdx.x; w < G; w += BLOCK64) {
            const unsigned long long sk = ((unsigned long long)s_word[3 * w + 1] << 32) | s_word[3 * w];
            const uint32_t si = s_word[3 * w + 2];
            if (sk < rk || (sk == rk && si < ri)) {
                rk = sk;
                ri = si;
            }
        }
        wg_lexmin(rk, ri, s_k, s_i); // ends with a barrier: s_word is free again
        if (ri != NO_IDX) {
            // the winner's position, from its workgroup's tagged words
            const unsigned long long *src = pw + (size_t)(ri / per_wg) * 2 * D;
            for (uint32_t w = threadIdx.x; w < 2 * (uint32_t)D; w += BLOCK64) {
                unsigned long long v;
                while (((v = __hip_atomic_load(&src[w], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) >> 32) != t1) {
                    __builtin_amdgcn_s_sleep(1);
                    if (wall_clock64() - w0 > GANG64_WAIT_TICKS) {
                        s_fail = 1;
                        break;
                    }
                }
                s_word[w] = (uint32_t)v;
            }
            __syncthreads();
            if (s_fail) { // uniform
                if (threadIdx.x == 0) atomicOr(&c->err, 1u);
                break;
            }
            for (int d = threadIdx.x; d < D; d += BLOCK64)
                s_g[d] = __longlong_as_double((long long)(((unsigned long long)s_word[2 * d + 1] << 32) | s_word[2 * d]));
            gk = rk;
            gi = ri;
            giter = t1;
        }
        t = t1;
        // every workgroup holds the same key, so all take the same decision
        stop = tol > 0.0 && fabs(ord64_value(gk) - fstar) < tol;
        __syncthreads();
    }
    for (size_t e = threadIdx.x; e < rows; e += BLOCK64) {
        const size_t d = e / per_wg, j = e % per_wg;
        if (j < n_loc) {
            const size_t g = d * Np + i_lo + j;
            a.x[g] = sx[e];
            a.v[g] = sv[e];
            a.p[g] = sp[e];
        }
    }
    for (uint32_t j = threadIdx.x; j < n_loc; j += BLOCK64) a.pf[i_lo + j] = spf[j];
    if (b == 0) {
        for (int d = threadIdx.x; d < D; d += BLOCK64) a.gpos[d] = s_g[d];
        if (threadIdx.x == 0) {
            c->gord = gk;
            c->gidx = gi;
            c->giter = giter;
            c->t = t;
            c->stop = stop ? 1u : 0u;
        }
    }
}

// Zeroes n words (the staged gang's tagged slots before a launch).
__global__ void k_zero64(unsigned long long *w, size_t n)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) w[i] = 0;
}

// Clears the control block (a kernel, not a memset: the call may be
// captured into a graph).
__global__ void k_reset64(Swarm64Args a)
{
    if (threadIdx.x == 0) *a.ctrl = Ctrl64{};
}

hipError_t launch64_reset(const Swarm64Args &a, hipStream_t stream)
{
    hipLaunchKernelGGL(k_reset64, dim3(1), dim3(64), 0, stream, a);
    return hipGetLastError();
}

__global__ void k_arm64(Swarm64Args a, double tol, double fstar)
{
    if (threadIdx.x != 0) return;
    Ctrl64 *c = a.ctrl;
    c->tol = tol;
    c->fstar = fstar;
    c->stop = (tol > 0.0 && fabs(a.pf[c->gidx] - fstar) < tol) ? 1u : 0u;
}

static inline dim3 grid64(const Swarm64Args &a) { return dim3((a.N + BLOCK64 - 1) / BLOCK64); }

// Dynamic LDS of the staged one-workgroup run: gbest position and shift, x,
// v, p (D x N doubles each) and pf; 0 where it does not fit one workgroup
// (or PSO64_BLOCK_STAGED=0 in the environment: the unstaged run, for tests).
static int lds64_max()
{
    static const int v = [] {
        int dev = 0, b = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&b, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
            return 0;
        return b;
    }();
    return v;
}

static size_t block64_staged_lds(const Swarm64Args &a)
{
    if (!lds64_max()) return 0;
    const char *env = getenv("PSO64_BLOCK_STAGED");
    if (env && !strcmp(env, "0")) return 0;
    const size_t bytes = sizeof(double) * (2 * (size_t)a.D + (3 * (size_t)a.D + 1) * a.N);
    return bytes + 1024 <= (size_t)lds64_max() ? bytes : 0;
}

// The grid step takes two particles per lane (k_step64w) from N = 2^14 on;
// PSO64_WIDE=0 or 1 in the environment forces either form (tests of both).
#ifndef PSO64_WIDE_MIN_N
#define PSO64_WIDE_MIN_N 16384
#endif
static bool step64_wide(const Swarm64Args &a)
{
    const char *env = getenv("PSO64_WIDE");
    if (env) return atoi(env) != 0;
    return a.N >= PSO64_WIDE_MIN_N;
}

// The split step (k_step64s) for N <= SPLIT64_MAX_N and D >= SPLIT64_MIN_D:
// P = 64 particles per workgroup from N = 32768, else 32, halved (down to
// 4) while fewer than 64 workgroups would run, and halved while the staged
// terms exceed 63 KiB of LDS; C dimensions per lane.  Measured (Cubic, us
// per iteration, split / one or two particles per lane): D = 120: N = 128
// 9.4 / 38.1, 1024 12.9 / 50.5, 8192 20.6 / 61.6, 16384 29.7 / 60.9, 32768
// 39.9 / 63.4, 65536 80.2 (P = 64) / 71.2; N = 2048, D = 32: 9.8 / 15.0;
// N = 4096, D = 64: 13.3 / 31.2; at D = 16 the split loses (N = 8192: 12.4 /
// 11.1; 30000: 28.2 / 15.0): a workgroup's fixed cost over too few updates.
// PSO64_SPLIT=0 or 1 in the environment turns it off or on wherever the
// terms of four particles fit (tests of both forms); PSO64_SPLIT_P sets P.
#ifndef SPLIT64_MIN_D
#define SPLIT64_MIN_D 32
#endif
#ifndef SPLIT64_MAX_N
#define SPLIT64_MAX_N 32768
#endif
static bool split64_shape(const Swarm64Args &a, int words, uint32_t *P, uint32_t *C)
{
    const char *env = getenv("PSO64_SPLIT");
    const bool forced = env && atoi(env) != 0;
    if (env && !forced) return false;
    if (!forced && (a.N > SPLIT64_MAX_N || a.D < SPLIT64_MIN_D)) return false;
    const size_t lds_cap = 63 * 1024;
    auto fits = [&](uint32_t p) { return sizeof(double) * (2 * (size_t)a.D + (size_t)words * a.D * p) <= lds_cap; };
    uint32_t p = a.N >= 32768 ? 64 : 32;
    while (p > SPLIT64_MIN_P && a.N / p < 64) p >>= 1;
    if (const char *e = getenv("PSO64_SPLIT_P")) p = (uint32_t)atoi(e);
    if (p < SPLIT64_MIN_P || p > (uint32_t)BLOCK64 || (p & (p - 1))) return false;
    while (p > SPLIT64_MIN_P && !fits(p)) p >>= 1;
    if (!fits(p)) return false;
    const uint32_t L = BLOCK64 / p;
    uint32_t c = ((uint32_t)a.D + L - 1) / L;
    c += c & 1u;
    *P = p;
    *C = c;
    return true;
}

#define PSO64_DISPATCH(FN, ...)                                                                                    \
    switch (fitness) {                                                                                             \
    case F_SPHERE: FN<F_SPHERE>(__VA_ARGS__); break;                                                               \
    case F_RASTRIGIN: FN<F_RASTRIGIN>(__VA_ARGS__); break;                                                         \
    case F_ROSENBROCK: FN<F_ROSENBROCK>(__VA_ARGS__); break;                                                       \
    case F_ACKLEY: FN<F_ACKLEY>(__VA_ARGS__); break;                                                               \
    case F_CUBIC: FN<F_CUBIC>(__VA_ARGS__); break;                                                                 \
    default: return hipErrorInvalidValue;                                                                          \
    }

// The binary64 fitness of the swarm's function (with its shift) at M points
// (row-major M x D), one lane per point, in dimension order.
template <int FIT>
__global__ void k_eval64(Swarm64Args a, const double *pts, uint64_t M, double *out)
{
    const uint64_t m = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= M) return;
    Fitness64<FIT> fit;
    for (int d = 0; d < a.D; ++d) fit.add(pts[m * (uint64_t)a.D + d] - a.shift[d], d);
    out[m] = fit.value(a.D);
}

template <int FIT>
static void eval64_f(const Swarm64Args &a, const double *pts, uint64_t M, double *out, hipStream_t s)
{
    hipLaunchKernelGGL(k_eval64<FIT>, dim3((unsigned)((M + 255) / 256)), dim3(256), 0, s, a, pts, M, out);
}

hipError_t launch64_eval(int fitness, const Swarm64Args &a, const double *pts, uint64_t M, double *out,
                         hipStream_t stream)
{
    PSO64_DISPATCH(eval64_f, a, pts, M, out, stream);
    return hipGetLastError();
}

template <int FIT>
static void init64_f(const Swarm64Args &a, hipStream_t s)
{
    hipLaunchKernelGGL(k_init64<FIT>, grid64(a), dim3(BLOCK64), sizeof(double) * a.D, s, a);
}
template <int FIT>
static void step64_f(const Swarm64Args &a, hipStream_t s)
{
    const size_t lds = 2 * sizeof(double) * a.D;
    uint32_t P = 0, C = 0;
    if (split64_shape(a, split64_words<FIT>(), &P, &C)) {
        const size_t lds_s = sizeof(double) * (2 * (size_t)a.D + (size_t)split64_words<FIT>() * a.D * P);
        hipLaunchKernelGGL(k_step64s<FIT>, dim3((a.N + P - 1) / P), dim3(BLOCK64), lds_s, s, a, P, C);
        return;
    }
    if (!step64_wide(a)) {
        hipLaunchKernelGGL(k_step64<FIT>, grid64(a), dim3(BLOCK64), lds, s, a);
        return;
    }
    const dim3 grid((a.Np / 2 + BLOCK64 - 1) / BLOCK64);
    // rows of doubles: the binary32 policy at twice the row pitch in floats
    switch (cache_policy(2 * (uint64_t)a.Np, a.D)) {
    case POL_STREAM: hipLaunchKernelGGL((k_step64w<FIT, POL_STREAM>), grid, dim3(BLOCK64), lds, s, a); break;
    case POL_X: hipLaunchKernelGGL((k_step64w<FIT, POL_X>), grid, dim3(BLOCK64), lds, s, a); break;
    case POL_XV: hipLaunchKernelGGL((k_step64w<FIT, POL_XV>), grid, dim3(BLOCK64), lds, s, a); break;
    default: hipLaunchKernelGGL((k_step64w<FIT, POL_ALL>), grid, dim3(BLOCK64), lds, s, a); break;
    }
}
// One workgroup: 256 lanes for up to 512 particle-dimensions, else 1024.
template <int FIT>
static void block64_f(const Swarm64Args &a, long long T, hipStream_t s)
{
    const size_t lds = 2 * sizeof(double) * a.D;
    const bool small = (uint64_t)a.N * (uint64_t)a.D <= 512;
    const size_t staged = block64_staged_lds(a);
    if (staged > 0) {
        const bool one = a.D == 1;
        const void *f = small ? (one ? reinterpret_cast<const void *>(k_block_run64s<FIT, 256, true>)
                                     : reinterpret_cast<const void *>(k_block_run64s<FIT, 256, false>))
                              : (one ? reinterpret_cast<const void *>(k_block_run64s<FIT, 1024, true>)
                                     : reinterpret_cast<const void *>(k_block_run64s<FIT, 1024, false>));
        // the most any swarm may ask for, so concurrent callers never lower it
        if (hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, lds64_max() - 1024) == hipSuccess) {
            const dim3 lanes(small ? 256 : 1024);
            if (small && one)
                hipLaunchKernelGGL((k_block_run64s<FIT, 256, true>), dim3(1), lanes, staged, s, a, T);
            else if (small)
                hipLaunchKernelGGL((k_block_run64s<FIT, 256, false>), dim3(1), lanes, staged, s, a, T);
            else if (one)
                hipLaunchKernelGGL((k_block_run64s<FIT, 1024, true>), dim3(1), lanes, staged, s, a, T);
            else
                hipLaunchKernelGGL((k_block_run64s<FIT, 1024, false>), dim3(1), lanes, staged, s, a, T);
            return;
        }
    }
    if (small)
        hipLaunchKernelGGL((k_block_run64<FIT, 256>), dim3(1), dim3(256), lds, s, a, T);
    else
        hipLaunchKernelGGL((k_block_run64<FIT, 1024>), dim3(1), dim3(1024), lds, s, a, T);
}

// Particles per lane of the gang kernel: fewer, fuller workgroups make the
// per-iteration meeting cheaper (measured with the slices in LDS, Cubic 1D,
// us per iteration at 1/2/4/8/16 particles per lane: N = 4096: 4.2/3.9/4.3/
// 5.8/8.4; 8192: 5.2/4.6/4.6/5.8/8.6; 16384: 7.0/5.6/5.2/6.0/8.6; 65536:
// 17.5/10.2/7.8/7.8/9.5; 131072: 37.9/18.1/12.2/9.7/10.7; in device memory
// the same choices are within 2 % of the best).  PSO64_GANG_PPL overrides it.
static int gang_ppl(uint64_t N)
{
    if (const char *env = getenv("PSO64_GANG_PPL")) {
        const int v = atoi(env);
        if (v >= 1 && v <= 64) return v;
    }
    return N <= 8192 ? 2 : N <= 65536 ? 4 : 8;
}

// The gang with its slices in LDS (k_gang64s) where a slice fits and the
// workgroups are co-resident; else k_gang64 at gang_ppl's count
// (PSO64_GANG_STAGED=0 in the environment: always k_gang64, for tests).
template <int FIT>
static hipError_t gang64_f(const Swarm64Args &a, long long T, hipStream_t s, bool *launched, bool staged_only)
{
    const int ppl0 = gang_ppl(a.N);
    // staged: the fence-free meeting is cheap, so as many workgroups as the
    // tagged words allow (Cubic 1D, us per iteration at 1/2/4/8 particles
    // per lane: N = 4096: 3.0/3.1/3.5/4.6; 16384: 3.6/3.8/4.0/5.0; 65536:
    // 4.3/4.3/4.7/5.7; 131072: -/4.8/5.0/5.9)
    const char *penv = getenv("PSO64_GANG_PPL");
    const int ppl_s = penv ? ppl0
                           : (int)std::max<uint64_t>(1, ((uint64_t)a.N + (uint64_t)BLOCK64 * GANG64S_MAX_G - 1) /
                                                             ((uint64_t)BLOCK64 * GANG64S_MAX_G));
    int per_cu = 0, dev = 0, cus = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if ((e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess) return e;
    const char *env = getenv("PSO64_GANG_STAGED");
    const bool one = a.D == 1;
    for (int ppl = ppl_s; !(env && !strcmp(env, "0")) && lds64_max() > 0 && ppl >= std::max(1, ppl_s / 2); ppl /= 2) {
        const uint64_t per_wg = BLOCK64 * (uint64_t)ppl; // particles per workgroup
        const uint64_t G = ((uint64_t)a.N + per_wg - 1) / per_wg;
        const size_t lds_s = sizeof(double) * (2 * (size_t)a.D + (3 * (size_t)a.D + 1) * per_wg);
        const size_t lds_static = sizeof(uint32_t) * 3 * GANG64S_MAX_G + 1024; // the kernel's own arrays, with room
        if (lds_s + lds_static > (size_t)lds64_max()) continue;
        const void *f = one ? reinterpret_cast<const void *>(k_gang64s<FIT, true>)
                            : reinterpret_cast<const void *>(k_gang64s<FIT, false>);
        // the most any swarm may ask for, so concurrent callers never lower it
        if ((e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     lds64_max() - (int)lds_static)) != hipSuccess)
            return e;
        e = one ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_gang64s<FIT, true>, BLOCK64, lds_s)
                : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_gang64s<FIT, false>, BLOCK64, lds_s);
        if (e != hipSuccess) return e;
        if (G > (uint64_t)std::max(1, per_cu * cus * 3 / 4) || G > GANG64S_MAX_G) continue; // co-resident with margin
        // the tagged words of both parities: keys in slot_ord, positions in cand_pos
        hipLaunchKernelGGL(k_zero64, dim3(4), dim3(256), 0, s, a.slot_ord, (size_t)6 * G);
        hipLaunchKernelGGL(k_zero64, dim3(4), dim3(256), 0, s, reinterpret_cast<unsigned long long *>(a.cand_pos),
                           (size_t)4 * G * a.D);
        if (one)
            hipLaunchKernelGGL((k_gang64s<FIT, true>), dim3((unsigned)G), dim3(BLOCK64), lds_s, s, a, T,
                               (uint32_t)per_wg);
        else
            hipLaunchKernelGGL((k_gang64s<FIT, false>), dim3((unsigned)G), dim3(BLOCK64), lds_s, s, a, T,
                               (uint32_t)per_wg);
        *launched = true;
        return hipGetLastError();
    }
    if (staged_only) {
        *launched = false;
        return hipSuccess;
    }
    const uint64_t per_wg = BLOCK64 * (uint64_t)ppl0;
    const uint64_t G = ((uint64_t)a.N + per_wg - 1) / per_wg;
    const size_t lds = 2 * sizeof(double) * a.D;
    if ((e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_gang64<FIT>, BLOCK64, lds)) != hipSuccess) return e;
    const uint64_t cap = (uint64_t)std::max(1, per_cu * cus * 3 / 4); // co-resident with margin
    if (G > cap) {
        *launched = false;
        return hipSuccess;
    }
    hipLaunchKernelGGL(k_gang64<FIT>, dim3((unsigned)G), dim3(BLOCK64), lds, s, a, T, (uint32_t)per_wg);
    *launched = true;
    return hipGetLastError();
}

hipError_t launch64_gang(int fitness, const Swarm64Args &a, long long T, hipStream_t stream, bool *launched,
                         bool staged_only)
{
    switch (fitness) {
    case F_SPHERE: return gang64_f<F_SPHERE>(a, T, stream, launched, staged_only);
    case F_RASTRIGIN: return gang64_f<F_RASTRIGIN>(a, T, stream, launched, staged_only);
    case F_ROSENBROCK: return gang64_f<F_ROSENBROCK>(a, T, stream, launched, staged_only);
    case F_ACKLEY: return gang64_f<F_ACKLEY>(a, T, stream, launched, staged_only);
    case F_CUBIC: return gang64_f<F_CUBIC>(a, T, stream, launched, staged_only);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch64_init(int fitness, const Swarm64Args &a, hipStream_t stream)
{
    PSO64_DISPATCH(init64_f, a, stream);
    return hipGetLastError();
}

hipError_t launch64_step(int fitness, const Swarm64Args &a, hipStream_t stream)
{
    PSO64_DISPATCH(step64_f, a, stream);
    return hipGetLastError();
}

bool block64_staged_fits(const Swarm64Args &a) { return block64_staged_lds(a) > 0; }

bool step64_split(int fitness, const Swarm64Args &a)
{
    uint32_t P = 0, C = 0;
    return split64_shape(a, fitness == F_ACKLEY ? 2 : 1, &P, &C);
}

hipError_t launch64_block_run(int fitness, const Swarm64Args &a, long long T, hipStream_t stream)
{
    PSO64_DISPATCH(block64_f, a, T, stream);
    return hipGetLastError();
}

hipError_t launch64_arm(const Swarm64Args &a, double tol, double fstar, hipStream_t stream)
{
    hipLaunchKernelGGL(k_arm64, dim3(1), dim3(64), 0, stream, a, tol, fstar);
    return hipGetLastError();
}

hipError_t launch64_flush(const Swarm64Args &a, hipStream_t stream)
{
    hipLaunchKernelGGL(k_flush64, grid64(a), dim3(BLOCK64), 0, stream, a);
    return hipGetLastError();
}

} // namespace pso

// ---------------------------------------------------------------------------
// C ABI of the binary64 path (include/pso.h).
// ---------------------------------------------------------------------------
struct pso_swarm64 {
    int fitness = 0;
    uint64_t N = 0;
    int D = 0;
    pso::Layout64 L{};
    pso::Swarm64Args a{};
    void *mem = nullptr;
    hipStream_t stream = nullptr;
};

namespace {

#define HIP64_TRY(expr)                                                                                            \
    do {                                                                                                           \
        hipError_t e_ = (expr);                                                                                    \
        if (e_ != hipSuccess) return pso_internal_fail(PSO_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_));      \
    } while (0)

// Paths of pso64_run (Cubic, us per iteration).  A swarm that the split grid
// step takes (D >= 32, N <= 32768) runs one grid launch per iteration: its
// lanes share each particle's dimensions, where one workgroup gives a lane a
// whole particle (grid / one workgroup: N = 32, D = 120: 8.8 / 31.1; 64,
// 100: 8.8 / 24.5; 128, 40: 8.4 / 10.9; 192, 32: 8.6 / 8.9).  Else a swarm
// whose state fits the LDS of one workgroup (x, v, p and pf: about 6 700
// particle-dimensions) runs there in one launch (256, 24: 7.1 against 12.7
// for the grid; 512, 8: 3.3 against 4.6 for the gang) unless the gang takes
// it (D <= GANG64_MAX_D and N >= GANG64_MIN_N; one workgroup / gang at D =
// 1: N = 3000: 2.55 / 2.82; 4096: 3.21 / 2.87; 5000: 3.86 / 3.03); else for
// D <= GANG64_MAX_D the persistent gang (N = 16384: 3.4; 131072: 4.7;
// D = 8, N = 16384: 5.7); else one grid launch per iteration (at D = 120
// the unstaged gang and the grid were within 2 % at N = 8192).  PSO64_PATH
// (block, gang, grid) overrides the choice (tests of every path); with
// PSO64_BLOCK_STAGED=0 the one-workgroup run keeps the state in device
// memory and takes up to BLOCK64_MAX_ND.
constexpr uint64_t BLOCK64_MAX_ND = 2048;
constexpr int GANG64_MAX_D = 8;
// with its slices in LDS the gang also beats the grid up to D = 31 (staged
// gang / grid: N = 4096, D = 12: 6.1 / 9.3; 16384, 16: 7.9 / 14.0; 16384,
// 24: 9.7 / 17.5); where the slices do not fit or co-reside (N = 65536, D =
// 16: 29.6 in device memory against 17.2) the grid runs
constexpr int GANG64_STAGED_MAX_D = 32;
constexpr uint32_t GANG64_MIN_N = 4096; // from here the gang beats one workgroup (D = 1, N = 4096: 2.9 / 3.2 us)

void free64(pso_swarm64 *s)
{
    if (!s) return;
    if (s->stream) (void)hipStreamSynchronize(s->stream);
    (void)hipFree(s->mem);
    if (s->stream) (void)hipStreamDestroy(s->stream);
    delete s;
}

int reinit64(pso_swarm64 *s)
{
    HIP64_TRY(pso::launch64_reset(s->a, s->stream));
    HIP64_TRY(pso::launch64_init(s->fitness, s->a, s->stream));
    return PSO_OK;
}

// Pitched (Np) device rows -> dense (N) host rows.
int rows_to_host(const pso_swarm64 *s, const double *src, double *dst)
{
    if (!dst) return PSO_OK;
    HIP64_TRY(hipMemcpy2D(dst, sizeof(double) * s->N, src, sizeof(double) * s->L.Np, sizeof(double) * s->N, s->D,
                          hipMemcpyDeviceToHost));
    return PSO_OK;
}

} // namespace

extern "C" {

int pso64_create(int fitness_id, int64_t N, int32_t D, const float bounds[2], float w, float c1, float c2,
                 float vmax, uint64_t seed, pso_swarm64 **out)
{
    return pso::guarded([&]() -> int {
        if (!out) return pso_internal_fail(PSO_EINVAL, "out is NULL");
        *out = nullptr;
        if (!bounds) return pso_internal_fail(PSO_EINVAL, "bounds is NULL");
        pso_desc d{};
        d.fitness_id = fitness_id;
        d.D = D;
        d.N = N;
        d.bounds[0] = bounds[0];
        d.bounds[1] = bounds[1];
        d.w = w;
        d.c1 = c1;
        d.c2 = c2;
        d.vmax = vmax;
        d.seed = seed;
        int rc = pso_internal_check_desc(&d);
        if (rc) return rc;
        pso_swarm64 *s = new (std::nothrow) pso_swarm64();
        if (!s) return pso_internal_fail(PSO_ENOMEM, "host allocation failed");
        s->fitness = fitness_id;
        s->N = (uint64_t)N;
        s->D = D;
        s->L = pso::layout64_of(s->N, D);
        if (hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking) != hipSuccess) {
            s->stream = nullptr;
            free64(s);
            return pso_internal_fail(PSO_EDEVICE, "hipStreamCreate failed");
        }
        if (hipMalloc(&s->mem, s->L.total) != hipSuccess) {
            s->mem = nullptr;
            free64(s);
            return pso_internal_fail(PSO_ENOMEM, "hipMalloc of %zu bytes failed", s->L.total);
        }
        s->a = pso::bind64(s->mem, s->L, s->N, D);
        s->a.lo = bounds[0];
        s->a.hi = bounds[1];
        s->a.w = w;
        s->a.c1 = c1;
        s->a.c2 = c2;
        s->a.vmax = vmax;
        s->a.k0 = (uint32_t)seed;
        s->a.k1 = (uint32_t)(seed >> 32);
        if (hipMemset(const_cast<double *>(s->a.shift), 0, sizeof(double) * D) != hipSuccess ||
            (rc = reinit64(s)) != PSO_OK) {
            free64(s);
            return rc ? rc : pso_internal_fail(PSO_EDEVICE, "shift initialisation failed");
        }
        *out = s;
        return PSO_OK;
    });
}

int pso64_set_shift(pso_swarm64 *s, const float *shift)
{
    return pso::guarded([&]() -> int {
        if (!s || !shift) return pso_internal_fail(PSO_EINVAL, "swarm or shift is NULL");
        std::vector<double> sh(s->D);
        for (int d = 0; d < s->D; ++d) {
            if (!std::isfinite(shift[d])) return pso_internal_fail(PSO_EINVAL, "shift[%d] is not finite", d);
            sh[d] = shift[d];
        }
        HIP64_TRY(hipStreamSynchronize(s->stream));
        HIP64_TRY(hipMemcpy(const_cast<double *>(s->a.shift), sh.data(), sizeof(double) * s->D, hipMemcpyHostToDevice));
        return reinit64(s);
    });
}

int pso64_reset(pso_swarm64 *s)
{
    return pso::guarded([&]() -> int {
        if (!s) return pso_internal_fail(PSO_EINVAL, "swarm is NULL");
        return reinit64(s);
    });
}

int pso64_step(pso_swarm64 *s)
{
    return pso::guarded([&]() -> int {
        if (!s) return pso_internal_fail(PSO_EINVAL, "swarm is NULL");
        HIP64_TRY(pso::launch64_step(s->fitness, s->a, s->stream));
        return PSO_OK;
    });
}

int pso64_run(pso_swarm64 *s, int64_t max_iter, double tol, double f_star, double *gbest_value, double *gbest_pos,
              int64_t *gbest_iter, int64_t *iters_done)
{
    return pso::guarded([&]() -> int {
        if (!s) return pso_internal_fail(PSO_EINVAL, "swarm is NULL");
        if (max_iter < 0) return pso_internal_fail(PSO_EINVAL, "max_iter < 0");
        pso::Ctrl64 c{};
        HIP64_TRY(hipStreamSynchronize(s->stream));
        HIP64_TRY(hipMemcpy(&c, s->a.ctrl, sizeof c, hipMemcpyDeviceToHost));
        const long long t0 = c.t;
        HIP64_TRY(pso::launch64_arm(s->a, tol, f_star, s->stream));
        const uint64_t nd = s->N * (uint64_t)s->D;
        const char *path = getenv("PSO64_PATH"); // tests of every path: block, gang, grid
        bool done_gang = false;
        const bool block = path ? !strcmp(path, "block")
                                : !pso::step64_split(s->fitness, s->a) &&
                                      !(s->D <= GANG64_MAX_D && s->N >= GANG64_MIN_N) &&
                                      (pso::block64_staged_fits(s->a) || nd <= BLOCK64_MAX_ND);
        // 8 < D < 32: the gang only with its slices in LDS, else the grid
        const bool gang_staged_only = !path && s->D > GANG64_MAX_D;
        const bool gang = !block && (path ? !strcmp(path, "gang") : s->D < GANG64_STAGED_MAX_D);
        // those paths write each pbest position at once: complete the
        // pending ones a wide grid step left
        if (block || gang) HIP64_TRY(pso::launch64_flush(s->a, s->stream));
        if (block) {
            HIP64_TRY(pso::launch64_block_run(s->fitness, s->a, max_iter, s->stream));
            done_gang = true;
        } else if (gang) {
            HIP64_TRY(hipMemsetAsync(&s->a.ctrl->gang_arrive, 0, sizeof(unsigned long long), s->stream));
            HIP64_TRY(pso::launch64_gang(s->fitness, s->a, max_iter, s->stream, &done_gang, gang_staged_only));
        }
        if (!done_gang) {
            // chunks of launches; every launch returns at once after the stop rule holds
            for (int64_t done = 0; done < max_iter;) {
                const int64_t n = std::min<int64_t>(256, max_iter - done);
                for (int64_t k = 0; k < n; ++k) HIP64_TRY(pso::launch64_step(s->fitness, s->a, s->stream));
                done += n;
                HIP64_TRY(hipStreamSynchronize(s->stream));
                HIP64_TRY(hipMemcpy(&c, s->a.ctrl, sizeof c, hipMemcpyDeviceToHost));
                if (c.stop) break;
            }
        }
        HIP64_TRY(hipStreamSynchronize(s->stream));
        HIP64_TRY(hipMemcpy(&c, s->a.ctrl, sizeof c, hipMemcpyDeviceToHost));
        if (c.err) return pso_internal_fail(PSO_EDEVICE, "a gang wait gave up (device error bits 0x%x)", c.err);
        if (gbest_value) HIP64_TRY(hipMemcpy(gbest_value, s->a.pf + c.gidx, sizeof(double), hipMemcpyDeviceToHost));
        if (gbest_pos) HIP64_TRY(hipMemcpy(gbest_pos, s->a.gpos, sizeof(double) * s->D, hipMemcpyDeviceToHost));
        if (gbest_iter) *gbest_iter = c.giter;
        if (iters_done) *iters_done = c.t - t0;
        return PSO_OK;
    });
}

int pso64_get_state(pso_swarm64 *s, double *x, double *v, double *p, double *pf, int64_t *gbest_index, int64_t *t)
{
    return pso::guarded([&]() -> int {
        if (!s) return pso_internal_fail(PSO_EINVAL, "swarm is NULL");
        HIP64_TRY(pso::launch64_flush(s->a, s->stream));
        HIP64_TRY(hipStreamSynchronize(s->stream));
        int rc;
        if ((rc = rows_to_host(s, s->a.x, x)) || (rc = rows_to_host(s, s->a.v, v)) || (rc = rows_to_host(s, s->a.p, p)))
            return rc;
        if (pf) HIP64_TRY(hipMemcpy(pf, s->a.pf, sizeof(double) * s->N, hipMemcpyDeviceToHost));
        pso::Ctrl64 c{};
        HIP64_TRY(hipMemcpy(&c, s->a.ctrl, sizeof c, hipMemcpyDeviceToHost));
        if (gbest_index) *gbest_index = c.gidx;
        if (t) *t = c.t;
        return PSO_OK;
    });
}

int pso64_eval(pso_swarm64 *s, const double *points, int64_t M, double *values)
{
    return pso::guarded([&]() -> int {
        if (!s) return pso_internal_fail(PSO_EINVAL, "swarm is NULL");
        if (M < 0 || M > (int64_t(1) << 30)) return pso_internal_fail(PSO_EINVAL, "M=%lld out of range", (long long)M);
        if (M == 0) return PSO_OK;
        if (!points || !values) return pso_internal_fail(PSO_EINVAL, "points or values is NULL");
        const size_t in_bytes = sizeof(double) * (size_t)M * (size_t)s->D, out_bytes = sizeof(double) * (size_t)M;
        void *buf = nullptr;
        if (hipMalloc(&buf, in_bytes + out_bytes) != hipSuccess)
            return pso_internal_fail(PSO_ENOMEM, "hipMalloc of %zu bytes failed", in_bytes + out_bytes);
        double *d_pts = static_cast<double *>(buf), *d_out = d_pts + (size_t)M * (size_t)s->D;
        hipError_t e = hipMemcpyAsync(d_pts, points, in_bytes, hipMemcpyHostToDevice, s->stream);
        if (e == hipSuccess) e = pso::launch64_eval(s->fitness, s->a, d_pts, (uint64_t)M, d_out, s->stream);
        if (e == hipSuccess) e = hipMemcpyAsync(values, d_out, out_bytes, hipMemcpyDeviceToHost, s->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
        (void)hipFree(buf);
        if (e != hipSuccess) return pso_internal_fail(PSO_EDEVICE, "pso64_eval: %s", hipGetErrorString(e));
        return PSO_OK;
    });
}

int pso64_destroy(pso_swarm64 *s)
{
    return pso::guarded([&]() -> int {
        if (!s) return pso_internal_fail(PSO_EINVAL, "swarm is NULL");
        free64(s);
        return PSO_OK;
    });
}

} // extern "C"

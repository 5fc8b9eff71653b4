// pso_device.hpp -- device building blocks of the PSO step for gfx950.
//
// Random numbers (Sec. 4.4 uses a library generator; here a counter-based
// one with no stored state), the binary32 fitness functions, the
// order-preserving (fitness, index) keys of the gbest aggregation (Sec. 3.1,
// Sec. 4.3 keeps indices rather than positions) and the wavefront minimum.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pso {

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds, each two
// 32x32->64 products feeding a bijection of the four counter words, the key
// advanced by the Weyl constants between rounds.  Counter words that are the
// same on every lane (dimension pair, iteration, tag) stay scalar, so the
// first rounds run on the scalar unit.
struct U4 {
    uint32_t a, b, c, d;
};

__device__ __forceinline__ U4 philox4x32_10(uint32_t k0, uint32_t k1, uint32_t c0, uint32_t c1, uint32_t c2,
                                            uint32_t c3)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        // one 32x32->64 product each (v_mad_u64_u32 on vector operands)
        const uint64_t m0 = (uint64_t)0xD2511F53u * c0;
        const uint64_t m1 = (uint64_t)0xCD9E8D57u * c2;
        c0 = (uint32_t)(m1 >> 32) ^ c1 ^ k0;
        c1 = (uint32_t)m1;
        c2 = (uint32_t)(m0 >> 32) ^ c3 ^ k1;
        c3 = (uint32_t)m0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return U4{c0, c1, c2, c3};
}

constexpr uint32_t TAG_VEL = 0u;  // velocity draws r1, r2 of an iteration
constexpr uint32_t TAG_INIT = 1u; // initial position and velocity

// 24 random bits as a float in [0, 1); exact in binary32.
__device__ __forceinline__ float unit_float(uint32_t u) { return (float)(u >> 8) * 0x1p-24f; }

// ---------------------------------------------------------------------------
// Binary32 cos(pi y) and exp(x) as explicit operation sequences, so that the
// result does not depend on a math library: float-rounded Taylor
// coefficients evaluated by Horner's rule with fused multiply-adds.
// ---------------------------------------------------------------------------
// (-1)^k pi^(2k) / (2k)!, k = 0..5 and (-1)^k pi^(2k+1) / (2k+1)!, k = 0..4.
__device__ __forceinline__ float cos_pi_series(float a)
{
    const float s = a * a;
    float q = -0x1.a6d1f2p-6f;
    q = __builtin_fmaf(q, s, 0x1.e1f506p-3f);
    q = __builtin_fmaf(q, s, -0x1.55d3c8p+0f);
    q = __builtin_fmaf(q, s, 0x1.03c1f0p+2f);
    q = __builtin_fmaf(q, s, -0x1.3bd3ccp+2f);
    return __builtin_fmaf(q, s, 0x1p+0f);
}

__device__ __forceinline__ float sin_pi_series(float b)
{
    const float s = b * b;
    float q = 0x1.507834p-4f;
    q = __builtin_fmaf(q, s, -0x1.32d2ccp-1f);
    q = __builtin_fmaf(q, s, 0x1.466bc6p+1f);
    q = __builtin_fmaf(q, s, -0x1.4abbcep+2f);
    q = __builtin_fmaf(q, s, 0x1.921fb6p+1f);
    return b * q;
}

// cos(pi y): y = n + r, n = rint(y), r exact in [-1/2, 1/2]; |r| <= 1/4 uses the
// cos series, otherwise sin(pi (1/2 - |r|)) (1/2 - |r| is exact); odd n negates.
// |y| >= 2^24 (every such binary32 is an even integer) gives 1, NaN and
// infinities the canonical NaN.  Every case is computed and selected, so the
// function has no branch.
__device__ __forceinline__ float cospi_f32(float y)
{
    const float n = __builtin_rintf(y);
    const float a = __builtin_fabsf(y - n);
    const float cc = cos_pi_series(a);
    const float ss = sin_pi_series(0.5f - a);
    const float c = (a <= 0.25f) ? cc : ss;
    const float h = 0.5f * n; // exact; an integer iff n is even (|n| < 2^24)
    const float r = (h != __builtin_rintf(h)) ? -c : c;
    const float big = (y != y || __builtin_isinf(y)) ? __builtin_nanf("") : 1.0f;
    return (__builtin_fabsf(y) < 0x1p24f) ? r : big;
}

// exp(x): k = rint(x log2 e), r = x - k ln2 in two fused steps (ln 2 split in
// a binary32 head and tail), sum_{j<=8} r^j / j! by Horner, times 2^k.
__device__ __forceinline__ float exp_f32(float x)
{
    if (x != x) return x;
    if (x > 100.0f) return __builtin_inff();
    if (x < -110.0f) return 0.0f;
    const float k = __builtin_rintf(x * 0x1.715476p+0f);
    float r = __builtin_fmaf(-k, 0x1.62e430p-1f, x);
    r = __builtin_fmaf(-k, -0x1.05c610p-29f, r);
    float q = 0x1.a01a02p-16f;          // 1/8!
    q = __builtin_fmaf(q, r, 0x1.a01a02p-13f); // 1/7!
    q = __builtin_fmaf(q, r, 0x1.6c16c2p-10f); // 1/6!
    q = __builtin_fmaf(q, r, 0x1.111112p-7f);  // 1/5!
    q = __builtin_fmaf(q, r, 0x1.555556p-5f);  // 1/4!
    q = __builtin_fmaf(q, r, 0x1.555556p-3f);  // 1/3!
    q = __builtin_fmaf(q, r, 0x1p-1f);         // 1/2!
    q = __builtin_fmaf(q, r, 0x1p+0f);         // 1/1!
    q = __builtin_fmaf(q, r, 0x1p+0f);         // 1/0!
    return __builtin_ldexpf(q, (int)k);
}

// ---------------------------------------------------------------------------
// Fitness accumulated one dimension at a time, in dimension order, so the
// kernel folds it into the update loop without storing the position first.
// ---------------------------------------------------------------------------
enum : int { F_SPHERE = 0, F_RASTRIGIN = 1, F_ROSENBROCK = 2, F_ACKLEY = 3, F_CUBIC = 4 };

template <int FIT>
struct Fitness {
    float acc = 0.0f; // running sum (Ackley: sum of z^2)
    float aux = 0.0f; // Ackley: sum of cos(2 pi z); Rosenbrock: previous z

    // z = x_d - shift_d of dimension d.
    __device__ __forceinline__ void add(float z, int d)
    {
        if constexpr (FIT == F_SPHERE) {
            acc = acc + z * z;
        } else if constexpr (FIT == F_RASTRIGIN) {
            acc = acc + (z * z - 10.0f * cospi_f32(2.0f * z));
        } else if constexpr (FIT == F_ROSENBROCK) {
            if (d > 0) {
                const float a = z - aux * aux;
                const float b = 1.0f - aux;
                acc = acc + (100.0f * (a * a) + b * b);
            }
            aux = z;
        } else if constexpr (FIT == F_ACKLEY) {
            acc = acc + z * z;
            aux = aux + cospi_f32(2.0f * z);
        } else { // F_CUBIC, Eq. 3 negated at the end
            const float z2 = z * z;
            acc = acc + (((z2 * z - 0.8f * z2) - 1000.0f * z) + 8000.0f);
        }
    }

    // The same sum split in two: stage(z) computes a dimension's terms
    // independently of the others (STAGE_WORDS floats), fold() adds staged
    // terms in dimension order.  stage then fold gives exactly add(z, d).
    static constexpr int STAGE_WORDS = FIT == F_ACKLEY ? 2 : 1;

    __device__ __forceinline__ static void stage(float z, float *s0, float *s1)
    {
        if constexpr (FIT == F_RASTRIGIN) {
            *s0 = z * z - 10.0f * cospi_f32(2.0f * z);
        } else if constexpr (FIT == F_ACKLEY) {
            *s0 = z * z;
            *s1 = cospi_f32(2.0f * z);
        } else if constexpr (FIT == F_CUBIC) {
            const float z2 = z * z;
            *s0 = ((z2 * z - 0.8f * z2) - 1000.0f * z) + 8000.0f;
        } else { // Sphere, Rosenbrock: z itself
            *s0 = z;
        }
    }

    __device__ __forceinline__ void fold(float s0, float s1, int d)
    {
        if constexpr (FIT == F_RASTRIGIN || FIT == F_CUBIC) {
            acc = acc + s0;
        } else if constexpr (FIT == F_ACKLEY) {
            acc = acc + s0;
            aux = aux + s1;
        } else {
            add(s0, d);
        }
    }

    __device__ __forceinline__ float value(int D) const
    {
        if constexpr (FIT == F_RASTRIGIN) {
            return (float)(10 * D) + acc;
        } else if constexpr (FIT == F_ACKLEY) {
            const float m1 = acc / (float)D;
            const float m2 = aux / (float)D;
            const float e1 = exp_f32(-0.2f * __builtin_sqrtf(m1));
            const float e2 = exp_f32(m2);
            return (20.0f - 20.0f * e1) + (exp_f32(1.0f) - e2);
        } else if constexpr (FIT == F_CUBIC) {
            return -acc;
        } else {
            return acc;
        }
    }
};

// ---------------------------------------------------------------------------
// (fitness, index) keys: the high word maps binary32 order onto unsigned
// order (+0 and -0 alike, NaN last), the low word is the particle index, so
// the unsigned minimum of keys is the best fitness with the lowest index.
// ---------------------------------------------------------------------------
constexpr unsigned long long NO_KEY = ~0ull;

__device__ __forceinline__ uint32_t order_bits(float f)
{
    if (f != f) return 0xFFFFFFFFu;
    const uint32_t b = (f == 0.0f) ? 0u : __float_as_uint(f);
    return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}

__device__ __forceinline__ unsigned long long make_key(float f, uint32_t i)
{
    return ((unsigned long long)order_bits(f) << 32) | i;
}

__host__ __device__ __forceinline__ float key_fitness(unsigned long long key)
{
    const uint32_t o = (uint32_t)(key >> 32);
    const uint32_t b = (o & 0x80000000u) ? (o & 0x7FFFFFFFu) : ~o;
    float f;
    __builtin_memcpy(&f, &b, sizeof f);
    return f;
}

// Minimum of a 64-bit value over the 64 lanes of a wavefront (butterfly over
// lane-index bits; every lane ends with the minimum).
__device__ __forceinline__ unsigned long long wave_min_u64(unsigned long long v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        const unsigned long long o = __shfl_xor(v, off, 64);
        v = o < v ? o : v;
    }
    return v;
}

} // namespace pso

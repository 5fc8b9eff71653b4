/*
 * pso_oracle.c -- plain CPU oracle for the global-best PSO step of cuPSO
 * (Wang, Ho, Tu, Hung, "cuPSO: GPU Parallelization for Particle Swarm
 * Optimization Algorithms", ACM SAC 2022).
 *
 * TEST INFRASTRUCTURE.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  The GPU library never
 * links, includes or calls it, and it shares no code with the GPU library.
 *
 * What it computes (one function per step of the method, each citing the
 * passage it follows):
 *   - Step 1, initialisation (Sec. 2.1, Alg. 1 Step 1): uniform random
 *     position and velocity inside fixed ranges, fitness, pbest <- pos, gbest.
 *   - Steps 2-5 of one iteration (Sec. 2.1, Eq. 1 and Eq. 2, Alg. 1 Steps 2-5)
 *     with the global best synchronised once per iteration, as in the
 *     two-kernel parallel PSO of Sec. 2.2 (Fig. 1): every particle of
 *     iteration t reads the gbest of iteration t-1.
 *   - The same iteration with the gbest updated inside the particle loop, the
 *     literal serial order of Alg. 1 ("serial_immediate").
 * The paper maximises; this oracle minimises (the paper's Cubic function of
 * Eq. 3 is offered negated, so its maximum is this oracle's minimum).
 *
 * Precision modes.  The paper computes in double precision (Sec. 5.1).  The
 * "_f32" functions compute in IEEE binary32 with a fixed operation order and
 * no contraction (build with -ffp-contract=off), so that a binary32 GPU
 * implementation of the same definition can be compared bit for bit; the
 * "_f64" functions compute in binary64 from the same binary32 inputs and the
 * same random draws, and serve to state the binary32 error.
 *
 * Definitions fixed here where the paper is silent (each is a reading):
 *   - Random numbers: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11),
 *     key = (seed mod 2^32, seed >> 32), counter = (d >> 1, i, t, tag),
 *     tag 0 for the velocity draws of iteration t, tag 1 for initialisation.
 *     Dimension d uses output words 2*(d&1) and 2*(d&1)+1.
 *     A word u becomes the uniform (u >> 8) * 2^-24 in [0, 1).
 *   - r1 and r2 are drawn per particle, per dimension, per iteration.
 *   - Clamps keep values in the closed intervals [-vmax, vmax] and [lo, hi]
 *     by comparison (a value equal to a bound, or a signed zero, is kept).
 *   - pbest improves only on a strictly smaller fitness (NaN never does);
 *     gbest is the lowest particle index among the smallest pbest fitness.
 *   - Fitness of x is F(z) with z = x - shift; cos(pi*y) and exp(x) in the
 *     binary32 mode are the polynomial evaluations cospi_f32 / exp_f32 below.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORACLE_TAG_VEL 0u
#define ORACLE_TAG_INIT 1u

enum { FIT_SPHERE = 0, FIT_RASTRIGIN = 1, FIT_ROSENBROCK = 2, FIT_ACKLEY = 3, FIT_CUBIC = 4 };

typedef struct oracle_problem {
    int32_t fitness_id; /* 0 Sphere, 1 Rastrigin, 2 Rosenbrock, 3 Ackley, 4 Cubic (Eq. 3, negated) */
    int32_t D;          /* dimensions */
    int64_t N;          /* particle_cnt */
    float lo, hi;       /* min_pos, max_pos (Table 1), same for every dimension */
    float w, c1, c2;    /* inertia, cognitive and social coefficients (Table 1) */
    float vmax;         /* max_v; min_v = -vmax (Table 1) */
    uint64_t seed;      /* Philox key */
    const float *shift; /* D values, or NULL for no shift */
    int32_t nthreads;   /* threads for the particle loop; <= 0 means the runtime default */
    int32_t pad_;
} oracle_problem;

/* ------------------------------------------------------------------------- */
/* Philox4x32-10, as published by Salmon et al. (SC'11): ten rounds of two    */
/* 32x32->64 multiplications with a Weyl-sequence key schedule.              */
/* ------------------------------------------------------------------------- */
void oracle_philox4x32_10(const uint32_t key[2], const uint32_t ctr[4], uint32_t out[4])
{
    uint32_t k0 = key[0], k1 = key[1];
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t m0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t m1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t n0 = (uint32_t)(m1 >> 32) ^ c1 ^ k0;
        uint32_t n1 = (uint32_t)m1;
        uint32_t n2 = (uint32_t)(m0 >> 32) ^ c3 ^ k1;
        uint32_t n3 = (uint32_t)m0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* A 32-bit word -> uniform in [0, 1) with 24 random bits (exact in binary32). */
float oracle_uniform_f32(uint32_t u) { return (float)(u >> 8) * 0x1p-24f; }

/* The two uniforms that dimension d of particle i uses at iteration t under
 * the given tag (r1, r2 for velocity; position and velocity for init). */
void oracle_draw(uint64_t seed, uint32_t tag, uint64_t t, uint64_t i, int32_t d, float out[2])
{
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t ctr[4] = {(uint32_t)d >> 1, (uint32_t)i, (uint32_t)t, tag};
    uint32_t r[4];
    oracle_philox4x32_10(key, ctr, r);
    out[0] = oracle_uniform_f32(r[2 * (d & 1)]);
    out[1] = oracle_uniform_f32(r[2 * (d & 1) + 1]);
}

/* ------------------------------------------------------------------------- */
/* Binary32 elementary functions used by the fitness functions.              */
/* ------------------------------------------------------------------------- */
/* Taylor coefficients of cos(pi*a) and sin(pi*a) in a, (-1)^k pi^(2k)/(2k)!
 * and (-1)^k pi^(2k+1)/(2k+1)!, each rounded to the nearest binary32. */
static const float COS_C[6] = {0x1p+0f, -0x1.3bd3ccp+2f, 0x1.03c1f0p+2f,
                               -0x1.55d3c8p+0f, 0x1.e1f506p-3f, -0x1.a6d1f2p-6f};
static const float SIN_C[5] = {0x1.921fb6p+1f, -0x1.4abbcep+2f, 0x1.466bc6p+1f,
                               -0x1.32d2ccp-1f, 0x1.507834p-4f};
/* 1/k! rounded to binary32, k = 0..8. */
static const float EXP_C[9] = {0x1p+0f, 0x1p+0f, 0x1p-1f, 0x1.555556p-3f, 0x1.555556p-5f,
                               0x1.111112p-7f, 0x1.6c16c2p-10f, 0x1.a01a02p-13f, 0x1.a01a02p-16f};
/* ln 2 split into its binary32 rounding and the binary32 rounding of the rest;
 * log2(e) rounded to binary32. */
static const float LN2_HI = 0x1.62e430p-1f;
static const float LN2_LO = -0x1.05c610p-29f;
static const float LOG2E = 0x1.715476p+0f;

/* Copies the constants above, in order COS_C, SIN_C, EXP_C, LN2_HI, LN2_LO,
 * LOG2E (23 values), so that tests can check the built library. */
void oracle_constants_f32(float out[23])
{
    int k = 0;
    for (int j = 0; j < 6; ++j) out[k++] = COS_C[j];
    for (int j = 0; j < 5; ++j) out[k++] = SIN_C[j];
    for (int j = 0; j < 9; ++j) out[k++] = EXP_C[j];
    out[k++] = LN2_HI;
    out[k++] = LN2_LO;
    out[k++] = LOG2E;
}

/* cos(pi*y) in binary32: y = n + r with n = rint(y) and r = y - n exact,
 * |r| <= 1/2; a = |r|; for a <= 1/4 the cos series in a, otherwise the sin
 * series in 1/2 - a (exact); negated when n is odd.  Horner with fmaf. */
float oracle_cospi_f32(float y)
{
    if (!(fabsf(y) < 0x1p24f)) {
        if (isnan(y) || isinf(y)) return NAN;
        return 1.0f; /* every binary32 of magnitude >= 2^24 is an even integer */
    }
    float n = rintf(y);
    float r = y - n;
    float a = fabsf(r);
    float c;
    if (a <= 0.25f) {
        float s = a * a;
        float q = COS_C[5];
        q = fmaf(q, s, COS_C[4]);
        q = fmaf(q, s, COS_C[3]);
        q = fmaf(q, s, COS_C[2]);
        q = fmaf(q, s, COS_C[1]);
        c = fmaf(q, s, COS_C[0]);
    } else {
        float b = 0.5f - a;
        float s = b * b;
        float q = SIN_C[4];
        q = fmaf(q, s, SIN_C[3]);
        q = fmaf(q, s, SIN_C[2]);
        q = fmaf(q, s, SIN_C[1]);
        q = fmaf(q, s, SIN_C[0]);
        c = b * q;
    }
    long long ni = (long long)n;
    return (ni & 1) ? -c : c;
}

/* exp(x) in binary32 by Cody-Waite reduction: k = rint(x*log2(e)),
 * r = (x - k*LN2_HI) - k*LN2_LO with fmaf, degree-8 Taylor series of exp(r)
 * by Horner with fmaf, then scaling by 2^k (ldexpf rounds once). */
float oracle_exp_f32(float x)
{
    if (isnan(x)) return x;
    if (x > 100.0f) return INFINITY;
    if (x < -110.0f) return 0.0f;
    float k = rintf(x * LOG2E);
    float r = fmaf(-k, LN2_HI, x);
    r = fmaf(-k, LN2_LO, r);
    float q = EXP_C[8];
    for (int j = 7; j >= 0; --j) q = fmaf(q, r, EXP_C[j]);
    return ldexpf(q, (int)k);
}

/* ------------------------------------------------------------------------- */
/* Fitness functions (minimised).  x[d*stride] is dimension d.               */
/* ------------------------------------------------------------------------- */
static float shift_f32(const oracle_problem *pr, int d) { return pr->shift ? pr->shift[d] : 0.0f; }

float oracle_fitness_f32(const oracle_problem *pr, const float *x, int64_t stride)
{
    const int D = pr->D;
    switch (pr->fitness_id) {
    case FIT_SPHERE: { /* sum z^2 */
        float acc = 0.0f;
        for (int d = 0; d < D; ++d) {
            float z = x[d * stride] - shift_f32(pr, d);
            acc = acc + z * z;
        }
        return acc;
    }
    case FIT_RASTRIGIN: { /* 10 D + sum (z^2 - 10 cos(2 pi z)) */
        float acc = 0.0f;
        for (int d = 0; d < D; ++d) {
            float z = x[d * stride] - shift_f32(pr, d);
            acc = acc + (z * z - 10.0f * oracle_cospi_f32(2.0f * z));
        }
        return (float)(10 * D) + acc;
    }
    case FIT_ROSENBROCK: { /* sum_{d<D-1} 100 (z_{d+1} - z_d^2)^2 + (1 - z_d)^2 */
        float acc = 0.0f;
        for (int d = 0; d + 1 < D; ++d) {
            float zd = x[d * stride] - shift_f32(pr, d);
            float zn = x[(d + 1) * stride] - shift_f32(pr, d + 1);
            float a = zn - zd * zd;
            float b = 1.0f - zd;
            acc = acc + (100.0f * (a * a) + b * b);
        }
        return acc;
    }
    case FIT_ACKLEY: { /* 20 - 20 exp(-0.2 sqrt(mean z^2)) + e - exp(mean cos(2 pi z)) */
        float s1 = 0.0f, s2 = 0.0f;
        for (int d = 0; d < D; ++d) {
            float z = x[d * stride] - shift_f32(pr, d);
            s1 = s1 + z * z;
            s2 = s2 + oracle_cospi_f32(2.0f * z);
        }
        float m1 = s1 / (float)D;
        float m2 = s2 / (float)D;
        float e1 = oracle_exp_f32(-0.2f * sqrtf(m1));
        float e2 = oracle_exp_f32(m2);
        return (20.0f - 20.0f * e1) + (oracle_exp_f32(1.0f) - e2);
    }
    case FIT_CUBIC: { /* -(sum z^3 - 0.8 z^2 - 1000 z + 8000), Eq. 3 negated */
        float acc = 0.0f;
        for (int d = 0; d < D; ++d) {
            float z = x[d * stride] - shift_f32(pr, d);
            float z2 = z * z;
            acc = acc + (((z2 * z - 0.8f * z2) - 1000.0f * z) + 8000.0f);
        }
        return -acc;
    }
    default:
        return NAN;
    }
}

/* cos(pi*y) in binary64 from the C library after exact reduction y = n + r. */
static double cospi_f64(double y)
{
    double n = rint(y);
    double r = y - n;
    double c = cos(M_PI * r);
    return fmod(n, 2.0) != 0.0 ? -c : c;
}

static double shift_f64(const oracle_problem *pr, int d) { return pr->shift ? (double)pr->shift[d] : 0.0; }

double oracle_fitness_f64(const oracle_problem *pr, const double *x, int64_t stride)
{
    const int D = pr->D;
    switch (pr->fitness_id) {
    case FIT_SPHERE: {
        double acc = 0.0;
        for (int d = 0; d < D; ++d) {
            double z = x[d * stride] - shift_f64(pr, d);
            acc += z * z;
        }
        return acc;
    }
    case FIT_RASTRIGIN: {
        double acc = 0.0;
        for (int d = 0; d < D; ++d) {
            double z = x[d * stride] - shift_f64(pr, d);
            acc += z * z - 10.0 * cospi_f64(2.0 * z);
        }
        return 10.0 * D + acc;
    }
    case FIT_ROSENBROCK: {
        double acc = 0.0;
        for (int d = 0; d + 1 < D; ++d) {
            double zd = x[d * stride] - shift_f64(pr, d);
            double zn = x[(d + 1) * stride] - shift_f64(pr, d + 1);
            double a = zn - zd * zd;
            double b = 1.0 - zd;
            acc += 100.0 * a * a + b * b;
        }
        return acc;
    }
    case FIT_ACKLEY: {
        double s1 = 0.0, s2 = 0.0;
        for (int d = 0; d < D; ++d) {
            double z = x[d * stride] - shift_f64(pr, d);
            s1 += z * z;
            s2 += cospi_f64(2.0 * z);
        }
        return 20.0 - 20.0 * exp(-0.2 * sqrt(s1 / D)) + M_E - exp(s2 / D);
    }
    case FIT_CUBIC: {
        double acc = 0.0;
        for (int d = 0; d < D; ++d) {
            double z = x[d * stride] - shift_f64(pr, d);
            acc += z * z * z - 0.8 * z * z - 1000.0 * z + 8000.0;
        }
        return -acc;
    }
    default:
        return NAN;
    }
}

/* ------------------------------------------------------------------------- */
/* Ordering of (fitness, index): the gbest is the lexicographic minimum.     */
/* ------------------------------------------------------------------------- */
/* Order-preserving map of a binary32 onto uint32: -0 and +0 map alike,
 * NaN maps above +inf. */
uint32_t oracle_ord_f32(float f)
{
    if (isnan(f)) return 0xFFFFFFFFu;
    if (f == 0.0f) f = 0.0f;
    uint32_t b;
    memcpy(&b, &f, sizeof b);
    return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}

uint64_t oracle_key_f32(float f, uint32_t i) { return ((uint64_t)oracle_ord_f32(f) << 32) | i; }

static uint64_t ord_f64(double f)
{
    if (isnan(f)) return UINT64_MAX;
    if (f == 0.0) f = 0.0;
    uint64_t b;
    memcpy(&b, &f, sizeof b);
    return (b & 0x8000000000000000ull) ? ~b : (b | 0x8000000000000000ull);
}

static int nthreads_of(const oracle_problem *pr)
{
#ifdef _OPENMP
    return pr->nthreads > 0 ? pr->nthreads : omp_get_max_threads();
#else
    (void)pr;
    return 1;
#endif
}

static float clampf(float v, float lo, float hi)
{
    if (v < lo) v = lo;
    if (v > hi) v = hi;
    return v;
}

static double clampd(double v, double lo, double hi)
{
    if (v < lo) v = lo;
    if (v > hi) v = hi;
    return v;
}

/* ------------------------------------------------------------------------- */
/* Binary32 mode.  State is structure-of-arrays (Sec. 4.1, Data Structure 2):*/
/* element (d, i) of x, v, p at d*N + i; pf[i]; gpos[d].                      */
/* ------------------------------------------------------------------------- */
static uint64_t lexmin_f32(const oracle_problem *pr, const float *pf)
{
    uint64_t best = UINT64_MAX;
    for (int64_t i = 0; i < pr->N; ++i) {
        uint64_t k = oracle_key_f32(pf[i], (uint32_t)i);
        if (k < best) best = k;
    }
    return best;
}

static void gather_f32(const oracle_problem *pr, const float *p, uint64_t gkey, float *gpos)
{
    int64_t gi = (int64_t)(gkey & 0xFFFFFFFFu);
    for (int d = 0; d < pr->D; ++d) gpos[d] = p[d * pr->N + gi];
}

/* Step 1 of Alg. 1: random pos, v in their ranges; fit; pbest <- pos; gbest. */
void oracle_init_f32(const oracle_problem *pr, float *x, float *v, float *p, float *pf,
                     float *gpos, uint64_t *gkey)
{
    const int64_t N = pr->N;
    const int D = pr->D;
    const float span = pr->hi - pr->lo;
    const float vspan = pr->vmax + pr->vmax;
#pragma omp parallel for schedule(static) num_threads(nthreads_of(pr))
    for (int64_t i = 0; i < N; ++i) {
        for (int d = 0; d < D; ++d) {
            float u[2];
            oracle_draw(pr->seed, ORACLE_TAG_INIT, 0, (uint64_t)i, d, u);
            float xi = clampf(pr->lo + span * u[0], pr->lo, pr->hi);
            float vi = clampf(-pr->vmax + vspan * u[1], -pr->vmax, pr->vmax);
            x[d * N + i] = xi;
            v[d * N + i] = vi;
            p[d * N + i] = xi;
        }
        pf[i] = oracle_fitness_f32(pr, x + i, N);
    }
    *gkey = lexmin_f32(pr, pf);
    gather_f32(pr, p, *gkey, gpos);
}

/* Steps 2-4 of Alg. 1 for particle i at iteration t, with gbest position g. */
static void particle_update_f32(const oracle_problem *pr, uint64_t t, int64_t i, float *x, float *v,
                                float *p, float *pf, const float *g)
{
    const int64_t N = pr->N;
    const int D = pr->D;
    for (int d = 0; d < D; ++d) {
        float r[2];
        oracle_draw(pr->seed, ORACLE_TAG_VEL, t, (uint64_t)i, d, r);
        const int64_t e = d * N + i;
        float xi = x[e], vi = v[e], pi = p[e];
        /* Eq. 1, evaluated left to right, then the velocity clamp. */
        float vn = ((pr->w * vi) + ((pr->c1 * r[0]) * (pi - xi))) + ((pr->c2 * r[1]) * (g[d] - xi));
        vn = clampf(vn, -pr->vmax, pr->vmax);
        /* Eq. 2, then the position clamp. */
        float xn = clampf(xi + vn, pr->lo, pr->hi);
        x[e] = xn;
        v[e] = vn;
    }
    /* Step 3: fitness of the new position; Step 4: strict pbest improvement. */
    float f = oracle_fitness_f32(pr, x + i, N);
    if (f < pf[i]) {
        pf[i] = f;
        for (int d = 0; d < D; ++d) p[d * N + i] = x[d * N + i];
    }
}

/* One iteration t >= 1, gbest synchronised per iteration (Sec. 2.2): every
 * particle uses the gbest position of iteration t-1; Step 5 then takes the
 * lexicographic minimum over all pbest.  Returns 1 if the gbest changed. */
int oracle_step_f32(const oracle_problem *pr, uint64_t t, float *x, float *v, float *p, float *pf,
                    float *gpos, uint64_t *gkey)
{
#pragma omp parallel for schedule(static) num_threads(nthreads_of(pr))
    for (int64_t i = 0; i < pr->N; ++i) particle_update_f32(pr, t, i, x, v, p, pf, gpos);
    uint64_t k = lexmin_f32(pr, pf);
    if (k == *gkey) return 0;
    *gkey = k;
    gather_f32(pr, p, k, gpos);
    return 1;
}

/* One iteration t in the literal order of Alg. 1: particles in index order,
 * each one's Step 5 updating the gbest before the next particle moves. */
int oracle_step_serial_immediate_f32(const oracle_problem *pr, uint64_t t, float *x, float *v,
                                     float *p, float *pf, float *gpos, uint64_t *gkey)
{
    int changed = 0;
    for (int64_t i = 0; i < pr->N; ++i) {
        particle_update_f32(pr, t, i, x, v, p, pf, gpos);
        uint64_t k = oracle_key_f32(pf[i], (uint32_t)i);
        if (k < *gkey) {
            *gkey = k;
            gather_f32(pr, p, k, gpos);
            changed = 1;
        }
    }
    return changed;
}

static float key_value_f32(uint64_t key)
{
    uint32_t o = (uint32_t)(key >> 32);
    uint32_t b = (o & 0x80000000u) ? (o & 0x7FFFFFFFu) : ~o;
    float f;
    memcpy(&f, &b, sizeof f);
    return f;
}

float oracle_key_value_f32(uint64_t key) { return key_value_f32(key); }

/* Init plus up to T iterations; stops early once |gbest_fit - f_star| < tol
 * (tol <= 0 never stops), tested after init and after every iteration.
 * hist[t] receives the gbest key after iteration t (hist[0] after init); the
 * return value is the number of iterations run. */
int64_t oracle_run_f32(const oracle_problem *pr, int64_t T, float tol, float f_star, int serial_immediate,
                       float *x, float *v, float *p, float *pf, float *gpos, uint64_t *hist,
                       int64_t *giter)
{
    uint64_t gkey;
    oracle_init_f32(pr, x, v, p, pf, gpos, &gkey);
    if (hist) hist[0] = gkey;
    *giter = 0;
    int64_t t = 0;
    while (t < T) {
        if (tol > 0.0f && fabsf(key_value_f32(gkey) - f_star) < tol) break;
        ++t;
        int changed = serial_immediate
                          ? oracle_step_serial_immediate_f32(pr, (uint64_t)t, x, v, p, pf, gpos, &gkey)
                          : oracle_step_f32(pr, (uint64_t)t, x, v, p, pf, gpos, &gkey);
        if (changed) *giter = t;
        if (hist) hist[t] = gkey;
    }
    return t;
}

/* ------------------------------------------------------------------------- */
/* Binary64 mode: the same definition in double, from the same binary32      */
/* parameters and the same 24-bit uniforms.                                  */
/* ------------------------------------------------------------------------- */
static int64_t lexmin_f64(const oracle_problem *pr, const double *pf)
{
    int64_t bi = 0;
    uint64_t bk = ord_f64(pf[0]);
    for (int64_t i = 1; i < pr->N; ++i) {
        uint64_t k = ord_f64(pf[i]);
        if (k < bk) {
            bk = k;
            bi = i;
        }
    }
    return bi;
}

void oracle_init_f64(const oracle_problem *pr, double *x, double *v, double *p, double *pf,
                     double *gpos, int64_t *gidx)
{
    const int64_t N = pr->N;
    const int D = pr->D;
    const double lo = pr->lo, hi = pr->hi, vmax = pr->vmax;
#pragma omp parallel for schedule(static) num_threads(nthreads_of(pr))
    for (int64_t i = 0; i < N; ++i) {
        for (int d = 0; d < D; ++d) {
            float u[2];
            oracle_draw(pr->seed, ORACLE_TAG_INIT, 0, (uint64_t)i, d, u);
            double xi = clampd(lo + (hi - lo) * u[0], lo, hi);
            double vi = clampd(-vmax + 2.0 * vmax * u[1], -vmax, vmax);
            x[d * N + i] = xi;
            v[d * N + i] = vi;
            p[d * N + i] = xi;
        }
        pf[i] = oracle_fitness_f64(pr, x + i, N);
    }
    *gidx = lexmin_f64(pr, pf);
    for (int d = 0; d < D; ++d) gpos[d] = p[d * N + *gidx];
}

int oracle_step_f64(const oracle_problem *pr, uint64_t t, double *x, double *v, double *p, double *pf,
                    double *gpos, int64_t *gidx)
{
    const int64_t N = pr->N;
    const int D = pr->D;
    const double lo = pr->lo, hi = pr->hi, vmax = pr->vmax;
    const double w = pr->w, c1 = pr->c1, c2 = pr->c2;
    const int64_t prev_i = *gidx;
    const double prev_f = pf[prev_i];
#pragma omp parallel for schedule(static) num_threads(nthreads_of(pr))
    for (int64_t i = 0; i < N; ++i) {
        for (int d = 0; d < D; ++d) {
            float r[2];
            oracle_draw(pr->seed, ORACLE_TAG_VEL, t, (uint64_t)i, d, r);
            const int64_t e = d * N + i;
            double vn = w * v[e] + c1 * r[0] * (p[e] - x[e]) + c2 * r[1] * (gpos[d] - x[e]);
            vn = clampd(vn, -vmax, vmax);
            x[e] = clampd(x[e] + vn, lo, hi);
            v[e] = vn;
        }
        double f = oracle_fitness_f64(pr, x + i, N);
        if (f < pf[i]) {
            pf[i] = f;
            for (int d = 0; d < D; ++d) p[d * N + i] = x[d * N + i];
        }
    }
    const int64_t gi = lexmin_f64(pr, pf);
    *gidx = gi;
    for (int d = 0; d < D; ++d) gpos[d] = p[d * N + gi];
    return gi != prev_i || pf[gi] != prev_f;
}

/* Init plus up to T iterations in binary64; hist_f[t] and hist_i[t] receive the
 * gbest fitness and index after iteration t. */
int64_t oracle_run_f64(const oracle_problem *pr, int64_t T, double tol, double f_star, double *x, double *v,
                       double *p, double *pf, double *gpos, double *hist_f, int64_t *hist_i, int64_t *giter)
{
    int64_t gi;
    oracle_init_f64(pr, x, v, p, pf, gpos, &gi);
    double gf = pf[gi];
    if (hist_f) hist_f[0] = gf;
    if (hist_i) hist_i[0] = gi;
    *giter = 0;
    int64_t t = 0;
    while (t < T) {
        if (tol > 0.0 && fabs(gf - f_star) < tol) break;
        ++t;
        if (oracle_step_f64(pr, (uint64_t)t, x, v, p, pf, gpos, &gi)) *giter = t;
        gf = pf[gi];
        if (hist_f) hist_f[t] = gf;
        if (hist_i) hist_i[t] = gi;
    }
    return t;
}

/* ------------------------------------------------------------------------- */
/* Array helpers for the tests (elementwise loops, no other arithmetic).     */
/* ------------------------------------------------------------------------- */
void oracle_cospi_f32_array(const float *y, float *out, int64_t n)
{
    for (int64_t k = 0; k < n; ++k) out[k] = oracle_cospi_f32(y[k]);
}

void oracle_exp_f32_array(const float *x, float *out, int64_t n)
{
    for (int64_t k = 0; k < n; ++k) out[k] = oracle_exp_f32(x[k]);
}

/* Fitness of M points stored as x[d*M + m]. */
void oracle_fitness_f32_batch(const oracle_problem *pr, const float *x, int64_t M, float *out)
{
#pragma omp parallel for schedule(static) num_threads(nthreads_of(pr))
    for (int64_t m = 0; m < M; ++m) out[m] = oracle_fitness_f32(pr, x + m, M);
}

void oracle_fitness_f64_batch(const oracle_problem *pr, const double *x, int64_t M, double *out)
{
#pragma omp parallel for schedule(static) num_threads(nthreads_of(pr))
    for (int64_t m = 0; m < M; ++m) out[m] = oracle_fitness_f64(pr, x + m, M);
}

void oracle_key_f32_array(const float *f, const uint32_t *idx, uint64_t *out, int64_t n)
{
    for (int64_t k = 0; k < n; ++k) out[k] = oracle_key_f32(f[k], idx[k]);
}

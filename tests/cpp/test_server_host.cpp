// CPU unit test of the request server's host code (pso_server.hip compiled
// with g++ against tests/cpp/stub/hip/hip_runtime.h, so also under
// ThreadSanitizer).  The batched kernel is replaced by a model that advances
// each swarm one iteration at a time with a deterministic pseudo-fitness of
// (seed, iteration), so a request's result is a function of its descriptor
// alone, however the scheduler splits it over launches and streams.  Checks:
//   - every result equals the model run alone, with requests from two
//     threads, slot reuse and one part per workgroup per launch (a launch
//     that reads a slot's item or loop state before that slot's upload ran,
//     or stale from the slot's previous request, gives a wrong result);
//   - submit-to-completion latency and its percentiles under a fake clock;
//   - cancel and deadlines for queued, waiting and running requests.
// Prints "ok" and exits 0 on success.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <map>
#include <vector>

#include "pso.h"

#include "../../paper_2205_01313_amd/csrc/pso_server.hip"

// ---------------------------------------------------------------------------
// Stand-ins for the library functions pso_server.hip calls.
// ---------------------------------------------------------------------------
static thread_local char g_msg[512];

int pso_internal_fail(int code, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(g_msg, sizeof g_msg, fmt, ap);
    va_end(ap);
    return code;
}

int pso_internal_check_desc(const pso_desc *d)
{
    if (d->N < 1 || d->D < 1 || d->max_iter < 0) return pso_internal_fail(PSO_EINVAL, "bad descriptor");
    return PSO_OK;
}

namespace model {
std::atomic<int> violations{0};      // a launch read a slot that was never uploaded
std::mutex gate_mu;
std::condition_variable gate_cv;
bool gate_open = true;               // closed: launches wait (bounded) before running

uint64_t mix(uint64_t x)
{
    x ^= x >> 33;
    x *= 0xff51afd7ed558ccdull;
    x ^= x >> 33;
    x *= 0xc4ceb9fe1a85ec53ull;
    return x ^ (x >> 33);
}

// the shift vector the load test gives the swarm with this seed; while
// check_shift is set the model counts a violation for any other shift it
// finds in a launched swarm's device state
bool check_shift = false;
float shift_of(uint64_t seed, int d) { return float(mix(seed * 7919u + (uint64_t)d) % 97) - 48.0f; }

// pseudo-fitness of the swarm with this seed at iteration t (t = 0: Step 1)
unsigned long long key_at(uint64_t seed, long long t, uint64_t N)
{
    const uint64_t h = mix(seed * 0x9E3779B97F4A7C15ull + (uint64_t)t);
    const float f = float(h >> 40) * 0x1p-24f * (1.0f + float(t % 7));
    return pso::make_key(f, (uint32_t)(mix(h) % N));
}

// what the server must return for a descriptor: the same iterations alone
pso::BatchResult alone(const pso_desc &d)
{
    pso::BatchResult r{pso::NO_KEY, 0, 0, 1u, 0u, 0u, 0u};
    r.gkey = key_at(d.seed, 0, d.N);
    auto met = [&] { return d.tol > 0.0f && std::fabs(pso::key_fitness(r.gkey) - d.f_star) < d.tol; };
    r.stop = met();
    while (!r.stop && r.iters < d.max_iter) {
        ++r.iters;
        const unsigned long long k = key_at(d.seed, r.iters, d.N);
        if (k < r.gkey) {
            r.gkey = k;
            r.giter = r.iters;
        }
        r.stop = met();
    }
    return r;
}

void wait_gate()
{
    std::unique_lock<std::mutex> lk(gate_mu);
    gate_cv.wait_for(lk, std::chrono::seconds(20), [] { return gate_open; });
}

// The batched launch, run on the stream's thread: for every swarm listed
// (its part 0), Step 1 if not started, then the entry's iterations.
void batch(const pso::BatchItem *items, const pso::BatchEntry *entries, pso::BatchResult *results, uint32_t count,
           long long chunk, long long iter_cap, pso::BatchResult *out_state, float *out_pos, int maxD)
{
    wait_gate();
    stub_delay();
    for (uint32_t j = 0; j < count; ++j) {
        const pso::BatchEntry e = entries[j];
        if (e.part != 0) continue;
        const pso::BatchItem &it = items[e.item];
        if (!it.a.x || it.a.N == 0 || it.a.D < 1 || it.a.D > maxD) {
            violations.fetch_add(1);
            continue;
        }
        pso::BatchResult &r = results[e.item];
        const uint64_t seed = (uint64_t)it.a.k0 | ((uint64_t)it.a.k1 << 32);
        if (check_shift)
            for (int d = 0; d < it.a.D; ++d)
                if (it.a.shift[d] != shift_of(seed, d)) {
                    violations.fetch_add(1);
                    break;
                }
        auto met = [&] { return it.tol > 0.0f && std::fabs(pso::key_fitness(r.gkey) - it.fstar) < it.tol; };
        if (!r.started) {
            r = pso::BatchResult{key_at(seed, 0, it.a.N), 0, 0, 1u, 0u, 0u, 0u};
            r.stop = met();
        }
        const long long work = (long long)it.a.N * it.a.D;
        const long long iters = e.iters ? e.iters : std::max(1LL, std::min(iter_cap, chunk / work));
        long long ran = 0;
        for (; ran < iters && !r.stop && r.iters < it.max_iter; ++ran) {
            ++r.iters;
            const unsigned long long k = key_at(seed, r.iters, it.a.N);
            if (k < r.gkey) {
                r.gkey = k;
                r.giter = r.iters;
            }
            r.stop = met();
        }
        r.ticks = (uint32_t)(100 * ran); // 1 us per iteration at 100 ticks per us
        // the gbest position: a function of the swarm and its gbest iteration
        for (int d = 0; d < it.a.D; ++d) it.a.gpos[d] = float(mix(seed + 31 * (uint64_t)r.giter + (uint64_t)d) % 1000);
        if (out_state) out_state[e.out] = r;
        if (out_pos)
            for (int d = 0; d < it.a.D; ++d) out_pos[(size_t)e.out * maxD + d] = it.a.gpos[d];
    }
}
} // namespace model

namespace pso {

static size_t al(size_t b) { return (b + 255) & ~size_t(255); }

Layout layout_of(uint64_t N, int D, bool control)
{
    Layout L{};
    L.control = control;
    L.Np = (N + 63) / 64 * 64;
    size_t o = 0;
    L.gpos = o;
    o += al(4 * (size_t)D);
    L.shift = o;
    o += al(4 * (size_t)D);
    L.pf = o;
    o += al(4 * L.Np);
    L.pend = o;
    o += al(L.Np);
    L.x = o;
    o += al(4 * L.Np * D);
    L.v = o;
    o += al(4 * L.Np * D);
    L.p = o;
    o += al(4 * L.Np * D);
    L.total = o;
    return L;
}

SwarmArgs bind(void *base, const Layout &L, uint64_t N, int D)
{
    char *b = static_cast<char *>(base);
    SwarmArgs a{};
    a.gpos = reinterpret_cast<float *>(b + L.gpos);
    a.shift = reinterpret_cast<const float *>(b + L.shift);
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

size_t gang_bytes(uint32_t parts, int D) { return parts <= 1 ? 0 : al(64) + al(16 * parts) + al(8 * parts * (size_t)D); }

void bind_gang(BatchItem *it, void *region, uint32_t parts)
{
    it->parts = parts < 1 ? 1 : parts;
    it->gang = it->parts > 1 ? static_cast<GangSync *>(region) : nullptr;
    it->cand_key = nullptr;
    it->cand_pos = nullptr;
}

// a part per 20 000 particle-dimensions, within the launch's workgroups
uint32_t staged_parts(uint64_t N, int D, int, int stage_kib, int grid_cap)
{
    if (stage_kib < 1) return 0;
    const uint64_t parts = (N * (uint64_t)D + 19999) / 20000;
    return parts <= (uint64_t)grid_cap ? (uint32_t)parts : 0;
}

uint32_t parts_for(uint64_t N, int D, int grid_cap, const BatchShape &)
{
    return (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>((N * (uint64_t)D + 49999) / 50000,
                                                                  (uint64_t)std::max(1, grid_cap)));
}

hipError_t batch_capacity(int, int, int *workgroups, int stage_kib)
{
    *workgroups = stage_kib > 0 ? 16 : 24; // small, so a burst needs many launches
    return hipSuccess;
}

hipError_t launch_batch(const BatchItem *items, const BatchEntry *entries, BatchResult *results, uint32_t count,
                        unsigned int *, int maxD, int, int, long long chunk, long long iter_cap, hipStream_t stream,
                        BatchResult *out_state, float *out_pos, unsigned int *, int)
{
    stub_enqueue(stream, [=] { model::batch(items, entries, results, count, chunk, iter_cap, out_state, out_pos, maxD); });
    return hipSuccess;
}

hipError_t launch_upload(const UploadRec *recs, uint32_t n, const float *pool, BatchItem *items, BatchResult *state,
                         hipStream_t stream)
{
    if (n == 0) return hipSuccess;
    stub_enqueue(stream, [=] {
        for (uint32_t r = 0; r < n; ++r) {
            const UploadRec &u = recs[r];
            items[u.slot] = u.item;
            state[u.slot] = u.state;
            if (u.reset_gang && u.item.gang) *u.item.gang = GangSync{};
            float *shift = const_cast<float *>(u.item.a.shift);
            for (int d = 0; d < u.item.a.D; ++d) shift[d] = pool[u.shift_at + d];
        }
    });
    return hipSuccess;
}

} // namespace pso

// ---------------------------------------------------------------------------
// Tests.
// ---------------------------------------------------------------------------
#define CHECK(c)                                                                        \
    do {                                                                                \
        if (!(c)) {                                                                     \
            std::printf("FAIL line %d: %s (%s)\n", __LINE__, #c, g_msg);               \
            std::exit(1);                                                               \
        }                                                                               \
    } while (0)

static pso_desc desc_of(uint64_t seed, int64_t N, int D, int64_t max_iter, float tol)
{
    pso_desc d{};
    d.fitness_id = PSO_SPHERE;
    d.D = D;
    d.N = N;
    d.bounds[0] = -1.0f;
    d.bounds[1] = 1.0f;
    d.w = 0.7f;
    d.c1 = d.c2 = 1.4f;
    d.vmax = 0.2f;
    d.seed = seed;
    d.max_iter = max_iter;
    d.tol = tol;
    d.f_star = 0.0f;
    return d;
}

static int wait_result(pso_server *srv, uint64_t t, pso_result *r, double *lat, int seconds = 60)
{
    const auto t0 = std::chrono::steady_clock::now();
    for (;;) {
        const int rc = pso_server_poll(srv, t, r, lat);
        if (rc != PSO_EAGAIN) return rc;
        CHECK(std::chrono::steady_clock::now() - t0 < std::chrono::seconds(seconds));
        std::this_thread::sleep_for(std::chrono::microseconds(200));
    }
}

static void set_gate(bool open)
{
    {
        std::lock_guard<std::mutex> g(model::gate_mu);
        model::gate_open = open;
    }
    model::gate_cv.notify_all();
}

// Results equal the model alone: two submitting threads, 64 slots reused
// many times, one part per workgroup per launch.
static void test_results_under_load()
{
    setenv("PSO_SERVER_LAUNCH_WAVES", "1", 1);
    pso_server *srv = nullptr;
    CHECK(pso_server_create(size_t(64) << 16, 0, &srv) == PSO_OK); // 64 slots
    const int n = 600;
    std::vector<pso_desc> descs(n);
    std::vector<std::vector<float>> shifts(n);
    std::mt19937 rng(5);
    for (int k = 0; k < n; ++k) {
        descs[k] = desc_of(1000 + k, 16 + rng() % 3000, 1 + rng() % 40, 1 + rng() % 300, k % 5 == 0 ? 0.05f : 0.0f);
        for (int d = 0; d < descs[k].D; ++d) shifts[k].push_back(model::shift_of(descs[k].seed, d));
        descs[k].shift = shifts[k].data();
    }
    model::check_shift = true;
    std::vector<uint64_t> tickets(n);
    std::vector<std::vector<float>> pos(n);
    auto submitter = [&](int lo) {
        for (int k = lo; k < n; k += 2) {
            CHECK(pso_server_submit(srv, &descs[k], &tickets[k]) == PSO_OK);
            if (k % 50 == 0) std::this_thread::sleep_for(std::chrono::microseconds(300));
        }
    };
    std::thread a(submitter, 0), b(submitter, 1);
    a.join();
    b.join();
    for (int k = 0; k < n; ++k) {
        pso_result r{};
        pos[k].assign(descs[k].D, -1.0f);
        r.gbest_pos = pos[k].data();
        double lat = 0;
        CHECK(wait_result(srv, tickets[k], &r, &lat) == PSO_OK);
        const pso::BatchResult m = model::alone(descs[k]);
        CHECK(r.iters == m.iters && r.gbest_iter == m.giter);
        CHECK(r.gbest_value == pso::key_fitness(m.gkey) || (std::isnan(r.gbest_value) && std::isnan(pso::key_fitness(m.gkey))));
        for (int d = 0; d < descs[k].D; ++d)
            CHECK(pos[k][d] == float(model::mix(descs[k].seed + 31 * (uint64_t)m.giter + (uint64_t)d) % 1000));
    }
    pso_server_counters st{};
    CHECK(pso_server_stats(srv, &st) == PSO_OK);
    CHECK(st.completed == (uint64_t)n && st.mem_used == 0 && st.launches > 20);
    CHECK(model::violations.load() == 0);
    CHECK(pso_server_destroy(srv) == PSO_OK);
    model::check_shift = false;
    unsetenv("PSO_SERVER_LAUNCH_WAVES");
}

// Latency accounting under a fake clock.
static std::atomic<long long> g_fake_ns{0};
static std::chrono::steady_clock::time_point fake_now()
{
    return std::chrono::steady_clock::time_point(std::chrono::nanoseconds(g_fake_ns.load()));
}
static void set_fake_ms(double ms) { g_fake_ns.store((long long)(ms * 1e6)); }

static void wait_launches(pso_server *srv, uint64_t at_least)
{
    const auto t0 = std::chrono::steady_clock::now();
    for (;;) {
        pso_server_counters st{};
        CHECK(pso_server_stats(srv, &st) == PSO_OK);
        if (st.launches >= at_least) return;
        CHECK(std::chrono::steady_clock::now() - t0 < std::chrono::seconds(30));
        std::this_thread::sleep_for(std::chrono::microseconds(200));
    }
}

static void test_latency_with_fake_clock()
{
    set_fake_ms(1000.0);
    set_gate(false);
    pso_server *srv = nullptr;
    CHECK(pso_server_create(size_t(1) << 26, 0, &srv) == PSO_OK);
    srv->clock.store(&fake_now);
    // three requests finished by their first launch (FIRST_ITERS covers 3)
    const pso_desc a = desc_of(1, 100, 4, 3, 0.0f), b = desc_of(2, 100, 4, 3, 0.0f), c = desc_of(3, 100, 4, 3, 0.0f);
    uint64_t ta, tb, tc;
    CHECK(pso_server_submit(srv, &a, &ta) == PSO_OK);
    set_fake_ms(1003.0);
    CHECK(pso_server_submit(srv, &b, &tb) == PSO_OK);
    set_fake_ms(1004.5);
    CHECK(pso_server_submit(srv, &c, &tc) == PSO_OK);
    wait_launches(srv, 1);
    set_fake_ms(1010.0); // every launch is held at the gate until now
    set_gate(true);
    pso_result r{};
    double la = 0, lb = 0, lc = 0;
    CHECK(wait_result(srv, ta, &r, &la) == PSO_OK);
    CHECK(wait_result(srv, tb, &r, &lb) == PSO_OK);
    CHECK(wait_result(srv, tc, &r, &lc) == PSO_OK);
    CHECK(la == 10.0 && lb == 7.0 && lc == 5.5);
    pso_server_counters st{};
    CHECK(pso_server_stats(srv, &st) == PSO_OK);
    // percentiles of {5.5, 7, 10}: nearest rank over the sorted latencies
    CHECK(st.completed == 3 && st.p50_ms == 7.0 && st.p99_ms == 10.0 && st.max_ms == 10.0);
    CHECK(pso_server_destroy(srv) == PSO_OK);
}

// Cancel and deadlines: a queued request, a waiting one, a running one.
static void test_cancel_and_deadlines()
{
    set_fake_ms(2000.0);
    set_gate(false);
    const pso_desc big = desc_of(7, 4000, 8, 100000, 0.0f); // never finishes in one launch
    const size_t one = pso::layout_of(4000, 8, false).total;
    pso_server *srv = nullptr;
    CHECK(pso_server_create(one + one / 2, 0, &srv) == PSO_OK); // room for one such request
    srv->clock.store(&fake_now);
    uint64_t t_run, t_wait, t_q;
    CHECK(pso_server_submit(srv, &big, &t_run) == PSO_OK);
    wait_launches(srv, 1); // admitted and launched, held at the gate
    CHECK(pso_server_submit(srv, &big, &t_wait) == PSO_OK); // waits for memory
    CHECK(pso_server_set_deadline(srv, t_wait, 5.0) == PSO_OK);
    CHECK(pso_server_submit(srv, &big, &t_q) == PSO_OK); // waits behind it
    CHECK(pso_server_set_deadline(srv, t_q, 0.0) == PSO_EINVAL);
    CHECK(pso_server_cancel(srv, t_q) == PSO_OK); // still queued: leaves at once
    pso_result r{};
    double lat = -1;
    CHECK(pso_server_poll(srv, t_q, &r, &lat) == PSO_ECANCELED && lat == 0.0);
    CHECK(pso_server_cancel(srv, t_q) == PSO_EINVAL); // forgotten after the poll
    set_fake_ms(2006.0); // the waiting request passes its deadline while queued
    CHECK(wait_result(srv, t_wait, &r, &lat) == PSO_ETIMEDOUT && lat == 6.0);
    // the running request: a deadline that passes while its launch is held
    CHECK(pso_server_set_deadline(srv, t_run, 8.0) == PSO_OK);
    set_fake_ms(2009.0);
    set_gate(true);
    CHECK(wait_result(srv, t_run, &r, &lat) == PSO_ETIMEDOUT);
    // its memory is back: a new request runs to its end
    const pso_desc small = desc_of(8, 200, 3, 50, 0.0f);
    uint64_t t_s;
    CHECK(pso_server_submit(srv, &small, &t_s) == PSO_OK);
    CHECK(wait_result(srv, t_s, &r, &lat) == PSO_OK && r.iters == 50);
    CHECK(pso_server_cancel(srv, 999999) == PSO_EINVAL);
    // cancel of an admitted request between launches
    uint64_t t_c;
    CHECK(pso_server_submit(srv, &big, &t_c) == PSO_OK);
    wait_launches(srv, 4);
    CHECK(pso_server_cancel(srv, t_c) == PSO_OK);
    CHECK(wait_result(srv, t_c, &r, &lat) == PSO_ECANCELED);
    pso_server_counters st{};
    CHECK(pso_server_stats(srv, &st) == PSO_OK);
    CHECK(st.cancelled == 2 && st.timed_out == 2 && st.completed == 1 && st.mem_used == 0);
    CHECK(pso_server_destroy(srv) == PSO_OK);
}

int main()
{
    test_results_under_load();
    test_latency_with_fake_clock();
    test_cancel_and_deadlines();
    CHECK(model::violations.load() == 0);
    std::printf("ok\n");
    return 0;
}

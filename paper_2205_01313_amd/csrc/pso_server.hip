// pso_server.hip -- request server with continuous batching.
//
// Motivation: the paper targets real-time uses of PSO (object tracking,
// posture estimation; Sec. 1), where solves arrive over time.  Requests
// (pso_desc) are admitted in arrival order as device memory frees up (the
// Arena/Admission bookkeeping of pso_arena.hpp), their swarm state stays
// resident on the device, and a scheduler thread keeps up to two batched
// launches in flight on two streams: each launch advances every swarm in its
// set by the iterations that fit a fixed time slice at that swarm's measured
// speed (Step 1 first for new swarms), so
// requests that arrive while a launch runs start on the other stream and
// overlap on the device.  Between launches a swarm's loop state stays in
// device memory, so its result is the same bits as running it alone.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "pso.h"
#include "pso_arena.hpp"
#include "pso_block.hpp"
#include "pso_guard.hpp"
#include "pso_device.hpp"
#include "pso_kernels.hpp"

int pso_internal_fail(int code, const char *fmt, ...);
int pso_internal_check_desc(const pso_desc *d);

namespace {

using Clock = std::chrono::steady_clock;

double ms_since(Clock::time_point t0, Clock::time_point t1)
{
    return std::chrono::duration<double, std::milli>(t1 - t0).count();
}

struct Req {
    uint64_t ticket = 0;
    pso_desc d{};
    std::vector<float> shift;
    Clock::time_point t_submit, t_done;
    int status = PSO_EAGAIN; // PSO_OK when done, PSO_ENOMEM rejected, PSO_ECANCELED / PSO_ETIMEDOUT dropped
    // set by pso_server_cancel or a passed deadline while the request is
    // admitted: the scheduler drops it at its next scheduling point
    std::atomic<int> drop_code{0};
    size_t off = 0;
    int slot = -1;
    uint32_t parts = 1;
    pso::BatchResult res{};
    std::vector<float> gpos;
    double us_per_iter = 0.0; // measured time of one iteration on the device (0: not yet)
    long long prev_iters = 0;
    bool staged = false;      // runs in LDS-staged launches (else streamed ones)
};

#ifndef PSO_SERVER_STREAMS
#define PSO_SERVER_STREAMS 2
#endif
constexpr int STREAMS = PSO_SERVER_STREAMS;
// Time slice of a launch: every swarm runs as many iterations as fit in it
// at its own measured speed (the device times each swarm's share of a
// launch), so a launch lasts about the slice whatever its mix, and a small
// swarm is not held behind a large one's iterations.  A swarm's first
// launch runs FIRST_ITERS iterations to measure it.  Measured on the
// serving workload (p50 / p99 ms at 2000 and 10 000 requests/s): 300 us
// 41 / 438 and 151 / 665; 1 ms 34 / 244 and 97 / 469; 2 ms 36 / 225 and
// 91 / 434; 4 ms 39 / 224 and 92 / 375 (iteration-count chunks before:
// 127 / 377 and 235 / 481).
constexpr double SLICE_US_DEFAULT = 2000.0;
constexpr uint32_t FIRST_ITERS = 4;
// Parts of one launch: at most this many per workgroup of its grid (a
// launch's swarms are the longest-waiting ready ones).  Measured on the
// serving workload with staged launches of half the co-resident workgroups
// (p99 ms and requests/s at 10 000 and 50 000 requests/s): 1: 227 / 4.7k,
// 397 / 4.5k; 2: 198 / 5.1k, 353 / 5.1k; 4: 156 / 5.8k, 308 / 5.7k; 8:
// 155 / 6.1k, 292 / 6.0k; 16: 204 / 5.9k, 290 / 6.1k; no limit: 295 /
// 5.1k, 451 / 4.1k; with launches of every co-resident workgroup (below),
// at 10 000 requests/s (p99 ms, requests/s): 2: 169 / 9.3k; 4: 165 / 9.4k;
// 8: 223 / 9.4k; 16: 274 / 9.3k.  PSO_SERVER_LAUNCH_WAVES overrides it.
constexpr int LAUNCH_WAVES_DEFAULT = 4;
constexpr uint32_t MAX_SLICE_ITERS = 4096;
constexpr int MAX_SERVER_D = 4096; // LDS of a launch is sized for the largest D it lists
// LDS-staged launches: one 1024-lane workgroup per compute unit with 158 KiB
// of staged state, which leaves room for the gbest position and shift of
// D <= SERVER_STAGE_MAX_D in the 160 KiB.  A request of such D whose staged
// parts fit a launch runs staged (its state in LDS for each launch), others
// streamed; each launch is of one kind, the kind of the longest-waiting
// ready request.  PSO_SERVER_STAGED=0 in the environment streams every
// request.
constexpr int SERVER_STAGE_LANES = 1024;
constexpr int SERVER_STAGE_KIB = 158;
constexpr int SERVER_STAGE_MAX_D = 64;

} // namespace

struct pso_server {
    // configuration
    size_t budget = 0;
    long long chunk = 1LL << 40; // at most this many particle-dimension updates per swarm and launch
    int max_slots = 0;
    int grid_cap = 1;            // parts of a streamed swarm at most: half the co-resident workgroups
    int grid_cap_staged = 0;     // the same for a staged swarm (0: staging off)
    int launch_cap_staged = 0;   // workgroups of a staged launch (a streamed one has grid_cap)
    double ticks_per_us = 100.0; // device wall clock
    double slice_us = SLICE_US_DEFAULT;
    int launch_waves = LAUNCH_WAVES_DEFAULT;
    // device memory
    void *base = nullptr;
    pso::BatchItem *d_items = nullptr;
    pso::BatchResult *d_state = nullptr;
    pso::BatchEntry *d_entries[STREAMS] = {};
    unsigned int *d_next[STREAMS] = {};
    unsigned int *d_err = nullptr;
    pso::BatchResult *d_out[STREAMS] = {}; // compact state of a launch's items
    float *d_opos[STREAMS] = {};           // compact gbest positions (cap_pos floats)
    size_t cap_pos[STREAMS] = {};
    pso::UploadRec *d_up[STREAMS] = {};    // a launch's first uploads (max_slots records)
    float *d_pool[STREAMS] = {};           // their shift vectors (cap_pool floats)
    size_t cap_pool[STREAMS] = {};
    int launch_maxD[STREAMS] = {};
    // pinned staging
    pso::BatchItem *h_items = nullptr;   // max_slots
    pso::BatchResult *h_state = nullptr; // max_slots (fresh state for new swarms)
    pso::BatchEntry *h_entries[STREAMS] = {};
    size_t cap_entries[STREAMS] = {};
    unsigned int *h_err[STREAMS] = {};
    pso::BatchResult *h_out[STREAMS] = {};
    float *h_opos[STREAMS] = {};        // cap_pos floats
    pso::UploadRec *h_up[STREAMS] = {}; // max_slots records
    float *h_pool[STREAMS] = {};        // cap_pool floats
    hipStream_t st[STREAMS] = {};
    hipEvent_t ev[STREAMS] = {};
    // bookkeeping (guarded by mu)
    std::mutex mu;
    std::condition_variable cv;
    pso::Arena arena;
    pso::Admission adm{&arena};
    std::unordered_map<uint64_t, std::unique_ptr<Req>> reqs;
    uint64_t next_ticket = 1;
    std::vector<int> free_slots;
    std::vector<Req *> slot_req;
    // scheduler-thread state
    std::vector<int> ready;              // started or new swarms not in flight
    std::vector<int> fresh;              // slots whose item/state must be uploaded
    std::vector<int> fresh_gang;         // of those, slots whose gang counter must be cleared
    std::vector<char> pending_upload;    // per slot: admitted, its upload not yet enqueued
    std::vector<int> inflight[STREAMS];  // slots of each in-flight launch
    bool busy[STREAMS] = {};
    std::thread th;
    std::atomic<bool> quit{false};
    std::atomic<int> device_error{0};
    std::atomic<int> order_error{0};     // a launch listed a slot whose upload was not enqueued first
    // statistics (guarded by mu)
    uint64_t submitted = 0, completed = 0, rejected = 0, launches = 0;
    uint64_t cancelled = 0, timed_out = 0;
    size_t peak_used = 0;
    std::vector<double> latencies;
    std::multimap<Clock::time_point, uint64_t> deadlines; // (deadline, ticket), guarded by mu
    // the server's clock (submit and completion times, deadlines); a unit
    // test of the host scheduler replaces it by a fake one
    std::atomic<Clock::time_point (*)()> clock{&Clock::now};
    Clock::time_point now() const { return clock.load()(); }
};

namespace {

void server_loop(pso_server *s);

void server_free(pso_server *s)
{
    if (!s) return;
    for (int k = 0; k < STREAMS; ++k) {
        if (s->st[k]) (void)hipStreamSynchronize(s->st[k]);
    }
    (void)hipFree(s->base);
    (void)hipFree(s->d_items);
    (void)hipFree(s->d_state);
    (void)hipFree(s->d_err);
    for (int k = 0; k < STREAMS; ++k) {
        (void)hipFree(s->d_entries[k]);
        (void)hipFree(s->d_next[k]);
        (void)hipFree(s->d_out[k]);
        (void)hipFree(s->d_opos[k]);
        (void)hipFree(s->d_up[k]);
        (void)hipFree(s->d_pool[k]);
        (void)hipHostFree(s->h_opos[k]);
        (void)hipHostFree(s->h_up[k]);
        (void)hipHostFree(s->h_pool[k]);
        (void)hipHostFree(s->h_entries[k]);
        (void)hipHostFree(s->h_err[k]);
        (void)hipHostFree(s->h_out[k]);
        if (s->ev[k]) (void)hipEventDestroy(s->ev[k]);
        if (s->st[k]) (void)hipStreamDestroy(s->st[k]);
    }
    (void)hipHostFree(s->h_items);
    (void)hipHostFree(s->h_state);
    delete s;
}

// Item of a newly admitted request, bound to its arena range.
pso::BatchItem make_item(pso_server *s, const Req &r)
{
    const pso::Layout L = pso::layout_of((uint64_t)r.d.N, r.d.D, false);
    pso::BatchItem it{};
    it.a = pso::bind(static_cast<char *>(s->base) + r.off, L, (uint64_t)r.d.N, r.d.D);
    it.a.lo = r.d.bounds[0];
    it.a.hi = r.d.bounds[1];
    it.a.w = r.d.w;
    it.a.c1 = r.d.c1;
    it.a.c2 = r.d.c2;
    it.a.vmax = r.d.vmax;
    it.a.k0 = (uint32_t)r.d.seed;
    it.a.k1 = (uint32_t)(r.d.seed >> 32);
    it.fitness = r.d.fitness_id;
    it.max_iter = r.d.max_iter;
    it.tol = r.d.tol;
    it.fstar = r.d.f_star;
    pso::bind_gang(&it, static_cast<char *>(s->base) + r.off + L.total, r.parts);
    return it;
}

// Ends an admitted request that was cancelled or passed its deadline and is
// not in flight: its memory and slot return to the pool, a pending upload is
// forgotten, and a poll then reports the code.  Scheduler thread.
void drop_slot(pso_server *s, int slot)
{
    Req *r = s->slot_req[slot];
    s->pending_upload[slot] = 0;
    s->fresh.erase(std::remove(s->fresh.begin(), s->fresh.end(), slot), s->fresh.end());
    s->fresh_gang.erase(std::remove(s->fresh_gang.begin(), s->fresh_gang.end(), slot), s->fresh_gang.end());
    std::lock_guard<std::mutex> g(s->mu);
    const int code = r->drop_code.load();
    r->status = code;
    r->t_done = s->now();
    ++(code == PSO_ETIMEDOUT ? s->timed_out : s->cancelled);
    s->arena.release(r->off);
    s->slot_req[slot] = nullptr;
    s->free_slots.push_back(slot);
    s->cv.notify_all();
}

// Requests whose deadline has passed: a queued one leaves the queue now, an
// admitted one is marked for drop_slot.  Under s->mu; true if any expired.
bool expire_deadlines(pso_server *s)
{
    bool any = false;
    const auto now = s->now();
    while (!s->deadlines.empty() && s->deadlines.begin()->first <= now) {
        const uint64_t t = s->deadlines.begin()->second;
        s->deadlines.erase(s->deadlines.begin());
        auto it = s->reqs.find(t);
        if (it == s->reqs.end()) continue;
        Req *r = it->second.get();
        if (r->status != PSO_EAGAIN) continue;
        any = true;
        if (r->slot < 0 && s->adm.cancel(t)) {
            r->status = PSO_ETIMEDOUT;
            r->t_done = now;
            ++s->timed_out;
            s->cv.notify_all();
        } else {
            int none = 0;
            r->drop_code.compare_exchange_strong(none, PSO_ETIMEDOUT);
        }
    }
    return any;
}

// Launches one chunk on stream k over ready swarms of one kind (staged or
// streamed): the kind of the ready swarm submitted first, and of that kind
// the longest-waiting swarms whose parts fit the launch's workgroups.
bool launch_ready(pso_server *s, int k)
{
    if (s->ready.empty()) return true;
    hipStream_t st = s->st[k];
    const Req *first = s->slot_req[s->ready[0]];
    for (int slot : s->ready)
        if (s->slot_req[slot]->t_submit < first->t_submit) first = s->slot_req[slot];
    const bool staged = first->staged;
    // the longest-waiting swarms of that kind, at most launch_waves parts per
    // workgroup, so that a launch lasts about that many slices and the two
    // streams take turns
    const int grid_cap = staged ? s->launch_cap_staged : s->grid_cap;
    std::stable_sort(s->ready.begin(), s->ready.end(),
                     [&](int x, int y) { return s->slot_req[x]->t_submit < s->slot_req[y]->t_submit; });
    std::vector<int> sel, rest;
    uint64_t parts = 0;
    for (int slot : s->ready) {
        const Req *r = s->slot_req[slot];
        if (r->staged == staged && parts + r->parts <= (uint64_t)grid_cap * s->launch_waves) {
            sel.push_back(slot);
            parts += r->parts;
        } else {
            rest.push_back(slot);
        }
    }
    // Upload the items, fresh loop states and shift vectors of the new swarms
    // this launch runs -- the slots in `sel`, nothing else.  An upload is
    // ordered before the launch on its own stream only, so a fresh slot left
    // for a later launch keeps its upload pending until that launch (on
    // either stream) takes it.  The uploads of a launch are packed into one
    // record array and one float pool: two copies and one scatter kernel
    // (one copy per table entry cost a dispatch each -- about 200 per launch
    // and 3 ms of stream time between launches at 10 000 requests/s).
    std::vector<char> in_sel(s->max_slots, 0);
    for (int slot : sel) in_sel[slot] = 1;
    std::vector<char> gang_due(s->max_slots, 0);
    for (int slot : s->fresh_gang) gang_due[slot] = 1;
    std::vector<int> fresh_rest, gang_rest;
    size_t pool_need = 0;
    for (int slot : s->fresh)
        if (in_sel[slot]) pool_need += (size_t)s->slot_req[slot]->d.D;
    if (pool_need > s->cap_pool[k]) { // grow this stream's float pool (the stream is idle)
        if (hipStreamSynchronize(st) != hipSuccess) return false;
        (void)hipFree(s->d_pool[k]);
        (void)hipHostFree(s->h_pool[k]);
        s->d_pool[k] = nullptr;
        s->h_pool[k] = nullptr;
        s->cap_pool[k] = std::max(pool_need, 2 * s->cap_pool[k]);
        if (hipMalloc(&s->d_pool[k], sizeof(float) * s->cap_pool[k]) != hipSuccess ||
            hipHostMalloc(reinterpret_cast<void **>(&s->h_pool[k]), sizeof(float) * s->cap_pool[k],
                          hipHostMallocDefault) != hipSuccess)
            return false;
    }
    uint32_t nup = 0, at = 0;
    for (int slot : s->fresh) {
        if (!in_sel[slot]) {
            fresh_rest.push_back(slot);
            continue;
        }
        const Req *r = s->slot_req[slot];
        pso::UploadRec &u = s->h_up[k][nup++];
        u.item = s->h_items[slot];
        u.state = s->h_state[slot];
        u.slot = (uint32_t)slot;
        u.shift_at = at;
        u.reset_gang = gang_due[slot] ? 1u : 0u;
        u.pad = 0;
        std::memcpy(s->h_pool[k] + at, r->shift.data(), sizeof(float) * r->d.D);
        at += (uint32_t)r->d.D;
        s->pending_upload[slot] = 0;
    }
    for (int slot : s->fresh_gang)
        if (!in_sel[slot]) gang_rest.push_back(slot);
    if (nup > 0) {
        if (hipMemcpyAsync(s->d_up[k], s->h_up[k], sizeof(pso::UploadRec) * nup, hipMemcpyHostToDevice, st) !=
                hipSuccess ||
            hipMemcpyAsync(s->d_pool[k], s->h_pool[k], sizeof(float) * at, hipMemcpyHostToDevice, st) != hipSuccess ||
            pso::launch_upload(s->d_up[k], nup, s->d_pool[k], s->d_items, s->d_state, st) != hipSuccess)
            return false;
    }
    s->fresh.swap(fresh_rest);
    s->fresh_gang.swap(gang_rest);
    // every slot of this launch has its upload ordered before the launch
    for (int slot : sel)
        if (s->pending_upload[slot]) {
            s->order_error.store(1);
            return false;
        }
    s->ready.swap(sel); // the launch's swarms, until they move to inflight
    // largest per-part work first; a swarm's parts are consecutive
    std::stable_sort(s->ready.begin(), s->ready.end(), [&](int x, int y) {
        const Req *a = s->slot_req[x], *b = s->slot_req[y];
        return double(a->d.N) * a->d.D / a->parts > double(b->d.N) * b->d.D / b->parts;
    });
    const int n = (int)s->ready.size();
    int maxD = 1;
    size_t need_entries = 0;
    for (int j = 0; j < n; ++j) need_entries += s->slot_req[s->ready[j]]->parts;
    if (need_entries > s->cap_entries[k]) { // grow the entry lists of this stream
        if (hipStreamSynchronize(st) != hipSuccess) return false;
        (void)hipFree(s->d_entries[k]);
        (void)hipHostFree(s->h_entries[k]);
        s->d_entries[k] = nullptr;
        s->h_entries[k] = nullptr;
        s->cap_entries[k] = std::max(need_entries, 2 * s->cap_entries[k]);
        if (hipMalloc(&s->d_entries[k], sizeof(pso::BatchEntry) * s->cap_entries[k]) != hipSuccess ||
            hipHostMalloc(reinterpret_cast<void **>(&s->h_entries[k]), sizeof(pso::BatchEntry) * s->cap_entries[k],
                          hipHostMallocDefault) != hipSuccess)
            return false;
    }
    uint32_t ne = 0;
    for (int j = 0; j < n; ++j) {
        const Req *r = s->slot_req[s->ready[j]];
        // iterations of this launch: the slice at the swarm's measured speed,
        // at most `chunk` updates' worth
        uint32_t iters = FIRST_ITERS;
        if (r->us_per_iter > 0.0) {
            const double by_time = s->slice_us / r->us_per_iter;
            const double by_work = double(s->chunk) / (double(r->d.N) * double(r->d.D));
            iters = (uint32_t)std::max(1.0, std::min({by_time, by_work, double(MAX_SLICE_ITERS)}));
        }
        for (uint32_t p = 0; p < r->parts; ++p)
            s->h_entries[k][ne++] = pso::BatchEntry{(uint32_t)s->ready[j], p, (uint32_t)j, iters};
        maxD = std::max(maxD, (int)r->d.D);
    }
    if (hipMemcpyAsync(s->d_entries[k], s->h_entries[k], sizeof(pso::BatchEntry) * ne, hipMemcpyHostToDevice, st) !=
        hipSuccess)
        return false;
    const size_t need = (size_t)n * maxD;
    if (need > s->cap_pos[k]) { // grow the compact position buffers
        if (hipStreamSynchronize(st) != hipSuccess) return false;
        (void)hipFree(s->d_opos[k]);
        (void)hipHostFree(s->h_opos[k]);
        s->d_opos[k] = nullptr;
        s->h_opos[k] = nullptr;
        s->cap_pos[k] = std::max(need, 2 * s->cap_pos[k]);
        if (hipMalloc(&s->d_opos[k], sizeof(float) * s->cap_pos[k]) != hipSuccess ||
            hipHostMalloc(reinterpret_cast<void **>(&s->h_opos[k]), sizeof(float) * s->cap_pos[k],
                          hipHostMallocDefault) != hipSuccess)
            return false;
    }
    const int grid = std::min<int>((int)ne, grid_cap);
    if (pso::launch_batch(s->d_items, s->d_entries[k], s->d_state, ne, s->d_next[k], maxD, grid,
                          staged ? SERVER_STAGE_LANES : pso::DEFAULT_BATCH_SHAPE.lanes, s->chunk, MAX_SLICE_ITERS, st,
                          s->d_out[k], s->d_opos[k], s->d_err, staged ? SERVER_STAGE_KIB : 0) != hipSuccess)
        return false;
    // the launch's results, positions included, come back before its event
    if (hipMemcpyAsync(s->h_out[k], s->d_out[k], sizeof(pso::BatchResult) * n, hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipMemcpyAsync(s->h_opos[k], s->d_opos[k], sizeof(float) * need, hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipMemcpyAsync(s->h_err[k], s->d_err, sizeof(unsigned int), hipMemcpyDeviceToHost, st) != hipSuccess)
        return false;
    if (hipEventRecord(s->ev[k], st) != hipSuccess) return false;
    s->launch_maxD[k] = maxD;
    s->inflight[k].swap(s->ready);
    s->ready.swap(rest);
    s->busy[k] = true;
    {
        std::lock_guard<std::mutex> g(s->mu);
        ++s->launches;
    }
    return true;
}

// Collects a finished launch (its compact states and positions are already on
// the host):
// completed swarms return their result and memory; the others become ready.
bool collect(pso_server *s, int k)
{
    if (*s->h_err[k]) return false; // parts of a swarm timed out waiting for each other
    const int n = (int)s->inflight[k].size();
    const int maxD = s->launch_maxD[k];
    std::vector<int> done_j;
    for (int j = 0; j < n; ++j) {
        const int slot = s->inflight[k][j];
        Req *r = s->slot_req[slot];
        r->res = s->h_out[k][j];
        const long long ran = r->res.iters - r->prev_iters;
        if (ran > 0 && r->res.ticks > 0) {
            const double us = double(r->res.ticks) / s->ticks_per_us / double(ran);
            r->us_per_iter = r->us_per_iter > 0.0 ? 0.5 * (r->us_per_iter + us) : us;
        }
        r->prev_iters = r->res.iters;
        if (r->res.stop || r->res.iters >= r->d.max_iter)
            done_j.push_back(j);
        else if (r->drop_code.load())
            drop_slot(s, slot); // cancelled or past its deadline, not finished by this launch
        else
            s->ready.push_back(slot);
    }
    {
        std::lock_guard<std::mutex> g(s->mu);
        const auto now = s->now();
        for (int j : done_j) {
            const int slot = s->inflight[k][j];
            Req *r = s->slot_req[slot];
            r->gpos.assign(s->h_opos[k] + (size_t)j * maxD, s->h_opos[k] + (size_t)j * maxD + r->d.D);
            r->t_done = now;
            r->status = PSO_OK;
            s->latencies.push_back(ms_since(r->t_submit, now));
            ++s->completed;
            s->arena.release(r->off);
            s->slot_req[slot] = nullptr;
            s->free_slots.push_back(slot);
        }
        if (!done_j.empty()) s->cv.notify_all();
    }
    s->inflight[k].clear();
    s->busy[k] = false;
    return true;
}

void server_pass_loop(pso_server *s);

// The scheduler thread: a failure inside it (a host allocation that throws)
// stops the server as a device error does -- submit and poll then report
// it -- instead of ending the process.
void server_loop(pso_server *s)
{
    try {
        server_pass_loop(s);
    } catch (...) {
        s->device_error.store(1);
        std::lock_guard<std::mutex> g(s->mu);
        s->cv.notify_all();
    }
}

void server_pass_loop(pso_server *s)
{
    while (!s->quit.load()) {
        bool progressed = false;
        // admission
        {
            std::vector<std::pair<uint64_t, size_t>> admitted;
            std::vector<uint64_t> rejected;
            std::lock_guard<std::mutex> g(s->mu);
            s->adm.admit(&admitted, &rejected, s->free_slots.size());
            for (uint64_t t : rejected) {
                Req *r = s->reqs[t].get();
                r->status = PSO_ENOMEM;
                r->t_done = s->now();
                ++s->rejected;
                progressed = true;
            }
            for (auto &ad : admitted) {
                Req *r = s->reqs[ad.first].get();
                r->off = ad.second;
                r->slot = s->free_slots.back();
                s->free_slots.pop_back();
                s->slot_req[r->slot] = r;
                s->h_items[r->slot] = make_item(s, *r);
                s->h_state[r->slot] = pso::BatchResult{pso::NO_KEY, 0, 0, 0u, 0u};
                s->fresh.push_back(r->slot);
                s->pending_upload[r->slot] = 1;
                if (r->parts > 1) s->fresh_gang.push_back(r->slot);
                s->ready.push_back(r->slot);
                progressed = true;
            }
            s->peak_used = std::max(s->peak_used, s->arena.used());
            if (!rejected.empty()) s->cv.notify_all();
            if (expire_deadlines(s)) progressed = true;
        }
        // admitted requests cancelled or past their deadline and not in
        // flight leave now; those in flight leave when their launch ends
        for (size_t j = 0; j < s->ready.size();) {
            const int slot = s->ready[j];
            if (s->slot_req[slot]->drop_code.load()) {
                s->ready[j] = s->ready.back();
                s->ready.pop_back();
                drop_slot(s, slot);
                progressed = true;
            } else {
                ++j;
            }
        }
        // collect finished launches, then launch on free streams
        for (int k = 0; k < STREAMS; ++k) {
            if (s->busy[k]) {
                const hipError_t q = hipEventQuery(s->ev[k]);
                if (q == hipSuccess) {
                    if (!collect(s, k)) s->device_error.store(1);
                    progressed = true;
                } else if (q != hipErrorNotReady) {
                    s->device_error.store(1);
                }
            }
        }
        for (int k = 0; k < STREAMS; ++k) {
            if (!s->busy[k] && !s->ready.empty()) {
                if (!launch_ready(s, k)) s->device_error.store(1);
                progressed = true;
            }
        }
        if (s->device_error.load()) {
            std::lock_guard<std::mutex> g(s->mu);
            s->cv.notify_all();
            break;
        }
        if (!progressed) {
            std::unique_lock<std::mutex> lk(s->mu);
            s->cv.wait_for(lk, std::chrono::microseconds(50));
        }
    }
}

} // namespace

extern "C" {

int pso_server_create(size_t mem_budget, int64_t chunk_updates, pso_server **out)
{
    return pso::guarded([&]() -> int {
        if (!out) return pso_internal_fail(PSO_EINVAL, "out is NULL");
        *out = nullptr;
        if (mem_budget < 4096) return pso_internal_fail(PSO_EINVAL, "mem_budget too small");
        pso_server *s = new (std::nothrow) pso_server();
        if (!s) return pso_internal_fail(PSO_ENOMEM, "host allocation failed");
        s->budget = mem_budget;
        s->chunk = chunk_updates > 0 ? chunk_updates : (1LL << 40);
        if (const char *env = getenv("PSO_SERVER_SLICE_US")) { // tuning override
            const double v = atof(env);
            if (v > 0.0) s->slice_us = v;
        }
        if (const char *env = getenv("PSO_SERVER_LAUNCH_WAVES")) { // tuning override
            const int v = atoi(env);
            if (v > 0) s->launch_waves = v;
        }
        s->arena = pso::Arena(mem_budget);
        // at most one slot per 64 KiB of budget, within [64, 65536]
        s->max_slots = (int)std::min<size_t>(65536, std::max<size_t>(64, mem_budget / 65536));
        // A multi-part swarm's parts meet every iteration, so they must all be
        // resident at once: a swarm has at most half the co-resident
        // workgroups as parts, and a streamed launch takes half of them.  A
        // staged launch (one 1024-lane workgroup per compute unit, whatever
        // its swarms) takes all of them (PSO_SERVER_GRID=half: half), so
        // while one launch drains, the other's workgroups take the compute
        // units it leaves (9.4k against 8.5k requests/s at 10 000/s).  Two
        // staged launches cannot wait on each other: in a launch only the
        // swarm whose parts are being dequeued can wait on workgroups not yet
        // resident, and only while every resident workgroup of that launch
        // holds one of its parts; both launches stuck needs more parts in the
        // two swarms than there are compute units, but each has at most half.
        int capacity = 0;
        if (pso::batch_capacity(MAX_SERVER_D, pso::DEFAULT_BATCH_SHAPE.lanes, &capacity) != hipSuccess || capacity < 2) {
            server_free(s);
            return pso_internal_fail(PSO_EDEVICE, "device query failed");
        }
        const char *genv = getenv("PSO_SERVER_GRID");
        const int share = (genv && !strcmp(genv, "half")) ? STREAMS : 1;
        s->grid_cap = capacity / STREAMS;
        {
            const char *env = getenv("PSO_SERVER_STAGED");
            int cap_staged = 0;
            if (!(env && !strcmp(env, "0")) &&
                pso::batch_capacity(SERVER_STAGE_MAX_D, SERVER_STAGE_LANES, &cap_staged, SERVER_STAGE_KIB) == hipSuccess &&
                cap_staged >= STREAMS) {
                s->grid_cap_staged = cap_staged / STREAMS;
                s->launch_cap_staged = cap_staged / share;
            }
        }
        {
            int dev = 0, khz = 0;
            if (hipGetDevice(&dev) == hipSuccess &&
                hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) == hipSuccess && khz > 0)
                s->ticks_per_us = khz / 1000.0;
        }
        bool ok = hipMalloc(&s->base, mem_budget) == hipSuccess &&
                  hipMalloc(&s->d_items, sizeof(pso::BatchItem) * s->max_slots) == hipSuccess &&
                  hipMalloc(&s->d_state, sizeof(pso::BatchResult) * s->max_slots) == hipSuccess &&
                  hipMalloc(&s->d_err, sizeof(unsigned int)) == hipSuccess &&
                  hipMemset(s->d_err, 0, sizeof(unsigned int)) == hipSuccess &&
                  hipHostMalloc(reinterpret_cast<void **>(&s->h_items), sizeof(pso::BatchItem) * s->max_slots,
                                hipHostMallocDefault) == hipSuccess &&
                  hipHostMalloc(reinterpret_cast<void **>(&s->h_state), sizeof(pso::BatchResult) * s->max_slots,
                                hipHostMallocDefault) == hipSuccess;
        for (int k = 0; ok && k < STREAMS; ++k) {
            ok = hipMalloc(&s->d_entries[k], sizeof(pso::BatchEntry) * s->max_slots) == hipSuccess &&
                 hipMalloc(&s->d_next[k], sizeof(unsigned int)) == hipSuccess &&
                 hipMalloc(&s->d_out[k], sizeof(pso::BatchResult) * s->max_slots) == hipSuccess &&
                 hipHostMalloc(reinterpret_cast<void **>(&s->h_out[k]), sizeof(pso::BatchResult) * s->max_slots,
                               hipHostMallocDefault) == hipSuccess &&
                 hipHostMalloc(reinterpret_cast<void **>(&s->h_entries[k]), sizeof(pso::BatchEntry) * s->max_slots,
                               hipHostMallocDefault) == hipSuccess &&
                 hipHostMalloc(reinterpret_cast<void **>(&s->h_err[k]), sizeof(unsigned int), hipHostMallocDefault) ==
                     hipSuccess &&
                 hipStreamCreateWithFlags(&s->st[k], hipStreamNonBlocking) == hipSuccess &&
                 hipEventCreateWithFlags(&s->ev[k], hipEventDisableTiming) == hipSuccess &&
                 hipMalloc(&s->d_up[k], sizeof(pso::UploadRec) * s->max_slots) == hipSuccess &&
                 hipHostMalloc(reinterpret_cast<void **>(&s->h_up[k]), sizeof(pso::UploadRec) * s->max_slots,
                               hipHostMallocDefault) == hipSuccess;
        }
        if (!ok) {
            server_free(s);
            return pso_internal_fail(PSO_ENOMEM, "device or pinned allocation for the server failed");
        }
        for (int k = 0; k < STREAMS; ++k) s->cap_entries[k] = (size_t)s->max_slots;
        s->slot_req.assign(s->max_slots, nullptr);
        s->pending_upload.assign(s->max_slots, 0);
        for (int k = s->max_slots - 1; k >= 0; --k) s->free_slots.push_back(k);
        try {
            s->th = std::thread(server_loop, s);
        } catch (...) {
            server_free(s);
            throw;
        }
        *out = s;
        return PSO_OK;
    });
}

int pso_server_submit(pso_server *s, const pso_desc *d, uint64_t *ticket)
{
    return pso::guarded([&]() -> int {
        if (!s || !d || !ticket) return pso_internal_fail(PSO_EINVAL, "NULL argument");
        int rc = pso_internal_check_desc(d);
        if (rc) return rc;
        if (s->device_error.load()) return pso_internal_fail(PSO_EDEVICE, "server stopped after a device error");
        auto r = std::make_unique<Req>();
        r->d = *d;
        r->shift.assign(d->D, 0.0f);
        if (d->shift) std::memcpy(r->shift.data(), d->shift, sizeof(float) * d->D);
        r->d.shift = nullptr;
        r->t_submit = s->now();
        const uint32_t staged_parts =
            s->grid_cap_staged > 0 && d->D <= SERVER_STAGE_MAX_D
                ? pso::staged_parts((uint64_t)d->N, d->D, d->fitness_id, SERVER_STAGE_KIB, s->grid_cap_staged)
                : 0;
        r->staged = staged_parts > 0;
        r->parts = r->staged ? staged_parts : pso::parts_for((uint64_t)d->N, d->D, s->grid_cap, pso::DEFAULT_BATCH_SHAPE);
        const size_t bytes = pso::layout_of((uint64_t)d->N, d->D, false).total + pso::gang_bytes(r->parts, d->D);
        std::lock_guard<std::mutex> g(s->mu);
        // the request is listed before it is queued, and a failure to queue
        // it unlists it, so the scheduler never admits an unlisted ticket
        const uint64_t t = s->next_ticket;
        r->ticket = t;
        auto ins = s->reqs.emplace(t, std::move(r));
        try {
            s->adm.push(pso::Pending{t, bytes});
        } catch (...) {
            s->reqs.erase(ins.first);
            throw;
        }
        ++s->next_ticket;
        *ticket = t;
        ++s->submitted;
        s->cv.notify_all();
        return PSO_OK;
    });
}

int pso_server_poll(pso_server *s, uint64_t ticket, pso_result *result, double *latency_ms)
{
    return pso::guarded([&]() -> int {
        if (!s) return pso_internal_fail(PSO_EINVAL, "server is NULL");
        std::lock_guard<std::mutex> g(s->mu);
        auto it = s->reqs.find(ticket);
        if (it == s->reqs.end()) return pso_internal_fail(PSO_EINVAL, "unknown ticket %llu", (unsigned long long)ticket);
        Req *r = it->second.get();
        if (r->status == PSO_EAGAIN) {
            if (s->device_error.load()) return pso_internal_fail(PSO_EDEVICE, "server stopped after a device error");
            return PSO_EAGAIN;
        }
        const int status = r->status;
        if (result) {
            result->status = status;
            if (status == PSO_OK) {
                result->gbest_value = pso::key_fitness(r->res.gkey);
                result->gbest_iter = r->res.giter;
                result->iters = r->res.iters;
                if (result->gbest_pos) std::memcpy(result->gbest_pos, r->gpos.data(), sizeof(float) * r->d.D);
            }
        }
        if (latency_ms) *latency_ms = ms_since(r->t_submit, r->t_done);
        s->reqs.erase(it);
        if (status == PSO_ENOMEM)
            return pso_internal_fail(status, "request %llu needs more device memory than the budget",
                                     (unsigned long long)ticket);
        if (status == PSO_ECANCELED) return pso_internal_fail(status, "request %llu was cancelled", (unsigned long long)ticket);
        if (status == PSO_ETIMEDOUT)
            return pso_internal_fail(status, "request %llu passed its deadline", (unsigned long long)ticket);
        return PSO_OK;
    });
}

int pso_server_cancel(pso_server *s, uint64_t ticket)
{
    return pso::guarded([&]() -> int {
        if (!s) return pso_internal_fail(PSO_EINVAL, "server is NULL");
        std::lock_guard<std::mutex> g(s->mu);
        auto it = s->reqs.find(ticket);
        if (it == s->reqs.end()) return pso_internal_fail(PSO_EINVAL, "unknown ticket %llu", (unsigned long long)ticket);
        Req *r = it->second.get();
        if (r->status != PSO_EAGAIN)
            return pso_internal_fail(PSO_ESTATE, "request %llu has already finished", (unsigned long long)ticket);
        if (r->slot < 0 && s->adm.cancel(ticket)) { // still queued: leaves now
            r->status = PSO_ECANCELED;
            r->t_done = s->now();
            ++s->cancelled;
        } else { // admitted: the scheduler drops it
            int none = 0;
            r->drop_code.compare_exchange_strong(none, PSO_ECANCELED);
        }
        s->cv.notify_all();
        return PSO_OK;
    });
}

int pso_server_set_deadline(pso_server *s, uint64_t ticket, double timeout_ms)
{
    return pso::guarded([&]() -> int {
        if (!s) return pso_internal_fail(PSO_EINVAL, "server is NULL");
        if (!(timeout_ms > 0.0) || !(timeout_ms < 1e12))
            return pso_internal_fail(PSO_EINVAL, "timeout_ms must be positive and finite");
        std::lock_guard<std::mutex> g(s->mu);
        auto it = s->reqs.find(ticket);
        if (it == s->reqs.end()) return pso_internal_fail(PSO_EINVAL, "unknown ticket %llu", (unsigned long long)ticket);
        Req *r = it->second.get();
        if (r->status != PSO_EAGAIN)
            return pso_internal_fail(PSO_ESTATE, "request %llu has already finished", (unsigned long long)ticket);
        const auto at = r->t_submit + std::chrono::duration_cast<Clock::duration>(
                                          std::chrono::duration<double, std::milli>(timeout_ms));
        s->deadlines.emplace(at, ticket);
        s->cv.notify_all();
        return PSO_OK;
    });
}

int pso_server_stats(pso_server *s, pso_server_counters *out)
{
    return pso::guarded([&]() -> int {
        if (!s || !out) return pso_internal_fail(PSO_EINVAL, "NULL argument");
        std::lock_guard<std::mutex> g(s->mu);
        out->submitted = s->submitted;
        out->completed = s->completed;
        out->rejected = s->rejected;
        out->cancelled = s->cancelled;
        out->timed_out = s->timed_out;
        out->queued = s->adm.queued();
        out->launches = s->launches;
        out->mem_budget = s->budget;
        out->mem_used = s->arena.used();
        out->mem_peak = s->peak_used;
        std::vector<double> l = s->latencies;
        out->p50_ms = out->p99_ms = out->max_ms = 0.0;
        if (!l.empty()) {
            std::sort(l.begin(), l.end());
            auto q = [&](double f) { return l[std::min(l.size() - 1, (size_t)(f * (l.size() - 1) + 0.5))]; };
            out->p50_ms = q(0.50);
            out->p99_ms = q(0.99);
            out->max_ms = l.back();
        }
        return PSO_OK;
    });
}

int pso_server_destroy(pso_server *s)
{
    return pso::guarded([&]() -> int {
        if (!s) return pso_internal_fail(PSO_EINVAL, "server is NULL");
        s->quit.store(true);
        {
            std::lock_guard<std::mutex> g(s->mu);
            s->cv.notify_all();
        }
        if (s->th.joinable()) s->th.join();
        server_free(s);
        return PSO_OK;
    });
}

} // extern "C"

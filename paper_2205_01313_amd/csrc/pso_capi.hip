// pso_capi.hip -- host runtime behind include/pso.h: argument checks, device
// memory and stream ownership, run loop with a device-side stop rule, and
// state transfer.  Every entry point returns a status and never aborts.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "pso.h"
#include "pso_block.hpp"
#include "pso_guard.hpp"
#include "pso_device.hpp"
#include "pso_kernels.hpp"

using pso::Ctrl;
using pso::Layout;
using pso::SwarmArgs;

namespace {

thread_local char g_err[512] = "";

int fail(int code, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return code;
}

#define HIP_TRY(expr)                                                                           \
    do {                                                                                        \
        hipError_t e_ = (expr);                                                                 \
        if (e_ != hipSuccess) return fail(PSO_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

constexpr int32_t MAX_D = 4096;
// Batch limits, checked before a batch allocates anything: swarms per batch,
// work-queue entries (parts) per batch -- a 32-bit count on the device -- and
// device bytes per batch (far above any device's memory, so only arithmetic
// overflow is excluded here; hipMalloc reports the real limit).
constexpr int64_t MAX_BATCH_SWARMS = int64_t(1) << 24;
constexpr uint64_t MAX_BATCH_ENTRIES = (uint64_t(1) << 32) - 1;
constexpr uint64_t MAX_BATCH_BYTES = uint64_t(1) << 52;

// A synchronous swarm of at most this many particle-dimensions whose state
// fits one workgroup's LDS runs its pso_run iterations in one workgroup (one
// launch for the whole run) instead of one grid launch per iteration.  A
// workgroup reading the state from device memory every iteration loses to
// the launches wherever the state does not fit (us per iteration, one
// workgroup / launches: Cubic 1D N = 16 384: 19.0 / 5.3, N = 8192: 9.7 /
// 5.2; Rastrigin D = 8, N = 2048: 13.7 / 10.7; D = 128, N = 512: 99.8 /
// 14.0; Ackley D = 32, N = 1024: 26.2 / 9.8), so it runs only under
// PSO_BLOCK_STAGED=0 (tests compare the two one-workgroup kernels).
#ifndef PSO_BLOCK_RUN_MAX_ND
#define PSO_BLOCK_RUN_MAX_ND 65536
#endif
constexpr int64_t BLOCK_RUN_MAX_ND = PSO_BLOCK_RUN_MAX_ND;

// pso_run enqueues its per-iteration step launches as replays of a graph of
// this many launches (captured once per swarm, variant and step path), the
// remainder directly: a graph's launches reach the device as one submission.
// PSO_RUN_GRAPH=0 in the environment launches every step directly.
constexpr int64_t RUN_GRAPH_STEPS = 8;

} // namespace

// Shared with pso_server.hip (C++ linkage, not part of the C ABI).
int pso_internal_fail(int code, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return code;
}

struct pso_swarm {
    int fitness = 0;
    int variant = PSO_SYNC;
    int64_t max_lead = 8; // PSO_PERSISTENT staleness bound
    uint64_t N = 0;
    int32_t D = 0;
    Layout L{};
    SwarmArgs args{};
    void *ws = nullptr;
    bool owns_ws = false;
    hipStream_t stream = nullptr;
    bool owns_stream = false;
    int device = 0;
    Ctrl *host_ctrl = nullptr; // pinned mirror of the control block
    float *host_gpos = nullptr; // pinned, D floats
    // RUN_GRAPH_STEPS step launches captured into a graph once (for the
    // variant and step path they were captured with) and replayed by pso_run
    hipGraph_t steps_graph = nullptr;
    hipGraphExec_t steps_exec = nullptr;
    int steps_key = -1;
    // the gang run's meeting words (allocated at its first run)
    unsigned long long *gang_words = nullptr;
    size_t gang_words_n = 0;
};

namespace {

int check_params(int fitness_id, int64_t N, int32_t D, const float bounds[2], float w, float c1, float c2,
                 float vmax)
{
    if (fitness_id < PSO_SPHERE || fitness_id > PSO_CUBIC) return fail(PSO_EINVAL, "unknown fitness_id %d", fitness_id);
    if (N < 1 || N > (int64_t(1) << 30)) return fail(PSO_EINVAL, "N=%lld outside [1, 2^30]", (long long)N);
    if (D < 1 || D > MAX_D) return fail(PSO_EINVAL, "D=%d outside [1, %d]", D, MAX_D);
    if (fitness_id == PSO_ROSENBROCK && D < 2) return fail(PSO_EINVAL, "Rosenbrock needs D >= 2");
    if (!bounds) return fail(PSO_EINVAL, "bounds is NULL");
    if (!std::isfinite(bounds[0]) || !std::isfinite(bounds[1]) || !(bounds[0] < bounds[1]))
        return fail(PSO_EINVAL, "bounds must be finite with bounds[0] < bounds[1]");
    if (!std::isfinite(w) || !std::isfinite(c1) || !std::isfinite(c2))
        return fail(PSO_EINVAL, "w, c1, c2 must be finite");
    if (!std::isfinite(vmax) || !(vmax > 0.0f)) return fail(PSO_EINVAL, "vmax must be finite and > 0");
    if (!std::isfinite(bounds[1] - bounds[0])) return fail(PSO_EINVAL, "bounds span overflows");
    return PSO_OK;
}

} // namespace

// Checks one request / batch descriptor (pso_create's rules plus the run
// limits); shared with pso_server.hip.
int pso_internal_check_desc(const pso_desc *d)
{
    int rc = check_params(d->fitness_id, d->N, d->D, d->bounds, d->w, d->c1, d->c2, d->vmax);
    if (rc) return rc;
    if (d->max_iter < 0 || d->max_iter >= (int64_t(1) << 32) - 1) return fail(PSO_EINVAL, "max_iter out of range");
    if (std::isnan(d->tol) || std::isnan(d->f_star)) return fail(PSO_EINVAL, "tol and f_star must not be NaN");
    if (d->shift)
        for (int k = 0; k < d->D; ++k)
            if (!std::isfinite(d->shift[k])) return fail(PSO_EINVAL, "shift[%d] is not finite", k);
    return PSO_OK;
}

namespace {

int enqueue_init(pso_swarm *s)
{
    HIP_TRY(pso::launch_reset(s->args, s->stream));
    HIP_TRY(pso::launch_init(s->fitness, s->args, s->stream));
    return PSO_OK;
}

int create_common(int fitness_id, int64_t N, int32_t D, const float bounds[2], float w, float c1, float c2,
                  float vmax, uint64_t seed, void *ws, size_t bytes, bool own, void *stream, pso_swarm **out)
{
    if (!out) return fail(PSO_EINVAL, "out is NULL");
    *out = nullptr;
    int rc = check_params(fitness_id, N, D, bounds, w, c1, c2, vmax);
    if (rc) return rc;
    pso_swarm *s = new (std::nothrow) pso_swarm();
    if (!s) return fail(PSO_ENOMEM, "host allocation failed");
    s->fitness = fitness_id;
    s->N = (uint64_t)N;
    s->D = D;
    s->L = pso::layout_of(s->N, D);
    auto cleanup = [&](int code) {
        if (s->owns_ws && s->ws) (void)hipFree(s->ws);
        if (s->owns_stream && s->stream) (void)hipStreamDestroy(s->stream);
        if (s->host_ctrl) (void)hipHostFree(s->host_ctrl);
        if (s->host_gpos) (void)hipHostFree(s->host_gpos);
        delete s;
        return code;
    };
    if (hipGetDevice(&s->device) != hipSuccess) return cleanup(fail(PSO_EDEVICE, "no HIP device"));
    if (own) {
        if (hipMalloc(&s->ws, s->L.total) != hipSuccess)
            return cleanup(fail(PSO_ENOMEM, "hipMalloc of %zu bytes failed", s->L.total));
        s->owns_ws = true;
        if (hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking) != hipSuccess)
            return cleanup(fail(PSO_EDEVICE, "hipStreamCreate failed"));
        s->owns_stream = true;
    } else {
        if (!ws) return cleanup(fail(PSO_EINVAL, "dev_workspace is NULL"));
        if (reinterpret_cast<uintptr_t>(ws) & 255) return cleanup(fail(PSO_EINVAL, "dev_workspace not 256-byte aligned"));
        if (bytes < s->L.total)
            return cleanup(fail(PSO_EINVAL, "workspace of %zu bytes < %zu needed", bytes, s->L.total));
        s->ws = ws;
        s->stream = static_cast<hipStream_t>(stream);
    }
    if (hipHostMalloc(reinterpret_cast<void **>(&s->host_ctrl), sizeof(Ctrl), hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc(reinterpret_cast<void **>(&s->host_gpos), sizeof(float) * D, hipHostMallocDefault) != hipSuccess)
        return cleanup(fail(PSO_ENOMEM, "pinned host allocation failed"));
    s->args = pso::bind(s->ws, s->L, s->N, D);
    s->args.lo = bounds[0];
    s->args.hi = bounds[1];
    s->args.w = w;
    s->args.c1 = c1;
    s->args.c2 = c2;
    s->args.vmax = vmax;
    s->args.k0 = (uint32_t)seed;
    s->args.k1 = (uint32_t)(seed >> 32);
    // shift = 0
    std::vector<float> zero(D, 0.0f);
    if (hipMemcpyAsync(const_cast<float *>(s->args.shift), zero.data(), sizeof(float) * D, hipMemcpyHostToDevice,
                       s->stream) != hipSuccess)
        return cleanup(fail(PSO_EDEVICE, "shift upload failed"));
    rc = enqueue_init(s);
    if (rc) return cleanup(rc);
    if (hipStreamSynchronize(s->stream) != hipSuccess) return cleanup(fail(PSO_EDEVICE, "init failed"));
    *out = s;
    return PSO_OK;
}

int fetch_ctrl(pso_swarm *s, bool with_gpos)
{
    HIP_TRY(hipMemcpyAsync(s->host_ctrl, s->args.ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, s->stream));
    if (with_gpos)
        HIP_TRY(hipMemcpyAsync(s->host_gpos, s->args.gpos, sizeof(float) * s->D, hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
    if (s->host_ctrl->err) return fail(PSO_EDEVICE, "device error bits 0x%x", s->host_ctrl->err);
    return PSO_OK;
}

} // namespace

extern "C" {

const char *pso_last_error(void) { return g_err; }

size_t pso_workspace_bytes(int64_t N, int32_t D)
{
    if (N < 1 || N > (int64_t(1) << 30) || D < 1 || D > MAX_D) return 0;
    return pso::layout_of((uint64_t)N, D).total;
}

int pso_create(int fitness_id, int64_t N, int32_t D, const float bounds[2], float w, float c1, float c2, float vmax,
               uint64_t seed, pso_swarm **out)
{
    return pso::guarded([&]() -> int {
        return create_common(fitness_id, N, D, bounds, w, c1, c2, vmax, seed, nullptr, 0, true, nullptr, out);
    });
}

int pso_create_in(int fitness_id, int64_t N, int32_t D, const float bounds[2], float w, float c1, float c2,
                  float vmax, uint64_t seed, void *dev_workspace, size_t bytes, void *hip_stream, pso_swarm **out)
{
    return pso::guarded([&]() -> int {
        return create_common(fitness_id, N, D, bounds, w, c1, c2, vmax, seed, dev_workspace, bytes, false, hip_stream,
                             out);
    });
}

int pso_set_shift(pso_swarm *s, const float *shift_host)
{
    return pso::guarded([&]() -> int {
        if (!s) return fail(PSO_EINVAL, "swarm is NULL");
        std::vector<float> h(s->D, 0.0f);
        if (shift_host) {
            for (int d = 0; d < s->D; ++d) {
                if (!std::isfinite(shift_host[d])) return fail(PSO_EINVAL, "shift[%d] is not finite", d);
                h[d] = shift_host[d];
            }
        }
        HIP_TRY(hipMemcpyAsync(const_cast<float *>(s->args.shift), h.data(), sizeof(float) * s->D,
                               hipMemcpyHostToDevice, s->stream));
        HIP_TRY(hipStreamSynchronize(s->stream)); // h is a stack buffer
        return enqueue_init(s);
    });
}

int pso_set_variant(pso_swarm *s, int variant)
{
    return pso::guarded([&]() -> int {
        if (!s) return fail(PSO_EINVAL, "swarm is NULL");
        if (variant < PSO_SYNC || variant > PSO_PERSISTENT) return fail(PSO_EINVAL, "unknown variant %d", variant);
        s->variant = variant;
        return PSO_OK;
    });
}

int pso_set_max_lead(pso_swarm *s, int64_t max_lead)
{
    return pso::guarded([&]() -> int {
        if (!s) return fail(PSO_EINVAL, "swarm is NULL");
        if (max_lead < 0) return fail(PSO_EINVAL, "max_lead < 0");
        s->max_lead = max_lead;
        return PSO_OK;
    });
}

int pso_reset(pso_swarm *s)
{
    return pso::guarded([&]() -> int {
        if (!s) return fail(PSO_EINVAL, "swarm is NULL");
        return enqueue_init(s);
    });
}

namespace {

void drop_steps_graph(pso_swarm *s)
{
    if (s->steps_exec) (void)hipGraphExecDestroy(s->steps_exec);
    if (s->steps_graph) (void)hipGraphDestroy(s->steps_graph);
    s->steps_exec = nullptr;
    s->steps_graph = nullptr;
    s->steps_key = -1;
}

// What a captured step launch depends on besides the swarm: its variant, the
// step path chosen from the environment (PSO_STEP_SPLIT, PSO_STEP_ONE,
// PSO_SPLIT_PHASES) and the asynchronous step's tiles per workgroup.
int steps_key_of(const pso_swarm *s)
{
    auto mode = [](const char *name) {
        const char *e = getenv(name);
        return e ? (atoi(e) == 0 ? 1 : 2) : 0;
    };
    const char *ph = getenv("PSO_SPLIT_PHASES");
    const int phases = ph ? std::min(std::max(atoi(ph), 0), 2) : 0;
    return (((s->variant * 3 + mode("PSO_STEP_SPLIT")) * 3 + mode("PSO_STEP_ONE")) * 3 + phases) * 65 +
           (int)pso::async_tiles_per_workgroup();
}

// Enqueues n step launches: replays of the captured graph of RUN_GRAPH_STEPS
// launches, then the rest directly.  The null stream cannot be captured; a
// swarm on it launches directly.
int enqueue_steps(pso_swarm *s, int64_t n)
{
    const char *env = getenv("PSO_RUN_GRAPH");
    const bool graphs = !(env && !strcmp(env, "0")) && s->stream != nullptr && n >= RUN_GRAPH_STEPS;
    if (graphs) {
        const int key = steps_key_of(s);
        if (s->steps_exec && s->steps_key != key) drop_steps_graph(s);
        if (!s->steps_exec) {
            HIP_TRY(hipStreamBeginCapture(s->stream, hipStreamCaptureModeThreadLocal));
            hipError_t le = hipSuccess;
            for (int64_t j = 0; j < RUN_GRAPH_STEPS && le == hipSuccess; ++j)
                le = pso::launch_step(s->fitness, s->variant, s->args, s->stream);
            hipGraph_t g = nullptr;
            const hipError_t ce = hipStreamEndCapture(s->stream, &g);
            if (le != hipSuccess || ce != hipSuccess) {
                if (g) (void)hipGraphDestroy(g);
                return fail(PSO_EDEVICE, "capturing the step launches failed: %s",
                            hipGetErrorString(le != hipSuccess ? le : ce));
            }
            s->steps_graph = g;
            if (hipGraphInstantiate(&s->steps_exec, g, nullptr, nullptr, 0) != hipSuccess) {
                drop_steps_graph(s);
                return fail(PSO_EDEVICE, "instantiating the step graph failed");
            }
            s->steps_key = key;
        }
        for (; n >= RUN_GRAPH_STEPS; n -= RUN_GRAPH_STEPS) HIP_TRY(hipGraphLaunch(s->steps_exec, s->stream));
    }
    for (int64_t j = 0; j < n; ++j) HIP_TRY(pso::launch_step(s->fitness, s->variant, s->args, s->stream));
    return PSO_OK;
}

// Persistent launches for T iterations (each clears its iteration counts).
int persistent_launch(pso_swarm *s, int64_t T)
{
    while (T > 0) {
        const uint32_t n = (uint32_t)std::min<int64_t>(T, int64_t(1) << 30);
        const uint32_t lead = (uint32_t)std::min<int64_t>(s->max_lead, int64_t(0xFFFFFFFF));
        HIP_TRY(pso::launch_persistent(s->fitness, s->args, n, lead, s->stream));
        T -= n;
    }
    return PSO_OK;
}

} // namespace

int pso_step(pso_swarm *s)
{
    return pso::guarded([&]() -> int {
        if (!s) return fail(PSO_EINVAL, "swarm is NULL");
        if (s->variant == PSO_PERSISTENT) return persistent_launch(s, 1);
        HIP_TRY(pso::launch_step(s->fitness, s->variant, s->args, s->stream));
        return PSO_OK;
    });
}

int pso_run(pso_swarm *s, int64_t max_iter, float tol, float f_star, float *gbest_value, float *gbest_pos_host,
            int64_t *gbest_iter, int64_t *iters_done)
{
    return pso::guarded([&]() -> int {
        if (!s) return fail(PSO_EINVAL, "swarm is NULL");
        if (max_iter < 0) return fail(PSO_EINVAL, "max_iter < 0");
        if (std::isnan(tol) || std::isnan(f_star)) return fail(PSO_EINVAL, "tol and f_star must not be NaN");
        HIP_TRY(pso::launch_arm(s->args, tol, f_star, s->stream));
        bool block_path = s->variant == PSO_SYNC && int64_t(s->N) * s->D <= BLOCK_RUN_MAX_ND &&
                          pso::block_run_suits(s->fitness, s->args);
        uint32_t gang_parts = s->variant == PSO_SYNC ? pso::gang_run_parts(s->fitness, s->args) : 0u;
        if (block_path) {
            // a gang of 8 or more parts meets in about 2 us per iteration and
            // overtakes one workgroup from N = 4096 or N*D = 8192 (Cubic 1D
            // N = 4096: 2.34 against 2.85 us; Rastrigin D = 4, N = 2048: 3.38
            // against 5.71; below, one workgroup: D = 2, N = 2048 2.00 against 2.25)
            const bool gang_first = gang_parts >= 8 && (s->N >= 4096 || int64_t(s->N) * s->D >= 8192);
            if (gang_first)
                block_path = false;
            else
                gang_parts = 0;
        }
        if (s->variant == PSO_PERSISTENT) {
            int rc = persistent_launch(s, max_iter);
            if (rc) return rc;
        } else if (block_path) {
            if (max_iter > 0) HIP_TRY(pso::launch_block_run(s->fitness, s->args, max_iter, s->stream));
        } else if (gang_parts > 0) {
            const size_t n = pso::gang_run_words(gang_parts, s->D);
            if (n > s->gang_words_n) {
                HIP_TRY(hipStreamSynchronize(s->stream));
                if (s->gang_words) (void)hipFree(s->gang_words);
                s->gang_words = nullptr;
                s->gang_words_n = 0;
                if (hipMalloc(reinterpret_cast<void **>(&s->gang_words), n * sizeof(unsigned long long)) != hipSuccess)
                    return fail(PSO_ENOMEM, "gang meeting words: device allocation failed");
                s->gang_words_n = n;
            }
            if (max_iter > 0)
                HIP_TRY(pso::launch_gang_run(s->fitness, s->args, max_iter, gang_parts, s->gang_words, s->stream));
        } else if (tol > 0.0f) {
            // Chunks of iterations with one chunk always queued ahead; the
            // device skips iterations once the stop rule holds, and the host
            // stops enqueueing when it sees the flag.
            const double work = double(s->N) * double(s->D);
            const int64_t chunk =
                std::max<int64_t>(8, std::min<int64_t>(256, int64_t((1 << 26) / work))) / RUN_GRAPH_STEPS *
                RUN_GRAPH_STEPS;
            hipEvent_t ev[2];
            HIP_TRY(hipEventCreateWithFlags(&ev[0], hipEventDisableTiming));
            if (hipEventCreateWithFlags(&ev[1], hipEventDisableTiming) != hipSuccess) {
                (void)hipEventDestroy(ev[0]);
                return fail(PSO_EDEVICE, "hipEventCreate failed");
            }
            unsigned int *flags = nullptr;
            if (hipHostMalloc(reinterpret_cast<void **>(&flags), 2 * sizeof(unsigned int), hipHostMallocDefault) !=
                hipSuccess) {
                (void)hipEventDestroy(ev[0]);
                (void)hipEventDestroy(ev[1]);
                return fail(PSO_ENOMEM, "pinned host allocation failed");
            }
            int rc = PSO_OK;
            int64_t done = 0;
            int k = 0, inflight = 0;
            while (done < max_iter && rc == PSO_OK) {
                const int64_t n = std::min(chunk, max_iter - done);
                rc = enqueue_steps(s, n);
                done += n;
                if (hipMemcpyAsync(&flags[k], &s->args.ctrl->stop, sizeof(unsigned int), hipMemcpyDeviceToHost,
                                   s->stream) != hipSuccess ||
                    hipEventRecord(ev[k], s->stream) != hipSuccess)
                    rc = fail(PSO_EDEVICE, "stop flag copy failed");
                ++inflight;
                k ^= 1;
                if (inflight == 2) { // wait for the older chunk
                    if (hipEventSynchronize(ev[k]) != hipSuccess) rc = fail(PSO_EDEVICE, "event wait failed");
                    --inflight;
                    if (flags[k]) break;
                }
            }
            (void)hipStreamSynchronize(s->stream);
            (void)hipHostFree(flags);
            (void)hipEventDestroy(ev[0]);
            (void)hipEventDestroy(ev[1]);
            if (rc) return rc;
        } else {
            int rc = enqueue_steps(s, max_iter);
            if (rc) return rc;
        }
        int rc = fetch_ctrl(s, true);
        if (rc) return rc;
        const Ctrl &c = *s->host_ctrl;
        if (gbest_value) *gbest_value = pso::key_fitness(c.gkey_prev);
        if (gbest_pos_host) std::memcpy(gbest_pos_host, s->host_gpos, sizeof(float) * s->D);
        if (gbest_iter) *gbest_iter = c.giter;
        if (iters_done) *iters_done = c.t - c.t_run0;
        return PSO_OK;
    });
}

int pso_get_best(pso_swarm *s, float *gbest_value, float *gbest_pos_host, int64_t *gbest_iter,
                 int64_t *iters_completed)
{
    return pso::guarded([&]() -> int {
        if (!s) return fail(PSO_EINVAL, "swarm is NULL");
        int rc = fetch_ctrl(s, true);
        if (rc) return rc;
        const Ctrl &c = *s->host_ctrl;
        if (gbest_value) *gbest_value = pso::key_fitness(c.gkey_prev);
        if (gbest_pos_host) std::memcpy(gbest_pos_host, s->host_gpos, sizeof(float) * s->D);
        if (gbest_iter) *gbest_iter = c.giter;
        if (iters_completed) *iters_completed = c.t;
        return PSO_OK;
    });
}

int pso_get_history(pso_swarm *s, int64_t t0, int64_t count, uint64_t *keys_host)
{
    return pso::guarded([&]() -> int {
        if (!s) return fail(PSO_EINVAL, "swarm is NULL");
        if (count < 0 || t0 < 0 || (count > 0 && !keys_host)) return fail(PSO_EINVAL, "bad history range");
        int rc = fetch_ctrl(s, false);
        if (rc) return rc;
        const int64_t t = s->host_ctrl->t;
        if (t0 + count > t + 1) return fail(PSO_ESTATE, "iterations %lld.. not run yet", (long long)(t + 1));
        if (count > 0 && t0 < t + 1 - pso::HIST_CAP) return fail(PSO_ESTATE, "iteration %lld left the history", (long long)t0);
        std::vector<unsigned long long> ring(pso::HIST_CAP);
        HIP_TRY(hipMemcpy(ring.data(), s->args.hist, sizeof(unsigned long long) * pso::HIST_CAP, hipMemcpyDeviceToHost));
        for (int64_t j = 0; j < count; ++j) keys_host[j] = ring[(t0 + j) & (pso::HIST_CAP - 1)];
        return PSO_OK;
    });
}

int pso_get_state(pso_swarm *s, float *x_host, float *v_host, float *p_host, float *pf_host, uint64_t *gbest_key,
                  float *gbest_pos_host, int64_t *gbest_iter, int64_t *iters_completed)
{
    return pso::guarded([&]() -> int {
        if (!s) return fail(PSO_EINVAL, "swarm is NULL");
        HIP_TRY(pso::launch_flush(s->args, s->stream));
        HIP_TRY(hipStreamSynchronize(s->stream));
        // device rows have pitch Np, host rows are dense (pitch N)
        const size_t row = sizeof(float) * s->N, pitch = sizeof(float) * s->L.Np;
        if (x_host) HIP_TRY(hipMemcpy2D(x_host, row, s->args.x, pitch, row, s->D, hipMemcpyDeviceToHost));
        if (v_host) HIP_TRY(hipMemcpy2D(v_host, row, s->args.v, pitch, row, s->D, hipMemcpyDeviceToHost));
        if (p_host) HIP_TRY(hipMemcpy2D(p_host, row, s->args.p, pitch, row, s->D, hipMemcpyDeviceToHost));
        if (pf_host) HIP_TRY(hipMemcpy(pf_host, s->args.pf, sizeof(float) * s->N, hipMemcpyDeviceToHost));
        int rc = fetch_ctrl(s, true);
        if (rc) return rc;
        const Ctrl &c = *s->host_ctrl;
        if (gbest_key) *gbest_key = c.gkey_prev;
        if (gbest_pos_host) std::memcpy(gbest_pos_host, s->host_gpos, sizeof(float) * s->D);
        if (gbest_iter) *gbest_iter = c.giter;
        if (iters_completed) *iters_completed = c.t;
        return PSO_OK;
    });
}

int pso_set_state(pso_swarm *s, const float *x_host, const float *v_host, const float *p_host, const float *pf_host,
                  uint64_t gbest_key, const float *gbest_pos_host, int64_t gbest_iter, int64_t iters_completed)
{
    return pso::guarded([&]() -> int {
        if (!s) return fail(PSO_EINVAL, "swarm is NULL");
        if (!x_host || !v_host || !p_host || !pf_host || !gbest_pos_host) return fail(PSO_EINVAL, "state buffer is NULL");
        if (iters_completed < 0 || iters_completed >= (int64_t(1) << 32) - 1 || gbest_iter < 0 || gbest_iter > iters_completed)
            return fail(PSO_EINVAL, "bad iteration counters");
        if ((gbest_key & 0xFFFFFFFFull) >= s->N) return fail(PSO_EINVAL, "gbest index out of range");
        HIP_TRY(hipStreamSynchronize(s->stream));
        const size_t row = sizeof(float) * s->N, pitch = sizeof(float) * s->L.Np;
        HIP_TRY(hipMemcpy2D(s->args.x, pitch, x_host, row, row, s->D, hipMemcpyHostToDevice));
        HIP_TRY(hipMemcpy2D(s->args.v, pitch, v_host, row, row, s->D, hipMemcpyHostToDevice));
        HIP_TRY(hipMemcpy2D(s->args.p, pitch, p_host, row, row, s->D, hipMemcpyHostToDevice));
        HIP_TRY(hipMemcpy(s->args.pf, pf_host, sizeof(float) * s->N, hipMemcpyHostToDevice));
        HIP_TRY(hipMemcpy(s->args.gpos, gbest_pos_host, sizeof(float) * s->D, hipMemcpyHostToDevice));
        Ctrl c;
        std::memset(&c, 0, sizeof c);
        c.gkey = gbest_key;
        c.gkey_prev = gbest_key;
        c.pubkey = gbest_key;
        c.giter = gbest_iter;
        c.t = iters_completed;
        c.t_run0 = iters_completed;
        HIP_TRY(hipMemcpy(s->args.ctrl, &c, sizeof c, hipMemcpyHostToDevice));
        HIP_TRY(pso::launch_clear_pending(s->args, s->stream));
        HIP_TRY(hipStreamSynchronize(s->stream));
        return PSO_OK;
    });
}

int pso_get_counters(pso_swarm *s, uint64_t *pbest_improvements)
{
    return pso::guarded([&]() -> int {
        if (!s) return fail(PSO_EINVAL, "swarm is NULL");
        int rc = fetch_ctrl(s, false);
        if (rc) return rc;
        if (pbest_improvements) *pbest_improvements = s->host_ctrl->improved;
        return PSO_OK;
    });
}

int pso_get_async_counters(pso_swarm *s, uint64_t *tiles, uint64_t *fresh_tiles)
{
    return pso::guarded([&]() -> int {
        if (!s) return fail(PSO_EINVAL, "swarm is NULL");
        int rc = fetch_ctrl(s, false);
        if (rc) return rc;
        if (tiles) *tiles = s->host_ctrl->tiles;
        if (fresh_tiles) *fresh_tiles = s->host_ctrl->fresh;
        return PSO_OK;
    });
}

int pso_sync(pso_swarm *s)
{
    return pso::guarded([&]() -> int {
        if (!s) return fail(PSO_EINVAL, "swarm is NULL");
        return fetch_ctrl(s, false);
    });
}

int pso_destroy(pso_swarm *s)
{
    return pso::guarded([&]() -> int {
        if (!s) return fail(PSO_EINVAL, "swarm is NULL");
        (void)hipStreamSynchronize(s->stream);
        drop_steps_graph(s);
        if (s->gang_words) (void)hipFree(s->gang_words);
        if (s->owns_ws) (void)hipFree(s->ws);
        if (s->owns_stream) (void)hipStreamDestroy(s->stream);
        (void)hipHostFree(s->host_ctrl);
        (void)hipHostFree(s->host_gpos);
        delete s;
        return PSO_OK;
    });
}

} // extern "C"

// ---------------------------------------------------------------------------
// Batches.
// ---------------------------------------------------------------------------
struct pso_batch {
    int64_t count = 0;
    int maxD = 1;
    int grid = 1;
    pso::BatchShape shape = pso::DEFAULT_BATCH_SHAPE;
    void *slab = nullptr;            // every swarm's state and gang region
    pso::BatchItem *d_items = nullptr;
    pso::BatchEntry *d_entries = nullptr;
    uint32_t n_entries = 0;
    uint32_t n_first = 0;  // entries of the first kernel (all of them unless some swarms stream after it)
    int grid_rest = 0;     // workgroups of the second (streamed) kernel
    pso::BatchResult *d_results = nullptr;
    unsigned int *d_next = nullptr;
    unsigned int *d_err = nullptr;
    std::vector<pso::BatchItem> items; // host copy (device pointers inside)
    std::vector<char *> gang;          // each swarm's gang region (sized for max_parts)
    std::vector<uint32_t> max_parts;
    std::vector<uint64_t> N;
    std::vector<int> D;
    std::vector<long long> max_iter;
    uint64_t signature = 0;
    hipStream_t stream = nullptr;
    bool owns_stream = false;
    hipGraph_t graph = nullptr;         // the captured launch of the current shape
    hipGraphExec_t graph_exec = nullptr;
};

namespace {

void drop_graph(pso_batch *b)
{
    if (b->graph_exec) (void)hipGraphExecDestroy(b->graph_exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->graph_exec = nullptr;
    b->graph = nullptr;
}

void batch_free(pso_batch *b)
{
    if (!b) return;
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    drop_graph(b);
    if (b->slab) (void)hipFree(b->slab);
    if (b->d_items) (void)hipFree(b->d_items);
    if (b->d_entries) (void)hipFree(b->d_entries);
    if (b->d_err) (void)hipFree(b->d_err);
    if (b->d_results) (void)hipFree(b->d_results);
    if (b->d_next) (void)hipFree(b->d_next);
    if (b->owns_stream && b->stream) (void)hipStreamDestroy(b->stream);
    delete b;
}

using pso::shape_grid;
using pso::staged_kib_fitting;

// The staged shape a new batch takes before any autotuning: one 1024-lane
// workgroup per compute unit with as much staged state as fits.
pso::BatchShape default_staged_shape(int maxD)
{
    pso::BatchShape sh = pso::DEFAULT_STAGED_SHAPE;
    sh.stage_kib = staged_kib_fitting(maxD, 1);
    return sh;
}

// The shapes the autotuner tries: streamed, lanes per workgroup x part size
// x co-resident workgroups (all of them, or half: a smaller working set);
// LDS-staged, lanes x staged KiB per workgroup (two or one workgroups per
// compute unit's 160 KiB, less the room each needs for maxD-float vectors;
// smaller parts meet too often: 38 KiB was 3x slower on the 4096-swarm
// batch).
std::vector<pso::BatchShape> tuner_candidates(int maxD)
{
    std::vector<pso::BatchShape> c;
    for (int lanes : {64, 128, 256})
        for (long long pw : {1LL << 15, 1LL << 17})
            for (int half : {0, 1}) c.push_back(pso::BatchShape{lanes, half ? -2 : 0, pw, 0});
    for (int lanes : {512, 1024})
        for (int per_cu : {2, 1})
            if (const int kib = staged_kib_fitting(maxD, per_cu)) c.push_back(pso::BatchShape{lanes, 0, 0, kib});
    return c;
}

// Process-wide choices of the autotuner, by batch signature and device.
std::mutex g_tuned_mu;
std::map<std::pair<uint64_t, int>, pso::BatchShape> g_tuned;

// Applies a shape: parts per swarm, gang bindings, the work queue (largest
// per-part work first, a swarm's parts consecutive) and the grid.
int batch_configure(pso_batch *b, const pso::BatchShape &sh)
{
    const bool staged = sh.stage_kib > 0;
    if (sh.stage_kib < 0 || !pso::batch_lanes_supported(sh.lanes, staged) || (!staged && sh.part_work < 1))
        return fail(PSO_EINVAL, "batch shape: lanes must be 64, 128 or 256 with part_work >= 1 (streamed), or 256, "
                                "512 or 1024 (LDS-staged, stage_kib > 0)");
    int grid = 0;
    HIP_TRY(shape_grid(b->maxD, sh, &grid));
    if (grid < 1) return fail(PSO_EINVAL, "batch shape: %d KiB of staged state per workgroup exceed the LDS", sh.stage_kib);
    // Under a staged shape, a swarm whose staged parts would be too many
    // (more than 512, than the grid, or than its gang region holds) streams:
    // the launch runs the staged kernel over the staged swarms, then the
    // streamed kernel (256 lanes, parts of 2^17 updates, its own co-resident
    // grid) over those.  Entries of the staged swarms come first.
    const pso::BatchShape stream_sh = staged ? pso::BatchShape{256, 0, 1LL << 17, 0} : sh;
    int grid_s = grid;
    if (staged) HIP_TRY(shape_grid(b->maxD, stream_sh, &grid_s));
    std::vector<uint32_t> parts(b->count);
    std::vector<char> streamed(b->count, 0);
    for (int64_t i = 0; i < b->count; ++i) {
        if (staged) {
            parts[i] = pso::staged_parts(b->N[i], b->D[i], b->items[i].fitness, sh.stage_kib, grid);
            if (parts[i] > 0 && parts[i] <= b->max_parts[i]) continue;
            streamed[i] = 1;
        }
        parts[i] = std::min(pso::parts_for(b->N[i], b->D[i], grid_s, stream_sh), b->max_parts[i]);
    }
    uint64_t n_entries = 0, n_first = 0;
    for (int64_t i = 0; i < b->count; ++i) {
        pso::bind_gang(&b->items[i], b->gang[i], parts[i]);
        n_entries += parts[i];
        if (!streamed[i]) n_first += parts[i];
    }
    std::vector<uint32_t> order(b->count);
    for (int64_t i = 0; i < b->count; ++i) order[i] = (uint32_t)i;
    std::stable_sort(order.begin(), order.end(), [&](uint32_t x, uint32_t y) {
        if (streamed[x] != streamed[y]) return streamed[x] < streamed[y];
        const double wx = double(b->N[x]) * b->D[x] * double(b->max_iter[x] + 1) / parts[x];
        const double wy = double(b->N[y]) * b->D[y] * double(b->max_iter[y] + 1) / parts[y];
        return wx > wy;
    });
    std::vector<pso::BatchEntry> entries;
    entries.reserve(n_entries);
    for (uint32_t i : order)
        for (uint32_t p = 0; p < parts[i]; ++p) entries.push_back(pso::BatchEntry{i, p, i, 0u});
    HIP_TRY(hipStreamSynchronize(b->stream));
    HIP_TRY(hipMemcpy(b->d_items, b->items.data(), sizeof(pso::BatchItem) * b->count, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(b->d_entries, entries.data(), sizeof(pso::BatchEntry) * n_entries, hipMemcpyHostToDevice));
    b->n_entries = (uint32_t)n_entries;
    b->n_first = (uint32_t)n_first;
    b->grid = (int)std::min<uint64_t>(n_first, (uint64_t)grid);
    b->grid_rest = (int)std::min<uint64_t>(n_entries - n_first, (uint64_t)grid_s);
    b->shape = sh;
    drop_graph(b); // the captured launch had the old grid and lanes
    return PSO_OK;
}

int batch_launch_iters(pso_batch *b, long long iter_cap, bool reset)
{
    if (reset) HIP_TRY(pso::launch_batch_reset(b->d_items, b->d_results, (uint32_t)b->count, b->d_next, b->stream));
    if (b->n_first > 0)
        HIP_TRY(pso::launch_batch(b->d_items, b->d_entries, b->d_results, b->n_first, b->d_next, b->maxD, b->grid,
                                  b->shape.lanes, (long long)1 << 62, iter_cap, b->stream, nullptr, nullptr, b->d_err,
                                  b->shape.stage_kib));
    if (b->n_entries > b->n_first) // the swarms too large to stage, streamed
        HIP_TRY(pso::launch_batch(b->d_items, b->d_entries + b->n_first, b->d_results, b->n_entries - b->n_first,
                                  b->d_next, b->maxD, b->grid_rest, 256, (long long)1 << 62, iter_cap, b->stream,
                                  nullptr, nullptr, b->d_err, 0));
    return PSO_OK;
}

} // namespace

extern "C" {

int pso_batch_create(const pso_desc *descs, int64_t count, void *hip_stream, pso_batch **out)
{
    return pso::guarded([&]() -> int {
        if (!out) return fail(PSO_EINVAL, "out is NULL");
        *out = nullptr;
        if (count < 1 || count > MAX_BATCH_SWARMS)
            return fail(PSO_EINVAL, "count=%lld outside [1, %lld]", (long long)count, (long long)MAX_BATCH_SWARMS);
        if (!descs) return fail(PSO_EINVAL, "descs is NULL");
        int maxD = 1;
        for (int64_t i = 0; i < count; ++i) {
            int rc = pso_internal_check_desc(&descs[i]);
            if (rc) return fail(rc, "descriptor %lld: %s", (long long)i, std::string(g_err).c_str());
            maxD = std::max(maxD, (int)descs[i].D);
        }
        // gang regions are sized for the most parts any tuner shape gives
        const std::vector<pso::BatchShape> cands = tuner_candidates(maxD);
        std::vector<int> cand_grid(cands.size());
        for (size_t c = 0; c < cands.size(); ++c)
            if (shape_grid(maxD, cands[c], &cand_grid[c]) != hipSuccess) return fail(PSO_EDEVICE, "device query failed");
        int def_grid = 0;
        if (shape_grid(maxD, pso::DEFAULT_BATCH_SHAPE, &def_grid) != hipSuccess)
            return fail(PSO_EDEVICE, "device query failed");
        std::vector<pso::Layout> lay(count);
        std::vector<size_t> off(count), goff(count);
        std::vector<uint32_t> maxp(count);
        size_t total = 0;
        uint64_t max_entries = 0, sig = 1469598103934665603ull;
        auto mix = [&](uint64_t v) { sig = (sig ^ v) * 1099511628211ull; };
        mix((uint64_t)count);
        for (int64_t i = 0; i < count; ++i) {
            const pso_desc &d = descs[i];
            lay[i] = pso::layout_of((uint64_t)d.N, d.D, false);
            uint32_t mp = pso::parts_for((uint64_t)d.N, d.D, def_grid, pso::DEFAULT_BATCH_SHAPE);
            for (size_t c = 0; c < cands.size(); ++c)
                mp = std::max(mp, cands[c].stage_kib > 0
                                      ? pso::staged_parts((uint64_t)d.N, d.D, d.fitness_id, cands[c].stage_kib, cand_grid[c])
                                      : pso::parts_for((uint64_t)d.N, d.D, cand_grid[c], cands[c]));
            maxp[i] = mp;
            off[i] = total;
            goff[i] = total + lay[i].total;
            total += lay[i].total + pso::gang_bytes(mp, d.D);
            max_entries += mp;
            // bounded before anything is allocated: the work queue's entry
            // count is a 32-bit value, and no device holds this many bytes
            if (total > MAX_BATCH_BYTES)
                return fail(PSO_ENOMEM, "the batch needs more than %llu bytes of device memory",
                            (unsigned long long)MAX_BATCH_BYTES);
            if (max_entries > MAX_BATCH_ENTRIES)
                return fail(PSO_EINVAL, "the batch's swarms need more than %llu work-queue entries",
                            (unsigned long long)MAX_BATCH_ENTRIES);
            mix((uint64_t)d.N);
            mix((uint64_t)d.D);
            mix((uint64_t)d.max_iter);
        }
        pso_batch *b = new (std::nothrow) pso_batch();
        if (!b) return fail(PSO_ENOMEM, "host allocation failed");
        b->count = count;
        b->maxD = maxD;
        b->signature = sig;
        if (hip_stream) {
            b->stream = static_cast<hipStream_t>(hip_stream);
        } else {
            if (hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking) != hipSuccess) {
                batch_free(b);
                return fail(PSO_EDEVICE, "hipStreamCreate failed");
            }
            b->owns_stream = true;
        }
        if (hipMalloc(&b->slab, total) != hipSuccess || hipMalloc(&b->d_items, sizeof(pso::BatchItem) * count) != hipSuccess ||
            hipMalloc(&b->d_entries, sizeof(pso::BatchEntry) * max_entries) != hipSuccess ||
            hipMalloc(&b->d_results, sizeof(pso::BatchResult) * count) != hipSuccess ||
            hipMalloc(&b->d_next, sizeof(unsigned int)) != hipSuccess ||
            hipMalloc(&b->d_err, sizeof(unsigned int)) != hipSuccess) {
            batch_free(b);
            return fail(PSO_ENOMEM, "hipMalloc of %zu bytes for the batch failed", total);
        }
        b->items.resize(count);
        b->gang.resize(count);
        b->max_parts = maxp;
        b->N.resize(count);
        b->D.resize(count);
        b->max_iter.resize(count);
        std::vector<float> shifts;
        for (int64_t i = 0; i < count; ++i) {
            const pso_desc &d = descs[i];
            pso::BatchItem &it = b->items[i];
            char *base = static_cast<char *>(b->slab) + off[i];
            it.a = pso::bind(base, lay[i], (uint64_t)d.N, d.D);
            it.a.lo = d.bounds[0];
            it.a.hi = d.bounds[1];
            it.a.w = d.w;
            it.a.c1 = d.c1;
            it.a.c2 = d.c2;
            it.a.vmax = d.vmax;
            it.a.k0 = (uint32_t)d.seed;
            it.a.k1 = (uint32_t)(d.seed >> 32);
            it.fitness = d.fitness_id;
            it.max_iter = d.max_iter;
            it.tol = d.tol;
            it.fstar = d.f_star;
            b->gang[i] = static_cast<char *>(b->slab) + goff[i];
            b->N[i] = (uint64_t)d.N;
            b->D[i] = d.D;
            b->max_iter[i] = d.max_iter;
            shifts.assign(d.D, 0.0f);
            if (d.shift) std::memcpy(shifts.data(), d.shift, sizeof(float) * d.D);
            if (hipMemcpy(const_cast<float *>(it.a.shift), shifts.data(), sizeof(float) * d.D, hipMemcpyHostToDevice) !=
                hipSuccess) {
                batch_free(b);
                return fail(PSO_EDEVICE, "shift upload failed");
            }
        }
        if (hipMemset(b->d_err, 0, sizeof(unsigned int)) != hipSuccess) {
            batch_free(b);
            return fail(PSO_EDEVICE, "descriptor upload failed");
        }
        // a shape the autotuner chose for the same workload on this device, else
        // the staged default where every swarm fits it, else the streamed one
        pso::BatchShape sh = default_staged_shape(maxD);
        bool tuned = false;
        int dev = 0;
        (void)hipGetDevice(&dev);
        {
            std::lock_guard<std::mutex> g(g_tuned_mu);
            auto f = g_tuned.find({sig, dev});
            if (f != g_tuned.end()) {
                sh = f->second;
                tuned = true;
            }
        }
        int rc = batch_configure(b, sh);
        if (rc == PSO_EINVAL && !tuned) rc = batch_configure(b, pso::DEFAULT_BATCH_SHAPE);
        if (rc) {
            batch_free(b);
            return rc;
        }
        *out = b;
        return PSO_OK;
    });
}

int pso_batch_launch(pso_batch *b)
{
    return pso::guarded([&]() -> int {
        if (!b) return fail(PSO_EINVAL, "batch is NULL");
        const char *env = getenv("PSO_BATCH_GRAPH");
        if (env && !strcmp(env, "0")) return batch_launch_iters(b, (long long)1 << 62, true);
        // the whole launch (reset kernel, counter kernel, persistent kernel; no
        // memset) is captured once per shape and replayed as one graph
        if (!b->graph_exec) {
            HIP_TRY(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
            int rc = batch_launch_iters(b, (long long)1 << 62, true);
            hipGraph_t g = nullptr;
            const hipError_t e = hipStreamEndCapture(b->stream, &g);
            if (rc) {
                if (g) (void)hipGraphDestroy(g);
                return rc;
            }
            if (e != hipSuccess) return fail(PSO_EDEVICE, "graph capture failed: %s", hipGetErrorString(e));
            b->graph = g;
            if (hipGraphInstantiate(&b->graph_exec, b->graph, nullptr, nullptr, 0) != hipSuccess) {
                drop_graph(b);
                return fail(PSO_EDEVICE, "graph instantiation failed");
            }
        }
        HIP_TRY(hipGraphLaunch(b->graph_exec, b->stream));
        return PSO_OK;
    });
}

int pso_batch_get_shape(pso_batch *b, pso_batch_shape *shape)
{
    return pso::guarded([&]() -> int {
        if (!b || !shape) return fail(PSO_EINVAL, "batch or shape is NULL");
        shape->lanes = b->shape.lanes;
        shape->grid = b->grid;
        shape->part_work = b->shape.part_work;
        shape->stage_kib = b->shape.stage_kib;
        return PSO_OK;
    });
}

int pso_batch_set_shape(pso_batch *b, const pso_batch_shape *shape)
{
    return pso::guarded([&]() -> int {
        if (!b || !shape) return fail(PSO_EINVAL, "batch or shape is NULL");
        if (shape->grid < 0) return fail(PSO_EINVAL, "grid must be >= 0 (0: the co-resident capacity)");
        return batch_configure(b, pso::BatchShape{shape->lanes, shape->grid, shape->part_work, shape->stage_kib});
    });
}

int pso_batch_autotune(pso_batch *b, int64_t probe_iters, pso_batch_shape *chosen)
{
    return pso::guarded([&]() -> int {
        if (!b) return fail(PSO_EINVAL, "batch is NULL");
        if (probe_iters < 1) return fail(PSO_EINVAL, "probe_iters must be >= 1");
        hipEvent_t e0 = nullptr, e1 = nullptr;
        HIP_TRY(hipEventCreate(&e0));
        if (hipEventCreate(&e1) != hipSuccess) {
            (void)hipEventDestroy(e0);
            return fail(PSO_EDEVICE, "hipEventCreate failed");
        }
        // A launch costs a fixed part (Step 1 aside: a staged shape loads and
        // stores every part's state once) plus a part per iteration.  Two
        // probe lengths, p and 3p iterations, give both; a shape is priced
        // at the batch's mean iteration limit, so the fixed cost of staging
        // is not weighed as if a launch ran p iterations only.
        double iters_run = 0.0;
        for (int64_t i = 0; i < b->count; ++i) iters_run += double(b->items[i].max_iter);
        iters_run = std::max(1.0, iters_run / double(b->count));
        double best_ms = -1.0;
        pso::BatchShape best = b->shape;
        int rc = PSO_OK;
        auto timed = [&](long long iters, float *ms) -> int {
            if (hipEventRecord(e0, b->stream) != hipSuccess) return fail(PSO_EDEVICE, "hipEventRecord failed");
            if (int r = batch_launch_iters(b, iters, false)) return r;
            if (hipEventRecord(e1, b->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                hipEventElapsedTime(ms, e0, e1) != hipSuccess)
                return fail(PSO_EDEVICE, "timing a probe launch failed");
            return PSO_OK;
        };
        for (const pso::BatchShape &sh : tuner_candidates(b->maxD)) {
            // Step 1 and one iteration untimed, then the two timed probes; a
            // staged shape that this batch's swarms do not fit is skipped
            if ((rc = batch_configure(b, sh))) {
                if (sh.stage_kib > 0 && rc == PSO_EINVAL) {
                    rc = PSO_OK;
                    continue;
                }
                break;
            }
            if ((rc = batch_launch_iters(b, 1, true))) break;
            float t1 = 0.0f, t3 = 0.0f;
            if ((rc = timed(probe_iters, &t1)) || (rc = timed(3 * probe_iters, &t3))) break;
            unsigned int err = 0;
            if (hipMemcpy(&err, b->d_err, sizeof err, hipMemcpyDeviceToHost) != hipSuccess || err) {
                rc = fail(PSO_EDEVICE, "a probe launch reported a device error");
                break;
            }
            const double per_iter = std::max(0.0, double(t3 - t1) / double(2 * probe_iters));
            const double fixed = std::max(0.0, double(t1) - per_iter * double(probe_iters));
            const double ms = fixed + per_iter * iters_run;
            if (best_ms < 0.0 || ms < best_ms) {
                best_ms = ms;
                best = sh;
            }
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        if (rc) return rc;
        if ((rc = batch_configure(b, best))) return rc;
        int dev = 0;
        (void)hipGetDevice(&dev);
        {
            std::lock_guard<std::mutex> g(g_tuned_mu);
            g_tuned[{b->signature, dev}] = best;
        }
        if (chosen) return pso_batch_get_shape(b, chosen);
        return PSO_OK;
    });
}

int pso_batch_results(pso_batch *b, pso_result *results)
{
    return pso::guarded([&]() -> int {
        if (!b) return fail(PSO_EINVAL, "batch is NULL");
        if (!results) return fail(PSO_EINVAL, "results is NULL");
        HIP_TRY(hipStreamSynchronize(b->stream));
        unsigned int err = 0;
        HIP_TRY(hipMemcpy(&err, b->d_err, sizeof err, hipMemcpyDeviceToHost));
        if (err) return fail(PSO_EDEVICE, "a batched swarm's parts timed out waiting for each other");
        std::vector<pso::BatchResult> r(b->count);
        HIP_TRY(hipMemcpy(r.data(), b->d_results, sizeof(pso::BatchResult) * b->count, hipMemcpyDeviceToHost));
        for (int64_t i = 0; i < b->count; ++i) {
            results[i].gbest_value = pso::key_fitness(r[i].gkey);
            results[i].status = PSO_OK;
            results[i].gbest_iter = r[i].giter;
            results[i].iters = r[i].iters;
            if (results[i].gbest_pos)
                HIP_TRY(hipMemcpy(results[i].gbest_pos, b->items[i].a.gpos, sizeof(float) * b->items[i].a.D,
                                  hipMemcpyDeviceToHost));
        }
        return PSO_OK;
    });
}

int pso_batch_destroy(pso_batch *b)
{
    return pso::guarded([&]() -> int {
        if (!b) return fail(PSO_EINVAL, "batch is NULL");
        batch_free(b);
        return PSO_OK;
    });
}

int pso_batch_run(const pso_desc *descs, int64_t count, pso_result *results)
{
    return pso::guarded([&]() -> int {
        pso_batch *b = nullptr;
        int rc = pso_batch_create(descs, count, nullptr, &b);
        if (rc) return rc;
        rc = pso_batch_launch(b);
        if (!rc) rc = pso_batch_results(b, results);
        batch_free(b);
        return rc;
    });
}

} // extern "C"

// Host-only stand-in for the part of the HIP runtime that the request
// server's host code calls, so that its scheduler can be unit-tested on the
// CPU (and under ThreadSanitizer) with no GPU.  A stream is a worker thread
// running its enqueued operations in order; an event completes when the
// stream reaches it; device and pinned memory are zeroed host memory.
// Enqueued copies wait a random 0-200 us before they run, so that work
// ordered on one stream only is visibly late for another stream.
#pragma once

#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstddef>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <functional>
#include <mutex>
#include <random>
#include <thread>

#define __device__
#define __host__
#define __global__
#define __shared__
#define __forceinline__ inline
#define __launch_bounds__(x)

enum hipError_t { hipSuccess = 0, hipErrorInvalidValue = 1, hipErrorOutOfMemory = 2, hipErrorNotReady = 600 };
enum hipMemcpyKind { hipMemcpyHostToHost, hipMemcpyHostToDevice, hipMemcpyDeviceToHost, hipMemcpyDeviceToDevice };
enum hipDeviceAttribute_t {
    hipDeviceAttributeWallClockRate,
    hipDeviceAttributeMultiprocessorCount,
    hipDeviceAttributeMaxSharedMemoryPerBlock
};
#define hipStreamNonBlocking 1u
#define hipEventDisableTiming 2u
#define hipHostMallocDefault 0u

template <class T>
inline T __shfl_xor(T v, int, int = 64) { return v; }
inline unsigned int __float_as_uint(float f)
{
    unsigned int u;
    std::memcpy(&u, &f, sizeof u);
    return u;
}

inline void stub_delay()
{
    thread_local std::mt19937 rng(std::hash<std::thread::id>()(std::this_thread::get_id()));
    const int us = int(rng() % 200);
    if (us > 20) std::this_thread::sleep_for(std::chrono::microseconds(us));
}

struct ihipStream_t {
    std::mutex mu;
    std::condition_variable cv;
    std::deque<std::function<void()>> q;
    bool busy = false, quit = false;
    std::thread th;
    ihipStream_t() : th([this] { run(); }) {}
    ~ihipStream_t()
    {
        {
            std::lock_guard<std::mutex> g(mu);
            quit = true;
        }
        cv.notify_all();
        th.join();
    }
    void run()
    {
        for (;;) {
            std::function<void()> f;
            {
                std::unique_lock<std::mutex> lk(mu);
                cv.wait(lk, [&] { return quit || !q.empty(); });
                if (q.empty()) return;
                f = std::move(q.front());
                q.pop_front();
                busy = true;
            }
            f();
            {
                std::lock_guard<std::mutex> g(mu);
                busy = false;
            }
            cv.notify_all();
        }
    }
    void push(std::function<void()> f)
    {
        {
            std::lock_guard<std::mutex> g(mu);
            q.push_back(std::move(f));
        }
        cv.notify_all();
    }
    void drain()
    {
        std::unique_lock<std::mutex> lk(mu);
        cv.wait(lk, [&] { return q.empty() && !busy; });
    }
};
typedef ihipStream_t *hipStream_t;

struct ihipEvent_t {
    std::atomic<uint64_t> recorded{0}, reached{0};
};
typedef ihipEvent_t *hipEvent_t;

// work on a stream (the null stream runs it at once)
inline void stub_enqueue(hipStream_t st, std::function<void()> f)
{
    if (st)
        st->push(std::move(f));
    else
        f();
}

inline hipError_t hipMalloc(void **p, size_t n)
{
    *p = std::calloc(1, n ? n : 1);
    return *p ? hipSuccess : hipErrorOutOfMemory;
}
template <class T>
inline hipError_t hipMalloc(T **p, size_t n) { return hipMalloc(reinterpret_cast<void **>(p), n); }
inline hipError_t hipHostMalloc(void **p, size_t n, unsigned int) { return hipMalloc(p, n); }
inline hipError_t hipFree(void *p)
{
    std::free(p);
    return hipSuccess;
}
inline hipError_t hipHostFree(void *p) { return hipFree(p); }
inline hipError_t hipMemset(void *p, int v, size_t n)
{
    std::memset(p, v, n);
    return hipSuccess;
}
inline hipError_t hipMemcpyAsync(void *dst, const void *src, size_t n, hipMemcpyKind, hipStream_t st)
{
    stub_enqueue(st, [=] {
        stub_delay();
        std::memcpy(dst, src, n);
    });
    return hipSuccess;
}
inline hipError_t hipStreamSynchronize(hipStream_t st)
{
    if (st) st->drain();
    return hipSuccess;
}
inline hipError_t hipStreamCreateWithFlags(hipStream_t *st, unsigned int)
{
    *st = new ihipStream_t();
    return hipSuccess;
}
inline hipError_t hipStreamDestroy(hipStream_t st)
{
    delete st;
    return hipSuccess;
}
inline hipError_t hipEventCreateWithFlags(hipEvent_t *ev, unsigned int)
{
    *ev = new ihipEvent_t();
    return hipSuccess;
}
inline hipError_t hipEventDestroy(hipEvent_t ev)
{
    delete ev;
    return hipSuccess;
}
inline hipError_t hipEventRecord(hipEvent_t ev, hipStream_t st)
{
    const uint64_t gen = ++ev->recorded;
    stub_enqueue(st, [ev, gen] { ev->reached.store(gen); });
    return hipSuccess;
}
inline hipError_t hipEventQuery(hipEvent_t ev)
{
    return ev->reached.load() >= ev->recorded.load() ? hipSuccess : hipErrorNotReady;
}
inline hipError_t hipGetDevice(int *d)
{
    *d = 0;
    return hipSuccess;
}
inline hipError_t hipDeviceGetAttribute(int *v, hipDeviceAttribute_t a, int)
{
    *v = a == hipDeviceAttributeWallClockRate ? 100000 : a == hipDeviceAttributeMultiprocessorCount ? 8 : 163840;
    return hipSuccess;
}
inline const char *hipGetErrorString(hipError_t) { return "stub HIP error"; }

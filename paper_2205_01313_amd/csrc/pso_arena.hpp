// pso_arena.hpp -- host-side bookkeeping of the request server, with no
// device code and no HIP dependency (unit-tested on the CPU):
//   Arena     first-fit sub-allocator of byte offsets inside one device
//             allocation, coalescing freed neighbours;
//   Admission FIFO admission of requests by memory: the head of the queue is
//             admitted while the arena can hold it; a request larger than the
//             whole arena is rejected at once; no request overtakes the head
//             (no starvation of large requests).
#pragma once

#include <cstddef>
#include <cstdint>
#include <deque>
#include <map>
#include <unordered_map>
#include <vector>

namespace pso {

class Arena {
public:
    explicit Arena(size_t capacity = 0, size_t align = 256) : cap_(capacity / align * align), align_(align)
    {
        if (cap_) free_[0] = cap_;
    }

    size_t capacity() const { return cap_; }
    size_t used() const { return used_bytes_; }
    size_t round(size_t bytes) const { return (bytes + align_ - 1) / align_ * align_; }

    // First fit; returns false if no free range is large enough.
    bool alloc(size_t bytes, size_t *offset)
    {
        const size_t need = round(bytes ? bytes : 1);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= need) {
                const size_t off = it->first, rest = it->second - need;
                free_.erase(it);
                if (rest) free_[off + need] = rest;
                live_[off] = need;
                used_bytes_ += need;
                *offset = off;
                return true;
            }
        }
        return false;
    }

    // Frees a range returned by alloc; false if offset is not live.
    bool release(size_t offset)
    {
        auto it = live_.find(offset);
        if (it == live_.end()) return false;
        size_t off = offset, len = it->second;
        live_.erase(it);
        used_bytes_ -= len;
        auto nx = free_.lower_bound(off);
        if (nx != free_.end() && nx->first == off + len) { // merge right
            len += nx->second;
            nx = free_.erase(nx);
        }
        if (nx != free_.begin()) { // merge left
            auto pv = std::prev(nx);
            if (pv->first + pv->second == off) {
                pv->second += len;
                return true;
            }
        }
        free_[off] = len;
        return true;
    }

    size_t largest_free() const
    {
        size_t m = 0;
        for (const auto &kv : free_) m = kv.second > m ? kv.second : m;
        return m;
    }

    size_t free_ranges() const { return free_.size(); }

private:
    size_t cap_, align_;
    size_t used_bytes_ = 0;
    std::map<size_t, size_t> free_;           // offset -> length
    std::unordered_map<size_t, size_t> live_; // offset -> length
};

// A request waiting for admission: its ticket and the bytes it needs.
struct Pending {
    uint64_t ticket;
    size_t bytes;
};

class Admission {
public:
    explicit Admission(Arena *arena) : arena_(arena) {}

    void push(const Pending &p) { q_.push_back(p); }
    size_t queued() const { return q_.size(); }

    // Admits from the head while memory allows, at most max_admit requests.
    // Fills `admitted` with (ticket, offset) and `rejected` with tickets that
    // can never fit.
    void admit(std::vector<std::pair<uint64_t, size_t>> *admitted, std::vector<uint64_t> *rejected,
               size_t max_admit = SIZE_MAX)
    {
        while (!q_.empty() && admitted->size() < max_admit) {
            const Pending &h = q_.front();
            if (arena_->round(h.bytes) > arena_->capacity()) {
                rejected->push_back(h.ticket);
                q_.pop_front();
                continue;
            }
            size_t off = 0;
            if (!arena_->alloc(h.bytes, &off)) break;
            admitted->emplace_back(h.ticket, off);
            q_.pop_front();
        }
    }

    // Drops a queued ticket (cancel); false if it is not queued.
    bool cancel(uint64_t ticket)
    {
        for (auto it = q_.begin(); it != q_.end(); ++it)
            if (it->ticket == ticket) {
                q_.erase(it);
                return true;
            }
        return false;
    }

private:
    Arena *arena_;
    std::deque<Pending> q_;
};

} // namespace pso

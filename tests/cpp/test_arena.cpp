// CPU unit test of the server's host bookkeeping (pso_arena.hpp): the arena
// against a byte-map model under random alloc/free, coalescing, and FIFO
// admission by memory.  Prints "ok" and exits 0 on success.
#include <cstdio>
#include <cstdlib>
#include <map>
#include <random>
#include <vector>

#include "../../paper_2205_01313_amd/csrc/pso_arena.hpp"

#define CHECK(c)                                                              \
    do {                                                                      \
        if (!(c)) {                                                           \
            std::printf("FAIL line %d: %s\n", __LINE__, #c);                 \
            return 1;                                                         \
        }                                                                     \
    } while (0)

int main()
{
    // random alloc/free against a byte map
    {
        const size_t cap = 1 << 20, align = 256;
        pso::Arena a(cap, align);
        std::vector<int> owner(cap / align, -1);
        std::map<size_t, size_t> live; // offset -> rounded length
        std::mt19937_64 rng(7);
        int id = 0;
        for (int step = 0; step < 200000; ++step) {
            if (live.empty() || rng() % 3 != 0) {
                const size_t want = 1 + rng() % 20000;
                size_t off = 0;
                const bool ok = a.alloc(want, &off);
                // a fit exists iff some free run of blocks is long enough
                const size_t blocks = (want + align - 1) / align;
                size_t run = 0, best = 0;
                for (int o : owner) {
                    run = (o < 0) ? run + 1 : 0;
                    best = run > best ? run : best;
                }
                CHECK(ok == (best >= blocks));
                if (ok) {
                    CHECK(off % align == 0 && off + blocks * align <= cap);
                    for (size_t b = off / align; b < off / align + blocks; ++b) {
                        CHECK(owner[b] < 0);
                        owner[b] = id;
                    }
                    live[off] = blocks * align;
                    ++id;
                }
            } else {
                auto it = live.begin();
                std::advance(it, rng() % live.size());
                CHECK(a.release(it->first));
                for (size_t b = it->first / align; b < (it->first + it->second) / align; ++b) owner[b] = -1;
                live.erase(it);
            }
            size_t used = 0;
            for (auto &kv : live) used += kv.second;
            CHECK(a.used() == used);
        }
        for (auto &kv : live) CHECK(a.release(kv.first));
        CHECK(a.used() == 0 && a.free_ranges() == 1 && a.largest_free() == cap);
        CHECK(!a.release(12345));
    }
    // admission: FIFO, head blocks, oversize rejected, slot limit
    {
        pso::Arena a(10 * 256);
        pso::Admission q(&a);
        q.push({1, 4 * 256});
        q.push({2, 4 * 256});
        q.push({3, 11 * 256}); // larger than the arena: rejected when it reaches the head
        q.push({4, 4 * 256});
        q.push({5, 1});
        std::vector<std::pair<uint64_t, size_t>> ad;
        std::vector<uint64_t> rej;
        q.admit(&ad, &rej);
        // 1 and 2 fit (8 of 10 blocks); 3 can never fit and is rejected; 4 waits at the head
        CHECK(ad.size() == 2 && ad[0].first == 1 && ad[1].first == 2);
        CHECK(rej.size() == 1 && rej[0] == 3 && q.queued() == 2);
        const size_t off1 = ad[0].second;
        // 5 (one block) would fit but must not overtake 4
        ad.clear();
        rej.clear();
        q.admit(&ad, &rej);
        CHECK(ad.empty() && rej.empty() && q.queued() == 2);
        CHECK(a.release(off1));
        q.admit(&ad, &rej, 1); // at most one
        CHECK(ad.size() == 1 && ad[0].first == 4 && q.queued() == 1);
        CHECK(q.cancel(5) && q.queued() == 0 && !q.cancel(5));
    }
    std::printf("ok\n");
    return 0;
}

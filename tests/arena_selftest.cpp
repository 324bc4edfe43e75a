// Randomised check of the serving engine's budget allocator against a
// byte-map model: blocks never overlap, stay inside the range, usage adds up,
// and freeing everything restores one run covering the whole range.
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include <random>
#include <vector>

#include "arena.hpp"

#define CHECK(c)                                                  \
    do {                                                          \
        if (!(c)) {                                               \
            fprintf(stderr, "check failed line %d: %s\n", __LINE__, #c); \
            return 1;                                             \
        }                                                         \
    } while (0)

int main() {
    const int64_t size = 1 << 20;
    rbsm::Arena a(size);
    CHECK(a.largest_free() == size && a.used() == 0);
    CHECK(a.alloc(size + 1) == -1);
    std::vector<uint8_t> owner(size / rbsm::Arena::kAlign, 0);
    struct Blk {
        int64_t off, bytes;
    };
    std::vector<Blk> live;
    std::mt19937_64 rng(12345);
    int64_t model_used = 0, fails = 0;
    for (int it = 0; it < 200000; ++it) {
        const bool do_alloc = live.empty() || (rng() % 100) < 55;
        if (do_alloc) {
            const int64_t bytes = 1 + (int64_t)(rng() % 40000);
            const int64_t off = a.alloc(bytes);
            if (off < 0) {
                ++fails;
                CHECK(a.largest_free() < rbsm::Arena::round_up(bytes));
                continue;
            }
            CHECK(off % rbsm::Arena::kAlign == 0);
            CHECK(off + bytes <= size);
            const int64_t r = rbsm::Arena::round_up(bytes);
            for (int64_t u = off / rbsm::Arena::kAlign; u < (off + r) / rbsm::Arena::kAlign; ++u) {
                CHECK(owner[u] == 0);
                owner[u] = 1;
            }
            live.push_back({off, bytes});
            model_used += r;
        } else {
            const size_t k = rng() % live.size();
            const Blk b = live[k];
            live[k] = live.back();
            live.pop_back();
            const int64_t r = rbsm::Arena::round_up(b.bytes);
            for (int64_t u = b.off / rbsm::Arena::kAlign; u < (b.off + r) / rbsm::Arena::kAlign; ++u) owner[u] = 0;
            a.release(b.off, b.bytes);
            model_used -= r;
        }
        CHECK(a.used() == model_used);
        CHECK(a.peak() >= a.used());
    }
    for (const Blk &b : live) a.release(b.off, b.bytes);
    CHECK(a.used() == 0);
    CHECK(a.free_runs() == 1 && a.largest_free() == size);
    CHECK(fails > 0);  // the run exercised a full arena
    printf("arena ok: %lld failed allocations, peak %lld of %lld\n", (long long)fails, (long long)a.peak(),
           (long long)size);
    return 0;
}

// Randomised check of the engine's first-fit pool allocator against a unit-bitmap model:
// allocations never overlap and stay inside the pool, used/peak bytes agree with the model,
// invalid releases are refused without changing anything, freed neighbours coalesce (a pool
// emptied in any order is one free range again), and first fit returns the lowest fitting
// offset.  Exit status 0 on success.
#include <cstdio>
#include <random>
#include <vector>

#include "pool.h"

#define CHECK(c)                                                    \
    do {                                                            \
        if (!(c)) {                                                 \
            std::fprintf(stderr, "check failed line %d: %s\n", __LINE__, #c); \
            return 1;                                               \
        }                                                           \
    } while (0)

int main() {
    using te::PoolAlloc;
    const uint64_t A = PoolAlloc::kAlign;
    {
        PoolAlloc p(10 * A + 17);  // size rounds down to whole units
        CHECK(p.size() == 10 * A);
        uint64_t a, b, c;
        CHECK(p.alloc(3 * A, &a) && a == 0);
        CHECK(p.alloc(1, &b) && b == 3 * A);     // rounds up to one unit
        CHECK(p.alloc(2 * A + 1, &c) && c == 4 * A);
        CHECK(p.used() == 7 * A);
        CHECK(!p.alloc(4 * A, &a));              // 3 units left
        CHECK(!p.release(5 * A, A));             // inside an allocation, not its start
        CHECK(!p.release(7 * A, A));             // free range
        CHECK(!p.release(A + 1, A));             // misaligned
        CHECK(p.release(3 * A, 1));
        CHECK(p.alloc(A, &a) && a == 3 * A);     // first fit reuses the hole
        CHECK(p.release(3 * A, A));
        CHECK(p.release(0, 3 * A));
        CHECK(p.ranges() == 2);                  // [0, 4A) and [7A, 10A)
        CHECK(p.largest_free() == 4 * A);
        CHECK(p.release(4 * A, 2 * A + 1));
        CHECK(p.ranges() == 1 && p.largest_free() == 10 * A && p.used() == 0);
        CHECK(p.peak() == 7 * A);
    }
    std::mt19937_64 rng(12345);
    for (int trial = 0; trial < 200; ++trial) {
        const uint64_t units = 1 + rng() % 300;
        PoolAlloc p(units * A);
        std::vector<int> owner(units, -1);
        struct Blk { uint64_t off, bytes; bool live; };
        std::vector<Blk> blocks;
        uint64_t used = 0, peak = 0;
        for (int step = 0; step < 400; ++step) {
            const bool do_alloc = blocks.empty() || rng() % 3 != 0;
            if (do_alloc) {
                const uint64_t bytes = 1 + rng() % (units * A / 4 + 1);
                const uint64_t need = (bytes + A - 1) / A;
                // model: lowest start of a free run of `need` units
                long expect = -1;
                for (uint64_t s = 0; s + need <= units && expect < 0; ++s) {
                    bool ok = true;
                    for (uint64_t u = s; u < s + need; ++u)
                        if (owner[u] >= 0) { ok = false; break; }
                    if (ok) expect = (long)s;
                }
                CHECK(p.fits(bytes) == (expect >= 0));
                uint64_t off = 0;
                const bool got = p.alloc(bytes, &off);
                CHECK(got == (expect >= 0));
                if (got) {
                    CHECK(off % A == 0 && off / A == (uint64_t)expect);
                    for (uint64_t u = off / A; u < off / A + need; ++u) owner[u] = (int)blocks.size();
                    blocks.push_back({off, bytes, true});
                    used += need * A;
                    if (used > peak) peak = used;
                }
            } else {
                const size_t i = rng() % blocks.size();
                Blk& b = blocks[i];
                if (!b.live && owner[b.off / A] >= 0) continue;  // offset reused by a live block
                const bool ok = p.release(b.off, b.bytes);
                CHECK(ok == b.live);
                if (b.live) {
                    const uint64_t need = (b.bytes + A - 1) / A;
                    for (uint64_t u = b.off / A; u < b.off / A + need; ++u) owner[u] = -1;
                    used -= need * A;
                    b.live = false;
                }
            }
            CHECK(p.used() == used && p.peak() == peak);
            uint64_t free_units = 0, run = 0, best = 0;
            for (uint64_t u = 0; u < units; ++u) {
                if (owner[u] < 0) { ++free_units; ++run; if (run > best) best = run; } else run = 0;
            }
            CHECK(p.largest_free() == best * A);
            CHECK(free_units * A + used == p.size());
        }
        for (auto& b : blocks)
            if (b.live) CHECK(p.release(b.off, b.bytes));
        CHECK(p.used() == 0 && p.ranges() == 1 && p.largest_free() == p.size());
    }
    std::printf("pool ok\n");
    return 0;
}

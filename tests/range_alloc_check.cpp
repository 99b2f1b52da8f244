// Host unit check of the scheduler's first-fit range allocator against a
// brute-force model of the pool (one flag per unit), on seeded random
// sequences of allocations and releases.  Built and run by
// tests/test_range_alloc.py with AddressSanitizer and UBSan.
#include "range_alloc.h"

#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

using dsdp::host::RangeAlloc;

static int fail(const char *what, int seed, int step)
{
    std::fprintf(stderr, "range allocator check failed: %s (seed %d, step %d)\n", what, seed, step);
    return 1;
}

int main()
{
    for (int seed = 0; seed < 200; seed++) {
        std::mt19937 rng(seed);
        const size_t total = 1 + rng() % 4096;
        RangeAlloc a;
        a.init(total);
        std::vector<char> taken(total, 0);
        struct Block { size_t off, n; };
        std::vector<Block> live;
        for (int step = 0; step < 2000; step++) {
            if (live.empty() || rng() % 3 != 0) {
                const size_t n = rng() % 97;   // 0 is rounded up to one unit
                const size_t need = n ? n : 1;
                // the model's first fit: the lowest offset with `need` free units
                size_t expect = total, run = 0;
                for (size_t u = 0; u < total; u++) {
                    run = taken[u] ? 0 : run + 1;
                    if (run == need) { expect = u + 1 - need; break; }
                }
                size_t off = 0;
                const bool ok = a.alloc(n, off);
                if (ok != (expect < total)) return fail("alloc success differs from the model", seed, step);
                if (!ok) continue;
                if (off != expect) return fail("not the first fit", seed, step);
                for (size_t u = off; u < off + need; u++) taken[u] = 1;
                live.push_back({off, n});
            } else {
                const size_t k = rng() % live.size();
                const Block b = live[k];
                live[k] = live.back();
                live.pop_back();
                a.release(b.off, b.n);
                for (size_t u = b.off; u < b.off + (b.n ? b.n : 1); u++) taken[u] = 0;
            }
            // invariants: used units, free ranges disjoint, sorted, never adjacent
            size_t used = 0;
            for (char t : taken) used += t;
            if (used != a.used) return fail("used count", seed, step);
            size_t prev_end = 0, free_units = 0;
            bool first = true;
            for (const auto &r : a.free_) {
                if (r.second == 0) return fail("empty free range", seed, step);
                if (!first && r.first <= prev_end) return fail("free ranges touch or overlap", seed, step);
                for (size_t u = r.first; u < r.first + r.second; u++)
                    if (u >= total || taken[u]) return fail("free range covers a taken unit", seed, step);
                prev_end = r.first + r.second;
                free_units += r.second;
                first = false;
            }
            if (free_units + used != total) return fail("free + used != total", seed, step);
        }
    }
    std::printf("range allocator: 200 seeds x 2000 operations match the model\n");
    return 0;
}

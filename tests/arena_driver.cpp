// CPU driver for the server's first-fit arena (csrc/arena.hpp): a seeded
// random sequence of allocations and releases, checked after every step
// against a plain list of live blocks (no overlap, inside the range, used
// bytes and coalescing consistent).  Exit status 0 on success.
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "arena.hpp"

int main(int argc, char **argv) {
    const unsigned seed = argc > 1 ? (unsigned)std::atoi(argv[1]) : 1u;
    std::mt19937_64 rng(seed);
    const size_t size = (size_t)1 << 24;
    grav::Arena a(size);
    struct Blk { size_t off, bytes; };
    std::vector<Blk> live;
    size_t fails = 0;
    for (int step = 0; step < 200000; ++step) {
        if (live.empty() || rng() % 3 != 0) {
            const size_t want = 1 + rng() % (size / 16);
            size_t off = 0;
            if (a.alloc(want, &off)) {
                const size_t b = grav::Arena::round(want);
                if (off % grav::Arena::kAlign || off + b > a.size()) { std::puts("out of range"); return 1; }
                for (auto &l : live)
                    if (off < l.off + grav::Arena::round(l.bytes) && l.off < off + b) { std::puts("overlap"); return 1; }
                live.push_back({off, want});
            } else {
                ++fails;
                if (a.largest_free() >= grav::Arena::round(want)) { std::puts("fit refused"); return 1; }
            }
        } else {
            const size_t k = rng() % live.size();
            a.release(live[k].off, live[k].bytes);
            live.erase(live.begin() + k);
        }
        size_t used = 0;
        for (auto &l : live) used += grav::Arena::round(l.bytes);
        if (used != a.used()) { std::puts("used bytes drift"); return 1; }
    }
    for (auto &l : live) a.release(l.off, l.bytes);
    if (a.used() != 0 || a.free_ranges() != 1 || a.largest_free() != a.size()) { std::puts("not coalesced"); return 1; }
    std::printf("ok: %zu refused allocations\n", fails);
    return 0;
}

// Randomised check of the serving arena's first-fit map against a byte-level
// model: every allocation lies inside the arena, overlaps no live one and
// starts at the lowest offset of a free run that holds it; largest() is the
// longest free run; releasing everything leaves one block.
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "arena_map.h"

int main(int argc, char** argv)
{
    const unsigned seed = argc > 1 ? (unsigned)atoi(argv[1]) : 1u;
    std::mt19937_64 rng(seed);
    const size_t unit = 256, units = 4096;   // a 1 MiB arena in 256-byte units
    lagp_rt::ArenaMap m;
    m.reset(units * unit + 100);             // the tail below 256 bytes is dropped
    std::vector<char> used(units, 0);
    struct Live { size_t off, bytes; };
    std::vector<Live> live;
    auto lowest_fit = [&](size_t need, size_t* at) {
        size_t run = 0;
        for (size_t u = 0; u < units; ++u) {
            run = used[u] ? 0 : run + 1;
            if (run == need) { *at = u + 1 - need; return true; }
        }
        return false;
    };
    auto longest = [&]() {
        size_t best = 0, run = 0;
        for (size_t u = 0; u < units; ++u) { run = used[u] ? 0 : run + 1; if (run > best) best = run; }
        return best;
    };
    for (int step = 0; step < 200000; ++step) {
        const bool grow = live.empty() || (rng() % 100) < 55;
        if (grow) {
            const size_t need = 1 + rng() % (rng() % 4 == 0 ? 1024 : 64);
            size_t off = 0, at = 0;
            const bool ok = m.alloc(need * unit, &off), fit = lowest_fit(need, &at);
            if (ok != fit) { printf("FAIL step %d: alloc %zu units returned %d, model %d\n", step, need, ok, fit); return 1; }
            if (!ok) continue;
            if (off % unit || off / unit != at) { printf("FAIL step %d: offset %zu, lowest fit %zu\n", step, off, at * unit); return 1; }
            for (size_t u = at; u < at + need; ++u) used[u] = 1;
            live.push_back({off, need * unit});
        } else {
            const size_t k = rng() % live.size();
            m.release(live[k].off, live[k].bytes);
            for (size_t u = live[k].off / unit; u < (live[k].off + live[k].bytes) / unit; ++u) used[u] = 0;
            live[k] = live.back();
            live.pop_back();
        }
        if (m.largest() != longest() * unit) { printf("FAIL step %d: largest %zu, model %zu\n", step, m.largest(), longest() * unit); return 1; }
    }
    for (const Live& l : live) m.release(l.off, l.bytes);
    if (m.blocks() != 1 || m.largest() != units * unit) { printf("FAIL: %zu blocks, largest %zu after releasing all\n", m.blocks(), m.largest()); return 1; }
    size_t off = 0;
    if (m.alloc(0, &off)) { printf("FAIL: a zero-byte allocation succeeded\n"); return 1; }
    printf("OK\n");
    return 0;
}

// Drives the serving loop's admission rules (rmpc_sched.h) with random arrivals and a fake
// completion source that finishes running launches in random order, and checks after every
// step: launches respect their capacities, requests start in submission order, staging
// ranges of running launches are disjoint and inside the staging memory, the allocator's
// books balance, and a free slot never idles while the queue holds requests and nothing runs.
// Usage: sched_check <seed> <steps>.  Prints "OK ..." and exits 0, or prints the violation
// and exits 1.
#include <cstdio>
#include <cstdlib>
#include <deque>
#include <random>
#include <vector>

#include "rmpc_sched.h"

namespace {

struct R {
    uint64_t ticket;
    int n_tiles;
    size_t stage_bytes;
    size_t stage_off;
};

int fail(const char *what, long step)
{
    std::printf("FAIL at step %ld: %s\n", step, what);
    return 1;
}

size_t rounded(size_t b) { return b ? (b + rmpc_sched::kAlign - 1) / rmpc_sched::kAlign * rmpc_sched::kAlign : 0; }

}  // namespace

int main(int argc, char **argv)
{
    const unsigned seed = argc > 1 ? (unsigned)std::atoi(argv[1]) : 1u;
    const long steps = argc > 2 ? std::atol(argv[2]) : 20000;
    std::mt19937_64 rng(seed);
    const int n_slots = 1 + (int)(rng() % 4);
    const rmpc_sched::Limits lim{1 + (int)(rng() % 64), 16 + (int)(rng() % 4096)};
    const size_t cap = (1 + rng() % 64) * 65536;

    rmpc_sched::Arena staging;
    staging.init(cap);
    std::deque<R> pending;
    std::vector<std::vector<R>> running((size_t)n_slots);
    std::vector<bool> busy((size_t)n_slots, false);
    uint64_t next_ticket = 1, last_started = 0, completed = 0, launches = 0, waits = 0;
    const long arrive_until = steps * 3 / 4;

    for (long step = 0; step < steps || !pending.empty() || completed + 1 < next_ticket; ++step) {
        if (step > steps * 4) return fail("requests never drain", step);
        // arrivals (none in the last quarter: everything must drain)
        if (step < arrive_until) {
            const int n_new = (int)(rng() % 4);
            for (int k = 0; k < n_new; ++k) {
                R r{next_ticket++, 1 + (int)(rng() % (uint64_t)lim.max_tiles), 0, 0};
                if (rng() % 2) r.stage_bytes = 1 + rng() % cap;   // a host scan
                pending.push_back(r);
            }
        }
        // fake completion source: each running launch finishes with probability 1/3
        for (int s = 0; s < n_slots; ++s) {
            if (!busy[(size_t)s] || rng() % 3) continue;
            rmpc_sched::release_launch(running[(size_t)s], staging);
            completed += running[(size_t)s].size();
            running[(size_t)s].clear();
            busy[(size_t)s] = false;
        }
        // admission into free slots, as the server thread does
        for (int s = 0; s < n_slots; ++s) {
            if (busy[(size_t)s] || pending.empty()) continue;
            std::vector<R> &out = running[(size_t)s];
            const rmpc_sched::Formed f = rmpc_sched::form_launch(pending, lim, staging, out);
            if (f.staging_wait) ++waits;
            if (f.n == 0) continue;
            if ((int)out.size() != f.n) return fail("count mismatch", step);
            if (f.n > lim.max_queries) return fail("too many queries in a launch", step);
            int tiles = 0;
            for (const R &r : out) {
                if (r.ticket != last_started + 1) return fail("request started out of order", step);
                last_started = r.ticket;
                tiles += r.n_tiles;
            }
            if (tiles != f.tiles || tiles > lim.max_tiles) return fail("tile capacity exceeded", step);
            if (f.staging_wait && (pending.empty() || pending.front().stage_bytes == 0))
                return fail("staging wait reported without a staged head", step);
            busy[(size_t)s] = true;
            ++launches;
        }
        // staging books: running ranges disjoint, inside [0, cap), and summing to in_use()
        std::vector<std::pair<size_t, size_t>> ranges;
        size_t total = 0;
        for (const auto &v : running)
            for (const R &r : v)
                if (r.stage_bytes) {
                    ranges.emplace_back(r.stage_off, r.stage_off + rounded(r.stage_bytes));
                    total += rounded(r.stage_bytes);
                }
        for (size_t i = 0; i < ranges.size(); ++i) {
            if (ranges[i].second > cap) return fail("staging range outside the memory", step);
            if (ranges[i].first % rmpc_sched::kAlign) return fail("staging range misaligned", step);
            for (size_t j = i + 1; j < ranges.size(); ++j)
                if (ranges[i].first < ranges[j].second && ranges[j].first < ranges[i].second)
                    return fail("staging ranges overlap", step);
        }
        if (total != staging.in_use()) return fail("staging allocator books do not balance", step);
        // progress: with nothing running, a non-empty queue must have been admitted
        bool any = false;
        for (int s = 0; s < n_slots; ++s) any = any || busy[(size_t)s];
        if (!any && !pending.empty()) return fail("idle with requests queued", step);
    }
    if (staging.in_use() != 0 || staging.n_free_ranges() != 1) return fail("staging not whole after draining", steps);
    std::printf("OK slots=%d max_q=%d max_tiles=%d cap=%zu requests=%llu launches=%llu waits=%llu\n", n_slots,
                lim.max_queries, lim.max_tiles, cap, (unsigned long long)(next_ticket - 1),
                (unsigned long long)launches, (unsigned long long)waits);
    return 0;
}

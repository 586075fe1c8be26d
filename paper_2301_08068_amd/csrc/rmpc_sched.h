// rmpc_sched.h -- host logic that decides what the serving loop launches: a first-fit
// allocator of byte ranges (the device arena and the staging memory are carved with it) and
// the rule that forms the next launch from the front of the FIFO queue.  Plain C++ with no
// HIP dependency, so the admission rules can be exercised on the CPU alone.
#pragma once

#include <cstddef>
#include <cstdint>
#include <deque>
#include <iterator>
#include <map>
#include <utility>
#include <vector>

namespace rmpc_sched {

constexpr size_t kAlign = 256;

// First-fit allocator of 256-byte aligned ranges of [0, bytes) (offsets only).
class Arena {
  public:
    void init(size_t bytes)
    {
        free_.clear();
        used_.clear();
        in_use_ = 0;
        if (bytes) free_[0] = bytes;
    }
    bool alloc(size_t bytes, size_t *off)
    {
        bytes = (bytes + kAlign - 1) / kAlign * kAlign;
        if (bytes == 0) bytes = kAlign;
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                *off = it->first;
                const size_t rest = it->second - bytes;
                const size_t noff = it->first + bytes;
                free_.erase(it);
                if (rest) free_[noff] = rest;
                used_[*off] = bytes;
                in_use_ += bytes;
                return true;
            }
        }
        return false;
    }
    void release(size_t off)
    {
        auto u = used_.find(off);
        if (u == used_.end()) return;
        size_t start = off, len = u->second;
        in_use_ -= len;
        used_.erase(u);
        auto nx = free_.lower_bound(start);
        if (nx != free_.end() && start + len == nx->first) { len += nx->second; nx = free_.erase(nx); }
        if (nx != free_.begin()) {
            auto pv = std::prev(nx);
            if (pv->first + pv->second == start) { start = pv->first; len += pv->second; free_.erase(pv); }
        }
        free_[start] = len;
    }
    size_t in_use() const { return in_use_; }
    size_t n_free_ranges() const { return free_.size(); }

  private:
    std::map<size_t, size_t> free_, used_;
    size_t in_use_ = 0;
};

// Capacity of one launch.
struct Limits {
    int max_queries;
    int max_tiles;
};

// What form_launch took.
struct Formed {
    int n = 0;                  // requests moved into the launch
    int tiles = 0;              // their tiles
    bool staging_wait = false;  // stopped because the head's points did not fit the staging memory
};

// Move requests from the front of `pending` into `out` while the launch has room: at most
// max_queries requests and max_tiles tiles, and each request's staging bytes (its field
// stage_bytes; 0 = none) must be allocated from `staging` (the offset goes to stage_off).
// The queue is served strictly in order: the first request that does not fit ends the
// launch, so no later request overtakes it.  R needs n_tiles, stage_bytes and stage_off.
template <class R>
Formed form_launch(std::deque<R> &pending, const Limits &lim, Arena &staging, std::vector<R> &out)
{
    Formed f;
    while (!pending.empty() && f.n < lim.max_queries) {
        R &r = pending.front();
        if (f.tiles + r.n_tiles > lim.max_tiles) break;
        if (r.stage_bytes) {
            size_t off = 0;
            if (!staging.alloc(r.stage_bytes, &off)) {
                f.staging_wait = true;
                break;
            }
            r.stage_off = off;
        }
        f.tiles += r.n_tiles;
        ++f.n;
        out.push_back(std::move(r));
        pending.pop_front();
    }
    return f;
}

// Return a finished launch's staging ranges.
template <class R>
void release_launch(const std::vector<R> &launched, Arena &staging)
{
    for (const R &r : launched)
        if (r.stage_bytes) staging.release(r.stage_off);
}

}  // namespace rmpc_sched

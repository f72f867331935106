// Host-only core of the request server: the device-memory arena, memory
// admission and the work-item schedule.  No HIP here, so the policy is tested
// on the CPU with a simulated executor; server.hip drives it with real
// launches.
//
// A request is run as work items: `chunks` launches of the transform, each
// over a consecutive group of its point slices (the work plan of the same call
// made alone, cut between slices, so the result is bitwise the solo result),
// then one finishing launch (the fixed-order reduction over the slices and the
// spectrum) once every chunk has completed.
//
// Memory admission: a waiting request is admitted (its scratch block taken
// from the arena) in arrival order; one that does not fit yet is passed over by
// later requests that do, until it has waited age_s since submission: from then
// on nothing behind it is admitted before it, so none starves.  A request whose
// footprint exceeds the whole arena is refused at submission.
//
// Work items go to free execution slots: among admitted requests with an item
// ready, requests that have waited longer than age_s come first (oldest
// first), then the one with the least remaining work (shortest remaining work
// first), ties by arrival.  So a small request that arrives behind large ones
// does not wait for them to finish: it waits at most for the items already
// running.
#pragma once

#include <cstddef>
#include <cstdint>
#include <iterator>
#include <map>
#include <vector>

namespace ptalm {
namespace serve {

constexpr size_t kArenaAlign = 256;

inline size_t round_up(size_t b) { return (b + kArenaAlign - 1) / kArenaAlign * kArenaAlign; }

// First-fit allocator over the byte range [0, size) of one device allocation.
// Blocks are kArenaAlign aligned; freed blocks merge with free neighbours.
class Arena {
  public:
    explicit Arena(size_t size) : size_(size / kArenaAlign * kArenaAlign) {
        if (size_ > 0) free_[0] = size_;
    }

    size_t size() const { return size_; }
    size_t in_use() const { return in_use_; }

    // Lowest-offset free block that holds `bytes` (rounded up); false if none.
    bool alloc(size_t bytes, size_t *offset) {
        const size_t need = round_up(bytes == 0 ? 1 : bytes);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < need) continue;
            const size_t off = it->first, len = it->second;
            free_.erase(it);
            if (len > need) free_[off + need] = len - need;
            used_[off] = need;
            in_use_ += need;
            *offset = off;
            return true;
        }
        return false;
    }

    // Returns the block at `offset` (must come from alloc) and merges free neighbours.
    bool release(size_t offset) {
        auto u = used_.find(offset);
        if (u == used_.end()) return false;
        size_t off = offset, len = u->second;
        used_.erase(u);
        in_use_ -= len;
        auto next = free_.lower_bound(off);
        if (next != free_.end() && off + len == next->first) {
            len += next->second;
            next = free_.erase(next);
        }
        if (next != free_.begin()) {
            auto prev = std::prev(next);
            if (prev->first + prev->second == off) {
                off = prev->first;
                len += prev->second;
                free_.erase(prev);
            }
        }
        free_[off] = len;
        return true;
    }

    size_t largest_free() const {
        size_t m = 0;
        for (const auto &kv : free_) m = kv.second > m ? kv.second : m;
        return m;
    }
    size_t free_blocks() const { return free_.size(); }

  private:
    size_t size_;
    size_t in_use_ = 0;
    std::map<size_t, size_t> free_;   // offset -> length
    std::map<size_t, size_t> used_;   // offset -> length
};

// A request admitted to the arena: where its scratch block lies.
struct Admitted {
    int64_t ticket;
    size_t offset;
    size_t bytes;
};

// One work item on one execution slot: chunk >= 0 is that chunk of the
// request's point slices, chunk == kFinish its finishing launch.
constexpr int kFinish = -1;
struct Item {
    int64_t ticket;
    int chunk;
    int slot;
};

class Scheduler {
  public:
    Scheduler(size_t arena_bytes, int slots, double age_s)
        : arena_(arena_bytes), busy_(slots > 0 ? slots : 1, false), age_s_(age_s) {}

    const Arena &arena() const { return arena_; }
    int slots() const { return (int)busy_.size(); }
    size_t waiting() const { return queue_.size(); }            // submitted, not admitted
    size_t active() const { return jobs_.size() - queue_.size(); }  // admitted, not complete
    int running() const { return running_; }                      // items in flight

    // Queues a request of `chunks` items (>= 0) plus its finish, each chunk
    // worth `chunk_work` (any unit: only compared between requests); false
    // (refused) if its footprint exceeds the arena.
    bool push(int64_t ticket, size_t bytes, int chunks, double chunk_work, double now) {
        if (round_up(bytes == 0 ? 1 : bytes) > arena_.size() || chunks < 0) return false;
        Job j;
        j.bytes = bytes;
        j.chunks = chunks;
        j.chunk_work = chunk_work;
        j.submit = now;
        j.order = next_order_++;
        jobs_[ticket] = j;
        queue_.push_back(ticket);
        return true;
    }

    // Memory admission (see the header): returns the requests admitted now.
    std::vector<Admitted> admit(double now) {
        std::vector<Admitted> out;
        for (size_t i = 0; i < queue_.size();) {
            Job &j = jobs_[queue_[i]];
            size_t off;
            if (arena_.alloc(j.bytes, &off)) {
                j.admitted = true;
                j.offset = off;
                out.push_back({queue_[i], off, j.bytes});
                queue_.erase(queue_.begin() + (std::ptrdiff_t)i);
                continue;
            }
            if (now - j.submit >= age_s_) break;   // aged: nothing behind it goes first
            ++i;
        }
        return out;
    }

    // The next work item for a free slot, if any is ready (see the header).
    bool next_item(double now, Item *out) {
        int slot = -1;
        for (int s = 0; s < (int)busy_.size(); ++s)
            if (!busy_[s]) {
                slot = s;
                break;
            }
        if (slot < 0) return false;
        int64_t best = 0;
        const Job *bj = nullptr;
        for (const auto &kv : jobs_) {
            const Job &j = kv.second;
            if (!j.admitted || !ready(j)) continue;
            if (bj == nullptr || better(j, *bj, now)) {
                bj = &j;
                best = kv.first;
            }
        }
        if (bj == nullptr) return false;
        Job &j = jobs_[best];
        out->ticket = best;
        out->slot = slot;
        if (j.issued < j.chunks) {
            out->chunk = j.issued++;
        } else {
            out->chunk = kFinish;
            j.finish_issued = true;
        }
        busy_[slot] = true;
        ++running_;
        return true;
    }

    // An item finished on its slot.  Returns true when it was the request's
    // finish: the request is complete and its arena block is free again.
    bool item_done(const Item &it) {
        if (it.slot >= 0 && it.slot < (int)busy_.size() && busy_[it.slot]) {
            busy_[it.slot] = false;
            --running_;
        }
        auto f = jobs_.find(it.ticket);
        if (f == jobs_.end()) return false;
        Job &j = f->second;
        if (it.chunk != kFinish) {
            ++j.done;
            return false;
        }
        arena_.release(j.offset);
        jobs_.erase(f);
        return true;
    }

    // Chunks of a request issued and completed so far (for tests).
    bool progress(int64_t ticket, int *issued, int *done) const {
        auto f = jobs_.find(ticket);
        if (f == jobs_.end()) return false;
        *issued = f->second.issued;
        *done = f->second.done;
        return true;
    }

  private:
    struct Job {
        size_t bytes = 0, offset = 0;
        int chunks = 0, issued = 0, done = 0;
        double chunk_work = 0.0, submit = 0.0;
        int64_t order = 0;
        bool admitted = false, finish_issued = false;
    };
    // an item is ready: a chunk not yet issued, or the finish once every chunk is done
    static bool ready(const Job &j) {
        return j.issued < j.chunks || (!j.finish_issued && j.done == j.chunks);
    }
    double remaining(const Job &j) const { return (j.chunks - j.issued) * j.chunk_work; }
    bool better(const Job &a, const Job &b, double now) const {
        const bool aa = now - a.submit >= age_s_, ab = now - b.submit >= age_s_;
        if (aa != ab) return aa;
        if (aa) return a.order < b.order;
        const double ra = remaining(a), rb = remaining(b);
        if (ra != rb) return ra < rb;
        return a.order < b.order;
    }

    Arena arena_;
    std::vector<bool> busy_;
    double age_s_;
    std::map<int64_t, Job> jobs_;
    std::vector<int64_t> queue_;   // waiting for memory, in arrival order
    int running_ = 0;
    int64_t next_order_ = 0;
};

}  // namespace serve
}  // namespace ptalm

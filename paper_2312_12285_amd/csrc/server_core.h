// Host-only core of the request server: the device-memory arena and the
// admission policy.  No HIP here, so the policy is tested on the CPU with a
// simulated executor; server.hip drives it with real launches.
//
// Admission is first-come first-served: the oldest waiting request is admitted
// as soon as an execution slot is free and its scratch footprint fits in the
// arena; requests behind it wait (no overtaking, so none starves).  A request
// whose footprint exceeds the whole arena is refused at submission.
#pragma once

#include <cstddef>
#include <cstdint>
#include <deque>
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

struct Admitted {
    int64_t ticket;
    int slot;
    size_t offset;
    size_t bytes;
};

// FIFO admission over `slots` execution slots and one arena.
class Admission {
  public:
    Admission(size_t arena_bytes, int slots) : arena_(arena_bytes), busy_(slots > 0 ? slots : 1, false) {}

    const Arena &arena() const { return arena_; }
    int slots() const { return (int)busy_.size(); }
    size_t waiting() const { return queue_.size(); }
    int running() const { return running_; }

    // Queues a request; false (refused) if its footprint exceeds the arena.
    bool push(int64_t ticket, size_t bytes) {
        if (round_up(bytes == 0 ? 1 : bytes) > arena_.size()) return false;
        queue_.push_back({ticket, bytes});
        return true;
    }

    // Admits, in arrival order, every waiting request that fits now; stops at the
    // first one that does not (no overtaking).
    std::vector<Admitted> admit() {
        std::vector<Admitted> out;
        while (!queue_.empty()) {
            int slot = -1;
            for (int s = 0; s < (int)busy_.size(); ++s)
                if (!busy_[s]) {
                    slot = s;
                    break;
                }
            if (slot < 0) break;
            size_t off;
            if (!arena_.alloc(queue_.front().bytes, &off)) break;
            busy_[slot] = true;
            ++running_;
            out.push_back({queue_.front().ticket, slot, off, queue_.front().bytes});
            queue_.pop_front();
        }
        return out;
    }

    // A running request finished: its slot and arena block become free.
    void complete(const Admitted &a) {
        arena_.release(a.offset);
        if (a.slot >= 0 && a.slot < (int)busy_.size() && busy_[a.slot]) {
            busy_[a.slot] = false;
            --running_;
        }
    }

  private:
    struct Wait {
        int64_t ticket;
        size_t bytes;
    };
    Arena arena_;
    std::vector<bool> busy_;
    std::deque<Wait> queue_;
    int running_ = 0;
};

}  // namespace serve
}  // namespace ptalm

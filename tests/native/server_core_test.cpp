// CPU test of the request server's arena, memory admission and work-item
// schedule (server_core.h), driven by a simulated executor: requests with
// random footprints, chunk counts and run times arrive over simulated time;
// items run on slots; completions free slots and memory.
#include <cassert>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <algorithm>
#include <iterator>
#include <vector>

#include "server_core.h"

using ptalm::serve::Admitted;
using ptalm::serve::Arena;
using ptalm::serve::Item;
using ptalm::serve::Scheduler;

#define CHECK(c)                                                                 \
    do {                                                                         \
        if (!(c)) {                                                              \
            std::fprintf(stderr, "%s:%d: check failed: %s\n", __FILE__, __LINE__, #c); \
            std::exit(1);                                                        \
        }                                                                        \
    } while (0)

static uint64_t rng_state = 0x9E3779B97F4A7C15ull;
static uint64_t next_u64() {   // splitmix64
    uint64_t z = (rng_state += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

static void arena_basics() {
    Arena a(10 * 256 + 100);           // rounded down to 10 blocks of 256
    CHECK(a.size() == 2560);
    size_t o1, o2, o3, o4;
    CHECK(a.alloc(1, &o1) && o1 == 0);          // rounds up to 256
    CHECK(a.alloc(300, &o2) && o2 == 256);      // 512 bytes
    CHECK(a.alloc(256, &o3) && o3 == 768);
    CHECK(a.in_use() == 1024);
    CHECK(!a.alloc(2000, &o4));                 // 1536 left
    CHECK(a.alloc(1536, &o4) && o4 == 1024);
    CHECK(a.largest_free() == 0);
    CHECK(a.release(o2));                       // hole of 512 at 256
    CHECK(!a.release(o2));                      // double free refused
    CHECK(!a.alloc(600, &o2));                  // hole too small
    CHECK(a.alloc(200, &o2) && o2 == 256);      // first fit, lowest offset
    CHECK(a.release(o1) && a.release(o2) && a.release(o3) && a.release(o4));
    CHECK(a.in_use() == 0 && a.free_blocks() == 1 && a.largest_free() == 2560);   // fully merged
}

static void admission_passing_and_aging() {
    Scheduler q(1024, 4, 10.0);
    CHECK(!q.push(1, 2000, 1, 1.0, 0.0));       // larger than the arena: refused
    CHECK(q.push(1, 700, 1, 1.0, 0.0));
    CHECK(q.push(2, 600, 1, 1.0, 0.0));         // does not fit next to 1
    CHECK(q.push(3, 100, 1, 1.0, 0.0));         // fits: passes 2, which is not yet aged
    std::vector<Admitted> a = q.admit(1.0);
    CHECK(a.size() == 2 && a[0].ticket == 1 && a[1].ticket == 3);
    CHECK(q.waiting() == 1);
    // 2 has waited past age_s: a later request that would fit may no longer pass it
    CHECK(q.push(4, 100, 1, 1.0, 11.0));
    CHECK(q.admit(11.5).empty());
    // finish 1 and 3 (one chunk + finish each); then 2 and 4 are admitted in order
    for (int64_t t : {1, 3}) {
        Item it;
        CHECK(q.next_item(12.0, &it) && it.chunk == 0);
        CHECK(!q.item_done(it));
        Item f;
        CHECK(q.next_item(12.0, &f) && f.chunk == ptalm::serve::kFinish && f.ticket == it.ticket);
        CHECK(q.item_done(f));
        (void)t;
    }
    a = q.admit(12.0);
    CHECK(a.size() == 2 && a[0].ticket == 2 && a[1].ticket == 4);
}

static void items_shortest_remaining_first() {
    Scheduler q(1 << 20, 2, 100.0);
    CHECK(q.push(1, 1000, 8, 10.0, 0.0));       // large: 8 chunks of 10
    CHECK(q.push(2, 1000, 2, 1.0, 0.1));        // small: 2 chunks of 1
    CHECK(q.admit(0.2).size() == 2);
    Item a, b, c;
    CHECK(q.next_item(0.2, &a) && a.ticket == 2 && a.chunk == 0);
    CHECK(q.next_item(0.2, &b) && b.ticket == 2 && b.chunk == 1 && b.slot != a.slot);
    CHECK(!q.next_item(0.2, &c));                // both slots busy
    CHECK(!q.item_done(a));
    // the small request's finish waits for its second chunk: the large one runs meanwhile
    CHECK(q.next_item(0.3, &c) && c.ticket == 1 && c.chunk == 0);
    CHECK(!q.item_done(b));
    Item f;
    CHECK(q.next_item(0.4, &f) && f.ticket == 2 && f.chunk == ptalm::serve::kFinish);
    CHECK(q.item_done(f));
    int issued = 0, done = 0;
    CHECK(q.progress(1, &issued, &done) && issued == 1 && done == 0);
    CHECK(!q.progress(2, &issued, &done));       // complete and gone
}

static void aged_requests_go_first() {
    Scheduler q(1 << 20, 1, 5.0);
    CHECK(q.push(1, 100, 3, 100.0, 0.0));        // large, arrives first
    CHECK(q.admit(0.0).size() == 1);
    Item it;
    CHECK(q.next_item(0.0, &it) && it.ticket == 1);
    q.item_done(it);
    CHECK(q.push(2, 100, 1, 1.0, 1.0));          // small
    CHECK(q.admit(1.0).size() == 1);
    CHECK(q.next_item(1.0, &it) && it.ticket == 2);   // shortest remaining first
    q.item_done(it);
    CHECK(q.push(3, 100, 1, 1.0, 6.0));
    CHECK(q.admit(6.0).size() == 1);
    CHECK(q.next_item(6.0, &it) && it.ticket == 1);   // 1 has waited past age_s: it goes first
    q.item_done(it);
}

static void simulated_stream() {
    // Requests with random footprints, chunk counts and chunk run times arrive over
    // simulated time; every item runs on a slot for its run time.
    const size_t budget = 64ull << 20;
    const int slots = 4, K = 3000;
    Scheduler q(budget, slots, 2.0);
    struct Job {
        int64_t ticket;
        double arrive, chunk_run, first = -1, end = -1;
        size_t bytes;
        int chunks;
        bool admitted = false;
        int chunks_done = 0;
    };
    std::vector<Job> jobs;
    double t = 0;
    for (int k = 0; k < K; ++k) {
        t += (next_u64() % 1000) * 1e-4;
        Job j;
        j.ticket = k + 1;
        j.arrive = t;
        j.chunks = (int)(next_u64() % 9);                  // 0 .. 8 chunks
        j.chunk_run = 0.0005 + (next_u64() % 1000) * 2e-4;
        j.bytes = 1 + next_u64() % (budget / 3);
        jobs.push_back(j);
    }
    struct Run {
        Item it;
        double end;
    };
    std::vector<Run> running;
    std::map<int64_t, Admitted> blocks;
    size_t next = 0;
    double now = 0;
    int done = 0;
    size_t overtakes = 0;
    while (done < K) {
        double t_arr = next < jobs.size() ? jobs[next].arrive : 1e300;
        double t_end = 1e300;
        for (const Run &r : running) t_end = std::min(t_end, r.end);
        now = std::min(t_arr, t_end);
        for (size_t i = 0; i < running.size();) {
            if (running[i].end <= now) {
                const Item it = running[i].it;
                Job &j = jobs[it.ticket - 1];
                if (it.chunk >= 0) {
                    ++j.chunks_done;
                    CHECK(!q.item_done(it));
                } else {
                    CHECK(j.chunks_done == j.chunks);     // the finish ran after every chunk
                    CHECK(q.item_done(it));
                    j.end = now;
                    blocks.erase(it.ticket);
                    ++done;
                }
                running[i] = running.back();
                running.pop_back();
            } else {
                ++i;
            }
        }
        while (next < jobs.size() && jobs[next].arrive <= now) {
            CHECK(q.push(jobs[next].ticket, jobs[next].bytes, jobs[next].chunks, jobs[next].chunk_run, now));
            ++next;
        }
        for (const Admitted &a : q.admit(now)) {
            Job &j = jobs[a.ticket - 1];
            CHECK(!j.admitted);
            j.admitted = true;
            for (const auto &kv : blocks) overtakes += kv.first > a.ticket;   // admitted after a later request
            blocks[a.ticket] = a;
        }
        Item it;
        while (q.next_item(now, &it)) {
            Job &j = jobs[it.ticket - 1];
            CHECK(j.admitted);
            if (j.first < 0) j.first = now;
            for (const Run &r : running) CHECK(r.it.slot != it.slot);
            running.push_back({it, now + (it.chunk >= 0 ? j.chunk_run : 1e-4)});
        }
        CHECK(q.arena().in_use() <= budget);
        CHECK(q.running() == (int)running.size() && q.running() <= slots);
        size_t held = 0;
        for (const auto &kv : blocks) held += ptalm::serve::round_up(kv.second.bytes);
        CHECK(held == q.arena().in_use());
        for (auto x = blocks.begin(); x != blocks.end(); ++x)      // no two blocks overlap
            for (auto y = std::next(x); y != blocks.end(); ++y)
                CHECK(x->second.offset + ptalm::serve::round_up(x->second.bytes) <= y->second.offset ||
                      y->second.offset + ptalm::serve::round_up(y->second.bytes) <= x->second.offset);
    }
    CHECK(q.arena().in_use() == 0 && q.arena().free_blocks() == 1 && q.waiting() == 0 && q.active() == 0);
    double worst_wait = 0;
    for (const Job &j : jobs) {
        CHECK(j.first >= j.arrive && j.end > j.first);
        worst_wait = std::max(worst_wait, j.first - j.arrive);
    }
    std::printf("simulated %d requests: %zu admissions ahead of an earlier request, worst wait %.3f s\n", K,
                overtakes, worst_wait);
}

int main() {
    arena_basics();
    admission_passing_and_aging();
    items_shortest_remaining_first();
    aged_requests_go_first();
    simulated_stream();
    std::printf("OK\n");
    return 0;
}

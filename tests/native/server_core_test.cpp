// CPU test of the request server's arena and admission policy (server_core.h),
// driven by a simulated executor: requests with random footprints and run
// times arrive over simulated time; completions free slots and memory.
#include <cassert>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "server_core.h"

using ptalm::serve::Admission;
using ptalm::serve::Admitted;
using ptalm::serve::Arena;

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

static void admission_fifo_no_overtaking() {
    Admission q(1024, 4);
    CHECK(!q.push(1, 2000));             // larger than the arena: refused
    CHECK(q.push(1, 700));
    CHECK(q.push(2, 600));               // does not fit next to 1
    CHECK(q.push(3, 100));               // would fit, but must not overtake 2
    std::vector<Admitted> a = q.admit();
    CHECK(a.size() == 1 && a[0].ticket == 1);
    CHECK(q.admit().empty());
    q.complete(a[0]);
    a = q.admit();
    CHECK(a.size() == 2 && a[0].ticket == 2 && a[1].ticket == 3);
    q.complete(a[1]);
    q.complete(a[0]);
    CHECK(q.running() == 0 && q.arena().in_use() == 0);
}

static void admission_slots() {
    Admission q(1 << 20, 2);
    for (int t = 1; t <= 5; ++t) CHECK(q.push(t, 1000));
    std::vector<Admitted> a = q.admit();
    CHECK(a.size() == 2 && a[0].slot != a[1].slot);
    q.complete(a[0]);
    std::vector<Admitted> b = q.admit();
    CHECK(b.size() == 1 && b[0].ticket == 3 && b[0].slot == a[0].slot);
}

static void simulated_stream() {
    const size_t budget = 64ull << 20;
    const int slots = 4, K = 3000;
    Admission q(budget, slots);
    struct Job { int64_t ticket; double arrive, run, start = -1, end = -1; size_t bytes; };
    std::vector<Job> jobs;
    double t = 0;
    for (int k = 0; k < K; ++k) {
        t += (next_u64() % 1000) * 1e-4;
        Job j;
        j.ticket = k + 1;
        j.arrive = t;
        j.run = 0.001 + (next_u64() % 1000) * 1e-3;
        j.bytes = 1 + next_u64() % (budget / 3);
        jobs.push_back(j);
    }
    std::vector<Admitted> running;
    size_t next = 0;
    int64_t last_admitted = 0;
    double now = 0;
    int done = 0;
    while (done < K) {
        // next event: an arrival or the earliest completion
        double t_arr = next < jobs.size() ? jobs[next].arrive : 1e300;
        double t_end = 1e300;
        for (const Admitted &a : running) t_end = std::min(t_end, jobs[a.ticket - 1].end);
        now = std::min(t_arr, t_end);
        for (size_t i = 0; i < running.size();) {
            if (jobs[running[i].ticket - 1].end <= now) {
                q.complete(running[i]);
                running[i] = running.back();
                running.pop_back();
                ++done;
            } else {
                ++i;
            }
        }
        while (next < jobs.size() && jobs[next].arrive <= now) {
            CHECK(q.push(jobs[next].ticket, jobs[next].bytes));
            ++next;
        }
        for (const Admitted &a : q.admit()) {
            CHECK(a.ticket == last_admitted + 1);          // first come, first served
            last_admitted = a.ticket;
            Job &j = jobs[a.ticket - 1];
            j.start = now;
            j.end = now + j.run;
            running.push_back(a);
        }
        CHECK(q.arena().in_use() <= budget);
        CHECK(q.running() == (int)running.size() && q.running() <= slots);
        size_t held = 0;
        for (const Admitted &a : running) held += ptalm::serve::round_up(a.bytes);
        CHECK(held == q.arena().in_use());
        // no two running blocks overlap
        for (size_t i = 0; i < running.size(); ++i)
            for (size_t k = i + 1; k < running.size(); ++k) {
                const Admitted &x = running[i], &y = running[k];
                CHECK(x.offset + ptalm::serve::round_up(x.bytes) <= y.offset ||
                      y.offset + ptalm::serve::round_up(y.bytes) <= x.offset);
                CHECK(x.slot != y.slot);
            }
    }
    CHECK(q.arena().in_use() == 0 && q.arena().free_blocks() == 1 && q.waiting() == 0);
    int concurrent_max = 0;
    for (const Job &j : jobs) {
        CHECK(j.start >= j.arrive && j.end > j.start);
        int c = 0;
        for (const Job &k : jobs) c += (k.start <= j.start && j.start < k.end);
        concurrent_max = std::max(concurrent_max, c);
    }
    CHECK(concurrent_max >= 2);      // requests did overlap
    std::printf("simulated %d requests: max concurrent %d\n", K, concurrent_max);
}

int main() {
    arena_basics();
    admission_fifo_no_overtaking();
    admission_slots();
    simulated_stream();
    std::printf("OK\n");
    return 0;
}

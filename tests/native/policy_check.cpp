// Host-only checks of the server's admission policy and arena allocator
// (server_policy.h).  Prints "ok <name>" per check; exits non-zero on failure.
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "../../paper_1803_11301_amd/csrc/server_policy.h"

using namespace fpmul_srv;

static int failures = 0;
#define CHECK(c)                                                          \
    do {                                                                  \
        if (!(c)) {                                                       \
            std::printf("FAIL %s:%d %s\n", __FILE__, __LINE__, #c);       \
            ++failures;                                                   \
        }                                                                 \
    } while (0)

static Footprint toy_fp()
{
    Footprint F;
    F.single = [](uint64_t lc) { return lc; };                         // bytes = bits, for the test
    F.batch = [](uint32_t count, uint64_t max_lc) { return (uint64_t)count * max_lc; };
    return F;
}

static Req req(uint64_t t, uint64_t la, uint64_t lb)
{
    Req r;
    r.ticket = t;
    r.la = la;
    r.lb = lb;
    return r;
}

static void arena_basics()
{
    Arena A(1 << 20);
    uint64_t o1, o2, o3;
    CHECK(A.alloc(1000, o1) && o1 == 0);
    CHECK(A.alloc(256, o2) && o2 == 1024);
    CHECK(A.alloc(1, o3) && o3 == 1280);
    A.release(o2, 256);
    uint64_t o4;
    CHECK(A.alloc(200, o4) && o4 == 1024);   // first fit reuses the hole
    A.release(o1, 1000);
    A.release(o4, 200);
    A.release(o3, 1);
    CHECK(A.free_bytes() == (1u << 20) && A.largest_free() == (1u << 20));
    uint64_t big;
    CHECK(!A.alloc((1 << 20) + 1, big));
    std::printf("ok arena_basics\n");
}

static void arena_random()
{
    const uint64_t size = 1 << 22;
    Arena A(size);
    std::mt19937_64 rng(7);
    std::vector<std::pair<uint64_t, uint64_t>> live;
    std::vector<uint8_t> used(size / 256, 0);
    for (int it = 0; it < 20000; ++it) {
        if (live.empty() || rng() % 3) {
            uint64_t bytes = 1 + rng() % 70000, off;
            if (A.alloc(bytes, off)) {
                CHECK(off % 256 == 0 && off + Arena::round(bytes) <= size);
                for (uint64_t k = off / 256; k < (off + Arena::round(bytes)) / 256; ++k) {
                    CHECK(!used[k]);
                    used[k] = 1;
                }
                live.push_back({off, bytes});
            }
        } else {
            size_t i = rng() % live.size();
            auto [off, bytes] = live[i];
            for (uint64_t k = off / 256; k < (off + Arena::round(bytes)) / 256; ++k) used[k] = 0;
            A.release(off, bytes);
            live.erase(live.begin() + (long)i);
        }
    }
    for (auto &p : live) A.release(p.first, p.second);
    CHECK(A.free_bytes() == size && A.largest_free() == size);
    std::printf("ok arena_random\n");
}

static void batches_small_in_order()
{
    Policy P;
    P.batch_limit_bits = 1000;
    Arena A(1 << 20);
    std::deque<Req> q;
    for (int t = 1; t <= 5; ++t) q.push_back(req(t, 100, 100));
    Plan p;
    CHECK(next_plan(q, A, P, toy_fp(), p));
    CHECK(p.batch && p.reqs.size() == 5 && q.empty());
    for (int k = 0; k < 5; ++k) CHECK(p.reqs[k].ticket == (uint64_t)k + 1);
    CHECK(p.max_lc == 199 && p.bytes == 5 * 199);
    std::printf("ok batches_small_in_order\n");
}

static void large_runs_alone_and_batch_skips_it()
{
    Policy P;
    P.batch_limit_bits = 1000;
    Arena A(1 << 20);
    std::deque<Req> q;
    q.push_back(req(1, 100, 100));
    q.push_back(req(2, 5000, 5000));
    q.push_back(req(3, 10, 10));
    Plan p;
    CHECK(next_plan(q, A, P, toy_fp(), p));
    CHECK(p.batch && p.reqs.size() == 2 && p.reqs[0].ticket == 1 && p.reqs[1].ticket == 3);
    CHECK(q.size() == 1 && q[0].ticket == 2 && q[0].skipped == 1);
    Plan p2;
    CHECK(next_plan(q, A, P, toy_fp(), p2));
    CHECK(!p2.batch && p2.reqs.size() == 1 && p2.reqs[0].ticket == 2 && p2.bytes == 9999);
    CHECK(q.empty());
    std::printf("ok large_runs_alone_and_batch_skips_it\n");
}

static void budget_and_starvation()
{
    Policy P;
    P.batch_limit_bits = 1000;
    P.starve_after = 3;
    Arena A(20000);
    uint64_t hold;
    CHECK(A.alloc(15000, hold));   // memory taken by a launch in flight
    std::deque<Req> q;
    q.push_back(req(1, 5000, 5000));   // needs 9999 bytes: does not fit now
    for (int t = 2; t <= 10; ++t) q.push_back(req(t, 50, 50));
    int admitted = 0;
    Plan p;
    P.max_batch = 1;                   // one small request per launch
    while (next_plan(q, A, P, toy_fp(), p)) {
        CHECK(p.batch && p.reqs[0].ticket != 1);
        A.release(p.off, p.bytes);     // that launch finishes at once
        ++admitted;
    }
    CHECK(admitted == 3);              // the head was passed three times, then blocks
    CHECK(q[0].ticket == 1 && q[0].skipped == 3 && q.size() == 7);
    A.release(hold, 15000);
    CHECK(next_plan(q, A, P, toy_fp(), p));
    CHECK(!p.batch && p.reqs[0].ticket == 1);
    std::printf("ok budget_and_starvation\n");
}

static void max_batch_respected()
{
    Policy P;
    P.batch_limit_bits = 1000;
    P.max_batch = 4;
    Arena A(1 << 20);
    std::deque<Req> q;
    for (int t = 1; t <= 10; ++t) q.push_back(req(t, 10, 10));
    Plan p;
    CHECK(next_plan(q, A, P, toy_fp(), p) && p.reqs.size() == 4 && p.reqs[3].ticket == 4);
    CHECK(next_plan(q, A, P, toy_fp(), p) && p.reqs.size() == 4 && p.reqs[0].ticket == 5);
    CHECK(next_plan(q, A, P, toy_fp(), p) && p.reqs.size() == 2 && q.empty());
    std::printf("ok max_batch_respected\n");
}

static void batch_shrinks_to_fit()
{
    Policy P;
    P.batch_limit_bits = 1000;
    Arena A(1000);
    std::deque<Req> q;
    for (int t = 1; t <= 4; ++t) q.push_back(req(t, 200, 200));   // 399 bytes each, 4 do not fit
    Plan p;
    CHECK(next_plan(q, A, P, toy_fp(), p) && p.reqs.size() == 1 && p.reqs[0].ticket == 1);
    std::printf("ok batch_shrinks_to_fit\n");
}

// event-driven run: random arrivals, 3 slots, launches finish after a time
// proportional to their bytes; every request is served, the arena is never
// over-committed and all memory comes back
static void simulated_stream()
{
    Policy P;
    P.batch_limit_bits = 4000;
    P.starve_after = 8;
    const uint64_t budget = 60000;
    Arena A(budget);
    std::mt19937_64 rng(11);
    std::deque<Req> q;
    struct Run { Plan p; double end; };
    std::vector<Run> running;
    std::vector<int> served(2001, 0);
    double now = 0;
    int next = 1;
    uint64_t in_use = 0, peak = 0;
    while (next <= 2000 || !q.empty() || !running.empty()) {
        if (next <= 2000 && rng() % 2) {
            uint64_t la = 1 + rng() % (rng() % 4 ? 1500 : 12000), lb = 1 + rng() % 1500;
            q.push_back(req(next++, la, lb));
        }
        for (size_t i = 0; i < running.size();) {
            if (running[i].end <= now) {
                A.release(running[i].p.off, running[i].p.bytes);
                in_use -= Arena::round(running[i].p.bytes);
                running.erase(running.begin() + (long)i);
            } else {
                ++i;
            }
        }
        while (running.size() < 3) {
            Plan p;
            if (!next_plan(q, A, P, toy_fp(), p)) break;
            in_use += Arena::round(p.bytes);
            peak = in_use > peak ? in_use : peak;
            for (auto &r : p.reqs) served[r.ticket]++;
            running.push_back({p, now + 1 + p.bytes / 5000.0});
        }
        now += 0.5;
        CHECK(now < 1e6);
        if (now >= 1e6) break;
    }
    for (int t = 1; t <= 2000; ++t) CHECK(served[t] == 1);
    CHECK(peak <= budget && A.free_bytes() == budget - (budget % 256 ? budget % 256 : 0));
    std::printf("ok simulated_stream peak=%llu\n", (unsigned long long)peak);
}

// a product on a resident operand's kept transform is never batched, even
// when it is short, and reserves the single-launch footprint of the resident
// transform length, not of its own product length
static void resident_runs_alone_at_its_length()
{
    Policy P;
    P.batch_limit_bits = 1000;
    Arena A(1 << 20);
    std::deque<Req> q;
    static const uint64_t fa = 0;
    q.push_back(req(1, 10, 10));
    Req r = req(2, 20, 20);
    r.fa = &fa;
    r.res_log2n = 12;
    q.push_back(r);
    q.push_back(req(3, 30, 30));
    Plan p;
    CHECK(next_plan(q, A, P, toy_fp(), p));
    CHECK(p.batch && p.reqs.size() == 2 && p.reqs[0].ticket == 1 && p.reqs[1].ticket == 3);
    CHECK(q.size() == 1 && q[0].ticket == 2);
    Plan p2;
    CHECK(next_plan(q, A, P, toy_fp(), p2));
    CHECK(!p2.batch && p2.reqs.size() == 1 && p2.reqs[0].ticket == 2 && p2.reqs[0].fa == &fa);
    CHECK(p2.bytes == 4096 && p2.max_lc == 4096);
    CHECK(q.empty());
    std::printf("ok resident_runs_alone_at_its_length\n");
}

int main()
{
    resident_runs_alone_at_its_length();
    arena_basics();
    arena_random();
    batches_small_in_order();
    large_runs_alone_and_batch_skips_it();
    budget_and_starvation();
    max_batch_respected();
    batch_shrinks_to_fit();
    simulated_stream();
    if (failures) {
        std::printf("%d failures\n", failures);
        return 1;
    }
    std::printf("all ok\n");
    return 0;
}

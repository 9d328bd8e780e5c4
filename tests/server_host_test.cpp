// Host test of the served form's logic (arena, admission, tick loop,
// tickets) with a test double in place of the GPU executor.  Built with g++
// under the address, undefined-behaviour or thread sanitizer by
// test_server_host.py; prints one line per check and exits non-zero on the
// first failure.  The double computes nothing: it checks the contract the
// core must keep with a device (a tick slot is reused only after its wait,
// a running request's arena block is never touched by another request) and
// returns a result that identifies the request and its step count, so that
// a result delivered to the wrong ticket, a lost step or an overlapping
// block is seen.
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>

#include <atomic>
#include <random>
#include <set>
#include <string>

#include "server_core.hpp"

namespace kl {
namespace {
thread_local std::string g_err;
}
int fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}
void clear_error() { g_err.clear(); }
}  // namespace kl

using namespace kl;
using served::Req;

#define CHECK(c)                                                               \
    do {                                                                       \
        if (!(c)) {                                                            \
            fprintf(stderr, "FAILED %s:%d: %s\n", __FILE__, __LINE__, #c);     \
            exit(1);                                                           \
        }                                                                      \
    } while (0)

constexpr uint64_t FAIL_SEED = 0xdead;

struct FakeExec {
    std::mutex mu;
    bool busy[2] = {false, false};       // slot recorded and not yet waited for
    std::atomic<int64_t> ticks{0};
    int delay_us = 50;

    size_t footprint(const kl_request_t &q, int64_t *off, int64_t *js, int64_t *ks, int64_t *alloc)
    {
        *off = 0;
        *js = q.itot + 2;
        *ks = *js * (q.jtot + 2);
        *alloc = *ks * (q.ktot + 2);
        return served::round_up((size_t)q.itot * q.jtot * q.ktot * (q.dtype == KL_F32 ? 4 : 8)) + served::ALIGN;
    }
    static unsigned char pattern(const Req &q) { return (unsigned char)(1 + q.ticket % 251); }
    int init_request(Req &q, char *block)
    {
        memset(block, pattern(q), q.bytes);  // the request's whole block
        q.f[0] = block;
        q.g.off = 0;
        q.checksum[0] = 0;
        q.dt = 0.1;
        return KL_OK;
    }
    int run_tick(int slot, const std::vector<Req *> &active, int64_t *launches)
    {
        {
            std::lock_guard<std::mutex> lk(mu);
            CHECK(!busy[slot]);  // the core waits for a slot's previous tick before reusing it
        }
        for (Req *q : active) {
            CHECK(q->state == 1);
            // no other request has written into this one's block (checked on
            // the server thread, which alone writes blocks)
            const unsigned char *p = (const unsigned char *)q->f[0];
            for (size_t b = 0; b < q->bytes; b += 61) CHECK(p[b] == pattern(*q));
            if (q->r.seed == FAIL_SEED) return fail(KL_ERR_DEVICE, "injected device error");
            q->checksum[0] += 1;  // one more step of this request
        }
        *launches += 1;
        ++ticks;
        return KL_OK;
    }
    int enqueue_checksums(const std::vector<Req *> &done, int64_t *launches)
    {
        for (Req *q : done) {
            q->checksum[1] = (double)q->r.seed;
            q->checksum[2] = (double)q->ticket;
        }
        *launches += (int64_t)done.size();
        return KL_OK;
    }
    int record(int slot)
    {
        std::lock_guard<std::mutex> lk(mu);
        busy[slot] = true;
        return KL_OK;
    }
    int wait(int slot)
    {
        if (delay_us) std::this_thread::sleep_for(std::chrono::microseconds(delay_us));
        std::lock_guard<std::mutex> lk(mu);
        CHECK(busy[slot]);
        busy[slot] = false;
        return KL_OK;
    }
    int fetch_checksum(Req &) { return KL_OK; }
    void thread_init() {}
};

typedef served::Server<FakeExec> Server;

struct Harness {
    std::vector<char> arena;
    Server *S;
    Harness(size_t arena_bytes, size_t budget) : arena(arena_bytes)
    {
        S = new Server(arena.data(), arena_bytes, budget);
        S->th = std::thread(served::server_loop<FakeExec>, S);
    }
    ~Harness()
    {
        served::shutdown(*S);
        delete S;
    }
};

kl_request_t req(int n, int steps, uint64_t seed, int dtype = KL_F32)
{
    kl_request_t r;
    memset(&r, 0, sizeof r);
    r.itot = n;
    r.jtot = n;
    r.ktot = n;
    r.dtype = dtype;
    r.bc = KL_BC_ZWALL_ZEROGRAD;
    r.nsteps = steps;
    r.seed = seed;
    return r;
}

int wait_done(Server &S, uint64_t t, kl_result_t *out)
{
    for (int n = 0; n < 200000; ++n) {
        const int rc = served::poll(S, t, out);
        if (rc != KL_ERR_AGAIN) return rc;
        std::this_thread::sleep_for(std::chrono::microseconds(20));
    }
    return KL_ERR_AGAIN;
}

void test_arena()
{
    const size_t cap = 1 << 20;
    served::Arena a(cap);
    std::vector<unsigned char> owner(cap / 16, 0);  // 16-byte granules
    std::mt19937_64 rng(7);
    std::vector<std::pair<size_t, size_t>> live;
    for (int it = 0; it < 20000; ++it) {
        if (live.empty() || rng() % 3) {
            const size_t bytes = 16 * (1 + rng() % 512);
            size_t off;
            if (a.alloc(bytes, &off)) {
                CHECK(off % 16 == 0 && off + bytes <= cap);
                for (size_t g = off / 16; g < (off + bytes) / 16; ++g) {
                    CHECK(owner[g] == 0);  // no overlap with a live block
                    owner[g] = 1;
                }
                live.push_back({off, bytes});
            }
        } else {
            const size_t k = rng() % live.size();
            const auto b = live[k];
            live[k] = live.back();
            live.pop_back();
            for (size_t g = b.first / 16; g < (b.first + b.second) / 16; ++g) owner[g] = 0;
            a.release(b.first, b.second);
        }
        // free blocks never touch each other (coalesced) and never cover a live granule
        size_t end = (size_t)-1;
        for (const auto &f : a.free_blocks()) {
            CHECK(f.first != end);
            end = f.first + f.second;
            for (size_t g = f.first / 16; g < end / 16; g += 7) CHECK(owner[g] == 0);
        }
    }
    for (const auto &b : live) a.release(b.first, b.second);
    CHECK(a.free_blocks().size() == 1 && a.free_blocks().begin()->second == cap);
    printf("ok arena: 20000 random allocations and frees, no overlap, frees coalesce\n");
}

void test_admission_fifo_and_budget()
{
    // budget for about three requests of 32^3 FP32 at a time
    const size_t one = served::round_up(32 * 32 * 32 * 4) + served::ALIGN;
    Harness h(64 << 20, 3 * one + one / 2);
    std::vector<uint64_t> tickets;
    for (int n = 0; n < 40; ++n) {
        uint64_t t;
        kl_request_t r = req(32, 1 + n % 5, 1000 + n);
        CHECK(served::submit(*h.S, &r, &t) == KL_OK);
        tickets.push_back(t);
    }
    int64_t last_admit = 0;
    for (size_t n = 0; n < tickets.size(); ++n) {
        kl_result_t out;
        CHECK(wait_done(*h.S, tickets[n], &out) == KL_OK);
        CHECK(out.state == 2 && out.err == 0);
        CHECK(out.checksum[0] == (double)(1 + n % 5));  // every step ran, once
        CHECK(out.checksum[1] == (double)(1000 + n) && out.checksum[2] == (double)tickets[n]);
        CHECK(out.t_admit_ns >= last_admit);  // admitted in arrival order
        last_admit = out.t_admit_ns;
        CHECK(out.t_done_ns >= out.t_admit_ns && out.t_admit_ns >= out.t_arrive_ns);
        CHECK(served::release(*h.S, tickets[n]) == KL_OK);
    }
    int64_t st[5];
    served::stats(*h.S, st);
    CHECK(st[2] == 40);
    CHECK((size_t)st[3] <= 3 * one + one / 2);  // peak bytes within the budget
    CHECK(h.S->used == 0);
    printf("ok admission: 40 requests in arrival order, peak %lld <= budget, all steps, results to their tickets\n",
           (long long)st[3]);
}

void test_errors()
{
    Harness h(1 << 20, 1 << 16);
    uint64_t t;
    kl_request_t big = req(64, 1, 1);  // 1 MiB of fields > 64 KiB budget
    CHECK(served::submit(*h.S, &big, &t) == KL_ERR_BUDGET);
    kl_request_t bad = req(0, 1, 1);
    CHECK(served::submit(*h.S, &bad, &t) == KL_ERR_INVALID);
    bad = req(8, 0, 1);
    CHECK(served::submit(*h.S, &bad, &t) == KL_ERR_INVALID);
    bad = req(8, 1, 1);
    bad.dtype = 7;
    CHECK(served::submit(*h.S, &bad, &t) == KL_ERR_INVALID);
    kl_result_t out;
    CHECK(served::poll(*h.S, 12345, &out) == KL_ERR_NOTFOUND);
    CHECK(served::release(*h.S, 12345) == KL_ERR_NOTFOUND);
    // release before the end is refused; a second release is unknown
    h.S->exec.delay_us = 2000;
    kl_request_t r = req(8, 50, 2);
    CHECK(served::submit(*h.S, &r, &t) == KL_OK);
    CHECK(served::release(*h.S, t) == KL_ERR_AGAIN);
    CHECK(wait_done(*h.S, t, &out) == KL_OK);
    CHECK(served::release(*h.S, t) == KL_OK);
    CHECK(served::release(*h.S, t) == KL_ERR_NOTFOUND);
    printf("ok errors: budget, invalid sizes and dtype, unknown ticket, early and double release\n");
}

void test_device_error()
{
    Harness h(16 << 20, 16 << 20);
    std::vector<uint64_t> before, after;
    uint64_t bad;
    for (int n = 0; n < 5; ++n) {
        uint64_t t;
        kl_request_t r = req(16, 3, 10 + n);
        CHECK(served::submit(*h.S, &r, &t) == KL_OK);
        before.push_back(t);
    }
    for (auto t : before) {
        kl_result_t out;
        CHECK(wait_done(*h.S, t, &out) == KL_OK && out.state == 2);
    }
    kl_request_t r = req(16, 3, FAIL_SEED);
    CHECK(served::submit(*h.S, &r, &bad) == KL_OK);
    kl_result_t out;
    CHECK(wait_done(*h.S, bad, &out) == KL_OK);
    CHECK(out.state == 3 && out.err == KL_ERR_DEVICE);  // the failed tick's request fails
    CHECK(served::release(*h.S, bad) == KL_OK);
    for (int n = 0; n < 5; ++n) {
        uint64_t t;
        kl_request_t q = req(16, 2, 20 + n);
        CHECK(served::submit(*h.S, &q, &t) == KL_OK);
        after.push_back(t);
    }
    for (auto t : after) {
        CHECK(wait_done(*h.S, t, &out) == KL_OK);
        CHECK(out.state == 2 && out.checksum[0] == 2.0);  // later requests are not blocked
    }
    printf("ok device error: the failing request ends failed, the ones after it finish\n");
}

void test_concurrent_clients()
{
    const size_t budget = 4 << 20;
    Harness h(budget + (1 << 20), budget);
    h.S->exec.delay_us = 20;
    std::atomic<int> okc{0};
    std::vector<std::thread> clients;
    for (int c = 0; c < 4; ++c) {
        clients.emplace_back([&, c] {
            std::mt19937 rng(100 + c);
            std::vector<std::pair<uint64_t, kl_request_t>> mine;
            for (int n = 0; n < 150; ++n) {
                const int sizes[4] = {8, 16, 24, 40};
                kl_request_t r = req(sizes[rng() % 4], 1 + rng() % 6, (uint64_t)(c * 1000 + n), rng() % 4 ? KL_F32 : KL_F64);
                uint64_t t;
                CHECK(served::submit(*h.S, &r, &t) == KL_OK);
                mine.push_back({t, r});
                if (rng() % 3 == 0) {  // poll and release some early ones while others run
                    kl_result_t out;
                    const auto &m = mine[rng() % mine.size()];
                    const int rc = served::poll(*h.S, m.first, &out);
                    CHECK(rc == KL_OK || rc == KL_ERR_AGAIN || rc == KL_ERR_NOTFOUND);
                }
            }
            for (const auto &m : mine) {
                kl_result_t out;
                CHECK(wait_done(*h.S, m.first, &out) == KL_OK);
                CHECK(out.state == 2 && out.checksum[0] == (double)m.second.nsteps);
                CHECK(out.checksum[1] == (double)m.second.seed && out.checksum[2] == (double)m.first);
                CHECK(served::release(*h.S, m.first) == KL_OK);
                ++okc;
            }
        });
    }
    for (auto &t : clients) t.join();
    CHECK(okc == 600);
    {
        std::lock_guard<std::mutex> lk(h.S->mu);
        CHECK(h.S->used == 0);
        CHECK(h.S->arena.free_blocks().size() == 1);
    }
    int64_t st[5];
    served::stats(*h.S, st);
    CHECK((size_t)st[3] <= budget);
    printf("ok concurrent clients: 4 threads x 150 requests submitted, polled and released while ticks run; "
           "arena whole again, peak %lld <= budget\n", (long long)st[3]);
}

void test_shutdown_with_work()
{
    Harness *h = new Harness(8 << 20, 8 << 20);
    h->S->exec.delay_us = 500;
    for (int n = 0; n < 20; ++n) {
        uint64_t t;
        kl_request_t r = req(16, 10, n);
        CHECK(served::submit(*h->S, &r, &t) == KL_OK);
    }
    delete h;  // stops the loop with work queued and running; frees every request
    printf("ok shutdown with requests queued and running\n");
}

int main()
{
    test_arena();
    test_admission_fifo_and_budget();
    test_errors();
    test_device_error();
    test_concurrent_clients();
    test_shutdown_with_work();
    printf("ALL OK\n");
    return 0;
}

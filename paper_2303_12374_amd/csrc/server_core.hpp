// Host logic of the served form, independent of the device: the arena
// sub-allocator, admission in arrival order under the memory budget, the
// request state machine, the tick loop that keeps one tick in flight while
// the next is prepared, and the ticket calls (submit, poll, release, stats,
// destroy).  All device work goes through an executor `Exec`, so the same
// logic runs against the GPU (server.hip) and against a host test double
// (tests), which is how admission, the arena and the tick pipeline are
// exercised, under the address, undefined-behaviour and thread sanitizers,
// on a machine without a GPU.
//
// Exec provides:
//   size_t footprint(const kl_request_t &, int64_t *off, int64_t *js, int64_t *ks, int64_t *alloc);
//   int init_request(Req &q, char *block);            // lay out and fill a newly admitted request
//   int run_tick(int slot, const std::vector<Req *> &active, int64_t *launches);
//   int enqueue_checksums(const std::vector<Req *> &done, int64_t *launches);
//   int record(int slot);                             // mark the end of the tick's work
//   int wait(int slot);                               // wait for it
//   int fetch_checksum(Req &q);                       // after wait: q.checksum from the device
//   void thread_init();                               // on the server thread before the loop
// Each returns KL_OK or a kl_status_t (after recording a message with fail()).
#pragma once

#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "kl.h"

namespace kl {

int fail(int code, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
void clear_error();

namespace served {

constexpr size_t ALIGN = 256;
inline size_t round_up(size_t x) { return (x + ALIGN - 1) / ALIGN * ALIGN; }

inline int64_t now_ns()
{
    return std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

// First-fit sub-allocator over [0, cap) with coalescing frees.
class Arena {
   public:
    explicit Arena(size_t cap) { free_[0] = cap; }
    bool alloc(size_t bytes, size_t *off)
    {
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                *off = it->first;
                const size_t rest = it->second - bytes, start = it->first + bytes;
                free_.erase(it);
                if (rest) free_[start] = rest;
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t bytes)
    {
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
    // free blocks (offset -> bytes), for tests and statistics
    const std::map<size_t, size_t> &free_blocks() const { return free_; }

   private:
    std::map<size_t, size_t> free_;
};

struct Req {
    uint64_t ticket = 0;
    kl_request_t r;
    int state = 0, err = 0;  // 0 queued, 1 running, 2 done, 3 failed
    int64_t t_arrive = 0, t_admit = 0, t_done = 0;
    int steps_left = 0;
    size_t off = 0, bytes = 0;
    int cur = 0;  // the state is in f[3*cur .. 3*cur+2]; the other three take the next step
    double dt = 0;
    kl_grid_t g;
    void *f[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
    double checksum[9];
    std::vector<char> metrics;  // host copy of dzi | dzhi in the field dtype
};

template <class Exec>
struct Server {
    char *base = nullptr;
    size_t arena_bytes = 0, budget = 0, used = 0, peak = 0;
    Arena arena{0};
    std::mutex mu;
    std::condition_variable cv;
    std::deque<Req *> queue;
    std::vector<Req *> active;
    std::unordered_map<uint64_t, Req *> reqs;
    uint64_t next_ticket = 1;
    bool stop = false;
    std::thread th;
    int64_t ticks = 0, launches = 0, ndone = 0, point_steps = 0;
    Exec exec;

    Server(void *arena_ptr, size_t ab, size_t bb) : base((char *)arena_ptr), arena_bytes(ab), budget(bb), arena(ab) {}
};

// A tick whose work is enqueued but not known to be complete.
struct InFlight {
    int slot;
    int rc;
    int64_t pts;
    std::vector<Req *> finishing;
};

// Wait for the oldest tick in flight and publish the requests it finished.
template <class Exec>
void complete(Server<Exec> &S, std::deque<InFlight> &inflight)
{
    InFlight t = inflight.front();
    inflight.pop_front();
    int rc = t.rc;
    if (rc == KL_OK) rc = S.exec.wait(t.slot);
    for (Req *q : t.finishing)
        if (rc == KL_OK) rc = S.exec.fetch_checksum(*q);
    const int64_t now = now_ns();
    std::lock_guard<std::mutex> lk(S.mu);
    ++S.ticks;
    if (rc == KL_OK) S.point_steps += t.pts;
    for (Req *q : t.finishing) {
        q->state = rc == KL_OK ? 2 : 3;
        q->err = rc;
        q->t_done = now;
        ++S.ndone;
    }
    S.cv.notify_all();
}

template <class Exec>
void server_loop(Server<Exec> *Sp)
{
    Server<Exec> &S = *Sp;
    S.exec.thread_init();
    std::deque<InFlight> inflight;  // at most one tick waits while the next is prepared
    int64_t tick = 0;
    for (;;) {
        std::vector<Req *> fresh;
        bool idle = false;
        {
            std::unique_lock<std::mutex> lk(S.mu);
            for (;;) {
                // admission in arrival order while the head fits budget and arena
                while (!S.queue.empty()) {
                    Req *q = S.queue.front();
                    if (S.used + q->bytes > S.budget) break;
                    size_t off;
                    if (!S.arena.alloc(q->bytes, &off)) break;
                    q->off = off;
                    S.used += q->bytes;
                    S.peak = std::max(S.peak, S.used);
                    q->state = 1;
                    q->t_admit = now_ns();
                    q->steps_left = q->r.nsteps;
                    S.queue.pop_front();
                    S.active.push_back(q);
                    fresh.push_back(q);
                }
                if (!S.active.empty()) break;
                if (!inflight.empty()) {
                    idle = true;  // nothing to enqueue: retire the tick in flight first
                    break;
                }
                if (S.stop) {
                    // nothing runs and the head cannot be admitted now: fail what is left
                    for (Req *q : S.queue) {
                        q->state = 3;
                        q->err = KL_ERR_BUDGET;
                        q->t_done = now_ns();
                    }
                    S.queue.clear();
                    return;
                }
                S.cv.wait(lk);
            }
        }
        if (idle) {
            complete(S, inflight);
            continue;
        }
        const int slot = (int)(tick & 1);
        int rc = KL_OK;
        for (Req *q : fresh)
            if (rc == KL_OK) rc = S.exec.init_request(*q, S.base + q->off);
        int64_t nl = 0;
        if (rc == KL_OK) rc = S.exec.run_tick(slot, S.active, &nl);
        InFlight t{slot, rc, 0, {}};
        std::vector<Req *> still;
        for (Req *q : S.active) {
            --q->steps_left;
            t.pts += (int64_t)q->r.itot * q->r.jtot * q->r.ktot;
            if (rc == KL_OK) q->cur ^= 1;
            if (q->steps_left == 0 || rc != KL_OK)
                t.finishing.push_back(q);
            else
                still.push_back(q);
        }
        if (rc == KL_OK) rc = S.exec.enqueue_checksums(t.finishing, &nl);
        if (rc == KL_OK) rc = S.exec.record(slot);
        t.rc = rc;
        {
            std::lock_guard<std::mutex> lk(S.mu);
            S.launches += nl;
            if (rc != KL_OK) {  // a failed tick fails every request it carried
                for (Req *q : still) t.finishing.push_back(q);
                still.clear();
            }
            S.active.swap(still);
        }
        inflight.push_back(t);
        ++tick;
        // keep one tick queued on the device while the host prepares the next
        while (inflight.size() > 1) complete(S, inflight);
    }
}

template <class Exec>
int submit(Server<Exec> &S, const kl_request_t *req, uint64_t *ticket)
{
    const kl_request_t &r = *req;
    if (r.itot < 1 || r.jtot < 1 || r.ktot < 1 || (r.bc != KL_BC_ZPERIODIC && r.ktot < 2))
        return fail(KL_ERR_INVALID, "request sizes %d x %d x %d", r.itot, r.jtot, r.ktot);
    if (r.dtype != KL_F32 && r.dtype != KL_F64) return fail(KL_ERR_INVALID, "request dtype %d", r.dtype);
    if (r.bc < 0 || r.bc > 2) return fail(KL_ERR_INVALID, "request bc %d", r.bc);
    if (r.nsteps < 1) return fail(KL_ERR_INVALID, "request nsteps %d", r.nsteps);
    Req *q = new (std::nothrow) Req();
    if (!q) return fail(KL_ERR_NOMEM, "request");
    q->r = r;
    int64_t off, js, ks, alloc;
    q->bytes = S.exec.footprint(r, &off, &js, &ks, &alloc);
    if (q->bytes > S.budget) {
        const size_t b = q->bytes;
        delete q;
        return fail(KL_ERR_BUDGET, "request needs %zu bytes, budget is %zu", b, S.budget);
    }
    q->t_arrive = now_ns();
    std::lock_guard<std::mutex> lk(S.mu);
    if (S.stop) {
        delete q;
        return fail(KL_ERR_INVALID, "server is stopping");
    }
    q->ticket = S.next_ticket++;
    S.reqs[q->ticket] = q;
    S.queue.push_back(q);
    *ticket = q->ticket;
    S.cv.notify_all();
    return KL_OK;
}

template <class Exec>
int poll(Server<Exec> &S, uint64_t ticket, kl_result_t *out)
{
    std::lock_guard<std::mutex> lk(S.mu);
    auto it = S.reqs.find(ticket);
    if (it == S.reqs.end()) return fail(KL_ERR_NOTFOUND, "ticket %llu", (unsigned long long)ticket);
    const Req &q = *it->second;
    memset(out, 0, sizeof *out);
    out->state = q.state;
    out->err = q.err;
    out->t_arrive_ns = q.t_arrive;
    out->t_admit_ns = q.t_admit;
    out->t_done_ns = q.t_done;
    if (q.state >= 2) {
        memcpy(out->checksum, q.checksum, sizeof q.checksum);
        for (int n = 0; n < 3; ++n) out->fields[n] = q.f[3 * q.cur + n];
        out->off = q.g.off;
        out->jstride = q.g.jstride;
        out->kstride = q.g.kstride;
        return KL_OK;
    }
    return KL_ERR_AGAIN;
}

template <class Exec>
int release(Server<Exec> &S, uint64_t ticket)
{
    std::lock_guard<std::mutex> lk(S.mu);
    auto it = S.reqs.find(ticket);
    if (it == S.reqs.end()) return fail(KL_ERR_NOTFOUND, "ticket %llu", (unsigned long long)ticket);
    Req *q = it->second;
    if (q->state < 2) return fail(KL_ERR_AGAIN, "ticket %llu is not finished", (unsigned long long)ticket);
    if (q->t_admit) {  // admitted requests hold an arena block until released
        S.arena.release(q->off, q->bytes);
        S.used -= q->bytes;
    }
    S.reqs.erase(it);
    delete q;
    S.cv.notify_all();
    return KL_OK;
}

template <class Exec>
void stats(Server<Exec> &S, int64_t out[5])
{
    std::lock_guard<std::mutex> lk(S.mu);
    out[0] = S.ticks;
    out[1] = S.launches;
    out[2] = S.ndone;
    out[3] = (int64_t)S.peak;
    out[4] = S.point_steps;
}

// Stop the loop (it fails the requests still queued once nothing runs) and
// free every request.
template <class Exec>
void shutdown(Server<Exec> &S)
{
    {
        std::lock_guard<std::mutex> lk(S.mu);
        S.stop = true;
        S.cv.notify_all();
    }
    if (S.th.joinable()) S.th.join();
    for (auto &kv : S.reqs) delete kv.second;
    S.reqs.clear();
}

}  // namespace served
}  // namespace kl

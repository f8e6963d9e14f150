// Request server core: tickets, the payload pool, admission, continuous batching and
// completion (see include/vnp_server.h).  Host code only: the device work is behind a
// backend B, so the same core runs with the HIP backend in the library and with a CPU
// stand-in under ThreadSanitizer in the tests.
//
// One batcher thread owns the launches.  Clients submit requests (host bookkeeping
// only); the batcher moves pending requests into a free stream slot and hands the batch to
// the backend (B::launch), which enqueues it and records a completion event.  Each slot
// has a completion thread that waits for its batch (B::wait), posts the results to the
// tickets, frees the pool blocks of copied payloads and wakes waiters and the batcher.
// With several slots, requests that arrive while batches run are launched on another
// stream and overlap on the device.
//
// Admission by device memory: a request submitted with a copy (submit with copy = true)
// gets a pool block of its payload's size when the batcher takes it, in arrival order among
// such requests; if the pool cannot hold it, it and every later copy request wait
// (back-pressure) until a completion or a client frees memory.  Requests that need no pool
// memory pass them.
//
// The batcher and the completion threads poll for new work for up to SPIN_NS before they
// block on a condition variable: waking a blocked thread takes longer than a small batch
// runs on the device.
//
// Backend interface (B):
//   struct SlotData;                                   per-slot device resources
//   int init(const vnp_server_config &, char **pool);  device pool (and device context)
//   void fini(char *pool);
//   int slot_init(SlotData &, const vnp_server_config &);
//   void slot_fini(SlotData &);
//   void thread_start();                               in every server thread
//   int launch(SlotData &, std::vector<Pending> &reqs, int *nlaunch);
//       enqueue the batch (may reorder reqs; result i belongs to reqs[i] afterwards)
//   int wait(SlotData &, int launch_rc);               block until the batch has completed
//   double result(const SlotData &, size_t i, const vnp_request &);
#pragma once
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/vnp_server.h"

namespace vnp {
namespace srv {

inline int64_t now_ns()
{
    return std::chrono::duration_cast<std::chrono::nanoseconds>(std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

constexpr int64_t SPIN_NS = 200000;  // busy-poll window before blocking

// Polls seq until it differs from seen (true) or spin_ns pass (false).
inline bool spin_until_changed(const std::atomic<uint64_t> &seq, uint64_t seen, int64_t spin_ns)
{
    const int64_t t0 = now_ns();
    while (seq.load(std::memory_order_acquire) == seen) {
        if (now_ns() - t0 > spin_ns) return false;
        std::this_thread::yield();
    }
    return true;
}

// First-fit allocator over one device allocation, 256-byte granules, with coalescing.
struct Pool {
    char *base = nullptr;
    uint64_t size = 0;
    std::map<uint64_t, uint64_t> free_;  // offset -> size
    std::map<uint64_t, uint64_t> used_;  // offset -> size
    uint64_t free_bytes = 0;

    static uint64_t granule(uint64_t bytes) { return (bytes + 255) & ~uint64_t(255); }
    void init(char *b, uint64_t s)
    {
        base = b;
        size = s;
        free_.clear();
        used_.clear();
        if (s) free_[0] = s;
        free_bytes = s;
    }
    void *alloc(uint64_t bytes)
    {
        const uint64_t need = granule(bytes);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= need) {
                const uint64_t off = it->first, rest = it->second - need;
                free_.erase(it);
                if (rest) free_[off + need] = rest;
                used_[off] = need;
                free_bytes -= need;
                return base + off;
            }
        }
        return nullptr;
    }
    bool release(void *p)
    {
        if (!p || static_cast<char *>(p) < base) return false;
        const uint64_t off = (uint64_t)(static_cast<char *>(p) - base);
        auto u = used_.find(off);
        if (u == used_.end()) return false;
        uint64_t start = off, len = u->second;
        used_.erase(u);
        free_bytes += len;
        auto nx = free_.lower_bound(start);
        if (nx != free_.end() && nx->first == start + len) {
            len += nx->second;
            nx = free_.erase(nx);
        }
        if (nx != free_.begin()) {
            auto pv = std::prev(nx);
            if (pv->first + pv->second == start) {
                start = pv->first;
                len += pv->second;
                free_.erase(pv);
            }
        }
        free_[start] = len;
        return true;
    }
};

struct Pending {
    uint64_t ticket;
    vnp_request req;
    int64_t t_submit;
    bool solo;         // rerun alone after an injected batch failure
    bool copy;         // the payload is copied into a pool block at admission
    void *blk;         // that block, once admitted
    int64_t t_blocked; // when admission first found the pool full (0: never)
};

struct Ticket {
    vnp_result r;
    bool done;
};

inline int64_t payload_bytes(const vnp_request &q) { return q.n * (q.dtype == VNP_F32 ? 4 : 8); }

enum class SlotState { Free, Launching, InFlight };

template <class B>
struct Slot {
    typename B::SlotData d;
    std::vector<Pending> reqs;
    SlotState state = SlotState::Free;
    int launch_rc = 0;
    int64_t t_enqueued = 0;
    std::thread done_thread;
};

template <class B>
struct Server {
    B be;
    vnp_server_config cfg{};
    Pool pool;
    std::mutex mu;
    std::condition_variable cv_work, cv_done, cv_slots, cv_left;
    std::deque<Pending> pending;
    std::unordered_map<uint64_t, Ticket> tickets;
    std::vector<Slot<B>> slots;
    std::thread worker;
    bool stop = false;
    int waiters = 0;  // threads blocked in wait
    // Bumped under mu whenever the batcher may have work (a request queued, a slot freed,
    // stop), and per slot whenever the slot's batch is in flight (or stop): the polled
    // change counters of the busy-poll phase.
    std::atomic<uint64_t> work_seq{0};
    std::unique_ptr<std::atomic<uint64_t>[]> flight_seq;
    uint64_t next_ticket = 1;
    int64_t nocopy_pending = 0;  // queued requests submitted without copy
    vnp_server_stats st{};
    int64_t batch_counter = 0;

    // --- set-up and tear-down -------------------------------------------------------
    int create(const vnp_server_config &c)
    {
        cfg = c;
        char *base = nullptr;
        int rc = be.init(cfg, &base);
        if (rc) return rc;
        pool.init(base, (uint64_t)cfg.pool_bytes);
        slots = std::vector<Slot<B>>((size_t)cfg.streams);
        flight_seq.reset(new (std::nothrow) std::atomic<uint64_t>[(size_t)cfg.streams]);
        if (!flight_seq) rc = VNP_ENOMEM;
        for (int k = 0; !rc && k < cfg.streams; ++k) flight_seq[k].store(0, std::memory_order_relaxed);
        for (size_t i = 0; !rc && i < slots.size(); ++i) rc = be.slot_init(slots[i].d, cfg);
        if (rc) {
            release_resources();
            return rc;
        }
        st.pool_bytes = cfg.pool_bytes;
        for (size_t i = 0; i < slots.size(); ++i) slots[i].done_thread = std::thread([this, i] { completion_loop(i); });
        worker = std::thread([this] { worker_loop(); });
        return 0;
    }

    void release_resources()
    {
        for (Slot<B> &sl : slots) be.slot_fini(sl.d);
        slots.clear();
        be.fini(pool.base);
        pool.base = nullptr;
    }

    // Requests not yet launched complete as cancelled; batches in flight finish; blocked
    // waiters return before the resources go.
    void destroy()
    {
        {
            std::lock_guard<std::mutex> lk(mu);
            stop = true;
            const int64_t t = now_ns();
            for (const Pending &p : pending) {
                auto it = tickets.find(p.ticket);
                if (it != tickets.end()) {
                    it->second.r.status = VNP_ECANCELED;
                    it->second.r.value = __builtin_nan("");
                    it->second.r.t_done_ns = t;
                    it->second.done = true;
                    st.cancelled += 1;
                }
                if (p.blk) pool.release(p.blk);
            }
            pending.clear();
            nocopy_pending = 0;
            work_seq.fetch_add(1, std::memory_order_release);
        }
        cv_done.notify_all();
        cv_work.notify_all();
        if (worker.joinable()) worker.join();
        {
            std::lock_guard<std::mutex> lk(mu);  // the batcher has stopped: no slot is Launching
            for (size_t k = 0; k < slots.size(); ++k) flight_seq[k].fetch_add(1, std::memory_order_release);
        }
        cv_slots.notify_all();
        for (Slot<B> &sl : slots)
            if (sl.done_thread.joinable()) sl.done_thread.join();  // in-flight batches complete first
        {
            std::unique_lock<std::mutex> lk(mu);
            cv_done.notify_all();
            cv_left.wait(lk, [this] { return waiters == 0; });
        }
        release_resources();
    }

    // --- completion -------------------------------------------------------------------
    // Posts the slot's results (status 0) or the error to its tickets, frees its copied
    // payloads and frees the slot.  Called with mu held.
    void complete(Slot<B> &s, int status)
    {
        const int64_t t = now_ns();
        if (s.t_enqueued) {
            st.batch_ns += t - s.t_enqueued;
            st.batch_ns_max = std::max<int64_t>(st.batch_ns_max, t - s.t_enqueued);
            s.t_enqueued = 0;
        }
        for (size_t i = 0; i < s.reqs.size(); ++i) {
            Pending &p = s.reqs[i];
            if (p.blk) {
                pool.release(p.blk);
                p.blk = nullptr;
            }
            auto it = tickets.find(p.ticket);
            if (it == tickets.end()) continue;
            Ticket &tk = it->second;
            tk.r.status = status;
            tk.r.value = status ? __builtin_nan("") : be.result(s.d, i, p.req);
            tk.r.t_done_ns = t;
            tk.done = true;
            st.completed += 1;
        }
        s.reqs.clear();
        s.state = SlotState::Free;
        work_seq.fetch_add(1, std::memory_order_release);
        cv_done.notify_all();
        cv_work.notify_one();
    }

    // Waits for slot i's batches, one at a time, and completes them.
    void completion_loop(size_t i)
    {
        be.thread_start();
        Slot<B> &s = slots[i];
        std::atomic<uint64_t> &seq = flight_seq[i];
        auto ready = [&] { return s.state == SlotState::InFlight || (stop && s.state == SlotState::Free); };
        std::unique_lock<std::mutex> lk(mu);
        for (;;) {
            while (!ready()) {
                const uint64_t seen = seq.load(std::memory_order_relaxed);
                lk.unlock();
                const bool changed = spin_until_changed(seq, seen, SPIN_NS);
                lk.lock();
                if (!changed)
                    cv_slots.wait(lk, [&] { return ready() || seq.load(std::memory_order_relaxed) != seen; });
            }
            if (s.state != SlotState::InFlight) break;
            const int lrc = s.launch_rc;
            lk.unlock();
            const int rc = be.wait(s.d, lrc);
            lk.lock();
            complete(s, lrc ? lrc : rc);
        }
    }

    // --- batching ---------------------------------------------------------------------
    // Chooses the next batch from the queue, in arrival order: requests that need no pool
    // memory (zero-copy, or admitted already) and copy requests that are admitted now while
    // the pool has room.  The first copy request that does not fit stops the admission of
    // later copies, which keep their order, but not requests that need no memory (a client
    // may hold pool memory until such a request completes).  A request rerun alone after an
    // injected failure is a batch of its own.  Returns the queue positions; *blocked: a copy
    // request waits for memory.  Called with mu held.
    std::vector<size_t> select(bool *blocked)
    {
        std::vector<size_t> pick;
        *blocked = false;
        const size_t limit = pending.front().solo ? 1 : (size_t)cfg.max_batch;
        // behind a blocked copy only requests that need no memory are taken: the scan stops
        // when none is left further back (and after a bounded window)
        int64_t nocopy_left = nocopy_pending;
        const size_t window = 4 * (size_t)cfg.max_batch + 4096;
        for (size_t k = 0; k < pending.size() && pick.size() < limit; ++k) {
            Pending &p = pending[k];
            if (p.solo && k > 0) break;
            if (*blocked && (nocopy_left == 0 || k >= window)) break;
            if (!p.copy) --nocopy_left;
            if (p.copy && !p.blk) {
                if (*blocked) continue;
                p.blk = pool.alloc((uint64_t)std::max<int64_t>(payload_bytes(p.req), 1));
                if (!p.blk) {
                    *blocked = true;
                    if (!p.t_blocked) {
                        p.t_blocked = now_ns();
                        st.admission_waits += 1;
                    }
                    if (limit == 1) break;
                    continue;
                }
                if (p.t_blocked) {
                    const int64_t w = now_ns() - p.t_blocked;
                    st.admission_wait_ns += w;
                    st.admission_wait_ns_max = std::max<int64_t>(st.admission_wait_ns_max, w);
                }
            }
            pick.push_back(k);
        }
        return pick;
    }

    void worker_loop()
    {
        be.thread_start();
        std::unique_lock<std::mutex> lk(mu);
        for (;;) {
            if (stop) break;
            Slot<B> *free_slot = nullptr;
            bool idle = true;
            for (Slot<B> &s : slots) {
                if (s.state == SlotState::Free && !free_slot) free_slot = &s;
                idle = idle && s.state == SlotState::Free;
            }
            bool go = false;
            int64_t wait_ns = -1;
            std::vector<size_t> pick;
            if (free_slot && !pending.empty()) {
                bool blocked = false;
                pick = select(&blocked);
                // an idle device starts at once; while batches run, a small batch may wait
                // up to max_wait_us for more requests (not while a request waits for memory)
                const int64_t age = pick.empty() ? 0 : now_ns() - pending[pick[0]].t_submit;
                go = !pick.empty() && (idle || cfg.max_wait_us == 0 || pick.size() >= (size_t)cfg.max_batch ||
                                       age >= (int64_t)cfg.max_wait_us * 1000 || pending.front().solo || blocked);
                if (!pick.empty() && !go) wait_ns = (int64_t)cfg.max_wait_us * 1000 - age;
            }
            if (!go) {
                if (wait_ns > 0) {
                    cv_work.wait_for(lk, std::chrono::nanoseconds(wait_ns));
                } else {
                    const uint64_t seen = work_seq.load(std::memory_order_relaxed);
                    lk.unlock();
                    const bool changed = spin_until_changed(work_seq, seen, SPIN_NS);
                    lk.lock();
                    if (!changed) cv_work.wait(lk, [&] { return work_seq.load(std::memory_order_relaxed) != seen; });
                }
                continue;
            }
            std::vector<Pending> batch;
            batch.reserve(pick.size());
            for (size_t k : pick) batch.push_back(pending[k]);
            if (pick.back() + 1 == pick.size()) {  // a prefix of the queue (the usual case)
                for (size_t k = 0; k < pick.size(); ++k) pending.pop_front();
            } else {
                for (auto it = pick.rbegin(); it != pick.rend(); ++it) pending.erase(pending.begin() + (ptrdiff_t)*it);
            }
            for (const Pending &p : batch) nocopy_pending -= p.copy ? 0 : 1;
            Slot<B> &s = *free_slot;
            const int64_t bno = ++batch_counter;
            st.batches += 1;
            st.max_batch_seen = std::max<int64_t>(st.max_batch_seen, (int64_t)batch.size());
            if (cfg.inject_failure_every > 0 && bno % cfg.inject_failure_every == 0 && batch.size() > 1) {
                // injected failure: nothing is launched; each request is rerun alone (keeping
                // its pool block)
                st.failed_batches += 1;
                for (auto it = batch.rbegin(); it != batch.rend(); ++it) {
                    Pending p = *it;
                    p.solo = true;
                    pending.push_front(p);
                    nocopy_pending += p.copy ? 0 : 1;
                }
                continue;
            }
            s.state = SlotState::Launching;
            lk.unlock();
            int nl = 0;
            const int64_t t_l = now_ns();
            const int rc = be.launch(s.d, batch, &nl);
            const int64_t t_e = now_ns();
            lk.lock();
            st.host_launch_ns += t_e - t_l;
            st.launches += nl;
            s.reqs = std::move(batch);
            s.launch_rc = rc;
            s.t_enqueued = t_e;
            s.state = SlotState::InFlight;
            flight_seq[(size_t)(&s - slots.data())].fetch_add(1, std::memory_order_release);
            cv_slots.notify_all();
        }
    }

    // --- client calls -----------------------------------------------------------------
    int alloc(int64_t bytes, void **dptr)
    {
        std::lock_guard<std::mutex> lk(mu);
        void *p = pool.alloc((uint64_t)bytes);
        if (!p) return VNP_EAGAIN;
        *dptr = p;
        return 0;
    }

    int release(void *dptr)
    {
        std::lock_guard<std::mutex> lk(mu);
        if (!pool.release(dptr)) return -2;
        work_seq.fetch_add(1, std::memory_order_release);  // memory for waiting admissions
        cv_work.notify_one();
        return 0;
    }

    // info: the request's INFO code (0 = valid); copy: admit a copy of the payload.
    void submit(const vnp_request &req, int info, bool copy, uint64_t *ticket)
    {
        const int64_t t = now_ns();
        if (!info && copy && Pool::granule((uint64_t)std::max<int64_t>(payload_bytes(req), 1)) > pool.size)
            info = VNP_ENOMEM;  // larger than the whole pool: never admitted
        {
            std::lock_guard<std::mutex> lk(mu);
            const uint64_t id = next_ticket++;
            Ticket tk{};
            tk.r.t_submit_ns = t;
            st.submitted += 1;
            if (info) {
                tk.r.status = info;
                tk.r.value = __builtin_nan("");
                tk.r.t_done_ns = t;
                tk.done = true;
                st.rejected += 1;
            } else {
                pending.push_back(Pending{id, req, t, false, copy, nullptr, 0});
                nocopy_pending += copy ? 0 : 1;
                work_seq.fetch_add(1, std::memory_order_release);
            }
            tickets.emplace(id, tk);
            *ticket = id;
        }
        if (info)
            cv_done.notify_all();
        else
            cv_work.notify_one();
    }

    int take(uint64_t ticket, vnp_result *out, int64_t timeout_us)
    {
        std::unique_lock<std::mutex> lk(mu);
        auto it = tickets.find(ticket);
        if (it == tickets.end()) return VNP_ENOTFOUND;
        if (!it->second.done && timeout_us != 0) {
            auto ready = [&] {
                auto j = tickets.find(ticket);
                return j == tickets.end() || j->second.done;
            };
            waiters += 1;
            if (timeout_us < 0)
                cv_done.wait(lk, ready);
            else
                cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), ready);
            waiters -= 1;
            if (stop && waiters == 0) cv_left.notify_all();
            it = tickets.find(ticket);
            if (it == tickets.end()) return VNP_ENOTFOUND;
        }
        if (!it->second.done) return VNP_EPENDING;
        if (out) *out = it->second.r;
        tickets.erase(it);
        return 0;
    }

    void stats(vnp_server_stats *out)
    {
        std::lock_guard<std::mutex> lk(mu);
        vnp_server_stats r = st;
        r.pool_free_bytes = (int64_t)pool.free_bytes;
        r.pending = (int64_t)pending.size();
        int64_t inflight = 0;
        for (const Slot<B> &sl : slots) inflight += sl.state != SlotState::Free ? (int64_t)sl.reqs.size() : 0;
        r.in_flight = inflight;
        *out = r;
    }
};

// Argument checks of a request (the INFO codes of vnp_server_submit); p_ok: the p-norm
// calls' test of p in the request's dtype.
template <class POk>
inline int request_info(const vnp_request &req, POk p_ok)
{
    if (req.dtype != VNP_F64 && req.dtype != VNP_F32) return -1;
    if (!p_ok(req)) return -2;
    if (req.n < 0 || req.n > VNP_MAX_N) return -3;
    if (req.n > 0 && !req.x) return -4;
    if (req.incx == 0) return -5;
    return 0;
}

}  // namespace srv
}  // namespace vnp

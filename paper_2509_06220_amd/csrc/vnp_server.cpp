// Request server: continuous batching of norm requests (see include/vnp_server.h).
//
// One batcher thread owns the launches.  Clients submit requests (host bookkeeping
// only); the batcher moves pending requests into a free stream slot, writes their
// descriptors and item offsets into the slot's pinned host buffer and enqueues the batch:
// a stage kernel copies the descriptors to the device, then one batched launch per
// (dtype, p) class writes the results straight into the slot's pinned result buffer, and
// an event is recorded.  A batch of one request is the single-vector call itself.  Each slot has a completion thread that waits for that event,
// posts the results to the tickets and wakes waiters and the batcher.  With several
// slots, requests that arrive while batches run are launched on another stream and
// overlap on the device.
//
// The batcher and the completion threads poll for new work for up to SPIN_NS before they
// block on a condition variable: waking a blocked thread takes longer than a small batch
// runs on the device.
#include <hip/hip_runtime.h>
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

#include "../../include/vnp.h"
#include "../../include/vnp_server.h"
#include "vnp_batch.hpp"
#include "vnp_internal.hpp"

namespace {

int64_t now_ns()
{
    return std::chrono::duration_cast<std::chrono::nanoseconds>(std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

constexpr int64_t SPIN_NS = 200000;  // busy-poll window before blocking

// Polls seq until it differs from seen (true) or spin_ns pass (false).
bool spin_until_changed(const std::atomic<uint64_t> &seq, uint64_t seen, int64_t spin_ns)
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

    void init(char *b, uint64_t s)
    {
        base = b;
        size = s;
        free_.clear();
        used_.clear();
        free_[0] = s;
        free_bytes = s;
    }
    void *alloc(uint64_t bytes)
    {
        const uint64_t need = (bytes + 255) & ~uint64_t(255);
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
    bool solo;  // rerun alone after an injected batch failure
};

struct Ticket {
    vnp_result r;
    bool done;
};

enum class SlotState { Free, Launching, InFlight };

struct Slot {
    hipStream_t st = nullptr;
    hipEvent_t ev = nullptr;
    vnp::BatchWorkspace ws;
    char *h_desc = nullptr, *h_desc_dev = nullptr;  // pinned descriptor words and their device view
    char *d_desc = nullptr;                         // device copy of the descriptor words
    char *h_res = nullptr, *h_res_dev = nullptr;    // pinned results [double cap | float cap]
    std::vector<Pending> reqs;
    SlotState state = SlotState::Free;
    int launch_rc = 0;
    int64_t t_enqueued = 0;
    std::thread done_thread;
};

bool same_class(const vnp_request &u, const vnp_request &v)
{
    return u.dtype == v.dtype && (u.p == v.p || (u.p != u.p && v.p != v.p));
}

}  // namespace

struct vnp_server {
    vnp_server_config cfg{};
    int device = 0;
    Pool pool;
    std::mutex mu;
    std::condition_variable cv_work, cv_done, cv_slots;
    std::deque<Pending> pending;
    std::unordered_map<uint64_t, Ticket> tickets;
    std::vector<Slot> slots;
    std::thread worker;
    bool stop = false;
    int waiters = 0;                 // threads blocked in vnp_server_wait
    std::condition_variable cv_left;  // signalled when the last waiter leaves after stop
    // Bumped under mu whenever the batcher may have work (a request queued, a slot freed,
    // stop), and per slot whenever the slot's batch is in flight (or stop): the polled
    // change counters of the busy-poll phase.
    std::atomic<uint64_t> work_seq{0};
    std::unique_ptr<std::atomic<uint64_t>[]> flight_seq;
    uint64_t next_ticket = 1;
    vnp_server_stats st{};
    int64_t batch_counter = 0;

    void worker_loop();
    void completion_loop(size_t i);
    int launch(Slot &s, std::vector<Pending> &reqs, int *nlaunch);
    void complete(Slot &s, int status);
};

// Fills the slot's pinned buffers for the batch and enqueues it.  Runs without the lock
// (the slot is owned by the batcher until it is handed to its completion thread).
int vnp_server::launch(Slot &s, std::vector<Pending> &reqs, int *nlaunch)
{
    *nlaunch = 0;
    const size_t cap = (size_t)cfg.max_batch;
    const int64_t n = (int64_t)reqs.size();
    if (n == 1) {
        // one request: the single-vector call itself on the slot's stream (no descriptor
        // staging), its result written to the slot's pinned result word
        const vnp_request &q = reqs[0].req;
        int rc;
        if (q.dtype == VNP_F32) {
            float *r = reinterpret_cast<float *>(s.h_res_dev + cap * 8);
            const float *x = static_cast<const float *>(q.x);
            rc = q.p == 2.0 ? vnp_snrmf(q.n, x, q.incx, r, s.st) : vnp_snrmp(q.n, x, q.incx, (float)q.p, r, s.st);
        } else {
            double *r = reinterpret_cast<double *>(s.h_res_dev);
            const double *x = static_cast<const double *>(q.x);
            rc = q.p == 2.0 ? vnp_dnrmf(q.n, x, q.incx, r, s.st) : vnp_dnrmp(q.n, x, q.incx, q.p, r, s.st);
        }
        if (rc) return rc;
        *nlaunch = 1;
        return (int)hipEventRecord(s.ev, s.st);
    }
    std::stable_sort(reqs.begin(), reqs.end(), [](const Pending &u, const Pending &v) {
        if (u.req.dtype != v.req.dtype) return u.req.dtype < v.req.dtype;
        return u.req.p < v.req.p;
    });
    int64_t *w = reinterpret_cast<int64_t *>(s.h_desc);
    void **hp = reinterpret_cast<void **>(w);
    int64_t *hl = w + n, *hi = w + 2 * n;
    double *rd = reinterpret_cast<double *>(s.h_res);
    float *rf = reinterpret_cast<float *>(s.h_res + cap * 8);
    std::vector<vnp::RequestClass> classes;
    for (int64_t i = 0; i < n; ++i) {
        const vnp_request &q = reqs[(size_t)i].req;
        const size_t esz = q.dtype == VNP_F32 ? 4 : 8;
        const char *x = static_cast<const char *>(q.x);
        hp[i] = const_cast<char *>(q.incx >= 0 || q.n <= 0 ? x : x + (size_t)((q.n - 1) * (-q.incx)) * esz);
        hl[i] = q.n;
        hi[i] = q.incx;
        if (q.n == 0) {  // no work item: the result is +0
            if (q.dtype == VNP_F32)
                rf[i] = 0.0f;
            else
                rd[i] = 0.0;
        }
        if (classes.empty() || !same_class(reqs[(size_t)classes.back().a].req, q))
            classes.push_back(vnp::RequestClass{q.dtype, q.p, i, 1, 0, 0, 0});
        else
            classes.back().n += 1;
    }
    for (size_t c = 0; c < classes.size(); ++c) {
        vnp::RequestClass &k = classes[c];
        int64_t *off = w + 3 * n + k.a + (int64_t)c;
        k.lwt = vnp::request_class_items(k.dtype, hl + k.a, k.n, off);
        k.items = off[k.n];
        for (int64_t i = 0; i < k.n && !k.multi; ++i) k.multi = off[i + 1] - off[i] > 1;
        *nlaunch += k.items > 0 ? 1 : 0;
    }
    int rc = vnp::enqueue_request_batch(s.h_desc_dev, s.d_desc, n, classes.data(), (int)classes.size(),
                                        reinterpret_cast<double *>(s.h_res_dev),
                                        reinterpret_cast<float *>(s.h_res_dev + cap * 8), s.ws, s.st);
    if (rc) return rc;
    return (int)hipEventRecord(s.ev, s.st);
}

// Posts the slot's results (status 0) or the error to its tickets and frees the slot.
// Called with mu held.
void vnp_server::complete(Slot &s, int status)
{
    const size_t cap = (size_t)cfg.max_batch;
    const double *rd = reinterpret_cast<const double *>(s.h_res);
    const float *rf = reinterpret_cast<const float *>(s.h_res + cap * 8);
    const int64_t t = now_ns();
    if (s.t_enqueued) {
        st.batch_ns += t - s.t_enqueued;
        st.batch_ns_max = std::max<int64_t>(st.batch_ns_max, t - s.t_enqueued);
        s.t_enqueued = 0;
    }
    for (size_t i = 0; i < s.reqs.size(); ++i) {
        auto it = tickets.find(s.reqs[i].ticket);
        if (it == tickets.end()) continue;
        Ticket &tk = it->second;
        tk.r.status = status;
        tk.r.value = status ? __builtin_nan("") : (s.reqs[i].req.dtype == VNP_F32 ? (double)rf[i] : rd[i]);
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
void vnp_server::completion_loop(size_t i)
{
    (void)hipSetDevice(device);
    Slot &s = slots[i];
    std::atomic<uint64_t> &seq = flight_seq[i];
    auto ready = [&] { return s.state == SlotState::InFlight || (stop && s.state == SlotState::Free); };
    std::unique_lock<std::mutex> lk(mu);
    for (;;) {
        while (!ready()) {
            const uint64_t seen = seq.load(std::memory_order_relaxed);
            lk.unlock();
            const bool changed = spin_until_changed(seq, seen, SPIN_NS);
            lk.lock();
            if (!changed) cv_slots.wait(lk, [&] { return ready() || seq.load(std::memory_order_relaxed) != seen; });
        }
        if (s.state != SlotState::InFlight) break;
        int rc = s.launch_rc;
        lk.unlock();
        if (rc)
            (void)hipStreamSynchronize(s.st);  // nothing of a failed batch may still run
        else
            rc = (int)hipEventSynchronize(s.ev);
        lk.lock();
        complete(s, rc);
    }
}

void vnp_server::worker_loop()
{
    (void)hipSetDevice(device);
    std::unique_lock<std::mutex> lk(mu);
    for (;;) {
        if (stop) break;
        Slot *free_slot = nullptr;
        for (Slot &s : slots)
            if (s.state == SlotState::Free) {
                free_slot = &s;
                break;
            }
        bool go = false;
        int64_t wait_ns = -1;
        if (free_slot && !pending.empty()) {
            // an idle device starts at once; while batches run, a small batch may wait up
            // to max_wait_us for more requests
            bool idle = true;
            for (const Slot &sl : slots) idle = idle && sl.state == SlotState::Free;
            const int64_t age = now_ns() - pending.front().t_submit;
            go = idle || cfg.max_wait_us == 0 || (int64_t)pending.size() >= cfg.max_batch ||
                 age >= (int64_t)cfg.max_wait_us * 1000 || pending.front().solo;
            if (!go) wait_ns = (int64_t)cfg.max_wait_us * 1000 - age;
        }
        if (!go) {
            if (wait_ns > 0) {
                cv_work.wait_for(lk, std::chrono::nanoseconds(wait_ns));
            } else {
                const uint64_t seen = work_seq.load(std::memory_order_relaxed);
                lk.unlock();
                const bool changed = spin_until_changed(work_seq, seen, SPIN_NS);
                lk.lock();
                if (!changed)
                    cv_work.wait(lk, [&] { return work_seq.load(std::memory_order_relaxed) != seen; });
            }
            continue;
        }
        std::vector<Pending> batch;
        if (pending.front().solo) {
            batch.push_back(pending.front());
            pending.pop_front();
        } else {
            while (!pending.empty() && (int)batch.size() < cfg.max_batch && !pending.front().solo) {
                batch.push_back(pending.front());
                pending.pop_front();
            }
        }
        Slot &s = *free_slot;
        const int64_t bno = ++batch_counter;
        st.batches += 1;
        st.max_batch_seen = std::max<int64_t>(st.max_batch_seen, (int64_t)batch.size());
        if (cfg.inject_failure_every > 0 && bno % cfg.inject_failure_every == 0 && batch.size() > 1) {
            // injected failure: nothing is launched; each request is rerun alone
            st.failed_batches += 1;
            for (auto it = batch.rbegin(); it != batch.rend(); ++it) {
                Pending p = *it;
                p.solo = true;
                pending.push_front(p);
            }
            continue;
        }
        s.state = SlotState::Launching;
        lk.unlock();
        int nl = 0;
        const int64_t t_l = now_ns();
        const int rc = launch(s, batch, &nl);
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

static void free_slots(vnp_server *s)
{
    for (Slot &sl : s->slots) {
        if (sl.st) (void)hipStreamSynchronize(sl.st);
        vnp::release_batch_ws(sl.ws);
        if (sl.d_desc) (void)hipFree(sl.d_desc);
        if (sl.h_desc) (void)hipHostFree(sl.h_desc);
        if (sl.h_res) (void)hipHostFree(sl.h_res);
        if (sl.ev) (void)hipEventDestroy(sl.ev);
        if (sl.st) (void)hipStreamDestroy(sl.st);
    }
    s->slots.clear();
    if (s->pool.base) (void)hipFree(s->pool.base);
    s->pool.base = nullptr;
}

extern "C" {

int64_t vnp_server_clock_ns(void) { return now_ns(); }

int vnp_server_create(vnp_server **srv, const vnp_server_config *cfg)
{
    if (!srv) return -1;
    *srv = nullptr;
    if (!cfg || cfg->pool_bytes < 0 || cfg->max_batch < 1 || cfg->max_batch > (1 << 20) || cfg->streams < 1 ||
        cfg->streams > 16 || cfg->max_wait_us < 0 || cfg->inject_failure_every < 0)
        return -2;
    vnp_server *s = new (std::nothrow) vnp_server;
    if (!s) return (int)hipErrorOutOfMemory;
    s->cfg = *cfg;
    hipError_t e = hipGetDevice(&s->device);
    char *pool = nullptr;
    if (e == hipSuccess && cfg->pool_bytes > 0) e = hipMalloc(reinterpret_cast<void **>(&pool), (size_t)cfg->pool_bytes);
    s->pool.init(pool, (uint64_t)cfg->pool_bytes);
    const size_t cap = (size_t)cfg->max_batch;
    // ptrs | lens | incs | item offsets (n_c + 1 per class): at most 3 cap + 2 cap words,
    // since a batch of cap requests has at most cap (dtype, p) classes
    const size_t desc_bytes = (5 * cap + 1) * 8;
    s->slots.resize((size_t)cfg->streams);
    s->flight_seq.reset(new (std::nothrow) std::atomic<uint64_t>[(size_t)cfg->streams]);
    if (!s->flight_seq) {
        delete s;
        return (int)hipErrorOutOfMemory;
    }
    for (int k = 0; k < cfg->streams; ++k) s->flight_seq[k].store(0, std::memory_order_relaxed);
    for (Slot &sl : s->slots) {
        if (e != hipSuccess) break;
        e = hipStreamCreateWithFlags(&sl.st, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&sl.ev, hipEventDisableTiming);
        if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void **>(&sl.d_desc), desc_bytes);
        if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void **>(&sl.h_desc), desc_bytes, hipHostMallocDefault);
        if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void **>(&sl.h_res), cap * 12, hipHostMallocDefault);
        if (e == hipSuccess) e = hipHostGetDevicePointer(reinterpret_cast<void **>(&sl.h_desc_dev), sl.h_desc, 0);
        if (e == hipSuccess) e = hipHostGetDevicePointer(reinterpret_cast<void **>(&sl.h_res_dev), sl.h_res, 0);
        if (e == hipSuccess) memset(sl.h_desc, 0, desc_bytes);
    }
    if (e != hipSuccess) {
        free_slots(s);
        delete s;
        return (int)e;
    }
    s->st.pool_bytes = cfg->pool_bytes;
    for (size_t i = 0; i < s->slots.size(); ++i) s->slots[i].done_thread = std::thread([s, i] { s->completion_loop(i); });
    s->worker = std::thread([s] { s->worker_loop(); });
    *srv = s;
    return 0;
}

int vnp_server_destroy(vnp_server *s)
{
    if (!s) return -1;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
        // requests not yet launched complete as cancelled (their waiters return)
        const int64_t t = now_ns();
        for (const Pending &p : s->pending) {
            auto it = s->tickets.find(p.ticket);
            if (it == s->tickets.end()) continue;
            it->second.r.status = VNP_ECANCELED;
            it->second.r.value = __builtin_nan("");
            it->second.r.t_done_ns = t;
            it->second.done = true;
            s->st.cancelled += 1;
        }
        s->pending.clear();
        s->work_seq.fetch_add(1, std::memory_order_release);
    }
    s->cv_done.notify_all();
    s->cv_work.notify_all();
    if (s->worker.joinable()) s->worker.join();
    {
        std::lock_guard<std::mutex> lk(s->mu);  // the batcher has stopped: no slot is Launching
        for (size_t k = 0; k < s->slots.size(); ++k) s->flight_seq[k].fetch_add(1, std::memory_order_release);
    }
    s->cv_slots.notify_all();
    for (Slot &sl : s->slots)
        if (sl.done_thread.joinable()) sl.done_thread.join();  // in-flight batches complete first
    {
        // every ticket is complete now: wait until the blocked waiters have returned
        std::unique_lock<std::mutex> lk(s->mu);
        s->cv_done.notify_all();
        s->cv_left.wait(lk, [s] { return s->waiters == 0; });
    }
    free_slots(s);
    delete s;
    return 0;
}

int vnp_server_alloc(vnp_server *s, int64_t bytes, void **dptr)
{
    if (!s) return -1;
    if (bytes <= 0) return -2;
    if (!dptr) return -3;
    std::lock_guard<std::mutex> lk(s->mu);
    void *p = s->pool.alloc((uint64_t)bytes);
    if (!p) return VNP_EAGAIN;
    *dptr = p;
    return 0;
}

int vnp_server_free(vnp_server *s, void *dptr)
{
    if (!s) return -1;
    std::lock_guard<std::mutex> lk(s->mu);
    return s->pool.release(dptr) ? 0 : -2;
}

int vnp_server_submit(vnp_server *s, const vnp_request *req, uint64_t *ticket)
{
    if (!s) return -1;
    if (!req) return -2;
    if (!ticket) return -3;
    int info = 0;
    if (req->dtype != VNP_F64 && req->dtype != VNP_F32)
        info = -1;
    else if (!(req->dtype == VNP_F32 ? vnp::p_ok((float)req->p) : vnp::p_ok(req->p)))
        info = -2;
    else if (req->n < 0 || req->n > VNP_MAX_N)
        info = -3;
    else if (req->n > 0 && !req->x)
        info = -4;
    else if (req->incx == 0)
        info = -5;
    const int64_t t = now_ns();
    {
        std::lock_guard<std::mutex> lk(s->mu);
        const uint64_t id = s->next_ticket++;
        Ticket tk{};
        tk.r.t_submit_ns = t;
        s->st.submitted += 1;
        if (info) {
            tk.r.status = info;
            tk.r.value = __builtin_nan("");
            tk.r.t_done_ns = t;
            tk.done = true;
            s->st.rejected += 1;
        } else {
            s->pending.push_back(Pending{id, *req, t, false});
            s->work_seq.fetch_add(1, std::memory_order_release);
        }
        s->tickets.emplace(id, tk);
        *ticket = id;
    }
    if (info)
        s->cv_done.notify_all();
    else
        s->cv_work.notify_one();
    return 0;
}

static int take_result(vnp_server *s, uint64_t ticket, vnp_result *out, std::unique_lock<std::mutex> &lk,
                       int64_t timeout_us)
{
    auto it = s->tickets.find(ticket);
    if (it == s->tickets.end()) return VNP_ENOTFOUND;
    if (!it->second.done && timeout_us != 0) {
        auto ready = [&] {
            auto j = s->tickets.find(ticket);
            return j == s->tickets.end() || j->second.done;
        };
        s->waiters += 1;
        if (timeout_us < 0)
            s->cv_done.wait(lk, ready);
        else
            s->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), ready);
        s->waiters -= 1;
        if (s->stop && s->waiters == 0) s->cv_left.notify_all();
        it = s->tickets.find(ticket);
        if (it == s->tickets.end()) return VNP_ENOTFOUND;
    }
    if (!it->second.done) return VNP_EPENDING;
    if (out) *out = it->second.r;
    s->tickets.erase(it);
    return 0;
}

int vnp_server_poll(vnp_server *s, uint64_t ticket, vnp_result *out)
{
    if (!s) return -1;
    std::unique_lock<std::mutex> lk(s->mu);
    return take_result(s, ticket, out, lk, 0);
}

int vnp_server_wait(vnp_server *s, uint64_t ticket, int64_t timeout_us, vnp_result *out)
{
    if (!s) return -1;
    std::unique_lock<std::mutex> lk(s->mu);
    return take_result(s, ticket, out, lk, timeout_us);
}

int vnp_server_get_stats(vnp_server *s, vnp_server_stats *out)
{
    if (!s) return -1;
    if (!out) return -2;
    std::lock_guard<std::mutex> lk(s->mu);
    vnp_server_stats r = s->st;
    r.pool_free_bytes = (int64_t)s->pool.free_bytes;
    r.pending = (int64_t)s->pending.size();
    int64_t inflight = 0;
    for (const Slot &sl : s->slots) inflight += sl.state != SlotState::Free ? (int64_t)sl.reqs.size() : 0;
    r.in_flight = inflight;
    *out = r;
    return 0;
}

}  // extern "C"

// Request server on one GPU (see include/vnp_server.h): the core of vnp_server_core.hpp
// with the HIP backend below.
//
// A batch on a slot's stream: for requests admitted by copy, the copy table and a gather
// kernel that moves their payloads into their pool blocks; then, for a batch of one
// request, the single-vector call itself, its result written to the slot's pinned result
// word; for larger batches a stage kernel copies the descriptors to the device and one
// batched launch per (dtype, p) class writes the results straight into the slot's pinned
// result buffer.  An event marks the batch's end.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <vector>

#include "../../include/vnp.h"
#include "../../include/vnp_server.h"
#include "vnp_batch.hpp"
#include "vnp_internal.hpp"
#include "vnp_server_core.hpp"

namespace vnp {
namespace {

using srv::Pending;

bool same_class(const vnp_request &u, const vnp_request &v)
{
    return u.dtype == v.dtype && (u.p == v.p || (u.p != u.p && v.p != v.p));
}

struct HipBackend {
    int device = 0;

    struct SlotData {
        hipStream_t st = nullptr;
        hipEvent_t ev = nullptr;
        BatchWorkspace ws;
        char *h_desc = nullptr, *h_desc_dev = nullptr;  // pinned descriptor words and their device view
        char *d_desc = nullptr;                         // device copy of the descriptor words
        char *h_res = nullptr, *h_res_dev = nullptr;    // pinned results [double cap | float cap]
        size_t cap = 0;
    };

    int init(const vnp_server_config &cfg, char **pool)
    {
        hipError_t e = hipGetDevice(&device);
        if (e == hipSuccess && cfg.pool_bytes > 0) e = hipMalloc(reinterpret_cast<void **>(pool), (size_t)cfg.pool_bytes);
        return (int)e;
    }
    void fini(char *pool)
    {
        if (pool) (void)hipFree(pool);
    }

    int slot_init(SlotData &d, const vnp_server_config &cfg)
    {
        d.cap = (size_t)cfg.max_batch;
        // ptrs | lens | incs | item offsets (n_c + 1 per class) | copy table (6 per copy + 1):
        // at most 3 cap + 2 cap + 6 cap + 1 words, since a batch of cap requests has at most
        // cap (dtype, p) classes and cap copies
        const size_t desc_bytes = (11 * d.cap + 2) * 8;
        hipError_t e = hipStreamCreateWithFlags(&d.st, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&d.ev, hipEventDisableTiming);
        if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void **>(&d.d_desc), desc_bytes);
        if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void **>(&d.h_desc), desc_bytes, hipHostMallocDefault);
        if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void **>(&d.h_res), d.cap * 12, hipHostMallocDefault);
        if (e == hipSuccess) e = hipHostGetDevicePointer(reinterpret_cast<void **>(&d.h_desc_dev), d.h_desc, 0);
        if (e == hipSuccess) e = hipHostGetDevicePointer(reinterpret_cast<void **>(&d.h_res_dev), d.h_res, 0);
        if (e == hipSuccess) memset(d.h_desc, 0, desc_bytes);
        return (int)e;
    }
    void slot_fini(SlotData &d)
    {
        if (d.st) (void)hipStreamSynchronize(d.st);
        release_batch_ws(d.ws);
        if (d.d_desc) (void)hipFree(d.d_desc);
        if (d.h_desc) (void)hipHostFree(d.h_desc);
        if (d.h_res) (void)hipHostFree(d.h_res);
        if (d.ev) (void)hipEventDestroy(d.ev);
        if (d.st) (void)hipStreamDestroy(d.st);
        d = SlotData{};
    }

    void thread_start() { (void)hipSetDevice(device); }

    // The copy table of the batch's admitted requests at w (words), and each such request
    // redirected to its contiguous pool block; returns the number of chunks.
    static int64_t copy_table(std::vector<Pending> &reqs, int64_t *w, int64_t ncopy)
    {
        int64_t c = 0, chunks = 0;
        int64_t *off = w + 5 * ncopy;
        for (Pending &p : reqs) {
            if (!p.blk) continue;
            vnp_request &q = p.req;
            const int64_t esz = q.dtype == VNP_F32 ? 4 : 8;
            const char *x = static_cast<const char *>(q.x);
            const char *x0 = q.incx >= 0 || q.n <= 0 ? x : x + (q.n - 1) * (-q.incx) * esz;
            w[5 * c + 0] = (int64_t)(uintptr_t)x0;
            w[5 * c + 1] = (int64_t)(uintptr_t)p.blk;
            w[5 * c + 2] = q.n;
            w[5 * c + 3] = q.incx;
            w[5 * c + 4] = esz;
            off[c] = chunks;
            chunks += copy_chunks(q.n);
            q.x = p.blk;  // the norm reads the copy
            q.incx = 1;
            ++c;
        }
        off[c] = chunks;
        return chunks;
    }

    // Fills the slot's pinned buffers for the batch and enqueues it.
    int launch(SlotData &s, std::vector<Pending> &reqs, int *nlaunch)
    {
        *nlaunch = 0;
        const int64_t n = (int64_t)reqs.size();
        int64_t ncopy = 0;
        for (const Pending &p : reqs) ncopy += p.blk ? 1 : 0;
        if (n == 1) {
            // one request: the single-vector call itself on the slot's stream (after one gather
            // launch for a copy), its result written to the slot's pinned result word
            int rc = 0;
            if (ncopy) {
                vnp_request &q = reqs[0].req;
                const int64_t esz = q.dtype == VNP_F32 ? 4 : 8;
                const char *x = static_cast<const char *>(q.x);
                const char *x0 = q.incx >= 0 || q.n <= 0 ? x : x + (q.n - 1) * (-q.incx) * esz;
                rc = enqueue_copy1(x0, reqs[0].blk, q.n, q.incx, esz, s.st);
                if (rc) return rc;
                q.x = reqs[0].blk;  // the norm reads the copy
                q.incx = 1;
            }
            const vnp_request &q = reqs[0].req;
            if (q.dtype == VNP_F32) {
                float *r = reinterpret_cast<float *>(s.h_res_dev + s.cap * 8);
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
        float *rf = reinterpret_cast<float *>(s.h_res + s.cap * 8);
        std::vector<RequestClass> classes;
        for (int64_t i = 0; i < n; ++i) {
            const vnp_request &q = reqs[(size_t)i].req;
            if (classes.empty() || !same_class(reqs[(size_t)classes.back().a].req, q))
                classes.push_back(RequestClass{q.dtype, q.p, i, 1, 0, 0, 0});
            else
                classes.back().n += 1;
        }
        const int64_t nwords = 4 * n + (int64_t)classes.size();
        const int64_t chunks = ncopy ? copy_table(reqs, w + nwords, ncopy) : 0;
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
        }
        for (size_t c = 0; c < classes.size(); ++c) {
            RequestClass &k = classes[c];
            int64_t *off = w + 3 * n + k.a + (int64_t)c;
            k.lwt = request_class_items(k.dtype, hl + k.a, k.n, off);
            k.items = off[k.n];
            for (int64_t i = 0; i < k.n && !k.multi; ++i) k.multi = off[i + 1] - off[i] > 1;
            *nlaunch += k.items > 0 ? 1 : 0;
        }
        int rc = enqueue_request_batch(s.h_desc_dev, s.d_desc, n, classes.data(), (int)classes.size(), ncopy, chunks,
                                       reinterpret_cast<double *>(s.h_res_dev),
                                       reinterpret_cast<float *>(s.h_res_dev + s.cap * 8), s.ws, s.st);
        if (rc) return rc;
        return (int)hipEventRecord(s.ev, s.st);
    }

    int wait(SlotData &s, int launch_rc)
    {
        if (launch_rc) {
            (void)hipStreamSynchronize(s.st);  // nothing of a failed batch may still run
            return 0;
        }
        return (int)hipEventSynchronize(s.ev);
    }

    double result(const SlotData &s, size_t i, const vnp_request &q) const
    {
        if (q.dtype == VNP_F32) return (double)reinterpret_cast<const float *>(s.h_res + s.cap * 8)[i];
        return reinterpret_cast<const double *>(s.h_res)[i];
    }
};

int check_request(const vnp_request &req)
{
    return srv::request_info(req, [](const vnp_request &q) {
        return q.dtype == VNP_F32 ? p_ok((float)q.p) : p_ok(q.p);
    });
}

}  // namespace
}  // namespace vnp

struct vnp_server {
    vnp::srv::Server<vnp::HipBackend> core;
};

extern "C" {

int64_t vnp_server_clock_ns(void) { return vnp::srv::now_ns(); }

int vnp_server_create(vnp_server **srv, const vnp_server_config *cfg)
{
    if (!srv) return -1;
    *srv = nullptr;
    if (!cfg || cfg->pool_bytes < 0 || cfg->max_batch < 1 || cfg->max_batch > (1 << 20) || cfg->streams < 1 ||
        cfg->streams > 16 || cfg->max_wait_us < 0 || cfg->inject_failure_every < 0)
        return -2;
    vnp_server *s = new (std::nothrow) vnp_server;
    if (!s) return (int)hipErrorOutOfMemory;
    const int rc = s->core.create(*cfg);
    if (rc) {
        delete s;
        return rc;
    }
    *srv = s;
    return 0;
}

int vnp_server_destroy(vnp_server *s)
{
    if (!s) return -1;
    s->core.destroy();
    delete s;
    return 0;
}

int vnp_server_alloc(vnp_server *s, int64_t bytes, void **dptr)
{
    if (!s) return -1;
    if (bytes <= 0) return -2;
    if (!dptr) return -3;
    return s->core.alloc(bytes, dptr);
}

int vnp_server_free(vnp_server *s, void *dptr)
{
    if (!s) return -1;
    return s->core.release(dptr);
}

int vnp_server_submit(vnp_server *s, const vnp_request *req, uint64_t *ticket)
{
    if (!s) return -1;
    if (!req) return -2;
    if (!ticket) return -3;
    s->core.submit(*req, vnp::check_request(*req), false, ticket);
    return 0;
}

int vnp_server_submit_copy(vnp_server *s, const vnp_request *req, uint64_t *ticket)
{
    if (!s) return -1;
    if (!req) return -2;
    if (!ticket) return -3;
    s->core.submit(*req, vnp::check_request(*req), true, ticket);
    return 0;
}

int vnp_server_poll(vnp_server *s, uint64_t ticket, vnp_result *out)
{
    if (!s) return -1;
    return s->core.take(ticket, out, 0);
}

int vnp_server_wait(vnp_server *s, uint64_t ticket, int64_t timeout_us, vnp_result *out)
{
    if (!s) return -1;
    return s->core.take(ticket, out, timeout_us);
}

int vnp_server_get_stats(vnp_server *s, vnp_server_stats *out)
{
    if (!s) return -1;
    if (!out) return -2;
    s->core.stats(out);
    return 0;
}

}  // extern "C"

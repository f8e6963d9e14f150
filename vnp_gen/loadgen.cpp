// Open-loop load generator for the request server (benchmark harness, no norm arithmetic).
//
// A submitter thread issues request i at its scheduled arrival time t0 + arrival[i]
// (never waiting for results), a collector gathers the results in submission order.
// The latency of request i is measured from its scheduled arrival to the server's
// completion stamp, so a backlog shows up as latency (no coordinated omission).
// The server is reached through function pointers passed in by the caller.
#include <stdint.h>
#include <time.h>

#include <atomic>
#include <thread>
#include <vector>

#include "../include/vnp_server.h"

typedef int (*submit_fn)(vnp_server *, const vnp_request *, uint64_t *);
typedef int (*wait_fn)(vnp_server *, uint64_t, int64_t, vnp_result *);
typedef int64_t (*clock_fn)(void);

extern "C" int vnpg_loadgen(void *srv, void *submit, void *wait, void *clock, int64_t nreq, const double *arrival_s,
                            const vnp_request *reqs, double *latency_s, double *values, int *status,
                            double *wall_s)
{
    submit_fn sub = (submit_fn)submit;
    wait_fn wt = (wait_fn)wait;
    clock_fn now = (clock_fn)clock;
    std::vector<uint64_t> tickets((size_t)nreq, 0);
    std::vector<int> sub_rc((size_t)nreq, 0);
    std::atomic<int64_t> issued{0};
    const int64_t t0 = now() + 2000000;  // start 2 ms from now
    std::thread submitter([&] {
        for (int64_t i = 0; i < nreq; ++i) {
            const int64_t target = t0 + (int64_t)(arrival_s[i] * 1e9);
            for (;;) {
                const int64_t d = target - now();
                if (d <= 0) break;
                if (d > 200000) {
                    struct timespec ts = {0, (long)(d - 100000)};
                    nanosleep(&ts, nullptr);
                }
            }
            sub_rc[(size_t)i] = sub((vnp_server *)srv, &reqs[i], &tickets[(size_t)i]);
            issued.store(i + 1, std::memory_order_release);
        }
    });
    int worst = 0;
    for (int64_t i = 0; i < nreq; ++i) {
        while (issued.load(std::memory_order_acquire) <= i) std::this_thread::yield();
        if (sub_rc[(size_t)i]) {
            status[i] = sub_rc[(size_t)i];
            values[i] = 0;
            latency_s[i] = -1;
            worst = sub_rc[(size_t)i];
            continue;
        }
        vnp_result r;
        const int rc = wt((vnp_server *)srv, tickets[(size_t)i], -1, &r);
        if (rc) {
            status[i] = rc;
            latency_s[i] = -1;
            worst = rc;
            continue;
        }
        status[i] = r.status;
        values[i] = r.value;
        latency_s[i] = (double)(r.t_done_ns - (t0 + (int64_t)(arrival_s[i] * 1e9))) * 1e-9;
    }
    submitter.join();
    *wall_s = (double)(now() - t0) * 1e-9;
    return worst;
}

// Baseline of the batched benchmark: nseg plain single-vector calls issued back to back
// from native code on one stream (no synchronisation), as a C caller would loop them.
// fn is a vnp_dnrmf/vnp_snrmf-shaped function; results go to res + i * res_bytes.
typedef int (*plain_fn)(int64_t, const void *, int64_t, void *, void *);

extern "C" int vnpg_loop_plain(void *fn, int64_t nseg, const int64_t *offsets, const void *x, int64_t esz,
                               void *res, int64_t res_bytes, void *stream)
{
    plain_fn f = (plain_fn)fn;
    const char *xb = static_cast<const char *>(x);
    char *rb = static_cast<char *>(res);
    for (int64_t i = 0; i < nseg; ++i) {
        const int rc = f(offsets[i + 1] - offsets[i], xb + offsets[i] * esz, 1, rb + i * res_bytes, stream);
        if (rc) return rc;
    }
    return 0;
}

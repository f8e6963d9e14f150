// The request server's host core (paper_2509_06220_amd/csrc/vnp_server_core.hpp) under
// ThreadSanitizer, with a CPU stand-in for the device backend: client threads submit (with
// and without copy admission), wait, poll, allocate and free pool blocks concurrently
// while the batcher and the completion threads run; the server is destroyed with requests
// still queued behind a held pool and a client blocked in wait.  Every result is checked
// against the payload it names; every ticket completes exactly once.
//
// Built and run by tests/test_server_core_tsan.py:
//   g++ -std=c++17 -O1 -g -fsanitize=thread -pthread -I paper_2509_06220_amd/csrc ...
// GCC 11's ThreadSanitizer does not intercept pthread_cond_clockwait, which libstdc++ uses
// for timed waits on the steady clock; it then sees every timed wait as a double lock.  This
// build takes libstdc++'s pthread_cond_timedwait path instead.
#include <bits/c++config.h>
#undef _GLIBCXX_USE_PTHREAD_COND_CLOCKWAIT

#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <atomic>
#include <chrono>
#include <random>
#include <thread>
#include <vector>

#include "vnp_server_core.hpp"

using vnp::srv::Pending;

// The stand-in device: a batch is "computed" at launch (the sum of the payload's logical
// elements, read from the pool block for copied payloads, which launch fills first) and
// completes after a short random delay.
struct FakeBackend {
    struct SlotData {
        std::vector<double> res;
        int64_t ready_ns = 0;
    };
    std::vector<char> pool_mem;
    std::atomic<uint64_t> rng{12345};

    int init(const vnp_server_config &cfg, char **pool)
    {
        pool_mem.assign((size_t)cfg.pool_bytes, 0);
        *pool = pool_mem.empty() ? nullptr : pool_mem.data();
        return 0;
    }
    void fini(char *) {}
    int slot_init(SlotData &d, const vnp_server_config &cfg)
    {
        d.res.assign((size_t)cfg.max_batch, 0.0);
        return 0;
    }
    void slot_fini(SlotData &) {}
    void thread_start() {}

    static double element(const vnp_request &q, const char *x0, int64_t k)
    {
        const int64_t esz = q.dtype == VNP_F32 ? 4 : 8;
        const char *a = x0 + k * q.incx * esz;
        if (esz == 4) {
            float f;
            memcpy(&f, a, 4);
            return f;
        }
        double d;
        memcpy(&d, a, 8);
        return d;
    }
    int launch(SlotData &d, std::vector<Pending> &reqs, int *nlaunch)
    {
        std::reverse(reqs.begin(), reqs.end());  // the backend may reorder the batch
        for (size_t i = 0; i < reqs.size(); ++i) {
            vnp_request &q = reqs[i].req;
            const int64_t esz = q.dtype == VNP_F32 ? 4 : 8;
            const char *x = static_cast<const char *>(q.x);
            const char *x0 = q.incx >= 0 || q.n <= 0 ? x : x + (q.n - 1) * (-q.incx) * esz;
            if (reqs[i].blk) {  // admission by copy: the logical elements into the block
                char *b = static_cast<char *>(reqs[i].blk);
                for (int64_t k = 0; k < q.n; ++k) memcpy(b + k * esz, x0 + k * q.incx * esz, (size_t)esz);
                q.x = b;
                q.incx = 1;
                x0 = b;
            }
            double s = 0;
            for (int64_t k = 0; k < q.n; ++k) s += element(q, x0, k);
            d.res[i] = s;
        }
        *nlaunch = 1;
        const uint64_t r = rng.fetch_add(0x9E3779B97F4A7C15ull) >> 40;
        d.ready_ns = vnp::srv::now_ns() + 5000 + (int64_t)(r % 150000);
        return 0;
    }
    int wait(SlotData &d, int)
    {
        while (vnp::srv::now_ns() < d.ready_ns) std::this_thread::sleep_for(std::chrono::microseconds(20));
        return 0;
    }
    double result(const SlotData &d, size_t i, const vnp_request &) const { return d.res[i]; }
};

using Server = vnp::srv::Server<FakeBackend>;

static int check(const vnp_request &q)
{
    return vnp::srv::request_info(q, [](const vnp_request &r) { return r.p > 0; });
}

static std::atomic<int> failures{0};
#define EXPECT(c)                                                             \
    do {                                                                      \
        if (!(c)) {                                                           \
            fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c);   \
            failures.fetch_add(1);                                            \
        }                                                                     \
    } while (0)

// Payload i of a client: n doubles (or floats) with small integer values, so every sum is
// exact in either order.
struct Payload {
    std::vector<double> d;
    std::vector<float> f;
    double sum = 0;
};

static void client(Server &s, int id, int nreq, int64_t pool_bytes)
{
    std::mt19937_64 g(1000 + id);
    for (int i = 0; i < nreq; ++i) {
        const int kind = (int)(g() % 8);
        const bool f32 = g() % 3 == 0;
        int64_t n = (int64_t)(g() % 3000);
        if (kind == 7) n = pool_bytes / 4 + 1000;  // larger than the whole pool (copy) or plain
        const int64_t inc = (g() % 4 == 0) ? -2 : 1;
        const int64_t span = n > 0 ? (n - 1) * (inc < 0 ? -inc : inc) + 1 : 1;
        Payload pl;
        if (f32)
            pl.f.assign((size_t)span, 0.0f);
        else
            pl.d.assign((size_t)span, 0.0);
        for (int64_t k = 0; k < n; ++k) {
            const double v = (double)((int64_t)(g() % 17) - 8);
            const int64_t pos = inc > 0 ? k * inc : (n - 1 - k) * (-inc);
            if (f32)
                pl.f[(size_t)pos] = (float)v;
            else
                pl.d[(size_t)pos] = v;
            pl.sum += v;
        }
        vnp_request q{f32 ? VNP_F32 : VNP_F64, (g() % 5 == 0) ? -1.0 : 2.0, n,
                      f32 ? (const void *)pl.f.data() : (const void *)pl.d.data(), inc};
        // a caller-held pool block as the payload, now and then
        void *held = nullptr;
        if (kind == 5 && n > 0 && n < 2000) {
            if (s.alloc(span * (f32 ? 4 : 8), &held) == 0) {
                memcpy(held, q.x, (size_t)(span * (f32 ? 4 : 8)));
                q.x = held;
            }
        }
        const bool copy = kind < 4 || kind == 7;
        uint64_t t = 0;
        s.submit(q, check(q), copy && !held, &t);
        vnp_result r{};
        int rc;
        if (kind == 2) {
            do {
                rc = s.take(t, &r, 0);
            } while (rc == VNP_EPENDING);
        } else if (kind == 3) {
            do {
                rc = s.take(t, &r, 50);
            } while (rc == VNP_EPENDING);
        } else {
            rc = s.take(t, &r, -1);
        }
        EXPECT(rc == 0);
        EXPECT(s.take(t, &r, 0) == VNP_ENOTFOUND);  // a ticket is released once
        if (q.p <= 0) {
            EXPECT(r.status == -2);
        } else if (kind == 7 && copy && !held) {
            EXPECT(r.status == VNP_ENOMEM);
        } else {
            EXPECT(r.status == 0);
            EXPECT(r.value == pl.sum);
        }
        if (held) EXPECT(s.release(held) == 0);
    }
}

int main()
{
    const int64_t pool_bytes = 32 << 10;  // small: copy admissions wait for each other
    {
        Server s;
        vnp_server_config cfg{pool_bytes, 16, 3, 50, 7};
        EXPECT(s.create(cfg) == 0);
        std::vector<std::thread> th;
        for (int c = 0; c < 6; ++c) th.emplace_back([&s, c, pool_bytes] { client(s, c, 400, pool_bytes); });
        for (auto &t : th) t.join();
        vnp_server_stats st{};
        s.stats(&st);
        EXPECT(st.submitted == 6 * 400);
        EXPECT(st.completed + st.rejected == st.submitted);
        EXPECT(st.pending == 0 && st.in_flight == 0);
        EXPECT(st.pool_free_bytes == pool_bytes);
        EXPECT(st.admission_waits > 0);  // the small pool made copies wait
        printf("phase 1: %lld requests, %lld batches, %lld failed batches, %lld admission waits\n",
               (long long)st.submitted, (long long)st.batches, (long long)st.failed_batches,
               (long long)st.admission_waits);
        s.destroy();
    }
    {
        // destroy with copy requests queued behind a held pool and a client blocked in wait
        Server s;
        vnp_server_config cfg{pool_bytes, 8, 2, 0, 0};
        EXPECT(s.create(cfg) == 0);
        void *all = nullptr;
        EXPECT(s.alloc(pool_bytes, &all) == 0);  // the pool is full: copies cannot be admitted
        std::vector<double> x(100, 1.0);
        vnp_request q{VNP_F64, 2.0, 100, x.data(), 1};
        std::vector<uint64_t> t(20);
        for (auto &k : t) s.submit(q, 0, true, &k);
        std::atomic<int> got{-1};
        vnp_result r{};
        std::thread w([&] { got = s.take(t.back(), &r, -1); });
        std::this_thread::sleep_for(std::chrono::milliseconds(20));
        vnp_server_stats st{};
        s.stats(&st);
        EXPECT(st.pending == 20);
        s.destroy();
        w.join();
        EXPECT(got == 0);
        EXPECT(r.status == VNP_ECANCELED);
        printf("phase 2: destroy cancelled the queued requests, the waiter returned\n");
    }
    if (failures.load()) {
        fprintf(stderr, "%d checks failed\n", failures.load());
        return 1;
    }
    printf("all checks passed\n");
    return 0;
}

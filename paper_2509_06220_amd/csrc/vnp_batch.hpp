// Host-side declarations shared by the batched launches and the request server.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "vnp_internal.hpp"

namespace vnp {

struct BatchShape {
    int lwt;     // log2(tiles per item)
    int wpb;     // waves per block
    int blocks;  // resident blocks
};

struct BatchWorkspace {
    void *roots = nullptr;
    size_t roots_cap = 0;  // bytes
    int64_t *item_off = nullptr;
    size_t item_cap = 0;  // entries
    void *vals = nullptr;  // intermediate segment norms (array norms)
    size_t vals_cap = 0;   // bytes
};

int release_workspaces();
int release_batch_workspaces();
// One class of a request batch: requests [a, a + n) of the batch (sorted by class) share
// dtype and p; items work items at lwt (from request_class_items).
struct RequestClass {
    int dtype;
    double p;
    int64_t a, n;
    int64_t items;
    int lwt;
    int multi;  // some request of the class spans more than one run
};
// Item offsets (n + 1 entries) of n requests of one dtype with lengths lens; returns the
// log2(tiles per item) they are computed for.
int request_class_items(int dtype, const int64_t *lens, int64_t n, int64_t *item_off);
// Enqueues one request batch on st: a stage kernel copies the descriptor words from h_src
// (device view of host-mapped memory; ptrs[nreq] | lens[nreq] | incs[nreq] | item
// offsets, class c's n_c + 1 entries at 3 nreq + a_c + c | for ncopy > 0 the copy table:
// {src, dst, n, inc, esz} per copy (src: logical element 0; inc in elements, may be
// negative), then ncopy + 1 prefix sums of copy_chunks(n), nchunks in all) to d_desc
// (device, at least 4 nreq + ncls + 6 ncopy + 1 words); a gather kernel copies the
// admitted payloads into their pool blocks; then one batched
// launch per class writes request i of class c to res_d[a_c + i] or res_s[a_c + i],
// followed by a finish launch for classes with requests of several runs.  ptrs are
// addresses of logical element 0 (moved for negative strides); lengths are >= 0.
int enqueue_request_batch(const void *h_src, void *d_desc, int64_t nreq, const RequestClass *cls, int ncls,
                          int64_t ncopy, int64_t nchunks, double *res_d, float *res_s, BatchWorkspace &ws,
                          hipStream_t st);
// Gather-kernel chunks of a copy of n elements.
int64_t copy_chunks(int64_t n);
// One copy of n elements (src: logical element 0, stride inc, esz bytes each) into the
// contiguous dst, by one gather launch on st.
int enqueue_copy1(const void *src, void *dst, int64_t n, int64_t inc, int64_t esz, hipStream_t st);
void release_batch_ws(BatchWorkspace &w);
int release_svd_workspaces();
int set_launch_shape(int wpb, int wt);

}  // namespace vnp

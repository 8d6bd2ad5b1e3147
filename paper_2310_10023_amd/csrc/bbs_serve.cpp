// Stream serving: many localization queries on one resident map.
//
// Workers are host threads, each owning a workspace and a HIP stream (default
// priority).  They take queries in arrival order from a shared counter, wait
// for the query's arrival time, and run bbs_localize on their stream.  The
// GPU interleaves the workers' kernels: while one search runs its
// single-workgroup serial phase, the scoring kernels of the others fill the
// remaining compute units.
#include <hip/hip_runtime.h>

#include <atomic>
#include <chrono>
#include <cstring>
#include <string>
#include <thread>
#include <vector>

#include "bbs_internal.h"

extern "C" bbs_status bbs_serve(const bbs_map *map, const bbs_query *queries, int64_t n, int32_t workers,
                                const bbs_options *opt, bbs_result *results, double *start_s, double *end_s)
{
    using bbs::fail;
    if (!map) return fail(BBS_ERR_INVALID_ARG, "bbs_serve: map is NULL");
    if (n < 0 || (n > 0 && (!queries || !results))) return fail(BBS_ERR_INVALID_ARG, "bbs_serve: bad query buffers");
    if (workers < 1 || workers > 64) return fail(BBS_ERR_INVALID_ARG, "bbs_serve: workers must be in [1, 64]");
    for (int64_t i = 0; i < n; ++i) {
        if (!(queries[i].arrival_s >= 0.0) || (i > 0 && queries[i].arrival_s < queries[i - 1].arrival_s))
            return fail(BBS_ERR_INVALID_ARG, "bbs_serve: arrival times must be >= 0 and non-decreasing");
    }
    if (n == 0) return BBS_OK;
    bbs_options o;
    bbs_default_options(&o);
    if (opt) o = *opt;
    // a persistent search is one cooperative grid sized to be resident on
    // every compute unit at once, so two of them cannot run side by side
    if (o.persistent && workers > 1)
        return fail(BBS_ERR_INVALID_ARG, "bbs_serve: the persistent kernel occupies the whole GPU; use one worker");
    int device = 0;
    hipError_t e = hipGetDevice(&device);
    if (e != hipSuccess) return bbs::hip_fail(e, "hipGetDevice");

    const int nw = (int)std::min<int64_t>(workers, n);
    std::vector<bbs_workspace *> ws(nw, nullptr);
    std::vector<hipStream_t> streams(nw, nullptr);
    bbs_status st = BBS_OK;
    for (int w = 0; w < nw && st == BBS_OK; ++w) {
        st = bbs_workspace_create(0, &ws[w]);
        if (st == BBS_OK) {
            e = hipStreamCreateWithFlags(&streams[w], hipStreamNonBlocking);
            if (e != hipSuccess) st = bbs::hip_fail(e, "hipStreamCreateWithFlags");
        }
    }
    std::atomic<int64_t> next{0};
    std::atomic<int> first_error{0};
    std::vector<std::string> errors(nw);
    const auto t0 = std::chrono::steady_clock::now();
    auto secs = [&]() { return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count(); };
    auto work = [&](int w) {
        (void)hipSetDevice(device);
        bbs_options ow = o;
        ow.stream = streams[w];
        for (;;) {
            const int64_t i = next.fetch_add(1);
            if (i >= n) break;
            const bbs_query &q = queries[i];
            double now = secs();
            if (q.arrival_s > now)
                std::this_thread::sleep_for(std::chrono::duration<double>(q.arrival_s - now));
            const double ts = secs();
            bbs_options oq = ow;
            if (q.prior) oq.prior = q.prior;
            bbs_status s = bbs_localize(map, ws[w], q.scan_xyz, q.k, q.scan_on_device, &q.range, q.score_threshold,
                                        &oq, &results[i]);
            const double te = secs();
            if (start_s) start_s[i] = ts;
            if (end_s) end_s[i] = te;
            if (s != BBS_OK) {
                std::memset(&results[i], 0, sizeof(bbs_result));
                int expect = 0;
                if (first_error.compare_exchange_strong(expect, (int)s)) errors[w] = bbs_last_error();
            }
        }
    };
    if (st == BBS_OK) {
        std::vector<std::thread> threads;
        for (int w = 0; w < nw; ++w) threads.emplace_back(work, w);
        for (auto &t : threads) t.join();
    }
    for (int w = 0; w < nw; ++w) {
        if (streams[w]) (void)hipStreamDestroy(streams[w]);
        if (ws[w]) bbs_workspace_free(ws[w]);
    }
    if (st != BBS_OK) return st;
    if (first_error.load()) {
        std::string msg;
        for (auto &m : errors)
            if (!m.empty()) msg = m;
        return fail((bbs_status)first_error.load(), "bbs_serve: " + msg);
    }
    return BBS_OK;
}

extern "C" bbs_status bbs_autotune(const bbs_map *map, const bbs_query *queries, int64_t n, const int32_t *batch_sizes,
                                   int32_t n_b, const int32_t *score_items, int32_t n_items, const bbs_options *base,
                                   bbs_tune_entry *best, bbs_tune_entry *all)
{
    using bbs::fail;
    if (!map || !queries || n < 1 || !batch_sizes || n_b < 1 || !score_items || n_items < 1 || !best)
        return fail(BBS_ERR_INVALID_ARG, "bbs_autotune: bad arguments");
    for (int i = 0; i < n_b; ++i)
        if (batch_sizes[i] < 1 || batch_sizes[i] > (1 << 24))
            return fail(BBS_ERR_INVALID_ARG, "bbs_autotune: batch size out of range");
    for (int i = 0; i < n_items; ++i)
        if (score_items[i] < 1 || score_items[i] > (1 << 20))
            return fail(BBS_ERR_INVALID_ARG, "bbs_autotune: score_items out of range");
    bbs_options o;
    bbs_default_options(&o);
    if (base) o = *base;
    o.profile = 0;
    bbs_workspace *ws = nullptr;
    bbs_status st = bbs_workspace_create(0, &ws);
    if (st) return st;
    bbs_result r;
    best->ms = -1.0;
    for (int ib = 0; ib < n_b && st == BBS_OK; ++ib)
        for (int ii = 0; ii < n_items && st == BBS_OK; ++ii) {
            o.batch_size = batch_sizes[ib];
            o.score_items = score_items[ii];
            // (a query's own prior replaces the options' prior, as in bbs_serve)
            auto run = [&](const bbs_query &Q) {
                bbs_options oq = o;
                if (Q.prior) oq.prior = Q.prior;
                return bbs_localize(map, ws, Q.scan_xyz, Q.k, Q.scan_on_device, &Q.range, Q.score_threshold, &oq, &r);
            };
            st = run(queries[0]);
            const auto t0 = std::chrono::steady_clock::now();
            for (int64_t q = 0; q < n && st == BBS_OK; ++q) st = run(queries[q]);
            const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
            if (st) break;
            if (all) all[ib * n_items + ii] = bbs_tune_entry{o.batch_size, o.score_items, ms};
            if (best->ms < 0.0 || ms < best->ms) *best = bbs_tune_entry{o.batch_size, o.score_items, ms};
        }
    bbs_workspace_free(ws);
    return st;
}

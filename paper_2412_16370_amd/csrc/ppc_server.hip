// ppc_server.hip -- serving form: count queries over device-resident columns
// with admission by memory, continuous batching over several HIP streams,
// and latency accounting.
//
// Model.  A pool of equal columns lives in device memory.  A request asks
// for pospopcnt_w of bytes [offset, offset+nbytes) of one column.  submit()
// admits a request if a result slot is free and the bytes of all admitted,
// unfinished requests stay within the in-flight budget (PPC_EBUSY
// otherwise).  The progress engine (run by poll() and by the trace driver)
// retires finished batches and, whenever one of its K streams is idle and
// requests are pending, launches them as one batch right away: pending
// requests that arrived while other batches were on the GPU are taken in
// arrival order, so work of several batches overlaps on the device.  The
// host writes a batch's tables into its stream's pinned staging buffer and
// replays that stream's graph, captured once: a kernel copies the tables to
// the device, the persistent batched kernel counts (the same arithmetic as
// the plain call), and an epilogue kernel writes the counters into pinned
// host memory, clears them and re-arms the work cursor.  An event recorded
// after the replay marks the batch done, so a batch costs the host one
// graph launch and one event record.  A request's result is identical to
// what the plain call computes for it alone.
//
// Threading: a server object is used from one host thread at a time.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <chrono>
#include <cstring>
#include <deque>
#include <new>
#include <thread>
#include <vector>

#include "ppc.h"
#include "ppc_batch.hpp"
#include "ppc_device.hpp"
#include "ppc_host.hpp"

namespace ppc {

static uint64_t now_ns() {
    return (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

struct Slot {
    ppc_request req;
    uint64_t t_submit = 0;
};

struct Lane {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    bool busy = false;
    uint64_t t_launch = 0;        // host time the batch in flight was launched
    bool failed = false;          // an enqueue of the batch in flight failed
    std::vector<uint32_t> slots;  // slot ids of the batch in flight
    // staging buffer: BatchHeader, ArrayInfo[max_batch], WorkItem[item_cap]
    // (pinned host, copied to stage_dev by the first kernel of the graph)
    uint8_t *stage_host = nullptr, *stage_dev = nullptr;
    unsigned long long *counts_dev = nullptr;  // max_batch x 64, kept zero between batches
    uint64_t *results_host = nullptr;          // max_batch x 64, written by the graph
    uint32_t *cursor_dev = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

}  // namespace ppc

using namespace ppc;

struct ppc_server {
    int device = 0;
    const uint8_t *pool = nullptr;
    uint64_t pool_bytes = 0, column_bytes = 0, n_columns = 0;
    ppc_server_cfg cfg{};
    uint32_t item_cap = 0;
    size_t items_off = 0, groups_off = 0, stage_bytes = 0;  // staging layout
    std::vector<Slot> slots;
    std::vector<uint32_t> free_slots;
    std::deque<uint32_t> pending;
    std::deque<ppc_result> completed;
    std::vector<Lane> lanes;
    uint64_t inflight_bytes = 0;
    uint32_t inflight = 0;
    uint64_t batches = 0, batched_requests = 0, max_batch_seen = 0;
    uint64_t host_dispatch_ns = 0, host_retire_ns = 0;  // host time spent enqueuing / retiring
    ppc_status sticky = PPC_OK;  // first device error
};

namespace {

void server_free(ppc_server *s) {
    if (!s) return;
    for (auto &l : s->lanes) {
        if (l.stream) (void)hipStreamSynchronize(l.stream);
        if (l.exec) (void)hipGraphExecDestroy(l.exec);
        if (l.graph) (void)hipGraphDestroy(l.graph);
        if (l.done) (void)hipEventDestroy(l.done);
        if (l.stream) (void)hipStreamDestroy(l.stream);
        if (l.stage_host) (void)hipHostFree(l.stage_host);
        if (l.results_host) (void)hipHostFree(l.results_host);
        if (l.stage_dev) (void)hipFree(l.stage_dev);
        if (l.counts_dev) (void)hipFree(l.counts_dev);
        if (l.cursor_dev) (void)hipFree(l.cursor_dev);
    }
    delete s;
}

// Retires finished batches: results move to the completed queue, slots and
// in-flight bytes are released.  A batch still running `batch_timeout_us` after its launch makes the
// server's status PPC_ETIMEDOUT: the batch stays in flight (its buffers are
// still the device's), and every later poll or trace returns that status.
void retire(ppc_server *s) {
    const uint64_t t_begin = now_ns();
    for (auto &l : s->lanes) {
        if (!l.busy) continue;
        hipError_t q = hipEventQuery(l.done);
        if (q == hipErrorNotReady) {
            if (t_begin - l.t_launch > (uint64_t)s->cfg.batch_timeout_us * 1000u && s->sticky == PPC_OK)
                s->sticky = PPC_ETIMEDOUT;
            continue;
        }
        if (l.failed) q = hipErrorUnknown;
        if (q != hipSuccess && s->sticky == PPC_OK) s->sticky = PPC_EDEVICE;
        const uint64_t t = now_ns();
        for (size_t i = 0; i < l.slots.size(); ++i) {
            const uint32_t id = l.slots[i];
            Slot &sl = s->slots[id];
            ppc_result r;
            r.tag = sl.req.tag;
            r.width = sl.req.width;
            r.status = q == hipSuccess ? PPC_OK : PPC_EDEVICE;
            r.t_submit_ns = sl.t_submit;
            r.t_done_ns = t;
            std::memcpy(r.counts, l.results_host + i * 64, sl.req.width * sizeof(uint64_t));
            std::memset(r.counts + sl.req.width, 0, (64 - sl.req.width) * sizeof(uint64_t));
            s->completed.push_back(r);
            s->inflight_bytes -= sl.req.nbytes;
            s->inflight -= 1;
            s->free_slots.push_back(id);
        }
        l.slots.clear();
        l.busy = false;
        l.failed = false;
    }
    s->host_retire_ns += now_ns() - t_begin;
}

uint32_t items_needed(const ArrayInfo &ai, uint32_t p) {
    if (ai.n_tiles == 0) return (ai.edge0_len + ai.edge1_len) ? 1u : 0u;
    return (ai.n_tiles + p - 1) / p;
}

// Launches pending requests on idle lanes.
void dispatch(ppc_server *s) {
    const uint64_t t_begin = now_ns();
    std::vector<WorkItem> items;
    for (auto &l : s->lanes) {
        if (s->pending.empty()) break;
        if (l.busy) continue;
        uint32_t n = 0, n_items = 0;
        items.clear();
        ArrayInfo *arrays = reinterpret_cast<ArrayInfo *>(l.stage_host + sizeof(BatchHeader));
        while (!s->pending.empty() && n < s->cfg.max_batch) {
            const uint32_t id = s->pending.front();
            const ppc_request &rq = s->slots[id].req;
            ArrayInfo ai;
            make_array_info(ai, s->pool + rq.column * s->column_bytes + rq.offset, rq.nbytes,
                            reinterpret_cast<uint64_t *>(l.counts_dev + (uint64_t)n * 64), rq.width);
            // a request never needs more than a quarter of the item table
            uint32_t p = s->cfg.tiles_per_item;
            while (items_needed(ai, p) > s->item_cap / 4 && p < kMaxItemTiles) p *= 2;
            p = std::min(p, kMaxItemTiles);
            const uint32_t need = items_needed(ai, p);
            if (n > 0 && n_items + need > s->item_cap) break;
            arrays[n] = ai;
            append_items(items, ai, n, p);
            n_items += need;
            l.slots.push_back(id);
            s->pending.pop_front();
            ++n;
        }
        sort_items_lpt(items);
        const std::vector<uint32_t> groups = build_groups(items, s->cfg.waves, kServedGroupCost);
        std::memcpy(l.stage_host + s->items_off, items.data(), items.size() * sizeof(WorkItem));
        std::memcpy(l.stage_host + s->groups_off, groups.data(), groups.size() * sizeof(uint32_t));
        BatchHeader *h = reinterpret_cast<BatchHeader *>(l.stage_host);
        h->n_arrays = n;
        h->n_items = (uint32_t)items.size();
        h->n_groups = (uint32_t)groups.size() - 1u;
        l.t_launch = now_ns();
        // with no other batch in flight the kernels go out directly, which
        // costs the host less than a graph launch; under load the graph
        bool others = false;
        for (const auto &o : s->lanes) others = others || (&o != &l && o.busy);
        hipError_t e = others ? hipGraphLaunch(l.exec, l.stream)
                              : enqueue_served_batch(l.stream, l.stage_host, l.stage_dev, s->items_off, s->groups_off,
                                                     l.counts_dev, l.results_host, l.cursor_dev, s->cfg.waves);
        if (e == hipSuccess) e = hipEventRecord(l.done, l.stream);
        if (e != hipSuccess) {
            l.failed = true;  // retire() reports the batch with status PPC_EDEVICE
            if (s->sticky == PPC_OK) s->sticky = PPC_EDEVICE;
        }
        l.busy = true;
        s->batches += 1;
        s->batched_requests += n;
        s->max_batch_seen = std::max<uint64_t>(s->max_batch_seen, n);
    }
    s->host_dispatch_ns += now_ns() - t_begin;
}

void progress(ppc_server *s) {
    retire(s);
    dispatch(s);
}

ppc_status validate(const ppc_server *s, const ppc_request *r) {
    if (!r) return PPC_EINVAL;
    if (!(r->width == 8 || r->width == 16 || r->width == 32 || r->width == 64)) return PPC_EINVAL;
    if (r->column >= s->n_columns) return PPC_EINVAL;
    if (r->offset > s->column_bytes || r->nbytes > s->column_bytes - r->offset) return PPC_EINVAL;
    // dispatch() fits one request into a quarter of the item table, with at
    // most kMaxItemTiles tiles per item: larger requests are refused
    const uint64_t tile_bytes = (uint64_t)kTileChunks * 16u;
    const uint64_t max_tiles = (uint64_t)(s->item_cap / 4u) * kMaxItemTiles;
    if (r->nbytes / tile_bytes + 2u > max_tiles) return PPC_EINVAL;
    return PPC_OK;
}

ppc_status admit(ppc_server *s, const ppc_request *r, uint64_t t_submit) {
    if (s->free_slots.empty()) return PPC_EBUSY;
    // an oversized request is admitted alone rather than never
    if (s->inflight > 0 && s->inflight_bytes + r->nbytes > s->cfg.inflight_bytes) return PPC_EBUSY;
    const uint32_t id = s->free_slots.back();
    s->free_slots.pop_back();
    Slot &sl = s->slots[id];
    sl.req = *r;
    sl.t_submit = t_submit;
    s->inflight_bytes += r->nbytes;
    s->inflight += 1;
    s->pending.push_back(id);
    return PPC_OK;
}

}  // namespace

extern "C" {

ppc_status ppc_server_create(ppc_server **out, const void *pool, uint64_t pool_bytes, uint64_t column_bytes,
                             const ppc_server_cfg *cfg) {
    if (!out) return PPC_EINVAL;
    *out = nullptr;
    if (!pool || pool_bytes == 0 || column_bytes == 0 || pool_bytes % column_bytes != 0) return PPC_EINVAL;
    ppc_server_cfg c{};
    if (cfg) c = *cfg;
    if (c.n_streams == 0) c.n_streams = 3;
    if (c.batch_timeout_us == 0) c.batch_timeout_us = 10000000u;  // 10 s
    if (c.max_batch == 0) c.max_batch = 4096;
    if (c.max_inflight == 0) c.max_inflight = 16384;
    if (c.tiles_per_item == 0) c.tiles_per_item = 16;
    // 16 GiB in flight lets 3 streams keep up at 0.9 of the plain call's
    // bandwidth with requests of up to 64 MiB (4 GiB caps them near 0.7)
    if (c.inflight_bytes == 0) c.inflight_bytes = (uint64_t)16 << 30;
    if (c.n_streams > 64 || c.max_batch > (1u << 20) || c.max_inflight > (1u << 24) ||
        c.tiles_per_item > kMaxItemTiles)
        return PPC_EINVAL;
    auto *s = new (std::nothrow) ppc_server();
    if (!s) return PPC_ENOMEM;
    if (hipGetDevice(&s->device) != hipSuccess) {
        server_free(s);
        return PPC_EDEVICE;
    }
    if (c.waves == 0) c.waves = 8u * (uint32_t)device_cus(s->device);
    s->pool = static_cast<const uint8_t *>(pool);
    s->pool_bytes = pool_bytes;
    s->column_bytes = column_bytes;
    s->n_columns = pool_bytes / column_bytes;
    s->cfg = c;
    s->item_cap = std::max<uint32_t>(4096u, 16u * c.max_batch);
    s->slots.resize(c.max_inflight);
    s->free_slots.reserve(c.max_inflight);
    for (uint32_t i = c.max_inflight; i-- > 0;) s->free_slots.push_back(i);
    s->lanes.resize(c.n_streams);
    s->items_off = sizeof(BatchHeader) + (size_t)c.max_batch * sizeof(ArrayInfo);
    s->groups_off = s->items_off + (size_t)s->item_cap * sizeof(WorkItem);
    s->stage_bytes = s->groups_off + ((size_t)s->item_cap + 1) * sizeof(uint32_t);
    const size_t counts_bytes = (size_t)c.max_batch * 64 * sizeof(uint64_t);
    for (auto &l : s->lanes) {
        bool ok = hipStreamCreateWithFlags(&l.stream, hipStreamNonBlocking) == hipSuccess &&
                  hipEventCreateWithFlags(&l.done, hipEventDisableTiming) == hipSuccess &&
                  // coherent (uncached on the device) so every batch sees the
                  // host's new tables and the host sees the new results
                  hipHostMalloc((void **)&l.stage_host, s->stage_bytes, hipHostMallocCoherent) == hipSuccess &&
                  hipHostMalloc((void **)&l.results_host, counts_bytes, hipHostMallocCoherent) == hipSuccess &&
                  hipMalloc(&l.stage_dev, s->stage_bytes) == hipSuccess &&
                  hipMalloc(&l.counts_dev, counts_bytes) == hipSuccess &&
                  hipMalloc(&l.cursor_dev, sizeof(uint32_t)) == hipSuccess;
        // counters and cursor start at zero; the graph's last kernel leaves
        // them at zero after every batch
        ok = ok && hipMemset(l.counts_dev, 0, counts_bytes) == hipSuccess &&
             hipMemset(l.cursor_dev, 0, sizeof(uint32_t)) == hipSuccess &&
             hipDeviceSynchronize() == hipSuccess;
        if (ok) std::memset(l.stage_host, 0, sizeof(BatchHeader));
        ok = ok && capture_served_graph(&l.graph, &l.exec, l.stage_host, l.stage_dev, s->items_off, s->groups_off,
                                        l.counts_dev, l.results_host, l.cursor_dev, c.waves) == hipSuccess;
        if (!ok) {
            server_free(s);
            return PPC_ENOMEM;
        }
        l.slots.reserve(c.max_batch);
    }
    *out = s;
    return PPC_OK;
}

ppc_status ppc_server_submit(ppc_server *s, const ppc_request *req) {
    if (!s) return PPC_EINVAL;
    if (s->sticky != PPC_OK) return s->sticky;  // failed or timed out: no new work
    ppc_status rc = validate(s, req);
    if (rc != PPC_OK) return rc;
    rc = admit(s, req, now_ns());
    progress(s);
    return rc;
}

ppc_status ppc_server_poll(ppc_server *s, ppc_result *out, size_t cap, size_t *n_out) {
    if (!s || !n_out || (cap > 0 && !out)) return PPC_EINVAL;
    progress(s);
    size_t n = 0;
    while (n < cap && !s->completed.empty()) {
        out[n++] = s->completed.front();
        s->completed.pop_front();
    }
    *n_out = n;
    return s->sticky;
}

ppc_status ppc_server_get_stats(const ppc_server *s, ppc_server_stats *st) {
    if (!s || !st) return PPC_EINVAL;
    st->inflight = s->inflight;
    st->pending = s->pending.size();
    st->inflight_bytes = s->inflight_bytes;
    st->batches = s->batches;
    st->batched_requests = s->batched_requests;
    st->max_batch_seen = s->max_batch_seen;
    st->host_dispatch_ns = s->host_dispatch_ns;
    st->host_retire_ns = s->host_retire_ns;
    return PPC_OK;
}

ppc_status ppc_server_run_trace(ppc_server *s, const ppc_request *reqs, const uint64_t *arrival_ns, size_t n,
                                ppc_result *results, ppc_trace_stats *stats) {
    if (!s || (n > 0 && (!reqs || !arrival_ns || !results))) return PPC_EINVAL;
    for (size_t i = 0; i < n; ++i) {
        if (validate(s, &reqs[i]) != PPC_OK) return PPC_EINVAL;
        if (i > 0 && arrival_ns[i] < arrival_ns[i - 1]) return PPC_EINVAL;
    }
    if (!s->completed.empty() || s->inflight != 0) return PPC_EBUSY;  // needs an idle server
    const uint64_t b0 = s->batches, r0 = s->batched_requests;
    const uint64_t d0 = s->host_dispatch_ns, rr0 = s->host_retire_ns;
    std::vector<uint64_t> lat(n, 0);
    std::deque<size_t> backlog;
    uint64_t rejections = 0, total_bytes = 0;
    size_t next = 0, done = 0;
    const uint64_t t0 = now_ns();
    uint64_t t_last = t0;
    while (done < n) {
        const uint64_t now = now_ns();
        while (next < n && t0 + arrival_ns[next] <= now) backlog.push_back(next++);
        while (!backlog.empty()) {
            const size_t i = backlog.front();
            ppc_request r = reqs[i];
            r.tag = i;
            if (admit(s, &r, t0 + arrival_ns[i]) != PPC_OK) {
                ++rejections;
                break;
            }
            backlog.pop_front();
        }
        progress(s);
        bool idle = true;
        while (!s->completed.empty()) {
            const ppc_result &r = s->completed.front();
            const size_t i = (size_t)r.tag;
            results[i] = r;
            lat[i] = r.t_done_ns - (t0 + arrival_ns[i]);
            t_last = std::max(t_last, r.t_done_ns);
            total_bytes += reqs[i].nbytes;
            s->completed.pop_front();
            ++done;
            idle = false;
        }
        if (s->sticky != PPC_OK) return s->sticky;
        if (idle && backlog.empty() && s->inflight == 0 && next < n) {
            // nothing in flight: sleep until shortly before the next arrival
            const uint64_t wake = t0 + arrival_ns[next];
            const uint64_t t = now_ns();
            if (wake > t + 50000) std::this_thread::sleep_for(std::chrono::nanoseconds(wake - t - 20000));
        }
    }
    if (stats) {
        std::memset(stats, 0, sizeof *stats);
        stats->n_requests = n;
        stats->total_bytes = total_bytes;
        stats->makespan_ns = t_last - t0;
        std::vector<uint64_t> sorted = lat;
        std::sort(sorted.begin(), sorted.end());
        if (n > 0) {
            stats->p50_ns = sorted[(n - 1) / 2];
            stats->p99_ns = sorted[std::min(n - 1, (size_t)((n - 1) * 0.99 + 0.5))];
            stats->max_ns = sorted[n - 1];
            long double sum = 0;
            for (uint64_t v : sorted) sum += v;
            stats->mean_ns = (uint64_t)(sum / n);
        }
        stats->batches = s->batches - b0;
        stats->mean_batch = stats->batches ? (double)(s->batched_requests - r0) / stats->batches : 0.0;
        stats->busy_rejections = rejections;
        stats->host_dispatch_ns = s->host_dispatch_ns - d0;
        stats->host_retire_ns = s->host_retire_ns - rr0;
        stats->gbps = stats->makespan_ns ? (double)total_bytes / (double)stats->makespan_ns : 0.0;
    }
    return PPC_OK;
}

ppc_status ppc_server_destroy(ppc_server *s) {
    if (!s) return PPC_EINVAL;
    server_free(s);
    return PPC_OK;
}

}  // extern "C"

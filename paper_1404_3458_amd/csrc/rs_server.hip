// rs_server.hip -- the serving loop of librs_nb.so (rs_server_* in rs.h):
// continuous batching of encode and decode requests over the batched codec
// calls, first-in first-out admission by a device-memory budget, several
// streams so that batches overlap, and completion tracking by events.
//
// One scheduler thread per server repeatedly (1) retires batches whose event
// has completed, stamping their requests' completion time and releasing
// their bytes, and (2) while a stream has no batch in flight, admits queued
// requests in arrival order while they fit the budget and launches them as
// one encode batch and one decode batch on that stream (after waiting, on
// that stream, for the events of the producer streams the requests name).
#include "rs.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

namespace {

int64_t now_ns()
{
    return std::chrono::duration_cast<std::chrono::nanoseconds>(std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

int pow2ceil(int v)
{
    int p = 1;
    while (p < v)
        p <<= 1;
    return p;
}

struct Req {
    rs_request r;
    std::vector<uint8_t> mask;
    size_t bytes;
    hipEvent_t ready;         // recorded on the request's producer stream, or null
};

struct Batch {
    int stream;
    hipEvent_t ev;
    std::vector<Req> reqs;
    std::vector<int> status;  // per request
    size_t bytes;
};

// Device bytes a request keeps in flight: its codeword rows, the scratch of
// the pass pipelines (mother codes over 256 points, and encodes over 256
// points with several parity blocks) and, for a decode, the per-point
// locator tables (20 dwords each at r = 16).
size_t request_bytes(const rs_request &q)
{
    const rs_stripe_desc &d = q.desc;
    const size_t rb = d.row_bytes;
    const int kp = pow2ceil(d.k), np = pow2ceil(kp + d.n - d.k);
    size_t b = (size_t)d.n * rb;
    if (q.op == RS_OP_DECODE) {
        b += (size_t)np * 80;
        if (np > 256)
            b += 2 * (size_t)np * rb;
    } else if (kp > 256 || (kp == 256 && np > 512)) {
        b += 2 * (size_t)kp * rb;
    }
    return b;
}

}  // namespace

namespace nb {
int check_stripe(rs_ctx *ctx, const rs_stripe_desc &d, bool decode, const uint8_t *mask);
}

struct rs_server {
    rs_ctx *ctx = nullptr;
    int device = 0;
    size_t budget = 0;
    int max_batch = 1;
    std::vector<hipStream_t> streams;
    std::vector<int> busy;                 // batches in flight per stream
    std::vector<hipEvent_t> ev_pool;

    std::mutex mu;
    std::condition_variable cv_work;       // new requests or stop
    std::condition_variable cv_done;       // new completions
    std::deque<Req> queue;                 // submitted, not admitted
    std::deque<Batch> inflight;
    std::deque<rs_completion> done;
    size_t inflight_bytes = 0;
    rs_server_stats stats = {};
    int pending = 0;
    bool stop = false;
    std::thread thr;

    hipEvent_t take_event();              // caller holds mu
    void launch(Batch &b);                // without mu
    void loop();
};

hipEvent_t rs_server::take_event()
{
    if (ev_pool.empty()) {
        hipEvent_t e;
        if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess)
            return nullptr;
        return e;
    }
    hipEvent_t e = ev_pool.back();
    ev_pool.pop_back();
    return e;
}

// Queue the batch's requests on its stream: first the waits on their
// producers, then one batched encode call and one batched decode call.  A
// batched call that fails is rerun request by request, so that every
// request gets its own status (the checks at submit make this rare: it
// takes a device or allocation failure).
void rs_server::launch(Batch &b)
{
    hipStream_t s = streams[b.stream];
    b.status.assign(b.reqs.size(), RS_OK);
    for (size_t i = 0; i < b.reqs.size(); i++)
        if (b.reqs[i].ready && hipStreamWaitEvent(s, b.reqs[i].ready, 0) != hipSuccess)
            b.status[i] = RS_EDEVICE;
    for (int op = RS_OP_ENCODE; op <= RS_OP_DECODE; op++) {
        std::vector<rs_stripe_desc> descs;
        std::vector<uint8_t> masks;
        std::vector<size_t> idx;
        for (size_t i = 0; i < b.reqs.size(); i++) {
            const Req &r = b.reqs[i];
            if (r.r.op != op || b.status[i] != RS_OK)
                continue;
            descs.push_back(r.r.desc);
            masks.insert(masks.end(), r.mask.begin(), r.mask.end());
            idx.push_back(i);
        }
        if (descs.empty())
            continue;
        int rc = op == RS_OP_ENCODE ? rs_encode_batch(ctx, descs.data(), (int)descs.size(), s)
                                    : rs_decode_batch(ctx, descs.data(), masks.data(), (int)descs.size(), s);
        if (rc == RS_OK)
            continue;
        size_t moff = 0;
        for (size_t j = 0; j < idx.size(); j++) {
            const Req &r = b.reqs[idx[j]];
            b.status[idx[j]] = op == RS_OP_ENCODE ? rs_encode_batch(ctx, &r.r.desc, 1, s)
                                                  : rs_decode_batch(ctx, &r.r.desc, masks.data() + moff, 1, s);
            moff += r.mask.size();
        }
        std::lock_guard<std::mutex> lk(mu);
        stats.retried += idx.size();
    }
}

void rs_server::loop()
{
    (void)hipSetDevice(device);
    std::unique_lock<std::mutex> lk(mu);
    while (true) {
        bool progress = false;
        // (1) retire completed batches
        for (auto it = inflight.begin(); it != inflight.end();) {
            const hipError_t q = hipEventQuery(it->ev);
            if (q == hipErrorNotReady) {
                ++it;
                continue;
            }
            const int64_t t = now_ns();
            for (size_t i = 0; i < it->reqs.size(); i++) {
                const Req &r = it->reqs[i];
                done.push_back({r.r.tag, q == hipSuccess ? it->status[i] : RS_EDEVICE, t});
                if (r.ready)
                    ev_pool.push_back(r.ready);
            }
            inflight_bytes -= it->bytes;
            busy[it->stream]--;
            ev_pool.push_back(it->ev);
            it = inflight.erase(it);
            progress = true;
        }
        if (progress)
            cv_done.notify_all();
        // (2) admit and launch on idle streams
        for (size_t si = 0; si < streams.size() && !queue.empty(); si++) {
            if (busy[si])
                continue;
            Batch b;
            b.stream = (int)si;
            b.bytes = 0;
            bool oversize = false;
            while (!queue.empty() && (int)b.reqs.size() < max_batch) {
                const size_t need = queue.front().bytes;
                const bool alone = inflight_bytes == 0 && b.reqs.empty();
                if (!alone && inflight_bytes + b.bytes + need > budget)
                    break;
                oversize = alone && need > budget;
                b.bytes += need;
                b.reqs.push_back(std::move(queue.front()));
                queue.pop_front();
                if (oversize)
                    break;                  // nothing joins a request above the budget
            }
            if (b.reqs.empty())
                break;                      // the head does not fit yet
            inflight_bytes += b.bytes;
            stats.admitted += b.reqs.size();
            stats.batches++;
            stats.peak_bytes = std::max<uint64_t>(stats.peak_bytes, inflight_bytes);
            if (oversize) {
                stats.oversize_admitted++;
                stats.largest_oversize = std::max<uint64_t>(stats.largest_oversize, b.bytes);
            } else {
                stats.peak_shared_bytes = std::max<uint64_t>(stats.peak_shared_bytes, inflight_bytes);
            }
            busy[si]++;
            b.ev = take_event();
            lk.unlock();
            launch(b);                      // outside the lock
            hipEvent_t unused = nullptr;
            if (b.ev && hipEventRecord(b.ev, streams[si]) != hipSuccess) {
                unused = b.ev;
                b.ev = nullptr;
            }
            if (!b.ev) {                    // no completion event: wait here instead
                (void)hipStreamSynchronize(streams[si]);
                for (int &st : b.status)
                    if (st == RS_OK)
                        st = RS_EDEVICE;
            }
            lk.lock();
            if (unused)
                ev_pool.push_back(unused);
            if (!b.ev) {                    // no event: waited for the stream above
                const int64_t t = now_ns();
                for (size_t i = 0; i < b.reqs.size(); i++) {
                    done.push_back({b.reqs[i].r.tag, b.status[i], t});
                    if (b.reqs[i].ready)
                        ev_pool.push_back(b.reqs[i].ready);
                }
                inflight_bytes -= b.bytes;
                busy[si]--;
                cv_done.notify_all();
            } else {
                inflight.push_back(std::move(b));
            }
            progress = true;
        }
        if (stop && queue.empty() && inflight.empty())
            break;
        if (!progress) {
            if (inflight.empty())
                cv_work.wait(lk, [&] { return stop || !queue.empty(); });
            else {
                // a batch is on the device: poll its event again shortly
                lk.unlock();
                std::this_thread::sleep_for(std::chrono::microseconds(20));
                lk.lock();
            }
        }
    }
}

extern "C" {

__attribute__((visibility("default"))) int rs_server_create(rs_ctx *ctx, size_t budget_bytes, int max_batch,
                                                            int nstreams, rs_server **out)
{
    if (!ctx || !out || budget_bytes == 0 || max_batch < 1 || nstreams < 1 || nstreams > 16)
        return RS_EINVAL;
    *out = nullptr;
    rs_server *s = new (std::nothrow) rs_server();
    if (!s)
        return RS_ENOMEM;
    if (hipGetDevice(&s->device) != hipSuccess) {
        delete s;
        return RS_EDEVICE;
    }
    s->ctx = ctx;
    s->budget = budget_bytes;
    s->max_batch = max_batch;
    for (int i = 0; i < nstreams; i++) {
        hipStream_t st;
        if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
            for (hipStream_t x : s->streams)
                (void)hipStreamDestroy(x);
            delete s;
            return RS_EDEVICE;
        }
        s->streams.push_back(st);
        s->busy.push_back(0);
    }
    s->thr = std::thread([s] { s->loop(); });
    *out = s;
    return RS_OK;
}

__attribute__((visibility("default"))) int rs_server_submit(rs_server *s, const rs_request *req)
{
    if (!s || !req)
        return RS_EINVAL;
    const rs_stripe_desc &d = req->desc;
    if (req->op != RS_OP_ENCODE && req->op != RS_OP_DECODE)
        return RS_EINVAL;
    const bool decode = req->op == RS_OP_DECODE;
    if (decode && !req->mask)
        return RS_EINVAL;
    const int rc = nb::check_stripe(s->ctx, d, decode, decode ? req->mask : nullptr);
    if (rc != RS_OK)
        return rc;
    Req r;
    r.r = *req;
    if (decode)
        r.mask.assign(req->mask, req->mask + d.n);
    r.r.mask = nullptr;
    r.r.after = nullptr;
    r.bytes = request_bytes(r.r);
    r.ready = nullptr;
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stop)
        return RS_EINVAL;
    if (req->after) {
        r.ready = s->take_event();
        if (!r.ready)
            return RS_EDEVICE;
        if (hipEventRecord(r.ready, (hipStream_t)req->after) != hipSuccess) {
            s->ev_pool.push_back(r.ready);
            return RS_EDEVICE;
        }
    }
    s->queue.push_back(std::move(r));
    s->pending++;
    s->cv_work.notify_one();
    return RS_OK;
}

__attribute__((visibility("default"))) int rs_server_poll(rs_server *s, rs_completion *out, int max, int timeout_ms)
{
    if (!s || (max > 0 && !out) || max < 0)
        return RS_EINVAL;
    std::unique_lock<std::mutex> lk(s->mu);
    if (s->done.empty() && timeout_ms != 0) {
        auto ready = [&] { return !s->done.empty(); };
        if (timeout_ms < 0)
            s->cv_done.wait(lk, [&] { return ready() || s->pending == 0; });
        else
            s->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), ready);
    }
    int n = 0;
    while (n < max && !s->done.empty()) {
        out[n++] = s->done.front();
        s->done.pop_front();
        s->pending--;
    }
    return n;
}

__attribute__((visibility("default"))) int rs_server_pending(rs_server *s)
{
    if (!s)
        return RS_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    return s->pending;
}

__attribute__((visibility("default"))) int rs_server_get_stats(rs_server *s, rs_server_stats *out)
{
    if (!s || !out)
        return RS_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    *out = s->stats;
    out->budget = s->budget;
    out->inflight_bytes = s->inflight_bytes;
    return RS_OK;
}

__attribute__((visibility("default"))) void rs_server_free(rs_server *s)
{
    if (!s)
        return;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv_work.notify_all();
    if (s->thr.joinable())
        s->thr.join();
    (void)hipSetDevice(s->device);
    for (hipStream_t x : s->streams) {
        (void)hipStreamSynchronize(x);
        (void)hipStreamDestroy(x);
    }
    for (hipEvent_t e : s->ev_pool)
        if (e)
            (void)hipEventDestroy(e);
    delete s;
}

}  // extern "C"

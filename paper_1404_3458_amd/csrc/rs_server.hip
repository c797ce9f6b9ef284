// rs_server.hip -- the serving loop of librs_nb.so (rs_server_* in rs.h):
// continuous batching of encode and decode requests over the batched codec
// calls, first-in first-out admission by a device-memory budget, several
// streams so that batches overlap, and completion tracking by events.
//
// One scheduler thread per server repeatedly (1) retires batches whose event
// has completed, stamping their requests' completion time and releasing
// their bytes, and (2) while a stream has no batch in flight, admits queued
// requests in arrival order while they fit the budget and launches them as
// one encode batch and one decode batch on that stream.
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
};

struct Batch {
    int stream;
    hipEvent_t ev;
    std::vector<Req> reqs;
    size_t bytes;
    int status;
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
    int pending = 0;
    bool stop = false;
    std::thread thr;

    void loop();
};

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
            const int st = q == hipSuccess ? it->status : RS_EDEVICE;
            for (const Req &r : it->reqs)
                done.push_back({r.r.tag, st, t});
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
            b.status = RS_OK;
            while (!queue.empty() && (int)b.reqs.size() < max_batch) {
                const size_t need = queue.front().bytes;
                const bool alone = inflight_bytes == 0 && b.reqs.empty();
                if (!alone && inflight_bytes + b.bytes + need > budget)
                    break;
                b.bytes += need;
                b.reqs.push_back(std::move(queue.front()));
                queue.pop_front();
            }
            if (b.reqs.empty())
                break;                      // the head does not fit yet
            inflight_bytes += b.bytes;
            busy[si]++;
            if (ev_pool.empty()) {
                hipEvent_t e;
                if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess)
                    e = nullptr;
                ev_pool.push_back(e);
            }
            b.ev = ev_pool.back();
            ev_pool.pop_back();
            lk.unlock();
            // build the two batches outside the lock
            std::vector<rs_stripe_desc> enc, dec;
            std::vector<uint8_t> masks;
            for (const Req &r : b.reqs) {
                if (r.r.op == RS_OP_ENCODE) {
                    enc.push_back(r.r.desc);
                } else {
                    dec.push_back(r.r.desc);
                    masks.insert(masks.end(), r.mask.begin(), r.mask.end());
                }
            }
            hipStream_t s = streams[si];
            int rc = RS_OK;
            if (!enc.empty())
                rc = rs_encode_batch(ctx, enc.data(), (int)enc.size(), s);
            if (!rc && !dec.empty())
                rc = rs_decode_batch(ctx, dec.data(), masks.data(), (int)dec.size(), s);
            if (!b.ev || hipEventRecord(b.ev, s) != hipSuccess) {
                if (!rc)
                    rc = RS_EDEVICE;
                (void)hipStreamSynchronize(s);
            }
            b.status = rc;
            lk.lock();
            if (!b.ev) {                    // no event: completed synchronously above
                const int64_t t = now_ns();
                for (const Req &r : b.reqs)
                    done.push_back({r.r.tag, rc, t});
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
    if (d.k < 1 || d.n <= d.k)
        return RS_ESHAPE;
    Req r;
    r.r = *req;
    if (req->op == RS_OP_DECODE) {
        if (!req->mask)
            return RS_EINVAL;
        r.mask.assign(req->mask, req->mask + d.n);
        int e = 0;
        for (int t = 0; t < d.n; t++)
            e += r.mask[t] ? 1 : 0;
        if (e > d.n - d.k)
            return RS_ETOOMANY;
    }
    r.r.mask = nullptr;
    r.bytes = request_bytes(r.r);
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->stop)
            return RS_EINVAL;
        s->queue.push_back(std::move(r));
        s->pending++;
    }
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

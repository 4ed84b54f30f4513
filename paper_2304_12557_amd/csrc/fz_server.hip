// fz_server.hip -- request server of libfzmi: compress and decompress
// requests on one GPU with continuous batching and HBM admission.
//
// Requests arrive from any host thread.  A worker thread moves them through
//   pending  -- waits for the HBM budget (admission, first come first served)
//   ready    -- admitted; launched at the next free slot
//   slot     -- a batch of up to max_batch ready requests running on the
//               slot's stream (batch plans of fz_batch.hip), finished when the
//               slot's event completes
// so requests that arrive while others are on the GPU join the next batch as
// soon as a slot and budget free up, and the batches of different slots
// overlap on the device.  Each slot owns preallocated device table areas and
// pinned staging for its plans: serving allocates nothing per request.  A
// request whose tables do not fit a slot's area runs through the per-field
// path on the slot's stream.  Every result is the per-field call's result:
// the batch kernels run the same per-chunk and per-field code.
//
// Latency is measured on the host from submit to the worker observing the
// completion of the request's batch (event polling every ~20 us).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "fz.h"
#include "fz_batch.hpp"
#include "fz_kernels.hpp"

using namespace fz;

namespace {

using Clock = std::chrono::steady_clock;

constexpr size_t kAreaBytes = 8u << 20;  // device tables of one plan kind, per slot

struct Req {
    fz_request r;
    uint64_t bytes = 0;  // admission charge
    uint64_t input_bytes = 0;
    Clock::time_point t_submit, t_done;
    int status = FZ_OK;
    bool done = false;
    bool waited_admission = false;
};

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t ev = nullptr;
    void* dev = nullptr;     // [compress area | decompress area]
    void* stage = nullptr;   // staging slots of the slot's compression batches
    void* pinned = nullptr;  // host staging of the same layout
    std::vector<uint64_t> tickets;
    bool busy = false;
};

}  // namespace

struct fz_server {
    int device = 0;
    uint64_t budget = 0, inflight = 0, inflight_max = 0;
    int max_batch = 1;
    std::vector<Slot> slots;
    std::deque<uint64_t> pending, ready;
    std::unordered_map<uint64_t, Req> reqs;
    uint64_t next_ticket = 1;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    bool stop = false;
    std::thread worker;
    // statistics
    std::vector<double> lat_ms;
    uint64_t submitted = 0, completed = 0, batches = 0, batched = 0, admission_waits = 0, input_bytes = 0;
    Clock::time_point t_first, t_last;
    bool any = false;
};

namespace {

uint64_t field_values(const fz_dims& d)
{
    uint64_t n = 1;
    for (uint32_t i = 0; i < d.rank && i < 3; i++) n *= d.n[i];
    return n;
}

// Launch one batch of requests on a slot (worker thread, lock held).
int launch(fz_server* S, Slot& sl, const std::vector<uint64_t>& tickets)
{
    std::vector<fz_compress_job> cj;
    std::vector<fz_decompress_job> dj;
    for (uint64_t t : tickets) {
        const fz_request& r = S->reqs[t].r;
        if (r.kind == FZ_REQ_COMPRESS) {
            fz_compress_job j;
            std::memset(&j, 0, sizeof(j));
            j.d_in = static_cast<const float*>(r.d_in);
            j.dims = r.dims;
            j.eb = r.eb;
            j.eb_mode = r.eb_mode;
            j.d_out = r.d_out;
            cj.push_back(j);
        } else {
            fz_decompress_job j;
            std::memset(&j, 0, sizeof(j));
            j.d_stream = r.d_in;
            j.dims = r.dims;
            j.d_out = static_cast<float*>(r.d_out);
            j.d_err = r.d_err;
            j.stream_bytes = r.stream_bytes;
            dj.push_back(j);
        }
    }
    // the caller's work that produces the inputs (and last uses the outputs)
    for (uint64_t t : tickets) {
        const fz_request& r = S->reqs[t].r;
        if (r.ready_event && hipStreamWaitEvent(sl.stream, static_cast<hipEvent_t>(r.ready_event), 0) != hipSuccess)
            return FZ_ERR_HIP;
    }
    uint8_t* dev = static_cast<uint8_t*>(sl.dev);
    uint8_t* pin = static_cast<uint8_t*>(sl.pinned);
    for (int kind = 0; kind < 2; kind++) {
        const int n = kind == 0 ? (int)cj.size() : (int)dj.size();
        if (n == 0) continue;
        Plan P;
        int rc = kind == 0 ? plan_compress(&P, n, cj.data()) : plan_decompress(&P, n, dj.data());
        if (rc != FZ_OK) return rc;
        std::vector<uint8_t> img;
        const size_t bytes = plan_layout(&P, 0, &img);
        if (bytes <= kAreaBytes) {
            std::memcpy(pin + kind * kAreaBytes, img.data(), bytes);
            if (hipMemcpyAsync(dev + kind * kAreaBytes, pin + kind * kAreaBytes, bytes, hipMemcpyHostToDevice,
                               sl.stream) != hipSuccess)
                return FZ_ERR_HIP;
            plan_bind(&P, dev + kind * kAreaBytes);
            P.d_stage = sl.stage;
            if (plan_run(&P, sl.stream) != hipSuccess) return FZ_ERR_HIP;
        } else {  // too many chunks for the slot's tables: per-field launches
            for (int i = 0; i < n; i++) {
                rc = kind == 0 ? fz_compress(cj[i].d_in, &cj[i].dims, cj[i].eb, cj[i].eb_mode, cj[i].d_out, sl.stream)
                               : fz_decompress(dj[i].d_stream, dj[i].stream_bytes, dj[i].d_out, &dj[i].dims,
                                               dj[i].d_err, sl.stream);
                if (rc != FZ_OK) return rc;
            }
        }
    }
    return hipEventRecord(sl.ev, sl.stream) == hipSuccess ? FZ_OK : FZ_ERR_HIP;
}

void finish(fz_server* S, uint64_t t, int status, Clock::time_point now)
{
    Req& R = S->reqs[t];
    R.done = true;
    R.status = status;
    R.t_done = now;
    S->inflight -= R.bytes;
    S->completed++;
    S->input_bytes += R.input_bytes;
    S->lat_ms.push_back(std::chrono::duration<double, std::milli>(now - R.t_submit).count());
    S->t_last = now;
}

void loop(fz_server* S)
{
    (void)hipSetDevice(S->device);
    std::unique_lock<std::mutex> lk(S->mu);
    for (;;) {
        bool progress = false, busy = false;
        // retire finished batches
        for (Slot& sl : S->slots) {
            if (!sl.busy) continue;
            const hipError_t q = hipEventQuery(sl.ev);
            if (q == hipErrorNotReady) {
                busy = true;
                continue;
            }
            const Clock::time_point now = Clock::now();
            for (uint64_t t : sl.tickets) finish(S, t, q == hipSuccess ? FZ_OK : FZ_ERR_HIP, now);
            sl.tickets.clear();
            sl.busy = false;
            progress = true;
        }
        if (progress) S->cv_done.notify_all();
        // admit in arrival order while the budget allows
        while (!S->pending.empty()) {
            Req& R = S->reqs[S->pending.front()];
            if (S->inflight + R.bytes > S->budget) {
                if (!R.waited_admission) {
                    R.waited_admission = true;
                    S->admission_waits++;
                }
                break;
            }
            S->inflight += R.bytes;
            S->inflight_max = std::max(S->inflight_max, S->inflight);
            S->ready.push_back(S->pending.front());
            S->pending.pop_front();
            progress = true;
        }
        // launch ready requests on free slots
        for (Slot& sl : S->slots) {
            if (S->ready.empty()) break;
            if (sl.busy) continue;
            std::vector<uint64_t> take;
            while (!S->ready.empty() && (int)take.size() < S->max_batch) {
                take.push_back(S->ready.front());
                S->ready.pop_front();
            }
            const int rc = launch(S, sl, take);
            if (rc != FZ_OK) {  // nothing of this batch can be trusted: finish it with the error
                (void)hipStreamSynchronize(sl.stream);
                const Clock::time_point now = Clock::now();
                for (uint64_t t : take) finish(S, t, rc, now);
                S->cv_done.notify_all();
            } else {
                sl.tickets = take;
                sl.busy = true;
                busy = true;
                S->batches++;
                S->batched += take.size();
            }
            progress = true;
        }
        if (S->stop && !busy && S->pending.empty() && S->ready.empty()) break;
        if (progress) continue;
        if (busy) {  // poll the running batches
            lk.unlock();
            std::this_thread::sleep_for(std::chrono::microseconds(20));
            lk.lock();
        } else {
            S->cv_work.wait(lk, [&] { return S->stop || !S->pending.empty(); });
        }
    }
}

void release(fz_server* S)
{
    for (Slot& sl : S->slots) {
        if (sl.ev) (void)hipEventDestroy(sl.ev);
        if (sl.stream) (void)hipStreamDestroy(sl.stream);
        if (sl.dev) (void)hipFree(sl.dev);
        if (sl.stage) (void)hipFree(sl.stage);
        if (sl.pinned) (void)hipHostFree(sl.pinned);
    }
    S->slots.clear();
}

}  // namespace

extern "C" {

int fz_server_create(uint64_t hbm_budget, int slots, int max_batch, fz_server** out)
{
    if (!out) return FZ_ERR_ARG;
    *out = nullptr;
    if (hbm_budget == 0 || slots < 1 || slots > 16 || max_batch < 1 || max_batch > 4096) return FZ_ERR_ARG;
    fz_server* S = new (std::nothrow) fz_server();
    if (!S) return FZ_ERR_ARG;
    S->budget = hbm_budget;
    S->max_batch = max_batch;
    if (hipGetDevice(&S->device) != hipSuccess) {
        delete S;
        return FZ_ERR_HIP;
    }
    S->slots.resize(slots);
    for (Slot& sl : S->slots) {
        if (hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&sl.ev, hipEventDisableTiming) != hipSuccess ||
            hipMalloc(&sl.dev, 2 * kAreaBytes) != hipSuccess || hipHostMalloc(&sl.pinned, 2 * kAreaBytes, 0) != hipSuccess ||
            hipMalloc(&sl.stage, stage_bytes(cu_count())) != hipSuccess) {
            release(S);
            delete S;
            return FZ_ERR_HIP;
        }
    }
    S->worker = std::thread(loop, S);
    *out = S;
    return FZ_OK;
}

int fz_server_submit(fz_server* S, const fz_request* r, uint64_t* ticket)
{
    if (!S || !r || !ticket) return FZ_ERR_ARG;
    Geom g;
    if (!r->d_in || !r->d_out || !make_geom((int)r->dims.rank, r->dims.n, &g)) return FZ_ERR_ARG;
    const uint64_t n = field_values(r->dims);
    uint64_t bytes = r->hbm_bytes;
    if (r->kind == FZ_REQ_COMPRESS) {
        if (!(r->eb > 0.0) || !std::isfinite(r->eb) || (r->eb_mode != FZ_EB_ABS && r->eb_mode != FZ_EB_REL))
            return FZ_ERR_ARG;
        if (!aligned_to(r->d_in, 4) || !aligned_to(r->d_out, 256)) return FZ_ERR_ARG;
        float e2, iv;
        if (r->eb_mode == FZ_EB_ABS && !abs_params(r->eb, &e2, &iv)) return FZ_ERR_EB_RANGE;
        if (!bytes) bytes = 4 * n + (uint64_t)g.bound;
    } else if (r->kind == FZ_REQ_DECOMPRESS) {
        if (!aligned_to(r->d_in, 256) || !aligned_to(r->d_out, 4) || !aligned_to(r->d_err, 4) ||
            r->stream_bytes < (uint64_t)g.payload_off)
            return FZ_ERR_ARG;
        if (!bytes) bytes = 4 * n + r->stream_bytes;
    } else {
        return FZ_ERR_ARG;
    }
    std::lock_guard<std::mutex> lk(S->mu);
    if (bytes > S->budget || S->stop) return FZ_ERR_ARG;  // could never be admitted
    const uint64_t t = S->next_ticket++;
    Req& R = S->reqs[t];
    R.r = *r;
    R.bytes = bytes;
    R.input_bytes = 4 * n;
    R.t_submit = Clock::now();
    if (!S->any) {
        S->any = true;
        S->t_first = R.t_submit;
    }
    S->submitted++;
    S->pending.push_back(t);
    *ticket = t;
    S->cv_work.notify_one();
    return FZ_OK;
}

int fz_server_wait(fz_server* S, uint64_t ticket, int* status)
{
    if (!S) return FZ_ERR_ARG;
    std::unique_lock<std::mutex> lk(S->mu);
    auto it = S->reqs.find(ticket);
    if (it == S->reqs.end()) return FZ_ERR_ARG;
    S->cv_done.wait(lk, [&] { return it->second.done; });
    if (status) *status = it->second.status;
    S->reqs.erase(it);
    return FZ_OK;
}

int fz_server_poll(fz_server* S, uint64_t ticket, int* done)
{
    if (!S || !done) return FZ_ERR_ARG;
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->reqs.find(ticket);
    if (it == S->reqs.end()) return FZ_ERR_ARG;
    *done = it->second.done ? 1 : 0;
    return FZ_OK;
}

int fz_server_stats(fz_server* S, fz_server_report* out)
{
    if (!S || !out) return FZ_ERR_ARG;
    std::lock_guard<std::mutex> lk(S->mu);
    std::memset(out, 0, sizeof(*out));
    out->submitted = S->submitted;
    out->completed = S->completed;
    out->queued = S->pending.size() + S->ready.size();
    out->batches = S->batches;
    out->mean_batch = S->batches ? (double)S->batched / (double)S->batches : 0.0;
    out->admission_waits = S->admission_waits;
    out->inflight_max_bytes = S->inflight_max;
    out->input_bytes = S->input_bytes;
    if (!S->lat_ms.empty()) {
        std::vector<double> v = S->lat_ms;
        std::sort(v.begin(), v.end());
        auto pct = [&](double p) {
            const size_t i = (size_t)std::ceil(p * (double)v.size()) - 1;
            return v[std::min(i, v.size() - 1)];
        };
        out->p50_ms = pct(0.50);
        out->p99_ms = pct(0.99);
        out->max_ms = v.back();
        double s = 0.0;
        for (double x : v) s += x;
        out->mean_ms = s / (double)v.size();
        out->wall_s = std::chrono::duration<double>(S->t_last - S->t_first).count();
    }
    return FZ_OK;
}

int fz_server_reset_stats(fz_server* S)
{
    if (!S) return FZ_ERR_ARG;
    std::lock_guard<std::mutex> lk(S->mu);
    S->lat_ms.clear();
    S->submitted = S->completed = S->batches = S->batched = S->admission_waits = S->input_bytes = 0;
    S->inflight_max = S->inflight;
    S->any = false;
    return FZ_OK;
}

int fz_server_destroy(fz_server* S)
{
    if (!S) return FZ_ERR_ARG;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop = true;
    }
    S->cv_work.notify_all();
    if (S->worker.joinable()) S->worker.join();
    release(S);
    delete S;
    return FZ_OK;
}

}  // extern "C"

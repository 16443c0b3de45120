// libfgs multi-stream server: many camera streams served from one GPU with their
// models resident in device memory and continuous batching.
//
//  * Admission: a stream is opened only if its model, its device input slots and
//    the server's share fit the HBM budget (else FGS_ERR_BUSY); closing frees it.
//  * Submit copies a host frame into the stream's pinned ring (kQueue slots; a
//    full ring returns FGS_ERR_BUSY) and returns a ticket at once.
//  * A scheduler thread forms a batch from every stream whose previous frame has
//    finished and whose next frame is queued (at most one frame per stream in
//    flight, so every stream's frames run in order), copies the inputs to the
//    device on a copy stream, launches ONE serving kernel over all tiles of all
//    entries (mixed resolutions, GMM and PBAS), and queues the masks' copy back
//    on a second stream.  It does not wait for the batch: frames that arrive while
//    it runs form the next batch, whose input copies overlap the running kernel.
//  * A completion thread waits for each batch, stamps the per-frame latency
//    (completion minus arrival) and releases the streams for their next frame.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "fgs.h"
#include "fgs_internal.h"
#include "model.h"

using namespace fgs;

namespace {

constexpr int kQueue = 4;        // frames per stream ring
constexpr int kDescRing = 16;    // descriptor buffers for batches in flight

double now_s() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

size_t align256(size_t n) { return (n + 255) & ~size_t(255); }

enum SlotState { kFree, kFilling, kQueued, kInflight, kDone, kDropped };

struct Slot {
    uint8_t* h_in = nullptr;    // pinned: rgb (dense, 256-aligned size) then depth
    uint8_t* d_in = nullptr;    // device copy of h_in
    uint8_t* h_mask = nullptr;  // pinned mask of this frame
    SlotState state = kFree;
    uint64_t ticket = 0;
    double t_arrival = 0.0, latency = 0.0;
};

struct Stream {
    int id = 0;
    fgs_model* model = nullptr;
    int algo = 0, H = 0, W = 0, npix = 0;
    size_t rgb_bytes = 0, in_bytes = 0, dev_bytes = 0;
    Slot slots[kQueue];
    int next_submit = 0, next_run = 0;
    int copying = 0;  // submits copying into a slot with the lock released
    bool inflight = false, closed = false;
};

struct Batch {
    std::vector<std::pair<Stream*, int>> items;
    hipEvent_t in_done = nullptr, done = nullptr;
    int ring = 0;
    hipError_t err = hipSuccess;
};

template <typename... A>
fgs_status fail(fgs_status s, const char* fmt, A... args) {
    return fgs::set_error(s, fmt, args...);
}

}  // namespace

struct fgs_server {
    size_t budget = 0, used = 0;
    int max_streams = 0;
    int device = 0;
    hipStream_t compute = nullptr, h2d = nullptr, d2h = nullptr;
    std::mutex mu;
    std::condition_variable cv_sched, cv_done, cv_compl;
    std::map<int, Stream*> streams;
    std::vector<Stream*> closed;
    std::map<uint64_t, std::pair<Stream*, int>> tickets;
    int next_id = 1;
    int opening = 0;  // opens past the stream-count check, not yet admitted or refused
    uint64_t next_ticket = 1;
    std::deque<Batch*> completion;
    std::vector<hipEvent_t> event_pool;
    bool stop_sched = false, stop_compl = false;
    std::thread sched, compl_thread;
    ServeEntry* h_desc[kDescRing] = {};
    int32_t* h_prefix[kDescRing] = {};
    uint8_t* d_ring = nullptr;
    hipEvent_t ring_ev[kDescRing] = {};
    bool ring_used[kDescRing] = {};
    int ring_next = 0;
    size_t desc_cap = 0;  // entries per descriptor buffer
    // statistics since the last reset
    std::vector<double> latencies;
    int64_t frames_done = 0, batches = 0, batch_frames = 0, pixels_done = 0;
    double t_stats0 = 0.0;
    bool device_error = false;
};

namespace {

hipEvent_t take_event(fgs_server* s) {  // caller holds s->mu
    if (!s->event_pool.empty()) {
        hipEvent_t e = s->event_pool.back();
        s->event_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return nullptr;
    return e;
}

bool ready(const Stream* st) {
    return !st->closed && !st->inflight && st->slots[st->next_run].state == kQueued;
}

// Serving classes.  The fused serving kernel runs GMM streams with Kc = Kd = K, K one
// of {3, 5}, one variance per Gaussian (any rate or decision variant), and PBAS streams
// with N <= 40, mixed, in ONE launch; its instance is chosen per batch (K: whichever of
// 3 and 5 has more of the batch's pixels; PBAS register class 24 or 40: the largest N
// among its PBAS streams).  Every other stream (the other K, any other (Kc, Kd),
// per-channel variances, N > 40) runs through the per-frame step kernels, grouped by
// kernel class, up to kBatchMax models per launch, after the fused launch on the same
// stream.  A stream's results are those of its model pushed alone either way.
bool fused_gmm(const fgs_model* m) {
    return m->gp.Kc == m->gp.Kd && (m->gp.Kc == 3 || m->gp.Kc == 5) && m->gp.var_mode == 0;
}
bool fused_pbas(const fgs_model* m) { return m->pp.N <= 40 && !m->pp.gradient; }

// Launches of the streams outside the fused kernel's class: models of one kind and
// batch key share a launch of up to kBatchMax; PBAS fill frames go alone.
hipError_t launch_other(const std::vector<std::pair<GmmStepArgs, const fgs_model*>>& og,
                        const std::vector<PbasStepArgs>& op, const std::vector<PbasGradArgs>& opg,
                        hipStream_t s) {
    for (const PbasGradArgs& a : opg) {  // the gradient-magnitude variant: one launch each
        const hipError_t e = pbas_grad_launch_step(a, s);
        if (e != hipSuccess) return e;
    }
    std::vector<char> used(og.size(), 0);
    for (size_t i = 0; i < og.size(); ++i) {
        if (used[i]) continue;
        const fgs_model* mi = og[i].second;
        const int key = gmm_batch_key(og[i].first, mi->gp.Kc, mi->gp.Kd);
        GmmStepArgs b[kBatchMax];
        int n = 0;
        for (size_t j = i; j < og.size() && n < kBatchMax; ++j) {
            if (used[j] || gmm_batch_key(og[j].first, og[j].second->gp.Kc, og[j].second->gp.Kd) != key) continue;
            used[j] = 1;
            b[n++] = og[j].first;
        }
        const hipError_t e = gmm_launch_step_batch(b, n, mi->gp.Kc, mi->gp.Kd, s);
        if (e != hipSuccess) return e;
    }
    std::vector<char> pused(op.size(), 0);
    for (size_t i = 0; i < op.size(); ++i) {
        if (pused[i]) continue;
        const int key = pbas_batch_key(op[i]);
        if (key < 0) {  // a fill frame
            pused[i] = 1;
            const hipError_t e = pbas_launch_step(op[i], s);
            if (e != hipSuccess) return e;
            continue;
        }
        PbasStepArgs b[kBatchMax];
        int n = 0;
        for (size_t j = i; j < op.size() && n < kBatchMax; ++j) {
            if (pused[j] || pbas_batch_key(op[j]) != key) continue;
            pused[j] = 1;
            b[n++] = op[j];
        }
        const hipError_t e = pbas_launch_step_batch(b, n, s);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// Enqueue one batch on the device (scheduler thread, lock not held).  Only the
// scheduler touches the models' frame bookkeeping.
hipError_t issue(fgs_server* s, Batch* b) {
    const int r = b->ring;
    if (s->ring_used[r]) {
        hipError_t e = hipEventSynchronize(s->ring_ev[r]);
        if (e != hipSuccess) return e;
    }
    for (auto& it : b->items) {
        Slot& sl = it.first->slots[it.second];
        hipError_t e = hipMemcpyAsync(sl.d_in, sl.h_in, it.first->in_bytes, hipMemcpyHostToDevice, s->h2d);
        if (e != hipSuccess) return e;
    }
    hipError_t e = hipEventRecord(b->in_done, s->h2d);
    if (e == hipSuccess) e = hipStreamWaitEvent(s->compute, b->in_done, 0);
    if (e != hipSuccess) return e;

    // the fused kernel's instance for this batch
    int64_t px3 = 0, px5 = 0;
    int pbas_n = 0;
    for (auto& it : b->items) {
        const fgs_model* m = it.first->model;
        if (it.first->algo == FGS_GMM && fused_gmm(m)) (m->gp.Kc == 3 ? px3 : px5) += it.first->npix;
        if (it.first->algo == FGS_PBAS && fused_pbas(m)) pbas_n = std::max(pbas_n, (int)m->pp.N);
    }
    const int kg = px5 >= px3 ? 5 : 3;
    const int np = serve_pbas_nmax(std::max(pbas_n, 2));

    ServeEntry* d = s->h_desc[r];
    int32_t* pre = s->h_prefix[r];
    int n = 0, total = 0;
    bool streaming = false;
    std::vector<std::pair<GmmStepArgs, const fgs_model*>> og;
    std::vector<PbasStepArgs> op;
    std::vector<PbasGradArgs> opg;
    for (auto& it : b->items) {
        Stream* st = it.first;
        Slot& sl = st->slots[it.second];
        const uint8_t* drgb = sl.d_in;
        const uint8_t* ddep = sl.d_in + st->rgb_bytes;
        fgs_model* m = st->model;
        if (st->algo == FGS_GMM) {
            GmmStepArgs ga;
            model_next_gmm(m, drgb, 3 * (int64_t)st->W, ddep, 2 * (int64_t)st->W, 0, 0, &ga);
            if (!(fused_gmm(m) && m->gp.Kc == kg)) {
                og.emplace_back(ga, m);
                continue;
            }
            ServeEntry& en = d[n];
            std::memset(&en, 0, sizeof en);
            en.algo = FGS_GMM;
            en.g = ga;
            en.ntiles = (st->npix + 255) / 256;
            streaming = streaming || ga.streaming;
        } else if (m->pp.gradient) {
            PbasGradArgs pa;
            model_next_pbas_grad(m, drgb, 3 * (int64_t)st->W, ddep, 2 * (int64_t)st->W, 0, 0, &pa);
            opg.push_back(pa);
            continue;
        } else {
            const int fill = m->t < m->pp.N ? 1 : 0;
            PbasStepArgs pa;
            model_next_pbas(m, drgb, 3 * (int64_t)st->W, ddep, 2 * (int64_t)st->W, 0, 0, &pa);
            if (!fused_pbas(m)) {
                op.push_back(pa);
                continue;
            }
            ServeEntry& en = d[n];
            std::memset(&en, 0, sizeof en);
            en.algo = FGS_PBAS;
            en.fill = fill;
            en.p = pa;
            en.tiles_x = (st->W + kPbasTileW - 1) / kPbasTileW;
            en.ntiles = fill ? (st->npix + 255) / 256 : en.tiles_x * ((st->H + kPbasTileH - 1) / kPbasTileH);
            streaming = streaming || pa.streaming;
        }
        pre[n] = total;
        total += d[n].ntiles;
        n += 1;
    }
    pre[n] = total;
    if (n > 0) {
        ServeEntry* dd = reinterpret_cast<ServeEntry*>(s->d_ring + r * (s->desc_cap * sizeof(ServeEntry) +
                                                                       align256((s->desc_cap + 1) * 4)));
        int32_t* dp = reinterpret_cast<int32_t*>(reinterpret_cast<uint8_t*>(dd) + s->desc_cap * sizeof(ServeEntry));
        e = hipMemcpyAsync(dd, d, n * sizeof(ServeEntry), hipMemcpyHostToDevice, s->compute);
        if (e == hipSuccess) e = hipMemcpyAsync(dp, pre, (n + 1) * sizeof(int32_t), hipMemcpyHostToDevice, s->compute);
        if (e == hipSuccess) e = serve_launch(dd, dp, n, total, kg, np, streaming, s->compute);
        if (e != hipSuccess) return e;
    }
    e = launch_other(og, op, opg, s->compute);
    if (e == hipSuccess) e = hipEventRecord(s->ring_ev[r], s->compute);
    if (e != hipSuccess) return e;
    s->ring_used[r] = true;
    e = hipStreamWaitEvent(s->d2h, s->ring_ev[r], 0);
    if (e != hipSuccess) return e;
    for (auto& it : b->items) {
        Slot& sl = it.first->slots[it.second];
        e = hipMemcpyAsync(sl.h_mask, it.first->model->mask, it.first->npix, hipMemcpyDeviceToHost, s->d2h);
        if (e != hipSuccess) return e;
    }
    return hipEventRecord(b->done, s->d2h);
}

void scheduler_loop(fgs_server* s) {
    (void)hipSetDevice(s->device);
    std::unique_lock<std::mutex> lk(s->mu);
    for (;;) {
        s->cv_sched.wait(lk, [&] {
            if (s->stop_sched) return true;
            for (auto& kv : s->streams)
                if (ready(kv.second)) return true;
            return false;
        });
        if (s->stop_sched) break;
        Batch* b = new Batch();
        for (auto& kv : s->streams) {
            Stream* st = kv.second;
            if (!ready(st)) continue;
            st->slots[st->next_run].state = kInflight;
            st->inflight = true;
            b->items.emplace_back(st, st->next_run);
            st->next_run = (st->next_run + 1) % kQueue;
        }
        b->ring = s->ring_next;
        s->ring_next = (s->ring_next + 1) % kDescRing;
        b->in_done = take_event(s);
        b->done = take_event(s);
        lk.unlock();
        b->err = (b->in_done && b->done) ? issue(s, b) : hipErrorOutOfMemory;
        lk.lock();
        s->completion.push_back(b);
        s->cv_compl.notify_one();
    }
}

void completion_loop(fgs_server* s) {
    (void)hipSetDevice(s->device);
    std::unique_lock<std::mutex> lk(s->mu);
    for (;;) {
        s->cv_compl.wait(lk, [&] { return !s->completion.empty() || s->stop_compl; });
        if (s->completion.empty()) break;
        Batch* b = s->completion.front();
        s->completion.pop_front();
        lk.unlock();
        hipError_t e = b->err;
        if (e == hipSuccess) e = hipEventSynchronize(b->done);
        const double t = now_s();
        lk.lock();
        if (e != hipSuccess) s->device_error = true;
        for (auto& it : b->items) {
            Stream* st = it.first;
            Slot& sl = st->slots[it.second];
            st->inflight = false;
            if (e == hipSuccess) {
                sl.state = kDone;
                sl.latency = t - sl.t_arrival;
                s->latencies.push_back(sl.latency);
                s->frames_done += 1;
                s->pixels_done += st->npix;
            } else {
                sl.state = kDropped;
            }
        }
        s->batches += 1;
        s->batch_frames += (int64_t)b->items.size();
        if (b->in_done) s->event_pool.push_back(b->in_done);
        if (b->done) s->event_pool.push_back(b->done);
        delete b;
        s->cv_done.notify_all();
        s->cv_sched.notify_one();
    }
}

void free_stream_device(Stream* st) {
    if (st->model) fgs_destroy(st->model);
    st->model = nullptr;
    for (Slot& sl : st->slots) {
        if (sl.d_in) (void)hipFree(sl.d_in);
        sl.d_in = nullptr;
    }
}

void free_stream_host(Stream* st) {
    for (Slot& sl : st->slots) {
        if (sl.h_in) (void)hipHostFree(sl.h_in);
        if (sl.h_mask) (void)hipHostFree(sl.h_mask);
        sl.h_in = sl.h_mask = nullptr;
    }
}

// A closed stream's host buffers are freed once nothing refers to them: no ticket
// (every slot collected) and no submit still copying into a slot (caller holds s->mu).
void reclaim_if_idle(fgs_server* s, Stream* st) {
    if (!st->closed || st->copying != 0) return;
    for (const Slot& sl : st->slots)
        if (sl.state != kFree) return;
    auto it = std::find(s->closed.begin(), s->closed.end(), st);
    if (it == s->closed.end()) return;
    s->closed.erase(it);
    free_stream_host(st);
    delete st;
}

// Holds one of the server's max_streams places from the count check until the stream
// is admitted (release_locked) or the open fails (destructor).
struct OpenReservation {
    fgs_server* s;
    bool held = true;
    void release_locked() {
        if (held) s->opening -= 1;
        held = false;
    }
    ~OpenReservation() {
        if (!held) return;
        std::lock_guard<std::mutex> lk(s->mu);
        s->opening -= 1;
    }
};

}  // namespace

extern "C" {

double fgs_server_now(void) { return now_s(); }

fgs_status fgs_server_create(size_t hbm_budget_bytes, int32_t max_streams, fgs_server** out) {
    if (!out) return fail(FGS_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (max_streams < 1 || max_streams > 1024)
        return fail(FGS_ERR_INVALID_ARG, "server needs 1 <= max_streams <= 1024 (got %d)", max_streams);
    fgs_server* s = new (std::nothrow) fgs_server();
    if (!s) return fail(FGS_ERR_OUT_OF_MEMORY, "host allocation");
    s->budget = hbm_budget_bytes;
    s->max_streams = max_streams;
    s->desc_cap = (size_t)max_streams;
    hipError_t e = hipGetDevice(&s->device);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&s->compute, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&s->h2d, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&s->d2h, hipStreamNonBlocking);
    const size_t per = s->desc_cap * sizeof(ServeEntry) + align256((s->desc_cap + 1) * 4);
    if (e == hipSuccess) e = hipMalloc((void**)&s->d_ring, per * kDescRing);
    for (int r = 0; r < kDescRing && e == hipSuccess; ++r) {
        e = hipHostMalloc((void**)&s->h_desc[r], s->desc_cap * sizeof(ServeEntry), hipHostMallocDefault);
        if (e == hipSuccess) e = hipHostMalloc((void**)&s->h_prefix[r], (s->desc_cap + 1) * 4, hipHostMallocDefault);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&s->ring_ev[r], hipEventDisableTiming);
    }
    if (e != hipSuccess) {
        fgs_status st = fail(FGS_ERR_DEVICE, "server set-up: %s", hipGetErrorString(e));
        fgs_server_destroy(s);
        return st;
    }
    s->used = per * kDescRing;
    s->t_stats0 = now_s();
    s->sched = std::thread(scheduler_loop, s);
    s->compl_thread = std::thread(completion_loop, s);
    *out = s;
    return FGS_OK;
}

fgs_status fgs_server_open(fgs_server* s, fgs_algo algo, int32_t H, int32_t W, const void* params,
                           int32_t* stream_id) {
    if (!s || !stream_id) return fail(FGS_ERR_INVALID_ARG, "NULL argument");
    if (algo != FGS_GMM && algo != FGS_PBAS) return fail(FGS_ERR_INVALID_ARG, "unknown algo %d", (int)algo);
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if ((int)s->streams.size() + s->opening >= s->max_streams)
            return fail(FGS_ERR_BUSY, "all %d stream slots in use", s->max_streams);
        s->opening += 1;
    }
    OpenReservation place{s};
    fgs_model* m = nullptr;
    fgs_status st = fgs_create(algo, H, W, params, s->compute, &m);
    if (st != FGS_OK) return st;
    Stream* sr = new (std::nothrow) Stream();
    if (!sr) {
        fgs_destroy(m);
        return fail(FGS_ERR_OUT_OF_MEMORY, "host allocation");
    }
    // The serving kernel keeps a PBAS pixel's previous value in its own plane (its one
    // instance serves every N up to the class bound): set before the first frame.
    if (algo == FGS_PBAS && !m->pp.gradient) m->pb.last_in_pad = 0;
    sr->model = m;
    sr->algo = algo;
    sr->H = H;
    sr->W = W;
    sr->npix = H * W;
    sr->rgb_bytes = align256((size_t)sr->npix * 3);
    sr->in_bytes = sr->rgb_bytes + (size_t)sr->npix * 2;
    size_t mb = 0;
    fgs_device_bytes(m, &mb);
    sr->dev_bytes = mb + kQueue * align256(sr->in_bytes);
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->used + sr->dev_bytes > s->budget) {
            const size_t need = sr->dev_bytes, have = s->budget - std::min(s->budget, s->used);
            fgs_destroy(m);
            delete sr;
            return fail(FGS_ERR_BUSY, "stream needs %zu device bytes, %zu left in the budget", need, have);
        }
        s->used += sr->dev_bytes;
    }
    hipError_t e = hipSuccess;
    for (Slot& sl : sr->slots) {
        if (e == hipSuccess) e = hipHostMalloc((void**)&sl.h_in, sr->in_bytes, hipHostMallocDefault);
        if (e == hipSuccess) e = hipHostMalloc((void**)&sl.h_mask, sr->npix, hipHostMallocDefault);
        if (e == hipSuccess) e = hipMalloc((void**)&sl.d_in, sr->in_bytes);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(s->compute);  // model initialised
    std::lock_guard<std::mutex> lk(s->mu);
    if (e != hipSuccess) {
        s->used -= sr->dev_bytes;
        free_stream_device(sr);
        free_stream_host(sr);
        delete sr;
        return fail(FGS_ERR_OUT_OF_MEMORY, "stream buffers: %s", hipGetErrorString(e));
    }
    place.release_locked();
    sr->id = s->next_id++;
    s->streams[sr->id] = sr;
    *stream_id = sr->id;
    return FGS_OK;
}

fgs_status fgs_server_submit(fgs_server* s, int32_t id, const uint8_t* rgb, const uint16_t* depth,
                             double t_arrival_s, uint64_t* ticket) {
    if (!s || !rgb || !depth || !ticket) return fail(FGS_ERR_INVALID_ARG, "NULL argument");
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->streams.find(id);
    if (it == s->streams.end()) return fail(FGS_ERR_INVALID_ARG, "no open stream %d", id);
    if (s->device_error) return fail(FGS_ERR_DEVICE, "the server hit a device error");
    Stream* st = it->second;
    const int k = st->next_submit;
    Slot& sl = st->slots[k];
    if (sl.state != kFree) return fail(FGS_ERR_BUSY, "stream %d has %d frames pending", id, kQueue);
    sl.state = kFilling;
    sl.ticket = s->next_ticket++;
    sl.t_arrival = t_arrival_s > 0.0 ? t_arrival_s : now_s();
    st->next_submit = (k + 1) % kQueue;
    s->tickets[sl.ticket] = {st, k};
    *ticket = sl.ticket;
    st->copying += 1;
    lk.unlock();
    std::memcpy(sl.h_in, rgb, (size_t)st->npix * 3);
    std::memcpy(sl.h_in + st->rgb_bytes, depth, (size_t)st->npix * 2);
    lk.lock();
    st->copying -= 1;
    // A close that ran during the copy marked the slot dropped (the copy counter kept its
    // host buffers): the ticket stays valid and its wait reports the drop.
    if (sl.state != kFilling) {
        reclaim_if_idle(s, st);
        return FGS_OK;
    }
    sl.state = kQueued;
    s->cv_sched.notify_one();
    return FGS_OK;
}

fgs_status fgs_server_wait(fgs_server* s, uint64_t ticket, uint8_t* mask, double* latency_s,
                           int32_t timeout_ms) {
    if (!s) return fail(FGS_ERR_INVALID_ARG, "server is NULL");
    std::unique_lock<std::mutex> lk(s->mu);
    if (s->tickets.find(ticket) == s->tickets.end())
        return fail(FGS_ERR_INVALID_ARG, "unknown ticket %llu", (unsigned long long)ticket);
    // Look the ticket up again on every wake-up: another wait may have collected it, and
    // its stream may then be gone.
    auto done = [&] {
        auto f = s->tickets.find(ticket);
        if (f == s->tickets.end()) return true;
        const SlotState q = f->second.first->slots[f->second.second].state;
        return q == kDone || q == kDropped;
    };
    if (timeout_ms < 0) {
        s->cv_done.wait(lk, done);
    } else if (!s->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), done)) {
        return fail(FGS_ERR_BUSY, "ticket %llu not finished", (unsigned long long)ticket);
    }
    auto it = s->tickets.find(ticket);
    if (it == s->tickets.end())
        return fail(FGS_ERR_INVALID_ARG, "ticket %llu was collected by another wait", (unsigned long long)ticket);
    Stream* st = it->second.first;
    Slot& sl = st->slots[it->second.second];
    const bool ok = sl.state == kDone;
    if (ok && mask) std::memcpy(mask, sl.h_mask, (size_t)st->npix);
    if (latency_s) *latency_s = ok ? sl.latency : -1.0;
    sl.state = kFree;
    s->tickets.erase(it);
    reclaim_if_idle(s, st);
    if (ok) return FGS_OK;
    return s->device_error ? fail(FGS_ERR_DEVICE, "frame lost to a device error")
                           : fail(FGS_ERR_BAD_STATE, "frame dropped: its stream was closed");
}

fgs_status fgs_server_close(fgs_server* s, int32_t id) {
    if (!s) return fail(FGS_ERR_INVALID_ARG, "server is NULL");
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->streams.find(id);
    if (it == s->streams.end()) return fail(FGS_ERR_INVALID_ARG, "no open stream %d", id);
    Stream* st = it->second;
    st->closed = true;  // no new batches; the running frame (if any) finishes
    s->cv_done.wait(lk, [&] { return !st->inflight; });
    s->streams.erase(it);
    for (Slot& sl : st->slots)
        if (sl.state == kQueued || sl.state == kFilling) sl.state = kDropped;
    s->used -= st->dev_bytes;
    free_stream_device(st);
    s->closed.push_back(st);  // host buffers stay until every ticket is collected
    reclaim_if_idle(s, st);
    s->cv_done.notify_all();
    return FGS_OK;
}

fgs_status fgs_server_get_stats(fgs_server* s, fgs_server_stats* out) {
    if (!s || !out) return fail(FGS_ERR_INVALID_ARG, "NULL argument");
    if (out->struct_size != sizeof(fgs_server_stats))
        return fail(FGS_ERR_INVALID_ARG, "fgs_server_stats.struct_size %u != %zu", out->struct_size,
                    sizeof(fgs_server_stats));
    std::lock_guard<std::mutex> lk(s->mu);
    std::vector<double> v = s->latencies;
    auto q = [&](double f) {
        if (v.empty()) return 0.0;
        const size_t i = std::min(v.size() - 1, (size_t)(f * (double)(v.size() - 1) + 0.5));
        std::nth_element(v.begin(), v.begin() + i, v.end());
        return v[i];
    };
    out->streams_open = (int32_t)s->streams.size();
    out->frames_done = s->frames_done;
    out->batches = s->batches;
    out->mean_batch_frames = s->batches ? (double)s->batch_frames / (double)s->batches : 0.0;
    out->p50_latency_s = q(0.50);
    out->p99_latency_s = q(0.99);
    out->max_latency_s = v.empty() ? 0.0 : *std::max_element(v.begin(), v.end());
    const double dt = now_s() - s->t_stats0;
    out->mpix_frames_per_s = dt > 0 ? (double)s->pixels_done / dt / 1e6 : 0.0;
    out->device_bytes_used = s->used;
    out->device_budget = s->budget;
    return FGS_OK;
}

fgs_status fgs_server_reset_stats(fgs_server* s) {
    if (!s) return fail(FGS_ERR_INVALID_ARG, "server is NULL");
    std::lock_guard<std::mutex> lk(s->mu);
    s->latencies.clear();
    s->frames_done = s->batches = s->batch_frames = s->pixels_done = 0;
    s->t_stats0 = now_s();
    return FGS_OK;
}

fgs_status fgs_server_destroy(fgs_server* s) {
    if (!s) return FGS_OK;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop_sched = true;
    }
    s->cv_sched.notify_all();
    if (s->sched.joinable()) s->sched.join();
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop_compl = true;
    }
    s->cv_compl.notify_all();
    if (s->compl_thread.joinable()) s->compl_thread.join();  // drains the batches in flight
    if (s->compute) (void)hipStreamSynchronize(s->compute);
    for (auto& kv : s->streams) {
        free_stream_device(kv.second);
        free_stream_host(kv.second);
        delete kv.second;
    }
    for (Stream* st : s->closed) {
        free_stream_host(st);
        delete st;
    }
    for (hipEvent_t e : s->event_pool) (void)hipEventDestroy(e);
    for (int r = 0; r < kDescRing; ++r) {
        if (s->h_desc[r]) (void)hipHostFree(s->h_desc[r]);
        if (s->h_prefix[r]) (void)hipHostFree(s->h_prefix[r]);
        if (s->ring_ev[r]) (void)hipEventDestroy(s->ring_ev[r]);
    }
    if (s->d_ring) (void)hipFree(s->d_ring);
    if (s->compute) (void)hipStreamDestroy(s->compute);
    if (s->h2d) (void)hipStreamDestroy(s->h2d);
    if (s->d2h) (void)hipStreamDestroy(s->d2h);
    delete s;
    return FGS_OK;
}

}  // extern "C"

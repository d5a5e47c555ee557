// Request API of the C ABI (solve_create / submit / poll / wait / destroy):
// HBM-budget admission, continuous batching over in-flight slots, and the
// plain one-request-per-synchronous-launch mode.
//
// Life of a request (batched mode):
//   submit   inputs copied to host memory owned by the request, validated
//            (n, order, sizes), footprint priced, queued (FIFO);
//   admit    the scheduler thread takes queued requests while the resident
//            footprint stays within the budget and the slot count (a bounded
//            look-ahead lets smaller requests pass a large head request,
//            until the head has been passed over too often);
//   launch   the admitted requests form one batch on a free in-flight slot:
//            inputs staged in pinned memory, copied to HBM, one persistent
//            fused launch builds and evaluates all of them (plus an explicit-
//            query kernel per request that brings its own points), results
//            copied back, an event recorded -- optionally as one hipGraph;
//   done     when the event completes, results reach the caller's buffers,
//            the footprint is released and the ticket turns DONE.
// New requests are admitted while earlier batches are still on the device
// (up to max_inflight batches overlap), which is continuous batching.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "batch.hpp"
#include "internal.hpp"
#include "spline_solve.h"

namespace {

using spl::Batch;

double now_s() {
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

// Device bytes held by a context's buffers, and their peak.
struct Held {
    std::atomic<uint64_t> now{0}, peak{0};
    void add(uint64_t b) {
        const uint64_t h = now.fetch_add(b) + b;
        uint64_t pk = peak.load();
        while (h > pk && !peak.compare_exchange_weak(pk, h)) {
        }
    }
    void sub(uint64_t b) { now.fetch_sub(b); }
};

// A device buffer whose allocation and release are ordered on its owner's
// stream (hipMallocAsync / hipFreeAsync): resizing one slot's buffers does
// not wait for the batches running on the other slots.
struct DevBuf {
    void* p = nullptr;
    size_t cap = 0;
    // Reallocate to exactly `want` bytes (the old contents are dropped).
    int resize(size_t want, hipStream_t s, Held& held) {
        drop(s, held);
        if (hipMallocAsync(&p, want, s) != hipSuccess) {
            p = nullptr;
            return SOLVE_E_DEVICE;
        }
        cap = want;
        held.add(cap);
        return SOLVE_OK;
    }
    void drop(hipStream_t s, Held& held) {
        if (p) {
            (void)hipFreeAsync(p, s);
            held.sub(cap);
        }
        p = nullptr;
        cap = 0;
    }
    template <typename T>
    T* as() const { return (T*)p; }
};

// Capacity for a buffer that must hold `bytes`: half again as much (fewer
// reallocations as batches grow) when `room` allows it, else exactly `bytes`.
size_t with_slack(size_t bytes, uint64_t room) {
    const size_t want = bytes + bytes / 2 + 256;
    return want <= room ? want : bytes;
}

struct HostBuf {  // pinned host staging
    void* p = nullptr;
    size_t cap = 0;
    int ensure(size_t bytes) {
        if (bytes <= cap && p) return SOLVE_OK;
        const size_t want = std::max(bytes, cap + cap / 2) + 256;
        if (p) (void)hipHostFree(p);
        p = nullptr;
        cap = 0;
        if (hipHostMalloc(&p, want, hipHostMallocDefault) != hipSuccess) {
            p = nullptr;
            return SOLVE_E_DEVICE;
        }
        cap = want;
        return SOLVE_OK;
    }
    void release() {
        if (p) (void)hipHostFree(p);
        p = nullptr;
        cap = 0;
    }
    template <typename T>
    T* as() const { return (T*)p; }
};

// With SOLVE_DEBUG set in the environment, failing HIP calls of the request
// path are reported on stderr (the C ABI itself only returns SOLVE_* codes).
int hip_fail(const char* what, hipError_t e) {
    static const bool debug = std::getenv("SOLVE_DEBUG") != nullptr;
    if (debug) std::fprintf(stderr, "solve: %s failed: %s (%d)\n", what, hipGetErrorString(e), (int)e);
    return SOLVE_E_DEVICE;
}

// Where a caller's pointer lives: device memory (or managed), pinned host
// memory (the device copies to and from it directly), or pageable host memory.
enum class Mem { kDevice, kPinned, kPageable };

Mem mem_kind(const void* p) {
    if (!p) return Mem::kPageable;
    hipPointerAttribute_t a;
    if (hipPointerGetAttributes(&a, p) != hipSuccess) {
        (void)hipGetLastError();  // clear the sticky error of an unknown host pointer
        return Mem::kPageable;
    }
    if (a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeManaged) return Mem::kDevice;
    if (a.type == hipMemoryTypeHost) return Mem::kPinned;
    return Mem::kPageable;
}

bool is_device_ptr(const void* p) { return mem_kind(p) == Mem::kDevice; }

struct Req {
    solve_ticket id = 0;
    int64_t n = 0, m = 0;
    double sd = 0, ed = 0;
    std::vector<double> x, y, xq;  // owned copies of the inputs
    double* yq_out = nullptr;
    double* ypp_out = nullptr;
    bool yq_dev = false, ypp_dev = false;
    bool yq_pinned = false, ypp_pinned = false;  // the device writes these directly
    int status = SOLVE_PENDING;
    int code = SOLVE_OK;
    double t[4] = {0, 0, 0, 0};
    uint64_t bytes = 0;
    int passed_over = 0;
    // recorded on the caller's stream at submit: the request's device outputs
    // are written only after it (null when no output is device memory)
    hipEvent_t ev = nullptr;
    bool explicit_q() const { return !xq.empty(); }
    // too long for the batched kernels: solved by the single-curve kernels
    bool solo() const { return n > SOLVE_MAX_N_BATCH; }
};
using ReqP = std::shared_ptr<Req>;

// Device bytes one request adds to a batch's buffers: knots, values and
// second derivatives (24 per knot), results (8 per query) and explicit query
// points (8 per query); its offsets, end derivatives, status and flag (40);
// and its work items, 48 bytes each: at most two per knot block of 255
// intervals and one per share of queries_per_tile queries.
uint64_t footprint(int64_t n, int64_t m, bool explicit_q, int64_t qpt) {
    const uint64_t blocks = (uint64_t)(n - 2) / 255 + 1;
    const uint64_t items = 2 * blocks + (uint64_t)m / (uint64_t)std::max<int64_t>(qpt, 1) + 1;
    return 8ull * (uint64_t)(3 * n + m + (explicit_q ? m : 0)) + 40ull + 48ull * items;
}

// A batch's buffers beyond its requests' footprints: the 256-byte alignment
// of its twelve regions.
constexpr uint64_t kBatchBytes = 4096;

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    std::unique_ptr<Batch> batch;
    bool busy = false;
    bool failed = false;
    std::vector<ReqP> reqs;
    uint64_t bytes = 0;
    // One packed input region and one packed output region per batch, each
    // with a pinned host mirror, so that a batch costs one copy each way.
    DevBuf din, dout;
    HostBuf hin, hout;
    std::vector<int64_t> koff, qoff;
    std::vector<uint8_t> uniform;
    size_t o_koff = 0, o_qoff = 0, o_sd = 0, o_ed = 0, o_x = 0, o_y = 0, o_xq = 0, o_tab = 0, in_bytes = 0;
    size_t o_status = 0, o_bad = 0, o_yq = 0, o_ypp = 0, out_bytes = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    void drop_graph() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        exec = nullptr;
        graph = nullptr;
    }
    template <typename T>
    T* din_at(size_t o) const { return (T*)((char*)din.p + o); }
    template <typename T>
    T* hin_at(size_t o) const { return (T*)((char*)hin.p + o); }
    template <typename T>
    T* dout_at(size_t o) const { return (T*)((char*)dout.p + o); }
    template <typename T>
    T* hout_at(size_t o) const { return (T*)((char*)hout.p + o); }
};

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

constexpr uint64_t kSpinPolls = 20000;  // about a few ms of yields before the scheduler sleeps between polls

constexpr int32_t kStatusUnset = 0x7fffffff;

}  // namespace

struct solve_ctx {
    solve_config cfg{};
    std::mutex mu;
    std::condition_variable cv_sched;
    std::condition_variable cv_done;
    std::deque<ReqP> queue;
    std::unordered_map<solve_ticket, ReqP> tickets;
    std::vector<std::unique_ptr<Slot>> slots;
    std::thread sched;
    bool stop = false;
    bool inject = false;
    bool failed_state = false;
    uint64_t spins = 0;  // scheduler polls since a batch last completed
    uint64_t next_ticket = 1;
    uint64_t resident = 0, peak_resident = 0, resident_reqs = 0;
    uint64_t n_submitted = 0, n_completed = 0, n_failed = 0, n_batches = 0, peak_batch = 0;
    spline_tuning tuning = spl::default_tuning();
    // copies of device-resident inputs (a stream of their own: a synchronous
    // copy on the legacy stream would collide with a batch being captured)
    std::mutex in_mu;
    hipStream_t in_stream = nullptr;
    // events recorded on the caller's stream (cfg.stream), reused
    std::mutex ev_mu;
    std::vector<hipEvent_t> ev_free;
    // plain mode
    std::mutex plain_mu;
    hipStream_t plain_stream = nullptr;
    DevBuf px, py, pypp, pyq, pxq, pstatus;
    // device bytes held by the slots' and the plain path's buffers
    Held held;
};

namespace {

struct DevCtx {
    int prev = -1;
    explicit DevCtx(int dev) {
        (void)hipGetDevice(&prev);
        if (prev != dev) (void)hipSetDevice(dev);
    }
    ~DevCtx() {
        int cur = -1;
        (void)hipGetDevice(&cur);
        if (prev >= 0 && cur != prev) (void)hipSetDevice(prev);
    }
};

void finish_locked(solve_ctx* c, const ReqP& r, int status, int code) {
    r->status = status;
    r->code = code;
    r->t[3] = now_s();
    if (status == SOLVE_DONE) ++c->n_completed; else ++c->n_failed;
}

hipEvent_t event_get(solve_ctx* c) {
    {
        std::lock_guard<std::mutex> g(c->ev_mu);
        if (!c->ev_free.empty()) {
            hipEvent_t e = c->ev_free.back();
            c->ev_free.pop_back();
            return e;
        }
    }
    hipEvent_t e = nullptr;
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return nullptr;
    return e;
}

void event_put(solve_ctx* c, hipEvent_t& e) {
    if (!e) return;
    std::lock_guard<std::mutex> g(c->ev_mu);
    c->ev_free.push_back(e);
    e = nullptr;
}

// Size slot s's device buffers for its batch (in_bytes, out_bytes) within
// the budget: the room is the budget less what the other slots hold; idle
// slots give up their buffers when the batch would not fit beside them.
// Admission keeps the running batches' footprints within the budget, so the
// bytes held exceed it only by spare capacity a running slot took earlier
// (at most half its batch).  Scheduler thread only.
int size_slot(solve_ctx* c, Slot& s) {
    const uint64_t budget = c->cfg.hbm_budget_bytes;
    const uint64_t need = s.in_bytes + s.out_bytes;
    auto others = [&]() { return c->held.now.load() - s.din.cap - s.dout.cap; };
    if (others() + need > budget)
        for (auto& t : c->slots)
            if (t.get() != &s && !t->busy) {
                t->din.drop(t->stream, c->held);
                t->dout.drop(t->stream, c->held);
            }
    const uint64_t room = budget > others() ? budget - others() : 0;
    // spare capacity (half again) only when both buffers can have it
    const size_t in_spare = s.in_bytes + s.in_bytes / 2 + 256, out_spare = s.out_bytes + s.out_bytes / 2 + 256;
    const bool slack = in_spare + out_spare <= room;
    const size_t in_want = slack ? in_spare : s.in_bytes;
    const size_t out_want = slack ? out_spare : s.out_bytes;
    // reallocate a buffer that is too small, or larger than it may be when
    // the slot holds more than its room
    const bool over = s.din.cap + s.dout.cap > room;
    int rc = SOLVE_OK;
    if (!s.din.p || s.din.cap < s.in_bytes || (over && s.din.cap > in_want)) rc = s.din.resize(in_want, s.stream, c->held);
    if (!rc && (!s.dout.p || s.dout.cap < s.out_bytes || (over && s.dout.cap > out_want)))
        rc = s.dout.resize(out_want, s.stream, c->held);
    return rc;
}

// Stage, copy and launch one batch on slot s (called without the lock; the
// slot is owned by the scheduler thread until its event completes).
int launch_batch(solve_ctx* c, Slot& s) {
    // requests with explicit points last, so that their points and results
    // are contiguous and one launch evaluates them all
    std::stable_partition(s.reqs.begin(), s.reqs.end(), [](const ReqP& r) { return !r->explicit_q(); });
    const int64_t count = (int64_t)s.reqs.size();
    int64_t nt = 0, mt = 0, xt = 0;
    bool host_yq = false, host_ypp = false;
    s.koff.assign(count + 1, 0);
    s.qoff.assign(count + 1, 0);
    s.uniform.assign(count, 1);
    for (int64_t i = 0; i < count; ++i) {
        const Req& r = *s.reqs[i];
        s.koff[i + 1] = s.koff[i] + r.n;
        s.qoff[i + 1] = s.qoff[i] + r.m;
        if (r.explicit_q()) {
            xt += r.m;
            s.uniform[i] = 0;
        }
        if (r.solo()) s.uniform[i] = spl::kCurveSkip;
        host_yq |= !r.yq_dev && !r.yq_pinned;
        host_ypp |= r.ypp_out && !r.ypp_dev && !r.ypp_pinned;
    }
    nt = s.koff[count];
    mt = s.qoff[count];
    if (!s.batch) s.batch.reset(new Batch(c->cfg.device));
    // (host tables only: they travel in the batch's input region)
    int rc = s.batch->plan(count, s.koff.data(), s.qoff.data(), c->tuning, c->cfg.precision, s.uniform.data(),
                           true);
    if (rc) return rc;
    // layouts
    size_t o = 0;
    s.o_koff = o; o = align256(o + 8 * (count + 1));
    s.o_qoff = o; o = align256(o + 8 * (count + 1));
    s.o_sd = o;   o = align256(o + 8 * count);
    s.o_ed = o;   o = align256(o + 8 * count);
    s.o_x = o;    o = align256(o + 8 * nt);
    s.o_y = o;    o = align256(o + 8 * nt);
    s.o_xq = o;   o = align256(o + 8 * xt);
    s.o_tab = o;  o = align256(o + s.batch->table_bytes());
    s.in_bytes = o;
    o = 0;
    s.o_status = o; o = align256(o + 4 * count);
    s.o_bad = o;    o = align256(o + (s.batch->needs_bad() ? 4 * count : 0));
    s.o_yq = o;     o = align256(o + 8 * mt);
    s.o_ypp = o;    o = align256(o + 8 * nt);
    s.out_bytes = o;
    rc = rc ? rc : s.hin.ensure(s.in_bytes);
    rc = rc ? rc : s.hout.ensure(s.out_bytes);
    rc = rc ? rc : size_slot(c, s);
    if (rc) return rc;
    // stage the inputs
    std::memcpy(s.hin_at<int64_t>(s.o_koff), s.koff.data(), 8 * (count + 1));
    std::memcpy(s.hin_at<int64_t>(s.o_qoff), s.qoff.data(), 8 * (count + 1));
    int64_t xo = 0;
    for (int64_t i = 0; i < count; ++i) {
        const Req& r = *s.reqs[i];
        s.hin_at<double>(s.o_sd)[i] = r.sd;
        s.hin_at<double>(s.o_ed)[i] = r.ed;
        std::memcpy(s.hin_at<double>(s.o_x) + s.koff[i], r.x.data(), 8 * r.n);
        std::memcpy(s.hin_at<double>(s.o_y) + s.koff[i], r.y.data(), 8 * r.n);
        if (r.explicit_q()) {
            std::memcpy(s.hin_at<double>(s.o_xq) + xo, r.xq.data(), 8 * r.m);
            xo += r.m;
        }
    }
    s.batch->write_tables(s.hin_at<char>(s.o_tab));

    const bool use_graph = !(c->cfg.flags & SOLVE_NO_GRAPH);
    hipStream_t st = s.stream;
    s.drop_graph();
    // device outputs are written only after the work the caller had queued
    // on its stream when it submitted them
    for (int64_t i = 0; i < count; ++i)
        if (s.reqs[i]->ev && hipStreamWaitEvent(st, s.reqs[i]->ev, 0) != hipSuccess) return SOLVE_E_DEVICE;
    if (use_graph && hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) != hipSuccess) return SOLVE_E_DEVICE;
    if (hipMemcpyAsync(s.din.p, s.hin.p, s.in_bytes, hipMemcpyHostToDevice, st) != hipSuccess) rc = SOLVE_E_DEVICE;
    double* dx = s.din_at<double>(s.o_x);
    double* dy = s.din_at<double>(s.o_y);
    double* dyq = s.dout_at<double>(s.o_yq);
    double* dypp = s.dout_at<double>(s.o_ypp);
    if (!rc)
        rc = s.batch->launch_with_tables(s.din_at<char>(s.o_tab), dx, dy, s.din_at<double>(s.o_sd),
                                         s.din_at<double>(s.o_ed), s.din_at<int64_t>(s.o_koff),
                                         s.din_at<int64_t>(s.o_qoff), dyq, dypp, s.dout_at<int32_t>(s.o_status), st,
                                         nullptr, s.dout_at<int32_t>(s.o_bad));
    // curves too long for the batched kernels: the single-curve kernels
    // (y'' only, and one throw-away query, when the queries are explicit)
    for (int64_t i = 0; i < count && !rc; ++i) {
        const Req& r = *s.reqs[i];
        if (!r.solo()) continue;
        rc = spl::launch_solve_uniform(dx + s.koff[i], dy + s.koff[i], r.n, r.sd, r.ed, r.explicit_q() ? 1 : r.m,
                                       dyq + s.qoff[i], dypp + s.koff[i], nullptr, nullptr, st);
    }
    // every request with explicit points (the last count - e0 of the batch)
    // in one launch, from the y'' the kernels above left
    if (!rc && xt > 0) {
        const int64_t e0 = count - (int64_t)std::count_if(s.reqs.begin(), s.reqs.end(),
                                                          [](const ReqP& r) { return r->explicit_q(); });
        rc = spl::launch_eval_points_batch(count - e0, xt, s.din_at<int64_t>(s.o_koff) + e0,
                                           s.din_at<int64_t>(s.o_qoff) + e0, dx, dy, dypp, s.din_at<double>(s.o_xq),
                                           dyq + s.qoff[e0], nullptr, nullptr, nullptr, st);
    }
    // Results: device-resident callers get a device-to-device copy; host
    // callers are served from one copy of the output region.
    for (int64_t i = 0; i < count && !rc; ++i) {
        const Req& r = *s.reqs[i];
        if ((r.yq_dev || r.yq_pinned) &&
            hipMemcpyAsync(r.yq_out, dyq + s.qoff[i], 8 * r.m,
                           r.yq_dev ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, st) != hipSuccess)
            rc = SOLVE_E_DEVICE;
        if (!rc && r.ypp_out && (r.ypp_dev || r.ypp_pinned) &&
            hipMemcpyAsync(r.ypp_out, dypp + s.koff[i], 8 * r.n,
                           r.ypp_dev ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, st) != hipSuccess)
            rc = SOLVE_E_DEVICE;
    }
    const size_t back = host_ypp ? s.out_bytes : host_yq ? s.o_ypp : s.o_yq;
    if (!rc && hipMemcpyAsync(s.hout.p, s.dout.p, back, hipMemcpyDeviceToHost, st) != hipSuccess) rc = SOLVE_E_DEVICE;
    if (use_graph) {
        hipGraph_t g = nullptr;
        const hipError_t e = hipStreamEndCapture(st, &g);
        if (!rc && (e != hipSuccess || !g)) rc = SOLVE_E_DEVICE;
        if (g && rc) (void)hipGraphDestroy(g);
        if (!rc) {
            s.graph = g;
            if (hipGraphInstantiate(&s.exec, s.graph, nullptr, nullptr, 0) != hipSuccess) {
                s.exec = nullptr;
                rc = SOLVE_E_DEVICE;
            }
        }
        if (!rc && hipGraphLaunch(s.exec, st) != hipSuccess) rc = SOLVE_E_DEVICE;
    }
    if (!rc && hipEventRecord(s.done, st) != hipSuccess) rc = SOLVE_E_DEVICE;
    return rc;
}

// Deliver the results of a completed slot (called without the lock).
void deliver(Slot& s) {
    for (size_t i = 0; i < s.reqs.size(); ++i) {
        Req& r = *s.reqs[i];
        if (s.failed) continue;
        // (the knots of every request were checked at submit; the batched
        // kernels still report per curve, the single-curve path needs not)
        r.code = r.solo() ? SOLVE_OK : s.hout_at<int32_t>(s.o_status)[i];
        if (!r.yq_dev && !r.yq_pinned) std::memcpy(r.yq_out, s.hout_at<double>(s.o_yq) + s.qoff[i], 8 * r.m);
        if (r.ypp_out && !r.ypp_dev && !r.ypp_pinned)
            std::memcpy(r.ypp_out, s.hout_at<double>(s.o_ypp) + s.koff[i], 8 * r.n);
    }
}

// Requests for the next batch: FIFO within the budget and the slot limit,
// with a bounded look-ahead past a head request that does not fit yet.
std::vector<ReqP> admit_locked(solve_ctx* c) {
    std::vector<ReqP> out;
    const size_t window = 64;
    const int64_t max_batch_queries = (int64_t)1 << 27;
    uint64_t bytes = kBatchBytes;
    int64_t queries = 0;
    size_t scanned = 0;
    bool head_blocked = false;
    for (auto it = c->queue.begin(); it != c->queue.end() && scanned < window;) {
        ++scanned;
        const ReqP& r = *it;
        if (c->resident_reqs + out.size() + 1 > c->cfg.max_slots) break;
        const bool fits = c->resident + bytes + r->bytes <= c->cfg.hbm_budget_bytes &&
                          (out.empty() || queries + r->m <= max_batch_queries);
        if (fits && !(head_blocked && c->queue.front()->passed_over > 8)) {
            bytes += r->bytes;
            queries += r->m;
            out.push_back(r);
            it = c->queue.erase(it);
            continue;
        }
        if (!head_blocked) {
            head_blocked = true;
            ++r->passed_over;
            if (r->passed_over > 8) break;  // let the resident set drain for it
        }
        ++it;
    }
    return out;
}

void scheduler(solve_ctx* c) {
    (void)hipSetDevice(c->cfg.device);
    std::unique_lock<std::mutex> lk(c->mu);
    for (;;) {
        // 1. retire completed batches
        for (auto& sp : c->slots) {
            Slot& s = *sp;
            if (!s.busy) continue;
            const hipError_t q = hipEventQuery(s.done);
            if (q == hipErrorNotReady) continue;
            if (q != hipSuccess) s.failed = true;
            lk.unlock();
            if (!s.failed && hipStreamSynchronize(s.stream) != hipSuccess) s.failed = true;
            deliver(s);
            s.drop_graph();
            for (auto& r : s.reqs) event_put(c, r->ev);
            lk.lock();
            for (auto& r : s.reqs) {
                if (s.failed) finish_locked(c, r, SOLVE_ERROR, SOLVE_E_DEVICE);
                else finish_locked(c, r, r->code == SOLVE_OK ? SOLVE_DONE : SOLVE_ERROR, r->code);
            }
            c->resident -= s.bytes;
            c->resident_reqs -= s.reqs.size();
            s.reqs.clear();
            s.bytes = 0;
            s.busy = false;
            s.failed = false;
            c->spins = 0;
            c->cv_done.notify_all();
        }
        // 2. cancel queued work on shutdown
        if (c->stop && !c->queue.empty()) {
            for (auto& r : c->queue) {
                event_put(c, r->ev);
                finish_locked(c, r, SOLVE_ERROR, SOLVE_E_STATE);
            }
            c->queue.clear();
            c->cv_done.notify_all();
        }
        // 3. launch a new batch on a free slot
        Slot* free_slot = nullptr;
        bool any_busy = false;
        for (auto& sp : c->slots) {
            if (sp->busy) any_busy = true;
            else if (!free_slot) free_slot = sp.get();
        }
        if (!c->stop && free_slot && !c->queue.empty()) {
            std::vector<ReqP> reqs = admit_locked(c);
            if (!reqs.empty()) {
                Slot& s = *free_slot;
                s.busy = true;
                s.reqs = std::move(reqs);
                s.bytes = kBatchBytes;
                const double ta = now_s();
                for (auto& r : s.reqs) {
                    s.bytes += r->bytes;
                    r->t[1] = ta;
                }
                c->resident += s.bytes;
                c->resident_reqs += s.reqs.size();
                c->peak_resident = std::max(c->peak_resident, c->resident);
                c->peak_batch = std::max<uint64_t>(c->peak_batch, s.reqs.size());
                ++c->n_batches;
                const bool fault = c->inject;
                c->inject = false;
                lk.unlock();
                int rc = fault ? SOLVE_E_DEVICE : launch_batch(c, s);
                const double tl = now_s();
                lk.lock();
                for (auto& r : s.reqs) r->t[2] = tl;
                if (rc) {
                    // nothing of this batch reached the device, or it failed to
                    // launch: wait for whatever was queued, then fail its tickets
                    lk.unlock();
                    (void)hipStreamSynchronize(s.stream);
                    (void)hipGetLastError();
                    s.drop_graph();
                    for (auto& r : s.reqs) event_put(c, r->ev);
                    lk.lock();
                    for (auto& r : s.reqs) finish_locked(c, r, SOLVE_ERROR, rc == SOLVE_E_ORDER ? rc : SOLVE_E_DEVICE);
                    c->resident -= s.bytes;
                    c->resident_reqs -= s.reqs.size();
                    s.reqs.clear();
                    s.bytes = 0;
                    s.busy = false;
                    c->cv_done.notify_all();
                }
                continue;
            }
        }
        if (c->stop && c->queue.empty() && !any_busy) break;
        if (any_busy) {
            // a batch is on the device: poll its event again at once (the
            // latency of a finished batch is what a waiting caller sees),
            // backing off to short sleeps only after a long wait
            if (++c->spins < kSpinPolls) {
                lk.unlock();
                std::this_thread::yield();
                lk.lock();
            } else {
                c->cv_sched.wait_for(lk, std::chrono::microseconds(50));
            }
        } else {
            c->spins = 0;
            c->cv_sched.wait(lk);
        }
    }
}

// Copy n doubles of a caller's input into dst; a device input is read after
// `after` (recorded on the caller's stream), so after the work that produced it.
int copy_in(solve_ctx* c, std::vector<double>& dst, const double* src, int64_t n, bool on_device, hipEvent_t after) {
    dst.resize((size_t)n);
    if (on_device) {
        std::lock_guard<std::mutex> g(c->in_mu);
        hipError_t e = after ? hipStreamWaitEvent(c->in_stream, after, 0) : hipSuccess;
        if (e == hipSuccess)
            e = hipMemcpyAsync(dst.data(), src, 8 * (size_t)n, hipMemcpyDeviceToHost, c->in_stream);
        if (e == hipSuccess) e = hipStreamSynchronize(c->in_stream);
        if (e != hipSuccess) return hip_fail("copy of a device input", e);
    } else {
        std::memcpy(dst.data(), src, 8 * (size_t)n);
    }
    return SOLVE_OK;
}

int run_plain(solve_ctx* c, Req& r) {
    std::lock_guard<std::mutex> g(c->plain_mu);
    hipStream_t s = c->plain_stream;
    int rc = SOLVE_OK;
    // one request at a time: its buffers, with spare capacity while the
    // budget has room for it
    DevBuf* bufs[6] = {&c->px, &c->py, &c->pypp, &c->pyq, &c->pstatus, &c->pxq};
    const size_t need[6] = {8 * (size_t)r.n, 8 * (size_t)r.n, 8 * (size_t)r.n, 8 * (size_t)r.m, 4,
                            r.explicit_q() ? 8 * (size_t)r.m : 0};
    for (int b = 0; b < 6 && !rc; ++b) {
        if (!need[b] || (bufs[b]->p && bufs[b]->cap >= need[b])) continue;
        const uint64_t others = c->held.now.load() - bufs[b]->cap;
        const uint64_t room = c->cfg.hbm_budget_bytes > others ? c->cfg.hbm_budget_bytes - others : 0;
        rc = bufs[b]->resize(with_slack(need[b], room), s, c->held);
    }
    if (rc) return rc;
    r.t[1] = r.t[2] = now_s();
    // device outputs: after the work the caller had queued when it submitted
    hipError_t e = r.ev ? hipStreamWaitEvent(s, r.ev, 0) : hipSuccess;
    if (e == hipSuccess) e = hipMemcpyAsync(c->px.p, r.x.data(), 8 * r.n, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(c->py.p, r.y.data(), 8 * r.n, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemsetAsync(c->pstatus.p, 0, 4, s);  // SOLVE_OK; the kernels set E_ORDER only
    if (e != hipSuccess) return hip_fail("plain: input copy", e);
    // the single-launch path of spline_solve_uniform (with explicit queries:
    // its y'' and one throw-away uniform query, then the explicit evaluation)
    rc = spl::launch_solve_uniform(c->px.as<double>(), c->py.as<double>(), r.n, r.sd, r.ed,
                                   r.explicit_q() ? 1 : r.m, c->pyq.as<double>(), c->pypp.as<double>(),
                                   c->pstatus.as<int32_t>(), nullptr, s);
    if (!rc && r.explicit_q()) {
        e = hipMemcpyAsync(c->pxq.p, r.xq.data(), 8 * r.m, hipMemcpyHostToDevice, s);
        if (e != hipSuccess) return hip_fail("plain: query copy", e);
        rc = spl::launch_eval_points(c->px.as<double>(), c->py.as<double>(), c->pypp.as<double>(), r.n,
                                     c->pxq.as<double>(), r.m, c->pyq.as<double>(), nullptr, nullptr, nullptr, s);
    }
    if (rc) return rc;
    const hipMemcpyKind kq = r.yq_dev ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    e = hipMemcpyAsync(r.yq_out, c->pyq.p, 8 * r.m, kq, s);
    if (e == hipSuccess && r.ypp_out) {
        const hipMemcpyKind kp = r.ypp_dev ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
        e = hipMemcpyAsync(r.ypp_out, c->pypp.p, 8 * r.n, kp, s);
    }
    int32_t st = kStatusUnset;
    if (e == hipSuccess) e = hipMemcpyAsync(&st, c->pstatus.p, 4, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail("plain: result copy", e);
    if (st != SOLVE_OK && st != SOLVE_E_ORDER) {
        hip_fail("plain: status word", hipSuccess);
        return SOLVE_E_DEVICE;
    }
    return st;
}

}  // namespace

extern "C" double solve_clock(void) { return now_s(); }

extern "C" int solve_create(const solve_config* cfg, solve_ctx** out) {
    if (!cfg || !out) return SOLVE_E_ARG;
    *out = nullptr;
    if (cfg->hbm_budget_bytes == 0 || cfg->max_slots == 0) return SOLVE_E_ARG;
    if (cfg->precision != SOLVE_FP64 && cfg->precision != SOLVE_FP32_REFINE) return SOLVE_E_ARG;
    if (cfg->flags & ~(SOLVE_PLAIN | SOLVE_NO_GRAPH)) return SOLVE_E_ARG;
    if (cfg->max_inflight > 8) return SOLVE_E_ARG;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || cfg->device < 0 || cfg->device >= ndev) return SOLVE_E_DEVICE;
    DevCtx g(cfg->device);
    solve_ctx* c = new solve_ctx();
    c->cfg = *cfg;
    if (c->cfg.max_inflight == 0) c->cfg.max_inflight = 2;
    if (hipStreamCreateWithFlags(&c->plain_stream, hipStreamNonBlocking) != hipSuccess) {
        delete c;
        return SOLVE_E_DEVICE;
    }
    if (hipStreamCreateWithFlags(&c->in_stream, hipStreamNonBlocking) != hipSuccess) {
        (void)hipStreamDestroy(c->plain_stream);
        delete c;
        return SOLVE_E_DEVICE;
    }
    if (!(cfg->flags & SOLVE_PLAIN)) {
        for (uint32_t i = 0; i < c->cfg.max_inflight; ++i) {
            std::unique_ptr<Slot> s(new Slot());
            if (hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking) != hipSuccess ||
                hipEventCreateWithFlags(&s->done, hipEventDisableTiming) != hipSuccess) {
                if (s->stream) (void)hipStreamDestroy(s->stream);
                for (auto& t : c->slots) {
                    (void)hipStreamDestroy(t->stream);
                    (void)hipEventDestroy(t->done);
                }
                (void)hipStreamDestroy(c->plain_stream);
                (void)hipStreamDestroy(c->in_stream);
                delete c;
                return SOLVE_E_DEVICE;
            }
            c->slots.push_back(std::move(s));
        }
        c->sched = std::thread(scheduler, c);
    }
    *out = c;
    return SOLVE_OK;
}

extern "C" int solve_submit(solve_ctx* c, const double* knots, const double* values, int64_t n, double start_deriv,
                            double end_deriv, const double* xq, int64_t m, double* yq_out, double* ypp_out,
                            solve_ticket* ticket_out) {
    if (!c || !knots || !values || !yq_out || !ticket_out) return SOLVE_E_ARG;
    const bool plain = (c->cfg.flags & SOLVE_PLAIN) != 0;
    if (n < 3 || m < 1 || n > SOLVE_MAX_N_SOLVE) return SOLVE_E_SIZE;
    DevCtx g(c->cfg.device);
    ReqP r = std::make_shared<Req>();
    r->t[0] = now_s();
    r->n = n;
    r->m = m;
    r->sd = start_deriv;
    r->ed = end_deriv;
    r->yq_out = yq_out;
    r->ypp_out = ypp_out;
    const Mem kq = mem_kind(yq_out);
    const Mem kp = ypp_out ? mem_kind(ypp_out) : Mem::kPageable;
    r->yq_dev = kq == Mem::kDevice;
    r->yq_pinned = kq == Mem::kPinned;
    r->ypp_dev = ypp_out && kp == Mem::kDevice;
    r->ypp_pinned = ypp_out && kp == Mem::kPinned;
    const bool dx = is_device_ptr(knots), dy = is_device_ptr(values), dq = xq && is_device_ptr(xq);
    // Device memory of the caller is ordered after the work queued on the
    // caller's stream (cfg.stream, NULL = the legacy stream) when this call
    // is made: inputs are read after it, outputs written after it.
    hipEvent_t after = nullptr;
    if (dx || dy || dq || r->yq_dev || r->ypp_dev) {
        after = event_get(c);
        if (!after) return SOLVE_E_DEVICE;
        if (hipEventRecord(after, (hipStream_t)c->cfg.stream) != hipSuccess) {
            event_put(c, after);
            return hip_fail("solve_submit: event on the caller's stream", hipErrorUnknown);
        }
    }
    int rc = copy_in(c, r->x, knots, n, dx, after);
    if (!rc) rc = copy_in(c, r->y, values, n, dy, after);
    if (!rc && xq) rc = copy_in(c, r->xq, xq, m, dq, after);
    if (!rc)
        for (int64_t j = 1; j < n; ++j)
            if (!(r->x[j] > r->x[j - 1])) {
                rc = SOLVE_E_ORDER;
                break;
            }
    r->bytes = footprint(n, m, xq != nullptr, c->tuning.queries_per_tile);
    if (!rc && r->bytes + kBatchBytes > c->cfg.hbm_budget_bytes) rc = SOLVE_E_BUDGET;
    if (!rc && (r->yq_dev || r->ypp_dev)) r->ev = after;  // kept until the outputs are written
    else event_put(c, after);
    if (rc) {
        event_put(c, r->ev);
        return rc;
    }
    if (plain) {
        {
            std::lock_guard<std::mutex> lk(c->mu);
            if (c->stop) {
                event_put(c, r->ev);
                return SOLVE_E_STATE;
            }
            r->id = c->next_ticket++;
            ++c->n_submitted;
            c->tickets[r->id] = r;
        }
        const int prc = run_plain(c, *r);
        event_put(c, r->ev);
        std::lock_guard<std::mutex> lk(c->mu);
        if (prc == SOLVE_OK) finish_locked(c, r, SOLVE_DONE, SOLVE_OK);
        else finish_locked(c, r, SOLVE_ERROR, prc);
        *ticket_out = r->id;
        c->cv_done.notify_all();
        return SOLVE_OK;
    }
    std::lock_guard<std::mutex> lk(c->mu);
    if (c->stop) {
        event_put(c, r->ev);
        return SOLVE_E_STATE;
    }
    r->id = c->next_ticket++;
    ++c->n_submitted;
    c->tickets[r->id] = r;
    c->queue.push_back(r);
    *ticket_out = r->id;
    c->cv_sched.notify_one();
    return SOLVE_OK;
}

extern "C" int solve_poll(solve_ctx* c, solve_ticket t, int* status) {
    if (!c || !status) return SOLVE_E_ARG;
    std::lock_guard<std::mutex> lk(c->mu);
    auto it = c->tickets.find(t);
    if (it == c->tickets.end()) return SOLVE_E_TICKET;
    *status = it->second->status;
    if (*status != SOLVE_PENDING) c->tickets.erase(it);
    return SOLVE_OK;
}

extern "C" int solve_wait(solve_ctx* c, solve_ticket t, int* status, int64_t timeout_ms) {
    if (!c || !status) return SOLVE_E_ARG;
    std::unique_lock<std::mutex> lk(c->mu);
    auto it = c->tickets.find(t);
    if (it == c->tickets.end()) return SOLVE_E_TICKET;
    ReqP r = it->second;
    auto ready = [&] { return r->status != SOLVE_PENDING; };
    if (timeout_ms < 0) c->cv_done.wait(lk, ready);
    else c->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), ready);
    *status = r->status;
    return SOLVE_OK;
}

extern "C" int solve_ticket_info(solve_ctx* c, solve_ticket t, double times[4], int* error_code) {
    if (!c || !times) return SOLVE_E_ARG;
    std::lock_guard<std::mutex> lk(c->mu);
    auto it = c->tickets.find(t);
    if (it == c->tickets.end()) return SOLVE_E_TICKET;
    for (int i = 0; i < 4; ++i) times[i] = it->second->t[i];
    if (error_code) *error_code = it->second->code;
    return SOLVE_OK;
}

extern "C" int solve_stats(solve_ctx* c, uint64_t out[8]) {
    if (!c || !out) return SOLVE_E_ARG;
    std::lock_guard<std::mutex> lk(c->mu);
    out[0] = c->n_submitted;
    out[1] = c->n_completed;
    out[2] = c->n_failed;
    out[3] = c->n_batches;
    out[4] = c->resident;
    out[5] = c->peak_resident;
    out[6] = c->queue.size();
    out[7] = c->peak_batch;
    return SOLVE_OK;
}

extern "C" int solve_memory(solve_ctx* c, uint64_t out[2]) {
    if (!c || !out) return SOLVE_E_ARG;
    out[0] = c->held.now.load();
    out[1] = c->held.peak.load();
    return SOLVE_OK;
}

extern "C" int solve_inject_fault(solve_ctx* c) {
    if (!c) return SOLVE_E_ARG;
    std::lock_guard<std::mutex> lk(c->mu);
    c->inject = true;
    return SOLVE_OK;
}

extern "C" int solve_destroy(solve_ctx* c) {
    if (!c) return SOLVE_E_ARG;
    {
        std::lock_guard<std::mutex> lk(c->mu);
        c->stop = true;
        c->cv_sched.notify_all();
    }
    if (c->sched.joinable()) c->sched.join();
    DevCtx g(c->cfg.device);
    {
        std::lock_guard<std::mutex> pg(c->plain_mu);
        (void)hipStreamSynchronize(c->plain_stream);
    }
    for (auto& s : c->slots) {
        (void)hipStreamSynchronize(s->stream);
        s->drop_graph();
        s->batch.reset();
        s->din.drop(s->stream, c->held);
        s->dout.drop(s->stream, c->held);
        (void)hipStreamSynchronize(s->stream);
        s->hin.release();
        s->hout.release();
        (void)hipEventDestroy(s->done);
        (void)hipStreamDestroy(s->stream);
    }
    for (DevBuf* d : {&c->px, &c->py, &c->pypp, &c->pyq, &c->pxq, &c->pstatus}) d->drop(c->plain_stream, c->held);
    (void)hipStreamSynchronize(c->plain_stream);
    for (hipEvent_t e : c->ev_free) (void)hipEventDestroy(e);
    (void)hipStreamDestroy(c->plain_stream);
    (void)hipStreamDestroy(c->in_stream);
    delete c;
    return SOLVE_OK;
}

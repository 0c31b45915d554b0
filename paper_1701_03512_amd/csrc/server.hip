// Continuous-batching pricing server on one device.
//
// Submitters (any thread) append requests to a queue.  One server thread
// loops:
//   1. retire batches whose completion event has fired: copy their results
//      out of pinned memory, release their device memory, and either finish
//      each request or, for a Monte Carlo request whose pilot missed the
//      target error, queue its second stage;
//   2. if a stream is idle, take the class (exact or Monte Carlo) of the
//      longest-waiting request and admit that class's queued requests in
//      arrival order (MC second stages first) while in-flight slots and the
//      device-memory budget allow; launch them together on that stream: the
//      exact requests as one plan (one persistent enumeration over all
//      their work items), every MC request as its own estimate.  A batch
//      holds one class, so a short MC stage never waits for the end of a
//      long enumeration in its own batch;
//   3. otherwise, while batches run, poll their events for up to kSpinNs
//      (short batches finish within that), then sleep until a batch's
//      completion callback (hipLaunchHostFunc, enqueued behind the batch)
//      or a submission wakes the thread; with nothing in flight, sleep
//      until a submission.
// Batches on different streams overlap on the device, so requests that
// arrive while others run are admitted as soon as a stream and memory free
// up.  Device memory comes from one arena of `mem_budget` bytes carved with a
// first-fit allocator; admission is by that budget.
//
// Results do not depend on the mix: an exact value is the fixed-order sum
// of its own work items, and the MC draws of a request are keyed by a hash
// of the option itself (plus the stage), not by its ticket or position.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdint>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "bt.h"
#include "bt_internal.hpp"
#include "host_common.hpp"

using namespace bt;

namespace {

constexpr int kMaxStreams = 4;
constexpr int64_t kSpinNs = 100000;  // poll in-flight events this long before sleeping
constexpr int kMaxBatch = 1024;
// doubles of results per request in a batch's pinned buffer: an exact
// request's value and error bound, or an MC estimate's outputs
constexpr int kPinnedPerRequest = 8;
constexpr int kMcOut = 4;  // an MC estimate's outputs: value, two variances, var_plain
constexpr size_t kAlign = 256;

int64_t now_ns()
{
    return std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

// First-fit allocator over [0, size) with coalescing.
class Arena {
public:
    void init(size_t size) { free_[0] = size; }
    bool alloc(size_t n, size_t *off)
    {
        n = (n + kAlign - 1) & ~(kAlign - 1);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= n) {
                *off = it->first;
                const size_t rest = it->second - n, at = it->first + n;
                free_.erase(it);
                if (rest) free_[at] = rest;
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t n)
    {
        n = (n + kAlign - 1) & ~(kAlign - 1);
        auto it = free_.emplace(off, n).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }

private:
    std::map<size_t, size_t> free_;
};

struct Request {
    uint64_t ticket = 0;
    bt_option opt{};
    bool exact = true;
    int stage = 0;       // MC: 0 = pilot, 1 = main
    int32_t r = 0, Rm = 0;
    size_t bytes = 0;    // reserved budget
    bt_result res{};
    bt_times times{};
    bool done = false;
};

struct Batch {
    std::vector<Request *> exact, mc;
    bt_plan *plan = nullptr;
    size_t off = 0, bytes = 0;
};

uint32_t option_hash(const bt_option &o)
{
    uint32_t h = 2166136261u;
    const unsigned char *p = reinterpret_cast<const unsigned char *>(&o);
    for (size_t i = 0; i < sizeof(o); ++i) h = (h ^ p[i]) * 16777619u;
    return h;
}

size_t align_up(size_t x) { return (x + kAlign - 1) & ~(kAlign - 1); }

}  // namespace

struct bt_server {
    bt_server_config cfg{};
    int device = -1;
    int nstreams = 1;
    hipStream_t streams[kMaxStreams] = {};
    hipEvent_t events[kMaxStreams] = {};
    double *pinned[kMaxStreams] = {};
    Batch *inflight[kMaxStreams] = {};
    char *mem = nullptr;
    Arena arena;
    std::mutex mu;
    std::condition_variable cv;
    std::deque<Request *> pend_exact, pend_mc, second;
    std::unordered_map<uint64_t, Request *> all;
    std::atomic<bool> stop{false};
    bool wake = false;      // a submission or a batch completion since the last wait
    bool callbacks = true;  // completion callbacks enqueued (else poll on a timer)
    std::thread th;
    uint64_t next_ticket = 1;
    uint64_t n_submitted = 0, n_admitted = 0, n_completed = 0;
    size_t reserved = 0, peak = 0;
    int inflight_reqs = 0;
    void loop();
    bool launch(int si);
    void retire(int si);
    void fail_batch(Batch *b, int rc);
};

namespace {

// Host callback behind each batch: flag the completion and wake the server
// thread.  Runs on the HIP runtime's callback thread; calls no HIP API.
void batch_done(void *arg)
{
    bt_server *srv = static_cast<bt_server *>(arg);
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        srv->wake = true;
    }
    srv->cv.notify_one();
}

// MC shape for a stage: strata on the first r steps, R_m draws each.
void mc_shape(const bt_server_config &cfg, const bt_option &o, int stage, double n_paths,
              int32_t *r, int32_t *Rm)
{
    const int rmax = std::min(o.N - 1, 24);
    if (stage == 0) {
        *r = std::min(rmax, 12);
        *Rm = 64;
        const double cap = (double)cfg.mc_max_paths;
        while (*r > 0 && std::ldexp((double)*Rm, *r) > cap) --*r;
        return;
    }
    // Second stage: 4 draws per stratum and as many strata as the paths
    // allow (deeper stratification gives a smaller variance for the same
    // paths; below 4 draws the unbiased variance estimate gets coarse).
    const double want = std::min(n_paths, (double)cfg.mc_max_paths);
    int rr = (int)std::floor(std::log2(std::max(want / 4.0, 1.0)));
    *r = std::max(0, std::min(rmax, rr));
    *Rm = (int32_t)std::max(4.0, std::floor(want / std::ldexp(1.0, *r)));
}

// Exact requests use the launch shapes made for one tree at a time, never
// the built-in or autotuned shapes made for throughput over batches.
PlanSpec exact_spec()
{
    PlanSpec ps;
    ps.one_tree_shape = true;
    return ps;
}

size_t request_bytes(const bt_server_config &cfg, Request *q)
{
    if (q->exact) {
        size_t b = 0;
        const PlanSpec ps = exact_spec();
        if (plan_bytes(&q->opt, 1, cfg.precision, nullptr, &b, &ps)) return 0;
        return align_up(b);
    }
    return align_up(mc_scratch_bytes(q->r, q->Rm, nullptr, nullptr)) + kAlign;
}

}  // namespace

bool bt_server::launch(int si)
{
    Batch *b = new Batch();
    {
        std::lock_guard<std::mutex> lk(mu);
        auto admit = [&](std::deque<Request *> &dq) {
            while (!dq.empty() && (int)(b->exact.size() + b->mc.size()) < kMaxBatch &&
                   inflight_reqs < cfg.max_inflight) {
                Request *q = dq.front();
                if (q->bytes > cfg.mem_budget) {  // can never fit
                    dq.pop_front();
                    q->res.status = BT_ENOMEM;
                    q->times.t_done = now_ns();
                    q->done = true;
                    ++n_completed;
                    continue;
                }
                if (reserved + q->bytes > cfg.mem_budget) break;
                dq.pop_front();
                reserved += q->bytes;
                peak = std::max(peak, reserved);
                ++inflight_reqs;
                if (q->stage == 0) {
                    q->times.t_admit = now_ns();
                    ++n_admitted;
                }
                (q->exact ? b->exact : b->mc).push_back(q);
            }
        };
        // the class of the longest-waiting request (second stages keep
        // their submission time, so they go first)
        auto front_t = [](const std::deque<Request *> &dq) {
            return dq.empty() ? INT64_MAX : dq.front()->times.t_submit;
        };
        const int64_t t_mc = std::min(front_t(second), front_t(pend_mc));
        const bool mc_first = t_mc < front_t(pend_exact);
        for (int pass = 0; pass < 2 && b->exact.empty() && b->mc.empty(); ++pass) {
            if (mc_first == (pass == 0)) {
                admit(second);
                admit(pend_mc);
            } else {
                admit(pend_exact);  // or when the MC head does not fit
            }
        }
    }
    if (b->exact.empty() && b->mc.empty()) {
        delete b;
        return false;
    }
    hipStream_t s = streams[si];
    // Memory: [plan | 4 outputs of every MC request | MC scratch ...]
    std::vector<bt_option> eo;
    for (Request *q : b->exact) eo.push_back(q->opt);
    size_t plan_b = 0;
    const PlanSpec ps = exact_spec();
    if (!eo.empty() && plan_bytes(eo.data(), (int)eo.size(), cfg.precision, nullptr, &plan_b, &ps))
        plan_b = 0;
    size_t total = align_up(plan_b) + align_up(b->mc.size() * kMcOut * sizeof(double));
    std::vector<size_t> mc_off;
    for (Request *q : b->mc) {
        mc_off.push_back(total);
        total += align_up(mc_scratch_bytes(q->r, q->Rm, nullptr, nullptr));
    }
    int rc = BT_OK;
    {
        std::lock_guard<std::mutex> lk(mu);
        if (!arena.alloc(total, &b->off)) {
            // Fragmented arena: hand the requests back, in order, and retry
            // once an in-flight batch has released its block.
            for (auto *vec : {&b->mc, &b->exact})
                for (auto it = vec->rbegin(); it != vec->rend(); ++it) {
                    Request *q = *it;
                    reserved -= q->bytes;
                    --inflight_reqs;
                    if (q->stage == 0) --n_admitted;
                    (q->exact ? pend_exact : q->stage ? second : pend_mc).push_front(q);
                }
            delete b;
            return false;
        }
    }
    b->bytes = total;
    char *base = mem + b->off;
    if (!rc && !eo.empty())
        rc = plan_create_in(eo.data(), (int)eo.size(), cfg.precision, nullptr, base, plan_b,
                            false, s, &b->plan, &ps);
    if (!rc && b->plan) {
        rc = bt_plan_tables(b->plan, s);
        if (!rc) rc = bt_plan_enumerate(b->plan, s);
        if (!rc) rc = bt_plan_reduce(b->plan, s);
        double *dv = nullptr;
        if (!rc) rc = bt_plan_device_values(b->plan, &dv);
        // the values and then their error bounds
        if (!rc && hipMemcpyAsync(pinned[si], dv, 2 * eo.size() * sizeof(double),
                                  hipMemcpyDeviceToHost, s) != hipSuccess)
            rc = BT_EDEVICE;
    }
    double *outs = reinterpret_cast<double *>(base + align_up(plan_b));
    for (size_t j = 0; !rc && j < b->mc.size(); ++j) {
        Request *q = b->mc[j];
        const uint32_t sid = option_hash(q->opt) ^ (uint32_t)(q->stage * 0x9E3779B9u);
        rc = mc_enqueue(&q->opt, q->r, q->Rm, cfg.mc_seed, sid, cfg.precision, outs + kMcOut * j,
                        base + mc_off[j], s);
    }
    if (!rc && !b->mc.empty() &&
        hipMemcpyAsync(pinned[si] + 2 * eo.size(), outs, b->mc.size() * kMcOut * sizeof(double),
                       hipMemcpyDeviceToHost, s) != hipSuccess)
        rc = BT_EDEVICE;
    if (!rc && hipEventRecord(events[si], s) != hipSuccess) rc = BT_EDEVICE;
    // wake the server thread when the stream gets here (it may be asleep)
    if (!rc && callbacks && hipLaunchHostFunc(s, batch_done, this) != hipSuccess) {
        (void)hipGetLastError();
        callbacks = false;  // fall back to timed polling
    }
    if (rc) {
        // Nothing usable was queued: fail the batch's requests.
        (void)hipStreamSynchronize(s);
        fail_batch(b, rc);
        return true;
    }
    inflight[si] = b;
    return true;
}

// Release a batch that produced no results and finish its requests with
// status rc.  Its stream must be idle.
void bt_server::fail_batch(Batch *b, int rc)
{
    if (b->plan) bt_plan_destroy(b->plan);
    std::lock_guard<std::mutex> lk(mu);
    arena.release(b->off, b->bytes);
    for (auto *vec : {&b->exact, &b->mc})
        for (Request *q : *vec) {
            reserved -= q->bytes;
            --inflight_reqs;
            q->res.status = rc;
            q->times.t_done = now_ns();
            q->done = true;
            ++n_completed;
        }
    delete b;
}

void bt_server::retire(int si)
{
    Batch *b = inflight[si];
    inflight[si] = nullptr;
    const double *h = pinned[si];
    const int64_t t = now_ns();
    if (b->plan) bt_plan_destroy(b->plan);
    std::lock_guard<std::mutex> lk(mu);
    arena.release(b->off, b->bytes);
    for (size_t i = 0; i < b->exact.size(); ++i) {
        Request *q = b->exact[i];
        std::memset(&q->res, 0, sizeof(q->res));
        q->res.value = h[i];
        q->res.err_bound = h[b->exact.size() + i];
        q->res.paths = (uint64_t)1 << q->opt.N;
        q->res.split = resolve_tuning(q->opt.N, cfg.precision, nullptr, true).k;
        q->res.status = BT_OK;
        q->times.t_done = t;
        q->done = true;
        reserved -= q->bytes;
        --inflight_reqs;
        ++n_completed;
    }
    const size_t ne = 2 * b->exact.size();  // values and bounds of the exact requests
    for (size_t j = 0; j < b->mc.size(); ++j) {
        Request *q = b->mc[j];
        const double *o = h + ne + kMcOut * j;
        const double v = o[0], var = o[1], vub = o[2];
        const double paths = std::ldexp((double)q->Rm, q->r);
        std::memset(&q->res, 0, sizeof(q->res));
        q->res.value = v;
        q->res.var_est = var;
        q->res.var_unbiased = vub;
        q->res.var_plain = o[3];
        // the 1/(R_m - 1) form: unbiased at any number of draws per stratum
        q->res.std_err = std::sqrt(std::isfinite(vub) ? vub : var);
        q->res.err_bound = q->res.std_err;  // statistical: one standard error
        q->res.paths = (uint64_t)paths;
        q->res.split = q->r;
        q->res.status = BT_OK;
        reserved -= q->bytes;
        --inflight_reqs;
        const double rel = v > 0 ? q->res.std_err / v : INFINITY;
        if (q->stage == 0 && v > 0 && rel > cfg.mc_target_rel_se &&
            paths < (double)cfg.mc_max_paths) {
            const double want = paths * (rel / cfg.mc_target_rel_se) * (rel / cfg.mc_target_rel_se);
            int32_t r1, Rm1;
            mc_shape(cfg, q->opt, 1, want, &r1, &Rm1);
            Request next = *q;
            next.stage = 1;
            next.r = r1;
            next.Rm = Rm1;
            next.bytes = request_bytes(cfg, &next);
            // (a second stage larger than the whole budget could never be
            // admitted: the pilot's estimate stands)
            if (std::ldexp((double)Rm1, r1) > paths && next.bytes <= cfg.mem_budget) {
                q->stage = 1;
                q->r = r1;
                q->Rm = Rm1;
                q->bytes = next.bytes;
                second.push_back(q);
                continue;
            }
        }
        q->times.t_done = t;
        q->done = true;
        ++n_completed;
    }
    delete b;
}

void bt_server::loop()
{
    (void)hipSetDevice(device);
    int64_t idle_since = 0;  // start of the current run of fruitless polls
    for (;;) {
        bool busy = false, any_inflight = false;
        for (int i = 0; i < nstreams; ++i) {
            if (inflight[i]) {
                const hipError_t e = hipEventQuery(events[i]);
                if (e == hipSuccess) {
                    retire(i);
                    busy = true;
                } else if (e != hipErrorNotReady) {
                    // the batch will never complete: fail its requests
                    (void)hipStreamSynchronize(streams[i]);
                    fail_batch(inflight[i], BT_EDEVICE);
                    inflight[i] = nullptr;
                    busy = true;
                } else {
                    any_inflight = true;
                }
            }
        }
        if (stop.load()) {
            if (!any_inflight) {
                bool more = false;
                for (int i = 0; i < nstreams; ++i) more = more || inflight[i];
                if (!more) {
                    std::lock_guard<std::mutex> lk(mu);
                    for (auto *dq : {&pend_exact, &pend_mc, &second})
                        for (Request *q : *dq) {
                            q->res.status = BT_ESHUTDOWN;
                            q->times.t_done = now_ns();
                            q->done = true;
                            ++n_completed;
                        }
                    pend_exact.clear();
                    pend_mc.clear();
                    second.clear();
                    return;
                }
            }
        } else {
            for (int i = 0; i < nstreams; ++i)
                if (!inflight[i] && launch(i)) busy = true;
        }
        if (busy) {
            idle_since = 0;
            continue;
        }
        const int64_t t = now_ns();
        if (!idle_since) idle_since = t;
        if (any_inflight && t - idle_since < kSpinNs) {
            // a short batch is about to finish: look again at once
            std::this_thread::yield();
            continue;
        }
        // Sleep until a submission or (callbacks) a batch completion; the
        // timeout only bounds a wait whose wake-up was missed.
        std::unique_lock<std::mutex> lk(mu);
        const auto limit = (any_inflight && !callbacks) ? std::chrono::microseconds(50)
                                                        : std::chrono::microseconds(2000);
        cv.wait_for(lk, limit, [&] { return wake || stop.load(); });
        wake = false;
        idle_since = 0;
    }
}

extern "C" int bt_server_create(const bt_server_config *cfg, bt_server **out)
{
    if (!cfg || !out) return BT_EINVAL;
    *out = nullptr;
    if (cfg->mem_budget < (1u << 20) || cfg->max_inflight < 1 || cfg->streams < 1 ||
        cfg->streams > kMaxStreams || (cfg->precision != BT_FP64 && cfg->precision != BT_FP32_KAHAN) ||
        cfg->exact_max_n < 1 || cfg->exact_max_n > kExactMaxN || !(cfg->mc_target_rel_se > 0) ||
        cfg->mc_max_paths < 64)
        return BT_EINVAL;
    DeviceInfo *dev = nullptr;
    int rc = ensure_device(&dev);
    if (rc) return rc;
    bt_server *s = new (std::nothrow) bt_server();
    if (!s) return BT_ENOMEM;
    s->cfg = *cfg;
    s->device = dev->device;
    s->nstreams = cfg->streams;
    bool ok = hipMalloc(&s->mem, cfg->mem_budget) == hipSuccess;
    for (int i = 0; ok && i < s->nstreams; ++i) {
        ok = hipStreamCreateWithFlags(&s->streams[i], hipStreamNonBlocking) == hipSuccess &&
             hipEventCreateWithFlags(&s->events[i], hipEventDisableTiming) == hipSuccess &&
             hipHostMalloc(&s->pinned[i], kMaxBatch * kPinnedPerRequest * sizeof(double),
                           hipHostMallocDefault) == hipSuccess;
    }
    if (!ok) {
        for (int i = 0; i < s->nstreams; ++i) {
            if (s->pinned[i]) (void)hipHostFree(s->pinned[i]);
            if (s->events[i]) (void)hipEventDestroy(s->events[i]);
            if (s->streams[i]) (void)hipStreamDestroy(s->streams[i]);
        }
        if (s->mem) (void)hipFree(s->mem);
        delete s;
        return BT_ENOMEM;
    }
    s->arena.init(cfg->mem_budget);
    s->th = std::thread([s] { s->loop(); });
    *out = s;
    return BT_OK;
}

extern "C" int bt_server_submit(bt_server *srv, const bt_option *opt, uint64_t *ticket)
{
    if (!srv || !opt || !ticket) return BT_EINVAL;
    int rc = check_option(opt, kMcMaxN);
    if (rc) return rc;
    if (srv->stop.load()) return BT_ESHUTDOWN;
    Request *q = new (std::nothrow) Request();
    if (!q) return BT_ENOMEM;
    q->opt = *opt;
    q->exact = opt->N <= srv->cfg.exact_max_n;
    if (!q->exact) mc_shape(srv->cfg, *opt, 0, 0.0, &q->r, &q->Rm);
    q->bytes = request_bytes(srv->cfg, q);
    q->times.t_submit = now_ns();
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        q->ticket = srv->next_ticket++;
        srv->all[q->ticket] = q;
        (q->exact ? srv->pend_exact : srv->pend_mc).push_back(q);
        ++srv->n_submitted;
        srv->wake = true;
    }
    srv->cv.notify_one();
    *ticket = q->ticket;
    return BT_OK;
}

extern "C" int bt_server_poll(bt_server *srv, uint64_t ticket, bt_result *out, bt_times *times)
{
    if (!srv || !out) return BT_EINVAL;
    std::lock_guard<std::mutex> lk(srv->mu);
    auto it = srv->all.find(ticket);
    if (it == srv->all.end()) return BT_ENOTFOUND;
    Request *q = it->second;
    if (!q->done) return BT_EAGAIN;
    *out = q->res;
    if (times) *times = q->times;
    srv->all.erase(it);
    delete q;
    return BT_OK;
}

extern "C" int bt_server_stats(bt_server *srv, uint64_t *submitted, uint64_t *admitted,
                               uint64_t *completed, uint64_t *peak_bytes)
{
    if (!srv) return BT_EINVAL;
    std::lock_guard<std::mutex> lk(srv->mu);
    if (submitted) *submitted = srv->n_submitted;
    if (admitted) *admitted = srv->n_admitted;
    if (completed) *completed = srv->n_completed;
    if (peak_bytes) *peak_bytes = srv->peak;
    return BT_OK;
}

extern "C" void bt_server_destroy(bt_server *srv)
{
    if (!srv) return;
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        srv->stop.store(true);
        srv->wake = true;
    }
    srv->cv.notify_all();
    if (srv->th.joinable()) srv->th.join();
    // completion callbacks may still be queued behind the last events: let
    // them run before the server they point at goes away
    for (int i = 0; i < srv->nstreams; ++i)
        if (srv->streams[i]) (void)hipStreamSynchronize(srv->streams[i]);
    for (auto &kv : srv->all) delete kv.second;
    for (int i = 0; i < srv->nstreams; ++i) {
        if (srv->pinned[i]) (void)hipHostFree(srv->pinned[i]);
        if (srv->events[i]) (void)hipEventDestroy(srv->events[i]);
        if (srv->streams[i]) (void)hipStreamDestroy(srv->streams[i]);
    }
    if (srv->mem) (void)hipFree(srv->mem);
    delete srv;
}

// Serving: a request loop over many concurrent simulations with continuous
// batching, device-resident per-simulation results and admission by memory
// footprint.  The worker thread owns every device call of the server; the
// public calls only queue requests and read or lease state under the lock.
// Which request runs when, which buffers it writes and what may be freed are
// decided by the host-only policy in server_core.h.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "qbvh_internal.h"
#include "server_core.h"

namespace qbi {
namespace {

using Clock = std::chrono::steady_clock;

double now_ms() {
    return std::chrono::duration<double, std::milli>(Clock::now().time_since_epoch()).count();
}

// Device bytes a stream's batch context holds for batches of up to n particles
// (workspace, sort counters and scan partials, per-system tables).
size_t lane_bytes(int32_t n) { return n > 0 ? workspace_bytes(n) + (size_t)n / 16 * 4 + (1 << 20) : 0; }

// The request's arguments, kept until it is launched.
struct Payload {
    qbvh_request_t r;
    std::vector<float> rcut;
};

struct HipLane {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
};

struct HipOps final : srv::DeviceOps {
    std::vector<HipLane> *lanes = nullptr;
    void *alloc(size_t bytes) override {
        void *p = nullptr;
        if (hipMalloc(&p, bytes) != hipSuccess) {
            (void)hipGetLastError();
            return nullptr;
        }
        return p;
    }
    void free(void *p) override { (void)hipFree(p); }
    void release_lane(int lane) override { nlist_batch_release((*lanes)[(size_t)lane].stream); }
};

}  // namespace
}  // namespace qbi

struct qbvh_server {
    int device = 0;
    qbvh_server_opts_t opts{};
    std::mutex mu;
    std::condition_variable cv_work;  // wakes the worker
    std::condition_variable cv_done;  // wakes waiters
    std::vector<qbi::HipLane> lanes;
    qbi::HipOps ops;
    qbi::srv::Core *core = nullptr;
    std::unordered_map<int64_t, qbi::Payload> payload;  // queued requests' arguments
    bool stop = false;
    std::thread worker;
};

namespace qbi {
namespace {

// Launch everything admissible on idle lane `li`.  Called with the lock held.
void launch(qbvh_server &s, int li) {
    std::vector<int64_t> failed;
    std::vector<srv::Admitted> adm = s.core->admit(li, now_ms(), &failed);
    for (int64_t t : failed) s.payload.erase(t);
    if (!failed.empty()) s.cv_done.notify_all();
    if (adm.empty()) return;
    std::vector<qbvh_system_t> sys(adm.size());
    std::vector<Payload> keep;
    keep.reserve(adm.size());
    for (size_t i = 0; i < adm.size(); ++i) {
        auto it = s.payload.find(adm[i].ticket);
        keep.push_back(std::move(it->second));
        s.payload.erase(it);
        const qbvh_request_t &r = keep.back().r;
        qbvh_system_t &y = sys[i];
        y.d_pos = r.d_pos;
        y.d_type = r.d_type;
        y.n = r.n;
        y.ntypes = r.ntypes;
        memcpy(y.box, r.box, sizeof(y.box));
        y.rcut = keep.back().rcut.data();
        y.skin = r.skin;
        y.max_nbr = r.max_nbr;
        y.d_nbr = adm[i].nbr;
        y.d_count = adm[i].count;
        y.d_overflow = adm[i].overflow;
    }
    const HipLane &l = s.lanes[(size_t)li];
    int rc = nlist_build_many((int32_t)sys.size(), sys.data(), &s.opts.batch, l.stream);
    if (rc == QBVH_OK && hipEventRecord(l.done, l.stream) != hipSuccess) rc = hip_fail(hipGetLastError());
    if (rc != QBVH_OK) {
        s.core->complete(li, rc, now_ms());
        s.cv_done.notify_all();
    }
}

void worker_main(qbvh_server *sp) {
    qbvh_server &s = *sp;
    (void)hipSetDevice(s.device);
    std::unique_lock<std::mutex> lk(s.mu);
    for (;;) {
        bool progressed = false;
        for (int li = 0; li < s.core->lanes(); ++li) {
            if (!s.core->lane_busy(li)) continue;
            const hipError_t e = hipEventQuery(s.lanes[(size_t)li].done);
            if (e == hipErrorNotReady) continue;
            s.core->complete(li, e == hipSuccess ? QBVH_OK : hip_fail(e), now_ms());
            progressed = true;
        }
        if (progressed) s.cv_done.notify_all();
        for (int li = 0; li < s.core->lanes(); ++li) {
            if (s.core->lane_busy(li) || s.core->queue_empty()) continue;
            const size_t before = s.payload.size();
            launch(s, li);
            progressed = progressed || s.core->lane_busy(li) || s.payload.size() != before;
        }
        const bool inflight = s.core->any_busy();
        if (s.stop && s.core->queue_empty() && !inflight) break;
        if (progressed) continue;
        if (inflight)
            s.cv_work.wait_for(lk, std::chrono::microseconds(20));
        else
            s.cv_work.wait(lk);
    }
}

}  // namespace
}  // namespace qbi

extern "C" {

int qbvh_server_create(qbvh_server_t **srv, const qbvh_server_opts_t *opts) {
    if (!srv || !opts || opts->budget_bytes == 0) return QBVH_EINVAL;
    qbvh_server_opts_t o = *opts;
    if (o.max_inflight == 0) o.max_inflight = 2;
    if (o.max_batch == 0) o.max_batch = 64;
    if (o.max_inflight < 1 || o.max_inflight > 8 || o.max_batch < 1) return QBVH_EINVAL;
    if (o.batch.leaf_size == 0) o.batch.leaf_size = 16;
    if (o.batch.qbits == 0) o.batch.qbits = 16;
    if (o.batch.block_size == 0) o.batch.block_size = 64;
    o.batch.eager = 1;
    if (!qbi::leaf_ok(o.batch.leaf_size) || !qbi::qbits_ok(o.batch.qbits) || !qbi::block_ok(o.batch.block_size))
        return QBVH_EINVAL;
    qbvh_server_t *s = new (std::nothrow) qbvh_server_t();
    if (!s) return QBVH_ENOMEM;
    s->opts = o;
    hipError_t e = hipGetDevice(&s->device);
    s->lanes.resize((size_t)o.max_inflight);
    for (qbi::HipLane &l : s->lanes) {
        if (e == hipSuccess) e = hipStreamCreateWithFlags(&l.stream, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&l.done, hipEventDisableTiming);
    }
    if (e == hipSuccess) {
        s->ops.lanes = &s->lanes;
        s->core = new (std::nothrow) qbi::srv::Core(o.budget_bytes, o.max_inflight, o.max_batch, &s->ops,
                                                    qbi::lane_bytes);
    }
    if (e != hipSuccess || !s->core) {
        for (qbi::HipLane &l : s->lanes) {
            if (l.done) (void)hipEventDestroy(l.done);
            if (l.stream) (void)hipStreamDestroy(l.stream);
        }
        delete s;
        return e != hipSuccess ? qbi::hip_fail(e) : QBVH_ENOMEM;
    }
    s->worker = std::thread(qbi::worker_main, s);
    *srv = s;
    return QBVH_OK;
}

int qbvh_server_submit(qbvh_server_t *srv, const qbvh_request_t *req, int64_t *ticket) {
    if (!srv || !req || !ticket) return QBVH_EINVAL;
    const qbvh_request_t &r = *req;
    if (r.sim_id < 0 || r.n < 1 || r.n > qbi::kMaxParticles || r.ntypes < 1 || r.ntypes > QBVH_MAX_TYPES ||
        !qbi::box_ok(r.box) || r.max_nbr < 1 || !r.d_pos || (r.ntypes > 1 && !r.d_type))
        return QBVH_EINVAL;
    double r2[QBVH_MAX_TYPES * QBVH_MAX_TYPES];
    int rc = qbi::list_radii(r.rcut, r.skin, r.ntypes, r.box, r2);
    if (rc != QBVH_OK) return rc;
    qbi::Payload p;
    p.r = r;
    p.rcut.assign(r.rcut, r.rcut + (size_t)r.ntypes * r.ntypes);
    p.r.rcut = nullptr;
    std::lock_guard<std::mutex> lk(srv->mu);
    int64_t t = 0;
    rc = srv->core->submit(r.sim_id, r.n, r.max_nbr, qbi::now_ms(), &t);
    if (rc != QBVH_OK) return rc;
    srv->payload[t] = std::move(p);
    *ticket = t;
    srv->cv_work.notify_one();
    return QBVH_OK;
}

int qbvh_server_poll(qbvh_server_t *srv, int64_t ticket, int32_t *done) {
    if (!srv || !done) return QBVH_EINVAL;
    std::lock_guard<std::mutex> lk(srv->mu);
    *done = 0;
    if (!srv->core->known(ticket)) return QBVH_EINVAL;
    const int st = srv->core->status(ticket, true);
    if (st == qbi::srv::kPending) return QBVH_OK;
    *done = 1;
    return st;
}

int qbvh_server_wait(qbvh_server_t *srv, int64_t ticket) {
    if (!srv) return QBVH_EINVAL;
    std::unique_lock<std::mutex> lk(srv->mu);
    if (!srv->core->known(ticket)) return QBVH_EINVAL;
    srv->cv_done.wait(lk, [&] { return srv->core->status(ticket, false) != qbi::srv::kPending; });
    return srv->core->status(ticket, true);
}

int qbvh_server_result(qbvh_server_t *srv, int32_t sim_id, const int32_t **d_nbr, const int32_t **d_count,
                       const int32_t **d_overflow, int32_t *n, int32_t *max_nbr) {
    if (!srv) return QBVH_EINVAL;
    std::lock_guard<std::mutex> lk(srv->mu);
    qbi::srv::Buffer b;
    const int rc = srv->core->lease(sim_id, &b);
    if (rc != QBVH_OK) return rc;
    if (d_nbr) *d_nbr = b.nbr();
    if (d_count) *d_count = b.count();
    if (d_overflow) *d_overflow = b.overflow();
    if (n) *n = b.res_n;
    if (max_nbr) *max_nbr = b.res_nbr;
    return QBVH_OK;
}

int qbvh_server_release(qbvh_server_t *srv, int32_t sim_id, const int32_t *d_nbr) {
    if (!srv) return QBVH_EINVAL;
    std::lock_guard<std::mutex> lk(srv->mu);
    const int rc = srv->core->release(sim_id, d_nbr);
    // memory may have become free for a queued request
    srv->cv_work.notify_one();
    return rc;
}

int qbvh_server_stats(qbvh_server_t *srv, qbvh_server_stats_t *st) {
    if (!srv || !st) return QBVH_EINVAL;
    std::vector<double> lat;
    qbi::srv::Stats s;
    size_t resident = 0;
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        s = srv->core->stats();
        lat = srv->core->latencies();
        resident = srv->core->bytes_buffers();
    }
    memset(st, 0, sizeof(*st));
    st->submitted = s.submitted;
    st->completed = s.completed;
    st->batches = s.batches;
    st->refused = s.refused;
    if (!lat.empty()) {
        std::sort(lat.begin(), lat.end());
        auto pct = [&](double p) {
            const size_t i = (size_t)std::min<double>((double)lat.size() - 1, ceil(p * (double)lat.size()) - 1);
            return lat[i];
        };
        st->p50_ms = pct(0.50);
        st->p99_ms = pct(0.99);
        double sum = 0;
        for (double x : lat) sum += x;
        st->mean_ms = sum / (double)lat.size();
        const double span = (s.last_done - s.first_submit) * 1e-3;
        if (span > 0) {
            st->requests_per_s = (double)s.completed / span;
            st->particles_per_s = s.particles_done / span;
        }
    }
    st->mean_batch = s.batches ? (double)s.batched_requests / (double)s.batches : 0.0;
    st->bytes_resident = resident;
    st->bytes_peak = s.bytes_peak;
    return QBVH_OK;
}

void qbvh_server_destroy(qbvh_server_t *srv) {
    if (!srv) return;
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        srv->stop = true;
    }
    srv->cv_work.notify_all();
    if (srv->worker.joinable()) srv->worker.join();
    (void)hipSetDevice(srv->device);
    delete srv->core;  // frees every session buffer
    for (qbi::HipLane &l : srv->lanes) {
        nlist_batch_release(l.stream);
        if (l.done) (void)hipEventDestroy(l.done);
        if (l.stream) (void)hipStreamDestroy(l.stream);
    }
    delete srv;
}

}  // extern "C"

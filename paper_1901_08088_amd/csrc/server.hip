// Serving: a request loop over many concurrent simulations with continuous
// batching, device-resident per-simulation lists and admission by memory
// footprint.  The worker thread owns every device call of the server; the
// public calls only queue requests and read state under the lock.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <set>
#include <thread>
#include <unordered_map>
#include <vector>

#include "qbvh_internal.h"

namespace qbi {
namespace {

using Clock = std::chrono::steady_clock;

double now_ms() {
    return std::chrono::duration<double, std::milli>(Clock::now().time_since_epoch()).count();
}

constexpr int kPending = 1;  // ticket status while queued or running

struct Session {
    int32_t cap_n = 0, cap_nbr = 0;  // buffer capacity (particles, row length)
    size_t bytes = 0;
    void *mem = nullptr;
    int32_t *nbr = nullptr, *count = nullptr, *overflow = nullptr;
    bool busy = false;         // a request of this sim is admitted and not finished
    bool has_result = false;
    int32_t res_n = 0, res_nbr = 0;
    uint64_t last_use = 0;
};

struct Request {
    int64_t ticket;
    qbvh_request_t r;
    std::vector<float> rcut;
    double t_submit;
};

struct Ticket {
    int status = kPending;
    int32_t sim = 0;
    int32_t n = 0;
    double t_submit = 0, t_done = 0;
};

struct Lane {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    bool busy = false;
    int32_t ws_cap = 0;  // largest batch (particles) this stream's batch context was sized for
    std::vector<int64_t> tickets;
    std::vector<int32_t> sims;
};

size_t session_bytes(int32_t n, int32_t max_nbr) {
    auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
    return al((size_t)n * (size_t)max_nbr * 4) + al((size_t)n * 4) + al(4);
}

// Device bytes a stream's batch context holds for batches of up to n particles.
size_t stream_bytes(int32_t n) { return n > 0 ? workspace_bytes(n) + (size_t)n / 16 * 4 + (1 << 20) : 0; }

}  // namespace
}  // namespace qbi

struct qbvh_server {
    int device = 0;
    qbvh_server_opts_t opts{};
    std::mutex mu;
    std::condition_variable cv_work;  // wakes the worker
    std::condition_variable cv_done;  // wakes waiters
    std::deque<qbi::Request> queue;
    std::unordered_map<int64_t, qbi::Ticket> tickets;
    std::map<int32_t, qbi::Session> sessions;
    std::vector<qbi::Lane> lanes;
    int64_t next_ticket = 1;
    uint64_t use_clock = 0;
    bool stop = false;
    size_t bytes_sessions = 0, bytes_peak = 0;
    // statistics
    int64_t submitted = 0, completed = 0, batches = 0, refused = 0, batched_requests = 0;
    double first_submit = -1, last_done = -1;
    double particles_done = 0;
    std::vector<double> latencies;
    std::thread worker;
};

namespace qbi {
namespace {

size_t lanes_bytes(const qbvh_server &s) {
    size_t b = 0;
    for (const Lane &l : s.lanes) b += stream_bytes(l.ws_cap);
    return b;
}

void finish_lane(qbvh_server &s, Lane &l, int status) {
    const double t = now_ms();
    for (size_t i = 0; i < l.tickets.size(); ++i) {
        Ticket &tk = s.tickets[l.tickets[i]];
        tk.status = status;
        tk.t_done = t;
        Session &ss = s.sessions[l.sims[i]];
        ss.busy = false;
        if (status == QBVH_OK) {
            ss.has_result = true;
            ++s.completed;
            s.latencies.push_back(t - tk.t_submit);
            s.particles_done += tk.n;
            s.last_done = t;
        }
    }
    l.tickets.clear();
    l.sims.clear();
    l.busy = false;
}

// Make room for `need` more bytes by evicting idle sessions (LRU), never one
// in `keep`.  Returns whether the bytes fit afterwards.
bool make_room(qbvh_server &s, size_t need, size_t extra_lanes, const std::set<int32_t> &keep) {
    const size_t budget = s.opts.budget_bytes;
    while (s.bytes_sessions + extra_lanes + need > budget) {
        int32_t victim = -1;
        uint64_t oldest = UINT64_MAX;
        for (auto &kv : s.sessions) {
            const Session &ss = kv.second;
            if (ss.busy || !ss.mem || keep.count(kv.first)) continue;
            if (ss.last_use < oldest) {
                oldest = ss.last_use;
                victim = kv.first;
            }
        }
        if (victim < 0) return false;
        Session &v = s.sessions[victim];
        (void)hipFree(v.mem);
        s.bytes_sessions -= v.bytes;
        s.sessions.erase(victim);
    }
    return true;
}

// Take every admissible queued request (FIFO, per-sim order kept) into one
// batch on lane `li`.  Called with the lock held.
void launch(qbvh_server &s, size_t li) {
    Lane &l = s.lanes[li];
    std::set<int32_t> seen;  // sims met in this scan: later requests of theirs wait
    std::set<int32_t> taken;
    std::vector<qbvh_system_t> sys;
    std::vector<std::vector<float>> rcuts;
    int64_t total = 0;
    size_t others = 0;
    for (size_t j = 0; j < s.lanes.size(); ++j)
        if (j != li) others += stream_bytes(s.lanes[j].ws_cap);
    for (auto it = s.queue.begin(); it != s.queue.end() && (int32_t)sys.size() < s.opts.max_batch;) {
        const qbvh_request_t &r = it->r;
        const int32_t sim = r.sim_id;
        if (seen.count(sim)) {
            ++it;
            continue;
        }
        seen.insert(sim);
        auto sit = s.sessions.find(sim);
        if (sit != s.sessions.end() && sit->second.busy) {
            ++it;
            continue;
        }
        // a batch holds at most kMaxParticles in all (the request waits for a later batch)
        if (total + r.n > qbi::kMaxParticles) {
            ++it;
            continue;
        }
        const bool fits_buffers = sit != s.sessions.end() && sit->second.cap_n >= r.n &&
                                  sit->second.cap_nbr >= r.max_nbr && sit->second.mem;
        const size_t new_bytes = fits_buffers ? 0 : session_bytes(r.n, r.max_nbr);
        const size_t old_bytes = (!fits_buffers && sit != s.sessions.end()) ? sit->second.bytes : 0;
        const int32_t lane_cap = (int32_t)std::max<int64_t>(l.ws_cap, total + r.n);
        const size_t lane_need = others + stream_bytes(lane_cap);
        std::set<int32_t> keep = taken;
        keep.insert(sim);
        const size_t need = new_bytes > old_bytes ? new_bytes - old_bytes : 0;
        if (!make_room(s, need, lane_need, keep)) {
            ++it;
            continue;
        }
        Session &ss = s.sessions[sim];
        if (!fits_buffers) {
            if (ss.mem) {
                (void)hipFree(ss.mem);
                s.bytes_sessions -= ss.bytes;
                ss = Session{};
            }
            void *mem = nullptr;
            if (hipMalloc(&mem, new_bytes) != hipSuccess) {
                (void)hipGetLastError();
                Ticket &tk = s.tickets[it->ticket];
                tk.status = QBVH_ENOMEM;
                s.sessions.erase(sim);
                it = s.queue.erase(it);
                s.cv_done.notify_all();
                continue;
            }
            ss.mem = mem;
            ss.bytes = new_bytes;
            ss.cap_n = r.n;
            ss.cap_nbr = r.max_nbr;
            char *p = (char *)mem;
            ss.nbr = (int32_t *)p;
            ss.count = (int32_t *)(p + (((size_t)r.n * r.max_nbr * 4 + 255) & ~(size_t)255));
            ss.overflow = (int32_t *)((char *)ss.count + (((size_t)r.n * 4 + 255) & ~(size_t)255));
            s.bytes_sessions += new_bytes;
        }
        ss.busy = true;
        ss.last_use = ++s.use_clock;
        ss.res_n = r.n;
        ss.res_nbr = r.max_nbr;
        qbvh_system_t y{};
        y.d_pos = r.d_pos;
        y.d_type = r.d_type;
        y.n = r.n;
        y.ntypes = r.ntypes;
        memcpy(y.box, r.box, sizeof(y.box));
        rcuts.push_back(it->rcut);
        y.skin = r.skin;
        y.max_nbr = r.max_nbr;
        y.d_nbr = ss.nbr;
        y.d_count = ss.count;
        y.d_overflow = ss.overflow;
        sys.push_back(y);
        l.tickets.push_back(it->ticket);
        l.sims.push_back(sim);
        taken.insert(sim);
        total += r.n;
        l.ws_cap = lane_cap;
        it = s.queue.erase(it);
    }
    if (sys.empty()) return;
    for (size_t i = 0; i < sys.size(); ++i) sys[i].rcut = rcuts[i].data();
    s.bytes_peak = std::max(s.bytes_peak, s.bytes_sessions + lanes_bytes(s));
    int rc = nlist_build_many((int32_t)sys.size(), sys.data(), &s.opts.batch, l.stream);
    if (rc == QBVH_OK && hipEventRecord(l.done, l.stream) != hipSuccess) rc = hip_fail(hipGetLastError());
    ++s.batches;
    s.batched_requests += (int64_t)sys.size();
    l.busy = true;
    if (rc != QBVH_OK) {
        finish_lane(s, l, rc);
        s.cv_done.notify_all();
    }
}

void worker_main(qbvh_server *sp) {
    qbvh_server &s = *sp;
    (void)hipSetDevice(s.device);
    std::unique_lock<std::mutex> lk(s.mu);
    for (;;) {
        bool progressed = false;
        for (Lane &l : s.lanes) {
            if (!l.busy) continue;
            const hipError_t e = hipEventQuery(l.done);
            if (e == hipErrorNotReady) continue;
            finish_lane(s, l, e == hipSuccess ? QBVH_OK : hip_fail(e));
            progressed = true;
        }
        if (progressed) s.cv_done.notify_all();
        bool inflight = false;
        for (size_t li = 0; li < s.lanes.size(); ++li) {
            if (!s.lanes[li].busy && !s.queue.empty()) {
                launch(s, li);
                progressed = progressed || s.lanes[li].busy;
            }
            inflight = inflight || s.lanes[li].busy;
        }
        if (s.stop && s.queue.empty() && !inflight) break;
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
    for (qbi::Lane &l : s->lanes) {
        if (e == hipSuccess) e = hipStreamCreateWithFlags(&l.stream, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&l.done, hipEventDisableTiming);
    }
    if (e != hipSuccess) {
        for (qbi::Lane &l : s->lanes) {
            if (l.done) (void)hipEventDestroy(l.done);
            if (l.stream) (void)hipStreamDestroy(l.stream);
        }
        delete s;
        return qbi::hip_fail(e);
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
    const size_t need = qbi::session_bytes(r.n, r.max_nbr) + qbi::stream_bytes(r.n);
    std::lock_guard<std::mutex> lk(srv->mu);
    if (need > srv->opts.budget_bytes) {
        ++srv->refused;
        return QBVH_EAGAIN;
    }
    qbi::Request q;
    q.ticket = srv->next_ticket++;
    q.r = r;
    q.rcut.assign(r.rcut, r.rcut + (size_t)r.ntypes * r.ntypes);
    q.r.rcut = nullptr;
    q.t_submit = qbi::now_ms();
    qbi::Ticket tk;
    tk.sim = r.sim_id;
    tk.n = r.n;
    tk.t_submit = q.t_submit;
    srv->tickets[q.ticket] = tk;
    if (srv->first_submit < 0) srv->first_submit = q.t_submit;
    ++srv->submitted;
    *ticket = q.ticket;
    srv->queue.push_back(std::move(q));
    srv->cv_work.notify_one();
    return QBVH_OK;
}

int qbvh_server_poll(qbvh_server_t *srv, int64_t ticket, int32_t *done) {
    if (!srv || !done) return QBVH_EINVAL;
    std::lock_guard<std::mutex> lk(srv->mu);
    auto it = srv->tickets.find(ticket);
    if (it == srv->tickets.end()) return QBVH_EINVAL;
    *done = it->second.status == qbi::kPending ? 0 : 1;
    return it->second.status == qbi::kPending ? QBVH_OK : it->second.status;
}

int qbvh_server_wait(qbvh_server_t *srv, int64_t ticket) {
    if (!srv) return QBVH_EINVAL;
    std::unique_lock<std::mutex> lk(srv->mu);
    auto it = srv->tickets.find(ticket);
    if (it == srv->tickets.end()) return QBVH_EINVAL;
    srv->cv_done.wait(lk, [&] { return srv->tickets[ticket].status != qbi::kPending; });
    return srv->tickets[ticket].status;
}

int qbvh_server_result(qbvh_server_t *srv, int32_t sim_id, const int32_t **d_nbr, const int32_t **d_count,
                       const int32_t **d_overflow, int32_t *n, int32_t *max_nbr) {
    if (!srv) return QBVH_EINVAL;
    std::lock_guard<std::mutex> lk(srv->mu);
    auto it = srv->sessions.find(sim_id);
    if (it == srv->sessions.end() || !it->second.has_result || !it->second.mem) return QBVH_EINVAL;
    const qbi::Session &ss = it->second;
    if (d_nbr) *d_nbr = ss.nbr;
    if (d_count) *d_count = ss.count;
    if (d_overflow) *d_overflow = ss.overflow;
    if (n) *n = ss.res_n;
    if (max_nbr) *max_nbr = ss.res_nbr;
    return QBVH_OK;
}

int qbvh_server_stats(qbvh_server_t *srv, qbvh_server_stats_t *st) {
    if (!srv || !st) return QBVH_EINVAL;
    std::lock_guard<std::mutex> lk(srv->mu);
    memset(st, 0, sizeof(*st));
    st->submitted = srv->submitted;
    st->completed = srv->completed;
    st->batches = srv->batches;
    st->refused = srv->refused;
    std::vector<double> lat = srv->latencies;
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
        const double span = (srv->last_done - srv->first_submit) * 1e-3;
        if (span > 0) {
            st->requests_per_s = (double)srv->completed / span;
            st->particles_per_s = srv->particles_done / span;
        }
    }
    st->mean_batch = srv->batches ? (double)srv->batched_requests / (double)srv->batches : 0.0;
    st->bytes_resident = srv->bytes_sessions;
    st->bytes_peak = srv->bytes_peak;
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
    for (auto &kv : srv->sessions)
        if (kv.second.mem) (void)hipFree(kv.second.mem);
    for (qbi::Lane &l : srv->lanes) {
        nlist_batch_release(l.stream);
        if (l.done) (void)hipEventDestroy(l.done);
        if (l.stream) (void)hipStreamDestroy(l.stream);
    }
    delete srv;
}

}  // extern "C"

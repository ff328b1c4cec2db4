// Admission, session and result-lifetime policy of the neighbor-list server.
//
// Host-only C++ (no HIP): the device operations it decides on -- allocating
// and freeing a session's result buffers, releasing a stream's batch
// workspace -- go through the DeviceOps interface, which the server
// implements with HIP and the unit tests with a fake.  Every method must be
// called with the server's lock held.
//
// Rules:
//   - A session (one per sim_id) holds one or more result buffers (list,
//     counts, overflow flag).  `pub` is the buffer of the sim's last completed
//     request: what qbvh_server_result hands out.
//   - qbvh_server_result leases the published buffer; a leased buffer is
//     neither written nor freed until every lease on it is released.
//   - A request needs one result buffer that no lease holds plus its share of
//     its lane's batch workspace.  In order of preference it writes a spare
//     buffer (neither published, leased nor being written) large enough; a
//     new buffer, if it fits after freeing spare buffers; the published
//     buffer, if no lease holds it (the sim then has no published result
//     until the request completes); a new buffer after evicting whole idle
//     sessions without leases, least recently used first.  It is admitted
//     when the bytes of all buffers and of every lane's workspace fit the
//     budget.  Requests of one sim run one at a time, in submission order; a
//     request that does not fit yet does not block smaller ones behind it.
//   - When no lane is running and the queue cannot make progress, the lanes'
//     workspaces are released and the scan repeated; requests that still do
//     not fit (the budget is held by leased buffers) fail with QBVH_EAGAIN.
//     So every queued request eventually runs or fails.
//   - A ticket is forgotten once its completion has been reported by poll or
//     wait.  Latency statistics keep the most recent kLatencyWindow requests.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include <algorithm>
#include <deque>
#include <map>
#include <set>
#include <unordered_map>
#include <vector>

#include "../../include/qbvh.h"

namespace qbi {
namespace srv {

constexpr int kPending = 1;  // ticket status while queued or running
constexpr size_t kLatencyWindow = 1u << 16;
constexpr int64_t kMaxBatchParticles = (1 << 27) - 1;  // particle runs address sorted positions in 27 bits

struct DeviceOps {
    virtual ~DeviceOps() = default;
    virtual void *alloc(size_t bytes) = 0;   // nullptr on failure
    virtual void free(void *p) = 0;
    virtual void release_lane(int lane) = 0; // drop the lane's batch workspace (the lane is idle)
};

inline size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

// Bytes of one result buffer: list [n][max_nbr], counts [n], overflow flag.
inline size_t buffer_bytes(int32_t n, int32_t max_nbr) {
    return align256((size_t)n * (size_t)max_nbr * 4) + align256((size_t)n * 4) + align256(4);
}

struct Buffer {
    void *mem = nullptr;
    size_t bytes = 0;
    int32_t cap_n = 0, cap_nbr = 0;  // capacity
    int32_t res_n = 0, res_nbr = 0;  // shape of the result it holds (or is being written)
    int32_t leases = 0;
    int32_t *nbr() const { return (int32_t *)mem; }
    int32_t *count() const { return (int32_t *)((char *)mem + align256((size_t)cap_n * (size_t)cap_nbr * 4)); }
    int32_t *overflow() const { return (int32_t *)((char *)count() + align256((size_t)cap_n * 4)); }
};

struct Session {
    std::vector<Buffer> bufs;
    int pub = -1;   // published buffer (last completed request), -1 if none
    int work = -1;  // buffer the running request writes, -1 when idle
    bool busy = false;
    uint64_t last_use = 0;
    bool leased() const {
        for (const Buffer &b : bufs)
            if (b.leases > 0) return true;
        return false;
    }
};

struct Request {
    int64_t ticket = 0;
    int32_t sim = 0, n = 0, max_nbr = 0;
    double t_submit = 0;
};

struct Ticket {
    int status = kPending;
    int32_t sim = 0, n = 0;
    double t_submit = 0, t_done = 0;
};

struct Lane {
    bool busy = false;
    int32_t ws_cap = 0;  // particles the lane's batch workspace is sized for
    std::vector<int64_t> tickets;
    std::vector<int32_t> sims;
};

// One admitted request: where its results go.
struct Admitted {
    int64_t ticket;
    int32_t sim;
    int32_t *nbr, *count, *overflow;
};

struct Stats {
    int64_t submitted = 0, completed = 0, batches = 0, refused = 0, failed = 0, batched_requests = 0;
    double first_submit = -1, last_done = -1, particles_done = 0;
    size_t bytes_peak = 0;
};

class Core {
public:
    // lane_bytes(n): device bytes of a lane's batch workspace sized for batches of n particles.
    Core(size_t budget, int lanes, int max_batch, DeviceOps *ops, size_t (*lane_bytes)(int32_t))
        : budget_(budget), max_batch_(max_batch), ops_(ops), lane_bytes_(lane_bytes), lanes_((size_t)lanes) {}

    ~Core() {
        for (auto &kv : sessions_)
            for (Buffer &b : kv.second.bufs)
                if (b.mem) ops_->free(b.mem);
    }

    // Queue a request; QBVH_EAGAIN (counted as refused) if it can never fit.
    int submit(int32_t sim, int32_t n, int32_t max_nbr, double now, int64_t *ticket) {
        if (buffer_bytes(n, max_nbr) + lane_bytes_(n) > budget_) {
            ++st_.refused;
            return QBVH_EAGAIN;
        }
        Request q;
        q.ticket = next_ticket_++;
        q.sim = sim;
        q.n = n;
        q.max_nbr = max_nbr;
        q.t_submit = now;
        Ticket tk;
        tk.sim = sim;
        tk.n = n;
        tk.t_submit = now;
        tickets_[q.ticket] = tk;
        if (st_.first_submit < 0) st_.first_submit = now;
        ++st_.submitted;
        queue_.push_back(q);
        *ticket = q.ticket;
        return QBVH_OK;
    }

    bool queue_empty() const { return queue_.empty(); }
    bool lane_busy(int li) const { return lanes_[(size_t)li].busy; }
    bool any_busy() const {
        for (const Lane &l : lanes_)
            if (l.busy) return true;
        return false;
    }
    int lanes() const { return (int)lanes_.size(); }

    // Take every admissible queued request into idle lane `li` (in FIFO
    // order, at most max_batch).  Requests failed on the way (allocation
    // failure, or no progress possible) get their status set and are
    // reported in *failed.  The lane is marked busy when something was
    // admitted.
    std::vector<Admitted> admit(int li, double now, std::vector<int64_t> *failed) {
        std::vector<Admitted> out = scan(li, now, failed);
        if (out.empty() && !queue_.empty() && !any_busy()) {
            // nothing runs, so nothing will free memory: drop the lanes'
            // workspaces and try again; what still does not fit is held out
            // by leased buffers and fails
            for (size_t j = 0; j < lanes_.size(); ++j)
                if (lanes_[j].ws_cap > 0) {
                    ops_->release_lane((int)j);
                    lanes_[j].ws_cap = 0;
                }
            std::vector<int64_t> unfit;
            out = scan(li, now, failed, &unfit);
            if (out.empty()) {
                for (int64_t t : unfit) fail_queued(t, QBVH_EAGAIN, now, failed);
            }
        }
        if (!out.empty()) {
            lanes_[(size_t)li].busy = true;
            ++st_.batches;
            st_.batched_requests += (int64_t)out.size();
            st_.bytes_peak = std::max(st_.bytes_peak, bytes_buffers_ + lanes_total());
        }
        return out;
    }

    // The lane's batch finished with `status`; publishes its results.
    void complete(int li, int status, double now) {
        Lane &l = lanes_[(size_t)li];
        for (size_t i = 0; i < l.tickets.size(); ++i) {
            auto it = tickets_.find(l.tickets[i]);
            if (it != tickets_.end()) {
                it->second.status = status;
                it->second.t_done = now;
            }
            auto sit = sessions_.find(l.sims[i]);
            if (sit != sessions_.end()) {
                Session &ss = sit->second;
                ss.busy = false;
                if (status == QBVH_OK && ss.work >= 0) ss.pub = ss.work;
                ss.work = -1;
            }
            if (status == QBVH_OK) {
                ++st_.completed;
                const double lat = now - (it != tickets_.end() ? it->second.t_submit : now);
                if (lat_.size() < kLatencyWindow) lat_.push_back(lat);
                else lat_[lat_next_] = lat;
                lat_next_ = (lat_next_ + 1) % kLatencyWindow;
                st_.particles_done += it != tickets_.end() ? it->second.n : 0;
                st_.last_done = now;
            } else {
                ++st_.failed;
            }
        }
        l.tickets.clear();
        l.sims.clear();
        l.busy = false;
    }

    // Status of a ticket (kPending while queued or running); QBVH_EINVAL for
    // an unknown or already reported ticket.  A finished ticket is forgotten
    // when `forget` is set.
    int status(int64_t ticket, bool forget) {
        auto it = tickets_.find(ticket);
        if (it == tickets_.end()) return QBVH_EINVAL;
        const int s = it->second.status;
        if (s != kPending && forget) tickets_.erase(it);
        return s;
    }
    bool known(int64_t ticket) const { return tickets_.count(ticket) != 0; }

    // Lease the published buffer of a sim; *out receives a copy of its description.
    int lease(int32_t sim, Buffer *out) {
        auto it = sessions_.find(sim);
        if (it == sessions_.end() || it->second.pub < 0) return QBVH_EINVAL;
        Buffer &b = it->second.bufs[(size_t)it->second.pub];
        ++b.leases;
        *out = b;
        return QBVH_OK;
    }

    // Release one lease of the sim's buffer whose list starts at `nbr`.
    int release(int32_t sim, const int32_t *nbr) {
        auto it = sessions_.find(sim);
        if (it == sessions_.end()) return QBVH_EINVAL;
        for (Buffer &b : it->second.bufs)
            if (b.mem && b.nbr() == nbr && b.leases > 0) {
                --b.leases;
                return QBVH_OK;
            }
        return QBVH_EINVAL;
    }

    // Fail every queued request (the server is shutting down).
    void cancel_queued(int status, double now, std::vector<int64_t> *failed) {
        while (!queue_.empty()) fail_queued(queue_.front().ticket, status, now, failed);
    }

    const Stats &stats() const { return st_; }
    std::vector<double> latencies() const { return lat_; }
    size_t bytes_buffers() const { return bytes_buffers_; }
    size_t lanes_total() const {
        size_t b = 0;
        for (const Lane &l : lanes_) b += lane_bytes_(l.ws_cap);
        return b;
    }
    const std::map<int32_t, Session> &sessions() const { return sessions_; }
    int32_t lane_cap(int li) const { return lanes_[(size_t)li].ws_cap; }

private:
    void fail_queued(int64_t ticket, int status, double now, std::vector<int64_t> *failed) {
        for (auto it = queue_.begin(); it != queue_.end(); ++it) {
            if (it->ticket != ticket) continue;
            queue_.erase(it);
            auto tk = tickets_.find(ticket);
            if (tk != tickets_.end()) {
                tk->second.status = status;
                tk->second.t_done = now;
            }
            ++st_.failed;
            if (failed) failed->push_back(ticket);
            return;
        }
    }

    void free_buffer(Buffer &b) {
        if (b.mem) ops_->free(b.mem);
        bytes_buffers_ -= b.bytes;
        b = Buffer{};
    }

    // Free spare buffers, then (with `evict`) whole idle sessions without
    // leases, least recently used first and never a session in `keep`, until
    // `need` more bytes of buffers fit next to `lanes` bytes of workspaces.
    bool make_room(size_t need, size_t lanes, const std::set<int32_t> &keep, bool evict) {
        while (bytes_buffers_ + lanes + need > budget_) {
            // a spare buffer: not published, not being written, not leased
            int32_t vs = -1;
            int vb = -1;
            uint64_t oldest = UINT64_MAX;
            for (auto &kv : sessions_) {
                const Session &ss = kv.second;
                if (ss.busy || keep.count(kv.first) || ss.last_use >= oldest) continue;
                for (size_t k = 0; k < ss.bufs.size(); ++k) {
                    const Buffer &b = ss.bufs[k];
                    if (b.mem && (int)k != ss.pub && (int)k != ss.work && b.leases == 0) {
                        vs = kv.first;
                        vb = (int)k;
                        oldest = ss.last_use;
                        break;
                    }
                }
            }
            if (vs >= 0) {
                free_buffer(sessions_[vs].bufs[(size_t)vb]);
                continue;
            }
            if (!evict) return false;
            // a whole session
            oldest = UINT64_MAX;
            for (auto &kv : sessions_) {
                const Session &ss = kv.second;
                if (ss.busy || keep.count(kv.first) || ss.leased()) continue;
                if (ss.last_use < oldest) {
                    oldest = ss.last_use;
                    vs = kv.first;
                }
            }
            if (vs < 0) return false;
            for (Buffer &b : sessions_[vs].bufs) free_buffer(b);
            sessions_.erase(vs);
        }
        return true;
    }

    std::vector<Admitted> scan(int li, double now, std::vector<int64_t> *failed,
                               std::vector<int64_t> *unfit = nullptr) {
        Lane &l = lanes_[(size_t)li];
        std::vector<Admitted> out;
        std::set<int32_t> seen, taken;
        int64_t total = 0;
        size_t others = 0;
        for (size_t j = 0; j < lanes_.size(); ++j)
            if ((int)j != li) others += lane_bytes_(lanes_[j].ws_cap);
        for (auto it = queue_.begin(); it != queue_.end() && (int)out.size() < max_batch_;) {
            const Request r = *it;
            if (!seen.insert(r.sim).second) {  // an earlier request of this sim waits
                ++it;
                continue;
            }
            auto sit = sessions_.find(r.sim);
            if ((sit != sessions_.end() && sit->second.busy) || total + r.n > kMaxBatchParticles) {
                ++it;
                continue;
            }
            // The buffer to write, in order of preference: a spare one large
            // enough; a new one that fits after freeing spare buffers only
            // (replacing a spare that is too small, if there is one); the
            // published one, if no lease holds it and it is large enough (the
            // sim then has no published result until this request completes);
            // a new one after evicting idle sessions.
            int reuse = -1, replace = -1;
            bool pub_ok = false;
            if (sit != sessions_.end()) {
                const Session &ss = sit->second;
                for (size_t k = 0; k < ss.bufs.size(); ++k) {
                    const Buffer &b = ss.bufs[k];
                    if (!b.mem || b.leases > 0) continue;
                    const bool big = b.cap_n >= r.n && b.cap_nbr >= r.max_nbr;
                    if ((int)k == ss.pub) {
                        pub_ok = big;
                        continue;
                    }
                    if (big && reuse < 0) reuse = (int)k;
                    if (!big && replace < 0) replace = (int)k;
                }
            }
            const int32_t cap = (int32_t)std::max<int64_t>(l.ws_cap, total + r.n);
            const size_t lane_need = others + lane_bytes_(cap);
            std::set<int32_t> keep = taken;
            keep.insert(r.sim);
            const size_t new_bytes = buffer_bytes(r.n, r.max_nbr);
            const size_t freed = replace >= 0 ? sit->second.bufs[(size_t)replace].bytes : 0;
            const size_t need = new_bytes > freed ? new_bytes - freed : 0;
            int target = -1;
            bool alloc_new = false;
            if (reuse >= 0) {
                if (make_room(0, lane_need, keep, true)) target = reuse;
            } else if (make_room(need, lane_need, keep, false)) {
                alloc_new = true;
            } else if (pub_ok) {
                if (make_room(0, lane_need, keep, true)) target = sit->second.pub;
            } else if (make_room(need, lane_need, keep, true)) {
                alloc_new = true;
            }
            if (target < 0 && !alloc_new) {
                if (unfit) unfit->push_back(r.ticket);
                ++it;
                continue;
            }
            Session &ss = sessions_[r.sim];
            if (target >= 0 && target == ss.pub) ss.pub = -1;
            if (alloc_new) {
                if (replace >= 0) free_buffer(ss.bufs[(size_t)replace]);
                void *mem = ops_->alloc(new_bytes);
                if (!mem) {
                    if (ss.bufs.empty()) sessions_.erase(r.sim);
                    it = queue_.erase(it);
                    auto tk = tickets_.find(r.ticket);
                    if (tk != tickets_.end()) {
                        tk->second.status = QBVH_ENOMEM;
                        tk->second.t_done = now;
                    }
                    ++st_.failed;
                    if (failed) failed->push_back(r.ticket);
                    continue;
                }
                Buffer b;
                b.mem = mem;
                b.bytes = new_bytes;
                b.cap_n = r.n;
                b.cap_nbr = r.max_nbr;
                bytes_buffers_ += new_bytes;
                if (replace >= 0) {
                    ss.bufs[(size_t)replace] = b;
                    target = replace;
                } else {
                    // an emptied slot (freed spare) is reused before the vector grows
                    for (size_t k = 0; k < ss.bufs.size() && target < 0; ++k)
                        if (!ss.bufs[k].mem && (int)k != ss.pub) target = (int)k;
                    if (target >= 0) {
                        ss.bufs[(size_t)target] = b;
                    } else {
                        ss.bufs.push_back(b);
                        target = (int)ss.bufs.size() - 1;
                    }
                }
            }
            Buffer &b = ss.bufs[(size_t)target];
            b.res_n = r.n;
            b.res_nbr = r.max_nbr;
            ss.work = target;
            ss.busy = true;
            ss.last_use = ++clock_;
            out.push_back(Admitted{r.ticket, r.sim, b.nbr(), b.count(), b.overflow()});
            l.tickets.push_back(r.ticket);
            l.sims.push_back(r.sim);
            taken.insert(r.sim);
            total += r.n;
            l.ws_cap = cap;
            it = queue_.erase(it);
        }
        return out;
    }

    size_t budget_;
    int max_batch_;
    DeviceOps *ops_;
    size_t (*lane_bytes_)(int32_t);
    std::vector<Lane> lanes_;
    std::deque<Request> queue_;
    std::unordered_map<int64_t, Ticket> tickets_;
    std::map<int32_t, Session> sessions_;
    std::vector<double> lat_;
    size_t lat_next_ = 0;
    int64_t next_ticket_ = 1;
    uint64_t clock_ = 0;
    size_t bytes_buffers_ = 0;
    Stats st_;
};

}  // namespace srv
}  // namespace qbi

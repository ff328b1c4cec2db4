// CPU unit test of the server's admission and result-lifetime policy
// (paper_1901_08088_amd/csrc/server_core.h) with a fake device: allocations
// are host blocks filled with a pattern, so a write into a buffer that a
// lease protects, or a free of one, is detected.  Built with g++ by
// tests/test_server_core.py; exits non-zero with a message on failure.
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <set>
#include <vector>

#include "../paper_1901_08088_amd/csrc/server_core.h"

using namespace qbi::srv;

static int g_fail = 0;
#define CHECK(c)                                                          \
    do {                                                                  \
        if (!(c)) {                                                       \
            fprintf(stderr, "%s:%d: check failed: %s\n", __FILE__, __LINE__, #c); \
            g_fail = 1;                                                   \
            return;                                                       \
        }                                                                 \
    } while (0)

struct FakeOps final : DeviceOps {
    std::set<void *> live;
    std::vector<int> released;
    size_t fail_next_alloc = 0;  // fail allocations of this size once
    void *alloc(size_t bytes) override {
        if (fail_next_alloc && bytes == fail_next_alloc) {
            fail_next_alloc = 0;
            return nullptr;
        }
        void *p = malloc(bytes);
        live.insert(p);
        return p;
    }
    void free(void *p) override {
        if (!live.erase(p)) {
            fprintf(stderr, "free of a block that is not live\n");
            exit(3);
        }
        ::free(p);
    }
    void release_lane(int lane) override { released.push_back(lane); }
};

// A lane's workspace: 100 bytes per particle (a round figure for the tests).
static size_t lane100(int32_t n) { return (size_t)n * 100; }

// Simulate the device work of a batch: every admitted request writes its sim
// id into its buffer's first list entry.
static void run(const std::vector<Admitted> &a) {
    for (const Admitted &x : a) x.nbr[0] = x.sim;
}

static void test_publish_is_never_overwritten() {
    FakeOps ops;
    Core c(1 << 30, 1, 8, &ops, lane100);
    int64_t t1, t2, t3;
    CHECK(c.submit(7, 10, 4, 0.0, &t1) == QBVH_OK);
    std::vector<int64_t> failed;
    auto a = c.admit(0, 0.0, &failed);
    CHECK(a.size() == 1 && failed.empty());
    run(a);
    c.complete(0, QBVH_OK, 1.0);
    CHECK(c.status(t1, true) == QBVH_OK);
    CHECK(c.status(t1, true) == QBVH_EINVAL);  // forgotten once reported
    Buffer b;
    CHECK(c.lease(7, &b) == QBVH_OK);
    int32_t *leased = b.nbr();
    CHECK(leased[0] == 7);
    leased[0] = 1234;  // the reader's marker
    // the next request of the sim is admitted while the lease is held and
    // writes another buffer
    CHECK(c.submit(7, 10, 4, 2.0, &t2) == QBVH_OK);
    a = c.admit(0, 2.0, &failed);
    CHECK(a.size() == 1 && a[0].nbr != leased);
    run(a);
    c.complete(0, QBVH_OK, 3.0);
    CHECK(leased[0] == 1234);
    // the published result is now the new buffer; the old one stays leased
    Buffer b2;
    CHECK(c.lease(7, &b2) == QBVH_OK && b2.nbr() == a[0].nbr);
    // a third request cannot take either leased buffer: a third buffer
    CHECK(c.submit(7, 10, 4, 4.0, &t3) == QBVH_OK);
    auto a3 = c.admit(0, 4.0, &failed);
    CHECK(a3.size() == 1 && a3[0].nbr != leased && a3[0].nbr != b2.nbr());
    run(a3);
    c.complete(0, QBVH_OK, 5.0);
    CHECK(c.sessions().at(7).bufs.size() == 3);
    CHECK(c.release(7, leased) == QBVH_OK);
    CHECK(c.release(7, leased) == QBVH_EINVAL);  // only one lease was taken
    CHECK(c.release(7, b2.nbr()) == QBVH_OK);
    // once released, the old buffer is reused instead of a fourth one
    int64_t t4;
    CHECK(c.submit(7, 10, 4, 6.0, &t4) == QBVH_OK);
    auto a4 = c.admit(0, 6.0, &failed);
    CHECK(a4.size() == 1 && c.sessions().at(7).bufs.size() == 3);
    c.complete(0, QBVH_OK, 7.0);
}

static void test_eviction_spares_leased_and_busy() {
    FakeOps ops;
    const size_t one = buffer_bytes(100, 8);
    // room for three buffers and one lane of 100 particles
    Core c(3 * one + lane100(100), 1, 8, &ops, lane100);
    std::vector<int64_t> failed;
    int64_t t;
    for (int sim = 0; sim < 3; ++sim) {
        CHECK(c.submit(sim, 100, 8, sim, &t) == QBVH_OK);
        auto a = c.admit(0, sim, &failed);
        CHECK(a.size() == 1);
        run(a);
        c.complete(0, QBVH_OK, sim + 0.5);
        CHECK(c.status(t, true) == QBVH_OK);
    }
    Buffer b0;
    CHECK(c.lease(0, &b0) == QBVH_OK);  // sim 0 is the least recently used, but leased
    int32_t *p0 = b0.nbr();
    // a fourth sim needs room: sim 1 (least recently used without a lease) goes
    CHECK(c.submit(3, 100, 8, 10.0, &t) == QBVH_OK);
    auto a = c.admit(0, 10.0, &failed);
    CHECK(a.size() == 1);
    CHECK(c.sessions().count(0) == 1 && c.sessions().count(1) == 0 && c.sessions().count(2) == 1);
    CHECK(p0[0] == 0);
    Buffer bx;
    CHECK(c.lease(1, &bx) == QBVH_EINVAL);  // evicted: its result is gone
    c.complete(0, QBVH_OK, 11.0);
    CHECK(c.bytes_buffers() + c.lanes_total() <= 3 * one + lane100(100));
    CHECK(c.stats().bytes_peak <= 3 * one + lane100(100));
    CHECK(c.release(0, p0) == QBVH_OK);
}

static void test_lease_held_budget_fails_instead_of_hanging() {
    FakeOps ops;
    const size_t one = buffer_bytes(100, 8);
    Core c(one + buffer_bytes(50, 8) + lane100(100), 2, 8, &ops, lane100);
    std::vector<int64_t> failed;
    int64_t t;
    CHECK(c.submit(0, 100, 8, 0.0, &t) == QBVH_OK);
    auto a = c.admit(0, 0.0, &failed);
    CHECK(a.size() == 1);
    c.complete(0, QBVH_OK, 1.0);
    CHECK(c.status(t, true) == QBVH_OK);
    Buffer b;
    CHECK(c.lease(0, &b) == QBVH_OK);
    int32_t *p = b.nbr();
    // a second request of the same sim needs a second buffer of 100: it fits
    // the budget on its own (so it is accepted) but not next to the leased
    // buffer; nothing runs, so it fails instead of waiting forever
    CHECK(c.submit(0, 100, 8, 2.0, &t) == QBVH_OK);
    a = c.admit(1, 2.0, &failed);
    CHECK(a.empty());
    CHECK(failed.size() == 1 && failed[0] == t);
    CHECK(ops.released.size() == 1 && ops.released[0] == 0);  // lane 0's workspace was dropped first
    CHECK(c.status(t, true) == QBVH_EAGAIN);
    CHECK(c.queue_empty());
    // after the release the same request runs
    CHECK(c.release(0, p) == QBVH_OK);
    CHECK(c.submit(0, 100, 8, 3.0, &t) == QBVH_OK);
    a = c.admit(1, 3.0, &failed);
    CHECK(a.size() == 1);
    c.complete(1, QBVH_OK, 4.0);
    CHECK(c.status(t, true) == QBVH_OK);
}

static void test_grown_lane_does_not_block_forever() {
    // lane 0 grew for a large batch; later a request whose session is large
    // only fits once that idle lane's workspace is released
    FakeOps ops;
    const size_t budget = buffer_bytes(1000, 8) + lane100(1000) + 1000;
    Core c(budget, 2, 8, &ops, lane100);
    std::vector<int64_t> failed;
    int64_t t;
    CHECK(c.submit(0, 1000, 8, 0.0, &t) == QBVH_OK);
    auto a = c.admit(0, 0.0, &failed);
    CHECK(a.size() == 1 && c.lane_cap(0) == 1000);
    c.complete(0, QBVH_OK, 1.0);
    CHECK(c.status(t, true) == QBVH_OK);
    // sim 1 on lane 1: sim 0's session is evicted, but lane 0 still holds
    // 1000 particles of workspace, so lane 1 cannot get its own until lane 0
    // is released
    CHECK(c.submit(1, 900, 8, 2.0, &t) == QBVH_OK);
    a = c.admit(1, 2.0, &failed);
    CHECK(a.size() == 1 && failed.empty());
    CHECK(ops.released.size() == 1 && c.lane_cap(0) == 0);
    c.complete(1, QBVH_OK, 3.0);
    CHECK(c.status(t, true) == QBVH_OK);
}

static void test_refusal_order_and_batching() {
    FakeOps ops;
    Core c(buffer_bytes(100, 8) * 4 + lane100(300), 1, 2, &ops, lane100);
    int64_t t;
    CHECK(c.submit(0, 100000, 8, 0.0, &t) == QBVH_EAGAIN);  // can never fit
    CHECK(c.stats().refused == 1);
    int64_t a1, a2, b1, c1;
    CHECK(c.submit(0, 100, 8, 0.0, &a1) == QBVH_OK);
    CHECK(c.submit(0, 100, 8, 0.0, &a2) == QBVH_OK);  // same sim: waits for a1
    CHECK(c.submit(1, 100, 8, 0.0, &b1) == QBVH_OK);
    CHECK(c.submit(2, 100, 8, 0.0, &c1) == QBVH_OK);
    std::vector<int64_t> failed;
    auto a = c.admit(0, 0.0, &failed);  // max_batch 2: a1 and b1 (a2 waits for a1)
    CHECK(a.size() == 2 && a[0].ticket == a1 && a[1].ticket == b1);
    CHECK(c.status(a2, false) == kPending && c.status(c1, false) == kPending);
    c.complete(0, QBVH_OK, 1.0);
    a = c.admit(0, 1.0, &failed);
    CHECK(a.size() == 2 && a[0].ticket == a2 && a[1].ticket == c1);
    c.complete(0, QBVH_OK, 2.0);
    CHECK(c.stats().completed == 4 && c.stats().batches == 2);
}

static void test_allocation_failure_and_cancel() {
    FakeOps ops;
    Core c(1 << 30, 1, 8, &ops, lane100);
    int64_t t1, t2;
    CHECK(c.submit(0, 10, 4, 0.0, &t1) == QBVH_OK);
    CHECK(c.submit(1, 20, 4, 0.0, &t2) == QBVH_OK);
    ops.fail_next_alloc = buffer_bytes(10, 4);
    std::vector<int64_t> failed;
    auto a = c.admit(0, 0.0, &failed);
    CHECK(a.size() == 1 && a[0].ticket == t2 && failed.size() == 1 && failed[0] == t1);
    CHECK(c.status(t1, true) == QBVH_ENOMEM);
    CHECK(c.sessions().count(0) == 0);
    c.complete(0, QBVH_OK, 1.0);
    int64_t t3;
    CHECK(c.submit(5, 10, 4, 2.0, &t3) == QBVH_OK);
    failed.clear();
    c.cancel_queued(QBVH_EAGAIN, 2.0, &failed);
    CHECK(failed.size() == 1 && c.status(t3, true) == QBVH_EAGAIN && c.queue_empty());
}

static void test_latency_window_is_bounded() {
    FakeOps ops;
    Core c(1 << 30, 1, 1, &ops, lane100);
    std::vector<int64_t> failed;
    for (int k = 0; k < (int)kLatencyWindow + 100; ++k) {
        int64_t t;
        if (c.submit(k % 3, 4, 4, k, &t) != QBVH_OK) {
            CHECK(false);
        }
        auto a = c.admit(0, k, &failed);
        CHECK(a.size() == 1);
        c.complete(0, QBVH_OK, k + 0.25);
        CHECK(c.status(t, true) == QBVH_OK);
    }
    CHECK(c.latencies().size() == kLatencyWindow);
    CHECK(c.stats().completed == (int64_t)kLatencyWindow + 100);
}

int main() {
    test_publish_is_never_overwritten();
    test_eviction_spares_leased_and_busy();
    test_lease_held_budget_fails_instead_of_hanging();
    test_grown_lane_does_not_block_forever();
    test_refusal_order_and_batching();
    test_allocation_failure_and_cancel();
    test_latency_window_is_bounded();
    if (g_fail) return 1;
    printf("server core: all checks passed\n");
    return 0;
}

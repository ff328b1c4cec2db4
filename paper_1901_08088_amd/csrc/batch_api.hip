// C interface of the batched form: per-stream batch contexts, the launch plan
// of each batch shape, the autotuner and hipGraph capture and replay.
//
// A batch shape is the list of (n, ntypes) of its systems plus whether every
// system's rows take 16-byte stores.  Per shape the library keeps the
// autotuner's measurements and one captured graph per configuration tried.
// Everything that may change between calls of one shape (input and output
// pointers, boxes, cutoffs, row capacities) lives in a device table that the
// graph's kernels read, so a replay only needs the table re-uploaded when its
// bytes differ from the last upload.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <new>
#include <utility>
#include <vector>

#include "qbvh_internal.h"

namespace qbi {
namespace {

constexpr int32_t kBuildBlock = 256;  // work-items per build workgroup (kBuildThreads)
constexpr int kTrialsPerCandidate = 2;

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }
int32_t div_up(int64_t a, int64_t b) { return (int32_t)((a + b - 1) / b); }

struct Cfg {
    int32_t leaf, qbits, block;
    bool operator<(const Cfg &o) const {
        return leaf != o.leaf ? leaf < o.leaf : (qbits != o.qbits ? qbits < o.qbits : block < o.block);
    }
    bool operator==(const Cfg &o) const { return leaf == o.leaf && qbits == o.qbits && block == o.block; }
};

struct Pending {
    int cand;
    hipEvent_t a, b;
};

// Launch plan of one batch shape.
struct Plan {
    std::vector<Cfg> cands;
    std::vector<float> best;  // fastest measured call per candidate (ms)
    std::vector<int> runs;    // measurements per candidate
    std::vector<Pending> pending;
    int next = 0;
    bool frozen = false;
    Cfg chosen{};
    std::map<Cfg, hipGraphExec_t> graphs;
    int64_t calls = 0;
    int32_t graphs_captured = 0;
};

// Byte offsets of the device table for a capacity of `cap` systems.  The
// first `upload` bytes are written by the host; the rest by the device.
struct TabLayout {
    size_t sys_off, blk_first, tile_first, tblk_first, sysb, trav, upload, type_count, meta, bytes;
    explicit TabLayout(int32_t cap) {
        size_t p = 0;
        auto take = [&](size_t b) {
            const size_t r = p;
            p += align256(b);
            return r;
        };
        const size_t ints = (size_t)(cap + 1) * sizeof(int32_t);
        sys_off = take(ints);
        blk_first = take(ints);
        tile_first = take(ints);
        tblk_first = take(ints);
        sysb = take((size_t)cap * sizeof(SysBuild));
        trav = take((size_t)cap * sizeof(TravArgs));
        upload = p;
        type_count = take((size_t)cap * QBVH_MAX_TYPES * sizeof(uint32_t));
        meta = take((size_t)cap * QBVH_MAX_TYPES * sizeof(TreeMeta));
        bytes = p;
    }
};

struct BatchCtx {
    int device = 0;
    hipStream_t stream = nullptr;
    hipStream_t cap_stream = nullptr;  // graphs are captured here, launched on `stream`
    // device memory
    void *ws_base = nullptr;
    int32_t cap_total = -1;
    Workspace ws;
    void *aux = nullptr;  // sort counters + scan partials
    int32_t cap_tiles = -1;
    size_t cap_scan = 0;
    uint32_t *hist = nullptr, *scan_part = nullptr;
    void *tab = nullptr;
    int32_t cap_nsys = 0;
    // host staging of the table (pinned, two slots) and the bytes last uploaded
    void *htab[2] = {nullptr, nullptr};
    size_t htab_bytes = 0;
    hipEvent_t hev[2] = {nullptr, nullptr};
    bool hev_used[2] = {false, false};
    int slot = 0;
    std::vector<char> last;
    std::map<std::vector<int64_t>, Plan> plans;
    Plan *last_plan = nullptr;
    std::vector<hipEvent_t> spare;
};

std::mutex g_mu;
std::map<std::pair<int, hipStream_t>, BatchCtx *> g_ctx;

void drop_graphs(BatchCtx &c) {
    for (auto &kv : c.plans) {
        for (auto &g : kv.second.graphs) (void)hipGraphExecDestroy(g.second);
        kv.second.graphs.clear();
    }
}

hipError_t get_event(BatchCtx &c, hipEvent_t *ev) {
    if (!c.spare.empty()) {
        *ev = c.spare.back();
        c.spare.pop_back();
        return hipSuccess;
    }
    return hipEventCreate(ev);
}

// Fold finished measurements into the plan; with `wait`, block on all of them.
hipError_t poll(BatchCtx &c, Plan &p, bool wait) {
    size_t keep = 0;
    for (size_t i = 0; i < p.pending.size(); ++i) {
        Pending &q = p.pending[i];
        hipError_t e = wait ? hipEventSynchronize(q.b) : hipEventQuery(q.b);
        if (e == hipErrorNotReady) {
            p.pending[keep++] = q;
            continue;
        }
        if (e != hipSuccess) return e;
        float ms = 0.f;
        e = hipEventElapsedTime(&ms, q.a, q.b);
        if (e != hipSuccess) return e;
        if (ms < p.best[q.cand]) p.best[q.cand] = ms;
        ++p.runs[q.cand];
        c.spare.push_back(q.a);
        c.spare.push_back(q.b);
    }
    p.pending.resize(keep);
    if (!p.frozen) {
        bool done = true;
        for (int r : p.runs) done = done && r >= kTrialsPerCandidate;
        if (done) {
            size_t bi = 0;
            for (size_t i = 1; i < p.cands.size(); ++i)
                if (p.best[i] < p.best[bi]) bi = i;
            p.chosen = p.cands[bi];
            p.frozen = true;
            for (auto it = p.graphs.begin(); it != p.graphs.end();) {
                if (it->first == p.chosen) {
                    ++it;
                } else {
                    (void)hipGraphExecDestroy(it->second);
                    it = p.graphs.erase(it);
                }
            }
        }
    }
    return hipSuccess;
}

// Candidate configurations: every fixed option as given, the free ones over
// the values that matter on this hardware (leaf runs of 4, 8 and 16
// particles; workgroups of 64, 128 and 256; the paper's 10-bit grid and the
// full 16-bit one).
std::vector<Cfg> candidates(const qbvh_batch_opts_t &o) {
    std::vector<int32_t> leaves = o.leaf_size ? std::vector<int32_t>{o.leaf_size} : std::vector<int32_t>{4, 8, 16};
    std::vector<int32_t> bits = o.qbits ? std::vector<int32_t>{o.qbits} : std::vector<int32_t>{10, 16};
    std::vector<int32_t> blocks = o.block_size ? std::vector<int32_t>{o.block_size}
                                               : std::vector<int32_t>{64, 128, 256};
    std::vector<Cfg> r;
    for (int32_t l : leaves)
        for (int32_t q : bits)
            for (int32_t b : blocks) r.push_back(Cfg{l, q, b});
    return r;
}

hipError_t ensure_capacity(BatchCtx &c, int32_t total, int32_t tiles, int32_t nsys) {
    const size_t scan_len = (size_t)std::max<int64_t>((int64_t)total + 1, (int64_t)256 * tiles);
    const size_t scan_need = (size_t)scan_blocks((int32_t)scan_len) + 1;
    const bool grow_ws = c.ws_base == nullptr || total > c.cap_total;
    const bool grow_aux = c.aux == nullptr || tiles > c.cap_tiles || scan_need > c.cap_scan;
    const bool grow_tab = c.tab == nullptr || nsys > c.cap_nsys;
    if (!grow_ws && !grow_aux && !grow_tab) return hipSuccess;
    hipError_t e = hipStreamSynchronize(c.stream);
    if (e != hipSuccess) return e;
    drop_graphs(c);  // they hold the old addresses
    if (grow_ws) {
        if (c.ws_base) (void)hipFree(c.ws_base);
        c.ws_base = nullptr;
        const int32_t cap = std::max(total, 1);
        e = hipMalloc(&c.ws_base, workspace_bytes(cap));
        if (e != hipSuccess) {
            c.cap_total = -1;
            return e;
        }
        workspace_carve(c.ws, c.ws_base, cap);
        c.cap_total = cap;
    }
    if (grow_aux) {
        if (c.aux) (void)hipFree(c.aux);
        c.aux = nullptr;
        const int32_t t = std::max(tiles, std::max(c.cap_tiles, 1));
        const size_t hist_bytes = align256((size_t)256 * t * sizeof(uint32_t));
        const size_t sc = std::max(scan_need, c.cap_scan);
        e = hipMalloc(&c.aux, hist_bytes + sc * sizeof(uint32_t));
        if (e != hipSuccess) {
            c.cap_tiles = -1;
            c.cap_scan = 0;
            return e;
        }
        c.hist = (uint32_t *)c.aux;
        c.scan_part = (uint32_t *)((char *)c.aux + hist_bytes);
        c.cap_tiles = t;
        c.cap_scan = sc;
    }
    if (grow_tab) {
        if (c.tab) (void)hipFree(c.tab);
        c.tab = nullptr;
        for (int i = 0; i < 2; ++i) {
            if (c.htab[i]) (void)hipHostFree(c.htab[i]);
            c.htab[i] = nullptr;
            c.hev_used[i] = false;
        }
        const int32_t cap = std::max(nsys, 2 * c.cap_nsys);
        const TabLayout lay(cap);
        e = hipMalloc(&c.tab, lay.bytes);
        if (e != hipSuccess) {
            c.cap_nsys = 0;
            return e;
        }
        for (int i = 0; i < 2; ++i) {
            e = hipHostMalloc(&c.htab[i], lay.upload, hipHostMallocDefault);
            if (e != hipSuccess) {
                c.cap_nsys = 0;
                return e;
            }
        }
        c.htab_bytes = lay.upload;
        c.cap_nsys = cap;
        c.last.clear();
    }
    return hipSuccess;
}

hipError_t get_ctx(hipStream_t stream, BatchCtx **out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    auto key = std::make_pair(dev, stream);
    auto it = g_ctx.find(key);
    if (it != g_ctx.end()) {
        *out = it->second;
        return hipSuccess;
    }
    BatchCtx *c = new (std::nothrow) BatchCtx();
    if (!c) return hipErrorOutOfMemory;
    c->device = dev;
    c->stream = stream;
    e = hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&c->hev[0], hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&c->hev[1], hipEventDisableTiming);
    if (e != hipSuccess) {
        delete c;
        return e;
    }
    g_ctx[key] = c;
    *out = c;
    return hipSuccess;
}

void destroy_ctx(BatchCtx *c) {
    (void)hipStreamSynchronize(c->stream);
    drop_graphs(*c);
    for (auto &kv : c->plans)
        for (auto &q : kv.second.pending) {
            (void)hipEventDestroy(q.a);
            (void)hipEventDestroy(q.b);
        }
    for (hipEvent_t ev : c->spare) (void)hipEventDestroy(ev);
    for (int i = 0; i < 2; ++i) {
        if (c->hev[i]) (void)hipEventDestroy(c->hev[i]);
        if (c->htab[i]) (void)hipHostFree(c->htab[i]);
    }
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    if (c->ws_base) (void)hipFree(c->ws_base);
    if (c->aux) (void)hipFree(c->aux);
    if (c->tab) (void)hipFree(c->tab);
    delete c;
}

// Host image of the uploaded part of the table for configuration `cfg`.
void fill_table(const BatchCtx &c, int32_t nsys, const qbvh_system_t *sys, const std::vector<TravArgs> &trav,
                const Cfg &cfg, int32_t qpw, std::vector<char> &img) {
    const TabLayout lay(c.cap_nsys);
    img.assign(lay.upload, 0);
    int32_t *sys_off = (int32_t *)(img.data() + lay.sys_off);
    int32_t *blk = (int32_t *)(img.data() + lay.blk_first);
    int32_t *tile = (int32_t *)(img.data() + lay.tile_first);
    int32_t *tblk = (int32_t *)(img.data() + lay.tblk_first);
    SysBuild *sb = (SysBuild *)(img.data() + lay.sysb);
    TravArgs *ta = (TravArgs *)(img.data() + lay.trav);
    const TreeMeta *meta_dev = (const TreeMeta *)((const char *)c.tab + lay.meta);
    int32_t off = 0, b = 0, t = 0, tb = 0;
    for (int32_t s = 0; s < nsys; ++s) {
        const qbvh_system_t &y = sys[s];
        sys_off[s] = off;
        blk[s] = b;
        tile[s] = t;
        tblk[s] = tb;
        SysBuild &q = sb[s];
        q.pos = y.d_pos;
        q.type = y.ntypes > 1 ? y.d_type : nullptr;
        q.n = y.n;
        q.ntypes = y.ntypes;
        q.off = off;
        double lmax = 0.0;
        for (int d = 0; d < 3; ++d) {
            q.scale[d] = 1023.0 / (double)y.box[d];
            lmax = fmax(lmax, (double)y.box[d]);
        }
        q.ext_floor = lmax * 0x1p-24;
        TravArgs a = trav[s];
        a.records = c.ws.records;
        a.ropes = c.ws.ropes;
        a.sorted = c.ws.sorted;
        a.meta = meta_dev + (size_t)s * QBVH_MAX_TYPES;
        a.start = off;
        a.qpw = qpw;
        ta[s] = a;
        off += y.n;
        b += div_up(y.n, kBuildBlock);
        t += seg_radix_tiles(y.n);
        tb += (int32_t)trav_blocks(y.n, y.ntypes, cfg.block, qpw);
    }
    sys_off[nsys] = off;
    blk[nsys] = b;
    tile[nsys] = t;
    tblk[nsys] = tb;
}

hipError_t upload_table(BatchCtx &c, const std::vector<char> &img) {
    if (img == c.last) return hipSuccess;
    const int sl = c.slot;
    if (c.hev_used[sl]) {
        // this slot's previous copy must have left the staging buffer
        hipError_t e = hipEventSynchronize(c.hev[sl]);
        if (e != hipSuccess) return e;
    }
    memcpy(c.htab[sl], img.data(), img.size());
    hipError_t e = hipMemcpyAsync(c.tab, c.htab[sl], img.size(), hipMemcpyHostToDevice, c.stream);
    if (e != hipSuccess) return e;
    e = hipEventRecord(c.hev[sl], c.stream);
    if (e != hipSuccess) return e;
    c.hev_used[sl] = true;
    c.slot ^= 1;
    c.last = img;
    return hipSuccess;
}

BatchLaunch make_launch(const BatchCtx &c, int32_t nsys, int32_t total, int32_t tiles, int32_t blocks,
                        int32_t tblocks, const Cfg &cfg, bool vec4) {
    const TabLayout lay(c.cap_nsys);
    char *tab = (char *)c.tab;
    BatchLaunch b{};
    b.ws = c.ws;
    b.hist = c.hist;
    b.scan_part = c.scan_part;
    b.sys_off = (const int32_t *)(tab + lay.sys_off);
    b.blk_first = (const int32_t *)(tab + lay.blk_first);
    b.tile_first = (const int32_t *)(tab + lay.tile_first);
    b.tblk_first = (const int32_t *)(tab + lay.tblk_first);
    b.sysb = (const SysBuild *)(tab + lay.sysb);
    b.trav = (const TravArgs *)(tab + lay.trav);
    b.type_count = (uint32_t *)(tab + lay.type_count);
    b.meta = (TreeMeta *)(tab + lay.meta);
    b.nsys = nsys;
    b.total = total;
    b.blocks = blocks;
    b.tiles = tiles;
    b.tblocks = tblocks;
    b.leaf_size = cfg.leaf;
    b.qbits = cfg.qbits;
    b.block_size = cfg.block;
    b.vec4 = vec4;
    return b;
}

hipError_t capture(BatchCtx &c, const BatchLaunch &b, hipGraphExec_t *exec) {
    hipError_t e = hipStreamBeginCapture(c.cap_stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return e;
    hipError_t le = launch_batch(b, c.cap_stream);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(c.cap_stream, &g);
    if (le != hipSuccess || e != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return le != hipSuccess ? le : e;
    }
    e = hipGraphInstantiate(exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    return e;
}

int run_many(int32_t nsys, const qbvh_system_t *sys, const qbvh_batch_opts_t *opts, hipStream_t stream) {
    qbvh_batch_opts_t o{};
    if (opts) o = *opts;
    if ((o.leaf_size && !leaf_ok(o.leaf_size)) || (o.qbits && !qbits_ok(o.qbits)) ||
        (o.block_size && !block_ok(o.block_size)) || o.eager < 0 || o.eager > 1)
        return QBVH_EINVAL;
    const bool use_graph = o.eager == 0;

    std::vector<TravArgs> trav((size_t)nsys);
    std::vector<int64_t> key;
    key.reserve(2 + 2 * (size_t)nsys);
    int64_t total = 0, tiles = 0, blocks = 0;
    bool vec4 = true;
    for (int32_t s = 0; s < nsys; ++s) {
        const qbvh_system_t &y = sys[s];
        if (y.n < 0 || y.n > kMaxParticles || y.ntypes < 1 || y.ntypes > QBVH_MAX_TYPES || !box_ok(y.box) ||
            y.max_nbr < 0 || !y.d_overflow)
            return QBVH_EINVAL;
        if (y.n > 0 && (!y.d_pos || !y.d_count || (y.max_nbr > 0 && !y.d_nbr) || (y.ntypes > 1 && !y.d_type)))
            return QBVH_EINVAL;
        TravArgs &a = trav[(size_t)s];
        a = TravArgs{};
        int rc = list_radii(y.rcut, y.skin, y.ntypes, y.box, a.rlist2);
        if (rc != QBVH_OK) return rc;
        fill_trav_box(a, y.box);
        a.nbr = y.d_nbr;
        a.count = y.d_count;
        a.overflow = y.d_overflow;
        a.n = y.n;
        a.ntypes = y.ntypes;
        a.max_nbr = y.max_nbr;
        if (y.n > 0) vec4 = vec4 && y.max_nbr > 0 && (y.max_nbr % 4) == 0 && (((uintptr_t)y.d_nbr) & 15u) == 0;
        total += y.n;
        tiles += seg_radix_tiles(y.n);
        blocks += div_up(y.n, kBuildBlock);
        key.push_back(y.n);
        key.push_back(y.ntypes);
    }
    if (total > kMaxParticles) return QBVH_EINVAL;
    key.push_back(vec4 ? 1 : 0);

    std::lock_guard<std::mutex> lock(g_mu);
    BatchCtx *c = nullptr;
    hipError_t e = get_ctx(stream, &c);
    if (e != hipSuccess) return hip_fail(e);
    auto pit = c->plans.find(key);
    if (pit == c->plans.end()) {
        Plan p;
        p.cands = candidates(o);
        p.best.assign(p.cands.size(), INFINITY);
        p.runs.assign(p.cands.size(), 0);
        if (p.cands.size() == 1) {
            p.frozen = true;
            p.chosen = p.cands[0];
        }
        pit = c->plans.emplace(key, std::move(p)).first;
    }
    Plan &p = pit->second;
    c->last_plan = &p;
    ++p.calls;

    e = poll(*c, p, p.pending.size() > 4 * p.cands.size());
    if (e != hipSuccess) return hip_fail(e);
    const bool tuning = !p.frozen;
    int cand = -1;
    Cfg cfg = p.chosen;
    if (tuning) {
        cand = p.next;
        p.next = (p.next + 1) % (int)p.cands.size();
        cfg = p.cands[(size_t)cand];
    }

    e = ensure_capacity(*c, (int32_t)total, (int32_t)tiles, nsys);
    if (e != hipSuccess) return hip_fail(e);
    // queries per wavefront from the batch's total: a batch of many systems
    // fills the GPU with 64-query wavefronts, a small one gets smaller ones
    const int32_t qpw = queries_per_wave(total);
    int64_t tblocks = 0;
    for (int32_t s = 0; s < nsys; ++s) tblocks += trav_blocks(sys[s].n, sys[s].ntypes, cfg.block, qpw);
    std::vector<char> img;
    fill_table(*c, nsys, sys, trav, cfg, qpw, img);
    e = upload_table(*c, img);
    if (e != hipSuccess) return hip_fail(e);
    const BatchLaunch b =
        make_launch(*c, nsys, (int32_t)total, (int32_t)tiles, (int32_t)blocks, (int32_t)tblocks, cfg, vec4);

    Pending q{cand, nullptr, nullptr};
    if (tuning) {
        e = get_event(*c, &q.a);
        if (e == hipSuccess) e = get_event(*c, &q.b);
        if (e == hipSuccess) e = hipEventRecord(q.a, stream);
        if (e != hipSuccess) return hip_fail(e);
    }
    if (use_graph) {
        auto git = p.graphs.find(cfg);
        if (git == p.graphs.end()) {
            hipGraphExec_t ex = nullptr;
            e = capture(*c, b, &ex);
            if (e != hipSuccess) return hip_fail(e);
            git = p.graphs.emplace(cfg, ex).first;
            ++p.graphs_captured;
        }
        e = hipGraphLaunch(git->second, stream);
    } else {
        e = launch_batch(b, stream);
    }
    if (e != hipSuccess) return hip_fail(e);
    if (tuning) {
        e = hipEventRecord(q.b, stream);
        if (e != hipSuccess) return hip_fail(e);
        p.pending.push_back(q);
    }
    return QBVH_OK;
}

}  // namespace
}  // namespace qbi

extern "C" {

int nlist_build_many(int32_t nsys, const qbvh_system_t *sys, const qbvh_batch_opts_t *opts, qbvh_stream_t stream) {
    if (nsys < 0 || (nsys > 0 && !sys)) return QBVH_EINVAL;
    if (nsys == 0) return QBVH_OK;
    return qbi::run_many(nsys, sys, opts, (hipStream_t)stream);
}

int nlist_batch_stats(qbvh_stream_t stream, qbvh_batch_stats_t *out) {
    if (!out) return QBVH_EINVAL;
    memset(out, 0, sizeof(*out));
    std::lock_guard<std::mutex> lock(qbi::g_mu);
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return qbi::hip_fail(e);
    auto it = qbi::g_ctx.find(std::make_pair(dev, (hipStream_t)stream));
    if (it == qbi::g_ctx.end() || !it->second->last_plan) return QBVH_OK;
    qbi::BatchCtx &c = *it->second;
    qbi::Plan &p = *c.last_plan;
    e = qbi::poll(c, p, false);
    if (e != hipSuccess) return qbi::hip_fail(e);
    out->tuned = p.frozen ? 1 : 0;
    const qbi::Cfg cfg = p.frozen ? p.chosen : p.cands[0];
    out->leaf_size = cfg.leaf;
    out->qbits = cfg.qbits;
    out->block_size = cfg.block;
    out->candidates = (int32_t)p.cands.size();
    out->graphs_captured = p.graphs_captured;
    out->calls = p.calls;
    float best = INFINITY;
    for (size_t i = 0; i < p.cands.size(); ++i)
        if (p.cands[i] == cfg) best = p.best[i];
    out->best_ms = isfinite(best) ? best : 0.0f;
    return QBVH_OK;
}

void nlist_batch_release(qbvh_stream_t stream) {
    std::lock_guard<std::mutex> lock(qbi::g_mu);
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return;
    auto it = qbi::g_ctx.find(std::make_pair(dev, (hipStream_t)stream));
    if (it == qbi::g_ctx.end()) return;
    qbi::destroy_ctx(it->second);
    qbi::g_ctx.erase(it);
}

}  // extern "C"

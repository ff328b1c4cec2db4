// C interface of the qbvh library: argument checks, workspace ownership and
// launch sequencing.  All device work is in build.hip, sort.hip and
// traverse.hip; nothing here computes on the host beyond the per-call
// constants (list radii, box scale factors).
#include <algorithm>
#include <math.h>
#include <string.h>

#include <mutex>
#include <new>
#include <vector>

#include "qbvh_internal.h"

using qbi::TreeMeta;
using qbi::Workspace;

struct qbvh {
    Workspace ws;
    int32_t n = 0;
    int32_t ntypes = 1;
    float box[3] = {0.f, 0.f, 0.f};
    qbvh_opts_t opts{};
    hipStream_t stream = nullptr;
    // fp64 particle data (qbvh_build_f64): the box in fp64 and, in one extra
    // allocation for cap64 particles, the sorted fp64 positions (the exact
    // decisions)
    int32_t f64 = 0;
    double box64[3] = {0.0, 0.0, 0.0};
    void *mem64 = nullptr;
    int32_t cap64 = 0;
    double *sorted64 = nullptr;
};

namespace {

thread_local int g_last_hip_error = 0;

int resolve_opts(const qbvh_opts_t *in, qbvh_opts_t *out) {
    qbvh_opts_t o{};
    if (in) o = *in;
    if (o.leaf_size == 0) o.leaf_size = 16;
    if (o.qbits == 0) o.qbits = 16;
    if (o.block_size == 0) o.block_size = 64;
    if (!qbi::leaf_ok(o.leaf_size) || !qbi::qbits_ok(o.qbits) || !qbi::block_ok(o.block_size)) return QBVH_EINVAL;
    if (o.validate != 0 && o.validate != 1) return QBVH_EINVAL;
    if (!(isfinite(o.collapse_radius) && o.collapse_radius >= 0.0f && o.collapse_radius < 1e30f)) return QBVH_EINVAL;
    if (!qbi::qpw_ok(o.queries_per_wave)) return QBVH_EINVAL;
    *out = o;
    return QBVH_OK;
}

}  // namespace

namespace qbi {

int hip_fail(hipError_t e) {
    g_last_hip_error = (int)e;
    (void)hipGetLastError();  // clear the sticky launch error
    return e == hipErrorOutOfMemory ? QBVH_ENOMEM : QBVH_EHIP;
}

bool box_ok(const float box[3]) {
    if (!box) return false;
    for (int d = 0; d < 3; ++d)
        if (!(isfinite(box[d]) && box[d] > 0.0f)) return false;
    return true;
}

// (rc + skin)^2 in fp64 from the fp32 inputs; -1 marks a pair never listed.
int list_radii(const float *rcut, float skin, int32_t ntypes, const float box[3],
               double rlist2[QBVH_MAX_TYPES * QBVH_MAX_TYPES]) {
    const double b[3] = {(double)box[0], (double)box[1], (double)box[2]};
    return list_radii(rcut, skin, ntypes, b, rlist2);
}

int list_radii(const float *rcut, float skin, int32_t ntypes, const double box[3],
               double rlist2[QBVH_MAX_TYPES * QBVH_MAX_TYPES]) {
    if (!rcut || !(isfinite(skin) && skin >= 0.0f)) return QBVH_EINVAL;
    double rmax = 0.0;
    for (int a = 0; a < QBVH_MAX_TYPES * QBVH_MAX_TYPES; ++a) rlist2[a] = -1.0;
    for (int a = 0; a < ntypes; ++a) {
        for (int b = 0; b < ntypes; ++b) {
            const float rc = rcut[a * ntypes + b];
            if (isnan(rc) || rc != rcut[b * ntypes + a]) return QBVH_EINVAL;
            if (!isfinite(rc) && rc > 0) return QBVH_EINVAL;
            if (rc > 0.0f) {
                const double r = (double)rc + (double)skin;
                rlist2[a * QBVH_MAX_TYPES + b] = r * r;
                rmax = r > rmax ? r : rmax;
            }
        }
    }
    const double lmin = fmin(box[0], fmin(box[1], box[2]));
    if (!(2.0 * rmax * (1.0 + 1e-9) < lmin)) return QBVH_EGEOM;
    return QBVH_OK;
}

void fill_trav_box(TravArgs &a, const float box[3]) {
    const double b[3] = {(double)box[0], (double)box[1], (double)box[2]};
    fill_trav_box(a, b);
}

void fill_trav_box(TravArgs &a, const double box[3]) {
    for (int d = 0; d < 3; ++d) {
        a.L[d] = box[d];
        a.Lf[d] = (float)box[d];
    }
    a.lmax = fmax(a.L[0], fmax(a.L[1], a.L[2]));
}

}  // namespace qbi

using qbi::box_ok;
using qbi::hip_fail;
using qbi::kMaxParticles;
using qbi::list_radii;

extern "C" {

const char *qbvh_strerror(int code) {
    switch (code) {
    case QBVH_OK: return "ok";
    case QBVH_EINVAL: return "invalid argument";
    case QBVH_EGEOM: return "list radius too large for the box (minimum image not unique)";
    case QBVH_ENOMEM: return "out of device memory";
    case QBVH_EHIP: return "HIP runtime error";
    case QBVH_EAGAIN: return "request does not fit the server budget now";
    case QBVH_ENOTSUP: return "not supported";
    case QBVH_ENOSPACE: return "n needs more than the fixed no-allocation workspace (QBVH_NOALLOC_BYTES)";
    default: return "unknown error";
    }
}

int qbvh_last_hip_error(void) { return g_last_hip_error; }

size_t qbvh_workspace_bytes(int32_t n, int32_t ntypes, const qbvh_opts_t *opts) {
    qbvh_opts_t o;
    if (n < 0 || n > kMaxParticles || ntypes < 1 || ntypes > QBVH_MAX_TYPES || resolve_opts(opts, &o) != QBVH_OK)
        return 0;
    return qbi::workspace_bytes(n);
}

void qbvh_free(qbvh_t *tree) {
    if (!tree) return;
    if (tree->ws.base) (void)hipFree(tree->ws.base);
    if (tree->mem64) (void)hipFree(tree->mem64);
    delete tree;
}

}  // extern "C"

namespace {

// The tree of a build call: `*tree` itself, or a new one; its workspace is
// kept when it holds n particles, otherwise reallocated after both streams
// drain.  Returns QBVH_OK and the tree in *out (stored in *tree on success).
int prepare_tree(qbvh_t **tree, int32_t n, hipStream_t s, qbvh_t **out) {
    qbvh_t *t = *tree;
    const bool fresh = (t == nullptr);
    if (fresh) {
        t = new (std::nothrow) qbvh_t();
        if (!t) return QBVH_ENOMEM;
    }
    if (t->ws.base == nullptr || t->ws.cap < n) {
        if (t->ws.base) {
            hipError_t e = hipStreamSynchronize(t->stream);
            if (e == hipSuccess) e = hipStreamSynchronize(s);
            if (e != hipSuccess) {
                if (fresh) delete t;
                return hip_fail(e);
            }
            (void)hipFree(t->ws.base);
            t->ws = Workspace{};
        }
        const int32_t cap = n > 0 ? n : 1;
        void *base = nullptr;
        hipError_t e = hipMalloc(&base, qbi::workspace_bytes(cap));
        if (e != hipSuccess) {
            if (fresh) delete t;
            else t->ws = Workspace{};
            return hip_fail(e);
        }
        qbi::workspace_carve(t->ws, base, cap);
    }
    *out = t;
    *tree = t;
    return QBVH_OK;
}

// Waits for the build and reads the device-side validation word.
int check_valid(const int32_t *d_err, hipStream_t s) {
    int32_t err = 0;
    hipError_t e = hipMemcpyAsync(&err, d_err, sizeof(err), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e);
    return err ? QBVH_EINVAL : QBVH_OK;
}

// The traversal of a built workspace into the caller's outputs; `a` carries
// the list radii, the box and (fp64 data) the sorted fp64 positions.
int launch_list(const Workspace &w, int32_t n, int32_t ntypes, const qbvh_opts_t &o, qbi::TravArgs &a,
                int32_t max_nbr, int32_t mode, int32_t *d_nbr, int32_t *d_count, int32_t *d_overflow,
                hipStream_t s) {
    a.records = w.records;
    a.ropes = w.ropes;
    a.sorted = w.sorted;
    a.meta = w.meta;
    a.nbr = d_nbr;
    a.count = d_count;
    a.overflow = d_overflow;
    a.n = n;
    a.ntypes = ntypes;
    a.max_nbr = max_nbr;
    a.qpw = o.queries_per_wave ? o.queries_per_wave : qbi::queries_per_wave(n);
    a.qbits = o.qbits;
    const bool vec4 = max_nbr > 0 && (max_nbr % 4) == 0 && (((uintptr_t)d_nbr) & 15u) == 0;
    const bool paper = mode == QBVH_LIST_PAPER;
    hipError_t e = hipSuccess;
    if (paper) e = qbi::launch_qpoint(w, n, ntypes, o.qbits, a.lmax, s);
    if (e == hipSuccess) e = qbi::launch_traverse(a, o.block_size, vec4, paper, w.qpoint, s);
    if (e != hipSuccess) return hip_fail(e);
    return QBVH_OK;
}

}  // namespace

extern "C" {

int qbvh_build(qbvh_t **tree, const float *d_pos, const int32_t *d_type, int32_t n, int32_t ntypes,
               const float box[3], const qbvh_opts_t *opts, qbvh_stream_t stream) {
    if (!tree || n < 0 || n > kMaxParticles || ntypes < 1 || ntypes > QBVH_MAX_TYPES || !box_ok(box))
        return QBVH_EINVAL;
    if (n > 0 && !d_pos) return QBVH_EINVAL;
    if (n > 0 && ntypes > 1 && !d_type) return QBVH_EINVAL;
    qbvh_opts_t o;
    int rc = resolve_opts(opts, &o);
    if (rc != QBVH_OK) return rc;
    hipStream_t s = (hipStream_t)stream;
    qbvh_t *t = nullptr;
    rc = prepare_tree(tree, n, s, &t);
    if (rc != QBVH_OK) return rc;
    t->n = n;
    t->ntypes = ntypes;
    memcpy(t->box, box, sizeof(t->box));
    t->f64 = 0;
    t->opts = o;
    t->stream = s;

    hipError_t e = qbi::launch_build(t->ws, d_pos, ntypes > 1 ? d_type : nullptr, n, ntypes, box, o.leaf_size,
                                      o.qbits, o.collapse_radius, o.validate, s);
    if (e != hipSuccess) return hip_fail(e);
    return o.validate ? check_valid(t->ws.err, s) : QBVH_OK;
}

int qbvh_build_f64(qbvh_t **tree, const double *d_pos, const int32_t *d_type, int32_t n, int32_t ntypes,
                   const double box[3], const qbvh_opts_t *opts, qbvh_stream_t stream) {
    if (!tree || n < 0 || n > kMaxParticles || ntypes < 1 || ntypes > QBVH_MAX_TYPES || !box)
        return QBVH_EINVAL;
    for (int d = 0; d < 3; ++d)
        if (!(isfinite(box[d]) && box[d] > 0.0 && box[d] < 3.0e38)) return QBVH_EINVAL;
    if (n > 0 && !d_pos) return QBVH_EINVAL;
    if (n > 0 && ntypes > 1 && !d_type) return QBVH_EINVAL;
    qbvh_opts_t o;
    int rc = resolve_opts(opts, &o);
    if (rc != QBVH_OK) return rc;
    hipStream_t s = (hipStream_t)stream;
    qbvh_t *t = nullptr;
    rc = prepare_tree(tree, n, s, &t);
    if (rc != QBVH_OK) return rc;
    if (t->mem64 == nullptr || t->cap64 < n) {
        if (t->mem64) {
            hipError_t e = hipStreamSynchronize(t->stream);
            if (e == hipSuccess) e = hipStreamSynchronize(s);
            if (e != hipSuccess) return hip_fail(e);
            (void)hipFree(t->mem64);
            t->mem64 = nullptr;
            t->cap64 = 0;
        }
        const int32_t cap = n > 0 ? n : 1;
        void *m = nullptr;
        hipError_t e = hipMalloc(&m, (size_t)cap * 32);
        if (e != hipSuccess) return hip_fail(e);
        t->mem64 = m;
        t->cap64 = cap;
        t->sorted64 = (double *)m;
    }
    t->n = n;
    t->ntypes = ntypes;
    for (int d = 0; d < 3; ++d) {
        t->box64[d] = box[d];
        t->box[d] = (float)box[d];
    }
    t->f64 = 1;
    t->opts = o;
    t->stream = s;

    // the build runs on the data rounded to fp32 (a point may round onto the
    // box edge, which the Morton bins clamp); validation is done in fp64
    hipError_t e = qbi::launch_build(t->ws, nullptr, ntypes > 1 ? d_type : nullptr, n, ntypes, t->box, o.leaf_size,
                                     o.qbits, o.collapse_radius, o.validate, s, d_pos, t->sorted64, box);
    if (e != hipSuccess) return hip_fail(e);
    return o.validate ? check_valid(t->ws.err, s) : QBVH_OK;
}

int nlist_build_ex(const qbvh_t *tree, const float *rcut, float skin, int32_t max_nbr, int32_t mode,
                   int32_t *d_nbr, int32_t *d_count, int32_t *d_overflow, qbvh_stream_t stream) {
    if (!tree || max_nbr < 0 || !d_overflow) return QBVH_EINVAL;
    if (mode != QBVH_LIST_EXACT && mode != QBVH_LIST_PAPER) return QBVH_EINVAL;
    if (tree->n > 0 && (!d_count || (max_nbr > 0 && !d_nbr))) return QBVH_EINVAL;
    if (tree->f64 && mode == QBVH_LIST_PAPER) return QBVH_ENOTSUP;
    qbi::TravArgs a{};
    int rc = tree->f64 ? list_radii(rcut, skin, tree->ntypes, tree->box64, a.rlist2)
                       : list_radii(rcut, skin, tree->ntypes, tree->box, a.rlist2);
    if (rc != QBVH_OK) return rc;
    if (tree->f64) {
        qbi::fill_trav_box(a, tree->box64);
        a.sorted64 = tree->sorted64;
    } else {
        qbi::fill_trav_box(a, tree->box);
    }
    return launch_list(tree->ws, tree->n, tree->ntypes, tree->opts, a, max_nbr, mode, d_nbr, d_count, d_overflow,
                       (hipStream_t)stream);
}

int nlist_build(const qbvh_t *tree, const float *rcut, float skin, int32_t max_nbr, int32_t *d_nbr,
                int32_t *d_count, int32_t *d_overflow, qbvh_stream_t stream) {
    return nlist_build_ex(tree, rcut, skin, max_nbr, QBVH_LIST_EXACT, d_nbr, d_count, d_overflow, stream);
}

int qbvh_info(const qbvh_t *tree, qbvh_info_t *info) {
    if (!tree || !info) return QBVH_EINVAL;
    memset(info, 0, sizeof(*info));
    info->n = tree->n;
    info->ntypes = tree->ntypes;
    info->leaf_size = tree->opts.leaf_size;
    info->qbits = tree->opts.qbits;
    if (!tree->ws.base) return QBVH_OK;
    TreeMeta m[QBVH_MAX_TYPES];
    hipError_t e = hipStreamSynchronize(tree->stream);
    if (e == hipSuccess) e = hipMemcpy(m, tree->ws.meta, sizeof(TreeMeta) * tree->ntypes, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e);
    int32_t nrec = 0;
    for (int t = 0; t < tree->ntypes; ++t) {
        info->tree_start[t] = m[t].start;
        info->tree_count[t] = m[t].count;
        info->tree_root[t] = m[t].root;
        info->tree_end[t] = m[t].end;
        for (int d = 0; d < 3; ++d) {
            info->root_lo[t][d] = m[t].lo[d];
            info->root_hi[t][d] = m[t].hi[d];
        }
        info->h[t] = m[t].h;
        nrec = m[t].end > nrec ? m[t].end : nrec;
    }
    info->nrecords = tree->n > 0 ? nrec : 0;
    return QBVH_OK;
}

int qbvh_export(const qbvh_t *tree, int32_t what, void *d_dst, size_t dst_bytes, qbvh_stream_t stream) {
    if (!tree || !d_dst) return QBVH_EINVAL;
    const Workspace &w = tree->ws;
    const size_t n = (size_t)tree->n;
    const void *src = nullptr;
    size_t bytes = 0;
    switch (what) {
    case QBVH_EXPORT_KEYS: src = w.keys; bytes = n * 4; break;
    case QBVH_EXPORT_PERM: src = w.vals; bytes = n * 4; break;
    case QBVH_EXPORT_SORTED: src = w.sorted; bytes = n * 16; break;
    case QBVH_EXPORT_LEFT: src = w.left; bytes = n * 4; break;
    case QBVH_EXPORT_RIGHT: src = w.right; bytes = n * 4; break;
    case QBVH_EXPORT_RANGE_F: src = w.rf; bytes = n * 4; break;
    case QBVH_EXPORT_RANGE_L: src = w.rl; bytes = n * 4; break;
    case QBVH_EXPORT_PARENT: src = w.parent; bytes = n * 4; break;
    case QBVH_EXPORT_LEAF_PARENT: src = w.leaf_parent; bytes = n * 4; break;
    case QBVH_EXPORT_BOX_LO:
    case QBVH_EXPORT_BOX_HI: {
        // the bounds are stored interleaved (lower, upper per node): a strided copy
        const size_t rows = std::min(n, dst_bytes / 16);
        if (rows == 0 || !w.box) return QBVH_OK;
        hipError_t e = hipMemcpy2DAsync(d_dst, 16, w.box + (what == QBVH_EXPORT_BOX_HI ? 1 : 0), 32, 16, rows,
                                        hipMemcpyDeviceToDevice, (hipStream_t)stream);
        return e == hipSuccess ? QBVH_OK : hip_fail(e);
    }
    case QBVH_EXPORT_RECORDS: src = w.records; bytes = n * 32; break;
    case QBVH_EXPORT_ROPES: src = w.ropes; bytes = n * 4; break;
    default: return QBVH_EINVAL;
    }
    if (bytes > dst_bytes) bytes = dst_bytes;
    if (bytes == 0 || !src) return QBVH_OK;
    hipError_t e = hipMemcpyAsync(d_dst, src, bytes, hipMemcpyDeviceToDevice, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e);
    return QBVH_OK;
}

}  // extern "C"

// ------------------------------------------------------------ no allocation

// The build workspace of nlist_build_noalloc: a fixed array in the library's
// code object, so every GPU the library runs on holds one copy of it from the
// library's first use on that GPU until the process ends.  Host code never
// passes the name itself to the device (on the host it is only a stand-in);
// it uses the device address taken once per device below.
static __device__ __align__(256) unsigned char scratch[QBVH_NOALLOC_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device, looked up on the first
// call made with that device current.
int scratch_address(void **out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e);
    if (dev < 0 || dev >= kMaxDevices) return QBVH_ENOTSUP;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e);
        if (!ptr || (((uintptr_t)ptr) & 255u) != 0) return QBVH_EHIP;
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return QBVH_OK;
}

}  // namespace

extern "C" {

int nlist_build_noalloc(const float *d_pos, const int32_t *d_type, int32_t n, int32_t ntypes, const float box[3],
                        const qbvh_opts_t *opts, const float *rcut, float skin, int32_t max_nbr, int32_t *d_nbr,
                        int32_t *d_count, int32_t *d_overflow, qbvh_stream_t stream) {
    // the checks of qbvh_build, then those of nlist_build
    if (n < 0 || n > kMaxParticles || ntypes < 1 || ntypes > QBVH_MAX_TYPES || !box_ok(box)) return QBVH_EINVAL;
    if (n > 0 && !d_pos) return QBVH_EINVAL;
    if (n > 0 && ntypes > 1 && !d_type) return QBVH_EINVAL;
    qbvh_opts_t o;
    int rc = resolve_opts(opts, &o);
    if (rc != QBVH_OK) return rc;
    if (max_nbr < 0 || !d_overflow) return QBVH_EINVAL;
    if (n > 0 && (!d_count || (max_nbr > 0 && !d_nbr))) return QBVH_EINVAL;
    qbi::TravArgs a{};
    rc = list_radii(rcut, skin, ntypes, box, a.rlist2);
    if (rc != QBVH_OK) return rc;
    const int32_t cap = n > 0 ? n : 1;
    if (qbi::workspace_bytes(cap) > (size_t)QBVH_NOALLOC_BYTES) return QBVH_ENOSPACE;
    void *base = nullptr;
    rc = scratch_address(&base);
    if (rc != QBVH_OK) return rc;

    // every array the build reads is written by the build first (as for a
    // tree rebuilt in place), so what an earlier call left needs no clearing
    Workspace w;
    qbi::workspace_carve(w, base, cap);
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = qbi::launch_build(w, d_pos, ntypes > 1 ? d_type : nullptr, n, ntypes, box, o.leaf_size, o.qbits,
                                     o.collapse_radius, o.validate, s);
    if (e != hipSuccess) return hip_fail(e);
    if (o.validate) {
        rc = check_valid(w.err, s);
        if (rc != QBVH_OK) return rc;
    }
    qbi::fill_trav_box(a, box);
    return launch_list(w, n, ntypes, o, a, max_nbr, QBVH_LIST_EXACT, d_nbr, d_count, d_overflow, s);
}

}  // extern "C"

// Tree build: Morton codes, Z-order sort, Karras radix tree, bottom-up boxes,
// quantized rope-linked records (Section 2.1 and Section 2.2, Fig. 3).
//
// Records (32 bytes, depth-first preorder per type tree), one per internal
// node whose particle range is longer than `leaf_size`:
//   words 0-2: quantized box of the left child,  w_d = q_lo_d | (q_hi_d << 16)
//   words 3-5: quantized box of the right child, same packing
//   word 6/7:  left/right child: record index (>= 0) or the particle run
//              ~((first << 4) | (count - 1)) when the child holds at most
//              `leaf_size` particles
// plus ropes[v], the record after v's subtree.  The left child's record is
// the next record.  Storing both child boxes in the parent lets one step of
// the walk test two boxes, halving the chain of dependent node loads.
//
// Record positions come from one scan instead of a top-down walk.  With C[f]
// the number of kept nodes whose particle range starts at sorted position f
// and P its exclusive scan:
//   kept node [f, l] -> record P[f] + (number of its ancestors that share f)
//   rope of [f, l]   -> record P[l + 1]
// because in preorder the records before a node are the kept nodes starting
// before f and its ancestors starting at f.
#include "build_common.h"

namespace qbi {
namespace {

__device__ __forceinline__ Segment segment_of(uint32_t key, int32_t n, int32_t ntypes,
                                              const uint32_t *__restrict__ type_count) {
    if (ntypes == 1) return {0, n};
    const uint32_t t = key >> 30;
    int32_t s = 0;
    for (uint32_t u = 0; u < t; ++u) s += (int32_t)type_count[u];
    return {s, s + (int32_t)type_count[t]};
}

__global__ __launch_bounds__(kBuildThreads) void k_init(uint32_t *type_count, int32_t *err) {
    if (threadIdx.x < QBVH_MAX_TYPES) type_count[threadIdx.x] = 0;
    if (threadIdx.x == 0) *err = 0;
}

// Morton keys from fp32 or fp64 positions.  fp64 data: the bins are taken
// from each coordinate rounded to nearest fp32 (what the tree is built on)
// and the optional checks 0 <= x < L are made in fp64 against the fp64 box;
// fp32 data: L is the fp32 box (compared exactly after promotion).
template <class T>
__global__ __launch_bounds__(kBuildThreads) void k_morton(const T *__restrict__ pos,
                                                          const int32_t *__restrict__ type, int32_t n,
                                                          int32_t ntypes, double Lx, double Ly, double Lz,
                                                          double sx, double sy, double sz, int32_t validate,
                                                          uint32_t *__restrict__ keys,
                                                          uint32_t *__restrict__ kept, int32_t *err) {
    const int32_t k = blockIdx.x * kBuildThreads + threadIdx.x;
    // the kept counts of positions < n are written by the tree build; the
    // scan's extra entry is cleared here
    if (k == n) kept[n] = 0;
    if (k < n) {
        const T x = pos[3 * (int64_t)k + 0];
        const T y = pos[3 * (int64_t)k + 1];
        const T z = pos[3 * (int64_t)k + 2];
        int32_t t = type ? type[k] : 0;
        if (validate) {
            const bool ok = ((double)x >= 0.0 && (double)x < Lx) && ((double)y >= 0.0 && (double)y < Ly) &&
                            ((double)z >= 0.0 && (double)z < Lz) && (t >= 0 && t < ntypes);
            if (!ok) atomicOr(err, 1);
        }
        t = t < 0 ? 0 : (t >= ntypes ? ntypes - 1 : t);
        keys[k] = morton_key((float)x, (float)y, (float)z, sx, sy, sz, t);
    }
}

// Particles per type, read off the sorted keys (type in bits 30-31) by binary
// search: no atomics on a few hot counters.
__global__ void k_type_count(const uint32_t *__restrict__ keys, int32_t n, uint32_t *__restrict__ type_count) {
    const uint32_t t = threadIdx.x;
    if (t < QBVH_MAX_TYPES)
        type_count[t] = (uint32_t)(type_start(keys, 0, n, t + 1) - type_start(keys, 0, n, t));
}

// Radix tree and node boxes in one bottom-up pass (Section 2.1: the hierarchy
// over the Z-ordered particles, its boxes fit from the leaves up).  The tree
// is the binary radix tree of the augmented keys (key, position): the split
// between sorted positions k and k + 1 has the weight delta(k), the common
// prefix length of the two augmented keys (-1 where k and k + 1 lie in
// different type trees), and every node's range [l, r] is bounded by two
// splits of smaller weight than any inside it.  So a node's parent is found
// from its two bounding splits alone: the heavier one (they never tie) is the
// parent's split.  A node that is the left child of its parent's split ends
// at that split, r = split, and takes r as its id; a right child starts just
// after it and takes l; the root of a tree takes its first position.  These
// are the ids of Karras's top-down construction (an internal node's range has
// its id at one end), which the tree is node for node; here no node searches
// for its range: every leaf climbs, and at each parent split an exchange lets
// the first arrival leave its far end and stop while the second merges both
// children and goes on (the agglomerative order of Apetrei's construction).
//
// The climb is split by sorted position into chunks, so that an exchange and
// the child boxes it hands over are synchronized within one workgroup: a
// split's two children meet only in a chunk holding both its neighbours.  (An
// agent-scope acquire/release on gfx950 writes back and invalidates the XCD's
// L2 at every step, far too slow for N atomic steps.)  The first level takes
// chunks of kFitChunk positions with keys, split weights, particles, boxes and
// exchange slots in LDS; every further level multiplies the chunk by
// kFitFanout and climbs in global memory from the nodes the level before left
// at its chunk borders (the "frontier": finished nodes whose parent did not
// finish there).  The last level has one chunk and reaches every root.  The
// unfinished nodes of a chunk nest along its two borders (a radix tree over
// 32-bit keys plus 32-bit positions has at most 64 internal levels) and each
// has at most one finished child in the chunk, so kFrontierCap suffices.
constexpr int kFitChunk = 1024;
constexpr int kFitThreads = 1024;
// A small fanout keeps every level's climbs short (about five tree levels from
// each frontier node) and its workgroups many; N = 8M takes three level launches.
constexpr int kFitFanout = 32;
constexpr int kFrontierCap = 160;
static_assert(kFrontierCap >= 2 * (64 + 1), "fit frontier bound");
// A level's climbs stop at most once each on a first arrival.
constexpr int kPendCap = kFitFanout * kFrontierCap;
// Exchange slot states besides a far end (a sorted position, >= 0).
constexpr int32_t kSlotEmpty = -1;
constexpr int32_t kSlotDone = -2;

// Sorted position i's particle (x, y, z, bits of ~input index within its system).
__device__ __forceinline__ float4 gather_particle(const TreeSource &src, const uint32_t *__restrict__ vals, int32_t i) {
    const uint32_t o = vals[i];
    if (src.sysb == nullptr)
        return make_float4(src.pos[3 * (int64_t)o + 0], src.pos[3 * (int64_t)o + 1], src.pos[3 * (int64_t)o + 2],
                           __int_as_float(~(int32_t)o));
    const SysBuild &y = src.sysb[find_seg(src.sys_off, src.nsys, i)];
    const int32_t li = (int32_t)o - y.off;
    return make_float4(y.pos[3 * (int64_t)li + 0], y.pos[3 * (int64_t)li + 1], y.pos[3 * (int64_t)li + 2],
                       __int_as_float(~li));
}

// Weight of the split between sorted positions k and k + 1 (both < n) with
// keys ka and kb: -1 across a type or a system boundary, else the common
// prefix length of the augmented keys (equal keys differ in the position).
__device__ __forceinline__ int32_t split_delta(const TreeSource &src, int32_t k, uint32_t ka, uint32_t kb) {
    if ((ka ^ kb) >> 30) return -1;
    if (src.sysb != nullptr) {
        const int32_t s = find_seg(src.sys_off, src.nsys, k);
        if (k + 1 >= src.sys_off[s + 1]) return -1;
    }
    return ka != kb ? (int32_t)__clz(ka ^ kb) : 32 + (int32_t)__clz((uint32_t)(k ^ (k + 1)));
}

// What the climb writes: the tree's node arrays (by Karras id), the Z-ordered
// particles, the kept-node counts, and the split weights and exchange slots
// the upper levels use.
struct TreeOut {
    float4 *sorted;
    int32_t *left, *right, *rf, *rl, *parent, *leaf_parent;
    float4 *box;      // [n][2]: lower and upper bound of each node
    uint32_t *kept;   // kept[l] counts the nodes [l, r] longer than kept_leaf
    float *cost;      // cost model only
    int32_t *delta;   // [n]: delta[k] for k < n - 1, delta[n - 1] = -1
    int32_t *slot;    // [n]: exchange slot of each split
    int32_t kept_leaf;
};

// Everything about a finished internal node K = [l, r] with children cl, cr.
template <bool kCost>
__device__ __forceinline__ void write_node(const TreeOut &o, int32_t K, int32_t l, int32_t r, int32_t cl, int32_t cr,
                                           const float lo[3], const float hi[3], float cst) {
    o.rf[K] = l;
    o.rl[K] = r;
    o.left[K] = cl;
    o.right[K] = cr;
    o.box[2 * (int64_t)K] = make_float4(lo[0], lo[1], lo[2], 0.0f);
    o.box[2 * (int64_t)K + 1] = make_float4(hi[0], hi[1], hi[2], 0.0f);
    if (kCost) o.cost[K] = cst;
    if (cl < 0) o.leaf_parent[~cl] = K; else o.parent[cl] = K;
    if (cr < 0) o.leaf_parent[~cr] = K; else o.parent[cr] = K;
    if (r - l + 1 > o.kept_leaf) atomicAdd(&o.kept[l], 1u);
}

__device__ __forceinline__ void frontier_push(int32_t c, uint32_t *s_fcount, int32_t *s_front, int32_t *err) {
    const uint32_t slot = atomicAdd(s_fcount, 1u);
    if (slot < (uint32_t)kFrontierCap)
        s_front[slot] = c;
    else
        atomicOr(err, 2);
}

// The child of split g whose far end is e: the left child [e, g] or the right
// child [g + 1, e], as a node id or a leaf (~position).
__device__ __forceinline__ int32_t child_at(int32_t g, int32_t e) {
    return e <= g ? (e == g ? ~g : g) : (e == g + 1 ? ~(g + 1) : g + 1);
}

// A node of the climb: range, bounding split weights, box, cost and children.
struct Climb {
    int32_t l, r, dl, dr, cl, cr;
    float lo[3], hi[3];
    float cost;
};

// First level: one chunk of kFitChunk sorted positions per workgroup; also
// gathers the chunk's particles in Z order and leaves its split weights and
// cleared exchange slots for the upper levels.  A node finished here has its
// id, range and children inside the chunk, so everything written about it
// (its range, split and box, its children's parent, the kept counts) is
// collected in LDS and written out at the end with coalesced stores.
constexpr int32_t kUnset = INT32_MIN;

template <bool kCost>
__global__ __launch_bounds__(kFitThreads) void k_tree_local(const uint32_t *__restrict__ keys,
                                                            const uint32_t *__restrict__ vals, int32_t n,
                                                            TreeSource src, TreeOut out, int32_t *__restrict__ front,
                                                            uint32_t *__restrict__ fcount, int32_t *err,
                                                            Collapse col) {
    __shared__ uint32_t s_keykept[kFitChunk + 2];  // keys c0 - 1 .. c0 + m, then kept counts by l - c0
    __shared__ int32_t s_delta[kFitChunk + 1];     // s_delta[j]: weight of split c0 - 1 + j
    __shared__ float s_pos[3][kFitChunk];
    __shared__ float s_box[6][kFitChunk];          // nodes by id - c0
    __shared__ float s_cost[kCost ? kFitChunk : 1];
    __shared__ int32_t s_nl[kFitChunk], s_nr[kFitChunk], s_ng[kFitChunk];  // range and split (s_nr < 0: none)
    __shared__ int32_t s_par[kFitChunk], s_lpar[kFitChunk];  // parent of node / leaf c0 + i
    __shared__ int32_t s_slot[kFitChunk];          // by split - c0
    __shared__ int32_t s_front[kFrontierCap];
    __shared__ uint32_t s_fcount;
    const int32_t c0 = blockIdx.x * kFitChunk;
    const int32_t m = min(kFitChunk, n - c0);
    const int32_t t = threadIdx.x;
    // the particle's loads go out first and complete while the keys are staged
    float4 p = make_float4(0.f, 0.f, 0.f, 0.f);
    if (t < m) {
        if (src.pos64 != nullptr) {
            // fp64 data: the particle rounded to fp32 for the tree (as the
            // Morton codes were), its fp64 position kept in Z order as well
            const uint32_t o = vals[c0 + t];
            const double x = src.pos64[3 * (int64_t)o + 0], y = src.pos64[3 * (int64_t)o + 1],
                         z = src.pos64[3 * (int64_t)o + 2];
            p = make_float4((float)x, (float)y, (float)z, __int_as_float(~(int32_t)o));
            double *q = src.sorted64 + 4 * (int64_t)(c0 + t);
            q[0] = x;
            q[1] = y;
            q[2] = z;
            q[3] = 0.0;
        } else {
            p = gather_particle(src, vals, c0 + t);
        }
    }
    for (int32_t j = t; j < m + 2; j += kFitThreads) {
        const int32_t k = c0 - 1 + j;
        s_keykept[j] = (k >= 0 && k < n) ? keys[k] : 0u;
    }
    if (t < m) {
        out.sorted[c0 + t] = p;
        s_pos[0][t] = p.x;
        s_pos[1][t] = p.y;
        s_pos[2][t] = p.z;
        s_slot[t] = kSlotEmpty;
        s_nr[t] = -1;
        s_par[t] = kUnset;
        s_lpar[t] = kUnset;
        out.slot[c0 + t] = kSlotEmpty;
    }
    if (t == 0) s_fcount = 0;
    __syncthreads();
    for (int32_t j = t; j <= m; j += kFitThreads) {
        const int32_t k = c0 - 1 + j;
        const int32_t d = (k < 0 || k + 1 >= n) ? -1 : split_delta(src, k, s_keykept[j], s_keykept[j + 1]);
        s_delta[j] = d;
        if (k >= c0) out.delta[k] = d;  // this chunk's splits c0 .. c0 + m - 1
    }
    __syncthreads();
    if (t < m) s_keykept[t] = 0u;
    __syncthreads();
    if (t < m) {
        Climb u;
        u.l = u.r = c0 + t;
        u.dl = s_delta[t];
        u.dr = s_delta[t + 1];
        u.cl = u.cr = 0;
        u.lo[0] = u.hi[0] = p.x;
        u.lo[1] = u.hi[1] = p.y;
        u.lo[2] = u.hi[2] = p.z;
        u.cost = col.kVball;
        int32_t split = 0;  // the split of the node being carried (internal nodes)
        for (int step = 0; step < kMaxDepth; ++step) {
            const bool leaf = u.l == u.r;
            const bool root = u.dl < 0 && u.dr < 0;
            const bool goes_left = u.dr > u.dl;  // the parent's split is r: this node is its left child
            const int32_t K = leaf ? ~u.l : (goes_left && !root ? u.r : u.l);
            if (!leaf) {
                const int32_t k = K - c0;
                s_nl[k] = u.l;
                s_nr[k] = u.r;
                s_ng[k] = split;
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    s_box[d][k] = u.lo[d];
                    s_box[3 + d][k] = u.hi[d];
                }
                if (kCost) s_cost[k] = u.cost;
                if (u.cl < 0) s_lpar[~u.cl - c0] = K; else s_par[u.cl - c0] = K;
                if (u.cr < 0) s_lpar[~u.cr - c0] = K; else s_par[u.cr - c0] = K;
                if (u.r - u.l + 1 > out.kept_leaf) atomicAdd(&s_keykept[u.l - c0], 1u);
            }
            if (root) {
                if (leaf) s_lpar[u.l - c0] = -1; else s_par[K - c0] = -1;
                break;
            }
            const int32_t g = goes_left ? u.r : u.l - 1;
            if (g < c0 || g >= c0 + m - 1) {  // a split on or past the chunk's border
                frontier_push(K, &s_fcount, s_front, err);
                break;
            }
            const int32_t e = __hip_atomic_exchange(&s_slot[g - c0], goes_left ? u.l : u.r, __ATOMIC_ACQ_REL,
                                                    __HIP_MEMORY_SCOPE_WORKGROUP);
            if (e == kSlotEmpty) break;  // the sibling finishes the parent
            s_slot[g - c0] = kSlotDone;
            const int32_t sib = child_at(g, e);
            float slo[3], shi[3], scost;
            if (sib < 0) {
#pragma unroll
                for (int d = 0; d < 3; ++d) slo[d] = shi[d] = s_pos[d][~sib - c0];
                scost = col.kVball;
            } else {
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    slo[d] = s_box[d][sib - c0];
                    shi[d] = s_box[3 + d][sib - c0];
                }
                scost = kCost ? fabsf(s_cost[sib - c0]) : 0.0f;
            }
            const float own = fabsf(u.cost);
            if (goes_left) {
                u.r = e;
                u.dr = s_delta[e - c0 + 1];
                u.cl = K;
                u.cr = sib;
            } else {
                u.l = e;
                u.dl = s_delta[e - c0];
                u.cl = sib;
                u.cr = K;
            }
            split = g;
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                u.lo[d] = fminf(u.lo[d], slo[d]);
                u.hi[d] = fmaxf(u.hi[d], shi[d]);
            }
            if (kCost)
                u.cost = node_cost(col, u.r - u.l + 1, u.lo[0], u.lo[1], u.lo[2], u.hi[0], u.hi[1], u.hi[2],
                                   goes_left ? own : scost, goes_left ? scost : own);
        }
    }
    __syncthreads();
    // first arrivals whose sibling never came: their parent straddles a border
    for (int32_t j = t; j < m - 1; j += kFitThreads) {
        const int32_t e = s_slot[j];
        if (e >= 0) frontier_push(child_at(c0 + j, e), &s_fcount, s_front, err);
    }
    if (t < m) {
        const int32_t K = c0 + t;
        const int32_t r = s_nr[t];
        if (r >= 0) {
            const int32_t l = s_nl[t], g = s_ng[t];
            out.rf[K] = l;
            out.rl[K] = r;
            out.left[K] = g == l ? ~l : g;
            out.right[K] = g + 1 == r ? ~r : g + 1;
            out.box[2 * (int64_t)K] = make_float4(s_box[0][t], s_box[1][t], s_box[2][t], 0.0f);
            out.box[2 * (int64_t)K + 1] = make_float4(s_box[3][t], s_box[4][t], s_box[5][t], 0.0f);
            if (kCost) out.cost[K] = s_cost[t];
        }
        if (s_par[t] != kUnset) out.parent[K] = s_par[t];
        if (s_lpar[t] != kUnset) out.leaf_parent[K] = s_lpar[t];
        out.kept[K] = s_keykept[t];  // the chunk's own nodes are the only ones starting here so far
    }
    __syncthreads();
    const uint32_t fc = min(s_fcount, (uint32_t)kFrontierCap);
    for (uint32_t i = t; i < fc; i += kFitThreads) front[(int64_t)blockIdx.x * kFrontierCap + i] = s_front[i];
    if (t == 0) fcount[blockIdx.x] = fc;
}

// One level above the first: chunks of `chunk` positions, climbing from the
// frontiers of the `fan` previous-level chunks each contains, with the
// exchange slots in global memory (workgroup-scope atomics: a split's two
// children meet in one chunk).  A step waits for two round trips: the
// exchange, then the sibling's box with the new bounding weight.
template <bool kCost>
__global__ __launch_bounds__(kFitThreads) void k_tree_level(int32_t n, int64_t chunk, int32_t nprev,
                                                            const int32_t *__restrict__ front_in,
                                                            const uint32_t *__restrict__ fcount_in, TreeOut out,
                                                            int32_t *__restrict__ front_out,
                                                            uint32_t *__restrict__ fcount_out, int32_t *err,
                                                            Collapse col) {
    __shared__ int32_t s_front[kFrontierCap];
    __shared__ uint32_t s_fcount;
    __shared__ uint32_t s_off[kFitFanout + 1];
    __shared__ int32_t s_pend[kPendCap];  // splits where a climb stopped as the first arrival
    __shared__ uint32_t s_npend;
    const int64_t c0 = (int64_t)blockIdx.x * chunk;
    const int64_t c1 = min(c0 + chunk, (int64_t)n);
    const int32_t j0 = blockIdx.x * kFitFanout;
    // The frontier entries of the fan-in chunks, numbered consecutively, so
    // that each thread climbs from at most a few of them.
    if (threadIdx.x < kFitFanout) {
        const int32_t jc = j0 + (int32_t)threadIdx.x;
        s_off[threadIdx.x + 1] = jc < nprev ? min(fcount_in[jc], (uint32_t)kFrontierCap) : 0u;
    }
    if (threadIdx.x == 0) {
        s_fcount = 0;
        s_npend = 0;
        s_off[0] = 0;
    }
    __syncthreads();
    if (threadIdx.x == 0)
        for (int k = 1; k <= kFitFanout; ++k) s_off[k] += s_off[k - 1];
    __syncthreads();
    const uint32_t total = s_off[kFitFanout];
    for (uint32_t e = threadIdx.x; e < total; e += kFitThreads) {
        // the chunk k holding entry e: s_off[k] <= e < s_off[k + 1]
        int lo = 0, hi = kFitFanout;
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (s_off[mid] <= e) lo = mid; else hi = mid;
        }
        const int32_t c = front_in[(int64_t)(j0 + lo) * kFrontierCap + (e - s_off[lo])];
        // the entry was written when its parent's split was found: restart there
        Climb u;
        u.cl = u.cr = 0;
        if (c < 0) {
            u.l = u.r = ~c;
            const float4 q = out.sorted[~c];
            u.lo[0] = u.hi[0] = q.x;
            u.lo[1] = u.hi[1] = q.y;
            u.lo[2] = u.hi[2] = q.z;
            u.cost = col.kVball;
        } else {
            u.l = out.rf[c];
            u.r = out.rl[c];
            const float4 a = out.box[2 * (int64_t)c], b = out.box[2 * (int64_t)c + 1];
            u.lo[0] = a.x; u.lo[1] = a.y; u.lo[2] = a.z;
            u.hi[0] = b.x; u.hi[1] = b.y; u.hi[2] = b.z;
            u.cost = kCost ? out.cost[c] : 0.0f;
        }
        u.dl = u.l > 0 ? out.delta[u.l - 1] : -1;
        u.dr = out.delta[u.r];
        bool fresh = false;
        for (int step = 0; step < kMaxDepth; ++step) {
            const bool leaf = u.l == u.r;
            const bool root = u.dl < 0 && u.dr < 0;
            const bool goes_left = u.dr > u.dl;
            const int32_t K = leaf ? ~u.l : (goes_left && !root ? u.r : u.l);
            if (fresh) write_node<kCost>(out, K, u.l, u.r, u.cl, u.cr, u.lo, u.hi, u.cost);
            if (root) {
                out.parent[K] = -1;  // (a climb reaches a root only through a merge)
                break;
            }
            const int32_t g = goes_left ? u.r : u.l - 1;
            if (g < c0 || g >= c1 - 1) {
                frontier_push(K, &s_fcount, s_front, err);
                break;
            }
            const int32_t ex = __hip_atomic_exchange(&out.slot[g], goes_left ? u.l : u.r, __ATOMIC_ACQ_REL,
                                                     __HIP_MEMORY_SCOPE_WORKGROUP);
            if (ex == kSlotEmpty) {
                const uint32_t at = atomicAdd(&s_npend, 1u);
                if (at < (uint32_t)kPendCap) s_pend[at] = g; else atomicOr(err, 2);
                break;
            }
            out.slot[g] = kSlotDone;
            const int32_t sib = child_at(g, ex);
            // the sibling's box and cost and the new far weight, loaded together
            const float4 *pa = sib < 0 ? out.sorted + ~sib : out.box + 2 * (int64_t)sib;
            const float4 *pb = sib < 0 ? out.sorted + ~sib : out.box + 2 * (int64_t)sib + 1;
            const float4 slo = *pa, shi = *pb;
            const float scost = kCost ? (sib < 0 ? col.kVball : fabsf(out.cost[sib])) : 0.0f;
            const int32_t dnew = goes_left ? out.delta[ex] : (ex > 0 ? out.delta[ex - 1] : -1);
            const float own = fabsf(u.cost);
            if (goes_left) {
                u.r = ex;
                u.dr = dnew;
                u.cl = K;
                u.cr = sib;
            } else {
                u.l = ex;
                u.dl = dnew;
                u.cl = sib;
                u.cr = K;
            }
            u.lo[0] = fminf(u.lo[0], slo.x);
            u.lo[1] = fminf(u.lo[1], slo.y);
            u.lo[2] = fminf(u.lo[2], slo.z);
            u.hi[0] = fmaxf(u.hi[0], shi.x);
            u.hi[1] = fmaxf(u.hi[1], shi.y);
            u.hi[2] = fmaxf(u.hi[2], shi.z);
            if (kCost)
                u.cost = node_cost(col, u.r - u.l + 1, u.lo[0], u.lo[1], u.lo[2], u.hi[0], u.hi[1], u.hi[2],
                                   goes_left ? own : scost, goes_left ? scost : own);
            fresh = true;
        }
    }
    __syncthreads();
    // first arrivals whose sibling never came go to the next level, with their
    // slots cleared for it
    const uint32_t np = min(s_npend, (uint32_t)kPendCap);
    for (uint32_t j = threadIdx.x; j < np; j += kFitThreads) {
        const int32_t g = s_pend[j];
        const int32_t ex = out.slot[g];
        if (ex >= 0) frontier_push(child_at(g, ex), &s_fcount, s_front, err);
        out.slot[g] = kSlotEmpty;
    }
    __syncthreads();
    const uint32_t fc = min(s_fcount, (uint32_t)kFrontierCap);
    for (uint32_t i = threadIdx.x; i < fc; i += kFitThreads) front_out[(int64_t)blockIdx.x * kFrontierCap + i] = s_front[i];
    if (threadIdx.x == 0) fcount_out[blockIdx.x] = fc;
}

// Root box, grid spacing and slot range of each type's tree.
__global__ void k_meta(int32_t n, int32_t ntypes, const uint32_t *__restrict__ type_count,
                       const float4 *__restrict__ sorted, const float4 *__restrict__ box,
                       const uint32_t *__restrict__ P, int32_t qbits,
                       int32_t leaf_size, const float *__restrict__ cost, double ext_floor,
                       TreeMeta *__restrict__ meta) {
    const int t = threadIdx.x;
    if (t >= ntypes) return;
    int32_t s = 0;
    for (int u = 0; u < t; ++u) s += (int32_t)type_count[u];
    const int32_t c = (ntypes == 1) ? n : (int32_t)type_count[t];
    float lo[3] = {0.f, 0.f, 0.f}, hi[3] = {0.f, 0.f, 0.f};
    if (c == 1) {
        const float4 p = sorted[s];
        lo[0] = hi[0] = p.x;
        lo[1] = hi[1] = p.y;
        lo[2] = hi[2] = p.z;
    } else if (c >= 2) {
        const float4 a = box[2 * (int64_t)s], b = box[2 * (int64_t)s + 1];
        lo[0] = a.x; lo[1] = a.y; lo[2] = a.z;
        hi[0] = b.x; hi[1] = b.y; hi[2] = b.z;
    }
    // the root (internal node s) is a run when its subtree was collapsed
    const bool root_run = cost ? (c < 2 || cost[s] < 0.0f) : c <= leaf_size;
    meta[t] = tree_meta(lo, hi, ext_floor, qbits, s, c, root_run, P);
}

// With the cost model: which internal nodes keep a record.  A node keeps one
// unless it or an ancestor became a run (only nodes of at most leaf_size
// particles can); kept_flag[i] records it for the emit, and kept[f] counts the
// kept nodes whose range starts at f (the layout's scan).
__global__ __launch_bounds__(kBuildThreads) void k_kept_collapse(int32_t n, int32_t ntypes,
                                                                 const uint32_t *__restrict__ keys,
                                                                 const uint32_t *__restrict__ type_count,
                                                                 const int32_t *__restrict__ rf,
                                                                 const int32_t *__restrict__ rl,
                                                                 const int32_t *__restrict__ parent,
                                                                 const float *__restrict__ cost, int32_t leaf_size,
                                                                 uint32_t *__restrict__ kept_flag,
                                                                 uint32_t *__restrict__ kept) {
    const int32_t i = blockIdx.x * kBuildThreads + threadIdx.x;
    if (i >= n) return;
    const Segment g = segment_of(keys[i], n, ntypes, type_count);
    if (i >= g.e - 1) return;  // not an internal node id
    const int32_t f = rf[i];
    bool keep = !(cost[i] < 0.0f);
    if (keep && rl[i] - f + 1 <= leaf_size) {
        // ancestors of at most leaf_size particles (the only ones that can be runs)
        int32_t u = parent[i];
        for (int step = 0; step < kMaxDepth && u >= 0 && rl[u] - rf[u] + 1 <= leaf_size; ++step) {
            if (cost[u] < 0.0f) {
                keep = false;
                break;
            }
            u = parent[u];
        }
    }
    kept_flag[i] = keep ? 1u : 0u;
    if (keep) atomicAdd(&kept[f], 1u);
}

// One record per kept internal node (Karras id i).  Only about one id in
// leaf_size keeps a record, so a workgroup first collects the kept ids of
// kEmitItems x kBuildThreads consecutive ids into LDS (one ballot per wave and
// step) and then writes their records with every lane busy.
constexpr int kEmitItems = 8;

__global__ __launch_bounds__(kBuildThreads) void k_emit(int32_t n, int32_t ntypes,
                                                        const uint32_t *__restrict__ keys,
                                                        const uint32_t *__restrict__ type_count,
                                                        const float4 *__restrict__ sorted,
                                                        const int32_t *__restrict__ left,
                                                        const int32_t *__restrict__ rf, const int32_t *__restrict__ rl,
                                                        const int32_t *__restrict__ parent,
                                                        const float4 *__restrict__ box,
                                                        const uint32_t *__restrict__ P,
                                                        const TreeMeta *__restrict__ meta, int32_t leaf_size,
                                                        const uint32_t *__restrict__ kept_flag, int32_t qbits,
                                                        uint4 *__restrict__ records, int32_t *__restrict__ ropes) {
    __shared__ int32_t s_ids[kEmitItems * kBuildThreads];
    __shared__ uint32_t s_count;
    if (threadIdx.x == 0) s_count = 0;
    __syncthreads();
    const int32_t lane = (int32_t)__lane_id();
    const int64_t b0 = (int64_t)blockIdx.x * (kEmitItems * kBuildThreads);
#pragma unroll
    for (int k = 0; k < kEmitItems; ++k) {
        const int64_t i = b0 + k * kBuildThreads + threadIdx.x;
        bool keep = false;
        if (i < n) {
            const Segment g = segment_of(ntypes == 1 ? 0u : keys[i], n, ntypes, type_count);
            // an internal node id outside every particle run
            if (i < g.e - 1)
                keep = kept_flag ? kept_flag[i] != 0u : rl[i] - rf[i] + 1 > leaf_size;
        }
        const uint64_t m = __ballot(keep);
        if (m == 0) continue;
        uint32_t at = 0;
        if (lane == 0) at = atomicAdd(&s_count, (uint32_t)__popcll(m));
        at = (uint32_t)__shfl((int32_t)at, 0);
        const uint32_t below =
            __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
        if (keep) s_ids[at + below] = (int32_t)i;
    }
    __syncthreads();
    const uint32_t count = s_count;
    for (uint32_t e = threadIdx.x; e < count; e += kBuildThreads) {
        const int32_t i = s_ids[e];
        const TreeMeta &m = meta[ntypes == 1 ? 0 : (keys[i] >> 30)];
        emit_record(i, rf[i], rl[i], m, sorted, left, parent, box, P, leaf_size, kept_flag, qbits, records,
                    ropes);
    }
}

// Cell box of every sorted particle in its type tree's grid (the leaf box of a
// one-particle leaf, Section 2.2), packed like a record box, plus its original
// index: what paper-mode lists test (Section 2.3).  The grid is the paper's:
// the root-node box split into 2^b - 1 bins along each axis, h_d =
// max(extent_d, ext_floor) / (2^b - 1).
__global__ __launch_bounds__(kBuildThreads) void k_qpoint(int32_t n, int32_t ntypes, const float4 *__restrict__ sorted,
                                                          const TreeMeta *__restrict__ meta, int32_t qbits,
                                                          double ext_floor, uint4 *__restrict__ qpoint) {
    const int32_t k = blockIdx.x * kBuildThreads + threadIdx.x;
    if (k >= n) return;
    int t = 0;
    for (int u = 1; u < ntypes; ++u)
        if (k >= meta[u].start && meta[u].count > 0) t = u;
    const TreeMeta &m = meta[t];
    const uint32_t qmax = (1u << qbits) - 1u;
    double h[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) h[d] = axis_spacing(m.lo[d], m.hi[d], ext_floor, qbits);
    const float4 p = sorted[k];
    qpoint[k] = make_uint4(quantize_axis(p.x, p.x, m.lo[0], h[0], qmax), quantize_axis(p.y, p.y, m.lo[1], h[1], qmax),
                           quantize_axis(p.z, p.z, m.lo[2], h[2], qmax), (uint32_t)~__float_as_int(p.w));
}

inline dim3 grid_for(int64_t items) { return dim3((unsigned)((items + kBuildThreads - 1) / kBuildThreads)); }

}  // namespace

int32_t fit_chunks0(int32_t cap) { return (cap + kFitChunk - 1) / kFitChunk; }

namespace {

template <bool kCost>
void launch_tree_t(const Workspace &w, int32_t n, const TreeSource &src, int32_t kept_leaf, const Collapse &col,
                   hipStream_t s) {
    const TreeOut out{w.sorted, w.left, w.right, w.rf, w.rl, w.parent, w.leaf_parent, w.box, w.kept,
                      w.cost, reinterpret_cast<int32_t *>(w.visit), reinterpret_cast<int32_t *>(w.keys2), kept_leaf};
    int32_t nchunks = fit_chunks0(n);
    hipLaunchKernelGGL(k_tree_local<kCost>, dim3(nchunks), dim3(kFitThreads), 0, s, w.keys, w.vals, n, src, out,
                       w.front[0], w.fcount[0], w.err, col);
    int64_t chunk = kFitChunk;
    int which = 0;
    while (chunk < n) {
        const int32_t nprev = nchunks;
        chunk *= kFitFanout;
        nchunks = (int32_t)((n + chunk - 1) / chunk);
        hipLaunchKernelGGL(k_tree_level<kCost>, dim3(nchunks), dim3(kFitThreads), 0, s, n, chunk, nprev,
                           w.front[which], w.fcount[which], out, w.front[which ^ 1], w.fcount[which ^ 1], w.err, col);
        which ^= 1;
    }
}

}  // namespace

hipError_t launch_tree(const Workspace &w, int32_t n, const TreeSource &src, int32_t kept_leaf, const Collapse &col,
                       hipStream_t s) {
    if (n <= 0) return hipSuccess;
    if (col.kVball > 0.0f)
        launch_tree_t<true>(w, n, src, kept_leaf, col, s);
    else
        launch_tree_t<false>(w, n, src, kept_leaf, col, s);
    return hipGetLastError();
}

hipError_t launch_qpoint(const Workspace &w, int32_t n, int32_t ntypes, int32_t qbits, double lmax, hipStream_t s) {
    if (n > 0)
        hipLaunchKernelGGL(k_qpoint, grid_for(n), dim3(kBuildThreads), 0, s, n, ntypes, w.sorted, w.meta, qbits,
                           lmax * 0x1p-24, w.qpoint);
    return hipGetLastError();
}

size_t workspace_bytes(int32_t cap) {
    const size_t c = cap > 0 ? (size_t)cap : 1;
    const size_t tiles = (size_t)radix_tiles((int32_t)c);
    const size_t sb = (size_t)scan_blocks((int32_t)c + 1) + 1;
    auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
    size_t b = 0;
    b += 4 * al(c * 4);                       // keys, vals, keys2, vals2
    b += al(256 * tiles * 4) + al(256 * 4);   // histograms
    b += al((c + kSortedPad) * 16);           // sorted (+ padding read by whole-run loads)
    b += 6 * al(c * 4);                       // left right rf rl parent leaf_parent
    b += al(c * 4);                           // visit (split weights, then kept flags)
    b += al(c * 4);                           // cost (subtree collapse)
    b += al(c * 32);                          // boxes (lower and upper bound per node)
    b += al((c + 1) * 4) + al(sb * 4);        // kept + scan partials
    b += al(c * 32) + al(c * 4);              // records + ropes
    b += al((c + kSortedPad) * 16);           // cell boxes (paper-mode lists)
    b += al(QBVH_MAX_TYPES * sizeof(TreeMeta)) + al(QBVH_MAX_TYPES * 4) + al(4);
    const size_t nf = (size_t)fit_chunks0((int32_t)c);
    b += 2 * (al(nf * kFrontierCap * 4) + al(nf * 4));  // tree-build frontiers (ping-pong)
    return b;
}

void workspace_carve(Workspace &w, void *base, int32_t cap) {
    const size_t c = cap > 0 ? (size_t)cap : 1;
    const size_t tiles = (size_t)radix_tiles((int32_t)c);
    const size_t sb = (size_t)scan_blocks((int32_t)c + 1) + 1;
    auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
    char *p = (char *)base;
    auto take = [&](size_t bytes) {
        void *r = p;
        p += al(bytes);
        return r;
    };
    w.cap = cap;
    w.tiles = (int32_t)tiles;
    w.base = base;
    w.keys = (uint32_t *)take(c * 4);
    w.vals = (uint32_t *)take(c * 4);
    w.keys2 = (uint32_t *)take(c * 4);
    w.vals2 = (uint32_t *)take(c * 4);
    w.hist = (uint32_t *)take(256 * tiles * 4);
    w.digit_total = (uint32_t *)take(256 * 4);
    w.sorted = (float4 *)take((c + kSortedPad) * 16);
    w.left = (int32_t *)take(c * 4);
    w.right = (int32_t *)take(c * 4);
    w.rf = (int32_t *)take(c * 4);
    w.rl = (int32_t *)take(c * 4);
    w.parent = (int32_t *)take(c * 4);
    w.leaf_parent = (int32_t *)take(c * 4);
    w.visit = (uint32_t *)take(c * 4);
    w.cost = (float *)take(c * 4);
    w.box = (float4 *)take(c * 32);
    w.kept = (uint32_t *)take((c + 1) * 4);
    w.scan_part = (uint32_t *)take(sb * 4);
    w.records = (uint4 *)take(c * 32);
    w.qpoint = (uint4 *)take((c + kSortedPad) * 16);
    w.ropes = (int32_t *)take(c * 4);
    w.meta = (TreeMeta *)take(QBVH_MAX_TYPES * sizeof(TreeMeta));
    w.type_count = (uint32_t *)take(QBVH_MAX_TYPES * 4);
    w.err = (int32_t *)take(4);
    const size_t nf = (size_t)fit_chunks0((int32_t)c);
    for (int i = 0; i < 2; ++i) {
        w.front[i] = (int32_t *)take(nf * kFrontierCap * 4);
        w.fcount[i] = (uint32_t *)take(nf * 4);
    }
    w.bytes = (size_t)(p - (char *)base);
}

Collapse collapse_model(float collapse_radius, int32_t leaf_size) {
    Collapse c{0.0f, 0.0f, 0.0f, leaf_size};
    if (collapse_radius > 0.0f) {
        const double R = (double)collapse_radius;
        const double pi = 3.141592653589793;
        c.k2R = (float)(2.0 * R);
        c.kPiR2 = (float)(pi * R * R);
        c.kVball = (float)(4.0 / 3.0 * pi * R * R * R);
    }
    return c;
}

hipError_t launch_build(const Workspace &w, const float *d_pos, const int32_t *d_type, int32_t n, int32_t ntypes,
                        const float box[3], int32_t leaf_size, int32_t qbits, float collapse_radius, int32_t validate,
                        hipStream_t s, const double *pos64, double *sorted64, const double *box64) {
    const Collapse col = collapse_model(collapse_radius, leaf_size);
    const bool by_cost = col.kVball > 0.0f;
    hipLaunchKernelGGL(k_init, dim3(1), dim3(64), 0, s, w.type_count, w.err);
    const double sx = 1023.0 / (double)box[0];
    const double sy = 1023.0 / (double)box[1];
    const double sz = 1023.0 / (double)box[2];
    if (pos64 != nullptr)
        hipLaunchKernelGGL(k_morton<double>, grid_for((int64_t)n + 1), dim3(kBuildThreads), 0, s, pos64, d_type, n,
                           ntypes, box64[0], box64[1], box64[2], sx, sy, sz, validate, w.keys, w.kept, w.err);
    else
        hipLaunchKernelGGL(k_morton<float>, grid_for((int64_t)n + 1), dim3(kBuildThreads), 0, s, d_pos, d_type, n,
                           ntypes, (double)box[0], (double)box[1], (double)box[2], sx, sy, sz, validate, w.keys,
                           w.kept, w.err);
    hipError_t e = launch_radix_sort(w.keys, w.vals, w.keys2, w.vals2, w.hist, w.digit_total, n, w.tiles, s);
    if (e != hipSuccess) return e;
    if (ntypes > 1) hipLaunchKernelGGL(k_type_count, dim3(1), dim3(64), 0, s, w.keys, n, w.type_count);
    if (n > 0) {
        // (with the cost model, which nodes keep a record is known only after the fit)
        e = launch_tree(w, n, TreeSource{d_pos, nullptr, nullptr, 0, pos64, sorted64}, by_cost ? INT32_MAX : leaf_size,
                        col, s);
        if (e != hipSuccess) return e;
        if (by_cost)
            hipLaunchKernelGGL(k_kept_collapse, grid_for(n), dim3(kBuildThreads), 0, s, n, ntypes, w.keys,
                               w.type_count, w.rf, w.rl, w.parent, w.cost, leaf_size, w.visit, w.kept);
    }
    e = launch_exclusive_scan(w.kept, n + 1, w.scan_part, s);
    if (e != hipSuccess) return e;
    const double lmax = (double)fmaxf(box[0], fmaxf(box[1], box[2]));
    const double ext_floor = lmax * 0x1p-24;
    hipLaunchKernelGGL(k_meta, dim3(1), dim3(64), 0, s, n, ntypes, w.type_count, w.sorted, w.box,
                       w.kept, qbits, leaf_size, by_cost ? w.cost : nullptr, ext_floor, w.meta);
    if (n > 0)
        hipLaunchKernelGGL(k_emit, grid_for((n + kEmitItems - 1) / kEmitItems), dim3(kBuildThreads), 0, s, n, ntypes,
                           w.keys, w.type_count,
                           w.sorted, w.left, w.rf, w.rl, w.parent, w.box, w.kept, w.meta,
                           leaf_size, by_cost ? w.visit : nullptr, qbits, w.records, w.ropes);
    return hipGetLastError();
}

}  // namespace qbi

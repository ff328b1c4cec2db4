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

__global__ __launch_bounds__(kBuildThreads) void k_morton(const float *__restrict__ pos,
                                                          const int32_t *__restrict__ type, int32_t n,
                                                          int32_t ntypes, float Lx, float Ly, float Lz,
                                                          double sx, double sy, double sz, int32_t validate,
                                                          uint32_t *__restrict__ keys, uint32_t *__restrict__ vals,
                                                          uint32_t *__restrict__ kept, int32_t *err) {
    const int32_t k = blockIdx.x * kBuildThreads + threadIdx.x;
    if (k <= n) kept[k] = 0;
    if (k < n) {
        const float x = pos[3 * (int64_t)k + 0];
        const float y = pos[3 * (int64_t)k + 1];
        const float z = pos[3 * (int64_t)k + 2];
        int32_t t = type ? type[k] : 0;
        if (validate) {
            bool ok = (x >= 0.0f && x < Lx) && (y >= 0.0f && y < Ly) && (z >= 0.0f && z < Lz) &&
                      (t >= 0 && t < ntypes);
            if (!ok) atomicOr(err, 1);
        }
        t = t < 0 ? 0 : (t >= ntypes ? ntypes - 1 : t);
        keys[k] = morton_key(x, y, z, sx, sy, sz, t);
        vals[k] = (uint32_t)k;
    }
}

// Particles per type, read off the sorted keys (type in bits 30-31) by binary
// search: no atomics on a few hot counters.
__global__ void k_type_count(const uint32_t *__restrict__ keys, int32_t n, uint32_t *__restrict__ type_count) {
    const uint32_t t = threadIdx.x;
    if (t < QBVH_MAX_TYPES)
        type_count[t] = (uint32_t)(type_start(keys, 0, n, t + 1) - type_start(keys, 0, n, t));
}

// fp64 particle data, before the build: each coordinate rounded to nearest
// fp32 (the tree is built and walked on these; the exact decisions use the
// fp64 values), with the fp64 checks 0 <= x < L and 0 <= type < ntypes when
// `validate` is set (*err, cleared by k_clear_err before, is set on failure).
__global__ void k_clear_err(int32_t *err) {
    if (threadIdx.x == 0) *err = 0;
}

__global__ __launch_bounds__(kBuildThreads) void k_to_f32(const double *__restrict__ pos64,
                                                          const int32_t *__restrict__ type, int32_t n,
                                                          int32_t ntypes, double Lx, double Ly, double Lz,
                                                          int32_t validate, float *__restrict__ pos32,
                                                          int32_t *err) {
    const int32_t i = blockIdx.x * kBuildThreads + threadIdx.x;
    if (i >= n) return;
    const double x = pos64[3 * (int64_t)i + 0], y = pos64[3 * (int64_t)i + 1], z = pos64[3 * (int64_t)i + 2];
    if (validate) {
        const int32_t t = type ? type[i] : 0;
        const bool ok = (x >= 0.0 && x < Lx) && (y >= 0.0 && y < Ly) && (z >= 0.0 && z < Lz) && t >= 0 && t < ntypes;
        if (!ok) atomicOr(err, 1);
    }
    pos32[3 * (int64_t)i + 0] = (float)x;
    pos32[3 * (int64_t)i + 1] = (float)y;
    pos32[3 * (int64_t)i + 2] = (float)z;
}

// fp64 particle data, after the build: the fp64 position of every sorted
// particle (its input index is the inverted w word of the fp32 copy).
__global__ __launch_bounds__(kBuildThreads) void k_gather64(const float4 *__restrict__ sorted, int32_t n,
                                                            const double *__restrict__ pos64,
                                                            double *__restrict__ sorted64) {
    const int32_t k = blockIdx.x * kBuildThreads + threadIdx.x;
    if (k >= n) return;
    const int64_t i = ~__float_as_int(sorted[k].w);
    double *o = sorted64 + 4 * (int64_t)k;
    o[0] = pos64[3 * i + 0];
    o[1] = pos64[3 * i + 1];
    o[2] = pos64[3 * i + 2];
    o[3] = 0.0;
}

// Karras's parallel construction: internal node i of a segment covers a
// range with i at one end; its direction, far end and split are found by
// exponential then binary search on the common-prefix length.  The same
// thread also writes sorted position i's particle in Z order (the gather):
// its loads from the unsorted input go out first and complete while the
// searches run, so the gather's memory latency and the searches' VALU work
// overlap in one launch instead of following each other.
__global__ __launch_bounds__(kBuildThreads) void k_karras(const uint32_t *__restrict__ keys, int32_t n,
                                                          int32_t ntypes, const uint32_t *__restrict__ type_count,
                                                          int32_t leaf_size, const float *__restrict__ pos,
                                                          const uint32_t *__restrict__ vals,
                                                          float4 *__restrict__ sorted, int32_t *__restrict__ left,
                                                          int32_t *__restrict__ right, int32_t *__restrict__ rf,
                                                          int32_t *__restrict__ rl, int32_t *__restrict__ parent,
                                                          int32_t *__restrict__ leaf_parent,
                                                          uint32_t *__restrict__ visit, uint32_t *__restrict__ kept) {
    __shared__ uint32_t s_keys[3 * kBuildThreads];
    const StagedKeys K = stage_keys(keys, s_keys, (int32_t)(blockIdx.x * kBuildThreads), 0, n);
    const int32_t i = blockIdx.x * kBuildThreads + threadIdx.x;
    if (i >= n) return;
    const uint32_t o = vals[i];
    const float4 p = make_float4(pos[3 * (int64_t)o + 0], pos[3 * (int64_t)o + 1], pos[3 * (int64_t)o + 2],
                                 __int_as_float(~(int32_t)o));
    const Segment g = segment_of(keys[i], n, ntypes, type_count);
    visit[i] = 0;
    if (i == g.e - 1) {  // no internal node carries the last position's id
        if (g.e - g.s == 1) leaf_parent[i] = -1;
    } else {
        const KarrasNode r = karras_node(K, i, g);
        const int32_t gamma = r.gamma, f = r.f, la = r.l, cl = r.left, cr = r.right;
        left[i] = cl;
        right[i] = cr;
        rf[i] = f;
        rl[i] = la;
        if (cl < 0) leaf_parent[gamma] = i; else parent[gamma] = i;
        if (cr < 0) leaf_parent[gamma + 1] = i; else parent[gamma + 1] = i;
        if (i == g.s) parent[i] = -1;
        if (la - f + 1 > leaf_size) atomicAdd(&kept[f], 1u);
    }
    sorted[i] = p;
}

// Bottom-up boxes (Section 2.1: boxes are fit by walking up the tree from the
// leaves).  Every leaf climbs; at each internal node an atomic visit counter
// lets the first arrival stop and the second merge both children and go on.
//
// The counters are synchronized within one workgroup only: an agent-scope
// acquire/release on gfx950 writes back and invalidates the XCD's L2 at every
// step, which is far too slow for N atomic steps.  So the climb is split by
// sorted position into chunks.  A node whose particle range lies inside one
// chunk has both children inside it, so only that chunk's workgroup ever
// touches its counter.  Level 0 uses chunks of kFitChunk positions with
// counters and boxes in LDS (60 KB, so two workgroups share a compute unit);
// every further level multiplies the chunk by
// kFitFanout and climbs in global memory with workgroup-scope atomics,
// starting from the nodes the previous level left at its chunk borders (the
// "frontier": finished nodes whose parent straddles a border).  The last
// level has one chunk and reaches every root.  A frontier holds at most two
// border chains of the tree (each at most 65 deep), so kFrontierCap suffices.
constexpr int kFitChunk = 1024;
constexpr int kFitThreads = 1024;
// A small fanout keeps every level's climbs short (about five tree levels from
// each frontier node) and its workgroups many; N = 8M takes three level launches.
constexpr int kFitFanout = 32;
constexpr int kFrontierCap = 160;
// A chunk's frontier holds nodes whose parent's range crosses one of the
// chunk's two borders; the nodes whose range crosses a border form one chain
// of the tree (they nest), so each border contributes at most one node per
// tree level.  Keys are 32 bits plus a 32-bit position, so a radix tree has
// at most 64 levels of internal nodes: 2 * (64 + 1) entries at most.
static_assert(kFrontierCap >= 2 * (64 + 1), "fit frontier bound");

__device__ __forceinline__ void frontier_push(int32_t c, uint32_t *s_fcount, int32_t *s_front, int32_t *err) {
    const uint32_t slot = atomicAdd(s_fcount, 1u);
    if (slot < (uint32_t)kFrontierCap)
        s_front[slot] = c;
    else
        atomicOr(err, 2);
}

// First level: the chunk's node links, its particles' positions, the visit
// counters and the boxes all live in LDS (loaded with coalesced reads), so a
// climb touches global memory only to read its leaf's parent.
template <bool kCost>
__global__ __launch_bounds__(kFitThreads) void k_fit_local(const float4 *__restrict__ sorted,
                                                           const int32_t *__restrict__ left,
                                                           const int32_t *__restrict__ right,
                                                           const int32_t *__restrict__ rf,
                                                           const int32_t *__restrict__ rl,
                                                           const int32_t *__restrict__ parent,
                                                           const int32_t *__restrict__ leaf_parent, int32_t n,
                                                           float4 *__restrict__ box_lo, float4 *__restrict__ box_hi,
                                                           int32_t *__restrict__ front, uint32_t *__restrict__ fcount,
                                                           int32_t *err, Collapse col, float *__restrict__ cost) {
    __shared__ float s_box[6][kFitChunk];
    __shared__ float s_cost[kCost ? kFitChunk : 1];
    __shared__ float s_pos[3][kFitChunk];
    __shared__ int32_t s_link[5][kFitChunk];  // left, right, range first, range last, parent
    __shared__ uint32_t s_visit[kFitChunk];
    __shared__ int32_t s_front[kFrontierCap];
    __shared__ uint32_t s_fcount;
    const int32_t c0 = blockIdx.x * kFitChunk;
    const int32_t m = min(kFitChunk, n - c0);
    for (int i = threadIdx.x; i < kFitChunk; i += kFitThreads) {
        s_visit[i] = 0;
        if (i < m) {
            // entries of ids that are not internal nodes (the last position of
            // a segment) are loaded but never referenced
            const int32_t k = c0 + i;
            s_link[0][i] = left[k];
            s_link[1][i] = right[k];
            s_link[2][i] = rf[k];
            s_link[3][i] = rl[k];
            s_link[4][i] = parent[k];
            const float4 q = sorted[k];
            s_pos[0][i] = q.x;
            s_pos[1][i] = q.y;
            s_pos[2][i] = q.z;
        }
    }
    if (threadIdx.x == 0) s_fcount = 0;
    __syncthreads();
    for (int32_t i0 = threadIdx.x; i0 < m; i0 += kFitThreads) {
        int32_t c = ~(c0 + i0);
        int32_t p = leaf_parent[c0 + i0];
        for (int step = 0; p >= 0 && step < kMaxDepth; ++step) {
            const int32_t j = p - c0;
            // a parent whose range leaves the chunk ends this level's climb
            if (j < 0 || j >= m || s_link[2][j] < c0 || s_link[3][j] >= c0 + kFitChunk) {
                frontier_push(c, &s_fcount, s_front, err);
                break;
            }
            const uint32_t old = __hip_atomic_fetch_add(&s_visit[j], 1u, __ATOMIC_ACQ_REL,
                                                        __HIP_MEMORY_SCOPE_WORKGROUP);
            if (old == 0) break;
            float lo[3], hi[3];
#pragma unroll
            for (int side = 0; side < 2; ++side) {
                const int32_t ch = s_link[side][j];
                float clo[3], chi[3];
                if (ch < 0) {
                    const int32_t t = ~ch - c0;
#pragma unroll
                    for (int d = 0; d < 3; ++d) clo[d] = chi[d] = s_pos[d][t];
                } else {
                    const int32_t t = ch - c0;
#pragma unroll
                    for (int d = 0; d < 3; ++d) {
                        clo[d] = s_box[d][t];
                        chi[d] = s_box[3 + d][t];
                    }
                }
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    lo[d] = side ? fminf(lo[d], clo[d]) : clo[d];
                    hi[d] = side ? fmaxf(hi[d], chi[d]) : chi[d];
                }
            }
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                s_box[d][j] = lo[d];
                s_box[3 + d][j] = hi[d];
            }
            if (kCost) {
                // children's costs: a particle, or an internal node of the chunk finished before
                float fc[2];
#pragma unroll
                for (int side = 0; side < 2; ++side) {
                    const int32_t ch = s_link[side][j];
                    fc[side] = ch < 0 ? col.kVball : fabsf(s_cost[ch - c0]);
                }
                s_cost[j] = node_cost(col, s_link[3][j] - s_link[2][j] + 1, lo[0], lo[1], lo[2], hi[0], hi[1], hi[2],
                                      fc[0], fc[1]);
            }
            c = p;
            p = s_link[4][j];
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < m; i += kFitThreads) {
        if (s_visit[i] == 2) {
            box_lo[c0 + i] = make_float4(s_box[0][i], s_box[1][i], s_box[2][i], 0.0f);
            box_hi[c0 + i] = make_float4(s_box[3][i], s_box[4][i], s_box[5][i], 0.0f);
            if (kCost) cost[c0 + i] = s_cost[i];
        }
    }
    const uint32_t fc = min(s_fcount, (uint32_t)kFrontierCap);
    for (uint32_t i = threadIdx.x; i < fc; i += kFitThreads) front[(int64_t)blockIdx.x * kFrontierCap + i] = s_front[i];
    if (threadIdx.x == 0) fcount[blockIdx.x] = fc;
}

// One level above the first: chunks of `chunk` positions, starting from the
// frontiers of the `fan` previous-level chunks each contains.
template <bool kCost>
__global__ __launch_bounds__(kFitThreads) void k_fit_level(const float4 *__restrict__ sorted,
                                                           const int32_t *__restrict__ left,
                                                           const int32_t *__restrict__ right,
                                                           const int32_t *__restrict__ rf,
                                                           const int32_t *__restrict__ rl,
                                                           const int32_t *__restrict__ parent,
                                                           const int32_t *__restrict__ leaf_parent, int64_t chunk,
                                                           int32_t nprev, const int32_t *__restrict__ front_in,
                                                           const uint32_t *__restrict__ fcount_in, uint32_t *visit,
                                                           float4 *box_lo, float4 *box_hi,
                                                           int32_t *__restrict__ front_out,
                                                           uint32_t *__restrict__ fcount_out, int32_t *err,
                                                           Collapse col, float *cost) {
    __shared__ int32_t s_front[kFrontierCap];
    __shared__ uint32_t s_fcount;
    __shared__ uint32_t s_off[kFitFanout + 1];
    const int64_t c0 = (int64_t)blockIdx.x * chunk;
    const int64_t c1 = c0 + chunk;
    const int32_t j0 = blockIdx.x * kFitFanout;
    // The frontier entries of the fan-in chunks, numbered consecutively, so
    // that each thread climbs from at most a few of them (the climbs are
    // chains of dependent loads: their count per thread sets the time).
    if (threadIdx.x < kFitFanout) {
        const int32_t jc = j0 + (int32_t)threadIdx.x;
        s_off[threadIdx.x + 1] = jc < nprev ? min(fcount_in[jc], (uint32_t)kFrontierCap) : 0u;
    }
    if (threadIdx.x == 0) {
        s_fcount = 0;
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
        const int32_t jc = j0 + lo;
        const uint32_t slot = e - s_off[lo];
        int32_t c = front_in[(int64_t)jc * kFrontierCap + slot];
        int32_t p = c < 0 ? leaf_parent[~c] : parent[c];
        for (int step = 0; p >= 0 && step < kMaxDepth; ++step) {
            // The links do not change during the fit: all of them are read
            // before the atomic, so that a step waits for three round trips
            // (links, counter, child boxes) rather than five.
            const int32_t pf = rf[p], pl = rl[p], c0i = left[p], c1i = right[p], pp = parent[p];
            // (sign bits rather than compares: both loads are then waited for together)
            if (((uint64_t)((int64_t)pf - c0) | (uint64_t)(c1 - 1 - (int64_t)pl)) >> 63) {
                frontier_push(c, &s_fcount, s_front, err);
                break;
            }
            const uint32_t old = __hip_atomic_fetch_add(&visit[p], 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_WORKGROUP);
            if (old == 0) break;
            // a leaf child's box is its particle: pointers are selected, not
            // branched on, so the four loads go out together
            const float4 *pa_lo = c0i < 0 ? sorted + ~c0i : box_lo + c0i;
            const float4 *pa_hi = c0i < 0 ? sorted + ~c0i : box_hi + c0i;
            const float4 *pb_lo = c1i < 0 ? sorted + ~c1i : box_lo + c1i;
            const float4 *pb_hi = c1i < 0 ? sorted + ~c1i : box_hi + c1i;
            const float4 alo = *pa_lo, ahi = *pa_hi, blo = *pb_lo, bhi = *pb_hi;
            const float4 nlo = make_float4(fminf(alo.x, blo.x), fminf(alo.y, blo.y), fminf(alo.z, blo.z), 0.0f);
            const float4 nhi = make_float4(fmaxf(ahi.x, bhi.x), fmaxf(ahi.y, bhi.y), fmaxf(ahi.z, bhi.z), 0.0f);
            box_lo[p] = nlo;
            box_hi[p] = nhi;
            if (kCost) {
                const float fa = c0i < 0 ? col.kVball : fabsf(cost[c0i]);
                const float fb = c1i < 0 ? col.kVball : fabsf(cost[c1i]);
                cost[p] = node_cost(col, pl - pf + 1, nlo.x, nlo.y, nlo.z, nhi.x, nhi.y, nhi.z, fa, fb);
            }
            c = p;
            p = pp;
        }
    }
    __syncthreads();
    const uint32_t fc = min(s_fcount, (uint32_t)kFrontierCap);
    for (uint32_t i = threadIdx.x; i < fc; i += kFitThreads) front_out[(int64_t)blockIdx.x * kFrontierCap + i] = s_front[i];
    if (threadIdx.x == 0) fcount_out[blockIdx.x] = fc;
}

// Root box, grid spacing and slot range of each type's tree.
__global__ void k_meta(int32_t n, int32_t ntypes, const uint32_t *__restrict__ type_count,
                       const float4 *__restrict__ sorted, const float4 *__restrict__ box_lo,
                       const float4 *__restrict__ box_hi, const uint32_t *__restrict__ P, int32_t qbits,
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
        const float4 a = box_lo[s], b = box_hi[s];
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
                                                        const int32_t *__restrict__ right,
                                                        const int32_t *__restrict__ rf, const int32_t *__restrict__ rl,
                                                        const int32_t *__restrict__ parent,
                                                        const float4 *__restrict__ box_lo,
                                                        const float4 *__restrict__ box_hi,
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
        emit_record(i, rf[i], rl[i], m, sorted, left, right, rf, rl, parent, box_lo, box_hi, P, leaf_size, kept_flag,
                    qbits, records, ropes);
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

hipError_t launch_to_f32(const double *pos64, const int32_t *type, int32_t n, int32_t ntypes, const double box[3],
                         int32_t validate, float *pos32, int32_t *err, hipStream_t s) {
    hipLaunchKernelGGL(k_clear_err, dim3(1), dim3(64), 0, s, err);
    if (n > 0)
        hipLaunchKernelGGL(k_to_f32, grid_for(n), dim3(kBuildThreads), 0, s, pos64, type, n, ntypes, box[0], box[1],
                           box[2], validate, pos32, err);
    return hipGetLastError();
}

hipError_t launch_gather64(const Workspace &w, int32_t n, const double *pos64, double *sorted64, hipStream_t s) {
    if (n > 0)
        hipLaunchKernelGGL(k_gather64, grid_for(n), dim3(kBuildThreads), 0, s, w.sorted, n, pos64, sorted64);
    return hipGetLastError();
}

namespace {

template <bool kCost>
void launch_fit_t(const Workspace &w, int32_t n, const Collapse &col, hipStream_t s) {
    int32_t nchunks = fit_chunks0(n);
    hipLaunchKernelGGL(k_fit_local<kCost>, dim3(nchunks), dim3(kFitThreads), 0, s, w.sorted, w.left, w.right, w.rf,
                       w.rl, w.parent, w.leaf_parent, n, w.box_lo, w.box_hi, w.front[0], w.fcount[0], w.err, col,
                       w.cost);
    int64_t chunk = kFitChunk;
    int which = 0;
    while (chunk < n) {
        const int32_t nprev = nchunks;
        chunk *= kFitFanout;
        nchunks = (int32_t)((n + chunk - 1) / chunk);
        hipLaunchKernelGGL(k_fit_level<kCost>, dim3(nchunks), dim3(kFitThreads), 0, s, w.sorted, w.left, w.right,
                           w.rf, w.rl, w.parent, w.leaf_parent, chunk, nprev, w.front[which], w.fcount[which],
                           w.visit, w.box_lo, w.box_hi, w.front[which ^ 1], w.fcount[which ^ 1], w.err, col, w.cost);
        which ^= 1;
    }
}

}  // namespace

hipError_t launch_fit(const Workspace &w, int32_t n, const Collapse &col, hipStream_t s) {
    if (col.kVball > 0.0f)
        launch_fit_t<true>(w, n, col, s);
    else
        launch_fit_t<false>(w, n, col, s);
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
    b += al(c * 4);                           // visit (fit counters, then kept flags)
    b += al(c * 4);                           // cost (subtree collapse)
    b += 2 * al(c * 16);                      // boxes
    b += al((c + 1) * 4) + al(sb * 4);        // kept + scan partials
    b += al(c * 32) + al(c * 4);              // records + ropes
    b += al((c + kSortedPad) * 16);           // cell boxes (paper-mode lists)
    b += al(QBVH_MAX_TYPES * sizeof(TreeMeta)) + al(QBVH_MAX_TYPES * 4) + al(4);
    const size_t nf = (size_t)fit_chunks0((int32_t)c);
    b += 2 * (al(nf * kFrontierCap * 4) + al(nf * 4));  // fit frontiers (ping-pong)
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
    w.box_lo = (float4 *)take(c * 16);
    w.box_hi = (float4 *)take(c * 16);
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
                        hipStream_t s) {
    const Collapse col = collapse_model(collapse_radius, leaf_size);
    const bool by_cost = col.kVball > 0.0f;
    hipLaunchKernelGGL(k_init, dim3(1), dim3(64), 0, s, w.type_count, w.err);
    const double sx = 1023.0 / (double)box[0];
    const double sy = 1023.0 / (double)box[1];
    const double sz = 1023.0 / (double)box[2];
    hipLaunchKernelGGL(k_morton, grid_for((int64_t)n + 1), dim3(kBuildThreads), 0, s, d_pos, d_type, n, ntypes,
                       box[0], box[1], box[2], sx, sy, sz, validate, w.keys, w.vals, w.kept, w.err);
    hipError_t e = launch_radix_sort(w.keys, w.vals, w.keys2, w.vals2, w.hist, w.digit_total, n, w.tiles, s);
    if (e != hipSuccess) return e;
    if (ntypes > 1) hipLaunchKernelGGL(k_type_count, dim3(1), dim3(64), 0, s, w.keys, n, w.type_count);
    if (n > 0) {
        // (with the cost model, which nodes keep a record is known only after the fit)
        hipLaunchKernelGGL(k_karras, grid_for(n), dim3(kBuildThreads), 0, s, w.keys, n, ntypes, w.type_count,
                           by_cost ? INT32_MAX : leaf_size, d_pos, w.vals, w.sorted, w.left, w.right, w.rf, w.rl,
                           w.parent, w.leaf_parent, w.visit, w.kept);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        e = launch_fit(w, n, col, s);
        if (e != hipSuccess) return e;
        if (by_cost)
            hipLaunchKernelGGL(k_kept_collapse, grid_for(n), dim3(kBuildThreads), 0, s, n, ntypes, w.keys,
                               w.type_count, w.rf, w.rl, w.parent, w.cost, leaf_size, w.visit, w.kept);
    }
    e = launch_exclusive_scan(w.kept, n + 1, w.scan_part, s);
    if (e != hipSuccess) return e;
    const double lmax = (double)fmaxf(box[0], fmaxf(box[1], box[2]));
    const double ext_floor = lmax * 0x1p-24;
    hipLaunchKernelGGL(k_meta, dim3(1), dim3(64), 0, s, n, ntypes, w.type_count, w.sorted, w.box_lo, w.box_hi,
                       w.kept, qbits, leaf_size, by_cost ? w.cost : nullptr, ext_floor, w.meta);
    if (n > 0)
        hipLaunchKernelGGL(k_emit, grid_for((n + kEmitItems - 1) / kEmitItems), dim3(kBuildThreads), 0, s, n, ntypes,
                           w.keys, w.type_count,
                           w.sorted, w.left, w.right, w.rf, w.rl, w.parent, w.box_lo, w.box_hi, w.kept, w.meta,
                           leaf_size, by_cost ? w.visit : nullptr, qbits, w.records, w.ropes);
    return hipGetLastError();
}

}  // namespace qbi

// Batched build: many independent systems built by one launch sequence, each
// kernel covering every system at once (Section 2.1 and Section 2.2 applied
// per system).  The systems' particles are laid end to end; system s owns
// positions [off_s, off_s + n_s) of every per-particle array, sorts inside
// that range only (segmented radix sort), and its type trees are the
// segments (s, type) of the concatenation.  Records of all trees share one
// array (their preorder positions come from one scan), and every tree keeps
// its own root box, grid and record range in meta[s][type].
//
// Workgroups of the per-particle kernels never straddle two systems (each
// system starts a new workgroup), so every per-system value is uniform in a
// workgroup and read from the system table with scalar loads.
#include "build_common.h"

namespace qbi {
namespace {

struct Item {
    int32_t sys;    // system of this workgroup
    int32_t local;  // index of this work-item inside the system
};

__device__ __forceinline__ Item item_of(const int32_t *__restrict__ blk_first, int32_t nsys) {
    Item it;
    it.sys = find_seg(blk_first, nsys, (int32_t)blockIdx.x);
    it.local = ((int32_t)blockIdx.x - blk_first[it.sys]) * kBuildThreads + (int32_t)threadIdx.x;
    return it;
}

// Segment of sorted position i of system s: its type's range inside the system.
__device__ __forceinline__ Segment batch_segment(uint32_t key, int32_t off, const uint32_t *__restrict__ tc) {
    const uint32_t t = key >> 30;
    int32_t s = off;
    for (uint32_t u = 0; u < t; ++u) s += (int32_t)tc[u];
    return {s, s + (int32_t)tc[t]};
}

// Clears the per-system type counters, the error word and every system's
// overflow flag (kernels, not memsets, so the sequence can be captured).
__global__ __launch_bounds__(kBuildThreads) void k_b_init(int32_t nsys, uint32_t *__restrict__ type_count,
                                                          const TravArgs *__restrict__ trav, int32_t *err) {
    const int32_t i = blockIdx.x * kBuildThreads + threadIdx.x;
    if (i < nsys * QBVH_MAX_TYPES) type_count[i] = 0;
    if (i < nsys) trav[i].overflow[0] = 0;
    if (i == 0) *err = 0;
}

__global__ __launch_bounds__(kBuildThreads) void k_b_morton(const int32_t *__restrict__ blk_first, int32_t nsys,
                                                            const SysBuild *__restrict__ sysb, int32_t total,
                                                            uint32_t *__restrict__ keys,
                                                            uint32_t *__restrict__ kept) {
    const Item it = item_of(blk_first, nsys);
    const SysBuild &y = sysb[it.sys];
    if (blockIdx.x == 0 && threadIdx.x == 0) kept[total] = 0;
    if (it.local < y.n) {
        const int32_t k = y.off + it.local;
        const float x = y.pos[3 * (int64_t)it.local + 0];
        const float yy = y.pos[3 * (int64_t)it.local + 1];
        const float z = y.pos[3 * (int64_t)it.local + 2];
        int32_t t = y.type ? y.type[it.local] : 0;
        t = t < 0 ? 0 : (t >= y.ntypes ? y.ntypes - 1 : t);
        keys[k] = morton_key(x, yy, z, y.scale[0], y.scale[1], y.scale[2], t);
    }
}

// Particles per (system, type), read off each system's sorted keys by binary
// search (every entry written, types a system lacks included).
__global__ __launch_bounds__(kBuildThreads) void k_b_type_count(int32_t nsys, const SysBuild *__restrict__ sysb,
                                                                const uint32_t *__restrict__ keys,
                                                                uint32_t *__restrict__ type_count) {
    const int32_t i = blockIdx.x * kBuildThreads + threadIdx.x;
    if (i >= nsys * QBVH_MAX_TYPES) return;
    const SysBuild &y = sysb[i / QBVH_MAX_TYPES];
    const uint32_t t = (uint32_t)(i % QBVH_MAX_TYPES);
    type_count[i] = (uint32_t)(type_start(keys, y.off, y.off + y.n, t + 1) - type_start(keys, y.off, y.off + y.n, t));
}

// Tree description of every (system, type).
__global__ __launch_bounds__(64) void k_b_meta(int32_t nsys, const SysBuild *__restrict__ sysb,
                                               const uint32_t *__restrict__ type_count,
                                               const float4 *__restrict__ sorted, const float4 *__restrict__ box,
                                               const uint32_t *__restrict__ P,
                                               int32_t qbits, int32_t leaf_size, TreeMeta *__restrict__ meta) {
    const int32_t idx = blockIdx.x * 64 + threadIdx.x;
    const int32_t sys = idx / QBVH_MAX_TYPES, t = idx % QBVH_MAX_TYPES;
    if (sys >= nsys) return;
    const SysBuild &y = sysb[sys];
    if (t >= y.ntypes) return;
    const uint32_t *tc = type_count + sys * QBVH_MAX_TYPES;
    int32_t s = y.off;
    for (int u = 0; u < t; ++u) s += (int32_t)tc[u];
    const int32_t c = (int32_t)tc[t];
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
    meta[idx] = tree_meta(lo, hi, y.ext_floor, qbits, s, c, c <= leaf_size, P);
}

__global__ __launch_bounds__(kBuildThreads) void k_b_emit(const int32_t *__restrict__ blk_first, int32_t nsys,
                                                          const SysBuild *__restrict__ sysb,
                                                          const uint32_t *__restrict__ keys,
                                                          const uint32_t *__restrict__ type_count,
                                                          const float4 *__restrict__ sorted,
                                                          const int32_t *__restrict__ left,
                                                          const int32_t *__restrict__ rf, const int32_t *__restrict__ rl,
                                                          const int32_t *__restrict__ parent,
                                                          const float4 *__restrict__ box,
                                                          const uint32_t *__restrict__ P,
                                                          const TreeMeta *__restrict__ meta, int32_t leaf_size,
                                                          int32_t qbits, uint4 *__restrict__ records,
                                                          int32_t *__restrict__ ropes) {
    // the workgroup's kept ids first (about one in leaf_size), so that the
    // record writes run on full wavefronts
    __shared__ int32_t s_ids[kBuildThreads];
    __shared__ uint32_t s_count;
    if (threadIdx.x == 0) s_count = 0;
    __syncthreads();
    const Item it = item_of(blk_first, nsys);
    const SysBuild &y = sysb[it.sys];
    const int32_t i = y.off + it.local;
    bool keep = false;
    if (it.local < y.n) {
        const Segment g = batch_segment(keys[i], y.off, type_count + it.sys * QBVH_MAX_TYPES);
        // an internal node id outside every particle run
        if (i < g.e - 1) keep = rl[i] - rf[i] + 1 > leaf_size;
    }
    const uint64_t mk = __ballot(keep);
    if (mk != 0) {
        uint32_t at = 0;
        if (__lane_id() == 0) at = atomicAdd(&s_count, (uint32_t)__popcll(mk));
        at = (uint32_t)__shfl((int32_t)at, 0);
        const uint32_t below =
            __builtin_amdgcn_mbcnt_hi((uint32_t)(mk >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mk, 0u));
        if (keep) s_ids[at + below] = i;
    }
    __syncthreads();
    if (threadIdx.x >= s_count) return;
    const int32_t k = s_ids[threadIdx.x];
    const TreeMeta &m = meta[it.sys * QBVH_MAX_TYPES + (keys[k] >> 30)];
    emit_record(k, rf[k], rl[k], m, sorted, left, parent, box, P, leaf_size, nullptr, qbits, records,
                ropes);
}

}  // namespace

hipError_t launch_batch(const BatchLaunch &b, hipStream_t s) {
    const Workspace &w = b.ws;
    const int32_t ninit = b.nsys * QBVH_MAX_TYPES;
    hipLaunchKernelGGL(k_b_init, dim3((unsigned)((ninit + kBuildThreads - 1) / kBuildThreads)), dim3(kBuildThreads),
                       0, s, b.nsys, b.type_count, b.trav, w.err);
    if (b.blocks > 0)
        hipLaunchKernelGGL(k_b_morton, dim3((unsigned)b.blocks), dim3(kBuildThreads), 0, s, b.blk_first, b.nsys,
                           b.sysb, b.total, w.keys, w.kept);
    hipError_t e = launch_radix_sort_segmented(w.keys, w.vals, w.keys2, w.vals2, b.hist, b.scan_part, b.total,
                                               b.tiles, b.tile_first, b.sys_off, b.nsys, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_b_type_count, dim3((unsigned)((ninit + kBuildThreads - 1) / kBuildThreads)),
                       dim3(kBuildThreads), 0, s, b.nsys, b.sysb, w.keys, b.type_count);
    if (b.total > 0) {
        e = launch_tree(w, b.total, TreeSource{nullptr, b.sysb, b.sys_off, b.nsys, nullptr, nullptr}, b.leaf_size,
                        Collapse{0.f, 0.f, 0.f, b.leaf_size}, s);
        if (e != hipSuccess) return e;
    }
    e = launch_exclusive_scan(w.kept, b.total + 1, b.scan_part, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_b_meta, dim3((unsigned)((ninit + 63) / 64)), dim3(64), 0, s, b.nsys, b.sysb, b.type_count,
                       w.sorted, w.box, w.kept, b.qbits, b.leaf_size, b.meta);
    if (b.total > 0)
        hipLaunchKernelGGL(k_b_emit, dim3((unsigned)b.blocks), dim3(kBuildThreads), 0, s, b.blk_first, b.nsys, b.sysb,
                           w.keys, b.type_count, w.sorted, w.left, w.rf, w.rl, w.parent, w.box,
                           w.kept, b.meta, b.leaf_size, b.qbits, w.records, w.ropes);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_traverse_batch(b, s);
}

}  // namespace qbi

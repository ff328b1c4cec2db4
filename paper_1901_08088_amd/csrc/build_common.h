// Device helpers shared by the single-system and batched builds: Morton bins,
// segment-bounded common prefixes, particle-run references and the outward
// quantization of box bounds (Section 2.1, Section 2.2).
#pragma once

#include "qbvh_internal.h"

namespace qbi {

constexpr int kBuildThreads = 256;
constexpr int kMaxDepth = 128;  // > 65, the deepest possible radix tree over 64-bit keys

__device__ __forceinline__ uint32_t spread10(uint32_t v) {
    v &= 0x3FFu;
    v = (v | (v << 16)) & 0x030000FFu;
    v = (v | (v << 8)) & 0x0300F00Fu;
    v = (v | (v << 4)) & 0x030C30C3u;
    v = (v | (v << 2)) & 0x09249249u;
    return v;
}

// Bin of one coordinate: floor(x * (1023 / L)) in fp64, clamped to [0, 1023].
__device__ __forceinline__ uint32_t morton_bin(float x, double scale) {
    double b = floor((double)x * scale);
    if (!(b >= 0.0)) b = 0.0;  // negative or NaN
    if (b > 1023.0) b = 1023.0;
    return (uint32_t)b;
}

__device__ __forceinline__ uint32_t morton_key(float x, float y, float z, double sx, double sy, double sz,
                                               int32_t type) {
    return spread10(morton_bin(x, sx)) | (spread10(morton_bin(y, sy)) << 1) | (spread10(morton_bin(z, sz)) << 2) |
           ((uint32_t)type << 30);
}

struct Segment {
    int32_t s, e;
};

// First position in [lo, hi) of sorted keys whose type (bits 30-31) is at
// least t; hi when there is none.
__device__ __forceinline__ int32_t type_start(const uint32_t *__restrict__ keys, int32_t lo, int32_t hi, uint32_t t) {
    while (lo < hi) {
        const int32_t mid = lo + ((hi - lo) >> 1);
        if ((keys[mid] >> 30) < t)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo;
}

// Particle run [first, first + count), count <= 16, as a negative reference.
__device__ __forceinline__ int32_t run_ref(int32_t first, int32_t count) {
    return ~((first << kRunCountBits) | (count - 1));
}

__device__ __forceinline__ uint32_t quantize_lo(float v, float root, double h, uint32_t qmax) {
    double q = floor(((double)v - (double)root) / h);
    if (!(q >= 0.0)) q = 0.0;
    if (q > (double)qmax) q = (double)qmax;
    return (uint32_t)q;
}

__device__ __forceinline__ uint32_t quantize_hi(float v, float root, double h, uint32_t qmax) {
    double q = ceil(((double)v - (double)root) / h);
    if (!(q >= 0.0)) q = 0.0;
    if (q > (double)qmax) q = (double)qmax;
    return (uint32_t)q;
}

__device__ __forceinline__ uint32_t quantize_axis(float lo, float hi, float root, double h, uint32_t qmax) {
    return quantize_lo(lo, root, h, qmax) | (quantize_hi(hi, root, h, qmax) << 16);
}

// Bin width along one axis of the paper's per-axis grid over a root box:
// max(hi - lo, ext_floor) / (2^b - 1) in fp64.
__host__ __device__ __forceinline__ double axis_spacing(float lo, float hi, double ext_floor, int32_t qbits) {
    double e = (double)hi - (double)lo;
    e = e > ext_floor ? e : ext_floor;
    return e / (double)((1 << qbits) - 1);
}

// Subtree collapse by cost (Section 2.3, last paragraph: build with one
// particle per leaf, then collapse subtrees by a heuristic).  For a search
// sphere of radius R, the chance that it meets a box is taken proportional to
// the volume of the box grown by R (Steiner's formula for an a x b x c box:
// abc + 2R(ab + bc + ca) + pi R^2 (a + b + c) + 4/3 pi R^3).  A node of at
// most leaf_size particles becomes a particle run when testing its particles
// (cost 1 each) costs no more than testing its children's boxes (one record,
// cost kRecordCost) plus the expected cost of the children; in volume-weighted
// form, with F the cost times the grown volume:
//   F(particle) = V(point)
//   F(node)     = min(count V(node), kRecordCost V(node) + F(left) + F(right))
// (the run when the first term is chosen).  fp32, in this order, with no
// fused multiply-add.  Collapse constants: k2R = 2R, kPiR2 = pi R^2,
// kVball = 4/3 pi R^3 (each computed in fp64, then rounded to fp32).
constexpr float kRecordCost = 4.0f;

struct Collapse {
    float k2R, kPiR2, kVball;  // kVball == 0: no cost model (runs are the subtrees of at most leaf_size)
    int32_t leaf_size;
};

__device__ __forceinline__ float grown_volume(const Collapse &c, float a, float b, float cz) {
    const float ab = a * b, bc = b * cz, ca = cz * a;
    return ((ab * cz + c.k2R * ((ab + bc) + ca)) + c.kPiR2 * ((a + b) + cz)) + c.kVball;
}

// F of a node of `count` particles with box lo/hi and children costs fl, fr;
// negative when the node becomes a run.
__device__ __forceinline__ float node_cost(const Collapse &c, int32_t count, float lx, float ly, float lz, float hx,
                                           float hy, float hz, float fl, float fr) {
    const float v = grown_volume(c, hx - lx, hy - ly, hz - lz);
    const float leafc = (float)count * v;
    const float split = kRecordCost * v + (fl + fr);
    return (count <= c.leaf_size && leafc <= split) ? -leafc : split;
}

// Tree description from the root box (exact fp32 min/max) of a segment;
// root_run: the whole tree is one particle run.
__device__ __forceinline__ TreeMeta tree_meta(const float lo[3], const float hi[3], double ext_floor, int32_t qbits,
                                              int32_t start, int32_t count, bool root_run,
                                              const uint32_t *__restrict__ P) {
    TreeMeta m;
    double ext = 0.0;
    for (int d = 0; d < 3; ++d) {
        m.lo[d] = lo[d];
        m.hi[d] = hi[d];
        const double e = (double)hi[d] - (double)lo[d];
        ext = e > ext ? e : ext;
    }
    ext = ext > ext_floor ? ext : ext_floor;
    m.h = ext / (double)((1 << qbits) - 1);
    m.inv_h = 1.0 / m.h;
    m.start = start;
    m.count = count;
    m.root = root_run ? run_ref(start, count > 0 ? count : 1) : (int32_t)P[start];
    m.end = (int32_t)P[start + count];
    m.pad[0] = m.pad[1] = 0;
    return m;
}

// Record of kept internal node i (a node with a record: particle range [f, l]
// longer than leaf_size, or with the cost model, kept_flag[i] set): both
// child boxes quantized against the tree's root box, both child references,
// written at its preorder position, plus its rope.  A child is a record when
// it is kept itself, otherwise a particle run.  The children are the left
// [f, g] and the right [g + 1, l] around the node's split g (ids g and g + 1
// when internal), so their ranges need no loads.
//
// Preorder position: the kept nodes starting before f (P[f]), then those
// starting at f that contain node i (they nest along a left spine and come
// before it in preorder; all of them are kept, being longer than i).  A node
// starting at f is a left child exactly when its id is not f (a left child
// takes the end of its range as id; a right child or a root takes f), so the
// ancestors starting at f are found by following parent links from i while
// the id differs from f: one load per step.
__device__ __forceinline__ void emit_record(int32_t i, int32_t f, int32_t l, const TreeMeta &m,
                                            const float4 *__restrict__ sorted, const int32_t *__restrict__ left,
                                            const int32_t *__restrict__ parent,
                                            const float4 *__restrict__ box,
                                            const uint32_t *__restrict__ P, int32_t leaf_size,
                                            const uint32_t *__restrict__ kept_flag, int32_t qbits,
                                            uint4 *__restrict__ records, int32_t *__restrict__ ropes) {
    const int32_t lc = left[i];
    const int32_t g = lc >= 0 ? lc : ~lc;
    const int32_t cf[2] = {f, g + 1}, cl[2] = {g, l};
    // A leaf child's box is its particle.
    float4 lo[2], hi[2];
#pragma unroll
    for (int side = 0; side < 2; ++side) {
        const bool leaf = cf[side] == cl[side];
        const int32_t k = side == 0 ? g : g + 1;
        lo[side] = *(leaf ? sorted + k : box + 2 * (int64_t)k);
        hi[side] = *(leaf ? sorted + k : box + 2 * (int64_t)k + 1);
    }
    const uint32_t right_rec = P[g + 1];
    const int32_t rope = (int32_t)P[l + 1];
    const uint32_t first_rec = P[f];
    // (issued after the loads above, so those overlap the chain)
    int32_t rank = 0;
    for (int32_t u = i; u != f && rank < kMaxDepth; ++rank) u = parent[u];
    const int32_t at = (int32_t)first_rec + rank;
    const float root[3] = {m.lo[0], m.lo[1], m.lo[2]};
    const double h = m.h;
    const uint32_t qmax = (1u << qbits) - 1u;
    uint32_t w[8];
#pragma unroll
    for (int side = 0; side < 2; ++side) {
        const int32_t count = cl[side] - cf[side] + 1;
        const int32_t id = side == 0 ? g : g + 1;
        const bool record = count > 1 && (kept_flag ? kept_flag[id] != 0u : count > leaf_size);
        int32_t ref;
        if (record)
            ref = side == 0 ? at + 1 : (int32_t)right_rec;
        else
            ref = run_ref(cf[side], count);
        w[3 * side + 0] = quantize_axis(lo[side].x, hi[side].x, root[0], h, qmax);
        w[3 * side + 1] = quantize_axis(lo[side].y, hi[side].y, root[1], h, qmax);
        w[3 * side + 2] = quantize_axis(lo[side].z, hi[side].z, root[2], h, qmax);
        w[6 + side] = (uint32_t)ref;
    }
    records[2 * (int64_t)at] = make_uint4(w[0], w[1], w[2], w[3]);
    records[2 * (int64_t)at + 1] = make_uint4(w[4], w[5], w[6], w[7]);
    ropes[at] = rope;
}

}  // namespace qbi

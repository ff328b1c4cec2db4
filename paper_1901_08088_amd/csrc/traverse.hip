// Neighbor-list traversal: one lane per Z-ordered particle, the lanes of a
// wavefront walking the rope-linked quantized tree together (Algorithm 1;
// Section 2.3; Section 3 runs the queries in Z order so that the lanes of a
// wavefront need similar subtrees).
//
// Per wavefront and per type tree:
//   1. image mask per lane: which of the 27 periodic images of its search
//      sphere touch the tree's root box (the image test of Algorithm 1); the wavefront
//      visits the union of its lanes' images;
//   2. per image, one stackless walk over the two-wide records, shared by the
//      wavefront.  A step loads one record (both child boxes and references)
//      and its rope with uniform (scalar) loads; every lane tests its own
//      sphere against both boxes in grid units (nearest point by a clamp per
//      axis, eq. (2)); a ballot over the lanes decides the step: the left
//      child's record if any lane hit that box, else the right child's record
//      if any lane hit that one, else the rope.  A lane whose sphere misses a
//      node misses everything below it, so the wavefront walks exactly the
//      union of the lanes' own walks and every record is fetched once for all
//      64 lanes instead of gathered lane by lane;
//   3. a hit particle run is fetched once (uniform loads) and decided by the
//      lanes that hit it: an fp32 distance with a proven error band accepts or
//      rejects almost every pair; pairs inside the band are decided with the
//      fp64 arithmetic of the list definition, so the result is the exact list.
//
// Grid-unit test.  With h the tree's bin width and g(x) = (x - root_lo) / h,
// a quantized bound q decodes exactly to the float 2^23 + q (bit trick: OR
// with 0x4B000000), and the query image is placed at 2^23 + g(x) rounded to
// fp32.  Rounding of the query position, of the differences and of the sum of
// squares is covered by comparing against
//   ((R / h) * (1 + 2^-20) + 2)^2 * (1 + 2^-20),
// a pad of two bins plus a relative 2^-20, so no true neighbor is lost.
//
// fp32 pair test.  With qs = fl(x_i + m L) per axis and a = fl(x_j - qs), each
// |a - dx| <= 2^-24 (2 L + |a|), so the computed distance differs from the
// definition's by at most eta = sqrt(3) 2^-22 (2 L_max + 2 R) while the pair
// is near the cutoff.  Pairs with d32^2 <= ((R - eta)(1 - 2^-20))^2 are in,
// pairs with d32^2 > ((R + eta)(1 + 2^-20))^2 are out, the rest (a shell a few
// 1e-4 wide) take the fp64 path.
#include "build_common.h"

namespace qbi {
namespace {

// Decoding a 16-bit bound q of a record word held in a scalar register: the
// float with bits 0x4B000000 | q is exactly 2^23 + q.  The lower bound is
// decoded by the scalar unit (s_pack_ll_b32_b16 puts 0x4B00 above the low half
// word), the upper one by the VALU (v_or_b32 with a 16-bit source select of
// the scalar word against the bias held in a VGPR).  Splitting the decodes
// balances the two issue slots of the shared walk, and leaves the clamp with
// one scalar and one vector bound (a VALU op may read one scalar operand).
__device__ __forceinline__ uint32_t vgpr_bias() {
    uint32_t v;
    asm volatile("v_mov_b32 %0, 0x4b000000" : "=v"(v));
    return v;
}

__device__ __forceinline__ float lo_bound(uint32_t w) {
    float r;
    asm("s_pack_ll_b32_b16 %0, %1, 0x4b00" : "=s"(r) : "s"(w));
    return r;
}

__device__ __forceinline__ float hi_bound(uint32_t w, uint32_t bias) {
    float r;
    asm("v_or_b32_sdwa %0, %1, %2 dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:WORD_1 src1_sel:DWORD"
        : "=v"(r)
        : "s"(w), "v"(bias));
    return r;
}

// Squared grid-unit distance from the query (ux, uy, uz) to a packed box.
__device__ __forceinline__ float box_d2(uint32_t wx, uint32_t wy, uint32_t wz, float ux, float uy, float uz,
                                        uint32_t bias) {
    const float cx = __builtin_amdgcn_fmed3f(ux, lo_bound(wx), hi_bound(wx, bias)) - ux;
    const float cy = __builtin_amdgcn_fmed3f(uy, lo_bound(wy), hi_bound(wy, bias)) - uy;
    const float cz = __builtin_amdgcn_fmed3f(uz, lo_bound(wz), hi_bound(wz, bias)) - uz;
    return __builtin_fmaf(cz, cz, __builtin_fmaf(cy, cy, cx * cx));
}

__device__ __forceinline__ int32_t uniform(int32_t x) { return __builtin_amdgcn_readfirstlane(x); }

// Row staging.  Each lane keeps its newest list entries in a ring of kRing
// LDS slots (its own column, so lanes never share a bank row) and writes them
// to its row kFlush at a time: with 16-byte aligned rows as two 16-byte
// stores.  A candidate's index is written to the lane's next free slot
// whether or not it is accepted, and the count advances only on acceptance,
// so the per-candidate path has no branch.  Runs are taken 8 particles at a
// time and the ring is flushed after each such part once kFlush entries wait,
// so no more than 15 entries are ever pending.
constexpr int kRing = 16;
constexpr int kFlush = 8;

struct Lane {
    float x, y, z;         // query position
    float qsx, qsy, qsz;   // fl(query + image shift)
    float ux, uy, uz;      // query image in grid units (2^23 offset form)
    float r2g;             // padded squared radius in grid units (negative: lane idle)
    float r2in, r2out;     // fp32 accept / reject thresholds
    double r2;             // exact squared list radius
    int32_t k, orig;
    int32_t cnt;           // entries of the list so far
    int32_t flushed;       // entries already written to the row (a multiple of kFlush)
    float px, py, pz;      // paper mode: query image in per-axis grid units (plain, not offset)
    float phx, phy, phz;   // paper mode: bin width of each axis
    float rp2;             // paper mode: squared tight radius (world units)
};

template <bool kVec4, int kBlock>
__device__ __forceinline__ void flush_ring(Lane &q, int32_t (*s_out)[kBlock], int32_t *nbr, int32_t max_nbr) {
    const int32_t f = q.flushed;
    const int s0 = f & (kRing - 1);
    int32_t *row = nbr + ((int64_t)q.orig * max_nbr + f);
    if (kVec4) {
        // f and max_nbr are multiples of 4 here; one compare covers the usual
        // case of a row with room for all eight
        const int4 lo = make_int4(s_out[s0][threadIdx.x], s_out[s0 + 1][threadIdx.x], s_out[s0 + 2][threadIdx.x],
                                  s_out[s0 + 3][threadIdx.x]);
        if (f <= max_nbr - 8) {
            *reinterpret_cast<int4 *>(row) = lo;
            *reinterpret_cast<int4 *>(row + 4) = make_int4(s_out[s0 + 4][threadIdx.x], s_out[s0 + 5][threadIdx.x],
                                                           s_out[s0 + 6][threadIdx.x], s_out[s0 + 7][threadIdx.x]);
        } else if (f <= max_nbr - 4) {
            *reinterpret_cast<int4 *>(row) = lo;
        }
    } else {
#pragma unroll
        for (int e = 0; e < kFlush; ++e)
            if (f + e < max_nbr) row[e] = s_out[s0 + e][threadIdx.x];
    }
    q.flushed = f + kFlush;
}

// The candidate's original index, inverted from its float4 w word (held in a
// scalar register) straight into a VGPR: one VALU op, no scalar op.
__device__ __forceinline__ int32_t orig_of(float w) {
    int32_t r;
    asm("v_not_b32 %0, %1" : "=v"(r) : "s"(__float_as_int(w)));
    return r;
}

// Particle u of a run, addressed as the array base plus a byte offset.
__device__ __forceinline__ float4 particle(const char *__restrict__ base, uint32_t off, uint32_t u) {
    return reinterpret_cast<const float4 *>(base + off)[u];
}

// fp32 pass over the particles of a run for every lane.  Accepts what is
// surely in (d2 <= thr; thr = r2in for hitting lanes, -1 otherwise) and
// returns whether some lane has a pair in the shell (thr, out] (out = r2out
// for hitting lanes, -1 otherwise), which then needs the exact test.  The
// whole run (8 float4, padding included) is fetched with uniform loads up
// front.  kSelf: the run may hold the lane's own particle at index `rel`,
// which is never listed (nor taken as a shell pair).
template <bool kSelf, int kBlock>
__device__ __forceinline__ bool run_fp32(const char *__restrict__ base, uint32_t roff, uint32_t count, uint32_t rel,
                                         float thr, float out, Lane &q, int32_t (*s_out)[kBlock]) {
    float4 p[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) p[u] = particle(base, roff, (uint32_t)u);
    // both halves of the run are requested before the first test (the
    // compiler would otherwise delay the second load behind the early exits)
    asm volatile("" ::"s"(p[0].x), "s"(p[4].x));
    // lanes with a pair in the shell: the band masks are combined on the
    // scalar unit, which leaves the VALU one compare per candidate for them
    uint64_t band = 0;
#pragma unroll
    for (int u = 0; u < 8; ++u) {
        if ((uint32_t)u >= count) break;
        const float ax = p[u].x - q.qsx, ay = p[u].y - q.qsy, az = p[u].z - q.qsz;
        const float d2 = __builtin_fmaf(az, az, __builtin_fmaf(ay, ay, ax * ax));
        const bool other = !kSelf || (uint32_t)u != rel;
        const bool in = d2 <= thr && other;
        s_out[q.cnt & (kRing - 1)][threadIdx.x] = orig_of(p[u].w);
        q.cnt += in ? 1 : 0;
        band |= __ballot(d2 <= out && other) & ~__ballot(in);
    }
    return band != 0;
}

// Sparse runs.  When at most 8 lanes hit a run, testing every particle on
// all 64 lanes wastes most of them.  Instead each lane takes one
// (hitting lane, particle) pair: lane l takes particle l % 8 of the (l / 8)-th
// hitting lane (lanes whose particle index reaches the run length idle).  The
// query's image and thresholds come from its lane by a cross-lane read, the
// particle by a vector load.  An accepted pair is written into the ring of its
// query's lane at that lane's count plus the number of accepted pairs of the
// same query before it, so every row receives exactly the entries, in exactly
// the order, of the per-lane pass.  Returns whether some pair fell in the
// shell (thr, out] (then the caller decides the shell exactly).  Never used
// for runs that may hold a lane's own particle.  s_src is the wavefront's
// 64-entry LDS table rank -> lane.  Every cross-lane read runs on all lanes:
// a lane left out of one would hand its readers 0.
template <int kBlock>
__device__ __forceinline__ bool run_sparse(const char *__restrict__ base, uint32_t roff, uint32_t count, bool hit,
                                           uint64_t hits,
                                           float thr, float out, Lane &q, int32_t (*s_out)[kBlock],
                                           int32_t *s_src) {
    const uint32_t lane = __lane_id();
    const uint32_t i = lane >> 3, j = lane & 7u;
    const uint32_t h = (uint32_t)__popcll(hits);
    const bool pv = i < h && j < count;
    const float4 p = particle(base, roff, j);  // j < 8: inside the run or its padding
    const uint32_t rank =
        __builtin_amdgcn_mbcnt_hi((uint32_t)(hits >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)hits, 0u));
    if (hit) s_src[rank] = (int32_t)lane;
    __builtin_amdgcn_wave_barrier();
    const int32_t src = s_src[i < h ? i : 0u];
    const float sx = __shfl(q.qsx, src), sy = __shfl(q.qsy, src), sz = __shfl(q.qsz, src);
    const float th = __shfl(thr, src), ou = __shfl(out, src);
    const int32_t c0 = __shfl(q.cnt, src);
    const float ax = p.x - sx, ay = p.y - sy, az = p.z - sz;
    const float d2 = __builtin_fmaf(az, az, __builtin_fmaf(ay, ay, ax * ax));
    const bool acc = pv && d2 <= th;
    const bool shell = __any(pv && !(d2 <= th) && d2 <= ou);
    const uint64_t A = __ballot(acc);
    const uint32_t below = __builtin_amdgcn_mbcnt_hi((uint32_t)(A >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)A, 0u));
    const uint32_t below0 = (uint32_t)__shfl((int32_t)below, (int32_t)(lane & ~7u));
    if (acc) {
        const uint32_t pos = (uint32_t)c0 + below - below0;
        s_out[pos & (kRing - 1)][(threadIdx.x & ~63u) + (uint32_t)src] = ~__float_as_int(p.w);
    }
    // every hitting lane adds the accepted pairs of its own 8 lanes
    const uint32_t e0 = (rank & 7u) << 3;
    const uint32_t b0 = (uint32_t)__shfl((int32_t)below, (int32_t)e0);
    const uint32_t b1r = (uint32_t)__shfl((int32_t)below, (int32_t)((e0 + 8u) & 63u));
    const uint32_t b1 = e0 + 8u < 64u ? b1r : (uint32_t)__popcll(A);
    if (hit) q.cnt += (int32_t)(b1 - b0);
    return shell;
}

// 16-bit bound of a record-style word held in a scalar register, as a float.
__device__ __forceinline__ float cvt_lo(uint32_t w) {
    float r;
    asm("v_cvt_f32_u32_sdwa %0, %1 dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:WORD_0" : "=v"(r) : "s"(w));
    return r;
}

__device__ __forceinline__ float cvt_hi(uint32_t w) {
    float r;
    asm("v_cvt_f32_u32_sdwa %0, %1 dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:WORD_1" : "=v"(r) : "s"(w));
    return r;
}

// Paper-mode pass (Section 2.3): a particle of the run is listed when the
// lane's sphere overlaps the particle's own cell box (its leaf box in the
// quantized tree, on the paper's per-axis grid), with no distance check.  The
// nearest point is found in each axis's grid units and scaled to world units
// by that axis's bin width; the test is against the tight radius
// R (1 + 2^-20) + 0.02 max_d h_d.
template <bool kSelf, int kBlock>
__device__ __forceinline__ void run_paper(const uint4 *__restrict__ qrun, uint32_t count, uint32_t rel, bool hit,
                                          Lane &q, int32_t (*s_out)[kBlock]) {
    uint4 b[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) b[u] = qrun[u];
    asm volatile("" ::"s"(b[0].x), "s"(b[4].x));
    const float r2 = hit ? q.rp2 : -1.0f;
#pragma unroll
    for (int u = 0; u < 8; ++u) {
        if ((uint32_t)u >= count) break;
        const float cx = (__builtin_amdgcn_fmed3f(q.px, cvt_lo(b[u].x), cvt_hi(b[u].x)) - q.px) * q.phx;
        const float cy = (__builtin_amdgcn_fmed3f(q.py, cvt_lo(b[u].y), cvt_hi(b[u].y)) - q.py) * q.phy;
        const float cz = (__builtin_amdgcn_fmed3f(q.pz, cvt_lo(b[u].z), cvt_hi(b[u].z)) - q.pz) * q.phz;
        const float d2 = __builtin_fmaf(cz, cz, __builtin_fmaf(cy, cy, cx * cx));
        const bool other = !kSelf || (uint32_t)u != rel;
        s_out[q.cnt & (kRing - 1)][threadIdx.x] = (int32_t)b[u].w;
        q.cnt += (d2 <= r2 && other) ? 1 : 0;
    }
}

// Decide the particles of one hit run for the lanes with `hit` set.  A run
// of up to 16 particles is taken in halves of at most 8: each half adds at
// most 8 entries to a ring holding fewer than kFlush, and the ring is
// flushed after every half.
template <bool kVec4, int kBlock, bool kPaper, bool kF64, class LArr>
__device__ __forceinline__ void take_run(int32_t ref, bool hit, uint64_t hits, Lane &q, int img, const LArr &L,
                                         const float4 *__restrict__ sorted, const uint4 *__restrict__ qpoint,
                                         const double *__restrict__ sorted64, uint32_t nend,
                                         int32_t (*s_out)[kBlock], int32_t *s_src, int32_t *nbr, int32_t max_nbr) {
    const int32_t v = ~ref;
    const uint32_t first = (uint32_t)uniform(v >> kRunCountBits);
    const uint32_t count = (uint32_t)uniform((v & kRunCountMask) + 1);
    // a well-formed tree never fails this; it keeps a corrupt reference from
    // reading outside the particle array
    if (first + count > nend) return;
    const float thr = hit ? q.r2in : -1.0f;
    const float out = hit ? q.r2out : -1.0f;
    // (two 32-bit counts keep the comparison on the scalar unit)
    const bool sparse = __popc((uint32_t)hits) + __popc((uint32_t)(hits >> 32)) <= 8;
    for (uint32_t h0 = 0; h0 < count; h0 += 8) {
        const uint32_t c8 = count - h0 < 8u ? count - h0 : 8u;
        const char *sbase = reinterpret_cast<const char *>(sorted);
        const uint32_t roff = (first + h0) * 16u;
        // the lane's own particle can only be accepted through the unshifted image
        const uint32_t rel = (uint32_t)(q.k - (int32_t)(first + h0));
        const bool self = img == 13 && __any(hit && rel < c8);
        if (kPaper) {
            if (self)
                run_paper<true, kBlock>(qpoint + first + h0, c8, rel, hit, q, s_out);
            else
                run_paper<false, kBlock>(qpoint + first + h0, c8, rel, hit, q, s_out);
        } else {
            bool shell;
            if (!self && sparse) {
                shell = run_sparse<kBlock>(sbase, roff, c8, hit, hits, thr, out, q, s_out, s_src);
            } else {
                shell = self ? run_fp32<true, kBlock>(sbase, roff, c8, rel, thr, out, q, s_out)
                             : run_fp32<false, kBlock>(sbase, roff, c8, rel, thr, out, q, s_out);
            }
            if (shell) {
                // some pair lies in the shell around the cutoff: decide the
                // shell pairs with the definition's fp64 arithmetic
                const double sx = (double)(img % 3 - 1) * L[0];
                const double sy = (double)((img / 3) % 3 - 1) * L[1];
                const double sz = (double)(img / 9 - 1) * L[2];
                // fp64 data: the query's and the candidates' own fp64 positions
                const double *q64 = kF64 ? sorted64 + 4 * (int64_t)(hit ? q.k : (int32_t)first) : nullptr;
                const double qx = kF64 ? q64[0] : (double)q.x, qy = kF64 ? q64[1] : (double)q.y,
                             qz = kF64 ? q64[2] : (double)q.z;
                for (uint32_t j = 0; j < c8; ++j) {
                    const float4 p = particle(sbase, roff, j);
                    const float ax = p.x - q.qsx, ay = p.y - q.qsy, az = p.z - q.qsz;
                    const float d2 = __builtin_fmaf(az, az, __builtin_fmaf(ay, ay, ax * ax));
                    if (hit && !(d2 <= thr) && d2 <= q.r2out && j != rel) {
                        const double *p64 = kF64 ? sorted64 + 4 * (int64_t)(first + h0 + j) : nullptr;
                        const double dx = ((kF64 ? p64[0] : (double)p.x) - qx) - sx;
                        const double dy = ((kF64 ? p64[1] : (double)p.y) - qy) - sy;
                        const double dz = ((kF64 ? p64[2] : (double)p.z) - qz) - sz;
                        if ((dx * dx + dy * dy) + dz * dz <= q.r2) {
                            s_out[q.cnt & (kRing - 1)][threadIdx.x] = ~__float_as_int(p.w);
                            ++q.cnt;
                        }
                    }
                }
            }
        }
        // a plain per-lane branch: the wavefront skips it when no lane's
        // condition holds, with one compare instead of a ballot and a test
        if (q.cnt - q.flushed >= kFlush)
            flush_ring<kVec4, kBlock>(q, s_out, nbr, max_nbr);
    }
}

// The read-only arrays come as separate __restrict__ parameters: that lets the
// compiler fetch wave-uniform records and particles with scalar loads.
template <bool kVec4, int kBlock, bool kPaper, bool kF64, class Args>
__device__ __forceinline__ void traverse_block(Args &a, int32_t li, const uint4 *__restrict__ records,
                                               const int32_t *__restrict__ ropes,
                                               const float4 *__restrict__ sorted,
                                               const uint4 *__restrict__ qpoint,
                                               const double *__restrict__ sorted64,
                                               const TreeMeta *__restrict__ meta, int32_t (*s_out)[kBlock],
                                               int32_t (*s_src)[64]);

// Workgroups are dealt round-robin to the 8 XCDs; each XCD gets one
// contiguous stretch of the Z-ordered queries so its L2 holds one region.
__device__ __forceinline__ int32_t xcd_logical_block() {
    const uint32_t nb = gridDim.x, b = blockIdx.x;
    const uint32_t xcd = b & 7u, qq = nb >> 3, rr = nb & 7u;
    return (int32_t)(xcd * qq + (xcd < rr ? xcd : rr) + (b >> 3));
}

// Query order.  A system of one type takes its queries in sorted (Z) order,
// a.qpw per wavefront.  In a system of several types, the workgroups form
// eight equal stretches (one per XCD when the system covers the whole
// launch); stretch x takes the x-th eighth of every type's queries, smallest
// type first, in wavefronts of type_qpw queries of one type.  A sparse type's
// wavefronts span the widest regions and run longest: this way they start
// first, are spread over the stretches, and each takes few queries, instead
// of closing the launch on one XCD.  `wg` is the system's workgroup in
// dispatch order and `nwg` its workgroup count (trav_blocks, an upper bound
// for several types); returns the lane's position in the system, or a.n for
// an idle lane.
template <int kBlock, class Args>
__device__ __forceinline__ int32_t query_position(Args &a, const TreeMeta *__restrict__ meta, int32_t wg,
                                                  int32_t nwg) {
    const int32_t lane = (int32_t)(threadIdx.x & 63u), wave = (int32_t)(threadIdx.x >> 6);
    if (a.ntypes <= 1) {
        // wavefronts of a.qpw queries: lanes past a.qpw idle
        const int32_t qpw = a.qpw;
        if (lane >= qpw) return a.n;
        return (wg * (kBlock / 64) + wave) * qpw + lane;
    }
    const int32_t per = nwg / 8;
    const int64_t part = wg / per;
    int32_t wi = (wg % per) * (kBlock / 64) + wave;  // wavefront of the stretch
    for (int r = 0; r < a.ntypes; ++r) {
        // the type of rank r by (count, type index)
        int t = 0;
        for (int u = 0; u < a.ntypes; ++u) {
            int rank = 0;
            for (int w = 0; w < a.ntypes; ++w)
                rank += (meta[w].count < meta[u].count || (meta[w].count == meta[u].count && w < u)) ? 1 : 0;
            if (rank == r) t = u;
        }
        const int64_t len = meta[t].count;
        const int32_t lo = stretch_lo(len, part), hi = stretch_lo(len, part + 1);
        const int32_t qt = type_qpw(len, a.n, a.qpw);
        const int32_t nw = type_waves(len, a.n, a.qpw, part);
        if (wi < nw) {
            const int32_t j = wi * qt + lane;
            return (lane < qt && j < hi - lo) ? meta[t].start - a.start + lo + j : a.n;
        }
        wi -= nw;
    }
    return a.n;
}

template <bool kVec4, int kBlock, bool kPaper, bool kF64>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(8))) void k_traverse(
    TravArgs a, const uint4 *__restrict__ records, const int32_t *__restrict__ ropes,
    const float4 *__restrict__ sorted, const uint4 *__restrict__ qpoint, const TreeMeta *__restrict__ meta) {
    __shared__ int32_t s_out[kRing][kBlock];
    __shared__ int32_t s_src[kBlock / 64][64];
    const int32_t li = query_position<kBlock>(a, meta, xcd_logical_block(), (int32_t)gridDim.x);
    traverse_block<kVec4, kBlock, kPaper, kF64, const TravArgs>(a, li, records, ropes, sorted, qpoint, a.sorted64, meta,
                                                                s_out, s_src);
}

// Batched form: the workgroups of all systems form one grid; each workgroup
// belongs to one system (found from the per-system first-workgroup table) and
// reads that system's arguments from the device table, so every per-system
// value stays wave-uniform.
template <bool kVec4, int kBlock>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(8))) void k_traverse_batch(
    const TravArgs *__restrict__ table, const int32_t *__restrict__ tblk_first, int32_t nsys,
    const uint4 *__restrict__ records, const int32_t *__restrict__ ropes, const float4 *__restrict__ sorted,
    const TreeMeta *__restrict__ meta_all) {
    __shared__ int32_t s_out[kRing][kBlock];
    __shared__ int32_t s_src[kBlock / 64][64];
    const int32_t logical = xcd_logical_block();
    const int32_t sys = find_seg(tblk_first, nsys, logical);
    // the system's arguments are read through the constant address space, as
    // kernel arguments are: the compiler may then fetch a field again where it
    // is needed instead of holding it in registers through the walk
    using ConstArgs = const TravArgs __attribute__((address_space(4)));
    ConstArgs *args = reinterpret_cast<ConstArgs *>(reinterpret_cast<uintptr_t>(table + sys));
    const TreeMeta *meta = meta_all + sys * QBVH_MAX_TYPES;
    const int32_t li = query_position<kBlock>(*args, meta, logical - tblk_first[sys], tblk_first[sys + 1] - tblk_first[sys]);
    traverse_block<kVec4, kBlock, false, false, ConstArgs>(*args, li, records, ropes, sorted, nullptr, nullptr, meta,
                                                           s_out, s_src);
}

// One workgroup of queries; this lane's query is position `li` of the system
// `a` (li >= a.n: an idle lane).
template <bool kVec4, int kBlock, bool kPaper, bool kF64, class Args>
__device__ __forceinline__ void traverse_block(Args &a, int32_t li, const uint4 *__restrict__ records,
                                               const int32_t *__restrict__ ropes,
                                               const float4 *__restrict__ sorted,
                                               const uint4 *__restrict__ qpoint,
                                               const double *__restrict__ sorted64,
                                               const TreeMeta *__restrict__ meta, int32_t (*s_out)[kBlock],
                                               int32_t (*s_src_all)[64]) {
    int32_t *s_src = s_src_all[threadIdx.x >> 6];
    const bool valid = li < a.n;  // idle lanes still take part in the shared walk
    const int32_t k = a.start + li;
    const uint32_t nend = (uint32_t)(a.start + a.n);

    Lane q;
    const float4 qp = sorted[valid ? k : a.start];
    q.x = qp.x;
    q.y = qp.y;
    q.z = qp.z;
    q.k = k;
    q.orig = ~__float_as_int(qp.w);
    int ta = 0;
    for (int t = 1; t < a.ntypes; ++t)
        if (k >= meta[t].start) ta = t;

    q.cnt = 0;
    q.flushed = 0;
    const uint32_t bias = vgpr_bias();
    for (int tb = 0; tb < a.ntypes; ++tb) {
        const TreeMeta &m = meta[tb];
        if (m.count == 0) continue;
        double r2 = a.rlist2[tb];
        for (int t = 1; t < a.ntypes; ++t)
            if (ta == t) r2 = a.rlist2[t * QBVH_MAX_TYPES + tb];
        const bool lane_on = valid && r2 >= 0.0;
        q.r2 = r2;
        const double R = lane_on ? sqrt(r2) : 0.0;

        // (1) image mask against the root box (the image test of Algorithm 1), in fp32
        // with an outward pad of 2^-18 of the largest box edge (far above the
        // fp32 rounding of the shifted coordinates) plus 2^-20 relative.
        uint32_t bits = 0;
        if (lane_on) {
            const float pad = (float)(a.lmax * 0x1p-18);
            const float rimg = (float)R * (1.0f + 0x1p-20f) + pad;
            const float rimg2 = rimg * rimg;
            float e2[3][3];
            const float xq[3] = {q.x, q.y, q.z};
#pragma unroll
            for (int dd = 0; dd < 3; ++dd) {
#pragma unroll
                for (int sh = 0; sh < 3; ++sh) {
                    const float p = xq[dd] + (float)(sh - 1) * a.Lf[dd];
                    const float e = fmaxf(fmaxf(m.lo[dd] - p, p - m.hi[dd]), 0.0f);
                    e2[dd][sh] = e * e;
                }
            }
#pragma unroll
            for (int img = 0; img < 27; ++img) {
                const float sum = (e2[0][img % 3] + e2[1][(img / 3) % 3]) + e2[2][img / 9];
                if (sum <= rimg2) bits |= 1u << img;
            }
        }
        uint32_t wave_bits = bits;
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) wave_bits |= (uint32_t)__shfl_xor((int)wave_bits, o, 64);
        wave_bits = (uint32_t)uniform((int32_t)wave_bits);

        // fp64 data: the tree and the query are the data rounded to fp32, which
        // moves each point by up to 2^-24 L_max per axis, so a pair's distance
        // by up to sqrt(3) 2^-23 L_max; the node test widens the sphere by that
        // much before the two-bin pad (which alone covers it only when the
        // tree's root box is not much smaller than the periodic box)
        const double rshift = kF64 ? 1.7320508075688772 * 0x1p-23 * a.lmax : 0.0;
        const double rg = (R + rshift) * m.inv_h;
        const double rgp = rg * (1.0 + 0x1p-20) + 2.0;
        const float r2g = lane_on ? (float)(rgp * rgp * (1.0 + 0x1p-20)) : -1.0f;
        // fp64 data adds the rounding of both points to fp32 (2^-24 L each per
        // axis); the band is doubled for it
        const double eta = (kF64 ? 2.0 : 1.0) * 1.7320508075688772 * 0x1p-22 * (2.0 * a.lmax + 2.0 * R);
        const double rin = fmax(R - eta, 0.0) * (1.0 - 0x1p-20);
        const double rout = (R + eta) * (1.0 + 0x1p-20);
        q.r2in = (float)(rin * rin * (1.0 - 0x1p-20));
        q.r2out = (float)(rout * rout * (1.0 + 0x1p-20));
        const int32_t root = m.root, end = m.end;
        double ph[3] = {1.0, 1.0, 1.0};
        if (kPaper) {
            // the paper's per-axis bins (as the cell boxes were quantized); the
            // pad covers the rounding of the query's grid position (at most
            // 2^-24 of 65535 bins per axis) and of the fp32 distance
            double hmax = 0.0;
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                ph[d] = axis_spacing(m.lo[d], m.hi[d], a.lmax * 0x1p-24, a.qbits);
                hmax = ph[d] > hmax ? ph[d] : hmax;
            }
            q.phx = (float)ph[0];
            q.phy = (float)ph[1];
            q.phz = (float)ph[2];
            const double rp = R * (1.0 + 0x1p-20) + 0.02 * hmax;
            q.rp2 = (float)(rp * rp * (1.0 + 0x1p-20));
        }

        // (2) one shared stackless walk per image in the union (the walk of Algorithm 1)
        while (wave_bits) {
            const int img = __builtin_ctz(wave_bits);
            wave_bits &= wave_bits - 1u;
            const bool on = (bits >> img) & 1u;
            q.r2g = on ? r2g : -1.0f;
            const double sx = (double)(img % 3 - 1) * a.L[0];
            const double sy = (double)((img / 3) % 3 - 1) * a.L[1];
            const double sz = (double)(img / 9 - 1) * a.L[2];
            q.qsx = (float)((double)q.x + sx);
            q.qsy = (float)((double)q.y + sy);
            q.qsz = (float)((double)q.z + sz);
            q.ux = (float)((((double)q.x + sx) - (double)m.lo[0]) * m.inv_h + 8388608.0);
            q.uy = (float)((((double)q.y + sy) - (double)m.lo[1]) * m.inv_h + 8388608.0);
            q.uz = (float)((((double)q.z + sz) - (double)m.lo[2]) * m.inv_h + 8388608.0);
            if (kPaper) {
                q.px = (float)((((double)q.x + sx) - (double)m.lo[0]) / ph[0]);
                q.py = (float)((((double)q.y + sy) - (double)m.lo[1]) / ph[1]);
                q.pz = (float)((((double)q.z + sz) - (double)m.lo[2]) / ph[2]);
            }
            if (root < 0) {  // a tree of at most leaf_size particles is one run
                take_run<kVec4, kBlock, kPaper, kF64>(root, on, __ballot(on), q, img, a.L, sorted, qpoint, sorted64,
                                                      nend, s_out,
                                                s_src, a.nbr, a.max_nbr);
                continue;
            }
            int32_t v = root;
            while (v < end) {
                // 32-bit byte offsets keep the address arithmetic to one scalar op
                const uint32_t off = (uint32_t)v << 5;
                const uint4 r0 = *reinterpret_cast<const uint4 *>(reinterpret_cast<const char *>(records) + off);
                const uint4 r1 = *reinterpret_cast<const uint4 *>(reinterpret_cast<const char *>(records) + off + 16u);
                const int32_t rope =
                    *reinterpret_cast<const int32_t *>(reinterpret_cast<const char *>(ropes) + ((uint32_t)v << 2));
                const bool hl = box_d2(r0.x, r0.y, r0.z, q.ux, q.uy, q.uz, bias) <= q.r2g;
                const uint64_t ml = __ballot(hl);
                const bool anyl = ml != 0;
                const int32_t cl = (int32_t)r1.z, cr = (int32_t)r1.w;
                if (cl < 0 && anyl)
                    take_run<kVec4, kBlock, kPaper, kF64>(cl, hl, ml, q, img, a.L, sorted, qpoint, sorted64, nend,
                                                          s_out, s_src, a.nbr, a.max_nbr);
                // Descending into an internal left child with an internal right
                // child, the right box is not needed: the walk reaches the right
                // child's record by the left subtree's rope and tests its
                // children there (they lie inside its box).
                int32_t next = cl;
                if (!(anyl && cl >= 0 && cr >= 0)) {
                    const bool hr = box_d2(r0.w, r1.x, r1.y, q.ux, q.uy, q.uz, bias) <= q.r2g;
                    const uint64_t mr = __ballot(hr);
                    const bool anyr = mr != 0;
                    if (cr < 0 && anyr)
                        take_run<kVec4, kBlock, kPaper, kF64>(cr, hr, mr, q, img, a.L, sorted, qpoint, sorted64, nend,
                                                              s_out, s_src, a.nbr, a.max_nbr);
                    next = (anyl && cl >= 0) ? cl : ((anyr && cr >= 0) ? cr : rope);
                }
                // references always point forward; max() makes progress unconditional
                v = uniform(max(next, v + 1));
            }
        }
    }

    if (!valid) return;
    a.count[q.orig] = q.cnt;
    // the last (fewer than kFlush) entries
    const int32_t f = q.flushed, s0 = f & (kRing - 1);
    int32_t *row = a.nbr + ((int64_t)q.orig * a.max_nbr + f);
    for (int32_t e = 0; e < q.cnt - f; ++e)
        if (f + e < a.max_nbr) row[e] = s_out[(s0 + e) & (kRing - 1)][threadIdx.x];
    if (q.cnt > a.max_nbr) atomicOr(a.overflow, 1);
}

__global__ void k_clear_flag(int32_t *f) {
    if (threadIdx.x == 0) *f = 0;
}

template <bool kVec4, int kBlock, bool kPaper, bool kF64>
void launch_one(const TravArgs &a, const uint4 *qpoint, hipStream_t s) {
    const unsigned grid = (unsigned)trav_blocks(a.n, a.ntypes, kBlock, a.qpw);
    hipLaunchKernelGGL((k_traverse<kVec4, kBlock, kPaper, kF64>), dim3(grid), dim3(kBlock), 0, s, a, a.records,
                       a.ropes, a.sorted, qpoint, a.meta);
}

template <bool kVec4, int kBlock>
void launch_one_batch(const BatchLaunch &b, hipStream_t s) {
    hipLaunchKernelGGL((k_traverse_batch<kVec4, kBlock>), dim3((unsigned)b.tblocks), dim3(kBlock), 0, s, b.trav,
                       b.tblk_first, b.nsys, b.ws.records, b.ws.ropes, b.ws.sorted, b.meta);
}

template <bool kVec4, bool kPaper, bool kF64>
void launch_block(const TravArgs &a, int32_t block, const uint4 *qpoint, hipStream_t s) {
    switch (block) {
    case 64: launch_one<kVec4, 64, kPaper, kF64>(a, qpoint, s); break;
    case 128: launch_one<kVec4, 128, kPaper, kF64>(a, qpoint, s); break;
    case 192: launch_one<kVec4, 192, kPaper, kF64>(a, qpoint, s); break;
    default: launch_one<kVec4, 256, kPaper, kF64>(a, qpoint, s); break;
    }
}

template <bool kVec4>
void launch_block_batch(const BatchLaunch &b, hipStream_t s) {
    switch (b.block_size) {
    case 64: launch_one_batch<kVec4, 64>(b, s); break;
    case 128: launch_one_batch<kVec4, 128>(b, s); break;
    case 192: launch_one_batch<kVec4, 192>(b, s); break;
    default: launch_one_batch<kVec4, 256>(b, s); break;
    }
}

}  // namespace

hipError_t launch_traverse(const TravArgs &a, int32_t block, bool vec4, bool paper, const uint4 *qpoint,
                           hipStream_t s) {
    hipLaunchKernelGGL(k_clear_flag, dim3(1), dim3(64), 0, s, a.overflow);
    if (a.n > 0) {
        if (paper) {  // fp32 data only
            if (vec4)
                launch_block<true, true, false>(a, block, qpoint, s);
            else
                launch_block<false, true, false>(a, block, qpoint, s);
        } else if (a.sorted64) {
            if (vec4)
                launch_block<true, false, true>(a, block, nullptr, s);
            else
                launch_block<false, false, true>(a, block, nullptr, s);
        } else {
            if (vec4)
                launch_block<true, false, false>(a, block, nullptr, s);
            else
                launch_block<false, false, false>(a, block, nullptr, s);
        }
    }
    return hipGetLastError();
}

// The overflow flags of a batch are cleared by the batch's first kernel.
hipError_t launch_traverse_batch(const BatchLaunch &b, hipStream_t s) {
    if (b.tblocks > 0) {
        if (b.vec4)
            launch_block_batch<true>(b, s);
        else
            launch_block_batch<false>(b, s);
    }
    return hipGetLastError();
}

}  // namespace qbi

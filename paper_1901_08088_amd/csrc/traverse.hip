// Neighbor-list traversal: one lane per Z-ordered particle, stackless walk of
// the rope-linked quantized tree (Algorithm 1; Section 2.3; Section 3 runs the
// queries in Z order so that the lanes of a wavefront walk similar subtrees).
//
// Per lane and per type tree:
//   1. image mask: which of the 27 periodic images of the search sphere touch
//      the tree's root box (Algorithm 1, line 4);
//   2. for each such image a walk over the two-wide records from the root to
//      the tree's end.  A step loads one record (both child boxes, both child
//      references) and its rope, and tests the sphere against both boxes in
//      grid units (nearest point by a clamp per axis, eq. (2)).  A hit
//      particle run is pushed into the lane's candidate buffer in LDS; the
//      walk continues at the left child's record if that box is hit, else at
//      the right child's record if that box is hit, else along the rope.
//      Every step runs the same instruction sequence on every lane;
//   3. whenever some lane's buffer is nearly full, and after every image, the
//      active lanes of the wavefront decide their candidates together with
//      the exact fp64 minimum-image distance of the list definition
//      (coordinates from the Z-ordered particle array) and append the
//      survivors to their rows.
//
// Grid-unit test.  With h the tree's bin width and g(x) = (x - root_lo) / h,
// a quantized bound q decodes exactly to the float 2^23 + q (bit trick: OR
// with 0x4B000000), and the query image is placed at 2^23 + g(x) rounded to
// fp32.  The clamp is v_med3_f32.  Rounding of the query position, of the
// differences and of the sum of squares is covered by comparing against
//   ((R / h) * (1 + 2^-20) + 2)^2 * (1 + 2^-20),
// a pad of two bins plus a relative 2^-20, so no true neighbor is lost; the
// exact filter removes everything the pad lets through.
#include "qbvh_internal.h"

namespace qbi {
namespace {

constexpr int kCand = 16;  // buffered particle runs per lane in LDS (64 B per lane)

__device__ __forceinline__ float grid_bound(uint32_t q16) { return __uint_as_float(0x4B000000u | q16); }

// Squared grid-unit distance from the query (ux, uy, uz) to a packed box.
__device__ __forceinline__ float box_d2(uint32_t wx, uint32_t wy, uint32_t wz, float ux, float uy, float uz) {
    const float cx = __builtin_amdgcn_fmed3f(ux, grid_bound(wx & 0xFFFFu), grid_bound(wx >> 16)) - ux;
    const float cy = __builtin_amdgcn_fmed3f(uy, grid_bound(wy & 0xFFFFu), grid_bound(wy >> 16)) - uy;
    const float cz = __builtin_amdgcn_fmed3f(uz, grid_bound(wz & 0xFFFFu), grid_bound(wz >> 16)) - uz;
    return __builtin_fmaf(cz, cz, __builtin_fmaf(cy, cy, cx * cx));
}

// Output row writer.  With 16-byte aligned rows the lane stages four indices
// in its LDS column and writes them with one 16-byte store.
template <bool kVec4, int kBlock>
__device__ __forceinline__ void append(int32_t j, int32_t &cnt, int32_t (*s_out)[kBlock], int32_t *nbr,
                                       int32_t orig, int32_t max_nbr) {
    if (kVec4) {
        s_out[cnt & 3][threadIdx.x] = j;
        if ((cnt & 3) == 3 && cnt < max_nbr)
            *reinterpret_cast<int4 *>(nbr + ((int64_t)orig * max_nbr + (cnt - 3))) =
                make_int4(s_out[0][threadIdx.x], s_out[1][threadIdx.x], s_out[2][threadIdx.x], j);
    } else {
        if (cnt < max_nbr) nbr[(int64_t)orig * max_nbr + cnt] = j;
    }
    ++cnt;
}

struct Query {
    float x, y, z;   // query position
    int32_t img;     // current periodic image (0..26)
    double r2;       // squared list radius for the current tree pair
    int32_t k;       // sorted position
    int32_t orig;    // original index (row)
};

// Exact decision for this lane's buffered particle runs (all from the current
// image): fp64 (x_j - x_i) - m L per axis, squares summed in the definition's
// order without fused multiply-add, compared with r_list^2.  Two particles
// per step so their loads overlap.
template <bool kVec4, int kBlock>
__device__ __forceinline__ void filter(const int32_t (*s_cand)[kBlock], int32_t nc, const Query &q,
                                       const double (&L)[3], const float4 *__restrict__ sorted, uint32_t n,
                                       int32_t &cnt, int32_t (*s_out)[kBlock], int32_t *nbr, int32_t max_nbr) {
    const int tid = threadIdx.x;
    const double sx = (double)(q.img % 3 - 1) * L[0];
    const double sy = (double)((q.img / 3) % 3 - 1) * L[1];
    const double sz = (double)(q.img / 9 - 1) * L[2];
    int32_t ci = 0, off = 0;
    while (ci < nc) {
        int32_t kk[2];
        bool ok[2];
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            ok[u] = ci < nc;
            kk[u] = 0;
            if (ok[u]) {
                const int32_t v = ~s_cand[ci][tid];
                // in range for any well-formed tree; the clamp keeps a corrupt
                // reference from ever reading outside the particle array
                kk[u] = (int32_t)min((uint32_t)((v >> 3) + off), n - 1u);
                if (++off > (v & 7)) {
                    off = 0;
                    ++ci;
                }
            }
        }
        float4 p[2];
#pragma unroll
        for (int u = 0; u < 2; ++u) p[u] = ok[u] ? sorted[kk[u]] : make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const double dx = ((double)p[u].x - (double)q.x) - sx;
            const double dy = ((double)p[u].y - (double)q.y) - sy;
            const double dz = ((double)p[u].z - (double)q.z) - sz;
            const double d2 = (dx * dx + dy * dy) + dz * dz;
            if (ok[u] && d2 <= q.r2 && kk[u] != q.k)
                append<kVec4, kBlock>(~__float_as_int(p[u].w), cnt, s_out, nbr, q.orig, max_nbr);
        }
    }
}

template <bool kVec4, int kBlock>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(8))) void k_traverse(TravArgs a) {
    __shared__ int32_t s_cand[kCand][kBlock];
    __shared__ int32_t s_out[4][kBlock];
    // Workgroups are dealt round-robin to the 8 XCDs; give each XCD one
    // contiguous stretch of the Z-ordered queries so its L2 holds one region.
    const uint32_t nb = gridDim.x, b = blockIdx.x;
    const uint32_t xcd = b & 7u, qq = nb >> 3, rr = nb & 7u;
    const uint32_t logical = xcd * qq + (xcd < rr ? xcd : rr) + (b >> 3);
    const int32_t k = (int32_t)(logical * kBlock + threadIdx.x);
    if (k >= a.n) return;

    const float4 qp = a.sorted[k];
    Query q;
    q.x = qp.x;
    q.y = qp.y;
    q.z = qp.z;
    q.img = 13;
    q.k = k;
    q.orig = ~__float_as_int(qp.w);
    int ta = 0;
    for (int t = 1; t < a.ntypes; ++t)
        if (k >= a.meta[t].start) ta = t;

    int32_t cnt = 0;

    for (int tb = 0; tb < a.ntypes; ++tb) {
        const TreeMeta &m = a.meta[tb];
        if (m.count == 0) continue;
        double r2 = a.rlist2[tb];
        for (int t = 1; t < a.ntypes; ++t)
            if (ta == t) r2 = a.rlist2[t * QBVH_MAX_TYPES + tb];
        if (r2 < 0.0) continue;
        q.r2 = r2;
        const double R = sqrt(r2);

        // (1) image mask against the root box (Algorithm 1, line 4), in fp32
        // with an outward pad of 2^-18 of the largest box edge (far above the
        // fp32 rounding of the shifted coordinates) plus 2^-20 relative.
        const float pad = (float)(a.lmax * 0x1p-18);
        const float rimg = (float)R * (1.0f + 0x1p-20f) + pad;
        const float rimg2 = rimg * rimg;
        float e2[3][3];
        const float xq[3] = {qp.x, qp.y, qp.z};
#pragma unroll
        for (int dd = 0; dd < 3; ++dd) {
#pragma unroll
            for (int sh = 0; sh < 3; ++sh) {
                const float p = xq[dd] + (float)(sh - 1) * a.Lf[dd];
                const float e = fmaxf(fmaxf(m.lo[dd] - p, p - m.hi[dd]), 0.0f);
                e2[dd][sh] = e * e;
            }
        }
        uint32_t bits = 0;
#pragma unroll
        for (int img = 0; img < 27; ++img) {
            const float sum = (e2[0][img % 3] + e2[1][(img / 3) % 3]) + e2[2][img / 9];
            if (sum <= rimg2) bits |= 1u << img;
        }

        const double rg = R * m.inv_h;
        const double rgp = rg * (1.0 + 0x1p-20) + 2.0;
        const float r2g = (float)(rgp * rgp * (1.0 + 0x1p-20));
        const int32_t root = m.root, end = m.end;

        // (2) one stackless walk per overlapping image (Algorithm 1, lines 5-19)
        while (bits) {
            const int img = __ffs(bits) - 1;
            bits &= bits - 1u;
            q.img = img;
            const double sx = (double)(img % 3 - 1) * a.L[0];
            const double sy = (double)((img / 3) % 3 - 1) * a.L[1];
            const double sz = (double)(img / 9 - 1) * a.L[2];
            const float ux = (float)((((double)q.x + sx) - (double)m.lo[0]) * m.inv_h + 8388608.0);
            const float uy = (float)((((double)q.y + sy) - (double)m.lo[1]) * m.inv_h + 8388608.0);
            const float uz = (float)((((double)q.z + sz) - (double)m.lo[2]) * m.inv_h + 8388608.0);
            int32_t nc = 0;
            if (root < 0) {  // a tree of at most leaf_size particles is one run
                s_cand[0][threadIdx.x] = root;
                nc = 1;
            }
            int32_t v = root < 0 ? end : root;
            for (;;) {
                // one filter call site: when the image's walk is over, or when
                // some lane of the wavefront could overflow its buffer
                const bool done = v >= end;
                if (__any(nc >= kCand - 1) || done) {
                    filter<kVec4, kBlock>(s_cand, nc, q, a.L, a.sorted, (uint32_t)a.n, cnt, s_out, a.nbr, a.max_nbr);
                    nc = 0;
                }
                if (done) break;
                const uint4 r0 = a.records[2 * (int64_t)v];
                const uint4 r1 = a.records[2 * (int64_t)v + 1];
                const int32_t rope = a.ropes[v];
                const bool hl = box_d2(r0.x, r0.y, r0.z, ux, uy, uz) <= r2g;
                const bool hr = box_d2(r0.w, r1.x, r1.y, ux, uy, uz) <= r2g;
                const int32_t cl = (int32_t)r1.z, cr = (int32_t)r1.w;
                if (hl && cl < 0) {
                    s_cand[nc][threadIdx.x] = cl;
                    ++nc;
                }
                if (hr && cr < 0) {
                    s_cand[nc][threadIdx.x] = cr;
                    ++nc;
                }
                const int32_t next = (hl && cl >= 0) ? cl : ((hr && cr >= 0) ? cr : rope);
                // references always point forward; max() makes progress unconditional
                v = max(next, v + 1);
            }
        }
    }

    a.count[q.orig] = cnt;
    if (kVec4) {
        const int32_t rem = cnt & 3;
        const int32_t at = cnt - rem;
        if (rem && at < a.max_nbr) {
            int32_t *row = a.nbr + (int64_t)q.orig * a.max_nbr;
            for (int32_t e = 0; e < rem; ++e) row[at + e] = s_out[e][threadIdx.x];
        }
    }
    if (cnt > a.max_nbr) atomicOr(a.overflow, 1);
}

__global__ void k_clear_flag(int32_t *f) {
    if (threadIdx.x == 0) *f = 0;
}

template <bool kVec4, int kBlock>
void launch_one(const TravArgs &a, hipStream_t s) {
    const unsigned grid = (unsigned)((a.n + kBlock - 1) / kBlock);
    hipLaunchKernelGGL((k_traverse<kVec4, kBlock>), dim3(grid), dim3(kBlock), 0, s, a);
}

template <bool kVec4>
void launch_block(const TravArgs &a, int32_t block, hipStream_t s) {
    switch (block) {
    case 64: launch_one<kVec4, 64>(a, s); break;
    case 128: launch_one<kVec4, 128>(a, s); break;
    case 192: launch_one<kVec4, 192>(a, s); break;
    default: launch_one<kVec4, 256>(a, s); break;
    }
}

}  // namespace

hipError_t launch_traverse(const TravArgs &a, int32_t block, bool vec4, hipStream_t s) {
    hipLaunchKernelGGL(k_clear_flag, dim3(1), dim3(64), 0, s, a.overflow);
    if (a.n > 0) {
        if (vec4)
            launch_block<true>(a, block, s);
        else
            launch_block<false>(a, block, s);
    }
    return hipGetLastError();
}

}  // namespace qbi

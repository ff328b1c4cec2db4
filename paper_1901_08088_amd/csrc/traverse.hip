// Neighbor-list traversal: one lane per Z-ordered particle, stackless walk of
// the rope-linked quantized tree (Algorithm 1; Section 2.3; Section 3 runs the
// queries in Z order so that the lanes of a wavefront walk similar subtrees).
//
// Per lane and per type tree:
//   1. image mask: which of the 27 periodic images of the search sphere touch
//      the tree's root box (fp64 test, padded outward);
//   2. for each image, a walk from the root slot to the tree's end:
//        internal slot: sphere-box test in grid units against the quantized
//          box (nearest point by a clamp per axis, eq. (2)); on overlap the
//          next slot (left child), else the rope;
//        particle slot: the exact fp64 minimum-image distance decides, then
//          the next slot.
//
// Grid-unit test.  With h the tree's bin width and g(x) = (x - root_lo) / h,
// a quantized bound q decodes exactly to the float 2^23 + q (bit trick: OR
// with 0x4B000000), and the query image is placed at 2^23 + g(x) rounded to
// fp32.  The clamp is v_med3_f32.  Rounding of the query position, of the
// differences and of the sum of squares is covered by comparing against
//   ((R / h) * (1 + 2^-20) + 2)^2 * (1 + 2^-20),
// a pad of two bins plus a relative 2^-20, so no true neighbor is lost; the
// exact filter at the particle slots removes everything the pad lets through.
#include "qbvh_internal.h"

namespace qbi {
namespace {

__device__ __forceinline__ float grid_bound(uint32_t q16) { return __uint_as_float(0x4B000000u | q16); }

template <bool kVec4>
__device__ __forceinline__ void append(int32_t j, int32_t &cnt, int32_t (&b)[4], int32_t *nbr, int32_t orig,
                                       int32_t max_nbr) {
    if (kVec4) {
        b[0] = b[1];
        b[1] = b[2];
        b[2] = b[3];
        b[3] = j;
        if ((cnt & 3) == 3 && cnt < max_nbr)
            *reinterpret_cast<int4 *>(nbr + ((int64_t)orig * max_nbr + (cnt - 3))) = make_int4(b[0], b[1], b[2], b[3]);
    } else {
        if (cnt < max_nbr) nbr[(int64_t)orig * max_nbr + cnt] = j;
    }
    ++cnt;
}

template <bool kVec4>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(8))) void k_traverse(TravArgs a) {
    // Workgroups are dealt round-robin to the 8 XCDs; give each XCD one
    // contiguous stretch of the Z-ordered queries so its L2 holds one region.
    const uint32_t nb = gridDim.x, b = blockIdx.x;
    const uint32_t xcd = b & 7u, q = nb >> 3, r = nb & 7u;
    const uint32_t logical = xcd * q + (xcd < r ? xcd : r) + (b >> 3);
    const int32_t k = (int32_t)(logical * blockDim.x + threadIdx.x);
    if (k >= a.n) return;

    const float4 qp = a.sorted[k];
    const int32_t orig = ~__float_as_int(qp.w);
    const double xd = qp.x, yd = qp.y, zd = qp.z;
    int ta = 0;
    for (int t = 1; t < a.ntypes; ++t)
        if (k >= a.meta[t].start) ta = t;

    int32_t cnt = 0;
    int32_t buf[4] = {0, 0, 0, 0};

    for (int tb = 0; tb < a.ntypes; ++tb) {
        const TreeMeta &m = a.meta[tb];
        if (m.count == 0) continue;
        double r2 = a.rlist2[tb];
        for (int t = 1; t < a.ntypes; ++t)
            if (ta == t) r2 = a.rlist2[t * QBVH_MAX_TYPES + tb];
        if (r2 < 0.0) continue;
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

        // (2) one stackless walk per overlapping image (Algorithm 1, lines 5-19)
        while (bits) {
            const int img = __ffs(bits) - 1;
            bits &= bits - 1u;
            const double sx = (double)(img % 3 - 1) * a.L[0];
            const double sy = (double)((img / 3) % 3 - 1) * a.L[1];
            const double sz = (double)(img / 9 - 1) * a.L[2];
            const float ux = (float)(((xd + sx) - (double)m.lo[0]) * m.inv_h + 8388608.0);
            const float uy = (float)(((yd + sy) - (double)m.lo[1]) * m.inv_h + 8388608.0);
            const float uz = (float)(((zd + sz) - (double)m.lo[2]) * m.inv_h + 8388608.0);
            int32_t nidx = m.root;
            const int32_t end = m.end;
            while (nidx < end) {
                const uint4 sl = a.slots[nidx];
                if ((int32_t)sl.w < 0) {
                    // particle: exact fp64 minimum-image distance, same operation
                    // order as the list definition, no fused multiply-add
                    const double dx = ((double)__uint_as_float(sl.x) - xd) - sx;
                    const double dy = ((double)__uint_as_float(sl.y) - yd) - sy;
                    const double dz = ((double)__uint_as_float(sl.z) - zd) - sz;
                    const double d2 = (dx * dx + dy * dy) + dz * dz;
                    const int32_t j = ~(int32_t)sl.w;
                    if (d2 <= r2 && j != orig) append<kVec4>(j, cnt, buf, a.nbr, orig, a.max_nbr);
                    ++nidx;
                } else {
                    // internal node: sphere vs quantized box in grid units (eq. (2))
                    const float cx = __builtin_amdgcn_fmed3f(ux, grid_bound(sl.x & 0xFFFFu), grid_bound(sl.x >> 16)) - ux;
                    const float cy = __builtin_amdgcn_fmed3f(uy, grid_bound(sl.y & 0xFFFFu), grid_bound(sl.y >> 16)) - uy;
                    const float cz = __builtin_amdgcn_fmed3f(uz, grid_bound(sl.z & 0xFFFFu), grid_bound(sl.z >> 16)) - uz;
                    const float d2 = __builtin_fmaf(cz, cz, __builtin_fmaf(cy, cy, cx * cx));
                    // ropes always point forward; max() makes progress unconditional
                    nidx = (d2 <= r2g) ? nidx + 1 : max((int32_t)sl.w, nidx + 1);
                }
            }
        }
    }

    a.count[orig] = cnt;
    if (kVec4) {
        const int32_t rem = cnt & 3;
        const int32_t at = cnt - rem;
        if (rem && at < a.max_nbr) {
            int32_t *row = a.nbr + (int64_t)orig * a.max_nbr;
            if (rem == 1) {
                row[at] = buf[3];
            } else if (rem == 2) {
                row[at] = buf[2];
                row[at + 1] = buf[3];
            } else {
                row[at] = buf[1];
                row[at + 1] = buf[2];
                row[at + 2] = buf[3];
            }
        }
    }
    if (cnt > a.max_nbr) atomicOr(a.overflow, 1);
}

__global__ void k_clear_flag(int32_t *f) {
    if (threadIdx.x == 0) *f = 0;
}

}  // namespace

hipError_t launch_traverse(const TravArgs &a, int32_t block, bool vec4, hipStream_t s) {
    hipLaunchKernelGGL(k_clear_flag, dim3(1), dim3(64), 0, s, a.overflow);
    if (a.n > 0) {
        const unsigned grid = (unsigned)((a.n + block - 1) / block);
        if (vec4)
            hipLaunchKernelGGL(k_traverse<true>, dim3(grid), dim3(block), 0, s, a);
        else
            hipLaunchKernelGGL(k_traverse<false>, dim3(grid), dim3(block), 0, s, a);
    }
    return hipGetLastError();
}

}  // namespace qbi

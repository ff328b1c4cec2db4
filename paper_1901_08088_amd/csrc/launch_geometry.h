// Traversal launch geometry shared by the host (workgroup counts) and the
// device (which queries a wavefront takes).  Plain C++ apart from the
// host/device qualifiers, so that a CPU test can check the host's bound
// against the device's mapping (tests/launch_geometry_test.cpp).
#pragma once

#include <stdint.h>

#ifdef __HIPCC__
#define QBVH_HD __host__ __device__
#else
#define QBVH_HD
#endif

namespace qbi {

// Queries per wavefront of one type of a system of several types.  A type
// with fewer than an eighth of the system's particles is sparse: its
// Z-consecutive queries lie far apart, so a wavefront of many of them walks a
// very wide union and runs far longer than the others; such a type takes at
// most kSparseQpw queries per wavefront.
constexpr int32_t kSparseQpw = 16;
QBVH_HD inline int32_t type_qpw(int64_t count, int64_t n, int32_t qpw) {
    return (count * 8 < n && qpw > kSparseQpw) ? kSparseQpw : qpw;
}

// A system of several types is traversed in eight stretches; stretch `part`
// takes queries [stretch_lo(count, part), stretch_lo(count, part + 1)) of a
// type of `count` particles, in type_waves(...) wavefronts.
QBVH_HD inline int32_t stretch_lo(int64_t count, int64_t part) { return (int32_t)(count * part / 8); }
QBVH_HD inline int32_t type_waves(int64_t count, int64_t n, int32_t qpw, int64_t part) {
    const int32_t len = stretch_lo(count, part + 1) - stretch_lo(count, part);
    const int32_t qt = type_qpw(count, n, qpw);
    return (len + qt - 1) / qt;
}

// Traversal workgroups of a system whose wavefronts take `qpw` queries each.
// A system of several types gets eight equal stretches, each with room for
// an eighth of every type (see the traversal's query order); the count is an
// upper bound there (the device knows the type sizes, the host does not), and
// wavefronts past a stretch's share exit at once.  Per stretch a type t takes
// len_t <= ceil(count_t / 8) queries in ceil(len_t / qpw_t) wavefronts, so
//   waves <= sum_t (len_t / qpw_t + 1)
//         <= (ceil(n/8) + ntypes) / qpw + (ntypes - 1) (ceil(n/64) + 1) / min(qpw, kSparseQpw) + ntypes,
// the second term bounding the sparse types (each has len_t <= ceil(n/64)).
inline int64_t trav_blocks(int64_t n, int32_t ntypes, int32_t block, int32_t qpw = 64) {
    const int64_t per_wg = (int64_t)(block / 64) * qpw;
    if (ntypes <= 1) return (n + per_wg - 1) / per_wg;
    const int64_t sq = qpw > kSparseQpw ? kSparseQpw : qpw;
    const int64_t dense = ((n + 7) / 8 + ntypes + qpw - 1) / qpw;
    const int64_t sparse = (int64_t)(ntypes - 1) * (((n + 63) / 64 + 1 + sq - 1) / sq);
    const int64_t waves = dense + sparse + ntypes;
    return 8 * ((waves + block / 64 - 1) / (block / 64));
}

}  // namespace qbi

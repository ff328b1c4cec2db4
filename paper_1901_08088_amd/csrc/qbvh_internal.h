// Internal declarations of the qbvh library (device structs and kernel launchers).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/qbvh.h"
#include "launch_geometry.h"

namespace qbi {

// Largest s in [0, nseg) with first[s] <= x (first is nondecreasing, first[0] = 0).
__device__ __forceinline__ int32_t find_seg(const int32_t *__restrict__ first, int32_t nseg, int32_t x) {
    int32_t lo = 0, hi = nseg - 1;
    while (lo < hi) {
        const int32_t mid = (lo + hi + 1) >> 1;
        if (first[mid] <= x) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// A particle run [first, first + count), count <= 16, is referenced as
// ~((first << kRunCountBits) | (count - 1)).
constexpr int kRunCountBits = 4;
constexpr int32_t kRunCountMask = (1 << kRunCountBits) - 1;

// Per-type tree description, written on the device after the bottom-up fit.
struct TreeMeta {
    float lo[3];      // root-node box (exact fp32 min over the type's particles)
    float hi[3];      // root-node box (exact fp32 max)
    double h;         // grid spacing of the quantized bounds
    double inv_h;     // 1 / h
    int32_t start;    // first sorted position of the type
    int32_t count;    // particles of the type
    int32_t root;     // root record index, or the particle run of a tree of <= leaf_size particles
    int32_t end;      // one past the last record of this tree
    int32_t pad[2];
};
static_assert(sizeof(TreeMeta) == 64, "TreeMeta is 64 bytes");

// The traversal loads the particles of a leaf run 8 float4 at a time from the
// run's start and from its ninth particle, whatever the run's length; the
// sorted array carries this many spare entries after its last particle so
// those loads stay inside the buffer.
constexpr int32_t kSortedPad = 16;

// Device workspace of one built tree (all arrays sized for `cap` particles).
struct Workspace {
    int32_t cap = 0;
    int32_t tiles = 0;        // radix-sort tiles for cap
    void *base = nullptr;     // single hipMalloc allocation
    size_t bytes = 0;
    uint32_t *keys = nullptr, *vals = nullptr;
    uint32_t *keys2 = nullptr, *vals2 = nullptr;  // sort ping-pong; keys2 then holds the tree build's exchange slots
    uint32_t *hist = nullptr;       // [256][tiles]
    uint32_t *digit_total = nullptr;// [256]
    float4 *sorted = nullptr;       // [cap + kSortedPad]
    int32_t *left = nullptr, *right = nullptr, *rf = nullptr, *rl = nullptr;
    int32_t *parent = nullptr, *leaf_parent = nullptr;
    uint32_t *visit = nullptr;      // split weights during the tree build; with the cost model, then kept flags
    float *cost = nullptr;          // subtree collapse: volume-weighted cost per internal node (negative: a run)
    float4 *box = nullptr;          // [cap][2]: node K's lower bound at 2K, its upper bound at 2K + 1
    uint32_t *kept = nullptr;       // [cap + 1]: kept-node counts, scanned in place
    uint32_t *scan_part = nullptr;  // [scan blocks + 1]
    uint4 *records = nullptr;       // [cap][2]: two-wide quantized records
    uint4 *qpoint = nullptr;        // [cap + kSortedPad]: per sorted particle, its quantized cell box
                                    // (words 0-2 as a record box) and original index (word 3);
                                    // written only for paper-mode lists
    int32_t *ropes = nullptr;       // [cap]
    TreeMeta *meta = nullptr;       // [QBVH_MAX_TYPES]
    uint32_t *type_count = nullptr; // [QBVH_MAX_TYPES]
    int32_t *err = nullptr;         // [1]
    int32_t *front[2] = {nullptr, nullptr};    // bottom-up fit frontiers (ping-pong)
    uint32_t *fcount[2] = {nullptr, nullptr};
};

size_t workspace_bytes(int32_t cap);
void workspace_carve(Workspace &w, void *base, int32_t cap);

// Traversal arguments (passed by value as the kernel argument block).
struct TravArgs {
    const uint4 *records;
    const int32_t *ropes;
    const float4 *sorted;
    const TreeMeta *meta;
    const double *sorted64;  // fp64 data: sorted positions [n][4] (x, y, z, unused); nullptr for fp32 data
    int32_t *nbr;
    int32_t *count;
    int32_t *overflow;
    double L[3];
    double rlist2[QBVH_MAX_TYPES * QBVH_MAX_TYPES];
    float Lf[3];
    float pad0;
    double lmax;
    int32_t n;        // particles of this system
    int32_t ntypes;
    int32_t max_nbr;
    int32_t start;    // first sorted position of this system (0 for a single system)
    int32_t qpw;      // queries per wavefront (64, or 32/16/8 for small systems)
    int32_t qbits;    // grid bits of the tree (paper-mode cell boxes)
};

// One system of a batch as the build kernels see it.
struct SysBuild {
    const float *pos;      // device float [n][3]
    const int32_t *type;   // device int32 [n], or nullptr when ntypes == 1
    int32_t n;
    int32_t ntypes;
    int32_t off;           // first position of the system in the concatenation
    int32_t pad;
    double scale[3];       // 1023 / L_d (Morton bins)
    double ext_floor;      // L_max 2^-24 (smallest root extent used for the grid)
};

// Device pointers and sizes of one batched launch sequence.  Every system s
// occupies positions [sys_off[s], sys_off[s + 1]) of the concatenated
// arrays; blk_first, tile_first and tblk_first give the first build block
// (kBuildThreads items), sort tile and traversal workgroup of each system.
struct BatchLaunch {
    Workspace ws;               // sized for the concatenation
    uint32_t *hist;             // 256 * tiles sort counters
    uint32_t *scan_part;        // scan partials for max(total + 1, 256 * tiles)
    const int32_t *sys_off, *blk_first, *tile_first, *tblk_first;  // [nsys + 1] each
    const SysBuild *sysb;       // [nsys]
    const TravArgs *trav;       // [nsys]
    uint32_t *type_count;       // [nsys][QBVH_MAX_TYPES]
    TreeMeta *meta;             // [nsys][QBVH_MAX_TYPES]
    int32_t nsys, total, blocks, tiles, tblocks;
    int32_t leaf_size, qbits, block_size;
    bool vec4;
};

// Host helpers shared by the interface files.

// Queries per wavefront of a single system.  A wavefront walks the union of
// its queries' paths, so a small system is faster with fewer queries per
// wavefront (a smaller union each, more wavefronts in parallel) until there
// are about two wavefronts per SIMD, and below 8 queries until there is about
// one; a large one keeps all 64 lanes busy.  (Measured on LJ fluids of 1000 to
// 260000 particles: 2 queries up to 4000, 8 at 15000 and 30000, 16 at 65000,
// 32 at 130000, 64 from 260000.)
inline int32_t queries_per_wave(int64_t n) {
    int32_t q = 64;
    while (q > 8 && (n + q - 1) / q < 2048) q /= 2;
    while (q > 2 && (n + q - 1) / q < 1024) q /= 2;
    return q;
}

constexpr int32_t kMaxParticles = (1 << 27) - 1;  // particle runs store a sorted position in 27 bits
inline bool leaf_ok(int32_t v) { return v >= 1 && v <= 16; }
inline bool qbits_ok(int32_t v) { return v >= 8 && v <= 16; }
// the traversal kernel is compiled for 64, 128, 192 and 256 work-items per group
inline bool block_ok(int32_t v) { return v >= 64 && v <= 256 && (v % 64) == 0; }
// queries per wavefront: 0 (automatic) or a power of 2 up to 64
inline bool qpw_ok(int32_t v) { return v >= 0 && v <= 64 && (v & (v - 1)) == 0; }
int hip_fail(hipError_t e);  // records the error for qbvh_last_hip_error, maps it to a code
bool box_ok(const float box[3]);
int list_radii(const float *rcut, float skin, int32_t ntypes, const float box[3],
               double rlist2[QBVH_MAX_TYPES * QBVH_MAX_TYPES]);
int list_radii(const float *rcut, float skin, int32_t ntypes, const double box[3],
               double rlist2[QBVH_MAX_TYPES * QBVH_MAX_TYPES]);
void fill_trav_box(TravArgs &a, const float box[3]);
void fill_trav_box(TravArgs &a, const double box[3]);

// Launchers (all asynchronous on `s`; return the launch status).
// collapse_radius > 0: subtrees of at most leaf_size particles become runs by
// the cost model (build_common.h); 0: every subtree of at most leaf_size.
// The build from positions d_pos [n][3] (fp32) in box `box`.  fp64 data:
// d_pos is null and pos64 [n][3] holds the data in the fp64 box box64 (box
// is box64 rounded to fp32): the tree is built on the data rounded to
// nearest fp32, validation is done in fp64, and sorted64 [n][4] receives the
// fp64 positions in Z order.
hipError_t launch_build(const Workspace &w, const float *d_pos, const int32_t *d_type, int32_t n,
                        int32_t ntypes, const float box[3], int32_t leaf_size, int32_t qbits,
                        float collapse_radius, int32_t validate, hipStream_t s, const double *pos64 = nullptr,
                        double *sorted64 = nullptr, const double *box64 = nullptr);
hipError_t launch_traverse(const TravArgs &a, int32_t block, bool vec4, bool paper, const uint4 *qpoint,
                           hipStream_t s);
// fp64 particle data: the positions rounded to fp32 for the build (with the
// fp64 range and type checks when validate is set), and after the build the
// fp64 positions in sorted order.
// Paper-mode cell boxes; lmax is the largest periodic box edge (the extent floor is lmax 2^-24).
hipError_t launch_qpoint(const Workspace &w, int32_t n, int32_t ntypes, int32_t qbits, double lmax, hipStream_t s);
hipError_t launch_traverse_batch(const BatchLaunch &b, hipStream_t s);
hipError_t launch_batch(const BatchLaunch &b, hipStream_t s);
// Stable sort of keys[0, n); vals receives each sorted key's input position
// (the caller writes only the keys).
hipError_t launch_radix_sort(uint32_t *keys, uint32_t *vals, uint32_t *keys2, uint32_t *vals2,
                             uint32_t *hist, uint32_t *digit_total, int32_t n, int32_t tiles,
                             hipStream_t s);
hipError_t launch_exclusive_scan(uint32_t *data, int32_t len, uint32_t *partials, hipStream_t s);
struct Collapse;
// Where the tree build takes its particles and tree boundaries from: a single
// system (pos: positions [n][3] in input order; the sort's values are input
// indices) or a batch (sysb and sys_off: system s owns sorted positions
// [sys_off[s], sys_off[s + 1]); the sort's values are concatenated indices).
struct TreeSource {
    const float *pos;
    const SysBuild *sysb;
    const int32_t *sys_off;
    int32_t nsys;
    // fp64 data (single system): the particles are gathered from pos64 [n][3]
    // instead, rounded to fp32 for the tree, and also written to sorted64
    // [n][4] (x, y, z, 0) in Z order
    const double *pos64;
    double *sorted64;
};
// Radix tree, Z-ordered particles, node boxes (and costs) and kept-node counts
// (nodes longer than kept_leaf) from the sorted keys and values.
hipError_t launch_tree(const Workspace &w, int32_t n, const TreeSource &src, int32_t kept_leaf, const Collapse &col,
                       hipStream_t s);
int32_t fit_chunks0(int32_t cap);
// Stable sort of each segment [seg_off[s], seg_off[s+1]) of keys on its own,
// vals receiving each sorted key's position in the concatenation; tile_first[s] = sum over earlier segments of seg_radix_tiles(size),
// tiles = tile_first[nseg]; hist holds 256 * tiles counters, scan_part
// scan_blocks(256 * tiles) + 1.
hipError_t launch_radix_sort_segmented(uint32_t *keys, uint32_t *vals, uint32_t *keys2, uint32_t *vals2,
                                       uint32_t *hist, uint32_t *scan_part, int32_t n, int32_t tiles,
                                       const int32_t *tile_first, const int32_t *seg_off, int32_t nseg,
                                       hipStream_t s);
int32_t seg_radix_tiles(int32_t n);
int32_t radix_tiles(int32_t n);
int32_t scan_blocks(int32_t len);

}  // namespace qbi

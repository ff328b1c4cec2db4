// Internal declarations of the qbvh library (device structs and kernel launchers).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/qbvh.h"

namespace qbi {

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

// Device workspace of one built tree (all arrays sized for `cap` particles).
struct Workspace {
    int32_t cap = 0;
    int32_t tiles = 0;        // radix-sort tiles for cap
    void *base = nullptr;     // single hipMalloc allocation
    size_t bytes = 0;
    uint32_t *keys = nullptr, *vals = nullptr, *keys2 = nullptr, *vals2 = nullptr;
    uint32_t *hist = nullptr;       // [256][tiles]
    uint32_t *digit_total = nullptr;// [256]
    float4 *sorted = nullptr;       // [cap]
    int32_t *left = nullptr, *right = nullptr, *rf = nullptr, *rl = nullptr;
    int32_t *parent = nullptr, *leaf_parent = nullptr;
    uint32_t *visit = nullptr;
    float4 *box_lo = nullptr, *box_hi = nullptr;
    uint32_t *kept = nullptr;       // [cap + 1]: kept-node counts, scanned in place
    uint32_t *scan_part = nullptr;  // [scan blocks + 1]
    uint4 *records = nullptr;       // [cap][2]: two-wide quantized records
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
    int32_t *nbr;
    int32_t *count;
    int32_t *overflow;
    double L[3];
    double rlist2[QBVH_MAX_TYPES * QBVH_MAX_TYPES];
    float Lf[3];
    float pad0;
    double lmax;
    int32_t n;
    int32_t ntypes;
    int32_t max_nbr;
    int32_t pad;
};

// Launchers (all asynchronous on `s`; return the launch status).
hipError_t launch_build(const Workspace &w, const float *d_pos, const int32_t *d_type, int32_t n,
                        int32_t ntypes, const float box[3], int32_t leaf_size, int32_t qbits,
                        int32_t validate, hipStream_t s);
hipError_t launch_traverse(const TravArgs &a, int32_t block, bool vec4, hipStream_t s);
hipError_t launch_radix_sort(uint32_t *keys, uint32_t *vals, uint32_t *keys2, uint32_t *vals2,
                             uint32_t *hist, uint32_t *digit_total, int32_t n, int32_t tiles,
                             hipStream_t s);
hipError_t launch_exclusive_scan(uint32_t *data, int32_t len, uint32_t *partials, hipStream_t s);
int32_t radix_tiles(int32_t n);
int32_t scan_blocks(int32_t len);

}  // namespace qbi

// Grid (cell list) neighbor search: the comparison method of the paper
// (Section 1 and Section 4: particles binned into a uniform grid of cells no
// narrower than the list radius, each particle scanning the 27 cells around
// its own), written for the same GPU so that the tree can be measured against
// it.  One particle type.  The lists are the exact lists of nlist_build: each
// candidate is decided by the same fp32 test with its error band and, inside
// the band, by the fp64 arithmetic of the definition.
//
// Steps (Section 3): cell index per particle; stable radix sort by cell (the
// sort of the tree build), so the particles of a cell are contiguous and in
// index order; cell ranges from the sorted keys; then the traversal in the
// sorted order with n lanes per particle (n a power of 2 below the wavefront
// width): the n lanes of a particle take the candidates of each of its 27
// cells in turn, n at a time (lane t the t-th of every n), and combine their
// accepted candidates with a ballot over the group (the wave64 form of the
// paper's warp shuffles), so the row is written n entries at a time in
// candidate order.  n = 1 is one lane per particle.
#include <math.h>
#include <string.h>

#include <new>

#include "qbvh_internal.h"

struct qgrid {
    void *mem = nullptr;
    size_t bytes = 0;
    int32_t cap = 0;
    int64_t cell_cap = 0;
    uint32_t *keys = nullptr, *vals = nullptr, *keys2 = nullptr, *vals2 = nullptr;
    uint32_t *hist = nullptr, *digit_total = nullptr;
    float4 *sorted = nullptr;
    int32_t *cell_start = nullptr, *cell_end = nullptr;
    hipStream_t stream = nullptr;
};

namespace qbi {
namespace {

constexpr int kGridThreads = 256;

struct GridGeom {
    int32_t nc[3];
    double inv_w[3];  // cells per unit length
    double L[3];
    float Lf[3];
};

__global__ __launch_bounds__(kGridThreads) void k_cell_key(const float *__restrict__ pos, int32_t n, GridGeom g,
                                                           uint32_t *__restrict__ keys) {
    const int32_t i = blockIdx.x * kGridThreads + threadIdx.x;
    if (i >= n) return;
    int32_t c[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        double v = floor((double)pos[3 * (int64_t)i + d] * g.inv_w[d]);
        if (!(v >= 0.0)) v = 0.0;
        if (v > (double)(g.nc[d] - 1)) v = (double)(g.nc[d] - 1);
        c[d] = (int32_t)v;
    }
    keys[i] = (uint32_t)((c[2] * g.nc[1] + c[1]) * g.nc[0] + c[0]);
}

__global__ __launch_bounds__(kGridThreads) void k_cell_clear(int32_t *__restrict__ start, int32_t *__restrict__ end,
                                                             int64_t ncells) {
    const int64_t c = (int64_t)blockIdx.x * kGridThreads + threadIdx.x;
    if (c >= ncells) return;
    start[c] = 0;
    end[c] = 0;
}

// Sorted particles (x, y, z, ~original index) and the range of every
// non-empty cell, from the boundaries between equal keys.
__global__ __launch_bounds__(kGridThreads) void k_cell_ranges(const float *__restrict__ pos,
                                                              const uint32_t *__restrict__ keys,
                                                              const uint32_t *__restrict__ vals, int32_t n,
                                                              float4 *__restrict__ sorted,
                                                              int32_t *__restrict__ start, int32_t *__restrict__ end) {
    const int32_t k = blockIdx.x * kGridThreads + threadIdx.x;
    if (k >= n) return;
    const uint32_t i = vals[k];
    sorted[k] = make_float4(pos[3 * (int64_t)i + 0], pos[3 * (int64_t)i + 1], pos[3 * (int64_t)i + 2],
                            __int_as_float(~(int32_t)i));
    const uint32_t key = keys[k];
    if (k == 0 || keys[k - 1] != key) start[key] = k;
    if (k == n - 1 || keys[k + 1] != key) end[key] = k + 1;
}

// The n = kN lanes of particle k (sorted position; lanes kN k .. kN k + kN - 1
// of the launch, inside one wavefront).
template <int kN>
__global__ __launch_bounds__(kGridThreads) void k_grid_nlist(const float4 *__restrict__ sorted,
                                                             const uint32_t *__restrict__ keys, int32_t n,
                                                             GridGeom g, const int32_t *__restrict__ start,
                                                             const int32_t *__restrict__ end, double r2, float r2in,
                                                             float r2out, int32_t max_nbr, int32_t *__restrict__ nbr,
                                                             int32_t *__restrict__ count, int32_t *overflow) {
    const int64_t t = (int64_t)blockIdx.x * kGridThreads + threadIdx.x;
    const int32_t k = (int32_t)(t / kN);
    if (k >= n) return;  // the kN lanes of a group share k: a group leaves whole
    const uint32_t lane = __lane_id();
    const int32_t sub = (int32_t)(lane & (kN - 1));
    // this group's lanes in the wavefront, and those below this lane
    const uint64_t gmask = kN == 64 ? ~0ull : (((1ull << kN) - 1ull) << (lane & ~(uint32_t)(kN - 1)));
    const uint64_t below = gmask & ((1ull << lane) - 1ull);
    const float4 q = sorted[k];
    const int32_t orig = ~__float_as_int(q.w);
    const uint32_t key = keys[k];
    const int32_t cx = (int32_t)(key % (uint32_t)g.nc[0]);
    const int32_t cy = (int32_t)((key / (uint32_t)g.nc[0]) % (uint32_t)g.nc[1]);
    const int32_t cz = (int32_t)(key / ((uint32_t)g.nc[0] * (uint32_t)g.nc[1]));
    int32_t *row = nbr + (int64_t)orig * max_nbr;
    int32_t cnt = 0;
    for (int oz = -1; oz <= 1; ++oz) {
        int32_t z = cz + oz, mz = 0;
        if (z < 0) { z += g.nc[2]; mz = 1; }
        if (z >= g.nc[2]) { z -= g.nc[2]; mz = -1; }
        for (int oy = -1; oy <= 1; ++oy) {
            int32_t y = cy + oy, my = 0;
            if (y < 0) { y += g.nc[1]; my = 1; }
            if (y >= g.nc[1]) { y -= g.nc[1]; my = -1; }
            for (int ox = -1; ox <= 1; ++ox) {
                int32_t x = cx + ox, mx = 0;
                if (x < 0) { x += g.nc[0]; mx = 1; }
                if (x >= g.nc[0]) { x -= g.nc[0]; mx = -1; }
                // a candidate p of this cell is compared with the query image
                // shifted by m L (dx = (p - q) - m L, as in the definition)
                const double sx = (double)mx * g.L[0], sy = (double)my * g.L[1], sz = (double)mz * g.L[2];
                const float qsx = (float)((double)q.x + sx), qsy = (float)((double)q.y + sy),
                            qsz = (float)((double)q.z + sz);
                const int32_t c = (z * g.nc[1] + y) * g.nc[0] + x;
                const int32_t j0 = start[c], j1 = end[c];
                // every lane of the group runs the same trips: the ballot sees the whole group
                for (int32_t jb = j0; jb < j1; jb += kN) {
                    const int32_t j = jb + sub;
                    bool in = false;
                    int32_t idx = 0;
                    if (j < j1 && j != k) {
                        const float4 p = sorted[j];
                        idx = ~__float_as_int(p.w);
                        const float ax = p.x - qsx, ay = p.y - qsy, az = p.z - qsz;
                        const float d2 = __builtin_fmaf(az, az, __builtin_fmaf(ay, ay, ax * ax));
                        in = d2 <= r2in;
                        if (!in && d2 <= r2out) {
                            const double dx = ((double)p.x - (double)q.x) - sx;
                            const double dy = ((double)p.y - (double)q.y) - sy;
                            const double dz = ((double)p.z - (double)q.z) - sz;
                            in = (dx * dx + dy * dy) + dz * dz <= r2;
                        }
                    }
                    const uint64_t acc = (uint64_t)__ballot(in) & gmask;
                    if (in) {
                        const int32_t pos = cnt + (int32_t)__popcll(acc & below);
                        if (pos < max_nbr) row[pos] = idx;
                    }
                    cnt += (int32_t)__popcll(acc);
                }
            }
        }
    }
    if (sub == 0) {
        count[orig] = cnt;
        if (cnt > max_nbr) atomicOr(overflow, 1);
    }
}

__global__ void k_grid_clear_flag(int32_t *f) {
    if (threadIdx.x == 0) *f = 0;
}

inline dim3 blocks_for(int64_t items) { return dim3((unsigned)((items + kGridThreads - 1) / kGridThreads)); }

template <int kN>
void launch_grid_n(int32_t n, hipStream_t s, const float4 *sorted, const uint32_t *keys, const GridGeom &g,
                   const int32_t *start, const int32_t *end, double r2, float r2in, float r2out, int32_t max_nbr,
                   int32_t *nbr, int32_t *count, int32_t *overflow) {
    hipLaunchKernelGGL(k_grid_nlist<kN>, blocks_for((int64_t)n * kN), dim3(kGridThreads), 0, s, sorted, keys, n, g,
                       start, end, r2, r2in, r2out, max_nbr, nbr, count, overflow);
}

void launch_grid_nlist(int32_t lanes, int32_t n, hipStream_t s, const float4 *sorted, const uint32_t *keys,
                       const GridGeom &g, const int32_t *start, const int32_t *end, double r2, float r2in,
                       float r2out, int32_t max_nbr, int32_t *nbr, int32_t *count, int32_t *overflow) {
    switch (lanes) {
    case 1: launch_grid_n<1>(n, s, sorted, keys, g, start, end, r2, r2in, r2out, max_nbr, nbr, count, overflow); break;
    case 2: launch_grid_n<2>(n, s, sorted, keys, g, start, end, r2, r2in, r2out, max_nbr, nbr, count, overflow); break;
    case 4: launch_grid_n<4>(n, s, sorted, keys, g, start, end, r2, r2in, r2out, max_nbr, nbr, count, overflow); break;
    case 8: launch_grid_n<8>(n, s, sorted, keys, g, start, end, r2, r2in, r2out, max_nbr, nbr, count, overflow); break;
    case 16: launch_grid_n<16>(n, s, sorted, keys, g, start, end, r2, r2in, r2out, max_nbr, nbr, count, overflow); break;
    default: launch_grid_n<32>(n, s, sorted, keys, g, start, end, r2, r2in, r2out, max_nbr, nbr, count, overflow); break;
    }
}

}  // namespace
}  // namespace qbi

using qbi::GridGeom;

extern "C" {

void qgrid_free(qgrid_t *grid) {
    if (!grid) return;
    if (grid->mem) (void)hipFree(grid->mem);
    delete grid;
}

int nlist_build_grid(qgrid_t **grid, const float *d_pos, int32_t n, const float box[3], float rcut, float skin,
                     int32_t lanes, int32_t max_nbr, int32_t *d_nbr, int32_t *d_count, int32_t *d_overflow,
                     qbvh_stream_t stream) {
    if (!grid || n < 0 || n > qbi::kMaxParticles || !qbi::box_ok(box) || max_nbr < 0 || !d_overflow) return QBVH_EINVAL;
    if (lanes == 0) lanes = 4;
    if (lanes < 1 || lanes > 32 || (lanes & (lanes - 1)) != 0) return QBVH_EINVAL;
    if (n > 0 && (!d_pos || !d_count || (max_nbr > 0 && !d_nbr))) return QBVH_EINVAL;
    if (!(isfinite(rcut) && rcut > 0.0f) || !(isfinite(skin) && skin >= 0.0f)) return QBVH_EINVAL;
    const double R = (double)rcut + (double)skin;
    const double r2 = R * R;
    GridGeom g{};
    int64_t ncells = 1;
    for (int d = 0; d < 3; ++d) {
        g.L[d] = (double)box[d];
        g.Lf[d] = box[d];
        if (!(2.0 * R * (1.0 + 1e-9) < g.L[d])) return QBVH_EGEOM;
        int64_t nc = (int64_t)floor(g.L[d] / (R * (1.0 + 1e-9)));
        if (nc > 1024) nc = 1024;
        if (nc < 3) return QBVH_ENOTSUP;  // the 27 cells around a cell would not be distinct
        g.nc[d] = (int32_t)nc;
        g.inv_w[d] = (double)nc / g.L[d];
        ncells *= nc;
    }
    hipStream_t s = (hipStream_t)stream;
    qgrid_t *G = *grid;
    const bool fresh = G == nullptr;
    if (fresh) {
        G = new (std::nothrow) qgrid_t();
        if (!G) return QBVH_ENOMEM;
    }
    if (G->mem == nullptr || G->cap < n || G->cell_cap < ncells) {
        if (G->mem) {
            hipError_t e = hipStreamSynchronize(G->stream);
            if (e == hipSuccess) e = hipStreamSynchronize(s);
            if (e != hipSuccess) {
                if (fresh) delete G;
                return qbi::hip_fail(e);
            }
            (void)hipFree(G->mem);
            G->mem = nullptr;
        }
        const int32_t cap = n > G->cap ? (n > 0 ? n : 1) : G->cap;
        const int64_t ccap = ncells > G->cell_cap ? ncells : G->cell_cap;
        const size_t tiles = (size_t)qbi::radix_tiles(cap);
        auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
        const size_t b_kv = al((size_t)cap * 4), b_hist = al(256 * tiles * 4), b_dt = al(256 * 4);
        const size_t b_sorted = al((size_t)cap * 16), b_cells = al((size_t)ccap * 4);
        const size_t bytes = 4 * b_kv + b_hist + b_dt + b_sorted + 2 * b_cells;
        void *m = nullptr;
        hipError_t e = hipMalloc(&m, bytes);
        if (e != hipSuccess) {
            if (fresh) delete G;
            else G->cap = 0;
            return qbi::hip_fail(e);
        }
        char *p = (char *)m;
        G->mem = m;
        G->bytes = bytes;
        G->cap = cap;
        G->cell_cap = ccap;
        G->keys = (uint32_t *)p; p += b_kv;
        G->vals = (uint32_t *)p; p += b_kv;
        G->keys2 = (uint32_t *)p; p += b_kv;
        G->vals2 = (uint32_t *)p; p += b_kv;
        G->hist = (uint32_t *)p; p += b_hist;
        G->digit_total = (uint32_t *)p; p += b_dt;
        G->sorted = (float4 *)p; p += b_sorted;
        G->cell_start = (int32_t *)p; p += b_cells;
        G->cell_end = (int32_t *)p;
    }
    G->stream = s;
    *grid = G;

    // the fp32 band of the tree's candidate test, with the same derivation
    const double lmax = fmax(g.L[0], fmax(g.L[1], g.L[2]));
    const double eta = 1.7320508075688772 * 0x1p-22 * (2.0 * lmax + 2.0 * R);
    const double rin = fmax(R - eta, 0.0) * (1.0 - 0x1p-20);
    const double rout = (R + eta) * (1.0 + 0x1p-20);
    const float r2in = (float)(rin * rin * (1.0 - 0x1p-20));
    const float r2out = (float)(rout * rout * (1.0 + 0x1p-20));

    hipLaunchKernelGGL(qbi::k_grid_clear_flag, dim3(1), dim3(64), 0, s, d_overflow);
    if (n > 0) {
        hipLaunchKernelGGL(qbi::k_cell_key, qbi::blocks_for(n), dim3(qbi::kGridThreads), 0, s, d_pos, n, g, G->keys);
        hipError_t e = qbi::launch_radix_sort(G->keys, G->vals, G->keys2, G->vals2, G->hist, G->digit_total, n,
                                              qbi::radix_tiles(n), s);
        if (e != hipSuccess) return qbi::hip_fail(e);
        hipLaunchKernelGGL(qbi::k_cell_clear, qbi::blocks_for(ncells), dim3(qbi::kGridThreads), 0, s, G->cell_start,
                           G->cell_end, ncells);
        hipLaunchKernelGGL(qbi::k_cell_ranges, qbi::blocks_for(n), dim3(qbi::kGridThreads), 0, s, d_pos, G->keys,
                           G->vals, n, G->sorted, G->cell_start, G->cell_end);
        qbi::launch_grid_nlist(lanes, n, s, G->sorted, G->keys, g, G->cell_start, G->cell_end, r2, r2in, r2out,
                               max_nbr, d_nbr, d_count, d_overflow);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return qbi::hip_fail(e);
    return QBVH_OK;
}

}  // extern "C"

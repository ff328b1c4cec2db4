// Stable LSD radix sort of (32-bit key, 32-bit value) pairs and a device-wide
// exclusive scan, written for wave64 (gfx950).
//
// The Z-order sort is the step the paper singles out as the largest part of
// the build (Section 2.2 opening; Section 3 uses a stable library sort so the
// result is deterministic).  Here it is four 8-bit passes of
// reduce-then-scan: per-tile digit histograms, a per-digit scan across tiles,
// then a scatter that ranks each tile stably with wave ballots (one peer mask
// per digit value and wave, popcount below the lane) and writes through LDS
// so that global stores land in contiguous runs.  No workgroup waits on
// another, so every wave always finishes.
#include "qbvh_internal.h"

namespace qbi {
namespace {

constexpr int kRadixBits = 8;
constexpr int kRadix = 1 << kRadixBits;
constexpr int kSortWaves = 8;
constexpr int kSortThreads = kSortWaves * 64;       // 512
constexpr int kSortItems = 8;
constexpr int kSortTile = kSortThreads * kSortItems;  // 4096 keys per tile
constexpr int kHistThreads = 256;

constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanThreads * kScanItems;  // 2048

__device__ __forceinline__ uint32_t wave_inclusive_scan(uint32_t v) {
    const int lane = __lane_id();
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        uint32_t t = __shfl_up(v, o, 64);
        if (lane >= o) v += t;
    }
    return v;
}

// Exclusive scan over a workgroup of NT threads; `total` receives the sum.
// `lds` needs NT/64 entries.  Contains barriers: every thread must call it.
template <int NT>
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t *lds, uint32_t &total) {
    constexpr int NW = NT / 64;
    const int lane = __lane_id();
    const int wave = threadIdx.x >> 6;
    uint32_t incl = wave_inclusive_scan(v);
    if (lane == 63) lds[wave] = incl;
    __syncthreads();
    uint32_t wsum = 0, wtot = 0;
#pragma unroll
    for (int w = 0; w < NW; ++w) {
        uint32_t x = lds[w];
        if (w < wave) wsum += x;
        wtot += x;
    }
    __syncthreads();
    total = wtot;
    return wsum + incl - v;
}

// Tile geometry.  Single array: tile t covers [4096 t, 4096 (t + 1)) and its
// count of digit d sits at hist[d * tiles + t].  Segmented (a batch of
// independent arrays laid end to end): tiles never straddle a segment, and
// the counts of segment s are stored digit-major after those of the segments
// before it, so one exclusive scan over the whole histogram array yields every
// tile's output offset for every digit directly (segment start + counts of
// smaller digits in the segment + counts of the same digit in earlier tiles).
struct TileView {
    int64_t base;     // first element of the tile
    int32_t nvalid;   // elements in the tile
    int64_t hbase;    // histogram index of digit 0
    int32_t hstride;  // histogram distance between digits
};

template <bool kSeg>
__device__ __forceinline__ TileView tile_view(int32_t tile, int32_t n, int32_t tiles, const int32_t *tile_first,
                                              const int32_t *seg_off, int32_t nseg) {
    TileView v;
    if (!kSeg) {
        v.base = (int64_t)tile * kSortTile;
        const int64_t rem = (int64_t)n - v.base;
        v.nvalid = rem < kSortTile ? (int32_t)rem : kSortTile;
        v.hbase = tile;
        v.hstride = tiles;
    } else {
        const int32_t s = find_seg(tile_first, nseg, tile);
        const int32_t lt = tile - tile_first[s];
        const int32_t ntl = tile_first[s + 1] - tile_first[s];
        v.base = (int64_t)seg_off[s] + (int64_t)lt * kSortTile;
        const int64_t rem = (int64_t)seg_off[s + 1] - v.base;
        v.nvalid = rem < kSortTile ? (int32_t)rem : kSortTile;
        v.hbase = (int64_t)kRadix * tile_first[s] + lt;
        v.hstride = ntl;
    }
    return v;
}

template <bool kSeg>
__global__ __launch_bounds__(kHistThreads) void k_radix_hist(const uint32_t *__restrict__ keys, int32_t n,
                                                             int32_t shift, uint32_t *__restrict__ hist,
                                                             int32_t tiles, const int32_t *__restrict__ tile_first,
                                                             const int32_t *__restrict__ seg_off, int32_t nseg) {
    __shared__ uint32_t h[kHistThreads / 64][kRadix];
    const int tid = threadIdx.x;
    const int wave = tid >> 6;
    const TileView tv = tile_view<kSeg>(blockIdx.x, n, tiles, tile_first, seg_off, nseg);
    for (int i = tid; i < (kHistThreads / 64) * kRadix; i += kHistThreads) (&h[0][0])[i] = 0;
    __syncthreads();
#pragma unroll 4
    for (int i = 0; i < kSortTile / kHistThreads; ++i) {
        const int j = i * kHistThreads + tid;
        if (j < tv.nvalid) atomicAdd(&h[wave][(keys[tv.base + j] >> shift) & (kRadix - 1)], 1u);
    }
    __syncthreads();
    uint32_t c = 0;
#pragma unroll
    for (int w = 0; w < kHistThreads / 64; ++w) c += h[w][tid];
    hist[tv.hbase + (int64_t)tid * tv.hstride] = c;
}

// One workgroup per digit: exclusive scan of that digit's tile counts in place.
__global__ __launch_bounds__(kScanThreads) void k_radix_digit_scan(uint32_t *__restrict__ hist, int32_t tiles,
                                                                   uint32_t *__restrict__ digit_total) {
    __shared__ uint32_t lds[kScanThreads / 64];
    uint32_t *row = hist + (int64_t)blockIdx.x * tiles;
    uint32_t carry = 0;
    for (int32_t b0 = 0; b0 < tiles; b0 += kScanThreads * 4) {
        uint32_t v[4];
        uint32_t s = 0;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            int32_t idx = b0 + threadIdx.x * 4 + k;
            v[k] = idx < tiles ? row[idx] : 0u;
            s += v[k];
        }
        uint32_t tot;
        uint32_t ex = block_exclusive_scan<kScanThreads>(s, lds, tot) + carry;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            int32_t idx = b0 + threadIdx.x * 4 + k;
            if (idx < tiles) row[idx] = ex;
            ex += v[k];
        }
        carry += tot;
    }
    if (threadIdx.x == 0) digit_total[blockIdx.x] = carry;
}

template <bool kSeg>
__global__ __launch_bounds__(kSortThreads) void k_radix_scatter(
    const uint32_t *__restrict__ keys_in, const uint32_t *__restrict__ vals_in, uint32_t *__restrict__ keys_out,
    uint32_t *__restrict__ vals_out, int32_t n, int32_t shift, const uint32_t *__restrict__ hist,
    const uint32_t *__restrict__ digit_total, int32_t tiles, const int32_t *__restrict__ tile_first,
    const int32_t *__restrict__ seg_off, int32_t nseg) {
    __shared__ uint32_t s_keys[kSortTile];
    __shared__ uint32_t s_vals[kSortTile];
    __shared__ uint32_t s_wcnt[kSortWaves][kRadix];
    __shared__ uint32_t s_dstart[kRadix];
    __shared__ uint32_t s_goff[kRadix];
    __shared__ uint32_t s_scan[kSortWaves];

    const int tid = threadIdx.x;
    const int lane = __lane_id();
    const int wave = tid >> 6;
    const TileView tv = tile_view<kSeg>(blockIdx.x, n, tiles, tile_first, seg_off, nseg);
    const int64_t base = tv.base;

    for (int i = tid; i < kSortWaves * kRadix; i += kSortThreads) (&s_wcnt[0][0])[i] = 0;

    if (!kSeg) {
        // global start of each digit: exclusive scan of the digit totals
        uint32_t dt = tid < kRadix ? digit_total[tid] : 0u;
        uint32_t tot;
        uint32_t gstart = block_exclusive_scan<kSortThreads>(dt, s_scan, tot);
        if (tid < kRadix) s_goff[tid] = gstart + hist[tv.hbase + (int64_t)tid * tv.hstride];
    } else if (tid < kRadix) {
        // the histogram array has been scanned as a whole: offsets are final
        s_goff[tid] = hist[tv.hbase + (int64_t)tid * tv.hstride];
    }
    __syncthreads();

    uint32_t k[kSortItems], v[kSortItems], r[kSortItems];
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
#pragma unroll
    for (int i = 0; i < kSortItems; ++i) {
        const int32_t j = wave * 64 * kSortItems + i * 64 + lane;
        const bool valid = j < tv.nvalid;
        const int64_t idx = base + j;
        k[i] = valid ? keys_in[idx] : 0u;
        v[i] = valid ? vals_in[idx] : 0u;
    }
    // Stable rank within the wave's chunk: items in order i, then lane.
#pragma unroll
    for (int i = 0; i < kSortItems; ++i) {
        const bool valid = wave * 64 * kSortItems + i * 64 + lane < tv.nvalid;
        uint32_t d = (k[i] >> shift) & (kRadix - 1);
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < kRadixBits; ++b) {
            bool bit = (d >> b) & 1u;
            uint64_t m = __ballot(bit);
            peers &= bit ? m : ~m;
        }
        if (valid) {
            uint32_t before = s_wcnt[wave][d];
            uint32_t rk = (uint32_t)__popcll(peers & lt_mask);
            r[i] = before + rk;
            if (rk == 0) s_wcnt[wave][d] = before + (uint32_t)__popcll(peers);
        }
    }
    __syncthreads();

    uint32_t cnt = 0;
    if (tid < kRadix) {
        uint32_t sum = 0;
#pragma unroll
        for (int w = 0; w < kSortWaves; ++w) {
            uint32_t c = s_wcnt[w][tid];
            s_wcnt[w][tid] = sum;
            sum += c;
        }
        cnt = sum;
    }
    {
        uint32_t tot;
        uint32_t ds = block_exclusive_scan<kSortThreads>(cnt, s_scan, tot);
        if (tid < kRadix) s_dstart[tid] = ds;
    }
    __syncthreads();

#pragma unroll
    for (int i = 0; i < kSortItems; ++i) {
        if (wave * 64 * kSortItems + i * 64 + lane < tv.nvalid) {
            uint32_t d = (k[i] >> shift) & (kRadix - 1);
            uint32_t p = s_dstart[d] + s_wcnt[wave][d] + r[i];
            s_keys[p] = k[i];
            s_vals[p] = v[i];
        }
    }
    __syncthreads();

    for (int j = tid; j < tv.nvalid; j += kSortThreads) {
        uint32_t key = s_keys[j];
        uint32_t d = (key >> shift) & (kRadix - 1);
        uint32_t g = s_goff[d] + (uint32_t)j - s_dstart[d];
        keys_out[g] = key;
        vals_out[g] = s_vals[j];
    }
}

// A whole sort of at most one tile in one workgroup: the four passes of the
// tile scatter above, each leaving the tile in LDS for the next (a small
// system's sort in one launch instead of twelve).
__global__ __launch_bounds__(kSortThreads) void k_radix_sort_tile(uint32_t *__restrict__ keys,
                                                                  uint32_t *__restrict__ vals, int32_t n) {
    __shared__ uint32_t s_keys[kSortTile];
    __shared__ uint32_t s_vals[kSortTile];
    __shared__ uint32_t s_wcnt[kSortWaves][kRadix];
    __shared__ uint32_t s_dstart[kRadix];
    __shared__ uint32_t s_scan[kSortWaves];

    const int tid = threadIdx.x;
    const int lane = __lane_id();
    const int wave = tid >> 6;
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    uint32_t k[kSortItems], v[kSortItems], r[kSortItems];
#pragma unroll
    for (int i = 0; i < kSortItems; ++i) {
        const int32_t j = wave * 64 * kSortItems + i * 64 + lane;
        k[i] = j < n ? keys[j] : 0u;
        v[i] = j < n ? vals[j] : 0u;
    }
    for (int pass = 0; pass < 32 / kRadixBits; ++pass) {
        const int shift = pass * kRadixBits;
        for (int i = tid; i < kSortWaves * kRadix; i += kSortThreads) (&s_wcnt[0][0])[i] = 0;
        __syncthreads();
        // stable rank within the wave's chunk: items in order i, then lane
#pragma unroll
        for (int i = 0; i < kSortItems; ++i) {
            const bool valid = wave * 64 * kSortItems + i * 64 + lane < n;
            const uint32_t d = (k[i] >> shift) & (kRadix - 1);
            uint64_t peers = __ballot(valid);
#pragma unroll
            for (int b = 0; b < kRadixBits; ++b) {
                const bool bit = (d >> b) & 1u;
                const uint64_t m = __ballot(bit);
                peers &= bit ? m : ~m;
            }
            if (valid) {
                const uint32_t before = s_wcnt[wave][d];
                const uint32_t rk = (uint32_t)__popcll(peers & lt_mask);
                r[i] = before + rk;
                if (rk == 0) s_wcnt[wave][d] = before + (uint32_t)__popcll(peers);
            }
        }
        __syncthreads();
        uint32_t cnt = 0;
        if (tid < kRadix) {
            uint32_t sum = 0;
#pragma unroll
            for (int w = 0; w < kSortWaves; ++w) {
                const uint32_t c = s_wcnt[w][tid];
                s_wcnt[w][tid] = sum;
                sum += c;
            }
            cnt = sum;
        }
        {
            uint32_t tot;
            const uint32_t ds = block_exclusive_scan<kSortThreads>(cnt, s_scan, tot);
            if (tid < kRadix) s_dstart[tid] = ds;
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < kSortItems; ++i) {
            if (wave * 64 * kSortItems + i * 64 + lane < n) {
                const uint32_t d = (k[i] >> shift) & (kRadix - 1);
                const uint32_t p = s_dstart[d] + s_wcnt[wave][d] + r[i];
                s_keys[p] = k[i];
                s_vals[p] = v[i];
            }
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < kSortItems; ++i) {
            const int32_t j = wave * 64 * kSortItems + i * 64 + lane;
            if (j < n) {
                k[i] = s_keys[j];
                v[i] = s_vals[j];
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < kSortItems; ++i) {
        const int32_t j = wave * 64 * kSortItems + i * 64 + lane;
        if (j < n) {
            keys[j] = k[i];
            vals[j] = v[i];
        }
    }
}

// ---------------------------------------------------------------- exclusive scan

// A thread's kScanItems consecutive entries: two 16-byte loads when all are in
// range (the array is 32-byte aligned, checked on the host), else one by one.
__device__ __forceinline__ void load_items(const uint32_t *__restrict__ data, int64_t base, int32_t len,
                                           uint32_t (&v)[kScanItems]) {
    static_assert(kScanItems == 8, "two 16-byte loads per thread");
    if (base + kScanItems <= len) {
        const uint4 a = reinterpret_cast<const uint4 *>(data + base)[0];
        const uint4 b = reinterpret_cast<const uint4 *>(data + base)[1];
        v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
        v[4] = b.x; v[5] = b.y; v[6] = b.z; v[7] = b.w;
    } else {
#pragma unroll
        for (int k = 0; k < kScanItems; ++k) v[k] = (base + k < len) ? data[base + k] : 0u;
    }
}

__global__ __launch_bounds__(kScanThreads) void k_scan_reduce(const uint32_t *__restrict__ data, int32_t len,
                                                              uint32_t *__restrict__ partials) {
    __shared__ uint32_t lds[kScanThreads / 64];
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    uint32_t v[kScanItems];
    load_items(data, base, len, v);
    uint32_t s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) s += v[k];
    uint32_t tot;
    (void)block_exclusive_scan<kScanThreads>(s, lds, tot);
    if (threadIdx.x == 0) partials[blockIdx.x] = tot;
}

__global__ __launch_bounds__(1024) void k_scan_partials(uint32_t *__restrict__ partials, int32_t nb) {
    __shared__ uint32_t lds[1024 / 64];
    uint32_t carry = 0;
    for (int32_t b0 = 0; b0 < nb; b0 += 1024) {
        int32_t idx = b0 + threadIdx.x;
        uint32_t v = idx < nb ? partials[idx] : 0u;
        uint32_t tot;
        uint32_t ex = block_exclusive_scan<1024>(v, lds, tot) + carry;
        if (idx < nb) partials[idx] = ex;
        carry += tot;
    }
}

// A short array in one workgroup: chunk by chunk with a running carry (one
// launch instead of three).
__global__ __launch_bounds__(kScanThreads) void k_scan_single(uint32_t *__restrict__ data, int32_t len) {
    __shared__ uint32_t lds[kScanThreads / 64];
    uint32_t carry = 0;
    for (int64_t b0 = 0; b0 < len; b0 += kScanTile) {
        const int64_t base = b0 + (int64_t)threadIdx.x * kScanItems;
        uint32_t v[kScanItems];
        uint32_t s = 0;
#pragma unroll
        for (int k = 0; k < kScanItems; ++k) {
            v[k] = (base + k < len) ? data[base + k] : 0u;
            s += v[k];
        }
        uint32_t tot;
        uint32_t ex = block_exclusive_scan<kScanThreads>(s, lds, tot) + carry;
#pragma unroll
        for (int k = 0; k < kScanItems; ++k) {
            if (base + k < len) data[base + k] = ex;
            ex += v[k];
        }
        carry += tot;
    }
}

__global__ __launch_bounds__(kScanThreads) void k_scan_down(uint32_t *__restrict__ data, int32_t len,
                                                            const uint32_t *__restrict__ partials) {
    __shared__ uint32_t lds[kScanThreads / 64];
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    uint32_t v[kScanItems];
    load_items(data, base, len, v);
    uint32_t s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) s += v[k];
    uint32_t tot;
    uint32_t ex = block_exclusive_scan<kScanThreads>(s, lds, tot) + partials[blockIdx.x];
    uint32_t o[kScanItems];
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        o[k] = ex;
        ex += v[k];
    }
    if (base + kScanItems <= len) {
        reinterpret_cast<uint4 *>(data + base)[0] = make_uint4(o[0], o[1], o[2], o[3]);
        reinterpret_cast<uint4 *>(data + base)[1] = make_uint4(o[4], o[5], o[6], o[7]);
    } else {
#pragma unroll
        for (int k = 0; k < kScanItems; ++k)
            if (base + k < len) data[base + k] = o[k];
    }
}

}  // namespace

int32_t radix_tiles(int32_t n) { return n <= 0 ? 1 : (n + kSortTile - 1) / kSortTile; }
int32_t scan_blocks(int32_t len) { return len <= 0 ? 1 : (len + kScanTile - 1) / kScanTile; }

hipError_t launch_radix_sort(uint32_t *keys, uint32_t *vals, uint32_t *keys2, uint32_t *vals2, uint32_t *hist,
                             uint32_t *digit_total, int32_t n, int32_t tiles, hipStream_t s) {
    if (n <= 1) return hipSuccess;
    if (n <= kSortTile) {
        hipLaunchKernelGGL(k_radix_sort_tile, dim3(1), dim3(kSortThreads), 0, s, keys, vals, n);
        return hipGetLastError();
    }
    const int32_t t = radix_tiles(n);
    (void)tiles;
    uint32_t *ki = keys, *vi = vals, *ko = keys2, *vo = vals2;
    for (int pass = 0; pass < 32 / kRadixBits; ++pass) {
        const int shift = pass * kRadixBits;
        hipLaunchKernelGGL(k_radix_hist<false>, dim3(t), dim3(kHistThreads), 0, s, ki, n, shift, hist, t,
                           nullptr, nullptr, 0);
        hipLaunchKernelGGL(k_radix_digit_scan, dim3(kRadix), dim3(kScanThreads), 0, s, hist, t, digit_total);
        hipLaunchKernelGGL(k_radix_scatter<false>, dim3(t), dim3(kSortThreads), 0, s, ki, vi, ko, vo, n, shift,
                           hist, digit_total, t, nullptr, nullptr, 0);
        uint32_t *tk = ki, *tv = vi;
        ki = ko;
        vi = vo;
        ko = tk;
        vo = tv;
    }
    // An even number of passes leaves the result in (keys, vals).
    static_assert((32 / kRadixBits) % 2 == 0, "result must end in the primary buffers");
    return hipGetLastError();
}

int32_t seg_radix_tiles(int32_t n) { return (n + kSortTile - 1) / kSortTile; }

hipError_t launch_radix_sort_segmented(uint32_t *keys, uint32_t *vals, uint32_t *keys2, uint32_t *vals2,
                                       uint32_t *hist, uint32_t *scan_part, int32_t n, int32_t tiles,
                                       const int32_t *tile_first, const int32_t *seg_off, int32_t nseg,
                                       hipStream_t s) {
    if (n <= 1 || tiles <= 0) return hipSuccess;
    uint32_t *ki = keys, *vi = vals, *ko = keys2, *vo = vals2;
    for (int pass = 0; pass < 32 / kRadixBits; ++pass) {
        const int shift = pass * kRadixBits;
        hipLaunchKernelGGL(k_radix_hist<true>, dim3(tiles), dim3(kHistThreads), 0, s, ki, n, shift, hist, tiles,
                           tile_first, seg_off, nseg);
        hipError_t e = launch_exclusive_scan(hist, kRadix * tiles, scan_part, s);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_radix_scatter<true>, dim3(tiles), dim3(kSortThreads), 0, s, ki, vi, ko, vo, n, shift,
                           hist, nullptr, tiles, tile_first, seg_off, nseg);
        uint32_t *tk = ki, *tv = vi;
        ki = ko;
        vi = vo;
        ko = tk;
        vo = tv;
    }
    return hipGetLastError();
}

hipError_t launch_exclusive_scan(uint32_t *data, int32_t len, uint32_t *partials, hipStream_t s) {
    if (len <= 0) return hipSuccess;
    if (len <= 4 * kScanTile) {
        hipLaunchKernelGGL(k_scan_single, dim3(1), dim3(kScanThreads), 0, s, data, len);
        return hipGetLastError();
    }
    if ((reinterpret_cast<uintptr_t>(data) & 31u) != 0) return hipErrorInvalidValue;
    const int32_t nb = scan_blocks(len);
    hipLaunchKernelGGL(k_scan_reduce, dim3(nb), dim3(kScanThreads), 0, s, data, len, partials);
    hipLaunchKernelGGL(k_scan_partials, dim3(1), dim3(1024), 0, s, partials, nb);
    hipLaunchKernelGGL(k_scan_down, dim3(nb), dim3(kScanThreads), 0, s, data, len, partials);
    return hipGetLastError();
}

}  // namespace qbi

// Device-wide exclusive prefix scan over a generated sequence.
//
// in(i) yields element i (computed on the fly, so flags need not be
// materialised); out(i, exclusive_prefix, value) consumes the result (it can
// write the prefix, or scatter/compact).  Tile sums, then the tiles
// re-scanned with their offsets; the offsets come from one workgroup scanning
// the tile sums, or, up to kScanInlineTiles tiles, each re-scanning tile adds
// up the sums before it itself (they stay in L2), which saves that launch.
// Integer sums only, so the result is independent of scheduling.
#pragma once
#include "common.hpp"

namespace bp {

constexpr int kScanItems = 8;
constexpr int kScanTile = kBlock * kScanItems;
constexpr int64_t kScanInlineTiles = 4096;

template <typename T, typename In>
__global__ __launch_bounds__(kBlock) void k_scan_tiles(In in, int64_t n, T *tile_sum)
{
    __shared__ T lds[16];
    int64_t base = (int64_t)blockIdx.x * kScanTile;
    T s = 0;
#pragma unroll
    for (int j = 0; j < kScanItems; j++) {
        int64_t i = base + j * kBlock + threadIdx.x;
        if (i < n) s += in(i);
    }
    s = block_sum(s, lds);
    if (threadIdx.x == 0) tile_sum[blockIdx.x] = s;
}

// One workgroup of 1024 threads scans the tile sums in place; total -> *total.
template <typename T> __global__ __launch_bounds__(1024) void k_scan_spine(T *tile_sum, int64_t nt, T *total)
{
    __shared__ T lds[16];
    T carry = 0;
    for (int64_t base = 0; base < nt; base += 1024) {
        int64_t i = base + threadIdx.x;
        T v = i < nt ? tile_sum[i] : T(0);
        T tot;
        T ex = block_excl_scan(v, lds, &tot);
        if (i < nt) tile_sum[i] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0) *total = carry;
}

// INLINE: tiles holds the tile sums (not yet their offsets); this tile adds
// up those before it, and the last tile writes the total.
template <typename T, typename In, typename Out, bool INLINE>
__global__ __launch_bounds__(kBlock) void k_scan_apply(In in, int64_t n, const T *tiles, Out out, T *total)
{
    __shared__ T lds[16], lds2[16];
    __shared__ T stage[kScanTile];
    T off;
    if (INLINE) {
        T s = 0;
        for (int64_t t = threadIdx.x; t < (int64_t)blockIdx.x; t += kBlock) s += tiles[t];
        off = block_sum(s, lds2);
    } else {
        off = tiles[blockIdx.x];
    }
    int64_t base = (int64_t)blockIdx.x * kScanTile;
    // coalesced load into LDS, then each thread scans a contiguous run
#pragma unroll
    for (int j = 0; j < kScanItems; j++) {
        int64_t i = base + j * kBlock + threadIdx.x;
        stage[j * kBlock + threadIdx.x] = i < n ? in(i) : T(0);
    }
    __syncthreads();
    T v[kScanItems];
    T local = 0;
#pragma unroll
    for (int j = 0; j < kScanItems; j++) {
        v[j] = stage[threadIdx.x * kScanItems + j];
        local += v[j];
    }
    T tot;
    T ex = block_excl_scan(local, lds, &tot) + off;
    if (INLINE && blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) *total = off + tot;
#pragma unroll
    for (int j = 0; j < kScanItems; j++) {
        int64_t i = base + threadIdx.x * kScanItems + j;
        if (i < n) out(i, ex, v[j]);
        ex += v[j];
    }
}

template <typename T> __global__ void k_scan_zero(T *p) { *p = T(0); }

// Scratch needed by scan(): tile sums + total.
struct ScanScratch {
    void *tiles = nullptr;
    void *total = nullptr;
    int64_t cap_tiles = 0;
};

template <typename T, typename In, typename Out>
inline void scan(LaunchCtx &lc, Arena &ar, const char *name, int64_t n, In in, Out out, T *d_total)
{
    int64_t nt = ceil_div(n > 0 ? n : 1, kScanTile);
    T *tiles = ar.get<T>(nt);
    double bytes = (double)n * 2 * sizeof(T);
    if (n <= 0) {
        launch(lc, name, 0.0, k_scan_zero<T>, 1, 1, 0, d_total);
        return;
    }
    launch(lc, name, bytes, k_scan_tiles<T, In>, nt, kBlock, 0, in, n, tiles);
    if (nt <= kScanInlineTiles) {
        launch(lc, name, bytes, k_scan_apply<T, In, Out, true>, nt, kBlock, 0, in, n, (const T *)tiles, out,
               d_total);
        return;
    }
    launch(lc, name, 0.0, k_scan_spine<T>, 1, 1024, 0, tiles, nt, d_total);
    launch(lc, name, bytes, k_scan_apply<T, In, Out, false>, nt, kBlock, 0, in, n, (const T *)tiles, out, d_total);
}

}  // namespace bp

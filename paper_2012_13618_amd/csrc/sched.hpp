// Degree-bucketed hyperedge schedules and block sorting helpers.
//
// A sweep over hyperedges runs as up to three launches: SMALL covers every
// hyperedge of degree <= 8 with one thread each (the vast majority in
// netlist and sparse-matrix hypergraphs), WAVE gives each listed hyperedge of
// degree 9..256 a wavefront (sweeps split by thread_split below take those of
// up to 32 pins one a thread as well), BLOCK gives each listed larger
// hyperedge a workgroup.  All per-pin updates are integer atomics (min/add), so
// results do not depend on which schedule processed a hyperedge.
#pragma once
#include "common.hpp"

namespace bp {

enum Sched { SMALL = 0, WAVE = 1, BLOCK = 2 };

// Sweeps whose per-hyperedge work is a plain loop over the pins take the
// listed hyperedges of up to kHedgeThreadMax pins one a thread as well: a
// wavefront on a 9..32-pin hyperedge leaves most lanes idle and adds a
// reduction.  thread_split<S>(d): whether schedule S takes a hyperedge of d
// pins in such a sweep (SMALL up to the limit, WAVE above it).
constexpr int32_t kHedgeThreadMax = 32;
template <int S> __device__ __forceinline__ bool thread_split(int32_t d)
{
    return S == SMALL ? d <= kHedgeThreadMax : (S == WAVE ? d > kHedgeThreadMax : true);
}

// Hyperedge handled by this thread's group in block vb of its schedule, or
// -1.  lane/stride give the thread's position within the group.  For SMALL
// the caller still has to skip hyperedges above kSmallMax (or, in a sweep
// split by thread_split, above kHedgeThreadMax, which WAVE then skips).
template <int S>
__device__ __forceinline__ int32_t sched_hedge_at(int64_t vb, int32_t count, const int32_t *list, int &lane,
                                                  int &stride)
{
    if (S == SMALL) {
        int64_t e = vb * blockDim.x + threadIdx.x;
        lane = 0;
        stride = 1;
        return e < count ? (int32_t)e : -1;
    } else if (S == WAVE) {
        int64_t w = (vb * blockDim.x + threadIdx.x) >> 6;
        lane = threadIdx.x & 63;
        stride = 64;
        return w < count ? list[w] : -1;
    } else {
        lane = threadIdx.x;
        stride = blockDim.x;
        return vb < count ? list[vb] : -1;
    }
}

template <int S>
__device__ __forceinline__ int32_t sched_hedge(int32_t count, const int32_t *list, int &lane,
                                               int &stride)
{
    return sched_hedge_at<S>(blockIdx.x, count, list, lane, stride);
}

// All three buckets of a hyperedge sweep in one launch: blocks [0, ns) take
// every hyperedge of degree <= kSmallMax one per thread, the next ones the
// listed mid hyperedges one per wavefront, the last ones the listed big
// hyperedges one per workgroup; op.run<S>(vb, count, list) does the work of
// block vb of schedule S.  The buckets are disjoint, so they run together.
inline int64_t buckets_grid(int64_t E, int64_t nmid, int64_t nbig)
{
    return ceil_div(E, kBlock) + ceil_div(nmid, kBlock / 64) + nbig;
}

template <typename Op>
__global__ __launch_bounds__(kBlock) void k_buckets(Op op, int32_t E, int32_t nmid, const int32_t *lmid,
                                                    int32_t nbig, const int32_t *lbig)
{
    int64_t b = blockIdx.x, ns = ceil_div(E, kBlock), nw = ceil_div(nmid, kBlock / 64);
    if (b < ns) op.template run<SMALL>(b, E, nullptr);
    else if (b < ns + nw) op.template run<WAVE>(b - ns, nmid, lmid);
    else op.template run<BLOCK>(b - ns - nw, nbig, lbig);
}

template <int S> inline int64_t sched_grid(int64_t count)
{
    if (S == SMALL) return ceil_div(count, kBlock);
    if (S == WAVE) return ceil_div(count, kBlock / kWave);
    return count;
}

// Group-wide reductions matching the schedule (SMALL: the thread is the group).
template <int S, typename T> __device__ __forceinline__ T group_sum(T v, T *lds)
{
    if (S == SMALL) return v;
    if (S == WAVE) return wave_sum(v);
    return block_sum(v, lds);
}
template <int S, typename T> __device__ __forceinline__ T group_min(T v, T *lds)
{
    if (S == SMALL) return v;
    if (S == WAVE) return wave_min(v);
    return block_min(v, lds);
}

// Ascending bitonic sort of n (a power of two) keys by the whole workgroup.
// a may point to LDS or to global memory private to the workgroup.
template <typename K> __device__ void block_bitonic_sort(K *a, int n)
{
    for (int k = 2; k <= n; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int i = threadIdx.x; i < n; i += blockDim.x) {
                int p = i ^ j;
                if (p > i) {
                    K x = a[i], y = a[p];
                    bool up = (i & k) == 0;
                    if ((x > y) == up) {
                        a[i] = y;
                        a[p] = x;
                    }
                }
            }
            __syncthreads();
        }
    }
}

// Ascending order of cnt distinct keys by counting: key i goes to out[rank],
// rank = the number of smaller keys.  One barrier instead of a bitonic
// network's log^2 ones; O(cnt^2 / threads) comparisons, for short lists.
template <typename K> __device__ __forceinline__ void block_rank_sort(const K *in, K *out, int cnt)
{
    // tpc adjacent lanes per key (a power of two up to 16, as the workgroup
    // allows), each counting every tpc-th key; cnt is the same in every thread
    int tpc = 1;
    while (tpc < 16 && cnt * 2 * tpc <= (int)blockDim.x) tpc <<= 1;
    for (int base = 0; base < cnt * tpc; base += blockDim.x) {
        int t = base + (int)threadIdx.x, i = t / tpc, part = t & (tpc - 1);
        K x = in[i < cnt ? i : 0];
        int r = 0;
        if (i < cnt) {
#pragma unroll 8
            for (int j = part; j < cnt; j += tpc) r += in[j] < x;
        }
        for (int o = 1; o < tpc; o <<= 1) r += __shfl_xor(r, o, 64);
        if (i < cnt && part == 0) out[r] = x;
    }
    __syncthreads();
}

// Same, but each wavefront sorts its own n-key slice (n a power of two); the
// loop shape is identical for every wave so a workgroup barrier can be used.
template <typename K> __device__ void wave_bitonic_sort(K *a, int n)
{
    int lane = threadIdx.x & 63;
    for (int k = 2; k <= n; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int i = lane; i < n; i += 64) {
                int p = i ^ j;
                if (p > i) {
                    K x = a[i], y = a[p];
                    bool up = (i & k) == 0;
                    if ((x > y) == up) {
                        a[i] = y;
                        a[p] = x;
                    }
                }
            }
            __syncthreads();
        }
    }
}

__host__ __device__ inline int next_pow2(int x)
{
    int p = 1;
    while (p < x) p <<= 1;
    return p;
}

template <typename T> __global__ void k_fill(T *p, int64_t n, T v)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

template <typename T> inline void fill(LaunchCtx &lc, T *p, int64_t n, T v)
{
    if (n <= 0) return;
    int64_t g = ceil_div(n, kBlock);
    if (g > 4096) g = 4096;
    launch(lc, "fill", (double)n * sizeof(T), k_fill<T>, g, kBlock, 0, p, n, v);
}

// Several arrays filled in one launch (grid y = array): up to kFillMax of
// them, elements of 1, 4 or 8 bytes.
constexpr int kFillMax = 6;
struct FillSet {
    void *p[kFillMax];
    int64_t n[kFillMax];
    uint64_t v[kFillMax];
    int32_t size[kFillMax];
};

__global__ __launch_bounds__(kBlock) void k_fill_set(FillSet fs)
{
    int k = blockIdx.y;
    int64_t n = fs.n[k];
    uint64_t v = fs.v[k];
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        if (fs.size[k] == 1) ((uint8_t *)fs.p[k])[i] = (uint8_t)v;
        else if (fs.size[k] == 4) ((uint32_t *)fs.p[k])[i] = (uint32_t)v;
        else ((uint64_t *)fs.p[k])[i] = v;
    }
}

class Fills {
  public:
    template <typename T> Fills &add(T *p, int64_t n, T v)
    {
        static_assert(sizeof(T) == 1 || sizeof(T) == 4 || sizeof(T) == 8, "element size");
        if (n <= 0) return *this;
        if (k_ == kFillMax) throw Error(BP_ERR_DEVICE, "too many arrays in one fill");
        uint64_t bits = 0;
        __builtin_memcpy(&bits, &v, sizeof(T));
        fs_.p[k_] = (void *)p;
        fs_.n[k_] = n;
        fs_.v[k_] = bits;
        fs_.size[k_] = (int32_t)sizeof(T);
        g_ = std::max<int64_t>(g_, std::min<int64_t>(ceil_div(n, kBlock), 4096));
        bytes_ += (double)n * sizeof(T);
        k_++;
        return *this;
    }
    void run(LaunchCtx &lc)
    {
        if (k_ == 0) return;
        launch3(lc, "fill", bytes_, k_fill_set, dim3((unsigned)g_, (unsigned)k_, 1), kBlock, 0, fs_);
        k_ = 0;
        g_ = 0;
        bytes_ = 0.0;
    }

  private:
    FillSet fs_{};
    int k_ = 0;
    int64_t g_ = 0;
    double bytes_ = 0.0;
};

}  // namespace bp

// Shared helpers of the gfx950 partitioner: error handling, launch wrapper,
// device memory arena, hashing and wave64/workgroup reductions and scans.
#pragma once
#include <atomic>

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <mutex>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/bipart.h"

namespace bp {

constexpr int kBlock = 256;           // threads per workgroup for sweeps
constexpr int kWave = 64;             // CDNA wavefront
constexpr int kSmallMax = 8;          // hyperedges up to this degree: one thread each
constexpr int kMidMax = 256;          // up to this degree: one wavefront each
constexpr int kBigMax = 8192;         // up to this degree: one workgroup, sorted in LDS
constexpr uint64_t kNoKey = ~0ull;

struct Error : std::runtime_error {
    bp_status status;
    Error(bp_status s, const std::string &m) : std::runtime_error(m), status(s) {}
};

inline void hip_check(hipError_t e, const char *what)
{
    if (e == hipSuccess) return;
    if (e == hipErrorOutOfMemory)
        throw Error(BP_ERR_OUT_OF_MEMORY, std::string(what) + ": " + hipGetErrorString(e));
    throw Error(BP_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}
#define BP_HIP(call) ::bp::hip_check((call), #call)

__host__ __device__ inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Reductions over all nodes that end in per-segment atomics run on at most
// this many workgroups, each over a contiguous chunk of whole tiles: a global
// atomic on one address costs about 11 ns and serialises across workgroups.
constexpr int64_t kReduceBlocks = 512;
__host__ __device__ inline int64_t reduce_grid(int64_t n)
{
    int64_t g = ceil_div(n, 256);
    return g < kReduceBlocks ? g : kReduceBlocks;
}
// Workgroups of a launch go to the 8 XCDs in turn (workgroup b to XCD b mod 8),
// and each XCD has its own L2.  xcd_block renumbers workgroups 0 .. n-1 so
// that each XCD takes one contiguous run of the n logical blocks: chunks
// that gather from the same neighbourhood (one graph of a batch) share an L2.
__device__ __forceinline__ int64_t xcd_block(int64_t b, int64_t n)
{
    constexpr int64_t X = 8;
    int64_t q = n / X, r = n % X, x = b % X, k = b / X;
    return x < r ? x * (q + 1) + k : r * (q + 1) + (x - r) * q + k;
}
// lists (two per segment) a chunk aggregates in LDS before its atomics
constexpr int kAggLists = 64;
// [lo, hi): chunk of workgroup b of g over n items, in tiles of 256
__host__ __device__ inline void reduce_chunk(int64_t n, int64_t g, int64_t b, int64_t &lo, int64_t &hi)
{
    int64_t per = ceil_div(ceil_div(n, 256), g) * 256;
    lo = b * per < n ? b * per : n;
    hi = lo + per < n ? lo + per : n;
}

// ---- per-kernel timing (bp_profile_*) ---------------------------------------

struct Profiler {
    std::mutex mu;
    bool on = false;
    struct Acc {
        std::string name;
        int64_t launches = 0;
        double ms = 0, bytes = 0;
    };
    std::vector<Acc> acc;
    static Profiler &get()
    {
        static Profiler p;
        return p;
    }
    void add(const char *name, double ms, double bytes)
    {
        std::lock_guard<std::mutex> g(mu);
        for (auto &a : acc)
            if (a.name == name) {
                a.launches++;
                a.ms += ms;
                a.bytes += bytes;
                return;
            }
        acc.push_back({name, 1, ms, bytes});
    }
    // bytes a family's kernels counted on the device (no launch, no time)
    void add_bytes(const char *name, double bytes)
    {
        std::lock_guard<std::mutex> g(mu);
        for (auto &a : acc)
            if (a.name == name) {
                a.bytes += bytes;
                return;
            }
        acc.push_back({name, 0, 0.0, bytes});
    }
};

// Launch bookkeeping for one call: counts launches, and when profiling is on
// brackets each launch with events on its stream.
struct LaunchCtx {
    hipStream_t stream = nullptr;
    int32_t launches = 0;
    int32_t syncs = 0;
    bool prof = false;
    struct Pending {
        const char *name;
        double bytes;
        hipEvent_t a, b;
        int64_t serial;
    };
    int64_t serial = 0;  // launches recorded so far (profiling)
    int hold = 0;        // > 0: keep timings pending (a chunk of rounds is open)
    std::vector<Pending> pending;
    std::vector<hipEvent_t> pool;

    hipEvent_t ev()
    {
        if (!pool.empty()) {
            hipEvent_t e = pool.back();
            pool.pop_back();
            return e;
        }
        hipEvent_t e;
        BP_HIP(hipEventCreate(&e));
        return e;
    }
    void flush()
    {
        if (pending.empty()) return;
        BP_HIP(hipStreamSynchronize(stream));
        for (auto &p : pending) {
            float ms = 0;
            BP_HIP(hipEventElapsedTime(&ms, p.a, p.b));
            Profiler::get().add(p.name, ms, p.bytes);
            pool.push_back(p.a);
            pool.push_back(p.b);
        }
        pending.clear();
    }
    ~LaunchCtx()
    {
        try {
            flush();
        } catch (...) {
        }
        for (auto e : pool) (void)hipEventDestroy(e);
    }
    void sync(bool flush_timings = true)
    {
        syncs++;
        BP_HIP(hipStreamSynchronize(stream));
        if (prof && flush_timings) flush();
    }
    // Launches with serial in [lo, hi) turned out to have no work (a round
    // that found nothing to do): they keep their time but count no bytes.
    void no_bytes(int64_t lo, int64_t hi)
    {
        for (auto &p : pending)
            if (p.serial >= lo && p.serial < hi) p.bytes = 0.0;
    }
};

template <typename K, typename... Args>
inline void launch3(LaunchCtx &lc, const char *name, double bytes, K kernel, dim3 grid, int block,
                    size_t lds, Args... args)
{
    if (grid.x == 0 || grid.y == 0 || grid.z == 0) return;
    hipEvent_t a = nullptr, b = nullptr;
    if (lc.prof) {
        a = lc.ev();
        b = lc.ev();
        BP_HIP(hipEventRecord(a, lc.stream));
    }
    hipLaunchKernelGGL(kernel, grid, dim3(block), lds, lc.stream, args...);
    BP_HIP(hipGetLastError());
    lc.launches++;
    if (lc.prof) {
        BP_HIP(hipEventRecord(b, lc.stream));
        lc.pending.push_back({name, bytes, a, b, lc.serial++});
        if (lc.pending.size() > 4096 && !lc.hold) lc.flush();
    }
}

template <typename K, typename... Args>
inline void launch(LaunchCtx &lc, const char *name, double bytes, K kernel, int64_t grid,
                   int block, size_t lds, Args... args)
{
    if (grid <= 0) return;
    if (grid > 0x7fffffff) throw Error(BP_ERR_INVALID_ARG, "grid too large");
    hipEvent_t a = nullptr, b = nullptr;
    if (lc.prof) {
        a = lc.ev();
        b = lc.ev();
        BP_HIP(hipEventRecord(a, lc.stream));
    }
    hipLaunchKernelGGL(kernel, dim3((unsigned)grid), dim3(block), lds, lc.stream, args...);
    BP_HIP(hipGetLastError());
    lc.launches++;
    if (lc.prof) {
        BP_HIP(hipEventRecord(b, lc.stream));
        lc.pending.push_back({name, bytes, a, b, lc.serial++});
        if (lc.pending.size() > 4096 && !lc.hold) lc.flush();
    }
}

// ---- device memory arena ----------------------------------------------------
// Bump allocator over large hipMalloc blocks; reset() keeps the blocks for
// reuse by the next call, so steady-state calls allocate nothing.  An arena
// made with adopt() works inside one caller-provided block instead and never
// allocates: running out of it is BP_ERR_OUT_OF_MEMORY.

// Process-wide ceiling on the device memory one arena may hold (0 = none).
inline std::atomic<int64_t> g_arena_limit{0};

class Arena {
  public:
    ~Arena() { release(); }
    // Use [base, base + size) as the only block; nothing is ever allocated or freed.
    void adopt(void *base, size_t size)
    {
        release();
        fixed_ = true;
        blocks_.push_back({(char *)base, size, 0});
    }
    void *alloc(size_t bytes)
    {
        bytes = (bytes + 255) & ~size_t(255);
        if (bytes == 0) bytes = 256;
        while (cur_ < blocks_.size()) {
            Block &b = blocks_[cur_];
            if (b.used + bytes <= b.size) {
                void *p = b.ptr + b.used;
                b.used += bytes;
                return p;
            }
            if (fixed_) break;
            cur_++;
        }
        if (fixed_)
            throw Error(BP_ERR_OUT_OF_MEMORY, "the fixed device workspace of " +
                                                  std::to_string(blocks_.empty() ? 0 : blocks_[0].size) +
                                                  " bytes is too small for this input");
        size_t sz = bytes > kChunk ? bytes : kChunk;
        int64_t lim = g_arena_limit.load();
        if (lim > 0 && (int64_t)(reserved() + sz) > lim)
            throw Error(BP_ERR_OUT_OF_MEMORY, "device memory limit of " + std::to_string(lim) +
                                                  " bytes per call reached");
        char *p = nullptr;
        hipError_t e = hipMalloc(&p, sz);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            throw Error(BP_ERR_OUT_OF_MEMORY, "hipMalloc of " + std::to_string(sz) + " bytes failed");
        }
        blocks_.push_back({p, sz, bytes});
        cur_ = blocks_.size() - 1;
        return p;
    }
    template <typename T> T *get(int64_t n) { return (T *)alloc(sizeof(T) * (size_t)(n > 0 ? n : 1)); }
    void reset()
    {
        for (auto &b : blocks_) b.used = 0;
        cur_ = 0;
    }
    // Frees every block beyond the first `keep` bytes' worth (blocks are
    // freed whole, last first); call only between calls (after reset()).
    void trim(size_t keep)
    {
        if (fixed_) return;
        size_t total = reserved();
        while (!blocks_.empty() && total > keep) {
            total -= blocks_.back().size;
            (void)hipFree(blocks_.back().ptr);
            blocks_.pop_back();
        }
        cur_ = 0;
    }
    void release()
    {
        if (!fixed_)
            for (auto &b : blocks_) (void)hipFree(b.ptr);
        blocks_.clear();
        cur_ = 0;
    }
    // bytes handed out since the last reset (what the current call holds)
    size_t used() const
    {
        size_t s = 0;
        for (auto &b : blocks_) s += b.used;
        return s;
    }
    size_t reserved() const
    {
        size_t s = 0;
        for (auto &b : blocks_) s += b.size;
        return s;
    }

  private:
    static constexpr size_t kChunk = size_t(64) << 20;
    struct Block {
        char *ptr;
        size_t size, used;
    };
    std::vector<Block> blocks_;
    size_t cur_ = 0;
    bool fixed_ = false;
};

// ---- hashing -----------------------------------------------------------------

// MurmurHash3 32-bit finalizer (Appleby); a bijection on 32-bit words.
__host__ __device__ __forceinline__ uint32_t fmix32(uint32_t x)
{
    x ^= x >> 16;
    x *= 0x85ebca6bu;
    x ^= x >> 13;
    x *= 0xc2b2ae35u;
    x ^= x >> 16;
    return x;
}

// Inverse of fmix32: undo each xorshift and multiply by the modular inverse.
__host__ __device__ __forceinline__ uint32_t fmix32_inv(uint32_t x)
{
    x ^= x >> 16;
    x *= 0x7ed1b41du;  // inverse of 0xc2b2ae35 mod 2^32
    x ^= (x >> 13) ^ (x >> 26);
    x *= 0xa5cb9243u;  // inverse of 0x85ebca6b mod 2^32
    x ^= x >> 16;
    return x;
}

// 64-bit mixer for pin-set fingerprints (SplitMix64 output function).
__device__ __forceinline__ uint64_t mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Priority of a hyperedge under a Table 1 policy (smaller = preferred),
// packed above the hash of its local id: the lexicographic (priority, hash)
// order of Algorithm 1 as one 64-bit key.
__device__ __forceinline__ uint64_t hedge_key(int policy, uint32_t local_id, int32_t degree,
                                              int32_t weight)
{
    uint32_t h = fmix32(local_id + 1u);
    uint32_t p;
    switch (policy) {
    case BP_HDH: p = 0xFFFFFFFFu - (uint32_t)degree; break;
    case BP_LWD: p = (uint32_t)weight; break;
    case BP_HWD: p = 0xFFFFFFFFu - (uint32_t)weight; break;
    case BP_RAND: p = h; break;
    default: p = (uint32_t)degree; break;
    }
    return ((uint64_t)p << 32) | h;
}

// Order key of (gain descending, node id ascending) as an ascending uint64.
__device__ __forceinline__ uint64_t gain_order_key(int32_t gain, uint32_t id)
{
    uint32_t g = (uint32_t)(-gain) ^ 0x80000000u;
    return ((uint64_t)g << 32) | id;
}

// ---- wave64 / workgroup collectives -------------------------------------------

template <typename T> __device__ __forceinline__ T wave_sum(T v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
template <typename T> __device__ __forceinline__ T wave_min(T v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        T u = __shfl_xor(v, o, 64);
        v = u < v ? u : v;
    }
    return v;
}
template <typename T> __device__ __forceinline__ T wave_max(T v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        T u = __shfl_xor(v, o, 64);
        v = u > v ? u : v;
    }
    return v;
}
// inclusive prefix sum across the wave
template <typename T> __device__ __forceinline__ T wave_incl_scan(T v)
{
    int lane = threadIdx.x & 63;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        T u = __shfl_up(v, o, 64);
        if (lane >= o) v += u;
    }
    return v;
}

// Workgroup sum; every thread gets the total.  All threads must call.
template <typename T> __device__ __forceinline__ T block_sum(T v, T *lds /* >= 16 */)
{
    v = wave_sum(v);
    int w = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) lds[w] = v;
    __syncthreads();
    T t = 0;
    for (int i = 0; i < nw; i++) t += lds[i];
    __syncthreads();
    return t;
}
template <typename T> __device__ __forceinline__ T block_min(T v, T *lds)
{
    v = wave_min(v);
    int w = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) lds[w] = v;
    __syncthreads();
    T t = lds[0];
    for (int i = 1; i < nw; i++) t = lds[i] < t ? lds[i] : t;
    __syncthreads();
    return t;
}
// Exclusive prefix over the workgroup; *total gets the sum.  All threads call.
template <typename T>
__device__ __forceinline__ T block_excl_scan(T v, T *lds /* >= 16 */, T *total)
{
    T inc = wave_incl_scan(v);
    int w = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 63 || threadIdx.x == blockDim.x - 1) lds[w] = inc;
    __syncthreads();
    T before = 0, t = 0;
    for (int i = 0; i < nw; i++) {
        if (i < w) before += lds[i];
        t += lds[i];
    }
    __syncthreads();
    *total = t;
    return before + inc - v;
}

// Slot of each taking lane in a list with counter *ctr (LDS or global): one
// atomic per wavefront; -1 for lanes not taking.  Lanes that do not call take
// nothing.
__device__ __forceinline__ int32_t lds_wave_slot(bool take, int32_t *ctr)
{
    unsigned long long m = __ballot(take);
    if (!m) return -1;
    int lane = threadIdx.x & 63, leader = __ffsll((long long)m) - 1;
    int32_t base = 0;
    if (lane == leader) base = atomicAdd(ctr, __popcll(m));
    base = __builtin_amdgcn_readlane(base, leader);
    return take ? base + __popcll(m & ((1ull << lane) - 1ull)) : -1;
}

// Histogram count of bin dig for every lane with act set: lanes sharing the
// bin of the first such lane (twice over) add with one atomic, the rest
// alone.  Selection keys crowd into few bins, where per-lane atomics on one
// LDS address serialize.  Lanes that do not call add nothing.
__device__ __forceinline__ void lds_hist_add(bool act, uint32_t dig, uint32_t *hist)
{
    int lane = threadIdx.x & 63;
    unsigned long long am = __ballot(act);
#pragma unroll
    for (int k = 0; k < 2; k++) {
        if (!am) return;
        int leader = __ffsll((long long)am) - 1;
        uint32_t ld = (uint32_t)__builtin_amdgcn_readlane((int)dig, leader);
        unsigned long long eq = __ballot(act && dig == ld);
        if (lane == leader) atomicAdd(&hist[ld], (uint32_t)__popcll(eq));
        act = act && dig != ld;
        am &= ~eq;
    }
    if (act) atomicAdd(&hist[dig], 1u);
}

// Appends id to list for every active lane with take set, using one atomic
// per wavefront.  Call from all active lanes (the ballot spans them).
__device__ __forceinline__ void wave_append(bool take, int32_t id, int32_t *list, int32_t *counter)
{
    unsigned long long m = __ballot(take);
    if (!m) return;
    int lane = threadIdx.x & 63;
    int leader = __ffsll((long long)m) - 1;
    int base = 0;
    if (lane == leader) base = atomicAdd(counter, __popcll(m));
    base = __shfl(base, leader, 64);
    if (take) list[base + __popcll(m & ((1ull << lane) - 1))] = id;
}

// wave_append into a workgroup-local list (LDS counter).
__device__ __forceinline__ void lds_append(bool take, int32_t id, int32_t *list, int32_t *counter)
{
    unsigned long long m = __ballot(take);
    if (!m) return;
    int lane = threadIdx.x & 63;
    int leader = __ffsll((long long)m) - 1;
    int base = 0;
    if (lane == leader) base = atomicAdd(counter, __popcll(m));
    base = __shfl(base, leader, 64);
    if (take) list[base + __popcll(m & ((1ull << lane) - 1))] = id;
}

// Smallest m with m*m >= n.
__host__ __device__ __forceinline__ int64_t ceil_sqrt_i64(int64_t n)
{
    if (n <= 0) return 0;
    int64_t m = (int64_t)sqrt((double)n);
    while (m * m < n) m++;
    while (m > 0 && (m - 1) * (m - 1) >= n) m--;
    return m;
}

}  // namespace bp

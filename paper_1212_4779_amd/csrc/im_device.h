// im_device.h -- device-side building blocks shared by the kernels of libim:
// the counter-based edge generator, wavefront/block scans and the
// level-synchronous word-parallel reachability engines.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define IM_WAVE 64
#define IM_EMPTY 0xFFFFFFFFu

// ---------------------------------------------------------------------------
// SplitMix64 (Steele, Lea & Flood, OOPSLA 2014), written from its published
// definition: output i (i >= 1) of a generator with state s is
// mix(s + i * 0x9e3779b97f4a7c15), mix = xorshift-30, multiply, xorshift-27,
// multiply, xorshift-31.
// ---------------------------------------------------------------------------
#define IM_GOLDEN 0x9e3779b97f4a7c15ull

__device__ __forceinline__ uint64_t sm64_finalise(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

// bits r0..r0+cnt-1 of the snapshots of word w that are set for a node
__device__ __forceinline__ uint64_t im_valid_bits(uint32_t R, uint32_t w)
{
    uint32_t lo = w * 64u;
    if (lo >= R) return 0ull;
    uint32_t cnt = R - lo;
    return cnt >= 64u ? ~0ull : ((1ull << cnt) - 1ull);
}

// Several independent instances laid side by side as one block-diagonal
// graph: instance i owns nodes [node_off[i], node_off[i+1]) and arcs
// [arc_off[i], arc_off[i+1]). count = 1 with null arrays is one graph whose
// parameters are passed as scalars.
struct Batch {
    uint32_t count;
    const uint32_t *node_inst;  // [N] instance of each node
    const uint32_t *R;          // [count] snapshots
    const uint32_t *k;          // [count] seeds wanted
    const uint32_t *kpre;       // [count] offset of the instance's outputs
    const uint32_t *node_off;   // [count+1]
    const uint64_t *arc_off;    // [count+1]
    const uint64_t *seed;       // [count]
};

// largest i with off[i] <= x (off[0] = 0 <= x < off[count])
template <typename T>
__device__ __forceinline__ uint32_t find_instance(const T *off, uint32_t count, T x)
{
    uint32_t lo = 0, hi = count;
    while (hi - lo > 1) {
        uint32_t mid = lo + (hi - lo) / 2;
        if (off[mid] <= x) lo = mid; else hi = mid;
    }
    return lo;
}

// ---------------------------------------------------------------------------
// Scans
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v)
{
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        uint32_t y = __shfl_up(v, d, 64);
        if (lane >= d) v += y;
    }
    return v;
}

__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t v)
{
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
    return v;
}

__device__ __forceinline__ unsigned long long wave_max_u64(unsigned long long v)
{
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
        unsigned long long o = __shfl_xor(v, d, 64);
        v = o > v ? o : v;
    }
    return v;
}

// Exclusive scan over a block of NT threads. s_w must hold NT/64 + 1 words.
// Returns the exclusive prefix; *total gets the block sum. Ends with a
// barrier, so s_w may be reused right after.
template <int NT>
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t *s_w, uint32_t *total)
{
    constexpr int NW = NT / 64;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    uint32_t incl = wave_incl_scan(v);
    if (lane == 63) s_w[wid] = incl;
    __syncthreads();
    if (wid == 0) {
        uint32_t x = lane < NW ? s_w[lane] : 0u;
        uint32_t xi = wave_incl_scan(x);
        if (lane < NW) s_w[lane] = xi - x;
        if (lane == NW - 1) s_w[NW] = xi;
    }
    __syncthreads();
    uint32_t r = incl - v + s_w[wid];
    *total = s_w[NW];
    __syncthreads();
    return r;
}

// largest k in [0, N) with a[k] <= j (a non-decreasing, a[0] <= j)
template <int N>
__device__ __forceinline__ int upper_index(const uint32_t *a, uint32_t j)
{
    int lo = 0;
#pragma unroll
    for (int step = N / 2; step >= 1; step >>= 1)
        if (a[lo + step] <= j) lo += step;
    return lo;
}

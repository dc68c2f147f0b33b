// Shared device helpers for the gfx950 kernels (wave64, LDS, int64 accumulation).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

typedef int64_t i64;
typedef int32_t i32;
typedef uint32_t u32;
typedef uint64_t u64;

#define WAVE 64

__device__ __forceinline__ int lane_id() { return (int)__lane_id(); }

__device__ __forceinline__ u64 lanemask_lt() {
    int l = lane_id();
    return l == 0 ? 0ull : (~0ull >> (64 - l));
}

// Wave-wide inclusive sum (int32), all 64 lanes participate.
__device__ __forceinline__ int wave_incl_sum(int v) {
#pragma unroll
    for (int o = 1; o < WAVE; o <<= 1) {
        int t = __shfl_up(v, o, WAVE);
        if (lane_id() >= o) v += t;
    }
    return v;
}

__device__ __forceinline__ i64 wave_sum64(i64 v) {
#pragma unroll
    for (int o = WAVE / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, WAVE);
    return v;
}

__device__ __forceinline__ int wave_sum32(int v) {
#pragma unroll
    for (int o = WAVE / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, WAVE);
    return v;
}

__device__ __forceinline__ int wave_max32(int v) {
#pragma unroll
    for (int o = WAVE / 2; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, WAVE));
    return v;
}

__device__ __forceinline__ void atomic_add_i64(i64 *p, i64 v) {
    atomicAdd(reinterpret_cast<unsigned long long *>(p), static_cast<unsigned long long>(v));
}

// Multiplicative hash into a power-of-two table.
__device__ __forceinline__ u32 hslot(u32 key, u32 mask) { return (key * 0x9E3779B1u >> 7) & mask; }

// Largest i in [lo, hi) with off[i] <= e, for a non-decreasing array off (lo valid).
template <typename T>
__device__ __forceinline__ int upper_index(const T *off, int lo, int hi, T e) {
    while (hi - lo > 1) {
        int mid = (lo + hi) >> 1;
        if (off[mid] <= e) lo = mid; else hi = mid;
    }
    return lo;
}

// First position p in the sorted range a[lo, hi) with a[p] >= key.
__device__ __forceinline__ i32 lower_bound_i32(const i32 *a, i32 lo, i32 hi, i32 key) {
    while (lo < hi) {
        i32 mid = lo + ((hi - lo) >> 1);
        if (a[mid] < key) lo = mid + 1; else hi = mid;
    }
    return lo;
}

#define HIP_CHECK_LAUNCH() (hipGetLastError())

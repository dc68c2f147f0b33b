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

// Wave-wide inclusive sum (int32), all 64 lanes active.  DPP row shifts build
// the prefix inside each 16-lane row; row broadcasts of lanes 15 and 31 carry it
// across rows (no LDS traffic).
__device__ __forceinline__ int wave_incl_sum(int v) {
    v += __builtin_amdgcn_update_dpp(0, v, 0x111, 0xf, 0xf, false);  // row_shr:1
    v += __builtin_amdgcn_update_dpp(0, v, 0x112, 0xf, 0xf, false);  // row_shr:2
    v += __builtin_amdgcn_update_dpp(0, v, 0x114, 0xf, 0xf, false);  // row_shr:4
    v += __builtin_amdgcn_update_dpp(0, v, 0x118, 0xf, 0xf, false);  // row_shr:8
    v += __builtin_amdgcn_update_dpp(0, v, 0x142, 0xa, 0xf, false);  // row_bcast:15 into rows 1, 3
    v += __builtin_amdgcn_update_dpp(0, v, 0x143, 0xc, 0xf, false);  // row_bcast:31 into rows 2, 3
    return v;
}

// Inclusive sum within each 16-lane row of the wave (DPP row shifts only).
__device__ __forceinline__ int row_incl_sum(int v) {
    v += __builtin_amdgcn_update_dpp(0, v, 0x111, 0xf, 0xf, false);  // row_shr:1
    v += __builtin_amdgcn_update_dpp(0, v, 0x112, 0xf, 0xf, false);  // row_shr:2
    v += __builtin_amdgcn_update_dpp(0, v, 0x114, 0xf, 0xf, false);  // row_shr:4
    v += __builtin_amdgcn_update_dpp(0, v, 0x118, 0xf, 0xf, false);  // row_shr:8
    return v;
}

// Adds, for every run of consecutive lanes holding the same index si, the run's
// total of val to dst[si] with one atomic (issued by the run's last lane).  All 64
// lanes active; lanes with nothing to add pass val = 0.  Values of 2^24 or more are
// added on their own, so that the 32-bit run sums cannot overflow.  dst is int64 or
// int32 (then the caller keeps every sum within int32).
template <typename T>
__device__ __forceinline__ void wave_run_add(T *dst, int si, int val) {
    const int lane = lane_id();
    if (val >= (1 << 24)) {
        if constexpr (sizeof(T) == 8) atomicAdd((unsigned long long *)&dst[si], (unsigned long long)(i64)val);
        else atomicAdd(&dst[si], (T)val);
        val = 0;
    }
    if (__ballot(val != 0) == 0) return;  // nothing to add anywhere in the wave
    const int incl = wave_incl_sum(val);
    const int prev = __shfl_up(si, 1, WAVE);
    const u64 starts = __ballot(lane == 0 || prev != si);
    const bool last = lane == WAVE - 1 || ((starts >> (lane + 1)) & 1ull);
    const u64 upto = lane == WAVE - 1 ? starts : (starts & ((2ull << lane) - 1ull));
    const int head = 63 - __clzll((long long)upto);
    const int before = __shfl(incl, head > 0 ? head - 1 : 0, WAVE);
    const int tot = incl - (head > 0 ? before : 0);
    if (last && tot) {
        if constexpr (sizeof(T) == 8) atomicAdd((unsigned long long *)&dst[si], (unsigned long long)(i64)tot);
        else atomicAdd(&dst[si], (T)tot);
    }
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

// Multiplicative hash into a power-of-two table (at most 2^15 entries), which
// scatters runs of consecutive keys (linear probing would turn them into long
// occupied runs).  The slot comes from bits 16..30 of a 24-bit product: the
// compiler then keeps the full-rate 24-bit multiply (it narrows a product whose low
// bits alone are used to a quarter-rate 32-bit one).
__device__ __forceinline__ u32 hslot(u32 key, u32 mask) {
    return (__umul24(key ^ (key >> 15), 0x9E3779u) >> 16) & mask;
}

// A value every lane of the wave holds alike, moved to a scalar register so that
// branches on it are scalar.
__device__ __forceinline__ i32 wave_uniform(i32 v) { return __builtin_amdgcn_readfirstlane(v); }

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

__device__ __forceinline__ void wave_fence() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// Segment index of element e0 + lane, for the 64 consecutive elements of one wave.
// Segments are given by a non-decreasing prefix off[0..nseg] (off[0] = 0, off[nseg] =
// total, e0 < total).  One binary search per wave finds the segment of e0; the later
// segment starts inside the 64-element window are marked in LDS and spread to the
// lanes by a prefix maximum.  All 64 lanes must call it with the same e0.  `mark`
// is this wave's 64-int LDS array, all -1 on entry and again on return.
__device__ __forceinline__ int locate64(const i32 *off, int nseg, i32 e0, i32 *mark) {
    const int lane = lane_id();
    const int lo = upper_index<i32>(off, 0, nseg, e0);
    for (int k0 = lo + 1; k0 < nseg; k0 += WAVE) {
        int j = k0 + lane;
        i32 st = j < nseg ? off[j] : 0x7fffffff;
        bool in = st < e0 + WAVE;
        if (in) atomicMax(&mark[st - e0], j);  // empty segments share a start: the last one wins
        if (!(__ballot(in) >> 63)) break;
    }
    wave_fence();
    int v = mark[lane];
    wave_fence();
    mark[lane] = -1;
    if (lane == 0) v = lo;
#pragma unroll
    for (int o = 1; o < WAVE; o <<= 1) {
        int t = __shfl_up(v, o, WAVE);
        if (lane >= o) v = max(v, t);
    }
    return v;
}

// Inclusive sum over runs of equal `key` in consecutive lanes; *last is set on the
// last lane of each run, which then holds the run total.
__device__ __forceinline__ i64 wave_run_sum(i64 v, int key, bool *last) {
    const int lane = lane_id();
#pragma unroll
    for (int o = 1; o < WAVE; o <<= 1) {
        i64 t = __shfl_up(v, o, WAVE);
        int k = __shfl_up(key, o, WAVE);
        if (lane >= o && k == key) v += t;
    }
    int nk = __shfl_down(key, 1, WAVE);
    *last = (lane == WAVE - 1) || nk != key;
    return v;
}

// Per-vertex passes: vertices of degree <= SG_MAXDEG (the ranks below a cut, since
// degrees ascend with rank) are handled by SG-lane groups, several per wave; the
// rest one per wave.
#define SG 16
#define SG_MAXDEG 64

// Smallest rank whose degree exceeds d (n if none): a binary search over the
// non-decreasing degrees by rank.
__device__ __forceinline__ i32 first_above(const u32 *__restrict__ ndeg, i32 n, u32 d) {
    i32 lo = 0, hi = n;
    while (lo < hi) {
        const i32 mid = lo + ((hi - lo) >> 1);
        if (ndeg[mid] <= d) lo = mid + 1; else hi = mid;
    }
    return lo;
}

template <int W>
__device__ __forceinline__ i64 group_sum64(i64 v) {
#pragma unroll
    for (int o = W / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, W);
    return v;
}

template <int W>
__device__ __forceinline__ int group_max32(int v) {
#pragma unroll
    for (int o = W / 2; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, W));
    return v;
}

#define HIP_CHECK_LAUNCH() (hipGetLastError())

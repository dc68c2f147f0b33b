// Host execution of the 4-cycle sweep kernels for tests: every lane of a workgroup
// is a host thread, and every cross-lane operation (shuffle, ballot, wave sum,
// wave barrier, workgroup barrier) is a rendezvous of the lanes involved.  Lanes
// run in no fixed order between rendezvous, which is stricter than a wave's
// lockstep: a read of LDS another lane writes without a barrier in between shows up
// as a wrong segment or count.  Every rendezvous also checks that all lanes of the
// wave arrive from the same collective (a collective some lanes skip aborts).
// LDS buffers and graph arrays are exact-size heap blocks, so a build with
// AddressSanitizer reports any access outside them.
#pragma once
#include <atomic>
#include <barrier>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <thread>
#include <vector>
#include <algorithm>
typedef int64_t i64;
typedef int32_t i32;
typedef uint32_t u32;
typedef uint64_t u64;
#define WAVE 64
#define __device__
#define __host__
#define __global__
#define __forceinline__ inline
#define __launch_bounds__(x)
#define amdgpu_waves_per_eu(x) unused
#define __align__(x) alignas(x)
struct dim3e { u32 x; };
inline thread_local dim3e threadIdx, blockIdx, gridDim, blockDim;
struct EmuSeqStore { u64 v[2][WAVE]; };
struct EmuBlock {
    int nt;
    std::barrier<> *bar;
    std::vector<std::barrier<> *> wbar;
    std::vector<i64> xch;  // [waves][64]
    std::mutex mu;
    std::map<int, void *> shared;
    char *dyn = nullptr;
    std::vector<EmuSeqStore> seqs;
};
inline thread_local EmuBlock *emu_blk = nullptr;
inline int lane_id() { return (int)(threadIdx.x % WAVE); }
inline int emu_wave() { return (int)(threadIdx.x / WAVE); }
inline thread_local u64 emu_seq = 0;
// every lane counts its wave rendezvous; all lanes of a wave must agree on the count
inline void emu_wsync() {
    EmuSeqStore &q = emu_blk->seqs[emu_wave()];
    const u64 my = ++emu_seq;
    q.v[my & 1][lane_id()] = my;
    emu_blk->wbar[emu_wave()]->arrive_and_wait();
    for (int i = 0; i < WAVE; i++)
        if (q.v[my & 1][i] != my) {
            fprintf(stderr, "DIVERGED wave %d: lane %d at rendezvous %llu, lane %d at %llu\n", emu_wave(), lane_id(),
                    (unsigned long long)my, i, (unsigned long long)q.v[my & 1][i]);
            abort();
        }
}
inline void __syncthreads() { emu_blk->bar->arrive_and_wait(); }
inline i64 *emu_x() { return &emu_blk->xch[(size_t)emu_wave() * WAVE]; }
template <typename T> inline T emu_get(T v, int src) {
    i64 *x = emu_x();
    x[lane_id()] = (i64)v;
    emu_wsync();
    T r = (T)x[src];
    emu_wsync();
    return r;
}
inline int __shfl(int v, int src, int w = WAVE) { return emu_get<int>(v, src & 63); }
inline int __shfl_up(int v, unsigned d, int w = WAVE) { int l = lane_id(); return emu_get<int>(v, l >= (int)d ? l - (int)d : l); }
inline int __shfl_down(int v, unsigned d, int w = WAVE) { int l = lane_id(); return emu_get<int>(v, l + (int)d < WAVE ? l + (int)d : l); }
inline u64 __ballot(bool p) {
    i64 *x = emu_x();
    x[lane_id()] = p ? 1 : 0;
    emu_wsync();
    u64 m = 0;
    for (int i = 0; i < WAVE; i++) if (x[i]) m |= 1ull << i;
    emu_wsync();
    return m;
}
inline int wave_incl_sum(int v) {
    i64 *x = emu_x();
    x[lane_id()] = v;
    emu_wsync();
    int s = 0;
    for (int i = 0; i <= lane_id(); i++) s += (int)x[i];
    emu_wsync();
    return s;
}
inline i64 wave_sum64(i64 v) {
    i64 *x = emu_x();
    x[lane_id()] = v;
    emu_wsync();
    i64 s = 0;
    for (int i = 0; i < WAVE; i++) s += x[i];
    emu_wsync();
    return s;
}
inline i32 wave_uniform(i32 v) { return emu_get<i32>(v, 0); }
inline int __popcll(u64 x) { return __builtin_popcountll(x); }
inline int __popc(u32 x) { return __builtin_popcount(x); }
inline int __clzll(long long x) { return x ? __builtin_clzll((u64)x) : 64; }
inline int __clz(int x) { return x ? __builtin_clz((u32)x) : 32; }
inline int __ffs(int x) { return __builtin_ffs(x); }
inline u32 __umul24(u32 a, u32 b) { return (u32)(((u64)(a & 0xffffff) * (u64)(b & 0xffffff)) & 0xffffffffu); }
inline u32 atomicAdd(u32 *p, u32 v) { return __atomic_fetch_add(p, v, __ATOMIC_SEQ_CST); }
inline i32 atomicAdd(i32 *p, i32 v) { return __atomic_fetch_add(p, v, __ATOMIC_SEQ_CST); }
inline unsigned long long atomicAdd(unsigned long long *p, unsigned long long v) { return __atomic_fetch_add(p, v, __ATOMIC_SEQ_CST); }
inline u32 atomicAnd(u32 *p, u32 v) { return __atomic_fetch_and(p, v, __ATOMIC_SEQ_CST); }
inline u32 atomicCAS(u32 *p, u32 c, u32 v) { __atomic_compare_exchange_n(p, &c, v, false, __ATOMIC_SEQ_CST, __ATOMIC_SEQ_CST); return c; }
inline i32 atomicCAS(i32 *p, i32 c, i32 v) { __atomic_compare_exchange_n(p, &c, v, false, __ATOMIC_SEQ_CST, __ATOMIC_SEQ_CST); return c; }
template <typename T> inline T *emu_shared(int id, size_t count) {
    std::lock_guard<std::mutex> g(emu_blk->mu);
    auto it = emu_blk->shared.find(id);
    if (it != emu_blk->shared.end()) return (T *)it->second;
    T *p = (T *)calloc(count, sizeof(T));
    emu_blk->shared[id] = p;
    return p;
}
inline int min(int a, int b) { return a < b ? a : b; }
inline int max(int a, int b) { return a > b ? a : b; }
inline i64 min(i64 a, i64 b) { return a < b ? a : b; }
inline i64 max(i64 a, i64 b) { return a > b ? a : b; }
inline int wave_incl_max(int v) {
    i64 *x = emu_x();
    x[lane_id()] = v;
    emu_wsync();
    int m = 0;
    for (int i = 0; i <= lane_id(); i++) m = std::max(m, (int)x[i]);
    emu_wsync();
    return m;
}

// Preprocessing kernels: degrees, degree-rank relabelling, oriented layout.
//
// The orientation follows the degree order r(v) = (deg v, v): vertices are
// renumbered by rank (stable LSD radix sort of the degrees, ties by id), so that
// "u ranks above v" is simply u > v.  Every relabelled row is stored as
//     [ N-(y) : neighbours with smaller rank, in input order | N+(y) sorted ascending ]
// and split[y] marks the boundary.  N+ lists are short (at most about sqrt(2m)),
// which is what the Stage I / Stage II / 4-cycle kernels intersect and probe.
#include "common.hpp"
#include "kernels.hpp"

// ---------------------------------------------------------------------------
// Degrees and the first statistics.
// ---------------------------------------------------------------------------
// A row whose bounds leave [0, nnz], run backwards or hold more than dcap entries
// (a bound on the degree the caller knows, which sizes the per-row buffers) gets
// degree 0 and raises bad_input, so no later kernel reads or writes outside its
// buffers.
// Grid-stride over the vertices; the maximum degree meets in LDS first, so that
// the shared statistic takes one atomic per workgroup (one per wave serialised
// tens of thousands of same-address atomics).
__global__ void k_degree(i32 n, i64 nnz, i64 dcap, const i64 *__restrict__ rp, u32 *__restrict__ deg,
                         u32 *__restrict__ vals, GraphStats *__restrict__ st) {
    __shared__ int s_max;
    if (threadIdx.x == 0) s_max = 0;
    __syncthreads();
    int dm = 0;
    for (i32 v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) {
        i64 b = rp[v], e = rp[v + 1];
        bool ok = b >= 0 && e >= b && e <= nnz && e - b <= dcap && (v > 0 || b == 0) && (v < n - 1 || e == nnz);
        if (!ok) atomicOr(&st->bad_input, 1);
        const int d = ok ? (int)(e - b) : 0;
        deg[v] = (u32)d;
        vals[v] = (u32)v;
        dm = max(dm, d);
    }
    dm = wave_max32(dm);
    if (lane_id() == 0 && dm > 0) atomicMax(&s_max, dm);
    __syncthreads();
    if (threadIdx.x == 0 && s_max > 0) atomicMax(&st->dmax, s_max);
}

// ---------------------------------------------------------------------------
// Device-wide exclusive scan (u32 or i64 elements), three kernels.
// ---------------------------------------------------------------------------
#define SCAN_NT 256
#define SCAN_PER 8
#define SCAN_TILE (SCAN_NT * SCAN_PER)

template <typename T>
__device__ T block_excl_scan(T v, T *total) {
    __shared__ T wsum[SCAN_NT / WAVE];
    T x = v;
#pragma unroll
    for (int o = 1; o < WAVE; o <<= 1) {
        T t = __shfl_up(x, o, WAVE);
        if (lane_id() >= o) x += t;
    }
    int w = threadIdx.x / WAVE;
    if (lane_id() == WAVE - 1) wsum[w] = x;
    __syncthreads();
    T before = 0, all = 0;
    for (int i = 0; i < SCAN_NT / WAVE; i++) {
        if (i < w) before += wsum[i];
        all += wsum[i];
    }
    __syncthreads();
    *total = all;
    return before + x - v;
}

template <typename Tin, typename Tout>
__global__ void k_scan_reduce(const Tin *__restrict__ in, i64 len, Tout *__restrict__ bsum) {
    i64 base = (i64)blockIdx.x * SCAN_TILE;
    Tout s = 0;
    for (int k = 0; k < SCAN_PER; k++) {
        i64 i = base + (i64)k * SCAN_NT + threadIdx.x;
        if (i < len) s += (Tout)in[i];
    }
    Tout tot;
    block_excl_scan<Tout>(s, &tot);
    if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

template <typename Tout>
__global__ void k_scan_top(Tout *__restrict__ bsum, i64 nb, Tout *__restrict__ grand) {
    Tout carry = 0;
    for (i64 base = 0; base < nb; base += SCAN_NT) {
        i64 i = base + threadIdx.x;
        Tout v = i < nb ? bsum[i] : 0;
        Tout tot;
        Tout ex = block_excl_scan<Tout>(v, &tot);
        if (i < nb) bsum[i] = carry + ex;
        carry += tot;
        __syncthreads();
    }
    if (threadIdx.x == 0 && grand) *grand = carry;
}

// out[i] = sum of in[0..i) ; out may alias a longer array (out[len] written if write_total).
template <typename Tin, typename Tout>
__global__ void k_scan_down(const Tin *__restrict__ in, i64 len, const Tout *__restrict__ bsum,
                            Tout *__restrict__ out, int write_total) {
    __shared__ Tout tile[SCAN_TILE];
    i64 base = (i64)blockIdx.x * SCAN_TILE;
    for (int k = 0; k < SCAN_PER; k++) {
        i64 i = base + (i64)k * SCAN_NT + threadIdx.x;
        tile[k * SCAN_NT + threadIdx.x] = i < len ? (Tout)in[i] : 0;
    }
    __syncthreads();
    Tout s = 0;
    for (int k = 0; k < SCAN_PER; k++) s += tile[threadIdx.x * SCAN_PER + k];
    Tout tot;
    Tout ex = block_excl_scan<Tout>(s, &tot) + bsum[blockIdx.x];
    for (int k = 0; k < SCAN_PER; k++) {
        Tout v = tile[threadIdx.x * SCAN_PER + k];
        tile[threadIdx.x * SCAN_PER + k] = ex;
        ex += v;
    }
    __syncthreads();
    for (int k = 0; k < SCAN_PER; k++) {
        i64 i = base + (i64)k * SCAN_NT + threadIdx.x;
        if (i < len) out[i] = tile[k * SCAN_NT + threadIdx.x];
    }
    if (write_total && blockIdx.x == gridDim.x - 1 && threadIdx.x == SCAN_NT - 1) {
        // last element of the array gets the grand total
        i64 last = len;
        Tout t = 0;
        (void)t;
        out[last] = ex;  // ex after the loop of the last thread = sum through its last element
    }
}

template <typename Tin, typename Tout>
static hipError_t excl_scan(const Tin *in, i64 len, Tout *out, Tout *bsum_ws, int write_total,
                            hipStream_t s) {
    if (len <= 0) {
        if (write_total) return hipMemsetAsync(out, 0, sizeof(Tout), s);
        return hipSuccess;
    }
    i64 nb = (len + SCAN_TILE - 1) / SCAN_TILE;
    hipLaunchKernelGGL((k_scan_reduce<Tin, Tout>), dim3((u32)nb), dim3(SCAN_NT), 0, s, in, len, bsum_ws);
    hipLaunchKernelGGL((k_scan_top<Tout>), dim3(1), dim3(SCAN_NT), 0, s, bsum_ws, nb, (Tout *)nullptr);
    hipLaunchKernelGGL((k_scan_down<Tin, Tout>), dim3((u32)nb), dim3(SCAN_NT), 0, s, in, len, bsum_ws, out,
                       write_total);
    return hipGetLastError();
}

i64 scan_ws_elems(i64 len) { return (len + SCAN_TILE - 1) / SCAN_TILE + 1; }

hipError_t scan_u32_to_i32(const u32 *in, i64 len, i32 *out, i32 *ws, int write_total, hipStream_t s) {
    return excl_scan<u32, i32>(in, len, out, ws, write_total, s);
}
hipError_t scan_i32_to_i32(const i32 *in, i64 len, i32 *out, i32 *ws, int write_total, hipStream_t s) {
    return excl_scan<i32, i32>(in, len, out, ws, write_total, s);
}

// ---------------------------------------------------------------------------
// Stable LSD radix sort of (key, value) u32 pairs, 8-bit digits.
// ---------------------------------------------------------------------------
#define RADIX_NT 256
#define RADIX_ROUNDS 16
#define RADIX_TILE (RADIX_NT * RADIX_ROUNDS)

__global__ void k_radix_hist(const u32 *__restrict__ keys, i64 n, int shift, i32 *__restrict__ hist,
                             i64 num_tiles) {
    __shared__ i32 cnt[256];
    cnt[threadIdx.x] = 0;
    __syncthreads();
    i64 base = (i64)blockIdx.x * RADIX_TILE;
    for (int r = 0; r < RADIX_ROUNDS; r++) {
        i64 i = base + (i64)r * RADIX_NT + threadIdx.x;
        if (i < n) atomicAdd(&cnt[(keys[i] >> shift) & 255u], 1);
    }
    __syncthreads();
    hist[(i64)threadIdx.x * num_tiles + blockIdx.x] = cnt[threadIdx.x];
}

__global__ void k_radix_scatter(const u32 *__restrict__ kin, const u32 *__restrict__ vin,
                                u32 *__restrict__ kout, u32 *__restrict__ vout, i64 n, int shift,
                                const i32 *__restrict__ offs, i64 num_tiles) {
    __shared__ i32 running[256];
    __shared__ i32 wcnt[RADIX_NT / WAVE][256];
    int t = threadIdx.x, w = t / WAVE;
    running[t] = offs[(i64)t * num_tiles + blockIdx.x];
    for (int k = 0; k < RADIX_NT / WAVE; k++) wcnt[k][t] = 0;
    __syncthreads();
    i64 base = (i64)blockIdx.x * RADIX_TILE;
    for (int r = 0; r < RADIX_ROUNDS; r++) {
        i64 i = base + (i64)r * RADIX_NT + t;
        bool valid = i < n;
        u32 key = valid ? kin[i] : 0u;
        u32 val = valid ? vin[i] : 0u;
        u32 d = (key >> shift) & 255u;
        u64 peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; b++) {
            u64 bb = __ballot((d >> b) & 1u);
            peers &= ((d >> b) & 1u) ? bb : ~bb;
        }
        int rank = __popcll(peers & lanemask_lt());
        int leader = peers ? (__ffsll((long long)peers) - 1) : -1;
        if (valid && lane_id() == leader) wcnt[w][d] = __popcll(peers);
        __syncthreads();
        if (valid) {
            i32 pos = running[d] + rank;
            for (int k = 0; k < w; k++) pos += wcnt[k][d];
            kout[pos] = key;
            vout[pos] = val;
        }
        __syncthreads();
        i32 add = 0;
        for (int k = 0; k < RADIX_NT / WAVE; k++) {
            add += wcnt[k][t];
            wcnt[k][t] = 0;
        }
        running[t] += add;
        __syncthreads();
    }
}

i64 radix_ws_elems(i64 n) { return 256 * ((n + RADIX_TILE - 1) / RADIX_TILE) + 1; }

__global__ void k_copy_pairs(const u32 *__restrict__ ks, const u32 *__restrict__ vs, u32 *__restrict__ kd,
                             u32 *__restrict__ vd, i64 n) {
    for (i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (i64)gridDim.x * blockDim.x) {
        kd[i] = ks[i];
        vd[i] = vs[i];
    }
}

// Sorts (k, v) stably by the low `bits` bits of k.  Result in (k, v); (k2, v2) are temporaries.
hipError_t radix_sort_pairs(u32 *k, u32 *v, u32 *k2, u32 *v2, i64 n, int bits, i32 *hist, i32 *scan_ws,
                            hipStream_t s) {
    if (n <= 1) return hipSuccess;
    i64 tiles = (n + RADIX_TILE - 1) / RADIX_TILE;
    u32 *ki = k, *vi = v, *ko = k2, *vo = v2;
    int passes = (bits + 7) / 8;
    for (int p = 0; p < passes; p++) {
        int shift = 8 * p;
        hipLaunchKernelGGL(k_radix_hist, dim3((u32)tiles), dim3(RADIX_NT), 0, s, ki, n, shift, hist, tiles);
        hipError_t e = scan_i32_to_i32(hist, 256 * tiles, hist, scan_ws, 0, s);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_radix_scatter, dim3((u32)tiles), dim3(RADIX_NT), 0, s, ki, vi, ko, vo, n, shift,
                           hist, tiles);
        u32 *tk = ki, *tv = vi;
        ki = ko; vi = vo; ko = tk; vo = tv;
    }
    if (ki != k) {
        i64 blocks = (n + 255) / 256;
        if (blocks > 65536) blocks = 65536;
        hipLaunchKernelGGL(k_copy_pairs, dim3((u32)blocks), dim3(256), 0, s, ki, vi, k, v, n);
    }
    return hipGetLastError();
}

// perm[order[y]] = y
__global__ void k_invert(i32 n, const u32 *__restrict__ order, i32 *__restrict__ perm) {
    i32 y = blockIdx.x * blockDim.x + threadIdx.x;
    if (y < n) perm[order[y]] = y;
}

// ---------------------------------------------------------------------------
// Relabelled rows: [N- in input order | N+ (unsorted yet)], one wave per row; the
// row's bounds go to vmeta as well (its heavy start follows once N+ is sorted).
// ---------------------------------------------------------------------------
// Column ids outside [0, n) raise bad_input and are read as y itself, which keeps
// every index in range; the host stops after this kernel when bad_input is set.
__device__ __forceinline__ i32 relabel_id(const i32 *__restrict__ col, const i32 *__restrict__ perm, i64 s, i32 n,
                                          i32 y, int &bad) {
    i32 a = col[s];
    if (a < 0 || a >= n) {
        bad = 1;
        return y;
    }
    return perm[a];
}

__global__ void k_relabel(i32 n, const i64 *__restrict__ rp, const i32 *__restrict__ col,
                          const u32 *__restrict__ order, const i32 *__restrict__ perm, const u32 *__restrict__ ndeg,
                          const i32 *__restrict__ nrp, i32 *__restrict__ nsplit, i32 *__restrict__ ncol,
                          int4 *__restrict__ vmeta, GraphStats *__restrict__ st) {
    int waves = gridDim.x * (blockDim.x / WAVE);
    int wid = blockIdx.x * (blockDim.x / WAVE) + threadIdx.x / WAVE;
    int dplus_max = 0, bad = 0;
    long long pairs = 0;
    for (i32 y = n - 1 - wid; y >= 0; y -= waves) {
        i32 x = (i32)order[y];
        i64 beg = rp[x];
        i32 len = (i32)ndeg[y];  // 0 for rows that failed the bounds check
        i32 nlow = 0, b_first = 0;  // the first 64 new ids stay in a register for the writes
        for (i32 c = 0; c < len; c += WAVE) {
            i32 j = c + lane_id();
            bool valid = j < len;
            i32 b = valid ? relabel_id(col, perm, beg + j, n, y, bad) : 0;
            if (c == 0) b_first = b;
            nlow += __popcll(__ballot(valid && b < y));
        }
        i32 ybase = nrp[y];
        i32 lowpos = ybase, uppos = ybase + nlow;
        if (lane_id() == 0) {
            nsplit[y] = uppos;
            vmeta[y] = make_int4(ybase, uppos, ybase + len, 0);  // heavy start: once sorted
        }
        dplus_max = max(dplus_max, len - nlow);
        pairs += (long long)(len - nlow) * (len - nlow - 1) / 2;
        for (i32 c = 0; c < len; c += WAVE) {
            i32 j = c + lane_id();
            bool valid = j < len;
            i32 b = c == 0 ? b_first : (valid ? relabel_id(col, perm, beg + j, n, y, bad) : 0);
            bool low = valid && b < y;
            u64 ml = __ballot(low), mu = __ballot(valid && !low);
            if (low) ncol[lowpos + __popcll(ml & lanemask_lt())] = b;
            else if (valid) ncol[uppos + __popcll(mu & lanemask_lt())] = b;
            lowpos += __popcll(ml);
            uppos += __popcll(mu);
        }
    }
    // the workgroup's statistics meet in LDS, then one atomic each
    __shared__ int s_dmax;
    __shared__ unsigned long long s_pairs;
    if (threadIdx.x == 0) {
        s_dmax = 0;
        s_pairs = 0;
    }
    __syncthreads();
    if (lane_id() == 0 && dplus_max > 0) atomicMax(&s_dmax, dplus_max);
    if (lane_id() == 0 && pairs > 0) atomicAdd(&s_pairs, (unsigned long long)pairs);
    __syncthreads();
    if (threadIdx.x == 0 && s_dmax > 0) atomicMax(&st->dplus_max, s_dmax);
    if (threadIdx.x == 0 && s_pairs > 0) atomicAdd((unsigned long long *)&st->pairs, s_pairs);
    if (bad) atomicOr(&st->bad_input, 1);
}

// ---------------------------------------------------------------------------
// Sorting of the N+ parts.  Rows of vertices of degree <= 16 are sorted four per
// wave, one per 16-lane group; other rows of length <= 64 by one wave (bitonic
// network over the lanes); longer rows are queued for the block kernel, which
// sorts in LDS.  hstart[y] (and vmeta[y]'s last field) = first slot of N+(y)
// holding an id >= h0.
// ---------------------------------------------------------------------------
__device__ __forceinline__ i32 bitonic64(i32 v) {
    int l = lane_id();
#pragma unroll
    for (int k = 2; k <= WAVE; k <<= 1) {
#pragma unroll
        for (int j = k >> 1; j > 0; j >>= 1) {
            i32 o = __shfl_xor(v, j, WAVE);
            bool up = (l & k) == 0;
            bool low = (l & j) == 0;
            v = (low == up) ? min(v, o) : max(v, o);
        }
    }
    return v;
}

// The same network within each aligned 16-lane group (xor distances below 16 stay
// inside the group).
__device__ __forceinline__ i32 bitonic16(i32 v) {
    int l = lane_id() & 15;
#pragma unroll
    for (int k = 2; k <= 16; k <<= 1) {
#pragma unroll
        for (int j = k >> 1; j > 0; j >>= 1) {
            i32 o = __shfl_xor(v, j, WAVE);
            bool up = (l & k) == 0;
            bool low = (l & j) == 0;
            v = (low == up) ? min(v, o) : max(v, o);
        }
    }
    return v;
}

__global__ void k_sort_upper_small(i32 n, const u32 *__restrict__ ndeg, const i32 *__restrict__ nrp,
                                   const i32 *__restrict__ nsplit, i32 *__restrict__ ncol,
                                   i32 *__restrict__ hstart, int4 *__restrict__ vmeta, i32 h0,
                                   i32 *__restrict__ longlist, i32 *__restrict__ longcount) {
    int waves = gridDim.x * (blockDim.x / WAVE);
    int wid = blockIdx.x * (blockDim.x / WAVE) + threadIdx.x / WAVE;
    // rows of degree <= 16 (so |N+| <= 16): four per wave, one per 16-lane group
    const i32 cut = first_above(ndeg, n, 16);
    for (i32 yb = wid * 4; yb < cut; yb += waves * 4) {
        const i32 y = yb + lane_id() / 16, l = lane_id() & 15;
        const bool act = y < cut;
        i32 b = 0, e = 0;
        if (act) {
            b = nsplit[y];
            e = nrp[y + 1];
        }
        const i32 len = e - b;
        const bool in = act && l < len;
        i32 v = in ? ncol[b + l] : 0x7fffffff;
        if (__ballot(act && len > 1)) v = bitonic16(v);
        if (in) ncol[b + l] = v;
        const u32 ge = (u32)(__ballot(in && v >= h0) >> (lane_id() & 48)) & 0xffffu;
        if (act && l == 0) {
            const i32 hs = ge ? b + (__ffs((int)ge) - 1) : e;
            hstart[y] = hs;
            reinterpret_cast<i32 *>(vmeta)[4 * (i64)y + 3] = hs;
        }
    }
    for (i32 y = cut + wid; y < n; y += waves) {
        i32 b = nsplit[y], e = nrp[y + 1], len = e - b;
        if (len > WAVE) {
            if (lane_id() == 0) longlist[atomicAdd(longcount, 1)] = y;
            continue;
        }
        i32 l = lane_id();
        i32 v = l < len ? ncol[b + l] : 0x7fffffff;
        if (len > 1) v = bitonic64(v);
        if (l < len) ncol[b + l] = v;
        u64 ge = __ballot(l < len && v >= h0);
        if (l == 0) {
            const i32 hs = ge ? b + (__ffsll((long long)ge) - 1) : e;
            hstart[y] = hs;
            reinterpret_cast<i32 *>(vmeta)[4 * (i64)y + 3] = hs;
        }
    }
}

__global__ void __launch_bounds__(LSORT_NT) k_sort_upper_large(const i32 *__restrict__ nrp,
                                                               const i32 *__restrict__ nsplit,
                                                               i32 *__restrict__ ncol, i32 *__restrict__ hstart,
                                                               int4 *__restrict__ vmeta, i32 h0,
                                                               const i32 *__restrict__ longlist,
                                                               const i32 *__restrict__ longcount) {
    __shared__ i32 a[LSORT_CAP];
    __shared__ i32 first;
    i32 cnt = *longcount;
    for (i32 it = blockIdx.x; it < cnt; it += gridDim.x) {
        i32 y = longlist[it];
        i32 b = nsplit[y], e = nrp[y + 1], len = e - b;
        int P = 1;
        while (P < len) P <<= 1;
        for (int i = threadIdx.x; i < P; i += LSORT_NT) a[i] = i < len ? ncol[b + i] : 0x7fffffff;
        if (threadIdx.x == 0) first = e;
        __syncthreads();
        for (int k = 2; k <= P; k <<= 1) {
            for (int j = k >> 1; j > 0; j >>= 1) {
                for (int i = threadIdx.x; i < P; i += LSORT_NT) {
                    int ixj = i ^ j;
                    if (ixj > i) {
                        i32 x = a[i], z = a[ixj];
                        bool up = (i & k) == 0;
                        if ((x > z) == up) { a[i] = z; a[ixj] = x; }
                    }
                }
                __syncthreads();
            }
        }
        for (int i = threadIdx.x; i < len; i += LSORT_NT) {
            i32 v = a[i];
            ncol[b + i] = v;
            if (v >= h0 && (i == 0 || a[i - 1] < h0)) first = b + i;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            hstart[y] = first;
            reinterpret_cast<i32 *>(vmeta)[4 * (i64)y + 3] = first;
        }
        __syncthreads();
    }
}

// Per-row sums of the mirror pass (over the row's W lanes) and their writes.
template <int W>
__device__ __forceinline__ void mirror_row_tail(i32 y, bool active, int l, i32 b0, i32 sp, i32 e0, i32 h0, i64 wl,
                                                i64 wh, i64 pr, i64 nds, int mx, i64 *__restrict__ wlight,
                                                i64 *__restrict__ wheavy, i64 *__restrict__ probes,
                                                float *__restrict__ feat) {
    wl = group_sum64<W>(wl);
    wh = group_sum64<W>(wh);
    pr = group_sum64<W>(pr);
    nds = group_sum64<W>(nds);
    mx = group_max32<W>(mx);
    if (active && l == 0) {
        wlight[y] = (y < h0) ? wl : 0;
        wheavy[y] = wh;
        probes[y] = pr;
        if (feat) {
            float *f = feat + (i64)y * 6;
            f[0] = log2f(1.0f + (float)(e0 - b0));
            f[1] = log2f(1.0f + (float)(e0 - sp));
            f[2] = log2f(1.0f + (float)(sp - b0));
            f[3] = log2f(1.0f + (float)nds);
            f[4] = log2f(1.0f + (float)pr);
            f[5] = log2f(1.0f + (float)mx);
        }
    }
}

// ---------------------------------------------------------------------------
// Mirror slots and per-vertex work of the 4-cycle passes, one wave per row y (or
// one 16-lane group for rows of degree <= SG_MAXDEG):
//   lower slot s (neighbour b < y): mirror[s] = slot of y inside N+(b);
//   wlight[y] = sum over lower slots of (mirror[s] - row start of b): the wedges
//               with y as the largest vertex;
//   wheavy[y] = sum over all slots of the heavy suffix lengths of N+(b) above
//               max(h0, y+1): the wedges with y opposite a heavy largest vertex;
//   probes[y] = sum of |N+(b)| over b in N+(y): the Stage I probes made from y.
// With feat != nullptr it also writes six cheap per-vertex features for the work
// model: log2(1 + x) of degree, |N+|, |N-|, neighbour-degree sum, probes and the
// largest |N+(b)| over b in N+(y).
// ---------------------------------------------------------------------------
template <int W>
__device__ __forceinline__ void mirror_row(i32 y, bool active, int l, const i32 *__restrict__ nrp,
                                           const i32 *__restrict__ nsplit, const i32 *__restrict__ ncol,
                                           const int4 *__restrict__ vmeta, i32 h0, i32 *__restrict__ mirror,
                                           int2 *__restrict__ hseg, i32 *__restrict__ lbeg, i32 *__restrict__ dslot,
                                           i64 *__restrict__ wlight, i64 *__restrict__ wheavy,
                                           i64 *__restrict__ probes, float *__restrict__ feat) {
    i32 b0 = 0, sp = 0, e0 = 0;
    if (active) {
        b0 = nrp[y];
        sp = nsplit[y];
        e0 = nrp[y + 1];
    }
    i64 wl = 0, wh = 0, pr = 0, nds = 0;
    int mx = 0;
    for (i32 s = b0 + l; s < e0; s += W) {
        i32 b = ncol[s];
        const int4 vb = vmeta[b];  // row start, N+ start, row end, heavy start of b
        i32 bb = vb.x, bend = vb.z;
        nds += bend - bb;
        dslot[s] = bend - bb;
        if (s < sp) {
            i32 m = lower_bound_i32(ncol, vb.y, bend, y);
            mirror[s] = m;
            lbeg[s] = bb;
            wl += m - bb;
            i32 st = (y >= h0) ? min(m + 1, bend) : vb.w;  // (m = bend only for asymmetric input)
            hseg[s] = make_int2(st, bend);
            wh += bend - st;
        } else {
            hseg[s] = make_int2(vb.w, bend);
            wh += bend - vb.w;
            i32 dpb = bend - vb.y;
            pr += dpb;
            mx = max(mx, dpb);
        }
    }
    mirror_row_tail<W>(y, active, l, b0, sp, e0, h0, wl, wh, pr, nds, mx, wlight, wheavy, probes, feat);
}

// Mirror slots (for each N- slot, the N+ slot of the reverse edge), the per-vertex
// work of the later passes (4-cycle wedges light and heavy, Stage I probes) and the
// work-model features.
__global__ void k_mirror(i32 n, const u32 *__restrict__ ndeg, const i32 *__restrict__ nrp,
                         const i32 *__restrict__ nsplit, const i32 *__restrict__ ncol,
                         const int4 *__restrict__ vmeta, i32 h0, i32 *__restrict__ mirror,
                         int2 *__restrict__ hseg, i32 *__restrict__ lbeg, i32 *__restrict__ dslot,
                         i64 *__restrict__ wlight, i64 *__restrict__ wheavy, i64 *__restrict__ probes,
                         float *__restrict__ feat) {
    const int waves = gridDim.x * (blockDim.x / WAVE);
    const int wid = blockIdx.x * (blockDim.x / WAVE) + threadIdx.x / WAVE;
    const i32 cut = first_above(ndeg, n, SG_MAXDEG);
    constexpr int GPW = WAVE / SG;
    for (i32 yb = wid * GPW; yb < cut; yb += waves * GPW) {
        const i32 y = yb + lane_id() / SG;
        mirror_row<SG>(y, y < cut, lane_id() % SG, nrp, nsplit, ncol, vmeta, h0, mirror, hseg, lbeg, dslot, wlight,
                       wheavy, probes, feat);
    }
    for (i32 y = n - 1 - wid; y >= cut; y -= waves)
        mirror_row<WAVE>(y, true, lane_id(), nrp, nsplit, ncol, vmeta, h0, mirror, hseg, lbeg, dslot, wlight, wheavy,
                         probes, feat);
}

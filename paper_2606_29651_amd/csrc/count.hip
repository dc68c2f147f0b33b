// Counting kernels on the relabelled, degree-oriented graph.
//
//   probe (TRI)  Stage I and Stage II: for every vertex u, the triangles with u as
//                lowest vertex are found by probing each N+(v), v in N+(u), against
//                an LDS hash of N+(u); every hit adds 1 to the three edges' t.  The
//                hits also form the graph H_u induced on N+(u), kept as an LDS
//                bitset; the 4-cliques with u lowest are the triangles of H_u
//                (Algorithm 2 counts each 4-clique once from a fixed vertex too).
//   probe (TAU)  after Stage I: tau(x) = sum over triangles at x of t(opposite edge).
//   sums         neighbour sums over the full row of x of t, t^2, t d(a), d(a), d(a)^2.
//   q (LIGHT)    4-cycles whose largest vertex u lies below h0, grouped by u:
//                cnt[w] = #v in N-(u) adjacent to w, w < u.
//   q (HEAVY)    4-cycles whose largest vertex u lies in [h0, n), grouped by the
//                vertex w opposite u: cnt[u] = #v in N(w) with u in N+(v), u > w.
//                Each 4-cycle is counted once, by (largest vertex, its opposite).
//   solve        the nine f-variables from those sums and the non-induced equations
//                (Section 5 and the Appendix), written in input vertex order.
#include "common.hpp"
#include "kernels.hpp"

// An item is worked on by NT threads: a 16-lane group of a wave (NT = 16), a wave
// (NT = 64) or a workgroup (NT a multiple of 64).
template <int NT>
__device__ __forceinline__ void item_sync() {
    if constexpr (NT <= WAVE) {
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
    } else {
        __syncthreads();
    }
}

// Sum over the NT threads of one item; red must hold NT/WAVE entries.
template <int NT>
__device__ __forceinline__ i64 item_sum(i64 v, i64 *red, int tid) {
    if constexpr (NT < WAVE) return group_sum64<NT>(v);
    v = wave_sum64(v);
    if constexpr (NT == WAVE) {
        return v;
    } else {
        if (lane_id() == 0) red[tid / WAVE] = v;
        __syncthreads();
        i64 s = 0;
        for (int k = 0; k < NT / WAVE; k++) s += red[k];
        __syncthreads();
        return s;
    }
}

// In-place inclusive prefix over a[1..len] (a[0] = 0 set here), NT threads.
template <int NT>
__device__ __forceinline__ void item_scan(i32 *a, int len, int tid, i32 *red32) {
    if (tid == 0) a[0] = 0;
    i32 carry = 0;
    for (int c = 0; c < len; c += NT) {
        int i = c + tid;
        i32 v = i < len ? a[i + 1] : 0;
        if constexpr (NT < WAVE) {
            static_assert(NT == 16, "sub-wave items are 16-lane rows");
            const i32 x = row_incl_sum(v);
            if (i < len) a[i + 1] = carry + x;
            carry += __shfl(x, (lane_id() & ~15) + 15, WAVE);
            continue;
        }
        i32 x = wave_incl_sum(v);
        if constexpr (NT == WAVE) {
            if (i < len) a[i + 1] = carry + x;
            carry += __shfl(x, WAVE - 1, WAVE);
        } else {
            int w = tid / WAVE;
            if (lane_id() == WAVE - 1) red32[w] = x;
            __syncthreads();
            i32 before = 0, all = 0;
            for (int k = 0; k < NT / WAVE; k++) {
                if (k < w) before += red32[k];
                all += red32[k];
            }
            if (i < len) a[i + 1] = carry + before + x;
            carry += all;
            __syncthreads();
        }
    }
    item_sync<NT>();
}

// ---------------------------------------------------------------------------
// Classification into work lists (workgroup-aggregated appends).
// ---------------------------------------------------------------------------
// The classes of one vertex: Stage I class (or -1) and the two 4-cycle classes
// (light: largest vertex u = y; heavy: opposite vertex y), with the work and row
// slots each one adds to the class statistics.
struct VertexClasses {
    int c[3];
    i64 work[3], slots[3];
};

__device__ __forceinline__ VertexClasses classify_vertex(const DevGraph &g, const i64 *__restrict__ wlight,
                                                         const i64 *__restrict__ wheavy,
                                                         const i64 *__restrict__ probes, const Thresholds &th,
                                                         i32 y) {
    VertexClasses v{{-1, -1, -1}, {0, 0, 0}, {0, 0, 0}};
    const i32 b = g.nrp[y], sp = g.nsplit[y], e = g.nrp[y + 1];
    const i32 du = e - sp, d = e - b, dm = sp - b;
    const i64 wl = wlight[y], wh = wheavy[y];
    // Stage I/II items: capacity decides first (|N+| sizes the LDS structures); items
    // that fit a wave may move to one lane or to a whole workgroup by predicted work.
    // An item whose neighbours above it have no neighbours above them closes no
    // triangle and is left out.
    if (du >= 2 && probes[y] > 0) {
        int tc;
        if (du > th.tri_block) tc = WC_TRI_LARGE;
        else if (du > th.tri_wave) tc = WC_TRI_BLOCK;
        else {
            tc = WC_TRI_WAVE;
            if (th.bin_mode == 1) {
                if (du <= TRI_THREAD_CAP && d <= th.deg_thread) tc = WC_TRI_THREAD;
                else if (du <= TRI_GROUP_CAP && d <= th.deg_group) tc = WC_TRI_GROUP;
                else if (d >= th.deg_block) tc = WC_TRI_BLOCK;
            } else if (th.bin_mode == 2) {
                float p = th.pred[y];
                if (du <= TRI_THREAD_CAP && p <= th.thr_thread) tc = WC_TRI_THREAD;
                else if (du <= TRI_GROUP_CAP && p <= th.thr_group) tc = WC_TRI_GROUP;
                else if (p >= th.thr_block) tc = WC_TRI_BLOCK;
            }
        }
        v.c[0] = tc;
        v.work[0] = probes[y];
        v.slots[0] = du;
    }
    if (wl > 0) {
        v.c[1] = wl <= th.ql_wave ? WC_QL_WAVE : (wl <= th.ql_block ? WC_QL_BLOCK : WC_QL_GLOBAL);
        v.work[1] = wl;
        v.slots[1] = dm;
    }
    // packed 17-bit and dense 16-bit counters need every count below 2^16; a count
    // is at most d(x), so vertices of degree >= 2^16 use int32 global counters
    if (wh > 0) {
        v.c[2] = d >= 65536 ? WC_QH_GLOBAL
                            : (wh <= th.qh_wave ? WC_QH_WAVE : (wh <= th.qh_block ? WC_QH_BLOCK : WC_QH_DENSE));
        v.work[2] = wh;
        v.slots[2] = d;
    }
    return v;
}

// Work lists per class.  A workgroup classifies CL_PER_THREAD vertices per thread
// per tile (hubs first), counts each class's members, work and slots in LDS, and
// reserves the class's list space with one global atomic per class and tile.
#define CL_NT 256
#define CL_PER_THREAD 4
__global__ void __launch_bounds__(CL_NT) k_classify(DevGraph g, const i64 *__restrict__ wlight,
                                                    const i64 *__restrict__ wheavy, const i64 *__restrict__ probes,
                                                    ListPtrs lists, GraphStats *__restrict__ st, Thresholds th) {
    __shared__ i32 s_cnt[WC_COUNT], s_base[WC_COUNT];
    __shared__ unsigned long long s_work[WC_COUNT], s_slots[WC_COUNT];
    constexpr int TILE = CL_NT * CL_PER_THREAD;
    const i32 tiles = (g.n + TILE - 1) / TILE;
    for (i32 tile = blockIdx.x; tile < tiles; tile += gridDim.x) {
        if (threadIdx.x < WC_COUNT) {
            s_cnt[threadIdx.x] = 0;
            s_work[threadIdx.x] = 0;
            s_slots[threadIdx.x] = 0;
        }
        __syncthreads();
        i32 ys[CL_PER_THREAD];
        int cls[CL_PER_THREAD][3], pos[CL_PER_THREAD][3];
#pragma unroll
        for (int k = 0; k < CL_PER_THREAD; k++) {
            const i32 idx = tile * TILE + k * CL_NT + threadIdx.x;
            const i32 y = g.n - 1 - idx;  // hubs first
            ys[k] = y;
            VertexClasses v{{-1, -1, -1}, {0, 0, 0}, {0, 0, 0}};
            if (y >= 0) v = classify_vertex(g, wlight, wheavy, probes, th, y);
#pragma unroll
            for (int j = 0; j < 3; j++) {
                cls[k][j] = v.c[j];
                pos[k][j] = -1;
                if (v.c[j] >= 0) {
                    pos[k][j] = atomicAdd(&s_cnt[v.c[j]], 1);
                    atomicAdd(&s_work[v.c[j]], (unsigned long long)v.work[j]);
                    atomicAdd(&s_slots[v.c[j]], (unsigned long long)v.slots[j]);
                }
            }
        }
        __syncthreads();
        if (threadIdx.x < WC_COUNT && s_cnt[threadIdx.x] > 0) {
            const int c = threadIdx.x;
            s_base[c] = atomicAdd(&st->cnt[c], s_cnt[c]);
            atomicAdd((unsigned long long *)&st->work[c], s_work[c]);
            atomicAdd((unsigned long long *)&st->slots[c], s_slots[c]);
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < CL_PER_THREAD; k++)
#pragma unroll
            for (int j = 0; j < 3; j++)
                if (cls[k][j] >= 0) lists.l[cls[k][j]][s_base[cls[k][j]] + pos[k][j]] = ys[k];
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Stage I / Stage II / tau probe kernels.
// ---------------------------------------------------------------------------
// Largest i in [0, len) with off[i] <= e, for the QK elements e = min(e0 + j*NT, emax)
// (j < nj) of one thread, searched together (power-of-two steps, independent LDS
// reads in flight).  off is non-decreasing with off[0] = 0 <= e; with emax below
// off[len], segment lo[j] holds e.
template <int NT, int QK>
__device__ __forceinline__ void q_locate(const i32 *off, int len, i32 e0, int nj, int *lo, i32 emax) {
#pragma unroll
    for (int j = 0; j < QK; j++) lo[j] = 0;
    int step = 1;
    while (2 * step < len) step <<= 1;
    for (; step > 0; step >>= 1) {
#pragma unroll
        for (int j = 0; j < QK; j++) {
            if (j < nj) {
                const i32 e = min(e0 + j * NT, emax);
                const int m = lo[j] + step;
                if (m < len && off[m] <= e) lo[j] = m;
            }
        }
    }
}

// Largest i in [0, len) with off[i] <= e (off non-decreasing, off[0] = 0 <= e).
__device__ __forceinline__ int seg_search(const i32 *off, int len, i32 e) {
    int s = 0;
    int step = 1;
    while (2 * step < len) step <<= 1;
    for (; step > 0; step >>= 1) {
        const int m = s + step;
        if (m < len && off[m] <= e) s = m;
    }
    return s;
}

// Segment of every element e in [eb, total), eb + NT*PER at most, of a run of
// segments with prefix offsets off[0..len], one byte each at byte e - eb of map (the
// segments number at most 256): thread t walks its run of PER consecutive elements
// from eb + t*PER on after one search, where a search per element would cost a
// logarithmic number of LDS reads for each.
template <int NT, int PER>
__device__ __forceinline__ void q_segmap(const i32 *off, int len, i32 eb, i32 total, int tid, u32 *map) {
    static_assert(PER % 4 == 0, "whole words per thread");
    const i32 e0 = eb + tid * PER;
    if (e0 >= total) return;
    int s = seg_search(off, len, e0);
    // off[len] = total > e, so the walk stops inside the chunk
    i32 nb = off[s + 1];
#pragma unroll
    for (int k4 = 0; k4 < PER / 4; k4++) {
        u32 w = 0;
#pragma unroll
        for (int b = 0; b < 4; b++) {
            const i32 e = e0 + 4 * k4 + b;
            if (e < total) {
                while (nb <= e) {
                    s++;
                    nb = off[s + 1];
                }
            }
            w |= (u32)s << (8 * b);
        }
        map[tid * (PER / 4) + k4] = w;
    }
}

__device__ __forceinline__ int seg_at(const u32 *map, i32 i) {
    return ((const unsigned char *)map)[i];
}

// The same map with one 16-bit entry per element (the absolute segment index, for
// items of up to 65536 segments): no block ever needs the search instead.
template <int NT, int PER>
__device__ __forceinline__ void q_segmap16(const i32 *off, int len, i32 eb, i32 total, int tid, u32 *map) {
    static_assert(PER % 2 == 0, "whole words per thread");
    const i32 e0 = eb + tid * PER;
    if (e0 >= total) return;
    int s = seg_search(off, len, e0);
    i32 nb = off[s + 1];
#pragma unroll
    for (int k2 = 0; k2 < PER / 2; k2++) {
        u32 w = 0;
#pragma unroll
        for (int b = 0; b < 2; b++) {
            const i32 e = e0 + 2 * k2 + b;
            if (e < total) {
                while (nb <= e) {
                    s++;
                    nb = off[s + 1];
                }
            }
            w |= (u32)s << (16 * b);
        }
        map[tid * (PER / 2) + k2] = w;
    }
}

__device__ __forceinline__ int seg_at16(const u32 *map, i32 i) {
    return ((const unsigned short *)map)[i];
}

// Wave-wide inclusive maximum of non-negative values, all 64 lanes active.
__device__ __forceinline__ int wave_incl_max(int v) {
    v = max(v, __builtin_amdgcn_update_dpp(0, v, 0x111, 0xf, 0xf, false));  // row_shr:1
    v = max(v, __builtin_amdgcn_update_dpp(0, v, 0x112, 0xf, 0xf, false));  // row_shr:2
    v = max(v, __builtin_amdgcn_update_dpp(0, v, 0x114, 0xf, 0xf, false));  // row_shr:4
    v = max(v, __builtin_amdgcn_update_dpp(0, v, 0x118, 0xf, 0xf, false));  // row_shr:8
    v = max(v, __builtin_amdgcn_update_dpp(0, v, 0x142, 0xa, 0xf, false));  // row_bcast:15
    v = max(v, __builtin_amdgcn_update_dpp(0, v, 0x143, 0xc, 0xf, false));  // row_bcast:31
    return v;
}

// The same byte map as q_segmap, built without a search per thread: every
// nonempty segment starting in the block writes its index at its first element, and
// a running maximum over the elements (within each thread's PER bytes, then across
// the item's threads, from the segment of element eb on) fills in the rest.  The
// indices of nonempty segments grow with their starts, so the maximum at e is the
// segment holding e.  NT is a multiple of the wave; red32 holds NT/WAVE entries.
template <int NT, int PER>
__device__ __forceinline__ void seg_map_scan(const i32 *off, int len, i32 eb, i32 total, int tid, u32 *map,
                                             i32 *red32) {
    static_assert(PER % 4 == 0 && NT % WAVE == 0, "whole words per thread, whole waves");
    constexpr int PW = PER / 4;
    u32 *mine = map + tid * PW;
#pragma unroll
    for (int k = 0; k < PW; k++) mine[k] = 0u;
    item_sync<NT>();
    const i32 eend = min(eb + NT * PER, total);
    for (int i = tid; i < len; i += NT) {
        const i32 o = off[i];
        if (o >= eb && o < eend && o < off[i + 1]) ((unsigned char *)map)[o - eb] = (unsigned char)i;
    }
    item_sync<NT>();
    u32 w[PW];
    int r = 0;
#pragma unroll
    for (int k = 0; k < PW; k++) {
        const u32 v = mine[k];
        u32 o = 0;
#pragma unroll
        for (int b = 0; b < 4; b++) {
            r = max(r, (int)((v >> (8 * b)) & 0xffu));
            o |= (u32)r << (8 * b);
        }
        w[k] = o;
    }
    const int incl = wave_incl_max(r);
    int c = __shfl_up(incl, 1, WAVE);
    if (lane_id() == 0) c = 0;
    if constexpr (NT > WAVE) {
        const int wv = tid / WAVE;
        if (lane_id() == WAVE - 1) red32[wv] = incl;
        item_sync<NT>();
        for (int k = 0; k < NT / WAVE; k++)
            if (k < wv) c = max(c, red32[k]);
    }
    if (eb > 0) c = max(c, seg_search(off, len, eb));
#pragma unroll
    for (int k = 0; k < PW; k++) {
        u32 o = 0;
#pragma unroll
        for (int b = 0; b < 4; b++) o |= (u32)max(c, (int)((w[k] >> (8 * b)) & 0xffu)) << (8 * b);
        mine[k] = o;
    }
    item_sync<NT>();
}

// Probe pass modes: Stage I/II (triangles and 4-cliques), tau, and Stage I/II with
// the 4-cliques through every edge credited as well (the `tau` argument of the
// kernels then carries that per-slot int64 array).
enum { PROBE_TRI = 0, PROBE_TAU = 1, PROBE_EK4 = 2 };

#define TAU_RK 4  // triangle records per thread in flight in the tau pass

#define QS 8  // wedges per thread per step in the 4-cycle sweeps

// Row pitch (in words) of the bitset of H_u: odd, so that lanes reading word k of
// consecutive rows hit distinct LDS banks.
__host__ __device__ constexpr int bit_pitch(int cap) { return ((cap + 31) / 32) | 1; }

struct ProbeMem {
    i32 *hkey;   // [hc]
    i32 *hpos;   // [hc]
    i32 *off;    // [cap+1]
    i32 *nb;     // [cap]
    i32 *beg;    // [cap]: first slot of N+(nb[i])
    i32 *tcnt;   // [cap]
    u32 *A;      // [cap*pitch]: row i is the bitset of i's neighbours in H_u
    i64 *acc;    // [cap]
    u32 *A_k4;   // where the 4-clique pass reads the bitset: A itself, or an LDS copy
                 // taken after the probes (over the then unused hash and slot arrays)
    u32 *seg;    // segment byte of each probe of a map block (NT*MP bytes), or null
                 // (nb may be null too: then neighbours are read from the row again)
    i32 *k4s;    // [cap] per-slot sums of the 4-clique pass over triangle records, or
                 // null for the scan over bitset rows
    i64 *acc_rec;  // [cap] per-slot sums of the tau pass over cached triangle records: acc
                   // itself, or LDS over the hash that this pass does not use
};

// Triangle records kept by Stage I for the tau pass: one u64 per triangle found at
// its lowest vertex u, (slot of v->w) << 32 | p << 16 | i, where i and p are the
// positions of v and w in N+(u).  Vertex u owns records [off[u], off[u]+cnt[u]);
// cnt[u] = -1 means its records were not kept and tau probes it again.  Space is
// handed out in chunks per wave/workgroup, so there is one global atomic per chunk;
// an item that may find more triangles than a chunk holds reserves its own space.
struct TriCache {
    u64 *rec;
    i64 cap;        // records
    u64 *bump;      // next free record
    i64 *off;       // int64[n]
    i32 *cnt;       // int32[n]
    i64 chunk;      // records reserved at a time
};

struct ItemState {  // per item group, in LDS
    i64 chunk_cur, chunk_end, item_base;
    i32 item_ok, item_cnt;
    i32 item_own;   // the item reserved its records outside the chunk
    i32 full;       // the record space ran out: stop asking for chunks
};

// Row bounds of a Stage I / tau item (and its kept triangles), loaded together so
// that the kernels can fetch them one item ahead.
struct PMeta {
    i32 u, base, du, tcnt;
    i64 toff;
};

template <int MODE>
__device__ __forceinline__ PMeta p_meta(const DevGraph &g, const TriCache &tc, i32 u) {
    PMeta m{u, 0, 0, -1, 0};
    if (u >= 0) {
        m.base = vmeta_at(g, u, VM_NSPLIT);
        m.du = vmeta_at(g, u, VM_END) - m.base;
        if (MODE == PROBE_TAU) {
            m.tcnt = tc.cnt[u];
            m.toff = tc.off[u];
        }
    }
    return m;
}

#define PL_NT 1024  // threads of a large Stage I item
typedef int v4i32 __attribute__((ext_vector_type(4)));
typedef int v16i32 __attribute__((ext_vector_type(16)));

// Sixteen bits of a bitset row as sixteen 0/1 bytes (bit q -> byte q): each nibble
// spread by one multiply whose shifted copies (0, 7, 14, 21) never overlap.
__device__ __forceinline__ v4i32 bits16_to_bytes(u32 w) {
    v4i32 r;
    r[0] = (int)(((w & 0xfu) * 0x204081u) & 0x01010101u);
    r[1] = (int)((((w >> 4) & 0xfu) * 0x204081u) & 0x01010101u);
    r[2] = (int)((((w >> 8) & 0xfu) * 0x204081u) & 0x01010101u);
    r[3] = (int)((((w >> 12) & 0xfu) * 0x204081u) & 0x01010101u);
    return r;
}

// The 4-clique pass of a large item as a dense contraction: with A the 0/1
// adjacency of H_u (the bitset, rows of `pitch` words), C = A*A counts the common
// neighbours of every pair, and sk[j] = sum over i of A[j][i] C[j][i] is twice the
// number of triangles of H_u through j (the per-slot sums the record pass builds).
// Each wave takes 32x32 tiles (J, I) with J <= I (C and A are symmetric, so an
// off-diagonal tile also serves its transpose) and runs one int8 MFMA
// (32x32x32, 0/1 bytes expanded from sixteen bits per lane) per 32 columns of A:
// lane l supplies row (or column) l % 32 and the bits (l / 32) * 16 .. + 16 of the
// word, and accumulator q holds row (q / 4) * 8 + (l / 32) * 4 + q % 4 of column
// l % 32 (the layout of the 32x32 MFMA forms).  Rows and columns past du read zero.
template <int NT>
__device__ __forceinline__ i64 dense_k4_sums(const u32 *A, int pitch, int du, int nw, i32 *sk, int tid) {
    const int wv = tid / WAVE, l = lane_id();
    const int nb = (du + 31) >> 5;
    const int ntiles = nb * (nb + 1) / 2;
    const int sh = (l >> 5) << 4;
    i64 words = 0;
    for (int tix = wv; tix < ntiles; tix += NT / WAVE) {
        int J = 0, rem = tix;
        while (rem >= nb - J) {
            rem -= nb - J;
            J++;
        }
        const int I = J + rem;
        const int ra = J * 32 + (l & 31), rb = I * 32 + (l & 31);
        const bool va = ra < du, vb = rb < du;
        v16i32 acc = {};
        for (int kw = 0; kw < nw; kw++) {
            const u32 wa = va ? A[ra * pitch + kw] : 0u;
            const u32 wb = vb ? A[rb * pitch + kw] : 0u;
            acc = __builtin_amdgcn_mfma_i32_32x32x32_i8(bits16_to_bytes((wa >> sh) & 0xffffu),
                                                         bits16_to_bytes((wb >> sh) & 0xffffu), acc, 0, 0, 0);
        }
        words += 2 * nw;
        const int i = I * 32 + (l & 31);
#pragma unroll
        for (int q = 0; q < 16; q++) {
            const int j = J * 32 + (q >> 2) * 8 + (l >> 5) * 4 + (q & 3);
            if (j < du && i < du && acc[q] && ((A[j * pitch + (i >> 5)] >> (i & 31)) & 1u)) {
                atomicAdd(&sk[j], acc[q]);
                if (J < I) atomicAdd(&sk[i], acc[q]);
            }
        }
    }
    return words;
}

template <int NT, int MODE, int QP, int MP = 0, int MAXDU = (1 << 30), bool WIDE = false>
__device__ __forceinline__ void probe_item(const DevGraph &g, const PMeta &pm, int tid, const ProbeMem &M, int hc,
                                           int pitch, i32 *__restrict__ t, i64 *__restrict__ K4,
                                           i64 *__restrict__ tau, i64 *red, i32 *red32, const TriCache &tc,
                                           ItemState *S, i64 *__restrict__ counters) {
    constexpr bool TRI = MODE != PROBE_TAU;  // Stage I/II work (with or without per-edge 4-cliques)
    const i64 t_start = (counters && TRI) ? (i64)clock64() : 0;
    const i32 u = pm.u, base = pm.base, du = pm.du;
    if (MODE == PROBE_TAU && pm.tcnt == 0) return;  // no triangle at u: nothing to add
    if (MODE == PROBE_TAU && pm.tcnt >= 0) {
        // cached triangles: tau from the records and the final t values
        i64 *const acc = M.acc_rec;
        for (int i = tid; i < du; i += NT) {
            M.nb[i] = g.ncol[base + i];
            M.tcnt[i] = t[base + i];
            acc[i] = 0;
        }
        item_sync<NT>();
        const i64 r0 = pm.toff, r1 = r0 + pm.tcnt;
        i64 tau_local = 0;
        // TAU_RK records per thread in flight; records of one probe batch are stored
        // in lane order, so runs of lanes share i and add to acc[i] once per run
        for (i64 rb = r0; rb < r1; rb += (i64)NT * TAU_RK) {
            u64 rec[TAU_RK];
            i32 tq[TAU_RK];
#pragma unroll
            for (int k = 0; k < TAU_RK; k++) {
                const i64 r = rb + tid + (i64)k * NT;
                rec[k] = r < r1 ? tc.rec[r] : ~0ull;
            }
#pragma unroll
            for (int k = 0; k < TAU_RK; k++) tq[k] = rec[k] != ~0ull ? t[(i32)(rec[k] >> 32)] : 0;
#pragma unroll
            for (int k = 0; k < TAU_RK; k++) {
                const bool ok = rec[k] != ~0ull;
                const int i = ok ? (int)(rec[k] & 0xffffu) : 0, p = ok ? (int)((rec[k] >> 16) & 0xffffu) : 0;
                tau_local += tq[k];
                if constexpr (NT >= WAVE) wave_run_add(acc, i, ok ? M.tcnt[p] : 0);
                else if (ok) atomicAdd((unsigned long long *)&acc[i], (unsigned long long)M.tcnt[p]);
                if (ok) atomicAdd((unsigned long long *)&acc[p], (unsigned long long)M.tcnt[i]);
            }
        }
        item_sync<NT>();
        for (int j = tid; j < du; j += NT) {
            i64 a = acc[j];
            if (a) atomic_add_i64(&tau[M.nb[j]], a);
        }
        i64 s = item_sum<NT>(tau_local, red, tid);
        if (tid == 0 && s) atomic_add_i64(&tau[u], s);
        item_sync<NT>();
        return;
    }
    const u32 hmask = (u32)hc - 1;
    const int nw = (du + 31) >> 5;
    for (int i = tid; i < hc; i += NT) M.hkey[i] = -1;
    item_sync<NT>();
    for (int i = tid; i < du; i += NT) {
        i32 v = g.ncol[base + i];
        const i32 b = vmeta_at(g, v, VM_NSPLIT);
        if (M.nb) M.nb[i] = v;
        M.beg[i] = b;
        M.off[i + 1] = vmeta_at(g, v, VM_END) - b;
        u32 sl = hslot((u32)v, hmask);
        while (atomicCAS(&M.hkey[sl], -1, v) != -1) sl = (sl + 1) & hmask;
        M.hpos[sl] = i;
        // acc serves the tau pass only; the triangle pass leaves it alone, so that
        // its kernels need no LDS for it
        if (MODE == PROBE_TAU) M.acc[i] = 0;
        if (TRI) {
            M.tcnt[i] = 0;
            for (int k = 0; k < nw; k++) M.A[i * pitch + k] = 0u;
        }
    }
    item_sync<NT>();
    item_scan<NT>(M.off, du, tid, red32);
    const i32 total = M.off[du];
    if (TRI && tid == 0) {
        // room for every possible triangle of this item: min(probes, C(du, 2))
        i64 ub = min((i64)total, (i64)du * (du - 1) / 2);
        S->item_ok = 0;
        S->item_cnt = 0;
        S->item_own = 0;
        if (tc.rec && ub > tc.chunk && !S->full) {
            // more than a chunk: the item reserves its own space
            u64 b = atomicAdd((unsigned long long *)tc.bump, (unsigned long long)ub);
            if ((i64)b + ub <= tc.cap) {
                S->item_ok = 1;
                S->item_own = 1;
                S->item_base = (i64)b;
            } else {
                S->full = 1;
            }
        } else if (tc.rec && !S->full) {
            if (S->chunk_end - S->chunk_cur < ub) {
                u64 b = atomicAdd((unsigned long long *)tc.bump, (unsigned long long)tc.chunk);
                if ((i64)b + tc.chunk <= tc.cap) {
                    S->chunk_cur = (i64)b;
                    S->chunk_end = (i64)b + tc.chunk;
                } else {
                    S->chunk_cur = S->chunk_end = 0;
                    S->full = 1;
                }
            }
            if (S->chunk_end - S->chunk_cur >= ub) {
                S->item_ok = 1;
                S->item_base = S->chunk_cur;
            }
        }
    }
    item_sync<NT>();
    const bool keep = TRI && S->item_ok;
    const i64 item_base = keep ? S->item_base : 0;
    // a bitset the 4-clique pass reads from an LDS copy is rebuilt there from the
    // item's triangle records (each an edge of H_u) after the probes, rather than
    // built in global memory with two device-scope atomics per hit
    const bool rebuild = keep && M.A_k4 != M.A;
    i64 tau_local = 0;
    // rounds of NT*QP probes: each thread locates its QP probes together, then
    // issues all their loads before the first hash lookup.  With MP > 0 the
    // probes are located through a segment map built every MP/QP rounds.
    static_assert(MP % QP == 0, "map blocks hold whole rounds");
    i32 mbase = 0;
    for (i32 eb = 0; eb < total; eb += NT * QP) {
        const int nj = min(QP, (total - eb + NT - 1) / NT);
        int lo[QP];
        i32 qq[QP], ww[QP];
        if constexpr (MP > 0 && WIDE) {
            if (eb % (NT * MP) == 0) {
                mbase = eb;
                item_sync<NT>();  // the previous block's map has been read
                q_segmap16<NT, MP>(M.off, du, eb, total, tid, M.seg);
                item_sync<NT>();
            }
#pragma unroll
            for (int j = 0; j < QP; j++) {
                const i32 e = eb + tid + j * NT;
                lo[j] = (j < nj && e < total) ? seg_at16(M.seg, e - mbase) : 0;
            }
        } else if constexpr (MP > 0) {
            static_assert(MAXDU <= 256, "a byte map holds the segment of items of at most 256 slots");
            if (eb % (NT * MP) == 0) {
                mbase = eb;
                item_sync<NT>();  // the previous block's map has been read
                q_segmap<NT, MP>(M.off, du, eb, total, tid, M.seg);
                item_sync<NT>();
            }
#pragma unroll
            for (int j = 0; j < QP; j++) {
                const i32 e = eb + tid + j * NT;
                lo[j] = (j < nj && e < total) ? seg_at(M.seg, e - mbase) : 0;
            }
        } else {
            q_locate<NT, QP>(M.off, du, eb + tid, nj, lo, total - 1);
        }
#pragma unroll
        for (int j = 0; j < QP; j++) {
            const i32 e = eb + tid + j * NT;
            qq[j] = (j < nj && e < total) ? M.beg[lo[j]] + (e - M.off[lo[j]]) : -1;
        }
#pragma unroll
        for (int j = 0; j < QP; j++) ww[j] = qq[j] >= 0 ? g.ncol[qq[j]] : -1;
#pragma unroll
        for (int j = 0; j < QP; j++) {
            if (j >= nj) break;
            const int i = lo[j];
            const i32 q = qq[j], w = ww[j];
            int p = -1;
            if (w >= 0) {
                u32 sl = hslot((u32)w, hmask);
                while (true) {
                    i32 k = M.hkey[sl];
                    if (k == w) { p = M.hpos[sl]; break; }
                    if (k == -1) break;
                    sl = (sl + 1) & hmask;
                }
            }
            if (p < 0) continue;
            if (TRI) {
                atomicAdd(&M.tcnt[i], 1);
                atomicAdd(&M.tcnt[p], 1);
                atomicAdd(&t[q], 1);
                if (!rebuild) {
                    atomicOr(&M.A[i * pitch + (p >> 5)], 1u << (p & 31));
                    atomicOr(&M.A[p * pitch + (i >> 5)], 1u << (i & 31));
                }
                if (keep) {
                    i32 r = atomicAdd(&S->item_cnt, 1);
                    tc.rec[item_base + r] = ((u64)(u32)q << 32) | ((u64)p << 16) | (u64)i;
                }
            } else {
                tau_local += t[q];
                atomicAdd((unsigned long long *)&M.acc[i], (unsigned long long)t[base + p]);
                atomicAdd((unsigned long long *)&M.acc[p], (unsigned long long)t[base + i]);
            }
        }
    }
    item_sync<NT>();
    if (TRI) {
        if (tid == 0) {
            if (keep) {
                tc.off[u] = item_base;
                tc.cnt[u] = S->item_cnt;
                if (!S->item_own) S->chunk_cur += S->item_cnt;
            } else {
                tc.cnt[u] = -1;
            }
        }
        i64 s_local = 0, tri2 = 0, words_scanned = 0;
        for (int j = tid; j < du; j += NT) {
            i32 c = M.tcnt[j];
            tri2 += c;
            if (c) atomicAdd(&t[base + j], c);
        }
        const u32 *A = M.A_k4;
        if (A != M.A) {
            item_sync<NT>();
            if (rebuild) {
                for (int i = tid; i < du * pitch; i += NT) M.A_k4[i] = 0u;
                item_sync<NT>();
                const i64 r1 = item_base + S->item_cnt;
                for (i64 r = item_base + tid; r < r1; r += NT) {
                    const u64 rec = tc.rec[r];
                    const int i = (int)(rec & 0xffffu), p = (int)((rec >> 16) & 0xffffu);
                    atomicOr(&M.A_k4[i * pitch + (p >> 5)], 1u << (p & 31));
                    atomicOr(&M.A_k4[p * pitch + (i >> 5)], 1u << (i & 31));
                }
            } else {
                for (int i = tid; i < du * pitch; i += NT) M.A_k4[i] = M.A[i];
            }
            item_sync<NT>();
        }
        if (NT == PL_NT && MODE == PROBE_TRI) {
            // large items: the dense contraction (H_u of such items is dense enough
            // that A*A on the matrix cores beats an intersection per edge)
            i32 *sk = M.k4s;
            item_sync<NT>();
            for (int j = tid; j < du; j += NT) sk[j] = 0;
            item_sync<NT>();
            words_scanned += dense_k4_sums<NT>(A, pitch, du, nw, sk, tid);
            item_sync<NT>();
            for (int j = tid; j < du; j += NT) {
                const i64 sj = sk[j];
                if (sj) atomic_add_i64(&K4[M.nb ? M.nb[j] : g.ncol[base + j]], sj >> 1);
                s_local += sj;
            }
        } else if (M.k4s && keep) {
            // every edge (i, p) of H_u once, from this item's triangle records: the
            // common neighbours of i and p in H_u close triangles of H_u through both,
            // summed per slot in k4s (which may share the spent tcnt)
            i32 *sk = M.k4s;
            item_sync<NT>();
            for (int j = tid; j < du; j += NT) sk[j] = 0;
            item_sync<NT>();
            const i64 r1 = item_base + S->item_cnt;
            for (i64 r = item_base + tid; r < r1; r += NT) {
                const u64 rec = tc.rec[r];
                const int i = (int)(rec & 0xffffu), p = (int)((rec >> 16) & 0xffffu);
                i32 c = 0;
                for (int k = 0; k < nw; k++) c += __popc(A[i * pitch + k] & A[p * pitch + k]);
                words_scanned += nw;
                if (c) {
                    atomicAdd(&sk[i], c);
                    atomicAdd(&sk[p], c);
                    // the record's probe slot is the edge (nb[i], nb[p]) itself
                    if constexpr (MODE == PROBE_EK4) atomic_add_i64(&tau[(i32)(rec >> 32)], c);
                }
            }
            item_sync<NT>();
            for (int j = tid; j < du; j += NT) {
                const i64 sj = sk[j];
                if (sj) atomic_add_i64(&K4[M.nb ? M.nb[j] : g.ncol[base + j]], sj >> 1);
                // sj / 2 = the 4-cliques through u and nb[j] with u lowest
                if constexpr (MODE == PROBE_EK4)
                    if (sj) atomic_add_i64(&tau[base + j], sj >> 1);
                s_local += sj;
            }
        } else {
            for (int j = tid; j < du; j += NT) {
                i64 sj = 0;
                for (int wd = 0; wd < nw; wd++) {
                    u32 bits = A[j * pitch + wd];
                    while (bits) {
                        int b = __ffs(bits) - 1;
                        bits &= bits - 1;
                        int i = wd * 32 + b;
                        words_scanned += nw;
                        if constexpr (MODE == PROBE_EK4) {
                            i32 c = 0;
                            for (int k = 0; k < nw; k++) c += __popc(A[i * pitch + k] & A[j * pitch + k]);
                            sj += c;
                            if (i < j && c) {
                                // edge (nb[i], nb[j]): nb[j] lies in N+(nb[i]), found by search
                                const i32 vi = M.nb ? M.nb[i] : g.ncol[base + i];
                                const i32 vj = M.nb ? M.nb[j] : g.ncol[base + j];
                                const i32 q = lower_bound_i32(g.ncol, vmeta_at(g, vi, VM_NSPLIT),
                                                              vmeta_at(g, vi, VM_END), vj);
                                atomic_add_i64(&tau[q], c);
                            }
                        } else {
                            for (int k = 0; k < nw; k++) sj += __popc(A[i * pitch + k] & A[j * pitch + k]);
                        }
                    }
                }
                // sj = 2 x (triangles of H_u through j) = 2 x (4-cliques containing u and nb[j])
                if (sj) atomic_add_i64(&K4[M.nb ? M.nb[j] : g.ncol[base + j]], sj >> 1);
                if constexpr (MODE == PROBE_EK4)
                    if (sj) atomic_add_i64(&tau[base + j], sj >> 1);
                s_local += sj;
            }
        }
        i64 s = item_sum<NT>(s_local, red, tid);
        if (tid == 0 && s) atomic_add_i64(&K4[u], s / 6);
        if (counters) {
            tri2 = item_sum<NT>(tri2, red, tid);
            words_scanned = item_sum<NT>(words_scanned, red, tid);
            if (tid == 0) {
                i64 *c = counters + (i64)u * NUM_COUNTERS;
                c[1] = tri2 >> 1;
                c[2] = words_scanned;
                c[6] = (i64)clock64() - t_start;
            }
        }
    } else {
        for (int j = tid; j < du; j += NT) {
            i64 a = M.acc[j];
            if (a) atomic_add_i64(&tau[M.nb ? M.nb[j] : g.ncol[base + j]], a);
        }
        i64 s = item_sum<NT>(tau_local, red, tid);
        if (tid == 0 && s) atomic_add_i64(&tau[u], s);
    }
    item_sync<NT>();
}

// One wave per vertex, |N+(u)| <= 64, four items per 256-thread block.
#define PW_QP 4   // probes per thread and round, wave items
#define PB_QP 8   // probes per thread and round, workgroup items
#define PL_QP 4   // probes per thread and round, large items
#define PW_MP 16  // probes per thread of a segment-map block, wave items (0: search)
#define PB_MP 8   // the same, workgroup items
#define PW_WPE 8  // waves per SIMD the wave kernel is compiled for: 64 registers (with
                  // one register more a SIMD holds a wave less, measured 30 % slower)
template <int MODE>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(PW_WPE))) k_probe_wave(DevGraph g, const i32 *__restrict__ list,
                                                    const GraphStats *__restrict__ st, i32 *t, i64 *K4,
                                                    i64 *tau, TriCache tc, i64 *counters) {
    constexpr int CAP = TRI_WAVE_CAP, HC = 2 * CAP, PITCH = bit_pitch(CAP);
    __shared__ i32 s_hkey[4][HC];
    __shared__ i32 s_hpos[4][HC];
    __shared__ i32 s_off[4][CAP + 1];
    __shared__ i32 s_nb[4][CAP];
    __shared__ i32 s_beg[4][CAP];
    __shared__ i32 s_tcnt[4][CAP];
    __shared__ u32 s_A[4][CAP * PITCH];
    __shared__ i64 s_acc[4][CAP];
    __shared__ u32 s_seg[4][PW_MP > 0 ? WAVE * PW_MP / 4 : 1];
    __shared__ ItemState s_st[4];
    const int w = threadIdx.x / WAVE, tid = lane_id();
    ProbeMem M{s_hkey[w], s_hpos[w], s_off[w], s_nb[w], s_beg[w], s_tcnt[w], s_A[w], s_acc[w], s_A[w], s_seg[w], nullptr,
               s_acc[w]};
    if (tid == 0) {
        s_st[w].chunk_cur = s_st[w].chunk_end = 0;
        s_st[w].full = 0;
    }
    item_sync<WAVE>();
    const i32 cnt = st->cnt[WC_TRI_WAVE];
    const int waves = gridDim.x * 4;
    i32 it = blockIdx.x * 4 + w;
    PMeta cur = p_meta<MODE>(g, tc, it < cnt ? list[it] : -1);
    i32 un = it + waves < cnt ? list[it + waves] : -1;
    for (; it < cnt; it += waves) {
        // the next item's row bounds and the one after's id load while this one runs
        const PMeta nxt = p_meta<MODE>(g, tc, un);
        un = it + 2 * waves < cnt ? list[it + 2 * waves] : -1;
        probe_item<WAVE, MODE, PW_QP, PW_MP, CAP>(g, cur, tid, M, HC, PITCH, t, K4, tau, nullptr, nullptr, tc,
                                             &s_st[w], counters);
        cur = nxt;
    }
}

// Sixteen lanes per vertex, |N+(u)| <= TRI_GROUP_CAP (16 items per 256-thread block):
// for items with little work, which would leave most of a wave idle.
#define PG_NT 16
#define PG_QP 4
template <int MODE>
__global__ void __launch_bounds__(256) k_probe_group(DevGraph g, const i32 *__restrict__ list,
                                                     const GraphStats *__restrict__ st, i32 *t, i64 *K4,
                                                     i64 *tau, TriCache tc, i64 *counters) {
    constexpr int CAP = TRI_GROUP_CAP, HC = 2 * CAP, PITCH = bit_pitch(CAP), NG = 256 / PG_NT;
    __shared__ i32 s_hkey[NG][HC];
    __shared__ i32 s_hpos[NG][HC];
    __shared__ i32 s_off[NG][CAP + 1];
    __shared__ i32 s_nb[NG][CAP];
    __shared__ i32 s_beg[NG][CAP];
    __shared__ i32 s_tcnt[NG][CAP];
    __shared__ u32 s_A[NG][CAP * PITCH];
    __shared__ i64 s_acc[NG][CAP];
    __shared__ ItemState s_st[NG];
    const int gr = threadIdx.x / PG_NT, tid = threadIdx.x % PG_NT;
    ProbeMem M{s_hkey[gr], s_hpos[gr], s_off[gr], s_nb[gr], s_beg[gr], s_tcnt[gr], s_A[gr], s_acc[gr], s_A[gr],
               nullptr, nullptr, s_acc[gr]};
    if (tid == 0) {
        s_st[gr].chunk_cur = s_st[gr].chunk_end = 0;
        s_st[gr].full = 0;
    }
    item_sync<PG_NT>();
    const i32 cnt = st->cnt[WC_TRI_GROUP];
    const int groups = gridDim.x * NG;
    i32 it = blockIdx.x * NG + gr;
    PMeta cur = p_meta<MODE>(g, tc, it < cnt ? list[it] : -1);
    i32 un = it + groups < cnt ? list[it + groups] : -1;
    for (; it < cnt; it += groups) {
        const PMeta nxt = p_meta<MODE>(g, tc, un);
        un = it + 2 * groups < cnt ? list[it + 2 * groups] : -1;
        probe_item<PG_NT, MODE, PG_QP>(g, cur, tid, M, HC, PITCH, t, K4, tau, nullptr, nullptr, tc, &s_st[gr],
                                       counters);
        cur = nxt;
    }
}

// One PB_NT-thread workgroup per vertex, 64 < |N+(u)| <= TRI_BLOCK_CAP.
#define PB_NT 512
template <int MODE>
__global__ void __launch_bounds__(PB_NT) k_probe_block(DevGraph g, const i32 *__restrict__ list,
                                                     const GraphStats *__restrict__ st, i32 *t, i64 *K4,
                                                     i64 *tau, TriCache tc, i64 *counters) {
    constexpr int CAP = TRI_BLOCK_CAP, HC = 1024, PITCH = bit_pitch(CAP);
    static_assert(HC >= 2 * CAP && (HC & (HC - 1)) == 0, "the hash: a power of two, at most half full");
    __shared__ i32 s_hkey[HC];
    __shared__ i32 s_hpos[HC];
    __shared__ i32 s_off[CAP + 1];
    __shared__ i32 s_nb[CAP];
    __shared__ i32 s_beg[CAP];
    __shared__ i32 s_tcnt[CAP];
    __shared__ u32 s_A[CAP * PITCH];
    __shared__ i64 s_acc[CAP];
    __shared__ u32 s_seg[PB_NT * PB_MP / 2];
    __shared__ i64 s_red[PB_NT / WAVE];
    __shared__ i32 s_red32[PB_NT / WAVE];
    __shared__ ItemState s_st;
    // the triangle pass reads neighbours from the row again (its LDS is full)
    ProbeMem M{s_hkey, s_hpos, s_off, MODE != PROBE_TAU ? nullptr : s_nb, s_beg, s_tcnt, s_A, s_acc, s_A, s_seg,
               s_tcnt, s_acc};
    if (threadIdx.x == 0) {
        s_st.chunk_cur = s_st.chunk_end = 0;
        s_st.full = 0;
    }
    __syncthreads();
    const i32 cnt = st->cnt[WC_TRI_BLOCK];
    i32 it = blockIdx.x;
    PMeta cur = p_meta<MODE>(g, tc, it < cnt ? list[it] : -1);
    i32 un = it + (i32)gridDim.x < cnt ? list[it + gridDim.x] : -1;
    for (; it < cnt; it += gridDim.x) {
        const PMeta nxt = p_meta<MODE>(g, tc, un);
        un = it + 2 * (i32)gridDim.x < cnt ? list[it + 2 * gridDim.x] : -1;
        probe_item<PB_NT, MODE, PB_QP, PB_MP, CAP, true>(g, cur, threadIdx.x, M, HC, PITCH, t, K4, tau, s_red,
                                                         s_red32, tc, &s_st, counters);
        cur = nxt;
    }
}

// One lane per vertex for tiny items (|N+(u)| <= 8): N+(u) in registers, the
// induced graph H_u as an 8x8 bit matrix in one 64-bit word, no LDS.  Triangles
// are not kept for tau; the tau pass probes these items again.
template <int MODE>
__global__ void __launch_bounds__(256) k_probe_thread(DevGraph g, const i32 *__restrict__ list,
                                                      const GraphStats *__restrict__ st, i32 *t, i64 *K4,
                                                      i64 *tau, TriCache tc, i64 *counters) {
    constexpr int C = TRI_THREAD_CAP;
    const i32 cnt = st->cnt[WC_TRI_THREAD];
    for (i32 it = blockIdx.x * blockDim.x + threadIdx.x; it < cnt; it += gridDim.x * blockDim.x) {
        const i64 t_start = (counters && MODE != PROBE_TAU) ? (i64)clock64() : 0;
        const i32 u = list[it];
        const i32 base = g.nsplit[u];
        const i32 du = g.nrp[u + 1] - base;
        i32 nu[C];
        i32 tcl[C];
        i64 acc[C];
#pragma unroll
        for (int j = 0; j < C; j++) {
            nu[j] = j < du ? g.ncol[base + j] : -1;
            tcl[j] = 0;
            acc[j] = 0;
        }
        u64 A = 0;
        i64 tau_local = 0, probes = 0;
#pragma unroll
        for (int i = 0; i < C; i++) {
            if (i >= du) break;
            const i32 v = nu[i];
            const i32 q0 = vmeta_at(g, v, VM_NSPLIT), q1 = vmeta_at(g, v, VM_END);
            probes += q1 - q0;
            for (i32 q = q0; q < q1; q++) {
                const i32 w = g.ncol[q];
                int p = -1;
#pragma unroll
                for (int j = 0; j < C; j++)
                    if (j > i && nu[j] == w) p = j;
                if (p < 0) continue;
                if (MODE != PROBE_TAU) {
#pragma unroll
                    for (int j = 0; j < C; j++) tcl[j] += (j == i) + (j == p);
                    atomicAdd(&t[q], 1);
                    A |= (1ull << (i * C + p)) | (1ull << (p * C + i));
                } else {
                    tau_local += t[q];
                    const i64 tup = t[base + p], tui = t[base + i];
#pragma unroll
                    for (int j = 0; j < C; j++) acc[j] += (j == i) ? tup : ((j == p) ? tui : 0);
                }
            }
        }
        if (MODE != PROBE_TAU) {
            i64 s = 0, tri2 = 0, words = 0;
#pragma unroll
            for (int j = 0; j < C; j++) {
                if (j >= du) break;
                tri2 += tcl[j];
                if (tcl[j]) atomicAdd(&t[base + j], tcl[j]);
                const u32 rj = (u32)(A >> (j * C)) & 0xffu;
                i64 sj = 0;
#pragma unroll
                for (int i = 0; i < C; i++)
                    if ((rj >> i) & 1u) {
                        const i32 c = __popc(((u32)(A >> (i * C)) & 0xffu) & rj);
                        sj += c;
                        words++;
                        if constexpr (MODE == PROBE_EK4) {
                            if (i < j && c) {
                                // edge (nu[i], nu[j]): nu[j] lies in N+(nu[i])
                                const i32 q = lower_bound_i32(g.ncol, vmeta_at(g, nu[i], VM_NSPLIT),
                                                              vmeta_at(g, nu[i], VM_END), nu[j]);
                                atomic_add_i64(&tau[q], c);
                            }
                        }
                    }
                if (sj) atomic_add_i64(&K4[nu[j]], sj >> 1);
                if constexpr (MODE == PROBE_EK4)
                    if (sj) atomic_add_i64(&tau[base + j], sj >> 1);
                s += sj;
            }
            if (s) atomic_add_i64(&K4[u], s / 6);
            tc.cnt[u] = -1;
            if (counters) {
                i64 *c = counters + (i64)u * NUM_COUNTERS;
                c[1] = tri2 >> 1;
                c[2] = words;
                c[6] = (i64)clock64() - t_start;
            }
        } else {
            if (tau_local) atomic_add_i64(&tau[u], tau_local);
#pragma unroll
            for (int j = 0; j < C; j++)
                if (j < du && acc[j]) atomic_add_i64(&tau[nu[j]], acc[j]);
        }
        (void)probes;
    }
}

// |N+(u)| > TRI_BLOCK_CAP: the same item code with larger structures, 1024 threads.
// Layouts (LAY): 2 -- hash and per-slot arrays in dynamic LDS during the probes, the
// bitset of H_u built in the global slice and copied into the same LDS (over the
// hash) for the 4-clique pass; 1 -- as 2 but the 4-clique pass reads the global
// bitset; 0 -- everything but the reductions in the global slice.
__host__ __device__ inline i64 probe_large_lds_bytes(int cap, int hc) {
    return (i64)sizeof(i32) * (2 * (i64)hc + 4 * (i64)cap + 1);
}
__host__ __device__ inline i64 probe_large_k4_bytes(int cap, int hc) {
    const i64 words = bit_pitch(cap);
    const i64 probe = (i64)sizeof(i32) * (2 * (i64)hc + 3 * (i64)cap + 1);
    const i64 k4 = (i64)sizeof(u32) * cap * words + (i64)sizeof(i32) * cap;  // bitset copy, per-slot sums
    return (i64)sizeof(i32) * cap + (probe > k4 ? probe : k4);
}

template <int MODE, int LAY>
__global__ void __launch_bounds__(PL_NT) k_probe_large(DevGraph g, const i32 *__restrict__ list,
                                                       const GraphStats *__restrict__ st, i32 *t, i64 *K4,
                                                       i64 *tau, TriCache tc, char *scratch, i64 slice_bytes,
                                                       int cap, int hc, i64 *counters) {
    extern __shared__ __align__(16) char s_dyn[];
    __shared__ i64 s_red[PL_NT / WAVE];
    __shared__ i32 s_red32[PL_NT / WAVE];
    const int words = bit_pitch(cap);
    char *p = scratch + (i64)blockIdx.x * slice_bytes;
    ProbeMem M;
    M.seg = nullptr;
    M.acc = (i64 *)p; p += sizeof(i64) * cap;
    M.A = (u32 *)p; p += sizeof(u32) * (i64)cap * words;
    M.A_k4 = M.A;
    if (LAY == 2) {
        M.nb = (i32 *)s_dyn;
        char *q = s_dyn + sizeof(i32) * cap;
        M.A_k4 = (u32 *)q;
        // the 4-clique sums follow the bitset copy
        M.k4s = (i32 *)(q + sizeof(u32) * (i64)cap * words);
        M.hkey = (i32 *)q; q += sizeof(i32) * hc;
        M.hpos = (i32 *)q; q += sizeof(i32) * hc;
        M.off = (i32 *)q; q += sizeof(i32) * (cap + 1);
        M.beg = (i32 *)q; q += sizeof(i32) * cap;
        M.tcnt = (i32 *)q;
    } else {
        char *q = LAY == 1 ? s_dyn : p;
        M.hkey = (i32 *)q; q += sizeof(i32) * hc;
        M.hpos = (i32 *)q; q += sizeof(i32) * hc;
        M.off = (i32 *)q; q += sizeof(i32) * (cap + 1);
        M.nb = (i32 *)q; q += sizeof(i32) * cap;
        M.beg = (i32 *)q; q += sizeof(i32) * cap;
        M.tcnt = (i32 *)q;
        M.k4s = M.tcnt;
    }
    // the tau pass over cached records keeps its sums in LDS over hkey and hpos (8 hc >= 16 cap
    // bytes, the start rounded up to 8 bytes), which that pass leaves unused
    M.acc_rec = LAY == 0 ? M.acc : (i64 *)(s_dyn + (LAY == 2 ? (sizeof(i32) * (i64)cap + 7) & ~7ll : 0));
    __shared__ ItemState s_st;
    if (threadIdx.x == 0) {
        s_st.chunk_cur = s_st.chunk_end = 0;
        s_st.full = 0;
    }
    __syncthreads();
    const i32 cnt = st->cnt[WC_TRI_LARGE];
    for (i32 it = blockIdx.x; it < cnt; it += gridDim.x)
        probe_item<PL_NT, MODE, PL_QP>(g, p_meta<MODE>(g, tc, list[it]), threadIdx.x, M, hc, words, t, K4, tau, s_red,
                                   s_red32, tc, &s_st, counters);
}

i64 probe_large_slice_bytes(int cap, int hc, i64 lds_max) {
    int words = bit_pitch(cap);
    i64 b = sizeof(i64) * cap + sizeof(u32) * (i64)cap * words;
    if (probe_large_lds_bytes(cap, hc) > lds_max) b += probe_large_lds_bytes(cap, hc);
    return (b + 255) & ~255ll;
}


template <int W>
__device__ __forceinline__ void sums_vertex(const DevGraph &g, const i32 *__restrict__ t, const Accum &acc, i32 x,
                                            bool active, int l) {
    i32 b0 = 0, sp = 0, e0 = 0;
    if (active) {
        b0 = g.nrp[x];
        sp = g.nsplit[x];
        e0 = g.nrp[x + 1];
    }
    i64 St = 0, Stt = 0, Std = 0, Sd = 0, Sdd = 0;
    for (i32 s = b0 + l; s < e0; s += W) {
        i64 ta = (s < sp) ? t[g.mirror[s]] : t[s];
        i64 da = g.dslot[s];
        St += ta;
        Stt += ta * ta;
        Std += ta * da;
        Sd += da;
        Sdd += da * da;
    }
    St = group_sum64<W>(St);
    Stt = group_sum64<W>(Stt);
    Std = group_sum64<W>(Std);
    Sd = group_sum64<W>(Sd);
    Sdd = group_sum64<W>(Sdd);
    if (active && l == 0) {
        acc.St[x] = St;
        acc.Stt[x] = Stt;
        acc.Std[x] = Std;
        acc.Sd[x] = Sd;
        acc.Sdd[x] = Sdd;
        acc.Tp[2 * (i64)x] = St >> 1;
        acc.Tp[2 * (i64)x + 1] = Sd - (e0 - b0);
    }
}

// ---------------------------------------------------------------------------
// Neighbour sums over full rows.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_sums(DevGraph g, const i32 *__restrict__ t, Accum acc) {
    const int waves = gridDim.x * (blockDim.x / WAVE);
    const int wid = blockIdx.x * (blockDim.x / WAVE) + threadIdx.x / WAVE;
    const i32 cut = first_above(g.ndeg, g.n, SG_MAXDEG);
    constexpr int GPW = WAVE / SG;
    for (i32 xb = wid * GPW; xb < cut; xb += waves * GPW) {
        const i32 x = xb + lane_id() / SG;
        sums_vertex<SG>(g, t, acc, x, x < cut, lane_id() % SG);
    }
    for (i32 x = g.n - 1 - wid; x >= cut; x -= waves) sums_vertex<WAVE>(g, t, acc, x, true, lane_id());
}

// ---------------------------------------------------------------------------
// Second neighbour sums and the equations.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void solve_vertex(i64 d, i64 T, i64 psi1, i64 St, i64 Stt, i64 Std, i64 Sd, i64 Sdd,
                                             i64 ST, i64 Spsi1, i64 tau, i64 Q, i64 k4, i64 *f, i64 *psi,
                                             int *err) {
    // f-variables (Table 1) as neighbour sums over a in N(x):
    const i64 f13 = Stt - St;                                   // sum t(t-1)
    const i64 f11 = (d - 1) * St - Stt;                         // sum t(d(x)-1-t)
    const i64 f12 = tau - T;                                    // sum over triangles (t(yz)-1)
    const i64 f10 = (Std - St) - 2 * tau;                       // sum t(d(a)-1) - 2 tau
    const i64 f5 = (d - 1) * (Sd - d) - (d - 1) * St - (Std - St) + Stt;
    const i64 f6 = (Sdd - 3 * Sd + 2 * d) - 2 * Std + 3 * St + Stt;
    const i64 f9 = 2 * ST - St - 2 * tau;
    const i64 f4 = Spsi1 - d * (d - 1) - (Std - St) - f9;
    const i64 f8 = 2 * Q - f13;
    f[0] = f12; f[1] = f10; f[2] = f13; f[3] = f11; f[4] = f5; f[5] = f6; f[6] = f9; f[7] = f4; f[8] = f8;
    const i64 h13 = f13, h11 = f11 + f13, h9 = f9, h8 = f13 + f8, h6 = f6 - f13;
    if ((h13 | h11 | h9 | h8 | h6) & 1) *err = 1;
    psi[0] = d;
    psi[1] = psi1;
    psi[2] = d * (d - 1) / 2;
    psi[3] = T;
    psi[4] = 2 * f12 + f4 + f10 + f9;
    psi[5] = 2 * f12 + f5 + f10 + f11;
    psi[6] = h6 / 2 + f10 + 2 * f12;
    psi[7] = d * (d - 1) * (d - 2) / 6;
    psi[8] = h8 / 2;
    psi[9] = f12 + h9 / 2;
    psi[10] = f10 + 2 * f12;
    psi[11] = h11 / 2;
    psi[12] = f12;
    psi[13] = h13 / 2;
    psi[14] = k4;
}

// Induced counts psi'_k from the non-induced psi_k of one vertex.  An induced
// occurrence of a graphlet on a vertex set S contains, as non-induced occurrences
// on S, its connected spanning subgraphs: psi = C psi', C unit upper triangular in
// this orbit numbering (C[k][j] = in how many connected spanning subgraphs of the
// graphlet of orbit j a vertex of orbit j has orbit k).  These are the rows of
// C^-1; three of them are the induced equations printed next to the non-induced
// ones (Section 5, relating ORCA and NI-ORCA): psi'_13 = psi_13 - 3 psi_14,
// psi'_11 = psi_11 - 2 psi_13 + 3 psi_14, psi'_10 = psi_10 - 2 psi_12 - 2 psi_13
// + 6 psi_14.
__device__ __forceinline__ void induced_from_noninduced(const i64 *p, i64 *o) {
    o[0] = p[0];
    o[1] = p[1] - 2 * p[3];
    o[2] = p[2] - p[3];
    o[3] = p[3];
    o[4] = p[4] - 2 * p[8] - 2 * p[9] - p[10] + 4 * p[12] + 2 * p[13] - 6 * p[14];
    o[5] = p[5] - 2 * p[8] - p[10] - 2 * p[11] + 2 * p[12] + 4 * p[13] - 6 * p[14];
    o[6] = p[6] - p[9] - p[10] + 2 * p[12] + p[13] - 3 * p[14];
    o[7] = p[7] - p[11] + p[13] - p[14];
    o[8] = p[8] - p[12] - p[13] + 3 * p[14];
    o[9] = p[9] - 2 * p[12] + 3 * p[14];
    o[10] = p[10] - 2 * p[12] - 2 * p[13] + 6 * p[14];
    o[11] = p[11] - 2 * p[13] + 3 * p[14];
    o[12] = p[12] - 3 * p[14];
    o[13] = p[13] - 3 * p[14];
    o[14] = p[14];
}

template <int W, bool INDUCED>
__device__ __forceinline__ void solve_one(const DevGraph &g, const Accum &acc, i64 *__restrict__ out,
                                          i64 *__restrict__ fvars, i32 x, bool active, int l, int *err) {
    i32 b0 = 0, e0 = 0;
    if (active) {
        b0 = g.nrp[x];
        e0 = g.nrp[x + 1];
    }
    i64 ST = 0, Sp = 0;
    for (i32 s = b0 + l; s < e0; s += W) {
        i32 a = g.ncol[s];
        const longlong2 tp = *reinterpret_cast<const longlong2 *>(acc.Tp + 2 * (i64)a);
        ST += tp.x;
        Sp += tp.y;
    }
    ST = group_sum64<W>(ST);
    Sp = group_sum64<W>(Sp);
    if (!active) return;
    // lanes 0..14 of the group each write one column; all compute the same row
    i64 f[9], psi[15];
    solve_vertex(e0 - b0, acc.Tp[2 * (i64)x], acc.Tp[2 * (i64)x + 1], acc.St[x], acc.Stt[x], acc.Std[x], acc.Sd[x],
                 acc.Sdd[x], ST, Sp, acc.tau[x], acc.Q[x], acc.K4[x], f, psi, err);
    if constexpr (INDUCED) {
        i64 ni[15];
#pragma unroll
        for (int k = 0; k < 15; k++) ni[k] = psi[k];
        induced_from_noninduced(ni, psi);
    }
    const i64 xo = g.order[x];
    if (out && l < 15) {
        i64 v = 0;
#pragma unroll
        for (int k = 0; k < 15; k++) v = (l == k) ? psi[k] : v;
        out[xo * 15 + l] = v;
    }
    if (fvars && l < 9) {
        i64 v = 0;
#pragma unroll
        for (int k = 0; k < 9; k++) v = (l == k) ? f[k] : v;
        fvars[xo * 9 + l] = v;
    }
}

template <bool INDUCED>
__global__ void __launch_bounds__(256) k_solve(DevGraph g, Accum acc, i64 *__restrict__ out,
                                               i64 *__restrict__ fvars, GraphStats *__restrict__ st) {
    const int waves = gridDim.x * (blockDim.x / WAVE);
    const int wid = blockIdx.x * (blockDim.x / WAVE) + threadIdx.x / WAVE;
    const i32 cut = first_above(g.ndeg, g.n, SG_MAXDEG);
    constexpr int GPW = WAVE / SG;
    int err = 0;
    for (i32 xb = wid * GPW; xb < cut; xb += waves * GPW) {
        const i32 x = xb + lane_id() / SG;
        solve_one<SG, INDUCED>(g, acc, out, fvars, x, x < cut, lane_id() % SG, &err);
    }
    for (i32 x = g.n - 1 - wid; x >= cut; x -= waves)
        solve_one<WAVE, INDUCED>(g, acc, out, fvars, x, true, lane_id(), &err);
    if (err) atomicOr(&st->err, 1);
}

// ---------------------------------------------------------------------------
// 4-cycles.
// ---------------------------------------------------------------------------
enum { Q_LIGHT = 0, Q_HEAVY = 1 };

// Segment (wedge run) of slot s of item x.
template <int MODE>
__device__ __forceinline__ void q_segment(const DevGraph &g, i32 x, i32 s, i32 sp, i32 &v, i32 &beg, i32 &end) {
    // the run bounds were written per slot next to the mirror slots, so that they
    // load alongside the neighbour rather than after it
    v = g.ncol[s];
    if (MODE == Q_LIGHT) {
        beg = g.lbeg[s];
        end = g.mirror[s];
    } else {
        const int2 h = g.hseg[s];
        beg = h.x;
        end = h.y;
    }
}

struct QChunk {
    i32 *off;    // [dc+1]
    i32 *vv;     // [dc]
    i32 *beg;    // [dc]
    i64 *mid;    // [dc]
    u32 *seg;    // segment byte of each wedge of a step (NT * max(QK, QS) bytes), or null
};

// How each 4-cycle kernel locates wedges (0 a search per wedge, 2 a byte map built by
// seg_map_scan, 3 the same map built by q_segmap: one search per thread, then a walk),
// chosen per kernel by measurement: a map costs LDS, and so occupancy, which the
// kernels win back by crediting middles straight to Q instead of through per-segment
// sums in LDS; the walk suits the heavy workgroup kernels, whose long segments make
// it short, the scan the light ones.
#define QMAP_QLW 2
#define QMAP_QLB 2
#define QMAP_QHW 2
#define QMAP_QHB 3
#define QMAP_QD 3
// Which ones credit middles straight to Q (and so keep no per-segment sums in LDS).
#define QGMID_QHW 1
#define QGMID_QHB 0
#define QGMID_QLW 1
#define QGMID_QLB 1


// Loads chunk [c0, c0+len) of the item's slots; returns its wedge count.
template <int NT, int MODE>
__device__ __forceinline__ i32 q_load_chunk(const DevGraph &g, i32 x, i32 s0, i32 sp, i32 c0, i32 len,
                                            const QChunk &C, int tid, i32 *red32) {
    for (int i = tid; i < len; i += NT) {
        i32 v, b, e;
        q_segment<MODE>(g, x, s0 + c0 + i, sp, v, b, e);
        C.vv[i] = v;
        C.beg[i] = b;
        C.off[i + 1] = e - b;
        if (C.mid) C.mid[i] = 0;
    }
    item_sync<NT>();
    item_scan<NT>(C.off, len, tid, red32);
    return C.off[len];
}

// Counter policies (inc / get of a key's count): LightHash (LDS hash of keys and
// counts), PackedHash (LDS hash of heavy key index and count in one word),
// DenseCounter (16-bit LDS counters over [h0, h0+K)), GlobalCounter (int32 counters
// over [0, n) in global scratch).

struct DenseCounter {
    static constexpr bool LOC_IS_KEY = true;  // a key's counter index is k - h0
    u32 *w;   // K/2 words
    i32 h0;
    __device__ int loc_of(i32 k) const { return k - h0; }
    // counts k; returns its counter's index, own set when this call took it from 0
    __device__ int inc_at(i32 k, bool &own) const {
        const i32 i = k - h0;
        const u32 old = atomicAdd(&w[i >> 1], 1u << ((i & 1) << 4));
        own = ((old >> ((i & 1) << 4)) & 0xffffu) == 0;
        return i;
    }
    __device__ void inc(i32 k) const {
        bool own;
        inc_at(k, own);
    }
    __device__ i32 at(int i) const { return (i32)((w[i >> 1] >> ((i & 1) << 4)) & 0xffffu); }
    __device__ i32 get(i32 k) const { return at(k - h0); }
    // count of an owned counter, which is returned to zero (the word's other half may
    // be taken at the same time)
    __device__ i32 take(int i) const {
        const int sh = (i & 1) << 4;
        const u32 old = atomicAnd(&w[i >> 1], ~(0xffffu << sh));
        return (i32)((old >> sh) & 0xffffu);
    }
};

struct GlobalCounter {
    static constexpr bool LOC_IS_KEY = false;
    i32 *c;       // [n] zero between items
    i32 *used;    // list of touched keys
    i32 *nused;   // LDS counter
    __device__ void inc(i32 k) const {
        if (atomicAdd(&c[k], 1) == 0) used[atomicAdd(nused, 1)] = k;
    }
    __device__ i32 get(i32 k) const { return c[k]; }
};

// Where C(c, 2) for a key with count c goes: Q of the key itself (light items, keys
// are vertices) or the heavy key's credit row.
struct CreditLight {
    i64 *Q;
    __device__ void operator()(i32 k, i64 cc) const { atomic_add_i64(&Q[k], cc); }
};
struct CreditHeavy {
    i64 *prow;
    i32 h0;
    __device__ void operator()(i32 k, i64 cc) const { atomic_add_i64(&prow[k - h0], cc); }
};

// Row bounds of a 4-cycle item and its wedge count, loaded together so that the
// kernels can fetch them one item ahead.
struct QMeta {
    i32 x, s0, sp, s1;
    i64 w;
};

template <int MODE>
__device__ __forceinline__ QMeta q_meta(const DevGraph &g, i32 x) {
    QMeta m{x, 0, 0, 0, 0};
    if (x >= 0) {
        m.s0 = vmeta_at(g, x, VM_BEGIN);
        m.sp = vmeta_at(g, x, VM_NSPLIT);
        m.s1 = vmeta_at(g, x, VM_END);
        m.w = (MODE == Q_LIGHT) ? g.wlight[x] : g.wheavy[x];
    }
    return m;
}

// Both sweeps over the item's wedges, chunk by chunk.  Each thread takes QS wedges
// per step (independent loads in flight); their segments come from a search over
// the chunk's prefix offsets in LDS or from a segment map.  When the whole item is
// one chunk of at most NT*QK wedges, every thread keeps its wedges' keys (and,
// unless the counter derives it from the key, where each key's count lives) in
// registers: the keys are read from memory once, all loads of a thread in flight
// together, and the second sweep needs neither loads nor lookups; the thread that
// created a key's counter then credits C(c, 2) through cr, adds it to *local and
// empties the counter, and the call returns true.  Otherwise (false) the counters
// are left for the caller to harvest.
// MAP: how wedges find their segments -- 0 a search each, 2 seg_map_scan, 3 q_segmap.
// GMID: middles' credits go straight to Q (runs of lanes in one segment add once)
// rather than through C.mid.
template <int NT, int MODE, int QK = 0, int MAP = 0, bool GMID = false, typename Ctr, typename Credit>
__device__ __forceinline__ bool q_sweeps(const DevGraph &g, const QMeta &mt, const Ctr &ctr, const QChunk &C, int dc,
                                         int tid, i32 *red32, i64 *__restrict__ Q, const Credit &cr, i64 *local) {
    const i32 x = mt.x, s0 = mt.s0, sp = mt.sp;
    const i32 ns = (MODE == Q_LIGHT) ? sp - s0 : mt.s1 - s0;
    const bool single = ns <= dc;
    if constexpr (QK > 0) {
        if (single) {
            const i32 total = wave_uniform(q_load_chunk<NT, MODE>(g, x, s0, sp, 0, ns, C, tid, red32));
            if (total <= NT * QK) {
                const int nj = (total + NT - 1) / NT;
                int lo[QK];
                i32 key[QK];
                if constexpr (MAP > 0) {
                    if constexpr (MAP == 3) {
                        q_segmap<NT, QK>(C.off, ns, 0, total, tid, C.seg);
                        item_sync<NT>();
                    } else {
                        seg_map_scan<NT, QK>(C.off, ns, 0, total, tid, C.seg, red32);
                    }
#pragma unroll
                    for (int j = 0; j < QK; j++) lo[j] = j < nj ? seg_at(C.seg, min(tid + j * NT, total - 1)) : 0;
                } else {
                    q_locate<NT, QK>(C.off, ns, tid, nj, lo, total - 1);
                }
                // lanes past the end repeat the last wedge's reads (in bounds, results
                // unused), so that the loads need no per-lane branch
#pragma unroll
                for (int j = 0; j < QK; j++) {
                    const i32 e = min(tid + j * NT, total - 1);
                    key[j] = j < nj ? C.beg[lo[j]] + (e - C.off[lo[j]]) : 0;
                }
#pragma unroll
                for (int j = 0; j < QK; j++) key[j] = j < nj ? g.ncol[key[j]] : -1;
#pragma unroll
                for (int j = 0; j < QK; j++)
                    if (tid + j * NT >= total) key[j] = -1;
                // where each key's count lives, so that the second sweep reads it
                // without a lookup; bit j of ownm: this thread created key j's count
                // (a dense counter's location is its key's offset, so it is not kept;
                // with a map the segments are read from it again rather than kept)
                int loc[QK];
                u32 ownm = 0;
#pragma unroll
                for (int j = 0; j < QK; j++) {
                    bool o = false;
                    const int l = key[j] >= 0 ? ctr.inc_at(key[j], o) : -1;
                    if constexpr (!Ctr::LOC_IS_KEY) loc[j] = l;
                    ownm |= (u32)o << j;
                }
                item_sync<NT>();
                // second sweep: each wedge's middle gains c - 1, summed over runs of
                // lanes in the same segment before the LDS atomic
#pragma unroll
                for (int j = 0; j < QK; j++) {
                    if (j < nj) {
                        int l;
                        if constexpr (Ctr::LOC_IS_KEY) l = key[j] >= 0 ? ctr.loc_of(key[j]) : -1;
                        else l = loc[j];
                        const int sj = MAP > 0 ? seg_at(C.seg, min(tid + j * NT, total - 1)) : lo[j];
                        const i32 c = l >= 0 ? ctr.at(l) : 0;
                        if constexpr (GMID) wave_run_add(Q, C.vv[sj], c > 1 ? c - 1 : 0);
                        else wave_run_add(C.mid, sj, c > 1 ? c - 1 : 0);
                    }
                }
                item_sync<NT>();
                i64 acc = 0;
#pragma unroll
                for (int j = 0; j < QK; j++) {
                    if ((ownm >> j) & 1u) {
                        int l;
                        if constexpr (Ctr::LOC_IS_KEY) l = ctr.loc_of(key[j]);
                        else l = loc[j];
                        const i64 c = ctr.take(l);
                        if (c >= 2) {
                            const i64 cc = c * (c - 1) / 2;
                            cr(key[j], cc);
                            acc += cc;
                        }
                    }
                }
                *local += acc;
                if constexpr (!GMID) {
                    for (int i = tid; i < ns; i += NT) {
                        i64 m = C.mid[i];
                        if (m) atomic_add_i64(&Q[C.vv[i]], m);
                    }
                }
                item_sync<NT>();
                return true;
            }
        }
    }
    for (int pass = 0; pass < 2; pass++) {
        for (i32 c0 = 0; c0 < ns; c0 += dc) {
            i32 len = min(dc, ns - c0);
            i32 total;
            // a single chunk stays loaded from the register-path check (loading it
            // again would race with waves still reading its total) and across passes
            if (!single || (pass == 0 && QK == 0)) {
                total = q_load_chunk<NT, MODE>(g, x, s0, sp, c0, len, C, tid, red32);
            } else {
                total = C.off[len];
            }
            total = wave_uniform(total);
            for (i32 eb = 0; eb < total; eb += NT * QS) {
                const int nj = min(QS, (total - eb + NT - 1) / NT);
                int si[QS];
                i32 key[QS];
                bool ok[QS];
                if constexpr (MAP > 0) {
                    // one map per block of NT*MQ wedges (the map's capacity), read by
                    // MQ/QS steps
                    constexpr int MQ = ((QK > QS ? QK : QS) / QS) * QS;  // whole steps
                    const i32 mb = eb - eb % (NT * MQ);
                    if (mb == eb) {
                        item_sync<NT>();  // the previous block's map has been read
                        if constexpr (MAP == 3) {
                            q_segmap<NT, MQ>(C.off, len, eb, total, tid, C.seg);
                            item_sync<NT>();
                        } else {
                            seg_map_scan<NT, MQ>(C.off, len, eb, total, tid, C.seg, red32);
                        }
                    }
#pragma unroll
                    for (int u = 0; u < QS; u++)
                        si[u] = u < nj ? seg_at(C.seg, min(eb + tid + u * NT, total - 1) - mb) : 0;
                } else {
                    q_locate<NT, QS>(C.off, len, eb + tid, nj, si, total - 1);
                }
#pragma unroll
                for (int u = 0; u < QS; u++) {
                    const i32 e = min(eb + tid + u * NT, total - 1);
                    ok[u] = u < nj && eb + tid + u * NT < total;
                    key[u] = u < nj ? C.beg[si[u]] + (e - C.off[si[u]]) : 0;
                }
#pragma unroll
                for (int u = 0; u < QS; u++) key[u] = u < nj ? g.ncol[key[u]] : 0;
#pragma unroll
                for (int u = 0; u < QS; u++) {
                    if (u >= nj) continue;
                    if (pass == 0) {
                        if (ok[u]) ctr.inc(key[u]);
                    } else {
                        const i32 c = ok[u] ? ctr.get(key[u]) : 0;
                        if constexpr (GMID) wave_run_add(Q, C.vv[si[u]], c > 1 ? c - 1 : 0);
                        else wave_run_add(C.mid, si[u], c > 1 ? c - 1 : 0);
                    }
                }
            }
            item_sync<NT>();
            if (pass == 1 && !GMID) {
                for (int i = tid; i < len; i += NT) {
                    i64 m = C.mid[i];
                    if (m) atomic_add_i64(&Q[C.vv[i]], m);
                }
                item_sync<NT>();
            }
        }
    }
    return false;
}


// Light items on one wave: an LDS hash (key, count) sized per item to twice its
// wedge count (at most hcw entries, given with the launch in dynamic LDS), harvested
// by scanning the item's part of the table.
struct LightHash {
    static constexpr bool LOC_IS_KEY = false;
    i32 *key;
    i32 *cnt;
    u32 mask;
    // counts k; returns its slot, own set when this call inserted the key
    __device__ int inc_at(i32 k, bool &own) const {
        u32 sl = hslot((u32)k, mask);
        own = false;
        while (true) {
            i32 cur = key[sl];
            if (cur == k) break;
            if (cur == -1) {
                i32 prev = atomicCAS(&key[sl], -1, k);
                if (prev == -1) {
                    own = true;
                    break;
                }
                if (prev == k) break;
            }
            sl = (sl + 1) & mask;
        }
        atomicAdd(&cnt[sl], 1);
        return (int)sl;
    }
    __device__ void inc(i32 k) const {
        bool own;
        inc_at(k, own);
    }
    __device__ i32 at(int sl) const { return cnt[sl]; }
    // count of an owned slot, which is emptied
    __device__ i32 take(int sl) const {
        const i32 c = cnt[sl];
        key[sl] = -1;
        cnt[sl] = 0;
        return c;
    }
    __device__ i32 get(i32 k) const {
        u32 sl = hslot((u32)k, mask);
        while (true) {
            i32 cur = key[sl];
            if (cur == k) return cnt[sl];
            if (cur == -1) return 0;
            sl = (sl + 1) & mask;
        }
    }
};

#define QLW_DC 64
#define QLW_QK 8
#define QLW_SEGB (QMAP_QLW ? WAVE * (QLW_QK > QS ? QLW_QK : QS) : 0)
#define QLW_MIDB (QGMID_QLW ? 0 : 8 * QLW_DC)
__host__ __device__ constexpr int qlw_wave_bytes(int hcw) {
    return ((QLW_MIDB + QLW_SEGB + 8 * hcw + 4 * (3 * QLW_DC + 1)) + 15) / 16 * 16;
}

template <int MODE>
__global__ void __launch_bounds__(256) k_q_wave(DevGraph g, const i32 *__restrict__ list,
                                                const GraphStats *__restrict__ st, int wc, i64 *Q, int hcw) {
    extern __shared__ __align__(16) char s_dyn[];
    const int w = threadIdx.x / WAVE, tid = lane_id();
    char *base = s_dyn + (size_t)w * qlw_wave_bytes(hcw);
    i64 *s_mid = QGMID_QLW ? nullptr : (i64 *)base;
    u32 *s_seg = (u32 *)(base + QLW_MIDB);
    i32 *s_key = (i32 *)(base + QLW_MIDB + QLW_SEGB);
    i32 *s_cnt = s_key + hcw;
    i32 *s_off = s_cnt + hcw;
    i32 *s_vv = s_off + QLW_DC + 1;
    i32 *s_beg = s_vv + QLW_DC;
    for (int i = tid; i < hcw; i += WAVE) {
        s_key[i] = -1;
        s_cnt[i] = 0;
    }
    item_sync<WAVE>();
    QChunk C{s_off, s_vv, s_beg, s_mid, s_seg};
    const i32 cnt = st->cnt[wc];
    const int waves = gridDim.x * 4;
    i32 it = blockIdx.x * 4 + w;
    QMeta cur = q_meta<MODE>(g, it < cnt ? list[it] : -1);
    i32 xn = it + waves < cnt ? list[it + waves] : -1;
    for (; it < cnt; it += waves) {
        // the next item's row bounds and the one after's id load while this one runs
        const QMeta nxt = q_meta<MODE>(g, xn);
        xn = it + 2 * waves < cnt ? list[it + 2 * waves] : -1;
        const i64 need = 2 * cur.w;
        const int hc = need >= hcw ? hcw : (need <= 64 ? 64 : (int)(1u << (32 - __clz((u32)(need - 1)))));
        LightHash H{s_key, s_cnt, (u32)hc - 1};
        i64 local = 0;
        const bool taken =
            q_sweeps<WAVE, MODE, QLW_QK, QMAP_QLW, QGMID_QLW>(g, cur, H, C, QLW_DC, tid, nullptr, Q, CreditLight{Q},
                                                              &local);
        for (int j = tid; !taken && j < hc; j += WAVE) {
            const i32 k = s_key[j];
            if (k >= 0) {
                const i64 c = s_cnt[j];
                if (c >= 2) {
                    const i64 cc = c * (c - 1) / 2;
                    atomic_add_i64(&Q[k], cc);
                    local += cc;
                }
                s_key[j] = -1;
                s_cnt[j] = 0;
            }
        }
        local = wave_sum64(local);
        if (tid == 0 && local) atomic_add_i64(&Q[cur.x], local);
        item_sync<WAVE>();
        cur = nxt;
    }
}

// Light items on one 256-thread workgroup: the same hash as the wave class, sized
// per item, at most hcb entries (dynamic LDS given with the launch).
#define QLB_DC 256
#define QLB_NT 256
#define QLB_QK 16
#define QLB_SEGB (QMAP_QLB ? QLB_NT * (QLB_QK > QS ? QLB_QK : QS) : 0)
#define QLB_MIDB (QGMID_QLB ? 0 : 8 * QLB_DC)
__host__ __device__ constexpr int qlb_bytes(int hcb) {
    return ((QLB_MIDB + QLB_SEGB + 8 * hcb + 4 * (3 * QLB_DC + 1)) + 15) / 16 * 16;
}

// Items of the list with wlo < wedges <= whi only (the class is split into two
// launches with different table sizes, so that small items keep a high occupancy).
template <int MODE>
__global__ void __launch_bounds__(QLB_NT) k_q_block(DevGraph g, const i32 *__restrict__ list,
                                                    const GraphStats *__restrict__ st, int wc, i64 *Q, int hcb,
                                                    i64 wlo, i64 whi) {
    extern __shared__ __align__(16) char s_dyn[];
    __shared__ i64 s_red[QLB_NT / WAVE];
    __shared__ i32 s_red32[QLB_NT / WAVE];
    i64 *s_mid = QGMID_QLB ? nullptr : (i64 *)s_dyn;
    u32 *s_seg = (u32 *)(s_dyn + QLB_MIDB);
    i32 *s_key = (i32 *)(s_dyn + QLB_MIDB + QLB_SEGB);
    i32 *s_cnt = s_key + hcb;
    i32 *s_off = s_cnt + hcb;
    i32 *s_vv = s_off + QLB_DC + 1;
    i32 *s_beg = s_vv + QLB_DC;
    for (int i = threadIdx.x; i < hcb; i += QLB_NT) {
        s_key[i] = -1;
        s_cnt[i] = 0;
    }
    __syncthreads();
    QChunk C{s_off, s_vv, s_beg, s_mid, s_seg};
    const i32 cnt = st->cnt[wc];
    i32 it = blockIdx.x;
    QMeta cur = q_meta<MODE>(g, it < cnt ? list[it] : -1);
    i32 xn = it + (i32)gridDim.x < cnt ? list[it + gridDim.x] : -1;
    for (; it < cnt; it += gridDim.x) {
        const QMeta nxt = q_meta<MODE>(g, xn);
        xn = it + 2 * (i32)gridDim.x < cnt ? list[it + 2 * gridDim.x] : -1;
        if (cur.w <= wlo || cur.w > whi) {
            cur = nxt;
            continue;
        }
        const i64 need = 2 * cur.w;
        const int hc = need >= hcb ? hcb : (need <= 64 ? 64 : (int)(1u << (32 - __clz((u32)(need - 1)))));
        LightHash H{s_key, s_cnt, (u32)hc - 1};
        i64 local = 0;
        const bool taken =
            q_sweeps<QLB_NT, MODE, QLB_QK, QMAP_QLB, QGMID_QLB>(g, cur, H, C, QLB_DC, threadIdx.x, s_red32, Q,
                                                                CreditLight{Q}, &local);
        for (int j = threadIdx.x; !taken && j < hc; j += QLB_NT) {
            const i32 k = s_key[j];
            if (k >= 0) {
                const i64 c = s_cnt[j];
                if (c >= 2) {
                    const i64 cc = c * (c - 1) / 2;
                    atomic_add_i64(&Q[k], cc);
                    local += cc;
                }
                s_key[j] = -1;
                s_cnt[j] = 0;
            }
        }
        local = item_sum<QLB_NT>(local, s_red, threadIdx.x);
        if (threadIdx.x == 0 && local) atomic_add_i64(&Q[cur.x], local);
        __syncthreads();
        cur = nxt;
    }
}

// ---------------------------------------------------------------------------
// Heavy largest vertices (keys u in [h0, n), at most QH_DENSE_K of them).
// Credits C(c,2) to a heavy key go to one of QH_PART_ROWS rows of `part`
// (int64[QH_PART_ROWS][K]), summed into Q by k_qh_reduce: every opposite vertex
// credits the same few thousand hubs, and one shared counter per hub would
// serialise those updates.  Workgroups are dealt to the 8 XCDs round robin, so
// row = blockIdx % QH_PART_ROWS keeps each XCD on its own 8 rows (2 MiB for
// K = 32768), which stay in that XCD's L2.
// ---------------------------------------------------------------------------
#define PK_SHIFT 17
#define PK_CMASK 0x1ffffu
#define PK_EMPTY 0xffffffffu

// Hash of (key index, count) packed in one 32-bit word: idx << 17 | count.
struct PackedHash {
    static constexpr bool LOC_IS_KEY = false;
    u32 *tab;
    u32 mask;
    i32 h0;
    // counts k; returns its slot, own set when this call inserted the key
    __device__ int inc_at(i32 k, bool &own) const {
        const u32 idx = (u32)(k - h0);
        u32 sl = hslot(idx, mask);
        own = false;
        while (true) {
            u32 cur = tab[sl];
            if (cur == PK_EMPTY) {
                u32 prev = atomicCAS(&tab[sl], PK_EMPTY, (idx << PK_SHIFT) | 1u);
                if (prev == PK_EMPTY) {
                    own = true;
                    return (int)sl;
                }
                cur = prev;
            }
            if ((cur >> PK_SHIFT) == idx) {
                atomicAdd(&tab[sl], 1u);
                return (int)sl;
            }
            sl = (sl + 1) & mask;
        }
    }
    __device__ void inc(i32 k) const {
        bool own;
        inc_at(k, own);
    }
    __device__ i32 at(int sl) const { return (i32)(tab[sl] & PK_CMASK); }
    // count of an owned slot, which is emptied
    __device__ i32 take(int sl) const {
        const u32 cur = tab[sl];
        tab[sl] = PK_EMPTY;
        return (i32)(cur & PK_CMASK);
    }
    __device__ i32 get(i32 k) const {
        const u32 idx = (u32)(k - h0);
        u32 sl = hslot(idx, mask);
        while (true) {
            u32 cur = tab[sl];
            if (cur == PK_EMPTY) return 0;
            if ((cur >> PK_SHIFT) == idx) return (i32)(cur & PK_CMASK);
            sl = (sl + 1) & mask;
        }
    }
};

template <int NT, int QK, int MAP, bool GMID>
__device__ __forceinline__ void qh_item_packed(const DevGraph &g, const QMeta &mt, const PackedHash &H0, int hc_max,
                                               const QChunk &C, int dc, int tid, i64 *red, i32 *red32,
                                               i64 *__restrict__ Q, i64 *__restrict__ prow) {
    const i32 x = mt.x;
    // the table used is the smallest power of two holding twice the item's wedges
    // (at least 64, at most hc_max)
    const i64 need = 2 * mt.w;
    const int hc = need >= hc_max ? hc_max : (need <= 64 ? 64 : (int)(1u << (32 - __clz((u32)(need - 1)))));
    PackedHash H{H0.tab, (u32)hc - 1, H0.h0};
    i64 local = 0;
    const bool taken =
        q_sweeps<NT, Q_HEAVY, QK, MAP, GMID>(g, mt, H, C, dc, tid, red32, Q, CreditHeavy{prow, H0.h0}, &local);
    for (int j = tid; !taken && j < hc; j += NT) {
        u32 cur = H.tab[j];
        if (cur != PK_EMPTY) {
            i64 c = cur & PK_CMASK;
            if (c >= 2) {
                i64 cc = c * (c - 1) / 2;
                atomic_add_i64(&prow[cur >> PK_SHIFT], cc);
                local += cc;
            }
            H.tab[j] = PK_EMPTY;
        }
    }
    i64 s = item_sum<NT>(local, red, tid);
    if (tid == 0 && s) atomic_add_i64(&Q[x], s);
    item_sync<NT>();
}

// One wave per item; the per-wave table size hcw (a power of two, at least twice
// the class's wedge bound) comes with the launch, in dynamic LDS.
#define QHW_DC 64
#define QHW_QK 8  // wedges per lane in registers: 512, the class's default bound
#define QHW_WPE 6  // waves per SIMD the heavy wave kernel is compiled for (80 registers)
#define QHW_GRID 6  // workgroups per CU (the class's grid is given per 4): all resident
#define QHW_SEGB (QMAP_QHW ? WAVE * (QHW_QK > QS ? QHW_QK : QS) : 0)
#define QHW_MIDB (QGMID_QHW ? 0 : 8 * QHW_DC)
__host__ __device__ constexpr int qhw_wave_bytes(int hcw) {
    return ((QHW_MIDB + QHW_SEGB + 4 * hcw + 4 * (3 * QHW_DC + 1)) + 15) / 16 * 16;
}
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(QHW_WPE))) k_qh_wave(DevGraph g, const i32 *__restrict__ list,
                                                 const GraphStats *__restrict__ st, i64 *Q, i64 *part, i32 K,
                                                 int hcw) {
    extern __shared__ __align__(16) char s_dyn[];
    const int w = threadIdx.x / WAVE, tid = lane_id();
    char *base = s_dyn + (size_t)w * qhw_wave_bytes(hcw);
    i64 *s_mid = QGMID_QHW ? nullptr : (i64 *)base;
    u32 *s_seg = (u32 *)(base + QHW_MIDB);
    u32 *s_tab = (u32 *)(base + QHW_MIDB + QHW_SEGB);
    i32 *s_off = (i32 *)(s_tab + hcw);
    i32 *s_vv = s_off + QHW_DC + 1;
    i32 *s_beg = s_vv + QHW_DC;
    for (int i = tid; i < hcw; i += WAVE) s_tab[i] = PK_EMPTY;
    item_sync<WAVE>();
    PackedHash H{s_tab, (u32)hcw - 1, g.h0};
    QChunk C{s_off, s_vv, s_beg, s_mid, s_seg};
    i64 *prow = part + (i64)(blockIdx.x % QH_PART_ROWS) * K;
    const i32 cnt = st->cnt[WC_QH_WAVE];
    const int waves = gridDim.x * 4;
    i32 it = blockIdx.x * 4 + w;
    QMeta cur = q_meta<Q_HEAVY>(g, it < cnt ? list[it] : -1);
    i32 xn = it + waves < cnt ? list[it + waves] : -1;
    for (; it < cnt; it += waves) {
        const QMeta nxt = q_meta<Q_HEAVY>(g, xn);
        xn = it + 2 * waves < cnt ? list[it + 2 * waves] : -1;
        qh_item_packed<WAVE, QHW_QK, QMAP_QHW, QGMID_QHW>(g, cur, H, hcw, C, QHW_DC, tid, nullptr, nullptr, Q, prow);
        cur = nxt;
    }
}

#define QHB_HC QH_BLOCK_HC
#define QHB_DC 256
#define QHB_QK 8  // wedges per thread kept in registers by the heavy workgroup kernel
                  // (2048, the class's default bound; 76 registers: six waves per SIMD)
#define QHB_NT 256
#define QHB_WPE 1
#define QHB_GRID 6  // workgroups per CU (the class's grid is given per 4): all resident
// The table (hcb entries, a power of two at least twice the class's wedge bound)
// comes with the launch in dynamic LDS.
__global__ void __launch_bounds__(QHB_NT) __attribute__((amdgpu_waves_per_eu(QHB_WPE)))
k_qh_block(DevGraph g, const i32 *__restrict__ list, const GraphStats *__restrict__ st, i64 *Q, i64 *part, i32 K,
           int hcb) {
    extern __shared__ __align__(16) char s_dyn[];
    u32 *s_tab = (u32 *)s_dyn;
    __shared__ u32 s_seg[QMAP_QHB ? QHB_NT * (QHB_QK > QS ? QHB_QK : QS) / 4 : 1];
    __shared__ i32 s_off[QHB_DC + 1];
    __shared__ i32 s_vv[QHB_DC];
    __shared__ i32 s_beg[QHB_DC];
    __shared__ i64 s_mid[QGMID_QHB ? 1 : QHB_DC];
    __shared__ i64 s_red[QHB_NT / WAVE];
    __shared__ i32 s_red32[QHB_NT / WAVE];
    for (int i = threadIdx.x; i < hcb; i += QHB_NT) s_tab[i] = PK_EMPTY;
    __syncthreads();
    PackedHash H{s_tab, (u32)hcb - 1, g.h0};
    QChunk C{s_off, s_vv, s_beg, QGMID_QHB ? nullptr : s_mid, s_seg};
    i64 *prow = part + (i64)(blockIdx.x % QH_PART_ROWS) * K;
    const i32 cnt = st->cnt[WC_QH_BLOCK];
    i32 it = blockIdx.x;
    QMeta cur = q_meta<Q_HEAVY>(g, it < cnt ? list[it] : -1);
    i32 xn = it + (i32)gridDim.x < cnt ? list[it + gridDim.x] : -1;
    for (; it < cnt; it += gridDim.x) {
        const QMeta nxt = q_meta<Q_HEAVY>(g, xn);
        xn = it + 2 * (i32)gridDim.x < cnt ? list[it + 2 * gridDim.x] : -1;
        qh_item_packed<QHB_NT, QHB_QK, QMAP_QHB, QGMID_QHB>(g, cur, H, hcb, C, QHB_DC, threadIdx.x,
                                                                         s_red, s_red32, Q, prow);
        cur = nxt;
    }
}

// part rows -> Q over the heavy range
__global__ void k_qh_reduce(const i64 *__restrict__ part, int rows, i32 K, i32 h0, i64 *__restrict__ Q) {
    i32 i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= K) return;
    i64 s = 0;
    for (int r = 0; r < rows; r++) s += part[(i64)r * K + i];
    if (s) Q[h0 + i] += s;
}

// Heavy largest vertices: dense 16-bit counters over [h0, n).
#define QD_NT 1024  // 16 waves per workgroup, two workgroups per CU (LDS)
#define QD_QK 8  // wedges per thread kept in registers by the dense kernel
#define QD_DC 256
#define QD_WPE 8  // 64 registers: eight waves per SIMD
__global__ void __launch_bounds__(QD_NT) __attribute__((amdgpu_waves_per_eu(QD_WPE))) k_q_dense(DevGraph g, const i32 *__restrict__ list,
                                                   const GraphStats *__restrict__ st, i64 *Q, i64 *part, i32 Kp) {
    __shared__ u32 s_w[QH_DENSE_K / 2];
    __shared__ u32 s_seg[QMAP_QD ? QD_NT * (QD_QK > QS ? QD_QK : QS) / 4 : 1];
    __shared__ i32 s_off[QD_DC + 1];
    __shared__ i32 s_vv[QD_DC];
    __shared__ i32 s_beg[QD_DC];
    __shared__ i64 s_mid[QD_DC];
    __shared__ i64 s_red[QD_NT / WAVE];
    __shared__ i32 s_red32[QD_NT / WAVE];
    const i32 K = g.n - g.h0;
    const i32 KW = (K + 1) >> 1;
    for (int i = threadIdx.x; i < KW; i += QD_NT) s_w[i] = 0u;
    __syncthreads();
    DenseCounter ctr{s_w, g.h0};
    QChunk C{s_off, s_vv, s_beg, s_mid, s_seg};
    i64 *prow = part + (i64)(blockIdx.x % QH_PART_ROWS) * Kp;
    const i32 cnt = st->cnt[WC_QH_DENSE];
    for (i32 it = blockIdx.x; it < cnt; it += gridDim.x) {
        i32 x = list[it];
        i64 local = 0;
        const bool taken = q_sweeps<QD_NT, Q_HEAVY, QD_QK, QMAP_QD>(g, q_meta<Q_HEAVY>(g, x), ctr, C, QD_DC,
                                                                     threadIdx.x, s_red32, Q,
                                                                     CreditHeavy{prow, g.h0}, &local);
        for (i32 i = threadIdx.x; !taken && i < KW; i += QD_NT) {
            u32 word = s_w[i];
            if (word) {
                i64 c0 = word & 0xffffu, c1 = word >> 16;
                if (c0 >= 2) {
                    i64 cc = c0 * (c0 - 1) / 2;
                    atomic_add_i64(&prow[2 * i], cc);
                    local += cc;
                }
                if (c1 >= 2) {
                    i64 cc = c1 * (c1 - 1) / 2;
                    atomic_add_i64(&prow[2 * i + 1], cc);
                    local += cc;
                }
                s_w[i] = 0u;
            }
        }
        i64 s = item_sum<QD_NT>(local, s_red, threadIdx.x);
        if (threadIdx.x == 0 && s) atomic_add_i64(&Q[x], s);
        __syncthreads();
    }
}

// Light largest vertices whose wedges overflow the LDS hash: int32 counters over
// [0, n) in per-workgroup global scratch, touched keys listed for clearing.
#define QG_NT 1024  // one workgroup per CU (a counter slice each): sixteen waves to hide the atomics' latency
#define QG_DC 1024
template <int MODE>
__global__ void __launch_bounds__(QG_NT) k_q_global(DevGraph g, const i32 *__restrict__ list,
                                                    const GraphStats *__restrict__ st, int wc, i64 *Q,
                                                    i32 *scratch, i64 slice_elems) {
    __shared__ i32 s_off[QG_DC + 1];
    __shared__ i32 s_vv[QG_DC];
    __shared__ i32 s_beg[QG_DC];
    __shared__ i64 s_mid[QG_DC];
    __shared__ i64 s_red[QG_NT / WAVE];
    __shared__ i32 s_red32[QG_NT / WAVE];
    __shared__ i32 s_nused;
    i32 *cnt_arr = scratch + (i64)blockIdx.x * slice_elems;
    i32 *used = cnt_arr + g.n;
    if (threadIdx.x == 0) s_nused = 0;
    __syncthreads();
    GlobalCounter ctr{cnt_arr, used, &s_nused};
    QChunk C{s_off, s_vv, s_beg, s_mid};
    const i32 cnt = st->cnt[wc];
    for (i32 it = blockIdx.x; it < cnt; it += gridDim.x) {
        i32 x = list[it];
        i64 unused = 0;
        q_sweeps<QG_NT, MODE>(g, q_meta<MODE>(g, x), ctr, C, QG_DC, threadIdx.x, s_red32, Q, CreditLight{Q}, &unused);
        __threadfence_block();
        const i32 nu = s_nused;
        i64 local = 0;
        for (i32 j = threadIdx.x; j < nu; j += QG_NT) {
            i32 k = used[j];
            i64 c = cnt_arr[k];
            if (c >= 2) {
                i64 cc = c * (c - 1) / 2;
                atomic_add_i64(&Q[k], cc);
                local += cc;
            }
            cnt_arr[k] = 0;
        }
        i64 s = item_sum<QG_NT>(local, s_red, threadIdx.x);
        if (threadIdx.x == 0) {
            if (s) atomic_add_i64(&Q[x], s);
            s_nused = 0;
        }
        __threadfence_block();
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Host-side launch helpers (called from the API file).
// ---------------------------------------------------------------------------
hipError_t launch_classify(const DevGraph &g, const i64 *wl, const i64 *wh, const i64 *probes, const ListPtrs &lists,
                           GraphStats *st, const Thresholds &th, hipStream_t s) {
    if (g.n == 0) return hipSuccess;
    const i32 tiles = (g.n + CL_NT * CL_PER_THREAD - 1) / (CL_NT * CL_PER_THREAD);
    hipLaunchKernelGGL(k_classify, dim3(tiles < 2048 ? tiles : 2048), dim3(CL_NT), 0, s, g, wl, wh, probes, lists, st,
                       th);
    return hipGetLastError();
}

template <int MODE>
static void launch_large(const DevGraph &g, const i32 *list, const GraphStats *st, i32 *t, i64 *K4, i64 *tau,
                         const TriCache &tc, char *scratch, i64 slice, int cap, int hc, int blocks, i64 lds_max,
                         i64 *counters, hipStream_t s) {
    const i64 k4 = probe_large_k4_bytes(cap, hc), lds = probe_large_lds_bytes(cap, hc);
    if (k4 <= lds_max)  // one workgroup per CU fits: launch no more than that
        hipLaunchKernelGGL((k_probe_large<MODE, 2>), dim3((blocks + 1) / 2), dim3(PL_NT), (size_t)k4, s, g, list, st,
                           t, K4,
                           tau, tc, scratch, slice, cap, hc, counters);
    else if (lds <= lds_max)
        hipLaunchKernelGGL((k_probe_large<MODE, 1>), dim3(blocks), dim3(PL_NT), (size_t)lds, s, g, list, st, t, K4,
                           tau, tc, scratch, slice, cap, hc, counters);
    else
        hipLaunchKernelGGL((k_probe_large<MODE, 0>), dim3(blocks), dim3(PL_NT), 0, s, g, list, st, t, K4, tau, tc,
                           scratch, slice, cap, hc, counters);
}

hipError_t launch_probe(int mode, const DevGraph &g, i32 *const *lists_host, const GraphStats *st, i32 *t,
                        i64 *K4, i64 *tau, const TriCacheArgs &tca, char *large_scratch, i64 large_slice,
                        int large_cap, int large_hc, int large_blocks, i64 large_lds_max, int grid_wave,
                        int grid_block, i64 *counters, const KernelEvents &kev, hipStream_t s) {
#define KMARK(i) \
    if (kev.ev) (void)hipEventRecord(kev.ev[i], s)
    TriCache tw{tca.rec, tca.cap, tca.bump, tca.off, tca.cnt, tca.chunk_wave};
    TriCache tb{tca.rec, tca.cap, tca.bump, tca.off, tca.cnt, tca.chunk_block};
    TriCache tg{tca.rec, tca.cap, tca.bump, tca.off, tca.cnt, tca.chunk_group};
    if (mode == PROBE_EK4) {
        // Stage I/II with per-edge 4-cliques into `tau` (an int64 per slot)
        hipLaunchKernelGGL(k_probe_thread<PROBE_EK4>, dim3(grid_wave), dim3(256), 0, s, g,
                           lists_host[WC_TRI_THREAD], st, t, K4, tau, tw, (i64 *)nullptr);
        hipLaunchKernelGGL(k_probe_wave<PROBE_EK4>, dim3(grid_wave), dim3(256), 0, s, g, lists_host[WC_TRI_WAVE], st,
                           t, K4, tau, tw, (i64 *)nullptr);
        hipLaunchKernelGGL(k_probe_block<PROBE_EK4>, dim3(grid_block), dim3(PB_NT), 0, s, g,
                           lists_host[WC_TRI_BLOCK], st, t, K4, tau, tb, (i64 *)nullptr);
        if (large_blocks > 0)
            launch_large<PROBE_EK4>(g, lists_host[WC_TRI_LARGE], st, t, K4, tau, tb, large_scratch, large_slice,
                                    large_cap, large_hc, large_blocks, large_lds_max, (i64 *)nullptr, s);
        hipLaunchKernelGGL(k_probe_group<PROBE_EK4>, dim3(grid_wave), dim3(256), 0, s, g,
                           lists_host[WC_TRI_GROUP], st, t, K4, tau, tg, (i64 *)nullptr);
    } else if (mode == PROBE_TRI) {
        KMARK(0);
        hipLaunchKernelGGL(k_probe_thread<PROBE_TRI>, dim3(grid_wave), dim3(256), 0, s, g,
                           lists_host[WC_TRI_THREAD], st, t, K4, tau, tw, counters);
        KMARK(1);
        hipLaunchKernelGGL(k_probe_wave<PROBE_TRI>, dim3(grid_wave), dim3(256), 0, s, g, lists_host[WC_TRI_WAVE], st,
                           t, K4, tau, tw, counters);
        KMARK(2);
        hipLaunchKernelGGL(k_probe_block<PROBE_TRI>, dim3(grid_block), dim3(PB_NT), 0, s, g,
                           lists_host[WC_TRI_BLOCK], st, t, K4, tau, tb, counters);
        KMARK(3);
        if (large_blocks > 0)
            launch_large<PROBE_TRI>(g, lists_host[WC_TRI_LARGE], st, t, K4, tau, tb, large_scratch, large_slice,
                                 large_cap, large_hc, large_blocks, large_lds_max, counters, s);
        KMARK(4);
        KMARK(13);
        hipLaunchKernelGGL(k_probe_group<PROBE_TRI>, dim3(grid_wave), dim3(256), 0, s, g,
                           lists_host[WC_TRI_GROUP], st, t, K4, tau, tg, counters);
        KMARK(14);
    } else {
        hipLaunchKernelGGL(k_probe_group<PROBE_TAU>, dim3(grid_wave), dim3(256), 0, s, g,
                           lists_host[WC_TRI_GROUP], st, t, K4, tau, tg, (i64 *)nullptr);
        hipLaunchKernelGGL(k_probe_thread<PROBE_TAU>, dim3(grid_wave), dim3(256), 0, s, g,
                           lists_host[WC_TRI_THREAD], st, t, K4, tau, tw, (i64 *)nullptr);
        hipLaunchKernelGGL(k_probe_wave<PROBE_TAU>, dim3(grid_wave), dim3(256), 0, s, g, lists_host[WC_TRI_WAVE], st,
                           t, K4, tau, tw, (i64 *)nullptr);
        hipLaunchKernelGGL(k_probe_block<PROBE_TAU>, dim3(grid_block), dim3(PB_NT), 0, s, g,
                           lists_host[WC_TRI_BLOCK], st, t, K4, tau, tb, (i64 *)nullptr);
        if (large_blocks > 0)
            launch_large<PROBE_TAU>(g, lists_host[WC_TRI_LARGE], st, t, K4, tau, tb, large_scratch, large_slice,
                                 large_cap, large_hc, large_blocks, large_lds_max, (i64 *)nullptr, s);
    }
    return hipGetLastError();
}

hipError_t launch_sums(const DevGraph &g, const i32 *t, const Accum &acc, int grid, hipStream_t s) {
    if (g.n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_sums, dim3(grid), dim3(256), 0, s, g, t, acc);
    return hipGetLastError();
}

hipError_t launch_solve(const DevGraph &g, const Accum &acc, i64 *out, i64 *fvars, GraphStats *st, int grid,
                        bool induced, hipStream_t s) {
    if (g.n == 0) return hipSuccess;
    if (induced)
        hipLaunchKernelGGL(k_solve<true>, dim3(grid), dim3(256), 0, s, g, acc, out, fvars, st);
    else
        hipLaunchKernelGGL(k_solve<false>, dim3(grid), dim3(256), 0, s, g, acc, out, fvars, st);
    return hipGetLastError();
}

hipError_t launch_q(const DevGraph &g, i32 *const *lists_host, const GraphStats *st, i64 *Q, i32 *gscratch,
                    i64 gslice, int gblocks, int grid_wave, int grid_block, int grid_dense, i64 *part, int part_rows,
                    i64 ql_wave_bound, i64 ql_block_bound, i64 ql_split, i64 qh_wave_bound, i64 qh_block_bound,
                    const KernelEvents &kev, hipStream_t s) {
    KMARK(5);
    {
        int hcw = 64;
        while ((i64)hcw < 2 * ql_wave_bound) hcw <<= 1;
        hipLaunchKernelGGL(k_q_wave<Q_LIGHT>, dim3(grid_wave), dim3(256), 4 * qlw_wave_bytes(hcw), s, g,
                           lists_host[WC_QL_WAVE], st, (int)WC_QL_WAVE, Q, hcw);
    }
    KMARK(6);
    {
        // one launch per window of wedge counts (ql_wave, ql_split], then doubling up to
        // ql_block, each with tables for its window only: small items keep many
        // workgroups per CU, large ones get the LDS they need
        auto table_for = [](i64 w) {
            int h = 64;
            while ((i64)h < 2 * w) h <<= 1;
            return h;
        };
        i64 lo = -1, hi = ql_split < ql_block_bound ? ql_split : ql_block_bound;
        if (hi <= 0) hi = ql_block_bound;
        while (lo < ql_block_bound && hi > 0) {
            const int hcb = table_for(hi);
            hipLaunchKernelGGL(k_q_block<Q_LIGHT>, dim3(grid_block), dim3(QLB_NT), qlb_bytes(hcb), s, g,
                               lists_host[WC_QL_BLOCK], st, (int)WC_QL_BLOCK, Q, hcb, lo, hi);
            lo = hi;
            hi = 2 * hi < ql_block_bound ? 2 * hi : ql_block_bound;
        }
    }
    KMARK(7);
    if (gblocks > 0)
        hipLaunchKernelGGL(k_q_global<Q_LIGHT>, dim3(gblocks), dim3(QG_NT), 0, s, g, lists_host[WC_QL_GLOBAL], st,
                           (int)WC_QL_GLOBAL, Q, gscratch, gslice);
    KMARK(8);
    const i32 K = g.n - g.h0;
    if (K > 0) {
        (void)part_rows;
        int hcw = 64;
        while ((i64)hcw < 2 * qh_wave_bound) hcw <<= 1;
        hipLaunchKernelGGL(k_qh_wave, dim3(grid_wave / 4 * QHW_GRID), dim3(256), 4 * qhw_wave_bytes(hcw), s, g,
                           lists_host[WC_QH_WAVE], st, Q, part, K, hcw);
        KMARK(9);
        int hcb = 64;
        while ((i64)hcb < 2 * qh_block_bound && hcb < QHB_HC) hcb <<= 1;
        hipLaunchKernelGGL(k_qh_block, dim3(grid_block / 4 * QHB_GRID), dim3(QHB_NT), (size_t)hcb * sizeof(u32), s, g,
                           lists_host[WC_QH_BLOCK], st, Q, part, K, hcb);
        KMARK(10);
        hipLaunchKernelGGL(k_q_dense, dim3(grid_dense), dim3(QD_NT), 0, s, g, lists_host[WC_QH_DENSE], st, Q, part,
                           K);
        KMARK(11);
        hipLaunchKernelGGL(k_qh_reduce, dim3((K + 255) / 256), dim3(256), 0, s, part, part_rows, K, g.h0, Q);
    } else {
        KMARK(9);
        KMARK(10);
        KMARK(11);
    }
    if (gblocks > 0)
        hipLaunchKernelGGL(k_q_global<Q_HEAVY>, dim3(gblocks), dim3(QG_NT), 0, s, g, lists_host[WC_QH_GLOBAL], st,
                           (int)WC_QH_GLOBAL, Q, gscratch, gslice);
    KMARK(12);
    return hipGetLastError();
}

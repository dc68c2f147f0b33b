// Host side of the C ABI declared in include/niorca.h: argument checks, the
// device workspace, and the order of the stages on the caller's stream.
#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/niorca.h"
#include "kernels.hpp"

struct niorca_ctx {
    int device = 0;
    int num_cu = 256;
    char *ws = nullptr;
    uint64_t ws_bytes = 0;
    uint64_t ws_limit = 0;
    std::string err;
    // cost model for NIORCA_BIN_MLP (host copy)
    std::vector<float> mlp;
    float thr_wave = 0.f, thr_block = 0.f;
    // work counters of the last counted graph
    int32_t counters_n = -1;
    bool counters_valid = false;
    GraphStats last{};
    // per-stage HIP events of the last call made with NIORCA_TIMING
    hipEvent_t ev[NIORCA_NUM_STAGES + 1] = {};
    bool ev_made = false;
    bool ev_valid = false;
    // tunable class thresholds and the size of the heavy 4-cycle key range
    Thresholds th{TRI_WAVE_CAP, TRI_BLOCK_CAP, QL_WAVE_HC / 2, QL_BLOCK_HC / 2, QH_WAVE_HC / 2, QH_BLOCK_HC / 2};
    int32_t heavy_k = QH_DENSE_K;
    int64_t tri_cache_records = (int64_t)1 << 29;  // 4 GiB of kept triangles for the tau pass
};

static niorca_status fail(niorca_ctx *c, niorca_status s, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (c) c->err = buf;
    return s;
}

#define HIP_TRY(expr)                                                                        \
    do {                                                                                     \
        hipError_t e_ = (expr);                                                              \
        if (e_ != hipSuccess)                                                                \
            return fail(ctx, NIORCA_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

// Bump allocator over the context workspace.
struct Arena {
    uint64_t off = 0;
    template <typename T>
    uint64_t take(uint64_t count) {
        uint64_t o = off;
        off += (sizeof(T) * count + 255) & ~255ull;
        return o;
    }
};

static niorca_status ensure_ws(niorca_ctx *ctx, uint64_t bytes) {
    if (bytes <= ctx->ws_bytes) return NIORCA_OK;
    if (ctx->ws_limit && bytes > ctx->ws_limit)
        return fail(ctx, NIORCA_ENOMEM, "workspace of %llu bytes exceeds the cap of %llu",
                    (unsigned long long)bytes, (unsigned long long)ctx->ws_limit);
    if (ctx->ws) {
        (void)hipDeviceSynchronize();
        (void)hipFree(ctx->ws);
        ctx->ws = nullptr;
        ctx->ws_bytes = 0;
    }
    uint64_t want = bytes + bytes / 8;
    if (ctx->ws_limit && want > ctx->ws_limit) want = bytes;
    if (hipMalloc((void **)&ctx->ws, want) != hipSuccess) {
        (void)hipGetLastError();
        return fail(ctx, NIORCA_ENOMEM, "hipMalloc of %llu bytes failed", (unsigned long long)want);
    }
    ctx->ws_bytes = want;
    return NIORCA_OK;
}

extern "C" niorca_status niorca_create(niorca_ctx **out, int device) {
    if (!out) return NIORCA_EINVAL;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return NIORCA_EDEVICE;
    if (hipSetDevice(device) != hipSuccess) return NIORCA_EDEVICE;
    niorca_ctx *c = new niorca_ctx();
    c->device = device;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) == hipSuccess && prop.multiProcessorCount > 0)
        c->num_cu = prop.multiProcessorCount;
    *out = c;
    return NIORCA_OK;
}

extern "C" void niorca_destroy(niorca_ctx *ctx) {
    if (!ctx) return;
    if (ctx->ev_made)
        for (auto &e : ctx->ev) (void)hipEventDestroy(e);
    if (ctx->ws) {
        (void)hipSetDevice(ctx->device);
        (void)hipDeviceSynchronize();
        (void)hipFree(ctx->ws);
    }
    delete ctx;
}

extern "C" const char *niorca_last_error(const niorca_ctx *ctx) { return ctx ? ctx->err.c_str() : ""; }

extern "C" niorca_status niorca_set_workspace_limit(niorca_ctx *ctx, uint64_t bytes) {
    if (!ctx) return NIORCA_EINVAL;
    ctx->ws_limit = bytes;
    return NIORCA_OK;
}

extern "C" uint64_t niorca_workspace_bytes(const niorca_ctx *ctx) { return ctx ? ctx->ws_bytes : 0; }

extern "C" niorca_status niorca_set_param(niorca_ctx *ctx, const char *name, int64_t value) {
    if (!ctx || !name) return NIORCA_EINVAL;
    std::string k(name);
    auto bad = [&](int64_t lo, int64_t hi) {
        return fail(ctx, NIORCA_EINVAL, "parameter %s = %lld outside [%lld, %lld]", name, (long long)value,
                    (long long)lo, (long long)hi);
    };
    if (k == "heavy_k") {
        if (value < 0 || value > QH_DENSE_K) return bad(0, QH_DENSE_K);
        ctx->heavy_k = (int32_t)value;
    } else if (k == "tri_cache") {
        if (value < 0 || value > ((int64_t)1 << 34)) return bad(0, (int64_t)1 << 34);
        ctx->tri_cache_records = value;
    } else if (k == "tri_wave") {
        if (value < 1 || value > TRI_WAVE_CAP) return bad(1, TRI_WAVE_CAP);
        ctx->th.tri_wave = (int)value;
    } else if (k == "tri_block") {
        if (value < 1 || value > TRI_BLOCK_CAP) return bad(1, TRI_BLOCK_CAP);
        ctx->th.tri_block = (int)value;
    } else if (k == "ql_wave") {
        if (value < 0 || value > QL_WAVE_HC / 2) return bad(0, QL_WAVE_HC / 2);
        ctx->th.ql_wave = value;
    } else if (k == "ql_block") {
        if (value < 0 || value > QL_BLOCK_HC / 2) return bad(0, QL_BLOCK_HC / 2);
        ctx->th.ql_block = value;
    } else if (k == "qh_wave") {
        if (value < 0 || value > QH_WAVE_HC / 2) return bad(0, QH_WAVE_HC / 2);
        ctx->th.qh_wave = value;
    } else if (k == "qh_block") {
        if (value < 0 || value > QH_BLOCK_HC / 2) return bad(0, QH_BLOCK_HC / 2);
        ctx->th.qh_block = value;
    } else {
        return fail(ctx, NIORCA_EINVAL, "unknown parameter %s", name);
    }
    return NIORCA_OK;
}

// ---------------------------------------------------------------------------
// Input validation (NIORCA_VALIDATE): one wave per input row.
// ---------------------------------------------------------------------------
__global__ void k_validate(int32_t n, int64_t nnz, const int64_t *__restrict__ rp, const int32_t *__restrict__ col,
                           int *__restrict__ bad) {
    int waves = gridDim.x * (blockDim.x / WAVE);
    int wid = blockIdx.x * (blockDim.x / WAVE) + threadIdx.x / WAVE;
    int flag = 0;
    if (wid == 0 && lane_id() == 0 && (rp[0] != 0 || rp[n] != nnz)) flag = 1;
    for (int32_t x = wid; x < n; x += waves) {
        int64_t b = rp[x], e = rp[x + 1];
        if (e < b || b < 0 || e > nnz) {
            flag = 1;
            continue;
        }
        for (int64_t s = b + lane_id(); s < e; s += WAVE) {
            int32_t a = col[s];
            if (a < 0 || a >= n || a == x) {
                flag = 1;
                continue;
            }
            if (s + 1 < e && col[s + 1] <= a) flag = 1;  // strictly ascending
            // symmetric: x must appear in row a
            int64_t lo = rp[a], hi = rp[a + 1];
            if (hi < lo || lo < 0 || hi > nnz) {
                flag = 1;
                continue;
            }
            while (lo < hi) {
                int64_t mid = lo + ((hi - lo) >> 1);
                if (col[mid] < x) lo = mid + 1; else hi = mid;
            }
            if (lo >= rp[a + 1] || col[lo] != x) flag = 1;
        }
    }
    if (flag) atomicOr(bad, 1);
}

// Stage I values in input slot order: t of input slot (x, a) from the relabelled layout.
__global__ void k_tri_to_input(int32_t n, const int64_t *__restrict__ rp, const int32_t *__restrict__ col,
                               const i32 *__restrict__ perm, DevGraph g, const i32 *__restrict__ t,
                               int32_t *__restrict__ tri) {
    int waves = gridDim.x * (blockDim.x / WAVE);
    int wid = blockIdx.x * (blockDim.x / WAVE) + threadIdx.x / WAVE;
    for (int32_t x = wid; x < n; x += waves) {
        i32 y = perm[x];
        for (int64_t s = rp[x] + lane_id(); s < rp[x + 1]; s += WAVE) {
            i32 b = perm[col[s]];
            i32 lo = b > y ? y : b, hi = b > y ? b : y;
            i32 slot = lower_bound_i32(g.ncol, g.nsplit[lo], g.nrp[lo + 1], hi);
            tri[s] = t[slot];
        }
    }
}

__global__ void k_k4_to_input(int32_t n, const u32 *__restrict__ order, const i64 *__restrict__ K4,
                              int64_t *__restrict__ out) {
    int32_t y = blockIdx.x * blockDim.x + threadIdx.x;
    if (y < n) out[order[y]] = K4[y];
}

// ---------------------------------------------------------------------------
// The pipeline.
// ---------------------------------------------------------------------------
struct Outputs {
    int64_t *psi = nullptr;    // [n*15] input order
    int64_t *fvars = nullptr;  // [n*9] input order
    int32_t *tri = nullptr;    // [nnz] input slot order
    int64_t *k4 = nullptr;     // [n] input order
};

static niorca_status check_graph_args(niorca_ctx *ctx, int32_t n, int64_t nnz, const int64_t *rp, const int32_t *col) {
    if (!ctx) return NIORCA_EINVAL;
    ctx->err.clear();
    if (n < 0) return fail(ctx, NIORCA_EINVAL, "n = %d is negative", n);
    if (nnz < 0 || (nnz & 1)) return fail(ctx, NIORCA_EINVAL, "nnz = %lld must be even and non-negative", (long long)nnz);
    if (n == 0 && nnz != 0) return fail(ctx, NIORCA_EINVAL, "nnz must be 0 for an empty graph");
    if (n > 0 && !rp) return fail(ctx, NIORCA_EINVAL, "row_ptr is NULL");
    if (nnz > 0 && !col) return fail(ctx, NIORCA_EINVAL, "col is NULL");
    if (nnz >= (int64_t)1 << 31) return fail(ctx, NIORCA_ENOTIMPL, "nnz = %lld is not below 2^31", (long long)nnz);
    if (nnz > (int64_t)n * (n - 1)) return fail(ctx, NIORCA_EINVAL, "nnz exceeds n(n-1)");
    return NIORCA_OK;
}

static niorca_status run(niorca_ctx *ctx, int32_t n, int64_t nnz, const int64_t *rp, const int32_t *col,
                         const Outputs &o, hipStream_t s, uint32_t flags) {
    HIP_TRY(hipSetDevice(ctx->device));
    const bool timing = (flags & NIORCA_TIMING) != 0;
    ctx->ev_valid = false;
    if (timing && !ctx->ev_made) {
        for (auto &e : ctx->ev) HIP_TRY(hipEventCreate(&e));
        ctx->ev_made = true;
    }
#define STAGE_MARK(i) \
    if (timing) HIP_TRY(hipEventRecord(ctx->ev[i], s))
    const int nthr = 256;
    const int cu = ctx->num_cu;
    // ---- workspace layout ----
    Arena A;
    const i64 radix_tiles_elems = radix_ws_elems(n);
    const i64 scan_elems = scan_ws_elems(radix_tiles_elems > n + 1 ? radix_tiles_elems : n + 1) + 8;
    uint64_t o_st = A.take<GraphStats>(1);
    uint64_t o_deg = A.take<u32>(n), o_val = A.take<u32>(n), o_k2 = A.take<u32>(n), o_v2 = A.take<u32>(n);
    uint64_t o_hist = A.take<i32>(radix_tiles_elems), o_scan = A.take<i32>(scan_elems);
    uint64_t o_perm = A.take<i32>(n), o_nrp = A.take<i32>(n + 1), o_nsplit = A.take<i32>(n);
    uint64_t o_hstart = A.take<i32>(n), o_long = A.take<i32>(n + 1);
    // slot arrays carry a pad so that a one-past-the-row read never leaves the buffer
    uint64_t o_ncol = A.take<i32>(nnz + 64), o_mirror = A.take<i32>(nnz + 64), o_t = A.take<i32>(nnz + 64);
    uint64_t o_wl = A.take<i64>(n), o_wh = A.take<i64>(n);
    uint64_t o_lists[WC_COUNT];
    for (int c = 0; c < WC_COUNT; c++) o_lists[c] = A.take<i32>(n);
    uint64_t o_acc = A.take<i64>((uint64_t)n * 10);
    uint64_t o_tcoff = A.take<i64>(n), o_tccnt = A.take<i32>(n), o_tcbump = A.take<u64>(1);
    const i64 tc_cap = ctx->tri_cache_records;
    uint64_t o_tcrec = A.take<u64>((uint64_t)(tc_cap > 0 ? tc_cap : 1));
    uint64_t base_bytes = A.off;

    // Validation first (it reads only the input).
    if (flags & NIORCA_VALIDATE) {
        niorca_status st = ensure_ws(ctx, base_bytes);
        if (st) return st;
        int *bad = (int *)(ctx->ws + o_st);
        HIP_TRY(hipMemsetAsync(bad, 0, sizeof(int), s));
        if (n > 0) hipLaunchKernelGGL(k_validate, dim3(cu * 8), dim3(nthr), 0, s, n, nnz, rp, col, bad);
        HIP_TRY(hipGetLastError());
        int hbad = 0;
        HIP_TRY(hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        if (hbad) return fail(ctx, NIORCA_ENOTSIMPLE, "the CSR is not a sorted, symmetric simple graph");
    }
    if (n == 0) return NIORCA_OK;
    {
        niorca_status st = ensure_ws(ctx, base_bytes);
        if (st) return st;
    }
    char *W = ctx->ws;
    GraphStats *dst = (GraphStats *)(W + o_st);
    u32 *deg = (u32 *)(W + o_deg), *val = (u32 *)(W + o_val), *k2 = (u32 *)(W + o_k2), *v2 = (u32 *)(W + o_v2);
    i32 *hist = (i32 *)(W + o_hist), *scanw = (i32 *)(W + o_scan);
    i32 *perm = (i32 *)(W + o_perm), *nrp = (i32 *)(W + o_nrp), *nsplit = (i32 *)(W + o_nsplit);
    i32 *hstart = (i32 *)(W + o_hstart), *longlist = (i32 *)(W + o_long);
    i32 *ncol = (i32 *)(W + o_ncol), *mirror = (i32 *)(W + o_mirror), *t = (i32 *)(W + o_t);
    i64 *wl = (i64 *)(W + o_wl), *wh = (i64 *)(W + o_wh);
    ListPtrs lists;
    for (int c = 0; c < WC_COUNT; c++) lists.l[c] = (i32 *)(W + o_lists[c]);
    i64 *accb = (i64 *)(W + o_acc);
    Accum acc{accb, accb + n, accb + 2 * (i64)n, accb + 3 * (i64)n, accb + 4 * (i64)n,
              accb + 5 * (i64)n, accb + 6 * (i64)n, accb + 7 * (i64)n, accb + 8 * (i64)n, accb + 9 * (i64)n};
    i32 *longcount = &dst->pad;

    STAGE_MARK(0);
    HIP_TRY(hipMemsetAsync(dst, 0, sizeof(GraphStats), s));
    // ---- a1: degrees and rank order (stable radix sort of degrees) ----
    hipLaunchKernelGGL(k_degree, dim3((n + nthr - 1) / nthr), dim3(nthr), 0, s, n, (i64)nnz, rp, deg, val, dst);
    HIP_TRY(hipGetLastError());
    int bits = 1;
    while (bits < 31 && ((int64_t)1 << bits) <= (int64_t)n) bits++;
    HIP_TRY(radix_sort_pairs(deg, val, k2, v2, n, bits, hist, scanw, s));
    // deg now holds degrees by new id, val the order (new id -> input id)
    hipLaunchKernelGGL(k_invert, dim3((n + nthr - 1) / nthr), dim3(nthr), 0, s, n, val, perm);
    HIP_TRY(scan_u32_to_i32(deg, n, nrp, scanw, 1, s));
    hipLaunchKernelGGL(k_relabel, dim3(cu * 8), dim3(nthr), 0, s, n, rp, col, val, perm, deg, nrp, nsplit, ncol,
                       dst);
    HIP_TRY(hipGetLastError());
    STAGE_MARK(1);
    // ---- the one wait: graph statistics ----
    GraphStats hs;
    HIP_TRY(hipMemcpyAsync(&hs, dst, sizeof(GraphStats), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (hs.bad_input)
        return fail(ctx, NIORCA_EINVAL, "row_ptr or col holds values outside the graph (use NIORCA_VALIDATE)");
    if (hs.dmax > 1200000)
        return fail(ctx, NIORCA_EOVERFLOW, "maximum degree %d could overflow int64 counts", hs.dmax);
    if (hs.dplus_max > LSORT_CAP)
        return fail(ctx, NIORCA_ENOTIMPL, "an oriented out-degree of %d exceeds %d", hs.dplus_max, LSORT_CAP);
    const i32 heavy_k = ctx->heavy_k;
    const i32 h0 = n > heavy_k ? n - heavy_k : 0;
    // ---- scratch for the large classes, sized by the statistics ----
    // vertices with |N+| above the workgroup threshold go to the global-scratch class
    const int large_cap = hs.dplus_max > ctx->th.tri_block ? hs.dplus_max : 0;
    int large_hc = 1;
    while (large_hc < 2 * large_cap) large_hc <<= 1;
    const int large_blocks = large_cap ? 2 * cu : 0;
    const i64 large_slice = large_cap ? probe_large_slice_bytes(large_cap, large_hc) : 0;
    uint64_t o_large = A.take<char>((uint64_t)large_slice * large_blocks);
    const int part_rows = QH_PART_ROWS;
    uint64_t o_part = A.take<i64>((uint64_t)part_rows * (uint64_t)(n - h0));
    const int gblocks = 32;
    const i64 gslice = 2 * (i64)n + 64;
    uint64_t o_g = A.take<i32>((uint64_t)gslice * gblocks);
    {
        niorca_status st = ensure_ws(ctx, A.off);
        if (st) return st;
        // The workspace grew and moved: start again; this time it is large enough.
        if (ctx->ws != W) return run(ctx, n, nnz, rp, col, o, s, flags & ~(uint32_t)NIORCA_VALIDATE);
    }
    char *large_scratch = W + o_large;
    i32 *gscratch = (i32 *)(W + o_g);
    i64 *qpart = (i64 *)(W + o_part);
    HIP_TRY(hipMemsetAsync(gscratch, 0, sizeof(i32) * (size_t)gslice * gblocks, s));
    // ---- oriented layout: sorted N+, mirror slots, per-vertex 4-cycle work ----
    HIP_TRY(hipMemsetAsync(longcount, 0, sizeof(i32), s));
    STAGE_MARK(2);
    hipLaunchKernelGGL(k_sort_upper_small, dim3(cu * 8), dim3(nthr), 0, s, n, nrp, nsplit, ncol, hstart, h0,
                       longlist, longcount);
    hipLaunchKernelGGL(k_sort_upper_large, dim3(cu), dim3(256), 0, s, nrp, nsplit, ncol, hstart, h0, longlist,
                       longcount);
    hipLaunchKernelGGL(k_mirror, dim3(cu * 8), dim3(nthr), 0, s, n, nrp, nsplit, ncol, hstart, h0, mirror, wl, wh);
    HIP_TRY(hipGetLastError());
    DevGraph g{n, (i32)nnz, h0, nrp, nsplit, ncol, mirror, hstart, deg, val, wl, wh};
    HIP_TRY(launch_classify(g, wl, wh, lists, dst, ctx->th, s));
    STAGE_MARK(3);
    i32 *lh[WC_COUNT];
    for (int c = 0; c < WC_COUNT; c++) lh[c] = lists.l[c];
    // ---- Stage I (t) and Stage II (K4) ----
    HIP_TRY(hipMemsetAsync(t, 0, sizeof(i32) * (size_t)nnz, s));
    HIP_TRY(hipMemsetAsync(accb, 0, sizeof(i64) * 10 * (size_t)n, s));
    TriCacheArgs tca{tc_cap > 0 ? (u64 *)(W + o_tcrec) : nullptr, tc_cap, (u64 *)(W + o_tcbump),
                     (i64 *)(W + o_tcoff), (i32 *)(W + o_tccnt), 1 << 14, 1 << 18};
    HIP_TRY(hipMemsetAsync(tca.bump, 0, sizeof(u64), s));
    STAGE_MARK(4);
    HIP_TRY(launch_probe(0, g, lh, dst, t, acc.K4, acc.tau, tca, large_scratch, large_slice, large_cap, large_hc,
                         large_blocks, cu * 8, cu * 2, s));
    STAGE_MARK(5);
    if (o.tri) {
        hipLaunchKernelGGL(k_tri_to_input, dim3(cu * 8), dim3(nthr), 0, s, n, rp, col, perm, g, t, o.tri);
        HIP_TRY(hipGetLastError());
    }
    if (o.k4 && !o.psi && !o.fvars) {
        hipLaunchKernelGGL(k_k4_to_input, dim3((n + nthr - 1) / nthr), dim3(nthr), 0, s, n, val, acc.K4, o.k4);
        HIP_TRY(hipGetLastError());
        return NIORCA_OK;
    }
    if (!o.psi && !o.fvars) return NIORCA_OK;
    // ---- Stage III-a: neighbour sums, tau, 4-cycles ----
    HIP_TRY(launch_sums(g, t, acc, cu * 8, s));
    STAGE_MARK(6);
    HIP_TRY(launch_probe(1, g, lh, dst, t, acc.K4, acc.tau, tca, large_scratch, large_slice, large_cap, large_hc,
                         large_blocks, cu * 8, cu * 2, s));
    STAGE_MARK(7);
    HIP_TRY(launch_q(g, lh, dst, acc.Q, gscratch, gslice, gblocks, cu * 4, cu * 4, cu * 2, qpart, part_rows, s));
    STAGE_MARK(8);
    // ---- Stage III-b: equations ----
    HIP_TRY(launch_solve(g, acc, o.psi, o.fvars, dst, cu * 8, s));
    STAGE_MARK(9);
    ctx->ev_valid = timing;
    if (o.k4) {
        hipLaunchKernelGGL(k_k4_to_input, dim3((n + nthr - 1) / nthr), dim3(nthr), 0, s, n, val, acc.K4, o.k4);
        HIP_TRY(hipGetLastError());
    }
    ctx->last = hs;
    return NIORCA_OK;
}

static hipStream_t as_stream(void *s) { return (hipStream_t)s; }

extern "C" niorca_status niorca_count(niorca_ctx *ctx, int32_t n, int64_t nnz, const int64_t *row_ptr,
                                      const int32_t *col, int64_t *out, void *stream, uint32_t flags) {
    niorca_status st = check_graph_args(ctx, n, nnz, row_ptr, col);
    if (st) return st;
    if (n > 0 && !out) return fail(ctx, NIORCA_EINVAL, "out is NULL");
    const uint32_t known = NIORCA_VALIDATE | NIORCA_BIN_DEGREE | NIORCA_BIN_MLP | NIORCA_COUNTERS | NIORCA_TIMING;
    if (flags & ~known) return fail(ctx, NIORCA_EINVAL, "unknown flag bits 0x%x", flags & ~known);
    Outputs o;
    o.psi = out;
    return run(ctx, n, nnz, row_ptr, col, o, as_stream(stream), flags);
}

extern "C" niorca_status niorca_edge_triangles(niorca_ctx *ctx, int32_t n, int64_t nnz, const int64_t *row_ptr,
                                               const int32_t *col, int32_t *tri, void *stream) {
    niorca_status st = check_graph_args(ctx, n, nnz, row_ptr, col);
    if (st) return st;
    if (nnz > 0 && !tri) return fail(ctx, NIORCA_EINVAL, "tri is NULL");
    Outputs o;
    o.tri = tri;
    return run(ctx, n, nnz, row_ptr, col, o, as_stream(stream), 0);
}

extern "C" niorca_status niorca_k4(niorca_ctx *ctx, int32_t n, int64_t nnz, const int64_t *row_ptr,
                                   const int32_t *col, int64_t *k4, void *stream) {
    niorca_status st = check_graph_args(ctx, n, nnz, row_ptr, col);
    if (st) return st;
    if (n > 0 && !k4) return fail(ctx, NIORCA_EINVAL, "k4 is NULL");
    Outputs o;
    o.k4 = k4;
    return run(ctx, n, nnz, row_ptr, col, o, as_stream(stream), 0);
}

extern "C" niorca_status niorca_fvars(niorca_ctx *ctx, int32_t n, int64_t nnz, const int64_t *row_ptr,
                                      const int32_t *col, int64_t *fvars, void *stream) {
    niorca_status st = check_graph_args(ctx, n, nnz, row_ptr, col);
    if (st) return st;
    if (n > 0 && !fvars) return fail(ctx, NIORCA_EINVAL, "fvars is NULL");
    Outputs o;
    o.fvars = fvars;
    return run(ctx, n, nnz, row_ptr, col, o, as_stream(stream), 0);
}

extern "C" niorca_status niorca_count_batched(niorca_ctx *ctx, int32_t num_graphs, const int64_t *vtx_off,
                                              const int64_t *row_ptr, const int32_t *col, int64_t *out,
                                              void *stream, uint32_t flags) {
    (void)num_graphs; (void)vtx_off; (void)row_ptr; (void)col; (void)out; (void)stream; (void)flags;
    return fail(ctx, NIORCA_ENOTIMPL, "batched counting is not built yet");
}

extern "C" niorca_status niorca_work_counters(niorca_ctx *ctx, int32_t n, int64_t *counters, void *stream) {
    (void)n; (void)counters; (void)stream;
    return fail(ctx, NIORCA_EINVAL, "no work counters were recorded");
}

extern "C" niorca_status niorca_stage_times(niorca_ctx *ctx, float *ms, int32_t count) {
    if (!ctx || !ms || count < NIORCA_NUM_STAGES) return fail(ctx, NIORCA_EINVAL, "need %d floats", NIORCA_NUM_STAGES);
    if (!ctx->ev_valid) return fail(ctx, NIORCA_EINVAL, "the last call did not record stage times");
    HIP_TRY(hipEventSynchronize(ctx->ev[NIORCA_NUM_STAGES]));
    for (int i = 0; i < NIORCA_NUM_STAGES; i++) HIP_TRY(hipEventElapsedTime(&ms[i], ctx->ev[i], ctx->ev[i + 1]));
    return NIORCA_OK;
}

extern "C" niorca_status niorca_set_cost_model(niorca_ctx *ctx, const float *weights, int32_t count, float thr_wave,
                                               float thr_block) {
    if (!ctx || !weights || count != NIORCA_MLP_PARAMS) return fail(ctx, NIORCA_EINVAL, "cost model needs %d floats", NIORCA_MLP_PARAMS);
    ctx->mlp.assign(weights, weights + count);
    ctx->thr_wave = thr_wave;
    ctx->thr_block = thr_block;
    return NIORCA_OK;
}

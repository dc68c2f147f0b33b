// Host side of the C ABI declared in include/niorca.h: argument checks, the
// device workspace, and the order of the stages on the caller's stream.
#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
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
    // cost model for NIORCA_BIN_MLP (host copy and device copy)
    std::vector<float> mlp;
    float *mlp_dev = nullptr;
    float thr_thread = 0.f, thr_group = -1e30f, thr_block = 0.f;
    // where the last count left its counters and features (offsets in the workspace)
    int32_t last_n = -1;
    uint64_t last_counters = 0, last_feat = 0, last_order = 0, last_stats_dev = 0;
    char *last_ws = nullptr;
    GraphStats last{};
    // per-stage HIP events of the last call made with NIORCA_TIMING
    hipEvent_t ev[NIORCA_NUM_STAGES + 1] = {};
    hipEvent_t kev[NUM_KERNEL_SLOTS] = {};
    bool ev_made = false;
    bool ev_valid = false;
    // tunable class thresholds and the size of the heavy 4-cycle key range
    // (degree binning: no one-lane items, sixteen lanes up to degree 32, no degree
    // promotion to workgroups -- the measured best on the Erdos-Renyi, Chung-Lu,
    // R-MAT and batched workloads)
    Thresholds th{TRI_WAVE_CAP, TRI_BLOCK_CAP, 0, 0, 1 << 30, 0.f, 0.f, nullptr,
                  512, 8192, 512, 2048, 2048, 32, -1e30f};
    // size of the heavy 4-cycle key range; -1 = chosen per call from the degrees
    int32_t heavy_k = -1;
    // the last captured batched sequence and the shape it was captured for
    hipGraphExec_t gexec = nullptr;
    uint64_t gkey = 0;
    // the region of global 4-cycle counters last cleared (kernels leave it zero)
    char *gz_ws = nullptr;
    uint64_t gz_off = 0, gz_bytes = 0;
    int64_t tri_cache_records = (int64_t)1 << 32;  // at most 32 GiB of kept triangles for the tau pass
    int64_t large_lds_max = PL_LDS_MAX;            // LDS bytes the large probe kernel may take
    int bin_default = 0;  // binning of calls whose flags ask for none: 0 none, 1 degree, 2 learned
    // set for the duration of a niorca_count_noalloc call: the fixed scratch it runs in
    char *fixed_ws = nullptr;
    uint64_t fixed_bytes = 0;
};

// ---------------------------------------------------------------------------
// The fixed workspace of niorca_count_noalloc: one device array, of which every GPU
// the library runs on holds its own copy until the process ends.  Host code never
// passes `scratch` itself to a kernel (in host code the name is a stand-in, not a
// device address): niorca_create looks up each device's address of it once, with
// that device current, and every later use goes through that address.
// ---------------------------------------------------------------------------
static __device__ __align__(256) char scratch[NIORCA_NOALLOC_BYTES];
#define MAX_DEVICES 64
static char *g_scratch[MAX_DEVICES];
static std::mutex g_scratch_mu;

// Device address of `scratch` on the current device `device` (looked up once).
static hipError_t scratch_address(int device, char **out) {
    *out = nullptr;
    if (device < 0 || device >= MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[device]) {
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch[device] = (char *)p;
    }
    *out = g_scratch[device];
    return hipSuccess;
}

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
    char *sp = nullptr;
    if (scratch_address(device, &sp) != hipSuccess) {
        (void)hipGetLastError();
        delete c;
        return NIORCA_EDEVICE;
    }
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) == hipSuccess && prop.multiProcessorCount > 0)
        c->num_cu = prop.multiProcessorCount;
    *out = c;
    return NIORCA_OK;
}

extern "C" void niorca_destroy(niorca_ctx *ctx) {
    if (!ctx) return;
    if (ctx->ev_made) {
        for (auto &e : ctx->ev) (void)hipEventDestroy(e);
        for (auto &e : ctx->kev) (void)hipEventDestroy(e);
    }
    if (ctx->gexec) (void)hipGraphExecDestroy(ctx->gexec);
    if (ctx->mlp_dev) (void)hipFree(ctx->mlp_dev);
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
        if (value < -1 || value > QH_DENSE_K) return bad(-1, QH_DENSE_K);
        ctx->heavy_k = (int32_t)value;
    } else if (k == "tri_cache") {
        if (value < 0 || value > ((int64_t)1 << 34)) return bad(0, (int64_t)1 << 34);
        ctx->tri_cache_records = value;
    } else if (k == "bin_deg_thread") {
        if (value < 0 || value > ((int64_t)1 << 30)) return bad(0, (int64_t)1 << 30);
        ctx->th.deg_thread = (int)value;
    } else if (k == "bin_deg_group") {
        if (value < 0 || value > ((int64_t)1 << 30)) return bad(0, (int64_t)1 << 30);
        ctx->th.deg_group = (int)value;
    } else if (k == "bin_deg_block") {
        if (value < 1 || value > ((int64_t)1 << 30)) return bad(1, (int64_t)1 << 30);
        ctx->th.deg_block = (int)value;
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
    } else if (k == "ql_split") {
        if (value < 0 || value > QL_BLOCK_HC / 2) return bad(0, QL_BLOCK_HC / 2);
        ctx->th.ql_split = value;
    } else if (k == "large_lds") {
        if (value < 0 || value > PL_LDS_MAX) return bad(0, PL_LDS_MAX);
        ctx->large_lds_max = value;
    } else if (k == "bin_mode") {
        if (value < 0 || value > 2) return bad(0, 2);
        if (value == 2 && !ctx->mlp_dev) return fail(ctx, NIORCA_EINVAL, "bin_mode 2 needs a cost model");
        ctx->bin_default = (int)value;
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

// Per-edge values in input slot order: the value of input slot (x, a) is kept on
// the N+ slot of the edge in the relabelled layout (Stage I t, per-edge 4-cliques).
template <typename T>
__global__ void k_slot_to_input(int32_t n, const int64_t *__restrict__ rp, const int32_t *__restrict__ col,
                                const i32 *__restrict__ perm, DevGraph g, const T *__restrict__ t,
                                T *__restrict__ tri) {
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

// Counters known before Stage I: probes, 4-cycle wedges, neighbour-sum slots.
__global__ void k_counters_base(int32_t n, const i32 *__restrict__ nrp, const i64 *__restrict__ probes,
                                const i64 *__restrict__ wl, const i64 *__restrict__ wh, i64 *__restrict__ c) {
    int32_t y = blockIdx.x * blockDim.x + threadIdx.x;
    if (y >= n) return;
    i64 *r = c + (i64)y * NUM_COUNTERS;
    r[0] = probes[y];
    r[3] = wl[y];
    r[4] = wh[y];
    r[5] = 2 * (i64)(nrp[y + 1] - nrp[y]);
}

// Rows of `k` values from new-id order to input order.
template <typename T>
__global__ void k_rows_to_input(int32_t n, int k, const u32 *__restrict__ order, const T *__restrict__ src,
                                T *__restrict__ dst) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)n * k) return;
    int64_t y = i / k, c = i % k;
    dst[(int64_t)order[y] * k + c] = src[i];
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
    int64_t *ek4 = nullptr;    // [nnz] input slot order: 4-cliques through each edge
};

// Internal flag of run(): Stage I/II also credits the 4-cliques through each edge.
#define RUN_EDGE_K4 0x80000000u

// Bounds the host already knows (batched calls): with them the pipeline needs no
// wait on the device, so the whole sequence can be captured into a hipGraph.
// Triangle records kept in batched (bounded) runs, whose triangle bound is unknown
// to the host: 4 GiB.
#define BOUNDED_TRI_CACHE ((i64)1 << 29)

struct HostBounds {
    int dmax;       // maximum degree
    int dplus_max;  // maximum |N+|
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

// Workspace layout of one count.
struct Layout {
    uint64_t st, deg, val, k2, v2, hist, scan, perm, nrp, nsplit, hstart, lng, ncol, mirror, t, wl, wh, vmeta;
    uint64_t hseg, lbeg;  // per-slot 4-cycle wedge runs (heavy: int2 bounds; light: start)
    uint64_t dslot;       // per-slot neighbour degree
    uint64_t lists[WC_COUNT];
    uint64_t acc, tcoff, tccnt, tcbump, tcrec, probes, feat, pred, counters, ek4;
    uint64_t base_end;  // everything above needs no graph statistics
    uint64_t large, part, gcnt, colg, voff;
    uint64_t total;
    i64 tc_cap;
    int large_cap, large_hc, large_blocks, part_rows, gblocks;
    i64 large_slice, gslice;
    i32 h0;
};

static void layout_base(Layout &L, const niorca_ctx *ctx, int32_t n, int64_t nnz, uint32_t flags, Arena &A) {
    const i64 radix_tiles_elems = radix_ws_elems(n);
    const i64 scan_elems = scan_ws_elems(radix_tiles_elems > n + 1 ? radix_tiles_elems : n + 1) + 8;
    L.st = A.take<GraphStats>(1);
    L.deg = A.take<u32>(n); L.val = A.take<u32>(n); L.k2 = A.take<u32>(n); L.v2 = A.take<u32>(n);
    L.hist = A.take<i32>(radix_tiles_elems); L.scan = A.take<i32>(scan_elems);
    L.perm = A.take<i32>(n); L.nrp = A.take<i32>(n + 1); L.nsplit = A.take<i32>(n);
    L.hstart = A.take<i32>(n); L.lng = A.take<i32>(n + 1);
    // slot arrays carry a pad so that a one-past-the-row read never leaves the buffer
    L.ncol = A.take<i32>(nnz + 64); L.mirror = A.take<i32>(nnz + 64); L.t = A.take<i32>(nnz + 64);
    L.hseg = A.take<int2>(nnz + 64); L.lbeg = A.take<i32>(nnz + 64);
    L.wl = A.take<i64>(n); L.wh = A.take<i64>(n);
    L.vmeta = A.take<int4>(n);
    for (int c = 0; c < WC_COUNT; c++) L.lists[c] = A.take<i32>(n);
    L.acc = A.take<i64>((uint64_t)n * 10);
    L.tcoff = A.take<i64>(n); L.tccnt = A.take<i32>(n); L.tcbump = A.take<u64>(1);
    L.probes = A.take<i64>(n);
    const bool mlp = (flags & NIORCA_BIN_MLP) || (!(flags & NIORCA_BIN_DEGREE) && ctx->bin_default == 2);
    const bool feats = mlp || (flags & NIORCA_COUNTERS);
    L.feat = feats ? A.take<float>((uint64_t)n * 6) : 0;
    L.pred = mlp ? A.take<float>(n) : 0;
    L.counters = (flags & NIORCA_COUNTERS) ? A.take<i64>((uint64_t)n * NUM_COUNTERS) : 0;
    L.ek4 = (flags & RUN_EDGE_K4) ? A.take<i64>((uint64_t)nnz + 64) : 0;
    L.base_end = A.off;
}

// The heavy 4-cycle range: the top QH_DENSE_K ranks when the graph has hubs (maximum
// degree above 8x the mean), none otherwise; batched runs (no statistics) use 4096.
static int32_t heavy_range(const niorca_ctx *ctx, int32_t n, int64_t nnz, int dmax, bool bounded) {
    if (ctx->heavy_k >= 0) return ctx->heavy_k;
    if (bounded) return 4096;
    const int64_t mean = n > 0 ? nnz / n : 0;
    return (int64_t)dmax > 8 * (mean > 1 ? mean : 1) ? QH_DENSE_K : 0;
}

// small: a fixed workspace (niorca_count_noalloc), where the scratch of the large
// Stage I class and of the 4-cycle global counters is kept to a few slices.
static void layout_rest_with(Layout &L, const niorca_ctx *ctx, int32_t n, int64_t nnz, int dmax, int dplus_max,
                             i64 tc_cap, bool bounded, bool small, Arena &A) {
    const int cu = ctx->num_cu;
    L.tc_cap = tc_cap;
    L.tcrec = A.take<u64>((uint64_t)(L.tc_cap > 0 ? L.tc_cap : 1));
    const int32_t hk = heavy_range(ctx, n, nnz, dmax, bounded);
    L.h0 = n > hk ? n - hk : 0;
    // vertices with |N+| above the workgroup threshold go to the global-scratch class
    L.large_cap = dplus_max > ctx->th.tri_block ? dplus_max : 0;
    L.large_hc = 1;
    while (L.large_hc < 2 * L.large_cap) L.large_hc <<= 1;
    L.large_blocks = L.large_cap ? (small ? (2 * cu < 32 ? 2 * cu : 32) : 2 * cu) : 0;
    L.large_slice = L.large_cap ? probe_large_slice_bytes(L.large_cap, L.large_hc, ctx->large_lds_max) : 0;
    L.large = A.take<char>((uint64_t)L.large_slice * L.large_blocks);
    L.part_rows = QH_PART_ROWS;
    L.part = A.take<i64>((uint64_t)L.part_rows * (uint64_t)(n - L.h0));
    // int32 counters over all vertices for the rare 4-cycle items that overflow LDS
    if (bounded) {
        L.gblocks = 2;
    } else if (small) {
        L.gblocks = 8;
    } else {
        // one slice per CU, within 8 GiB of the 288 GB
        const i64 fit = ((i64)8 << 30) / ((2 * (i64)n + 64) * 4);
        L.gblocks = (int)(fit < cu ? (fit < 8 ? 8 : fit) : cu);
    }
    L.gslice = 2 * (i64)n + 64;
    L.gcnt = A.take<i32>((uint64_t)L.gslice * L.gblocks);
    // last, so that adding it moved no other array: the 4-cycle kernels measured
    // about 10% slower on one heavy-tailed graph with every later array shifted
    L.dslot = A.take<i32>(nnz + 64);
    L.total = A.off;
}

// budget > 0: the layout must end within budget bytes (a fixed workspace); the
// triangle records kept for the tau pass then get what the rest leaves (vertices
// whose records do not fit are probed again).
static void layout_rest(Layout &L, const niorca_ctx *ctx, int32_t n, int64_t nnz, int dmax, int dplus_max,
                        i64 pairs, bool bounded, Arena &A, uint64_t budget = 0) {
    // triangle records for the tau pass: no more than the graph can have
    i64 cap = ctx->tri_cache_records < pairs ? ctx->tri_cache_records : pairs;
    if (budget) {
        Layout D = L;
        Arena B = A;
        layout_rest_with(D, ctx, n, nnz, dmax, dplus_max, 0, bounded, true, B);
        const i64 room = B.off < budget ? (i64)((budget - B.off) / sizeof(u64)) : 0;
        if (cap > room) cap = room;
    }
    layout_rest_with(L, ctx, n, nnz, dmax, dplus_max, cap, bounded, budget != 0, A);
}

// Fill kernels (no memset nodes: the sequence may be captured into a hipGraph).
__global__ void k_fill32(u32 *__restrict__ p, i64 words, u32 v) {
    for (i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x; i < words; i += (i64)gridDim.x * blockDim.x) p[i] = v;
}

static hipError_t fill32(void *p, i64 bytes, u32 v, hipStream_t s) {
    i64 words = bytes / 4;
    if (words <= 0) return hipSuccess;
    i64 blocks = (words + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(k_fill32, dim3((u32)blocks), dim3(256), 0, s, (u32 *)p, words, v);
    return hipGetLastError();
}

// A call that stopped after Stage I/II: its statistics (device_status) stay
// readable, the counters and features of an earlier count do not.
static void mark_partial(niorca_ctx *ctx, uint64_t st_off, char *W) {
    ctx->last_stats_dev = st_off;
    ctx->last_ws = W;
    ctx->last_n = -1;
    ctx->last_counters = 0;
    ctx->last_feat = 0;
}

static niorca_status run(niorca_ctx *ctx, int32_t n, int64_t nnz, const int64_t *rp, const int32_t *col,
                         const Outputs &o, hipStream_t s, uint32_t flags, const HostBounds *hb) {
    HIP_TRY(hipSetDevice(ctx->device));
    const bool timing = (flags & NIORCA_TIMING) != 0;
    ctx->ev_valid = false;
    if (timing && !ctx->ev_made) {
        for (auto &e : ctx->ev) HIP_TRY(hipEventCreate(&e));
        for (auto &e : ctx->kev) HIP_TRY(hipEventCreate(&e));
        ctx->ev_made = true;
    }
    const KernelEvents kev{timing ? ctx->kev : nullptr};
    const KernelEvents nokev{nullptr};
#define STAGE_MARK(i) \
    if (timing) HIP_TRY(hipEventRecord(ctx->ev[i], s))
    const int nthr = 256;
    const int cu = ctx->num_cu;
    Layout L;
    Arena A;
    layout_base(L, ctx, n, nnz, flags, A);
    if (hb) layout_rest(L, ctx, n, nnz, hb->dmax, hb->dplus_max, BOUNDED_TRI_CACHE, true, A);
    const uint64_t need_now = hb ? A.off : L.base_end;

    // a fixed workspace (niorca_count_noalloc) is never allocated, only checked
    const bool fixed = ctx->fixed_ws != nullptr;
    auto have = [&](uint64_t need) -> niorca_status {
        if (!fixed) return ensure_ws(ctx, need);
        if (need > ctx->fixed_bytes)
            return fail(ctx, NIORCA_ENOMEM, "this graph needs %llu bytes of workspace; the fixed scratch holds %llu",
                        (unsigned long long)need, (unsigned long long)ctx->fixed_bytes);
        return NIORCA_OK;
    };
    // Validation first (it reads only the input).
    if (flags & NIORCA_VALIDATE) {
        niorca_status st = have(need_now);
        if (st) return st;
        int *bad = (int *)((fixed ? ctx->fixed_ws : ctx->ws) + L.st);
        HIP_TRY(fill32(bad, sizeof(int), 0u, s));
        if (n > 0) hipLaunchKernelGGL(k_validate, dim3(cu * 8), dim3(nthr), 0, s, n, nnz, rp, col, bad);
        HIP_TRY(hipGetLastError());
        int hbad = 0;
        HIP_TRY(hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        if (hbad) return fail(ctx, NIORCA_ENOTSIMPLE, "the CSR is not a sorted, symmetric simple graph");
    }
    if (n == 0) return NIORCA_OK;
    {
        niorca_status st = have(need_now);
        if (st) return st;
    }
    char *W = fixed ? ctx->fixed_ws : ctx->ws;
    GraphStats *dst = (GraphStats *)(W + L.st);
    u32 *deg = (u32 *)(W + L.deg), *val = (u32 *)(W + L.val), *k2 = (u32 *)(W + L.k2), *v2 = (u32 *)(W + L.v2);
    i32 *hist = (i32 *)(W + L.hist), *scanw = (i32 *)(W + L.scan);
    i32 *perm = (i32 *)(W + L.perm), *nrp = (i32 *)(W + L.nrp), *nsplit = (i32 *)(W + L.nsplit);
    i32 *hstart = (i32 *)(W + L.hstart), *longlist = (i32 *)(W + L.lng);
    i32 *ncol = (i32 *)(W + L.ncol), *mirror = (i32 *)(W + L.mirror), *t = (i32 *)(W + L.t);
    int2 *hseg = (int2 *)(W + L.hseg);
    i32 *lbeg = (i32 *)(W + L.lbeg);
    i64 *wl = (i64 *)(W + L.wl), *wh = (i64 *)(W + L.wh);
    int4 *vmeta = (int4 *)(W + L.vmeta);
    ListPtrs lists;
    for (int c = 0; c < WC_COUNT; c++) lists.l[c] = (i32 *)(W + L.lists[c]);
    i64 *accb = (i64 *)(W + L.acc);
    // (T, psi1) pairs first, so that they are 16-byte aligned
    Accum acc{accb + 2 * (i64)n, accb + 3 * (i64)n, accb + 4 * (i64)n, accb + 5 * (i64)n, accb + 6 * (i64)n,
              accb, accb + 7 * (i64)n, accb + 8 * (i64)n, accb + 9 * (i64)n};
    i32 *longcount = &dst->pad;

    STAGE_MARK(0);
    HIP_TRY(fill32(dst, sizeof(GraphStats), 0u, s));
    // ---- a1: degrees and rank order (stable radix sort of degrees) ----
    // bounded runs size their per-row buffers from the host's degree bound: longer
    // rows are refused by the degree pass (degree 0, bad_input)
    const i64 dcap = hb ? (i64)hb->dmax : (i64)INT32_MAX;
    hipLaunchKernelGGL(k_degree, dim3(cu * 8), dim3(nthr), 0, s, n, (i64)nnz, dcap, rp, deg, val, dst);
    HIP_TRY(hipGetLastError());
    int bits = 1;
    while (bits < 31 && ((int64_t)1 << bits) <= (int64_t)n) bits++;
    HIP_TRY(radix_sort_pairs(deg, val, k2, v2, n, bits, hist, scanw, s));
    // deg now holds degrees by new id, val the order (new id -> input id)
    hipLaunchKernelGGL(k_invert, dim3((n + nthr - 1) / nthr), dim3(nthr), 0, s, n, val, perm);
    HIP_TRY(scan_u32_to_i32(deg, n, nrp, scanw, 1, s));
    hipLaunchKernelGGL(k_relabel, dim3(cu * 8), dim3(nthr), 0, s, n, rp, col, val, perm, deg, nrp, nsplit, ncol,
                       vmeta, dst);
    HIP_TRY(hipGetLastError());
    STAGE_MARK(1);
    GraphStats hs{};
    if (!hb) {
        // ---- the one wait: graph statistics ----
        HIP_TRY(hipMemcpyAsync(&hs, dst, sizeof(GraphStats), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        if (hs.bad_input)
            return fail(ctx, NIORCA_EINVAL, "row_ptr or col holds values outside the graph (use NIORCA_VALIDATE)");
        if (hs.dmax > 1200000)
            return fail(ctx, NIORCA_EOVERFLOW, "maximum degree %d could overflow int64 counts", hs.dmax);
        if (hs.dplus_max > LSORT_CAP)
            return fail(ctx, NIORCA_ENOTIMPL, "an oriented out-degree of %d exceeds %d", hs.dplus_max, LSORT_CAP);
        layout_rest(L, ctx, n, nnz, hs.dmax, hs.dplus_max, hs.pairs, false, A, fixed ? ctx->fixed_bytes : 0);
        niorca_status st = have(A.off);
        if (st) return st;
        // The workspace grew and moved: start again; this time it is large enough.
        if (!fixed && ctx->ws != W) return run(ctx, n, nnz, rp, col, o, s, flags & ~(uint32_t)NIORCA_VALIDATE, hb);
    } else {
        hs.dmax = hb->dmax;
        hs.dplus_max = hb->dplus_max;
    }
    const i32 h0 = L.h0;
    char *large_scratch = W + L.large;
    i32 *gscratch = (i32 *)(W + L.gcnt);
    i64 *qpart = (i64 *)(W + L.part);
    i32 *dslot = (i32 *)(W + L.dslot);
    // The global 4-cycle counters are returned to zero by the kernels that use them,
    // so they are cleared only when their place in the workspace changes -- and on
    // every bounded (possibly captured) run, whose replays may follow other calls.
    // A fixed workspace is shared by every context on the device: always cleared.
    if (hb || fixed || ctx->gz_ws != W || ctx->gz_off != L.gcnt ||
        ctx->gz_bytes != (uint64_t)L.gslice * L.gblocks * 4) {
        HIP_TRY(fill32(gscratch, (i64)L.gslice * L.gblocks * 4, 0u, s));
        ctx->gz_ws = fixed ? nullptr : W;
        ctx->gz_off = L.gcnt;
        ctx->gz_bytes = (uint64_t)L.gslice * L.gblocks * 4;
    }
    // ---- oriented layout: sorted N+, mirror slots, per-vertex 4-cycle work ----
    HIP_TRY(fill32(longcount, sizeof(i32), 0u, s));
    STAGE_MARK(2);
    hipLaunchKernelGGL(k_sort_upper_small, dim3(cu * 8), dim3(nthr), 0, s, n, deg, nrp, nsplit, ncol, hstart, vmeta,
                       h0, longlist, longcount);
    hipLaunchKernelGGL(k_sort_upper_large, dim3(cu * LSORT_GRID), dim3(LSORT_NT), 0, s, nrp, nsplit, ncol, hstart,
                       vmeta, h0, longlist, longcount);
    i64 *probes = (i64 *)(W + L.probes);
    float *feat = L.feat ? (float *)(W + L.feat) : nullptr;
    float *pred = L.pred ? (float *)(W + L.pred) : nullptr;
    i64 *counters = L.counters ? (i64 *)(W + L.counters) : nullptr;
    hipLaunchKernelGGL(k_mirror, dim3(cu * 8), dim3(nthr), 0, s, n, deg, nrp, nsplit, ncol, vmeta, h0, mirror, hseg, lbeg, dslot, wl,
                       wh, probes, feat);
    HIP_TRY(hipGetLastError());
    Thresholds th = ctx->th;
    th.bin_mode = (flags & NIORCA_BIN_MLP) ? 2 : ((flags & NIORCA_BIN_DEGREE) ? 1 : ctx->bin_default);
    if (th.bin_mode == 2) {
        HIP_TRY(mlp_predict(n, feat, ctx->mlp_dev, pred, s));
        th.pred = pred;
        th.thr_thread = ctx->thr_thread;
        th.thr_group = ctx->thr_group;
        th.thr_block = ctx->thr_block;
    }
    DevGraph g{n, (i32)nnz, h0, nrp, nsplit, ncol, mirror, hstart, deg, val, wl, wh, vmeta, hseg, lbeg, dslot};
    HIP_TRY(launch_classify(g, wl, wh, probes, lists, dst, th, s));
    if (counters) {
        HIP_TRY(fill32(counters, (i64)sizeof(i64) * NUM_COUNTERS * n, 0u, s));
        hipLaunchKernelGGL(k_counters_base, dim3((n + nthr - 1) / nthr), dim3(nthr), 0, s, n, nrp, probes, wl, wh,
                           counters);
        HIP_TRY(hipGetLastError());
    }
    STAGE_MARK(3);
    i32 *lh[WC_COUNT];
    for (int c = 0; c < WC_COUNT; c++) lh[c] = lists.l[c];
    // ---- Stage I (t) and Stage II (K4) ----
    HIP_TRY(fill32(t, sizeof(i32) * nnz, 0u, s));
    HIP_TRY(fill32(accb, sizeof(i64) * 10 * (i64)n, 0u, s));
    // records are handed out in chunks: about two per wave (workgroup) of the Stage I
    // grid, but never less than the largest item of the class needs, C(64, 2)
    // (C(512, 2)), and never more than 2^14 (2^18)
    auto chunk_for = [&](i64 holders, i64 lo, i64 hi) {
        i64 c = L.tc_cap / (2 * holders);
        return c < lo ? lo : (c > hi ? hi : c);
    };
    TriCacheArgs tca{L.tc_cap > 0 ? (u64 *)(W + L.tcrec) : nullptr, L.tc_cap, (u64 *)(W + L.tcbump),
                     (i64 *)(W + L.tcoff), (i32 *)(W + L.tccnt), chunk_for((i64)cu * 8 * 4, 2048, 1 << 14),
                     chunk_for((i64)cu * 2, 1 << 17, 1 << 18), chunk_for((i64)cu * 8 * 16, 256, 1 << 12)};
    HIP_TRY(fill32(tca.bump, sizeof(u64), 0u, s));
    STAGE_MARK(4);
    if (o.ek4) {
        // Stage I/II with the 4-cliques through every edge (on its N+ slot)
        i64 *ek4 = (i64 *)(W + L.ek4);
        HIP_TRY(fill32(ek4, sizeof(i64) * nnz, 0u, s));
        HIP_TRY(launch_probe(2, g, lh, dst, t, acc.K4, ek4, tca, large_scratch, L.large_slice, L.large_cap,
                             L.large_hc, L.large_blocks, ctx->large_lds_max, cu * 8, cu * PB_GRID, nullptr, nokev, s));
        hipLaunchKernelGGL(k_slot_to_input<i64>, dim3(cu * 8), dim3(nthr), 0, s, n, rp, col, perm, g,
                           (const i64 *)ek4, o.ek4);
        HIP_TRY(hipGetLastError());
        mark_partial(ctx, L.st, W);
        return NIORCA_OK;
    }
    HIP_TRY(launch_probe(0, g, lh, dst, t, acc.K4, acc.tau, tca, large_scratch, L.large_slice, L.large_cap,
                         L.large_hc, L.large_blocks, ctx->large_lds_max, cu * 8, cu * PB_GRID, counters, kev, s));
    STAGE_MARK(5);
    if (o.tri) {
        hipLaunchKernelGGL(k_slot_to_input<i32>, dim3(cu * 8), dim3(nthr), 0, s, n, rp, col, perm, g,
                           (const i32 *)t, (i32 *)o.tri);
        HIP_TRY(hipGetLastError());
    }
    if (o.k4 && !o.psi && !o.fvars) {
        hipLaunchKernelGGL(k_k4_to_input, dim3((n + nthr - 1) / nthr), dim3(nthr), 0, s, n, val, acc.K4, o.k4);
        HIP_TRY(hipGetLastError());
        mark_partial(ctx, L.st, W);
        return NIORCA_OK;
    }
    if (!o.psi && !o.fvars) {
        mark_partial(ctx, L.st, W);
        return NIORCA_OK;
    }
    // ---- Stage III-a: neighbour sums, tau, 4-cycles ----
    HIP_TRY(launch_sums(g, t, acc, cu * 8, s));
    STAGE_MARK(6);
    HIP_TRY(launch_probe(1, g, lh, dst, t, acc.K4, acc.tau, tca, large_scratch, L.large_slice, L.large_cap,
                         L.large_hc, L.large_blocks, ctx->large_lds_max, cu * 8, cu * PB_GRID_TAU, nullptr, nokev, s));
    STAGE_MARK(7);
    if (n - h0 > 0) HIP_TRY(fill32(qpart, (i64)sizeof(i64) * L.part_rows * (n - h0), 0u, s));
    HIP_TRY(launch_q(g, lh, dst, acc.Q, gscratch, L.gslice, L.gblocks, cu * 4, cu * 4, cu * 2, qpart, L.part_rows,
                     th.ql_wave, th.ql_block, th.ql_split, th.qh_wave, th.qh_block, kev, s));
    STAGE_MARK(8);
    // ---- Stage III-b: equations ----
    HIP_TRY(launch_solve(g, acc, o.psi, o.fvars, dst, cu * 8, (flags & NIORCA_INDUCED) != 0, s));
    STAGE_MARK(9);
    ctx->ev_valid = timing;
    if (o.k4) {
        hipLaunchKernelGGL(k_k4_to_input, dim3((n + nthr - 1) / nthr), dim3(nthr), 0, s, n, val, acc.K4, o.k4);
        HIP_TRY(hipGetLastError());
    }
    ctx->last = hs;
    ctx->last_stats_dev = L.st;
    ctx->last_n = n;
    ctx->last_counters = counters ? L.counters : 0;
    ctx->last_feat = feat ? L.feat : 0;
    ctx->last_order = L.val;
    ctx->last_ws = W;
    if (flags & NIORCA_VALIDATE) {
        // validated calls wait anyway: report the equations' evenness check too
        GraphStats fin{};
        HIP_TRY(hipMemcpyAsync(&fin, dst, sizeof(GraphStats), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        if (fin.err) return fail(ctx, NIORCA_EINTERNAL, "an equation's numerator that must be even was odd");
    }
    return NIORCA_OK;
}

static hipStream_t as_stream(void *s) { return (hipStream_t)s; }

extern "C" niorca_status niorca_count(niorca_ctx *ctx, int32_t n, int64_t nnz, const int64_t *row_ptr,
                                      const int32_t *col, int64_t *out, void *stream, uint32_t flags) {
    niorca_status st = check_graph_args(ctx, n, nnz, row_ptr, col);
    if (st) return st;
    if (n > 0 && !out) return fail(ctx, NIORCA_EINVAL, "out is NULL");
    const uint32_t known =
        NIORCA_VALIDATE | NIORCA_BIN_DEGREE | NIORCA_BIN_MLP | NIORCA_COUNTERS | NIORCA_TIMING | NIORCA_INDUCED;
    if (flags & ~known) return fail(ctx, NIORCA_EINVAL, "unknown flag bits 0x%x", flags & ~known);
    if ((flags & NIORCA_BIN_MLP) && !ctx->mlp_dev)
        return fail(ctx, NIORCA_EINVAL, "NIORCA_BIN_MLP needs a cost model (niorca_set_cost_model)");
    if ((flags & NIORCA_BIN_MLP) && (flags & NIORCA_BIN_DEGREE))
        return fail(ctx, NIORCA_EINVAL, "choose one of NIORCA_BIN_MLP and NIORCA_BIN_DEGREE");
    Outputs o;
    o.psi = out;
    return run(ctx, n, nnz, row_ptr, col, o, as_stream(stream), flags, nullptr);
}

extern "C" niorca_status niorca_count_noalloc(niorca_ctx *ctx, int32_t n, int64_t nnz, const int64_t *row_ptr,
                                              const int32_t *col, int64_t *out, void *stream, uint32_t flags) {
    niorca_status st = check_graph_args(ctx, n, nnz, row_ptr, col);
    if (st) return st;
    if (n > 0 && !out) return fail(ctx, NIORCA_EINVAL, "out is NULL");
    const uint32_t known = NIORCA_VALIDATE | NIORCA_BIN_DEGREE | NIORCA_BIN_MLP | NIORCA_INDUCED;
    if (flags & ~known) return fail(ctx, NIORCA_EINVAL, "unknown or unsupported flag bits 0x%x", flags & ~known);
    if ((flags & NIORCA_BIN_MLP) && !ctx->mlp_dev)
        return fail(ctx, NIORCA_EINVAL, "NIORCA_BIN_MLP needs a cost model (niorca_set_cost_model)");
    if ((flags & NIORCA_BIN_MLP) && (flags & NIORCA_BIN_DEGREE))
        return fail(ctx, NIORCA_EINVAL, "choose one of NIORCA_BIN_MLP and NIORCA_BIN_DEGREE");
    HIP_TRY(hipSetDevice(ctx->device));
    char *sp = nullptr;
    HIP_TRY(scratch_address(ctx->device, &sp));
    Outputs o;
    o.psi = out;
    ctx->fixed_ws = sp;
    ctx->fixed_bytes = NIORCA_NOALLOC_BYTES;
    st = run(ctx, n, nnz, row_ptr, col, o, as_stream(stream), flags, nullptr);
    ctx->fixed_ws = nullptr;
    ctx->fixed_bytes = 0;
    return st;
}

extern "C" niorca_status niorca_edge_triangles(niorca_ctx *ctx, int32_t n, int64_t nnz, const int64_t *row_ptr,
                                               const int32_t *col, int32_t *tri, void *stream) {
    niorca_status st = check_graph_args(ctx, n, nnz, row_ptr, col);
    if (st) return st;
    if (nnz > 0 && !tri) return fail(ctx, NIORCA_EINVAL, "tri is NULL");
    Outputs o;
    o.tri = tri;
    return run(ctx, n, nnz, row_ptr, col, o, as_stream(stream), 0, nullptr);
}

extern "C" niorca_status niorca_edge_k4(niorca_ctx *ctx, int32_t n, int64_t nnz, const int64_t *row_ptr,
                                        const int32_t *col, int64_t *k4e, void *stream) {
    niorca_status st = check_graph_args(ctx, n, nnz, row_ptr, col);
    if (st) return st;
    if (nnz > 0 && !k4e) return fail(ctx, NIORCA_EINVAL, "k4e is NULL");
    Outputs o;
    o.ek4 = k4e;
    return run(ctx, n, nnz, row_ptr, col, o, as_stream(stream), RUN_EDGE_K4, nullptr);
}

extern "C" niorca_status niorca_k4(niorca_ctx *ctx, int32_t n, int64_t nnz, const int64_t *row_ptr,
                                   const int32_t *col, int64_t *k4, void *stream) {
    niorca_status st = check_graph_args(ctx, n, nnz, row_ptr, col);
    if (st) return st;
    if (n > 0 && !k4) return fail(ctx, NIORCA_EINVAL, "k4 is NULL");
    Outputs o;
    o.k4 = k4;
    return run(ctx, n, nnz, row_ptr, col, o, as_stream(stream), 0, nullptr);
}

extern "C" niorca_status niorca_fvars(niorca_ctx *ctx, int32_t n, int64_t nnz, const int64_t *row_ptr,
                                      const int32_t *col, int64_t *fvars, void *stream) {
    niorca_status st = check_graph_args(ctx, n, nnz, row_ptr, col);
    if (st) return st;
    if (n > 0 && !fvars) return fail(ctx, NIORCA_EINVAL, "fvars is NULL");
    Outputs o;
    o.fvars = fvars;
    return run(ctx, n, nnz, row_ptr, col, o, as_stream(stream), 0, nullptr);
}

// Packed batch -> one disjoint union: column ids local to graph g become global by
// adding vtx_off[g].  The slots of graph g are the contiguous range
// [row_ptr[vtx_off[g]], row_ptr[vtx_off[g+1]]), so one wave per graph streams it
// (coalesced, no per-row search).  An id outside [0, n_g) becomes -1, which the
// relabel pass refuses (bad_input); a graph whose slot range leaves [0, nnz] is
// skipped (the degree pass refuses its rows).
__global__ void k_localize(int32_t G, int64_t nnz, const int64_t *__restrict__ voff, const int64_t *__restrict__ rp,
                           const int32_t *__restrict__ col, int32_t *__restrict__ colg) {
    const int waves = gridDim.x * (blockDim.x / WAVE);
    const int wid = blockIdx.x * (blockDim.x / WAVE) + threadIdx.x / WAVE;
    for (int32_t g = wid; g < G; g += waves) {
        const int64_t v0 = voff[g], v1 = voff[g + 1];
        const int32_t base = (int32_t)v0, ng = (int32_t)(v1 - v0);
        const int64_t b = rp[v0], e = rp[v1];
        if (b < 0 || e < b || e > nnz) continue;
        for (int64_t s = b + lane_id(); s < e; s += WAVE) {
            const int32_t c = col[s];
            colg[s] = (c >= 0 && c < ng) ? c + base : -1;
        }
    }
}

static uint32_t f32_bits(float x) {
    uint32_t u;
    memcpy(&u, &x, sizeof u);
    return u;
}

static uint64_t mix64(uint64_t h, uint64_t v) {
    h ^= v + 0x9E3779B97F4A7C15ull + (h << 6) + (h >> 2);
    return h;
}

extern "C" niorca_status niorca_count_batched(niorca_ctx *ctx, int32_t num_graphs, const int64_t *vtx_off,
                                              int64_t nnz, const int64_t *row_ptr, const int32_t *col,
                                              int64_t *out, void *stream, uint32_t flags) {
    if (!ctx) return NIORCA_EINVAL;
    ctx->err.clear();
    if (num_graphs < 0) return fail(ctx, NIORCA_EINVAL, "num_graphs is negative");
    if (num_graphs == 0) return NIORCA_OK;
    if (!vtx_off) return fail(ctx, NIORCA_EINVAL, "vtx_off is NULL");
    const uint32_t known = NIORCA_VALIDATE | NIORCA_GRAPH_CAPTURE | NIORCA_TIMING | NIORCA_INDUCED;
    if (flags & ~known) return fail(ctx, NIORCA_EINVAL, "unknown or unsupported flag bits 0x%x", flags & ~known);
    const bool capture = (flags & NIORCA_GRAPH_CAPTURE) != 0;
    if (capture && (flags & (NIORCA_VALIDATE | NIORCA_TIMING)))
        return fail(ctx, NIORCA_EINVAL, "NIORCA_GRAPH_CAPTURE cannot be combined with VALIDATE or TIMING");
    if (capture && !stream) return fail(ctx, NIORCA_EINVAL, "NIORCA_GRAPH_CAPTURE needs a non-null stream");
    if (vtx_off[0] != 0) return fail(ctx, NIORCA_EINVAL, "vtx_off[0] must be 0");
    int64_t max_n = 0;
    uint64_t vh = 0;
    for (int32_t g = 0; g < num_graphs; g++) {
        int64_t ng = vtx_off[g + 1] - vtx_off[g];
        if (ng < 0) return fail(ctx, NIORCA_EINVAL, "vtx_off decreases at graph %d", g);
        if (ng > max_n) max_n = ng;
        vh = mix64(vh, (uint64_t)vtx_off[g + 1]);
    }
    const int64_t total = vtx_off[num_graphs];
    if (total >= ((int64_t)1 << 31)) return fail(ctx, NIORCA_ENOTIMPL, "more than 2^31 - 1 vertices in the batch");
    const int32_t n = (int32_t)total;
    niorca_status st = check_graph_args(ctx, n, nnz, row_ptr, col);
    if (st) return st;
    if (n > 0 && !out) return fail(ctx, NIORCA_EINVAL, "out is NULL");
    if (n == 0) return NIORCA_OK;
    hipStream_t s = as_stream(stream);
    HIP_TRY(hipSetDevice(ctx->device));
    // Bounds known on the host: no vertex has more than max_n - 1 neighbours.
    HostBounds hb{(int)(max_n - 1), (int)(max_n - 1)};
    if (hb.dplus_max > LSORT_CAP)
        return fail(ctx, NIORCA_ENOTIMPL, "a graph of %lld vertices exceeds the batched size limit %d",
                    (long long)max_n, LSORT_CAP + 1);
    Layout L;
    Arena A;
    layout_base(L, ctx, n, nnz, flags, A);
    layout_rest(L, ctx, n, nnz, hb.dmax, hb.dplus_max, BOUNDED_TRI_CACHE, true, A);
    L.colg = A.take<int32_t>(nnz + 64);
    L.voff = A.take<int64_t>(num_graphs + 1);
    st = ensure_ws(ctx, A.off);
    if (st) return st;
    int32_t *colg = (int32_t *)(ctx->ws + L.colg);
    int64_t *dvoff = (int64_t *)(ctx->ws + L.voff);
    HIP_TRY(hipMemcpyAsync(dvoff, vtx_off, sizeof(int64_t) * (num_graphs + 1), hipMemcpyHostToDevice, s));
    Outputs o;
    o.psi = out;
    const int cu = ctx->num_cu;
    if (!capture) {
        hipLaunchKernelGGL(k_localize, dim3(cu * 8), dim3(256), 0, s, num_graphs, nnz, dvoff, row_ptr, col, colg);
        HIP_TRY(hipGetLastError());
        return run(ctx, n, nnz, row_ptr, colg, o, s, flags, &hb);
    }
    // Replay the captured sequence when the call has the same shape and buffers.
    uint64_t key = 0;
    for (uint64_t v : {(uint64_t)n, (uint64_t)nnz, (uint64_t)num_graphs, (uint64_t)(uintptr_t)row_ptr,
                       (uint64_t)(uintptr_t)col, (uint64_t)(uintptr_t)out, (uint64_t)(uintptr_t)ctx->ws,
                       ctx->ws_bytes, vh, (uint64_t)ctx->heavy_k, (uint64_t)ctx->tri_cache_records,
                       (uint64_t)ctx->th.tri_wave, (uint64_t)ctx->th.tri_block, (uint64_t)ctx->th.ql_wave,
                       (uint64_t)ctx->th.ql_block, (uint64_t)ctx->th.qh_wave, (uint64_t)ctx->th.qh_block,
                       (uint64_t)ctx->th.ql_split, (uint64_t)ctx->large_lds_max, (uint64_t)flags,
                       // binning: mode, degree bounds and the learned bounds are launch arguments too
                       (uint64_t)ctx->bin_default, (uint64_t)ctx->th.deg_thread, (uint64_t)ctx->th.deg_group,
                       (uint64_t)ctx->th.deg_block, (uint64_t)f32_bits(ctx->thr_thread),
                       (uint64_t)f32_bits(ctx->thr_group), (uint64_t)f32_bits(ctx->thr_block),
                       (uint64_t)(uintptr_t)ctx->mlp_dev})
        key = mix64(key, v);
    if (!ctx->gexec || ctx->gkey != key) {
        if (ctx->gexec) {
            (void)hipGraphExecDestroy(ctx->gexec);
            ctx->gexec = nullptr;
        }
        HIP_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
        hipLaunchKernelGGL(k_localize, dim3(cu * 8), dim3(256), 0, s, num_graphs, nnz, dvoff, row_ptr, col, colg);
        niorca_status rs = run(ctx, n, nnz, row_ptr, colg, o, s, flags & ~(uint32_t)NIORCA_GRAPH_CAPTURE, &hb);
        hipGraph_t graph = nullptr;
        hipError_t ce = hipStreamEndCapture(s, &graph);
        if (rs != NIORCA_OK) {
            if (graph) (void)hipGraphDestroy(graph);
            return rs;
        }
        if (ce != hipSuccess) return fail(ctx, NIORCA_EDEVICE, "hipStreamEndCapture: %s", hipGetErrorString(ce));
        hipError_t ie = hipGraphInstantiate(&ctx->gexec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (ie != hipSuccess) {
            ctx->gexec = nullptr;
            return fail(ctx, NIORCA_EDEVICE, "hipGraphInstantiate: %s", hipGetErrorString(ie));
        }
        ctx->gkey = key;
    }
    HIP_TRY(hipGraphLaunch(ctx->gexec, s));
    return NIORCA_OK;
}

extern "C" niorca_status niorca_work_counters(niorca_ctx *ctx, int32_t n, int64_t *counters, void *stream) {
    if (!ctx) return NIORCA_EINVAL;
    if (!counters && n > 0) return fail(ctx, NIORCA_EINVAL, "counters is NULL");
    if (ctx->last_n != n || !ctx->last_counters || ctx->last_ws != ctx->ws)
        return fail(ctx, NIORCA_EINVAL, "the last count on this context did not record counters for n = %d", n);
    if (n == 0) return NIORCA_OK;
    HIP_TRY(hipSetDevice(ctx->device));
    int64_t tot = (int64_t)n * NUM_COUNTERS;
    hipLaunchKernelGGL(k_rows_to_input<i64>, dim3((u32)((tot + 255) / 256)), dim3(256), 0, as_stream(stream), n,
                       NUM_COUNTERS, (const u32 *)(ctx->ws + ctx->last_order),
                       (const i64 *)(ctx->ws + ctx->last_counters), counters);
    HIP_TRY(hipGetLastError());
    return NIORCA_OK;
}

extern "C" niorca_status niorca_last_features(niorca_ctx *ctx, int32_t n, float *features, void *stream) {
    if (!ctx) return NIORCA_EINVAL;
    if (!features && n > 0) return fail(ctx, NIORCA_EINVAL, "features is NULL");
    if (ctx->last_n != n || !ctx->last_feat || ctx->last_ws != ctx->ws)
        return fail(ctx, NIORCA_EINVAL, "the last count on this context did not compute features for n = %d", n);
    if (n == 0) return NIORCA_OK;
    HIP_TRY(hipSetDevice(ctx->device));
    int64_t tot = (int64_t)n * 6;
    hipLaunchKernelGGL(k_rows_to_input<float>, dim3((u32)((tot + 255) / 256)), dim3(256), 0, as_stream(stream), n,
                       6, (const u32 *)(ctx->ws + ctx->last_order), (const float *)(ctx->ws + ctx->last_feat),
                       features);
    HIP_TRY(hipGetLastError());
    return NIORCA_OK;
}

static uint64_t splitmix64(uint64_t *x) {
    uint64_t z = (*x += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

struct DevBufs {
    std::vector<void *> p;
    ~DevBufs() {
        for (void *q : p) (void)hipFree(q);
    }
    template <typename T>
    T *get(int64_t count) {
        void *q = nullptr;
        if (hipMalloc(&q, sizeof(T) * (count > 0 ? count : 1)) != hipSuccess) return nullptr;
        p.push_back(q);
        return (T *)q;
    }
};

extern "C" niorca_status niorca_mlp_train(niorca_ctx *ctx, const float *X, const float *y, int64_t N, int32_t epochs,
                                          int32_t batch, float lr, uint64_t seed, float *model, double *mse,
                                          void *stream) {
    if (!ctx) return NIORCA_EINVAL;
    ctx->err.clear();
    if (N <= 0 || !X || !y || !model || epochs < 0 || batch <= 0 || batch > (1 << 20) || !(lr > 0.0f) ||
        N >= ((int64_t)1 << 31))
        return fail(ctx, NIORCA_EINVAL, "bad training arguments");
    HIP_TRY(hipSetDevice(ctx->device));
    hipStream_t s = as_stream(stream);
    const int nall = mlp_num_all(), ntr = mlp_num_trained();
    DevBufs B;
    float *P = B.get<float>(nall), *grad = B.get<float>(ntr), *m1 = B.get<float>(ntr), *m2 = B.get<float>(ntr);
    float *A1 = B.get<float>((int64_t)batch * 32), *A2 = B.get<float>((int64_t)batch * 32);
    float *D1 = B.get<float>((int64_t)batch * 32), *D2 = B.get<float>((int64_t)batch * 32);
    float *G3 = B.get<float>(batch), *lossp = B.get<float>(batch), *pred = B.get<float>(N);
    int32_t *idx = B.get<int32_t>(N);
    const int nblocks = 512;
    double *part = B.get<double>(nblocks * 12);
    float *ys = B.get<float>(N), *ms = B.get<float>(2);
    if (!P || !grad || !m1 || !m2 || !A1 || !A2 || !D1 || !D2 || !G3 || !lossp || !pred || !idx || !part || !ys ||
        !ms)
        return fail(ctx, NIORCA_ENOMEM, "training buffers");
    // seeded initialisation: uniform(-a, a), a = sqrt(6 / fan_in); zero biases
    std::vector<float> h(nall, 0.0f);
    uint64_t rs = seed;
    auto uni = [&](float a) { return (float)((double)(splitmix64(&rs) >> 11) * (1.0 / 9007199254740992.0) * 2.0 - 1.0) * a; };
    for (int i = 0; i < 32 * 6; i++) h[i] = uni(sqrtf(6.0f / 6.0f));
    for (int i = 0; i < 32 * 32; i++) h[224 + i] = uni(sqrtf(6.0f / 32.0f));
    for (int i = 0; i < 32; i++) h[1280 + i] = uni(sqrtf(6.0f / 32.0f));
    HIP_TRY(hipMemcpyAsync(P, h.data(), sizeof(float) * nall, hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemsetAsync(m1, 0, sizeof(float) * ntr, s));
    HIP_TRY(hipMemsetAsync(m2, 0, sizeof(float) * ntr, s));
    HIP_TRY(mlp_feature_stats(N, X, part, nblocks, P, s));
    // training runs on standardised targets; the output layer is rescaled at the end
    HIP_TRY(mlp_standardise_targets(N, y, part, nblocks, ms, ys, s));
    std::vector<int32_t> perm(N);
    int step = 0;
    for (int ep = 0; ep < epochs; ep++) {
        for (int64_t i = 0; i < N; i++) perm[i] = (int32_t)i;
        for (int64_t i = N - 1; i > 0; i--) {
            int64_t j = (int64_t)(splitmix64(&rs) % (uint64_t)(i + 1));
            std::swap(perm[i], perm[j]);
        }
        HIP_TRY(hipMemcpyAsync(idx, perm.data(), sizeof(int32_t) * N, hipMemcpyHostToDevice, s));
        HIP_TRY(hipStreamSynchronize(s));  // perm is reused by the next epoch
        for (int64_t b0 = 0; b0 + batch <= N || (b0 == 0 && N < batch); b0 += batch) {
            int32_t bs = (int32_t)(N < batch ? N : batch);
            HIP_TRY(mlp_train_step(bs, idx + b0, X, ys, P, A1, A2, D1, D2, G3, lossp, grad, m1, m2, lr, ++step, s));
            if (N < batch) break;
        }
    }
    HIP_TRY(mlp_fold_output(P, ms, s));
    HIP_TRY(mlp_predict(N, X, P, pred, s));
    HIP_TRY(mlp_sse(N, pred, y, part, nblocks, s));
    std::vector<double> hp(nblocks);
    HIP_TRY(hipMemcpyAsync(hp.data(), part, sizeof(double) * nblocks, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(model, P, sizeof(float) * nall, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    double sse = 0;
    for (double v : hp) sse += v;
    if (mse) *mse = sse / (double)N;
    return NIORCA_OK;
}

extern "C" niorca_status niorca_mlp_predict(niorca_ctx *ctx, const float *model, const float *X, int64_t N,
                                            float *pred, void *stream) {
    if (!ctx) return NIORCA_EINVAL;
    ctx->err.clear();
    if (N < 0 || !model || (N > 0 && (!X || !pred))) return fail(ctx, NIORCA_EINVAL, "bad prediction arguments");
    if (N == 0) return NIORCA_OK;
    HIP_TRY(hipSetDevice(ctx->device));
    hipStream_t s = as_stream(stream);
    DevBufs B;
    float *P = B.get<float>(mlp_num_all());
    if (!P) return fail(ctx, NIORCA_ENOMEM, "model buffer");
    HIP_TRY(hipMemcpyAsync(P, model, sizeof(float) * mlp_num_all(), hipMemcpyHostToDevice, s));
    HIP_TRY(mlp_predict(N, X, P, pred, s));
    HIP_TRY(hipStreamSynchronize(s));  // P is freed on return
    return NIORCA_OK;
}

extern "C" niorca_status niorca_stage_times(niorca_ctx *ctx, float *ms, int32_t count) {
    if (!ctx || !ms || count < NIORCA_NUM_STAGES) return fail(ctx, NIORCA_EINVAL, "need %d floats", NIORCA_NUM_STAGES);
    if (!ctx->ev_valid) return fail(ctx, NIORCA_EINVAL, "the last call did not record stage times");
    HIP_TRY(hipEventSynchronize(ctx->ev[NIORCA_NUM_STAGES]));
    for (int i = 0; i < NIORCA_NUM_STAGES; i++) HIP_TRY(hipEventElapsedTime(&ms[i], ctx->ev[i], ctx->ev[i + 1]));
    return NIORCA_OK;
}

extern "C" niorca_status niorca_kernel_times(niorca_ctx *ctx, float *ms, int32_t count) {
    if (!ctx || !ms || count < NIORCA_NUM_KERNEL_TIMES)
        return fail(ctx, NIORCA_EINVAL, "need %d floats", NIORCA_NUM_KERNEL_TIMES);
    if (!ctx->ev_valid) return fail(ctx, NIORCA_EINVAL, "the last call did not record kernel times");
    HIP_TRY(hipEventSynchronize(ctx->ev[NIORCA_NUM_STAGES]));
    // events 0..4 bracket the Stage I/II launches, 5..12 the 4-cycle launches, 13..14
    // the sixteen-lane Stage I launch
    static const int first[NIORCA_NUM_KERNEL_TIMES] = {0, 1, 2, 3, 5, 6, 7, 8, 9, 10, 11, 13};
    for (int i = 0; i < NIORCA_NUM_KERNEL_TIMES; i++)
        HIP_TRY(hipEventElapsedTime(&ms[i], ctx->kev[first[i]], ctx->kev[first[i] + 1]));
    return NIORCA_OK;
}

extern "C" niorca_status niorca_device_status(niorca_ctx *ctx, void *stream) {
    if (!ctx) return NIORCA_EINVAL;
    ctx->err.clear();
    // the last call's statistics: in the context's workspace, or in the fixed scratch
    // after niorca_count_noalloc (until the next call on the device overwrites it)
    char *sp = nullptr;
    if (ctx->last_ws && ctx->last_ws != ctx->ws && scratch_address(ctx->device, &sp) == hipSuccess &&
        ctx->last_ws != sp)
        return NIORCA_OK;
    if (!ctx->last_ws) return NIORCA_OK;  // nothing counted yet
    HIP_TRY(hipSetDevice(ctx->device));
    hipStream_t s = as_stream(stream);
    GraphStats hs;
    HIP_TRY(hipMemcpyAsync(&hs, ctx->last_ws + ctx->last_stats_dev, sizeof hs, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (hs.bad_input)
        return fail(ctx, NIORCA_EINVAL, "row_ptr or col held values outside the graph or its degree bound");
    if (hs.err) return fail(ctx, NIORCA_EINTERNAL, "an equation's numerator that must be even was odd");
    return NIORCA_OK;
}

extern "C" niorca_status niorca_load_tuning(niorca_ctx *ctx, const char *path, const char *key) {
    if (!ctx) return NIORCA_EINVAL;
    ctx->err.clear();
    if (!path || !key) return fail(ctx, NIORCA_EINVAL, "path or key is NULL");
    FILE *f = fopen(path, "r");
    if (!f) return fail(ctx, NIORCA_EINVAL, "cannot read %s", path);
    char line[512];
    int applied = 0;
    niorca_status st = NIORCA_OK;
    while (st == NIORCA_OK && fgets(line, sizeof line, f)) {
        char *hash = strchr(line, '#');
        if (hash) *hash = 0;
        char k[128], name[128];
        long long v;
        if (sscanf(line, "%127s %127s %lld", k, name, &v) != 3 || strcmp(k, key) != 0) continue;
        st = niorca_set_param(ctx, name, (int64_t)v);
        applied++;
    }
    fclose(f);
    if (st) return st;
    if (!applied) return fail(ctx, NIORCA_EINVAL, "no entry for %s in %s", key, path);
    return NIORCA_OK;
}

extern "C" niorca_status niorca_class_stats(niorca_ctx *ctx, int64_t *out, int32_t count) {
    if (!ctx || !out || count < 3 * WC_COUNT) return fail(ctx, NIORCA_EINVAL, "need %d int64", 3 * WC_COUNT);
    if (ctx->last_n < 0 || ctx->last_ws != ctx->ws) return fail(ctx, NIORCA_EINVAL, "no count to report on");
    GraphStats hs;
    HIP_TRY(hipDeviceSynchronize());
    HIP_TRY(hipMemcpy(&hs, ctx->ws + ctx->last_stats_dev, sizeof hs, hipMemcpyDeviceToHost));
    for (int c = 0; c < WC_COUNT; c++) {
        out[c] = hs.cnt[c];
        out[WC_COUNT + c] = hs.work[c];
        out[2 * WC_COUNT + c] = hs.slots[c];
    }
    return NIORCA_OK;
}

extern "C" niorca_status niorca_set_cost_model(niorca_ctx *ctx, const float *weights, int32_t count,
                                               float thr_thread, float thr_group, float thr_block) {
    if (!ctx || !weights || count != NIORCA_MLP_PARAMS) return fail(ctx, NIORCA_EINVAL, "cost model needs %d floats", NIORCA_MLP_PARAMS);
    ctx->mlp.assign(weights, weights + count);
    ctx->thr_thread = thr_thread;
    ctx->thr_group = thr_group;
    ctx->thr_block = thr_block;
    HIP_TRY(hipSetDevice(ctx->device));
    if (!ctx->mlp_dev && hipMalloc((void **)&ctx->mlp_dev, sizeof(float) * NIORCA_MLP_PARAMS) != hipSuccess) {
        ctx->mlp_dev = nullptr;
        return fail(ctx, NIORCA_ENOMEM, "model buffer");
    }
    HIP_TRY(hipMemcpy(ctx->mlp_dev, weights, sizeof(float) * NIORCA_MLP_PARAMS, hipMemcpyHostToDevice));
    return NIORCA_OK;
}

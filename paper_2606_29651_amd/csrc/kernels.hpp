// Internal interfaces between the host API and the kernel files.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#ifndef __HIPCC_RTC__
#include "common.hpp"
#endif

// Statistics gathered on the device and read back once per count.
struct GraphStats {
    int dmax;        // largest degree
    int dplus_max;   // largest |N+|
    int err;         // device-side consistency flag (odd numerator)
    int pad;         // counter of long N+ rows queued for the workgroup sort
    int bad_input;   // row_ptr or col out of range (checked before any use)
    int pad2;
    long long pairs; // sum over vertices of C(|N+|, 2): a bound on the triangle count
    // work-class list sizes (filled by the classification kernel)
    int cnt[16];
    // per class: work units (Stage I probes or 4-cycle wedges) and row slots handled
    long long work[16];
    long long slots[16];
};

// Optional HIP events around each kernel launch of the probe and 4-cycle stages
// (NIORCA_TIMING): ev[k] before launch k, ev[k+1] after it.
struct KernelEvents {
    hipEvent_t *ev;   // nullptr: no events
};
#define NUM_KERNEL_SLOTS 15  // probe: thread, wave, block, large; q: ql wave, ql block,
                             // ql global, qh wave, qh block, qh dense, qh global, reduce;
                             // probe: group

// Classes of work items (indices into GraphStats::cnt and the list table).
enum WorkClass {
    WC_TRI_WAVE = 0,   // Stage I/II/tau, 2 <= |N+(u)| <= 64, one wave per vertex
    WC_TRI_THREAD,     // |N+(u)| <= 8 and little predicted work: one lane per vertex
    WC_TRI_BLOCK,      // 64 < |N+(u)| <= 512, one workgroup
    WC_TRI_LARGE,      // |N+(u)| > 512, one workgroup with global scratch
    WC_QL_WAVE,        // 4-cycles, u as largest vertex (u < h0), small hash per wave
    WC_QL_BLOCK,       // larger LDS hash per workgroup
    WC_QL_GLOBAL,      // dense counters in global scratch
    WC_QH_WAVE,        // 4-cycles, w opposite a heavy largest vertex, small hash per wave
    WC_QH_BLOCK,       // hash per workgroup
    WC_QH_DENSE,       // dense 16-bit LDS counters over the heavy range
    WC_QH_GLOBAL,      // heavy-range items of degree >= 2^16: int32 counters in global scratch
    WC_TRI_GROUP,      // |N+(u)| <= 16 and little predicted work: sixteen lanes per vertex
    WC_COUNT
};

struct ListPtrs {
    i32 *l[WC_COUNT];
};

// Runtime class thresholds (each at most the capacity of its kernel).
#define TRI_THREAD_CAP 8
struct Thresholds {
    int tri_wave;    // |N+| <= tri_wave -> wave class (<= TRI_WAVE_CAP)
    int tri_block;   // |N+| <= tri_block -> workgroup class (<= TRI_BLOCK_CAP)
    // work binning of the Stage I/II items that fit a wave (they never change a count):
    int bin_mode;    // 0 capacity only, 1 degree thresholds, 2 learned model
    int deg_thread;  // mode 1: degree <= deg_thread (and |N+| <= 8) -> one lane
    int deg_block;   // mode 1: degree >= deg_block -> one workgroup
    float thr_thread, thr_block;  // mode 2: predicted log2 work bounds of the same two classes
    const float *pred;            // mode 2: predictions by new id
    i64 ql_wave;     // wedges <= ql_wave -> wave hash (<= QL_WAVE_HC/2)
    i64 ql_block;    // wedges <= ql_block -> workgroup hash (<= QL_BLOCK_HC/2)
    i64 qh_wave;
    i64 qh_block;
    i64 ql_split;    // light workgroup items up to this many wedges use the small-table launch
    int deg_group;   // mode 1: degree <= deg_group (and |N+| <= 16) -> sixteen lanes
    float thr_group; // mode 2: predicted log2 work bound of the sixteen-lane class
};

#define NUM_COUNTERS 7   // per-vertex work counters (see include/niorca.h)

// Class capacities (shared by classification and kernels).
#define TRI_WAVE_CAP 64
#define TRI_GROUP_CAP 16
#define TRI_BLOCK_CAP 480  // 51 KB of LDS per workgroup item, so three share a CU's 160 KB
#define PB_GRID 3          // workgroups per CU of the Stage I/II workgroup kernel
#define PB_GRID_TAU 2      // ... and of its tau pass (more per CU measured no faster)
#define QL_WAVE_HC 4096     // largest hash per wave, light 4-cycle items (sized per launch)
#define QL_WAVE_DC 64       // segment (row slot) capacity per wave item
#define QL_BLOCK_HC 16384    // largest hash per workgroup, light 4-cycle items (sized per launch)
#define QH_WAVE_HC 4096     // largest packed (key, count) table per wave (sized per launch)
#define QH_BLOCK_HC 8192    // packed entries per workgroup
#define QH_PART_ROWS 64     // rows of heavy-key credits (8 per XCD)
#define QH_DENSE_K 32768    // size of the heavy key range (top-ranked vertices)
#define QH_DENSE_DC 4096    // middles accumulated in LDS by the dense kernel (else global)

// Per-vertex accumulators (new vertex ids), all int64[n].
struct Accum {
    i64 *St, *Stt, *Std, *Sd, *Sdd;  // neighbour sums of t, t^2, t*d(a), d(a), d(a)^2
    i64 *Tp;                         // pairs (T, psi1) per vertex: triangles at x, non-induced
                                     // 3-path ends (one 16-byte load per neighbour)
    i64 *tau;                        // sum over triangles at x of t(opposite edge)
    i64 *Q;                          // 4-cycles through x
    i64 *K4;                         // 4-cliques containing x
};

// Everything the counting kernels read about the relabelled graph.
struct DevGraph {
    i32 n;
    i32 nnz;
    i32 h0;                 // first id of the heavy range (top QH_DENSE_K ranks)
    const i32 *nrp;         // int32[n+1]
    const i32 *nsplit;      // int32[n]: first slot of N+(y)
    const i32 *ncol;        // int32[nnz]
    const i32 *mirror;      // int32[nnz]: for lower slots, slot of y inside N+(b)
    const i32 *hstart;      // int32[n]: first slot of N+(y) with id >= h0
    const u32 *ndeg;        // uint32[n]: degree by new id
    const u32 *order;       // uint32[n]: new id -> input id
    const i64 *wlight;      // int64[n]: 4-cycle wedges with y as largest (light) vertex
    const i64 *wheavy;      // int64[n]: 4-cycle wedges with y opposite a heavy largest vertex
    const int4 *vmeta;      // int4[n]: {nrp[y], nsplit[y], nrp[y+1], hstart[y]}, one line
                            // for kernels that visit y as some other vertex's neighbour
    const int2 *hseg;       // int2[nnz]: slot s of y (neighbour b) -> first and end slot of
                            // the heavy 4-cycle tops u > y in N+(b) (wedges y-b-u)
    const i32 *lbeg;        // int32[nnz]: lower slot s of y (neighbour b) -> row start of b
                            // (light wedges y-b-w, w < y, end at mirror[s])
    const i32 *dslot;       // int32[nnz]: slot s -> degree of its neighbour, so that the
                            // neighbour sums stream it instead of gathering it
};

enum { VM_BEGIN = 0, VM_NSPLIT = 1, VM_END = 2, VM_HSTART = 3 };
// One field of vmeta[v] (fields of one vertex share a cache line; loading only the
// fields used keeps registers free).
__device__ __forceinline__ i32 vmeta_at(const DevGraph &g, i32 v, int f) {
    return reinterpret_cast<const i32 *>(g.vmeta)[4 * (i64)v + f];
}

// prep.hip
i64 scan_ws_elems(i64 len);
i64 radix_ws_elems(i64 n);
hipError_t scan_u32_to_i32(const u32 *in, i64 len, i32 *out, i32 *ws, int write_total, hipStream_t s);
hipError_t scan_i32_to_i32(const i32 *in, i64 len, i32 *out, i32 *ws, int write_total, hipStream_t s);
hipError_t radix_sort_pairs(u32 *k, u32 *v, u32 *k2, u32 *v2, i64 n, int bits, i32 *hist, i32 *scan_ws,
                            hipStream_t s);
__global__ void k_degree(i32 n, i64 nnz, i64 dcap, const i64 *rp, u32 *deg, u32 *vals, GraphStats *st);
__global__ void k_invert(i32 n, const u32 *order, i32 *perm);
__global__ void k_relabel(i32 n, const i64 *rp, const i32 *col, const u32 *order, const i32 *perm,
                          const u32 *ndeg, const i32 *nrp, i32 *nsplit, i32 *ncol, int4 *vmeta, GraphStats *st);
__global__ void k_sort_upper_small(i32 n, const u32 *ndeg, const i32 *nrp, const i32 *nsplit, i32 *ncol,
                                   i32 *hstart, int4 *vmeta, i32 h0, i32 *longlist, i32 *longcount);
__global__ void k_sort_upper_large(const i32 *nrp, const i32 *nsplit, i32 *ncol, i32 *hstart, int4 *vmeta, i32 h0,
                                   const i32 *longlist, const i32 *longcount);
__global__ void k_mirror(i32 n, const u32 *ndeg, const i32 *nrp, const i32 *nsplit, const i32 *ncol,
                         const int4 *vmeta, i32 h0, i32 *mirror, int2 *hseg, i32 *lbeg, i32 *dslot, i64 *wlight,
                         i64 *wheavy, i64 *probes, float *feat);
#define LSORT_CAP 16384
#define LSORT_NT 512  // threads of the long-row sort
#define LSORT_GRID 2  // its workgroups per CU (64 KiB of LDS each)

// count.hip
hipError_t launch_classify(const DevGraph &g, const i64 *wl, const i64 *wh, const i64 *probes, const ListPtrs &lists,
                           GraphStats *st, const Thresholds &th, hipStream_t s);
struct TriCacheArgs {
    u64 *rec;
    i64 cap;
    u64 *bump;
    i64 *off;
    i32 *cnt;
    i64 chunk_wave, chunk_block, chunk_group;
};
hipError_t launch_probe(int mode, const DevGraph &g, i32 *const *lists_host, const GraphStats *st, i32 *t,
                        i64 *K4, i64 *tau, const TriCacheArgs &tca, char *large_scratch, i64 large_slice,
                        int large_cap, int large_hc, int large_blocks, i64 large_lds_max, int grid_wave,
                        int grid_block, i64 *counters, const KernelEvents &kev, hipStream_t s);

// mlp.hip
int mlp_num_trained();
int mlp_num_all();
hipError_t mlp_predict(i64 n, const float *X, const float *P, float *pred, hipStream_t s);
hipError_t mlp_feature_stats(i64 n, const float *X, double *part, int nblocks, float *P, hipStream_t s);
hipError_t mlp_train_step(i32 B, const i32 *idx, const float *X, const float *y, float *P, float *A1, float *A2,
                          float *D1, float *D2, float *G3, float *lossp, float *grad, float *m1, float *m2, float lr,
                          int step, hipStream_t s);
hipError_t mlp_sse(i64 n, const float *pred, const float *y, double *part, int nblocks, hipStream_t s);
hipError_t mlp_standardise_targets(i64 n, const float *y, double *part, int nblocks, float *ms, float *ys,
                                   hipStream_t s);
hipError_t mlp_fold_output(float *P, const float *ms, hipStream_t s);
hipError_t launch_sums(const DevGraph &g, const i32 *t, const Accum &acc, int grid, hipStream_t s);
hipError_t launch_solve(const DevGraph &g, const Accum &acc, i64 *out, i64 *fvars, GraphStats *st, int grid,
                        bool induced, hipStream_t s);
hipError_t launch_q(const DevGraph &g, i32 *const *lists_host, const GraphStats *st, i64 *Q, i32 *gscratch,
                    i64 gslice, int gblocks, int grid_wave, int grid_block, int grid_dense, i64 *part, int part_rows,
                    i64 ql_wave_bound, i64 ql_block_bound, i64 ql_split, i64 qh_wave_bound, i64 qh_block_bound,
                    const KernelEvents &kev, hipStream_t s);
i64 probe_large_slice_bytes(int cap, int hc, i64 lds_max);
#define PL_LDS_MAX (150 * 1024)  // largest dynamic LDS of the large probe kernel

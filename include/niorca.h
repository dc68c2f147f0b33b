/*
 * niorca.h -- C ABI of the MI355X (gfx950) library that counts, for every vertex
 * of an undirected simple graph, the 15 orbits of the non-induced connected
 * graphlets on 2 to 4 vertices.
 *
 * What is computed (Section 3, Definitions 3-5; Section 5): psi_k(x) is the number
 * of pairs (S, E') with S a set of 2..4 vertices containing x, E' a subset of the
 * edges of G inside S such that (S, E') is connected, and x in orbit k of (S, E').
 * Orbits: 0 edge end; 1, 2 end and middle of a 3-path; 3 triangle; 4, 5 end and
 * inner vertex of a 4-path; 6, 7 leaf and centre of a 3-star; 8 4-cycle; 9, 10,
 * 11 tail, degree-2 and degree-3 vertex of a tailed triangle; 12, 13 degree-2 and
 * degree-3 vertex of a diamond; 14 4-clique.
 *
 * Method (Algorithm 1): Stage I per-edge triangle counts, Stage II per-vertex
 * 4-clique counts (Algorithm 2 in spirit, run on a degree-ordered orientation),
 * Stage III the nine f-variables of Table 1 and the non-induced equations of
 * Section 5 and the Appendix, all in int64.
 *
 * Conventions shared by every entry point
 *   - Graph: CSR in DEVICE memory.  row_ptr is int64[n+1] with row_ptr[0] = 0 and
 *     row_ptr[n] = nnz; col is int32[nnz]; row v lists N(v) sorted ascending, with
 *     no self-loop, no duplicate, and (u in N(v)) <=> (v in N(u)).  nnz = 2|E|.
 *     The library never modifies the graph and keeps no pointer after a call.
 *   - Outputs are DEVICE buffers owned by the caller, written completely.
 *   - stream: a hipStream_t passed as void*; NULL means the null stream.  Work is
 *     enqueued on it; entry points return once the work is enqueued (they wait on
 *     the stream only where stated).  The caller synchronises before reading.
 *   - A context is single-threaded: calls on one context must not overlap in time
 *     (they share its workspace).  Different contexts are independent.
 *   - Errors: every entry point returns a niorca_status; on failure nothing has
 *     been enqueued unless stated, and niorca_last_error() describes the cause.
 *   - Malformed input: row bounds outside [0, nnz] and column ids outside [0, n)
 *     are detected on the device and never lead to a read or write outside the
 *     buffers (niorca_count refuses them with EINVAL; calls that do not wait report
 *     them through niorca_device_status).  The other preconditions (rows sorted,
 *     no duplicate, no self-loop, symmetric) are not checked unless NIORCA_VALIDATE
 *     is given; a graph violating them gets meaningless counts.
 *   - Size limits: n < 2^31, nnz < 2^31 (ENOTIMPL above), and every vertex has at
 *     most 16384 neighbours of higher degree rank |N+(v)| (ENOTIMPL above; a
 *     simple graph reaches it only with more than 1.3e8 edges, since |N+(v)| is at
 *     most sqrt(2|E|)).
 */
#ifndef NIORCA_H
#define NIORCA_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    NIORCA_OK = 0,
    NIORCA_EINVAL = 1,      /* bad argument: NULL pointer, negative or odd size, unknown flag */
    NIORCA_ENOTSIMPLE = 2,  /* NIORCA_VALIDATE found an unsorted/asymmetric/looped/duplicated CSR */
    NIORCA_EOVERFLOW = 3,   /* some count could exceed int64 for this degree sequence */
    NIORCA_ENOMEM = 4,      /* device workspace allocation failed or exceeded the cap */
    NIORCA_EDEVICE = 5,     /* a HIP runtime call failed */
    NIORCA_ENOTIMPL = 6,    /* a size beyond the supported range (e.g. nnz >= 2^31) */
    NIORCA_EINTERNAL = 7    /* a device-side consistency check failed */
} niorca_status;

/* Flags (bitmask). */
#define NIORCA_VALIDATE   0x1u  /* check the CSR precondition on the device; waits on the stream */
#define NIORCA_BIN_DEGREE 0x2u  /* Stage I work classes from degree thresholds */
#define NIORCA_BIN_MLP    0x4u  /* Stage I work classes from the loaded work model (niorca_set_cost_model) */
#define NIORCA_COUNTERS   0x8u  /* record per-vertex work counters (niorca_work_counters) */
#define NIORCA_TIMING     0x10u /* record HIP events between stages (niorca_stage_times) */
#define NIORCA_INDUCED    0x20u /* write the induced counts psi'_k instead (see niorca_count) */

typedef struct niorca_ctx niorca_ctx;

/* Create a context on HIP device `device`; it owns a grow-only device workspace.
 * Returns EINVAL for a NULL ctx pointer, EDEVICE if the device cannot be set. */
niorca_status niorca_create(niorca_ctx **ctx, int device);

/* Release the context and its workspace (waits for the device).  NULL-safe. */
void niorca_destroy(niorca_ctx *ctx);

/* Message for the last failure on this context ("" if none).  The pointer stays
 * valid until the next call on the context. */
const char *niorca_last_error(const niorca_ctx *ctx);

/* Cap on the workspace in bytes (0 = no cap).  Calls needing more fail with ENOMEM. */
niorca_status niorca_set_workspace_limit(niorca_ctx *ctx, uint64_t bytes);

/* Workspace bytes currently held by the context. */
uint64_t niorca_workspace_bytes(const niorca_ctx *ctx);

/* Tuning knobs of the work classes (they change which kernel shape handles a vertex,
 * never a count).  Names and ranges:
 *   "tri_wave"  1..64    vertices with |N+| up to this use one wave (Stage I/II, tau)
 *   "tri_block" 1..480   ... up to this one workgroup with LDS; above, one 1024-thread
 *                        workgroup per vertex (LDS where it fits, else global scratch)
 *   "ql_wave"   0..2048  4-cycle wedges (largest vertex light) up to this: wave hash
 *                        (default 512; the per-wave table is sized from it)
 *   "ql_block"  0..8192  ... up to this: workgroup hash (default 8192, table sized
 *                        from it); above: global counters
 *   "ql_split"  0..8192  the workgroup class runs in launches by wedge count:
 *                        up to ql_split, then windows doubling up to ql_block, each
 *                        with tables sized for its window (default 2048)
 *   "qh_wave"   0..2048  4-cycle wedges opposite a heavy largest vertex: wave hash
 *                        (default 512; the per-wave table is sized from it)
 *   "qh_block"  0..4096  ... workgroup hash (default 2048); above: dense LDS counters
 *   "heavy_k"   -1..32768 how many top-ranked vertices form the heavy range; -1
 *                        (default): 32768 when the maximum degree exceeds 8x the
 *                        mean degree, else 0; 4096 in niorca_count_batched
 *   "bin_mode"  0..2     work binning of calls whose flags ask for none, including the
 *                        intermediate entry points: 0 capacity only (default), 1 as
 *                        NIORCA_BIN_DEGREE, 2 as NIORCA_BIN_MLP (needs a cost model)
 *   "bin_deg_thread" (NIORCA_BIN_DEGREE) degree up to which a vertex with |N+| <= 8
 *               goes to the one-lane Stage I class (default 0: none)
 *   "bin_deg_group"  (NIORCA_BIN_DEGREE) degree up to which a vertex with |N+| <= 16
 *               (and not one-lane) goes to the sixteen-lane Stage I class (default 32)
 *   "bin_deg_block"  (NIORCA_BIN_DEGREE) degree from which a vertex goes to the
 *               workgroup Stage I class (default 2^30: none)
 *   "tri_cache" 0..2^34  most triangles kept from Stage I for the tau pass (8 bytes
 *                        each, default 2^32; a call reserves no more than the sum over
 *                        vertices of C(|N+|, 2); vertices whose triangles do not fit
 *                        are probed again)
 *   "large_lds" 0..153600 LDS bytes the |N+| > tri_block class may use (default
 *                        153600): hash and per-slot arrays, and for the 4-clique pass
 *                        a copy of the bitset of H_u when that fits too; what does not
 *                        fit lives in global scratch
 * Returns EINVAL for an unknown name or a value out of range. */
niorca_status niorca_set_param(niorca_ctx *ctx, const char *name, int64_t value);

/* The 15 orbit counts of every vertex (Algorithm 1, Section 5, Appendix).
 *   n        number of vertices, 0 <= n < 2^31 (n = 0 is a no-op returning OK)
 *   nnz      row_ptr[n] = 2|E|, even, < 2^31
 *   row_ptr  device int64[n+1]; col device int32[nnz] (see conventions)
 *   out      device int64[n*15], row-major: out[x*15 + k] = psi_k(x)
 *   flags    NIORCA_* bits
 * With NIORCA_INDUCED, out[x*15 + k] = psi'_k(x) instead: the counts of induced
 * graphlets (Section 3, Definition 2: one occurrence per connected vertex set S,
 * the subgraph of all edges inside S), same numbering.  They follow from the
 * non-induced counts of the same vertex by the triangular system relating them
 * (the section on ORCA and NI-ORCA prints three of its equations, e.g.
 * psi'_13 = f13_14 / 2 - 3 psi_14).
 * Waits once on `stream` to read a few graph statistics (degree maximum, work
 * class sizes) that size the launches and the overflow check; everything after
 * that is enqueued without waiting.  With NIORCA_VALIDATE it also waits at the end
 * and returns EINTERNAL if the device's evenness check of the halved equations
 * (Section 5: every halving is exact) failed; otherwise niorca_device_status
 * reports that check. */
niorca_status niorca_count(niorca_ctx *ctx, int32_t n, int64_t nnz, const int64_t *row_ptr,
                           const int32_t *col, int64_t *out, void *stream, uint32_t flags);

/* niorca_count for callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid hipMalloc): the same computation,
 * with the workspace in a fixed device array of NIORCA_NOALLOC_BYTES that the
 * library holds on every GPU it runs on until the process ends; the call makes no
 * hipMalloc, hipFree or other allocation.  Graphs whose workspace does not fit are
 * refused with ENOMEM, the message giving the size needed (about 12 bytes per CSR
 * slot and 300 per vertex, plus 16 MiB when the graph has hubs: 10^5 vertices with
 * 2x10^6 edges fit); Stage I triangles that do not fit the space left are probed
 * again in the tau pass, which changes no count.
 * Flags: VALIDATE, BIN_DEGREE, BIN_MLP, INDUCED (not TIMING or COUNTERS).  Every
 * call on a GPU shares that GPU's array, whatever the context: calls that overlap
 * in time on one GPU race and give wrong counts.  Afterwards niorca_device_status
 * reads the shared array (valid until the next call on the device), and the
 * per-vertex introspection calls (counters, features, class statistics) refuse. */
#define NIORCA_NOALLOC_BYTES (128ull << 20)
niorca_status niorca_count_noalloc(niorca_ctx *ctx, int32_t n, int64_t nnz, const int64_t *row_ptr,
                                   const int32_t *col, int64_t *out, void *stream, uint32_t flags);

/* Many small graphs in one call.  Graph g owns vertices vtx_off[g]..vtx_off[g+1]-1
 * of a packed CSR whose row_ptr is global (device int64[total_n+1], nnz = row_ptr[total_n])
 * and whose column ids are LOCAL to the graph (0..n_g-1); out is device
 * int64[total_n*15] in packed vertex order.  vtx_off is a HOST int64[num_graphs+1]
 * array with vtx_off[0] = 0; each graph has at most 16385 vertices.
 * The batch is counted as one disjoint union, one launch sequence for all graphs,
 * with launch sizes taken from host-known bounds (no row longer than the largest
 * graph's n - 1), so nothing waits on the device.  NIORCA_INDUCED as for
 * niorca_count.  With NIORCA_GRAPH_CAPTURE (non-null stream; not with VALIDATE or
 * TIMING) that sequence is captured once into a hipGraph and replayed by later calls
 * of the same shape (sizes, buffers, vtx_off, flags and tuning parameters).  A row
 * longer than the bound, a row bound outside [0, nnz] or a column id outside its
 * graph is refused on the device (that vertex is counted as isolated, nothing
 * outside the buffers is touched) and reported by niorca_device_status; unsorted,
 * duplicated or asymmetric rows give meaningless counts.  NIORCA_VALIDATE checks
 * the whole precondition first (and waits). */
#define NIORCA_GRAPH_CAPTURE 0x100u
niorca_status niorca_count_batched(niorca_ctx *ctx, int32_t num_graphs, const int64_t *vtx_off, int64_t nnz,
                                   const int64_t *row_ptr, const int32_t *col, int64_t *out,
                                   void *stream, uint32_t flags);

/* ---- Introspection: intermediate results of the last stages, same conventions ---- */

/* Stage I: tri[s] = |N(x) and N(y)| for the edge in input CSR slot s (Algorithm 1,
 * the tri array indexed by edge).  tri is device int32[nnz]. */
niorca_status niorca_edge_triangles(niorca_ctx *ctx, int32_t n, int64_t nnz, const int64_t *row_ptr,
                                    const int32_t *col, int32_t *tri, void *stream);

/* Stage II: k4[x] = number of 4-cliques containing x (Algorithm 2).  device int64[n]. */
niorca_status niorca_k4(niorca_ctx *ctx, int32_t n, int64_t nnz, const int64_t *row_ptr,
                        const int32_t *col, int64_t *k4, void *stream);

/* Per-edge Stage II: k4e[s] = number of 4-cliques containing both ends of the edge
 * in input CSR slot s (Algorithm 2 finds each 4-clique once; here it is credited to
 * its six edges).  These per-edge counts, with tri of niorca_edge_triangles, are
 * the per-edge inputs 5-vertex methods start from (Section 3, complexity of the
 * 4- and 5-vertex counts).  k4e is device int64[nnz], written completely. */
niorca_status niorca_edge_k4(niorca_ctx *ctx, int32_t n, int64_t nnz, const int64_t *row_ptr,
                             const int32_t *col, int64_t *k4e, void *stream);

/* Stage III-a: the nine f-variables of Table 1 per vertex, device int64[n*9] in the
 * order f12_14, f10_13, f13_14, f11_13, f5_8, f6_9, f9_12, f4_8, f8_12. */
niorca_status niorca_fvars(niorca_ctx *ctx, int32_t n, int64_t nnz, const int64_t *row_ptr,
                           const int32_t *col, int64_t *fvars, void *stream);

/* Waits on `stream` for the last call on this context and reports what its kernels
 * flagged: EINVAL if a row bound, a column id or a row length was outside the graph
 * or its bound (the vertex was counted as isolated), EINTERNAL if a halved equation
 * had an odd numerator (Section 5 says every halving is exact, so this means a
 * fault), OK otherwise (also when nothing was counted yet). */
niorca_status niorca_device_status(niorca_ctx *ctx, void *stream);

/* Applies the knobs stored under `key` in a tuning file through niorca_set_param.
 * The file is text, one "key name value" triple per line ('#' starts a comment), as
 * the package's autotuner writes it.  EINVAL if the file cannot be read, holds no
 * line for `key`, or a value is out of range (lines before it stay applied). */
niorca_status niorca_load_tuning(niorca_ctx *ctx, const char *path, const char *key);

/* Durations in ms, measured with HIP events on the call's stream, of the stages of
 * the last niorca_count made with NIORCA_TIMING; waits for that call to finish.
 *   0 degrees, rank sort, relabelled rows         1 statistics wait and setup
 *   2 N+ sort, mirror slots, work classes          3 zeroing of the accumulators
 *   4 Stage I + Stage II (probe kernels)           5 neighbour sums
 *   6 tau (probe kernels)                          7 4-cycles (light and heavy kernels)
 *   8 equations and output
 * ms must hold NIORCA_NUM_STAGES floats. */
#define NIORCA_NUM_STAGES 9
niorca_status niorca_stage_times(niorca_ctx *ctx, float *ms, int32_t count);

/* Durations in ms of the kernel launches of the last NIORCA_TIMING count, from HIP
 * events recorded around each launch on the call's stream (a launch with nothing to
 * do still appears, with its near-zero time).  ms holds NIORCA_NUM_KERNEL_TIMES floats:
 *   0 Stage I/II one-lane   1 Stage I/II wave   2 Stage I/II workgroup   3 Stage I/II large
 *   4 4-cycles light, wave  5 light, workgroup   6 light, global counters
 *   7 4-cycles heavy, wave  8 heavy, workgroup   9 heavy, dense LDS counters
 *   10 heavy, global counters and the heavy-key reduction
 *   11 Stage I/II sixteen-lane
 * Waits for the call to finish. */
#define NIORCA_NUM_KERNEL_TIMES 12
niorca_status niorca_kernel_times(niorca_ctx *ctx, float *ms, int32_t count);

/* Work classes of the last count: out HOST int64[3*NIORCA_NUM_CLASSES]: vertices per
 * class, then their work units (Stage I probes for the first four classes, 4-cycle
 * wedges for the others), then their row slots (|N+| for the first four, |N-| for the
 * light 4-cycle classes, degree for the heavy ones).  Class order: Stage I/II wave,
 * one-lane, workgroup, large; 4-cycles light wave, light workgroup, light global;
 * heavy wave, heavy workgroup, heavy dense, heavy global; Stage I/II sixteen-lane.
 * Waits for the device. */
#define NIORCA_NUM_CLASSES 12
niorca_status niorca_class_stats(niorca_ctx *ctx, int64_t *out, int32_t count);

/* Number of per-vertex work counters written by niorca_work_counters. */
#define NIORCA_NUM_COUNTERS 7
/* Per-vertex work of the last niorca_count on this context made with
 * NIORCA_COUNTERS: device int64[n*NIORCA_NUM_COUNTERS], in input vertex order:
 *   0 Stage I probes made from x (sum of |N+(v)| over v in N+(x))
 *   1 triangles found with x as lowest vertex
 *   2 bitset words scanned for the 4-cliques with x as lowest vertex
 *   3 4-cycle wedges with x as largest vertex (largest vertex below the heavy range)
 *   4 4-cycle wedges with x opposite a heavy largest vertex
 *   5 neighbour-sum slots read (2 d(x))
 *   6 shader-clock cycles of x's Stage I/II item (0 if x had no item)
 * Must follow that count directly (the next call reuses the workspace).  EINVAL if
 * the last count recorded no counters or had another n. */
niorca_status niorca_work_counters(niorca_ctx *ctx, int32_t n, int64_t *counters, void *stream);

/* The six cheap features of every vertex computed by the last niorca_count made with
 * NIORCA_COUNTERS or NIORCA_BIN_MLP: device float[n*6] in input vertex order,
 * log2(1 + .) of degree, |N+|, |N-|, neighbour-degree sum, Stage I probes and the
 * largest |N+(v)| over v in N+(x).  Same lifetime rule as niorca_work_counters. */
niorca_status niorca_last_features(niorca_ctx *ctx, int32_t n, float *features, void *stream);

/* Work model for NIORCA_BIN_MLP: an FP32 MLP 6 -> 32 -> 32 -> 1 (ReLU hidden layers)
 * predicting log2(1 + work) of a vertex's Stage I/II item from its six features.
 * weights is a HOST float array: W1[32][6], b1[32], W2[32][32], b2[32], W3[32], b3,
 * then the feature normalisation mean[6] and inv_std[6] (1325 floats).  Items that
 * fit one wave go to the one-lane class when |N+| <= 8 and the prediction is at
 * most thr_thread, else to the sixteen-lane class when |N+| <= 16 and the
 * prediction is at most thr_group, and to the workgroup class when the prediction
 * is at least thr_block; capacity limits always take precedence, so no count depends
 * on the model.  Copied into the context (and to the device); waits for the copy. */
#define NIORCA_MLP_PARAMS 1325
niorca_status niorca_set_cost_model(niorca_ctx *ctx, const float *weights, int32_t count, float thr_thread,
                                    float thr_group, float thr_block);

/* Train the work model with the library's FP32 kernels: Adam on the mean squared
 * error between the prediction and y, minibatches of `batch` rows drawn by a
 * seeded shuffle each epoch, seeded initialisation; reproducible for a given seed.
 * X device float[N*6] (features), y device float[N] (targets, e.g. log2(1 + cycles)),
 * model HOST float[1325] (output, normalisation included), mse HOST double (output,
 * final mean squared error over all rows; may be NULL).  Waits for completion. */
niorca_status niorca_mlp_train(niorca_ctx *ctx, const float *X, const float *y, int64_t N, int32_t epochs,
                               int32_t batch, float lr, uint64_t seed, float *model, double *mse, void *stream);

/* Predictions of a model (HOST float[1325]) for device features X[N*6] into device
 * pred[N].  Waits for completion. */
niorca_status niorca_mlp_predict(niorca_ctx *ctx, const float *model, const float *X, int64_t N, float *pred,
                                 void *stream);

#ifdef __cplusplus
}
#endif

#endif /* NIORCA_H */

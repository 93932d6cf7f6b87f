/*
 * hnv.h -- C ABI of the MI355X (gfx950) HyperNetVec refinement library.
 *
 * HyperNetVec (Maleki, Saless, Wall, Pingali, arXiv 2103.09660) embeds a
 * hypergraph H = (V, E) (Section 1) by coarsening it (Section 3.1,
 * Algorithm 1), embedding the coarsest level, and refining the embedding
 * level by level back to the finest (Section 3.3, Algorithm 2).  This library
 * runs the refinement on the GPU: per level, the projection of the coarser
 * embedding and repeated smoothing sweeps over the star expansion H*
 * (Section 1.1), plus the reverse mode of both.  Coarsening runs on the host
 * or on the GPU, with identical results, and a plan can be built from host or
 * from device-resident levels.
 *
 * Conventions used by every call
 *   - Star-expansion rows of a level: nodes first, then hyperedges.  Row v is
 *     node v, row n_nodes + e is hyperedge e.  rows = n_nodes + n_edges.
 *   - An embedding Z of a level is a row-major [rows x d] matrix of the
 *     plan's storage type (HNV_F32: float, HNV_BF16: bfloat16 bit patterns,
 *     round-to-nearest-even), 16-byte aligned, in device memory.
 *   - A hyperedge is a nonempty set of nodes (Section 1): its member list is
 *     strictly ascending.  Weights are finite and > 0; a NULL weight array
 *     means unit weights (Section 3.3 takes unit weights when none are given).
 *   - The star edge between node v and hyperedge e carries the weight w_e in
 *     both directions.  So a hyperedge row is relaxed towards the plain mean
 *     of its members and a node row towards the w-weighted mean of its
 *     hyperedges.
 *   - One sweep is the Jacobi form of Algorithm 2: every row reads the
 *     previous iterate; a row without neighbours keeps its value.
 *   - Every call returns an hnv_status; nothing aborts and no C++ exception
 *     crosses this boundary.  On failure hnv_last_error() describes it.
 *   - Device work is enqueued on the caller's HIP stream (hipStream_t passed
 *     as void*; NULL = the default stream) and is asynchronous unless stated.
 *     The library allocates no device memory: it carves the caller's
 *     workspace.  A plan is not thread-safe, and its device calls share
 *     scratch space in its workspace, so calls on one plan must not overlap
 *     on the device (one stream per plan, or streams ordered by events);
 *     distinct plans are independent and may run on different streams.
 */
#ifndef HNV_H
#define HNV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define HNV_ABI_VERSION 2

typedef enum {
    HNV_OK = 0,
    HNV_EINVAL = 1,        /* null pointer, negative size, bad parameter */
    HNV_ERANGE = 2,        /* an index or map entry out of range */
    HNV_EUNSORTED = 3,     /* a member list not strictly ascending */
    HNV_EUNSUPPORTED = 4,  /* a size or width outside what the kernels handle */
    HNV_EWORKSPACE = 5,    /* workspace too small or not 256-byte aligned */
    HNV_EDEVICE = 6,       /* a HIP runtime error (message has the HIP text) */
    HNV_ENOMEM = 7         /* host allocation failed */
} hnv_status;

typedef enum { HNV_F32 = 0, HNV_BF16 = 1 } hnv_dtype;

/* One hypergraph of the hierarchy, in HOST memory: the incidence of the
 * star expansion H* (Section 1.1) in both directions.
 * edge_ptr[n_edges+1] (edge_ptr[0] = 0, edge_ptr[n_edges] = nnz) and
 * edge_idx[nnz] list each hyperedge's members (node ids in [0, n_nodes),
 * strictly ascending): the CSR, hyperedge -> members.  edge_w[n_edges] or
 * NULL.  node_ptr[n_nodes+1] and node_idx[nnz] are the CSC, node -> its
 * hyperedges (each list strictly ascending), or both NULL: the library then
 * derives it from the CSR.  A CSC given by the caller is used by the plan
 * builders in place of the derived one and is always checked to be the
 * exact transpose of the CSR (HNV_EINVAL otherwise; only one of the two
 * pointers NULL is HNV_EINVAL too).  Coarsening ignores it.  Limits: nnz,
 * n_nodes + n_edges < 2^31. */
typedef struct {
    int64_t n_nodes;
    int64_t n_edges;
    int64_t nnz;
    const int64_t *edge_ptr;
    const int32_t *edge_idx;
    const float *edge_w;
    const int64_t *node_ptr;
    const int32_t *node_idx;
} hnv_level;

/* Coarsening maps from level l to level l+1, in HOST memory (Section 3.1:
 * rep(v) and rep(e)).  node_rep[n_nodes_l] in [0, n_nodes_{l+1});
 * edge_rep[n_edges_l] in [0, n_edges_{l+1}) or -1 for a hyperedge that was
 * removed because all of its members were merged into one coarse node. */
typedef struct {
    const int32_t *node_rep;
    const int32_t *edge_rep;
} hnv_map;

/* Tuning knobs; zero fields take the library's defaults. */
#define HNV_ORDER_JACOBI 0      /* every row reads the previous iterate (Algorithm 2 as written) */
#define HNV_ORDER_EDGE_FIRST 1  /* hyperedge rows first, then node rows from the new hyperedge rows */
typedef struct {
    int32_t panel_cols;  /* columns per pass of a forward sweep (divides d, multiple of 8) */
    int32_t small_max;   /* rows with at most this many neighbours go to a lane group (capped
                            at 4 lanes' worth of indices per lane of the group) */
    int32_t chunk;       /* neighbours per wavefront work item; longer rows are split */
    int32_t order;       /* HNV_ORDER_*: update order of a sweep (Section 3.3 describes both; the
                            edge-first order is the text's SOR reading, two half-sweeps that may
                            run in place; the reverse sweep follows the plan's order) */
} hnv_options;

typedef struct hnv_plan hnv_plan;

/* HNV_ABI_VERSION of the built library. */
int hnv_abi_version(void);

/* Message for the last non-OK status returned on this thread ("" if none).
 * The pointer stays valid until the next hnv_* call on this thread. */
const char *hnv_last_error(void);

/* Checks a level: offsets, index range, ascending unique member lists,
 * weights finite and > 0, size limits, and a CSC if one is given (the exact
 * transpose of the CSR).  Host only. */
hnv_status hnv_validate_level(const hnv_level *level);

/* One step of Algorithm 1 without node features (Section 3.1), on the host.
 * Each node v with hyperedges is assigned to c(v), the hyperedge of N(v)
 * with the largest weight, then the fewest members, then the lowest id (the
 * paper's featureless rule, which assigns by hyperedge weight or degree, with its
 * random tie-break replaced by a fixed order so the maps are reproducible).
 * Nodes with the same c(v) merge into one coarse node; a node without
 * hyperedges stays a node of its own.  Coarse node ids follow the smallest
 * fine node of each group.  A hyperedge all of whose members chose it is
 * removed (edge_rep = -1), every other hyperedge is kept in order with the
 * coarse member set {rep(v) : v in e} (ascending, repeats collapsed) and the
 * same weight.
 * Outputs (HOST, caller-allocated, sized for the fine level):
 *   node_rep[n_nodes], edge_rep[n_edges], c_edge_ptr[n_edges+1],
 *   c_edge_idx[nnz], c_edge_w[n_edges] (may be NULL if fine->edge_w is NULL);
 *   *c_n_nodes, *c_n_edges, *c_nnz receive the coarse sizes.
 * The input is validated first (errors as hnv_validate_level). */
hnv_status hnv_coarsen_level(const hnv_level *fine, int32_t *node_rep, int32_t *edge_rep,
                             int64_t *c_edge_ptr, int32_t *c_edge_idx, float *c_edge_w,
                             int64_t *c_n_nodes, int64_t *c_n_edges, int64_t *c_nnz);

/* The same coarsening step on the GPU, with the same maps and coarse level
 * bit for bit as hnv_coarsen_level (Section 3.1, Algorithm 1; the choice
 * c(v) is an atomic minimum of each hyperedge's rank in the key order, so it
 * does not depend on scheduling).  Arrays are in DEVICE memory with 32-bit
 * offsets, so that the output of one call is the input of the next:
 *   edge_ptr[n_edges+1] (int32), edge_idx[nnz], edge_w[n_edges] or NULL;
 *   outputs node_rep[n_nodes], edge_rep[n_edges], c_edge_ptr[n_edges+1],
 *   c_edge_idx[nnz], c_edge_w[n_edges] (may be NULL), sized for the fine
 *   level and owned by the caller; only the first c_n_edges+1 / c_nnz /
 *   c_n_edges entries of the coarse arrays are written.
 * c_sizes: HOST int64[3] receiving coarse n_nodes, n_edges, nnz.  The call
 * checks the input on the device (same statuses as hnv_validate_level),
 * enqueues the step's kernels behind the checks on `stream` and waits once,
 * for the checks' result and the sizes together, so it returns with the
 * outputs complete.  The kernels that follow the input's offsets or member
 * ids read the checks' result first and do nothing on invalid input, which
 * therefore leaves every access inside the given arrays; the outputs are
 * then unspecified.  workspace: DEVICE,
 * >= hnv_coarsen_workspace_bytes, 256-byte aligned; its contents need not
 * be initialised and are scratch afterwards.  Calls sharing a workspace on
 * different streams race.  The workspace size includes the temporary
 * storage of the GPU sorts and scans, which is queried from the device, so
 * hnv_coarsen_workspace_bytes needs a visible GPU (HNV_EDEVICE otherwise). */
hnv_status hnv_coarsen_workspace_bytes(int64_t n_nodes, int64_t n_edges, int64_t nnz, size_t *bytes);
hnv_status hnv_coarsen_level_device(int64_t n_nodes, int64_t n_edges, int64_t nnz, const int32_t *edge_ptr,
                                    const int32_t *edge_idx, const float *edge_w, int32_t *node_rep,
                                    int32_t *edge_rep, int32_t *c_edge_ptr, int32_t *c_edge_idx, float *c_edge_w,
                                    int64_t *c_sizes, void *workspace, size_t ws_bytes, void *stream);

/* The same step with node features (Section 3.1, Algorithm 1 with X):
 * ComputeEdgeFeature takes f(e) = the mean of the member rows of X;
 * AssignHyperedge takes c(v) = the hyperedge of N(v) with the largest cosine
 * of f(e) and f(v), and among equal scores the first in the featureless
 * order above (in place of the paper's random choice); the coarse feature
 * matrix X' gives each coarse node the sum of its fine nodes' rows (merged
 * bags of words).  Maps and coarse level as hnv_coarsen_level_device; this
 * step reads the input checks' result back before its feature kernels run
 * (two waits: the checks', then the sizes').
 *   x: DEVICE int32 [n_nodes x k], row-major, 16-byte aligned: counts >= 0
 *      whose total is below 2^31 (checked; HNV_EINVAL otherwise), k a
 *      multiple of 4 up to 65536 (pad with zero columns: they change no
 *      cosine and no sum).
 *   c_x: DEVICE int32 [n_nodes x k], 16-byte aligned: the first c_n_nodes
 *      rows receive X'.
 * The cosine is compared exactly as far as the arithmetic goes: member sums,
 * dot products d and squared norms |s_e|^2 are exact integers, the score
 * d|d| / |s_e|^2 (an increasing function of the cosine for a fixed node) is
 * evaluated in IEEE FP64 with one rounding per operation, and a hyperedge
 * with s_e = 0 scores 0.  workspace: >= hnv_coarsen_features_workspace_bytes. */
hnv_status hnv_coarsen_features_workspace_bytes(int64_t n_nodes, int64_t n_edges, int64_t nnz, int k,
                                                size_t *bytes);
hnv_status hnv_coarsen_level_features_device(int64_t n_nodes, int64_t n_edges, int64_t nnz,
                                             const int32_t *edge_ptr, const int32_t *edge_idx,
                                             const float *edge_w, const int32_t *x, int k, int32_t *node_rep,
                                             int32_t *edge_rep, int32_t *c_edge_ptr, int32_t *c_edge_idx,
                                             float *c_edge_w, int32_t *c_x, int64_t *c_sizes, void *workspace,
                                             size_t ws_bytes, void *stream);

/* Device workspace a plan over these levels needs, in bytes.  levels[0] is
 * the finest, levels[n_levels-1] the coarsest; maps[l] maps level l to l+1
 * (n_levels-1 entries, may be NULL if n_levels == 1).  d: embedding width,
 * a multiple of 8 up to 512.  opts may be NULL.  No level may have more rows
 * (n_nodes + n_edges) than levels[0]: the refinement keeps every level's
 * iterates in buffers of the finest level's size (HNV_EUNSUPPORTED
 * otherwise; coarsening never grows a level).  Host only. */
hnv_status hnv_plan_workspace_bytes(const hnv_level *levels, const hnv_map *maps, int n_levels,
                                    int d, hnv_dtype dtype, const hnv_options *opts, size_t *bytes);

/* Builds a plan: the star-expansion adjacency of every level in both
 * directions (Section 1.1: V* = V and E, with an edge between each
 * hyperedge and each of its members), the degree-tiered work lists, the row
 * maps of the projection (Section 3.3, last paragraph before Algorithm 2),
 * their inverse, and the FP64-computed reciprocals of the row weight sums
 * (the denominators of the neighbour mean in Section 3.3).
 * Everything is copied into `workspace` (device memory of ws_bytes >=
 * hnv_plan_workspace_bytes, 256-byte aligned, owned by the caller, must
 * outlive the plan).  The host arrays are not retained.  validate != 0 runs
 * hnv_validate_level on every level and checks the maps.  Synchronises
 * `stream` before returning. */
hnv_status hnv_plan_create(const hnv_level *levels, const hnv_map *maps, int n_levels, int d,
                           hnv_dtype dtype, const hnv_options *opts, int validate, void *workspace,
                           size_t ws_bytes, void *stream, hnv_plan **out);

/* A level in DEVICE memory with 32-bit offsets: the form the GPU coarsening
 * (hnv_coarsen_level_device) takes and returns.  Same meaning and limits as
 * hnv_level. */
typedef struct {
    int64_t n_nodes;
    int64_t n_edges;
    int64_t nnz;
    const int32_t *edge_ptr;   /* DEVICE [n_edges+1] */
    const int32_t *edge_idx;   /* DEVICE [nnz] */
    const float *edge_w;       /* DEVICE [n_edges] or NULL */
} hnv_level_dev;

/* The same plan built on the GPU from device-resident levels and maps (the
 * hnv_map pointers are then DEVICE pointers), so that coarsening, plan and
 * refinement never leave the device.  The plan is identical to the one
 * hnv_plan_create builds from host copies of the same levels: the same
 * adjacency, work lists in the same order, the same reciprocals, hence
 * bit-identical results from every call that takes a plan.
 * hnv_plan_workspace_bytes_device gives the workspace size from the level
 * sizes alone (no device reads; the work lists are sized at their upper
 * bounds, and the build's temporaries use the plan's scratch embedding when
 * it is large enough, else extra space after it).  No level may have more
 * rows than levels[0], as for hnv_plan_workspace_bytes.  The temporary storage of
 * the GPU sorts and scans is queried from the device, so both calls need a
 * visible GPU.  validate != 0 runs, on the device, the checks that
 * hnv_validate_level and hnv_plan_create(validate = 1) run; offsets, index
 * ranges and map ranges are always checked.  The level and map arrays are
 * read during the call only.  Synchronises `stream` once, before returning:
 * the checks' flags and the work-list sizes of every level are read back
 * together once the whole build is enqueued (the kernels that follow a
 * level's offsets, ids or map entries read its flags first and write empty
 * but well-formed arrays when a check failed). */
hnv_status hnv_plan_workspace_bytes_device(const hnv_level_dev *levels, const hnv_map *maps, int n_levels, int d,
                                           hnv_dtype dtype, const hnv_options *opts, size_t *bytes);
hnv_status hnv_plan_create_device(const hnv_level_dev *levels, const hnv_map *maps, int n_levels, int d,
                                  hnv_dtype dtype, const hnv_options *opts, int validate, void *workspace,
                                  size_t ws_bytes, void *stream, hnv_plan **out);

/* Frees the plan's host state; the workspace stays the caller's. */
hnv_status hnv_plan_destroy(hnv_plan *plan);

/* Sizes of one level of the plan (any pointer may be NULL). */
hnv_status hnv_plan_level_info(const hnv_plan *plan, int level, int64_t *n_nodes, int64_t *n_edges,
                               int64_t *nnz);

/* Replaces the hyperedge weights of one level with w_dev[n_edges] (DEVICE,
 * finite, > 0; not checked on the device) and recomputes the row
 * reciprocals 1 / sum_{e ∋ v} w_e in FP64 (Section 3.3: the weight w_uv of
 * a star edge normalised by the sum over the row's neighbours; a hyperedge
 * row's own weight cancels in its mean). */
hnv_status hnv_set_edge_weights(hnv_plan *plan, int level, const float *w_dev, void *stream);

/* As hnv_set_edge_weights with w = exp(theta): theta_dev[n_edges] DEVICE
 * log-weights (the learnable parameterisation); w_out_dev[n_edges] (DEVICE,
 * may be NULL) receives w. */
hnv_status hnv_set_edge_logweights(hnv_plan *plan, int level, const float *theta_dev,
                                   float *w_out_dev, void *stream);

/* Multi-level refinement (Section 3.3): starting from z_coarsest (DEVICE,
 * [rows of the coarsest level x d]), run sweeps_per_level[L] sweeps at the
 * coarsest level L, then for l = L-1 .. 0 project onto level l (a merged
 * node's row goes to every fine node of its set; a kept hyperedge takes
 * rep(e)'s row, a removed one its members' common coarse node row) and run
 * sweeps_per_level[l] sweeps.  The projection is fused into the first sweep
 * of a level.  Writes z_finest (DEVICE, [rows of level 0 x d]; must not
 * alias z_coarsest).
 *   sweeps_per_level: HOST [n_levels], index = level, each >= 0.
 *   omega: relaxation, 0 <= omega <= 1 (Algorithm 2).
 *   tol: <= 0 runs the fixed counts; > 0 also stops a level after the first
 *        sweep whose change ||Z^i - Z^{i-1}||_F is <= tol (Section 4 names a
 *        difference of epsilon between consecutive iterations as the
 *        alternative to a fixed count; the test is absolute, on the whole
 *        level's matrix, and ends that level only; the next finer level
 *        starts from the projection and runs its own sweeps).  The test is made
 *        on the device: once a level has stopped, its remaining sweeps return
 *        without work.  The host enqueues a level's sweeps in batches of 1,
 *        2, 4, .. 16 and reads the level's stop flag between batches (a few
 *        waits per level, none per sweep); while the stream is being
 *        captured into a HIP graph it enqueues every sweep and never waits
 *        (sweeps_done must then be NULL: HNV_EINVAL otherwise).
 *   residuals_dev: DEVICE double [sum of sweeps_per_level] or NULL; entry k
 *        receives ||Z^i - Z^{i-1}||_F of the k-th sweep run (coarsest level
 *        first), reduced in FP64 in a fixed order.  Entries past the last
 *        sweep run (when tol stops levels early) are left untouched.  With
 *        tol <= 0 the residuals of up to 8 consecutive sweeps of a level are
 *        reduced together after the last of them (same values); the entries
 *        are all written once the call's work on `stream` has completed.
 *   sweeps_done: HOST int32 [n_levels] or NULL: sweeps actually run.  With
 *        tol > 0 the counts are known on the device only, and a non-NULL
 *        sweeps_done makes the call wait for the stream to read them. */
hnv_status hnv_refine(hnv_plan *plan, const void *z_coarsest, void *z_finest,
                      const int32_t *sweeps_per_level, float omega, double tol,
                      double *residuals_dev, int32_t *sweeps_done, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the sweep of
 * hnv_sweep, with the same kernels and bit-identical results, whose scratch --
 * the FP32 partial sums of rows split over several wavefronts and, when
 * resid_dev is given, the per-block FP64 residual partials and their two
 * reduction buffers -- lives in a static device array of
 * HNV_NOALLOC_SCRATCH_BYTES instead of the plan's workspace.  Each GPU the
 * library runs on holds that array until the process ends; its address is
 * looked up once per device, on the first call with the device current.  The
 * call allocates nothing (no hipMalloc, no hipFree, no allocating library
 * routine) and enqueues only kernels.  A level whose sweep needs more scratch
 * than the array holds (reported in the message) returns HNV_EUNSUPPORTED;
 * hnv_sweep still serves it.  The array keeps the last call's contents and
 * nothing in it has to start cleared (every entry is written before it is
 * read).  Every call on one GPU shares that GPU's array: calls that overlap on
 * one GPU, from any plan or stream, race.  Arguments and the other statuses
 * as hnv_sweep. */
#define HNV_NOALLOC_SCRATCH_BYTES (64u * 1024u * 1024u)
hnv_status hnv_sweep_noalloc(hnv_plan *plan, int level, const void *z_in, void *z_out, float omega,
                             int from_coarse, double *resid_dev, void *stream);

/* Projection alone onto level `level` (< L): z_fine[u] = z_coarse[rowmap(u)]
 * (Section 3.3: the embedding of a coarse node is given to every fine node
 * merged into it; a kept hyperedge takes rep(e)'s row and a removed one the
 * row of the coarse node its members were merged into, Section 3.1). */
hnv_status hnv_project(hnv_plan *plan, int level, const void *z_coarse, void *z_fine, void *stream);

/* One sweep at `level` (Algorithm 2, one iteration).  If from_coarse != 0,
 * z_in is the embedding of level+1 and the sweep runs on its projection
 * (fused; equal to hnv_project then hnv_sweep).  z_out must not alias z_in,
 * except for an edge-first plan with from_coarse = 0 (in place).
 * resid_dev: DEVICE double[1] or NULL, receives ||z_out - z_start||_F. */
hnv_status hnv_sweep(hnv_plan *plan, int level, const void *z_in, void *z_out, float omega,
                     int from_coarse, double *resid_dev, void *stream);

/* Reverse mode of one sweep at `level` (from_coarse = 0), in the plan's
 * sweep order.  With y = z_prev (the sweep's input), z = z_cur (its output)
 * and g_in = dL/dz, writes g_out = dL/dy.  Jacobi order:
 *   node v:      (1-omega) g_v + omega sum_{e ∋ v} g_e / |e|
 *   hyperedge e: (1-omega) g_e + omega w_e sum_{v in e} g_v / S_v,
 *                S_v = sum_{e' ∋ v} w_e'
 *   rows without neighbours: g_out = g_in,
 * and if dw_accum != NULL adds dL/dw_e = omega sum_{v in e}
 * <g_v, y_e - zt_v> / S_v to dw_accum[e] (DEVICE float [n_edges]), where
 * zt_v = (z_v - (1-omega) y_v) / omega is node v's neighbour mean.
 * Edge-first order (hyperedge rows relaxed from the old node rows, then node
 * rows from the new hyperedge rows e'_e = z_e): with
 * ge_e = g_e + omega w_e sum_{v in e} g_v / S_v (= dL/de'_e),
 *   hyperedge e: (1-omega) ge_e
 *   node v:      (1-omega) g_v + omega sum_{e ∋ v} ge_e / |e|
 *   rows without neighbours: g_out = g_in,
 * and dL/dw_e = omega sum_{v in e} <g_v, e'_e - zt_v> / S_v, zt_v as above
 * (the mean of the new hyperedge rows).  This order uses the plan's scratch
 * embedding for ge.  Needs omega > 0.  All matrices [rows x d] of the plan's
 * storage type; g_out must not alias g_in.  With dw_accum = NULL, z_prev and
 * z_cur are not read. */
hnv_status hnv_sweep_adjoint(hnv_plan *plan, int level, const void *g_in, void *g_out,
                             const void *z_prev, const void *z_cur, float *dw_accum, float omega,
                             void *stream);

/* The same reverse sweep with the weight gradient split in two, for several
 * reverse sweeps in a row whose weight gradients add up.  The hyperedge part
 * omega <sum_{v in e} g_v / S_v, y_e> (e'_e in place of y_e in the
 * edge-first order) is added to dw_accum[e] (DEVICE float
 * [n_edges]) and the node part omega <g_v, zt_v> / S_v to node_accum[v]
 * (DEVICE float [n_nodes], zeroed by the caller before the first sweep).
 * hnv_weight_grad_finish then subtracts from every dw_accum[e] the sum of
 * node_accum over the members of e.  After the finish, dw_accum holds what
 * hnv_sweep_adjoint calls would have added over the same sweeps, up to
 * rounding; the node part is gathered per incidence once instead of in every
 * sweep.  g_out and the other arguments as hnv_sweep_adjoint. */
hnv_status hnv_sweep_adjoint_split(hnv_plan *plan, int level, const void *g_in, void *g_out,
                                   const void *z_prev, const void *z_cur, float *dw_accum, float *node_accum,
                                   float omega, void *stream);
hnv_status hnv_weight_grad_finish(hnv_plan *plan, int level, const float *node_accum, float *dw_accum,
                                  void *stream);

/* Reverse mode of the projection onto `level` (the transpose of the copy
 * rule of Section 3.3 quoted at hnv_project): g_coarse[r] = sum of g_fine[u]
 * over the fine rows u with rowmap(u) = r, summed in ascending u.  Coarse
 * rows with no preimage get 0. */
hnv_status hnv_project_adjoint(hnv_plan *plan, int level, const void *g_fine, void *g_coarse,
                               void *stream);

/* Chain rule for log-weights: dtheta[e] = w[e] * dw[e] with the level's
 * current weights (DEVICE float [n_edges] each; dtheta may alias dw). */
hnv_status hnv_logweight_grad(hnv_plan *plan, int level, const float *dw, float *dtheta, void *stream);

/* Kernel timing, for profiling and tracing.  While enabled, every launch of
 * a sweep's main kernel is bracketed by two hipEvents recorded on the
 * launch stream (a few microseconds of host time per launch).  Kinds:
 *   HNV_PROF_SWEEP     forward sweep (reads this level's previous iterate)
 *   HNV_PROF_FUSED     forward sweep fused with the projection
 *   HNV_PROF_ADJ_NODE  reverse sweep, node rows
 *   HNV_PROF_ADJ_EDGE  reverse sweep, hyperedge rows
 * enable = 0 stops recording and discards what was recorded. */
#define HNV_PROF_SWEEP 0
#define HNV_PROF_FUSED 1
#define HNV_PROF_ADJ_NODE 2
#define HNV_PROF_ADJ_EDGE 3
hnv_status hnv_plan_set_profiling(hnv_plan *plan, int enable);

/* Waits for the recorded events and returns, for one kind and one level
 * (level = -1: all levels), the number of launches and their summed
 * durations in milliseconds.  Host call; records are kept until
 * hnv_plan_set_profiling(plan, 0). */
hnv_status hnv_plan_profile_read(hnv_plan *plan, int kind, int level, int64_t *launches, double *total_ms);

/* Hyperedge-prediction features (Section 4, hyperedge prediction): for each
 * candidate node set c, out[c, :] = a per-dimension statistic of the member
 * rows z[v, :] (node embeddings of level 0):
 *   HNV_SCORE_VARIANCE  population variance (the paper's choice)
 *   HNV_SCORE_MEAN, HNV_SCORE_MIN, HNV_SCORE_MAX  the alternatives it names.
 * A score plan holds the candidates: cand_ptr[n_cand+1] (int64) and
 * cand_idx[cand_ptr[n_cand]] (int32) are HOST arrays listing each
 * candidate's members, ids in [0, z_rows) (checked: HNV_ERANGE otherwise).
 * The plan tiers the candidates by size like the sweep's rows and copies
 * itself into `workspace` (DEVICE, >= hnv_score_workspace_bytes, 256-byte
 * aligned, the caller's; it must outlive the plan), then synchronises
 * `stream`.  Scoring visits members in list order with Welford's FP32
 * update; partial results of long candidates are combined in a fixed
 * order, so the output is reproducible.  An empty candidate gets a row of
 * NaN. */
#define HNV_SCORE_VARIANCE 0
#define HNV_SCORE_MEAN 1
#define HNV_SCORE_MIN 2
#define HNV_SCORE_MAX 3
typedef struct hnv_score_plan hnv_score_plan;
hnv_status hnv_score_workspace_bytes(const int64_t *cand_ptr, int64_t n_cand, int d, hnv_dtype dtype,
                                     size_t *bytes);
hnv_status hnv_score_plan_create(const int64_t *cand_ptr, const int32_t *cand_idx, int64_t n_cand, int64_t z_rows,
                                 int d, hnv_dtype dtype, void *workspace, size_t ws_bytes, void *stream,
                                 hnv_score_plan **out);
hnv_status hnv_score_plan_destroy(hnv_score_plan *plan);
/* z: DEVICE [z_rows x d] of the plan's dtype, 16-byte aligned; out: DEVICE
 * float [n_cand x d], 16-byte aligned; op: HNV_SCORE_*. */
hnv_status hnv_score_candidates(hnv_score_plan *plan, const void *z, int op, float *out, void *stream);

/* The same score plan built on the GPU from DEVICE candidate arrays (for
 * candidates generated on the device): cand_ptr[n_cand+1] (int32, starts at
 * 0, never decreases, ends at n_members) and cand_idx[n_members], ids in
 * [0, z_rows) (checked on the device: HNV_EINVAL / HNV_ERANGE).  The work
 * lists are those hnv_score_plan_create builds, so the scores are
 * identical.  The workspace size comes from the sizes alone, with the work
 * lists at their upper bounds; its sort storage is queried from the device,
 * so hnv_score_workspace_bytes_device needs a visible GPU.  The candidate
 * arrays are read during the call only; the call synchronises `stream`. */
hnv_status hnv_score_workspace_bytes_device(int64_t n_cand, int64_t n_members, int d, hnv_dtype dtype,
                                            size_t *bytes);
hnv_status hnv_score_plan_create_device(const int32_t *cand_ptr, const int32_t *cand_idx, int64_t n_cand,
                                        int64_t n_members, int64_t z_rows, int d, hnv_dtype dtype, void *workspace,
                                        size_t ws_bytes, void *stream, hnv_score_plan **out);

/* Element-wise conversion between storage types on the device (FP32 ->
 * BF16 rounds to nearest even; BF16 -> FP32 is exact).  n elements. */
hnv_status hnv_cast(const void *src, hnv_dtype src_dtype, void *dst, hnv_dtype dst_dtype,
                    int64_t n, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* HNV_H */

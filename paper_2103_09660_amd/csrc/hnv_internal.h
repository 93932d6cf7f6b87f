// Internal declarations shared by the host code (hnv_host.cpp) and the HIP
// kernels (hnv_kernels.hip).  Not part of the public ABI.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "hnv.h"

typedef struct ihipStream_t *hipStream_t;

namespace hnv {

constexpr int kBlock = 256;   // threads per workgroup (4 wavefronts of 64)
constexpr int kWave = 64;
constexpr int kWavesPerBlock = kBlock / kWave;
#ifndef HNV_ROWS_PER_GROUP
#define HNV_ROWS_PER_GROUP 1
#endif
constexpr int kRowsPerGroup = HNV_ROWS_PER_GROUP;   // lane-group tier rows a group handles in turn

// A work item: `len` neighbours of side-local row `row` starting at `start`
// in the side's neighbour array.
//   lane-group tier: len = the row's degree, aux = the row of the next
//     coarser level its value is projected from (0 at the coarsest level);
//   wavefront tier: aux = -1 if the wavefront owns the whole row (len = its
//     degree), else the partial slot it writes; a finalize pass combines a
//     split row's slots in order.
struct alignas(16) Item {
    int32_t row, start, len, aux;
};
// The first kInlineIds neighbour ids of a lane-group row (unused entries 0),
// kept beside its work item so that a row of that many neighbours or fewer
// needs no load of its own index list.
constexpr int kInlineIds = 4;
struct alignas(16) InlineIds {
    int32_t id[kInlineIds];
};
// A row split over n_slots consecutive partial slots starting at first_slot.
struct alignas(16) Split {
    int32_t row, first_slot, n_slots, deg;
};

// One side of the star expansion of a level, as device arrays.
//   side 0: hyperedge rows, neighbours = member nodes (hyperedge->members)
//   side 1: node rows, neighbours = incident hyperedges (node->hyperedges)
struct DevSide {
    int32_t n_rows = 0;
    int32_t row_base = 0;            // Z row of local row 0 (n_nodes for side 0, 0 for side 1)
    const int32_t *ptr = nullptr;    // [n_rows + 1]
    const int32_t *idx = nullptr;    // [nnz] neighbour Z row at this level
    const int32_t *cidx = nullptr;   // [nnz] neighbour Z row at the next coarser level, or null
    float *wn = nullptr;             // [nnz] weight of each star edge (side 1 only)
    float *sn = nullptr;             // [nnz] reverse-mode scale: reciprocal of the neighbour's row sum
    const Item *small = nullptr;
    const InlineIds *small_ids = nullptr;    // [n_small] first ids of each small row, from idx
    const InlineIds *small_cids = nullptr;   // [n_small] the same from cidx, or null
    int32_t n_small = 0;
    const Item *chunks = nullptr;
    int32_t n_chunks = 0;
    const Split *splits = nullptr;
    int32_t n_splits = 0;
};

// Device-side state of a refinement that stops a level early (Section 3.3's
// epsilon rule) without reading residuals back on the host.  The sweeps and
// projections of such a refinement take their input and output matrices
// from here; the last kernel of each operation advances them, and the
// residual of each sweep is compared with tol on the device, setting the
// level's stop flag, after which that level's remaining sweeps do nothing.
struct SweepCtl {
    const void *cur;      // matrix holding the latest iterate
    void *next;           // buffer the next operation writes
    void *buf[2];         // the two buffers the refinement alternates between
    double *res;          // residual of each sweep run, packed in run order, or null
    double *res_tmp;      // [1] residual of the last sweep when res is null
    int32_t *stop;        // [n_levels] 1 once a sweep of the level changed Z by <= tol
    int32_t *done;        // [n_levels] sweeps run per level
    double tol;
    int64_t n_res;        // sweeps run so far (next index into res)
};

struct LevelPlan {
    int64_t n_nodes = 0, n_edges = 0, nnz = 0, rows = 0;
    int64_t rows_coarse = 0;         // rows of level + 1 (0 at the coarsest level)
    bool has_coarse = false;
    bool unit_w = true;
    bool scales_ready = false;       // the reverse-mode scales (side[*].sn) hold the current weights
    DevSide side[2];
    float *r = nullptr;              // [rows] 1 / (row weight sum), 0 for rows without neighbours
    float *w = nullptr;              // [n_edges] current hyperedge weights
    int32_t *rowmap = nullptr;       // [rows] -> row of level + 1
    int32_t *inv_ptr = nullptr;      // [rows_coarse + 1]
    int32_t *inv_idx = nullptr;      // [rows] fine rows grouped by coarse row, ascending
    int32_t n_slots = 0;             // partial slots used by split rows (both sides)
    // host copies of the work-list sizes (for launch geometry)
    int32_t n_small[2] = {0, 0}, n_chunks[2] = {0, 0}, n_splits[2] = {0, 0};
};

}  // namespace hnv

namespace hnv {
// Sweeps of one level whose residuals a fixed-count refinement reduces
// together (their per-block partials wait in as many slots).
constexpr int kResidBatch = 8;
}  // namespace hnv

struct hnv_plan {
    int n_levels = 0;
    int d = 0;
    hnv_dtype dtype = HNV_F32;
    hnv_options opts{};
    std::vector<hnv::LevelPlan> lv;
    void *zbuf = nullptr;            // scratch embedding [rows of level 0 x d]
    float *partials = nullptr;       // [max_slots x pstride]
    int32_t pstride = 0;             // floats per partial slot (d + 8)
    int64_t max_slots = 0;
    double *resid_part = nullptr;    // [kResidBatch x max_resid_blocks] per-block partials, one slot per sweep
    int64_t max_resid_blocks = 0;
    double *resid_stage = nullptr;   // [2 x kResidBatch x resid_stage_len] partial sums of the residual stages
    int64_t resid_stage_len = 0;
    float *cscratch = nullptr;       // [max n_nodes] per-node scalar of the reverse sweep
    double *resid_tmp = nullptr;     // [1]
    hnv::SweepCtl *ctl = nullptr;    // [1] early-stop control (device)
    int32_t *ctl_flags = nullptr;    // [2 x n_levels] its stop flags and sweep counts
    int panels = 1;                  // column passes of a forward sweep
    int dp = 0;                      // columns per pass
    int g_fwd = 1;                   // lanes per row in a forward pass
    int epl_fwd = 8;                 // elements per lane in a forward pass
    int g_full = 1;                  // lanes per full-width row
    int epl_full = 8;                // elements per lane of a full-width row
    int small_max = 0;               // effective lane-group tier bound
    size_t ws_bytes = 0;
    // kernel timing (hnv_plan_set_profiling)
    struct ProfRecord {
        int kind, level;
        void *ev_begin, *ev_end;   // hipEvent_t
    };
    bool profiling = false;
    std::vector<ProfRecord> prof;
    std::vector<void *> ev_pool;
    ~hnv_plan();
};

namespace hnv {

// thread-local error text
hnv_status fail(hnv_status st, const std::string &msg);
void clear_error();

int next_pow2(int x);
// Lane layout of a row slice of `cols` elements of `elem` bytes: lanes move
// 16 B each, or 32 B for FP32 slices of 128 columns or more.
void lane_layout(int cols, int elem, int *lanes, int *elems_per_lane);
constexpr int kIdxRegs = 4;          // neighbour indices a lane preloads in the lane-group tier
int64_t blocks_for(int64_t items, int64_t per_block);

// Sizes and work-list counts of one level of a plan.
struct LevelShape {
    int64_t nV = 0, nE = 0, nnz = 0, rows = 0, rows_c = 0;
    bool has_coarse = false, unit_w = true;
    int32_t n_small[2] = {0, 0}, n_chunks[2] = {0, 0}, n_splits[2] = {0, 0};
    int32_t n_slots = 0;
};

// Plan set-up shared by the host-built and the device-built plan
// (hnv_host.cpp): option defaults and limits, the plan's shape, and the
// workspace layout (base == nullptr: sizing only; sets p->ws_bytes).
void resolve_options(const hnv_options *in, int d, hnv_dtype dtype, hnv_options *out);
hnv_status check_plan_options(int d, hnv_dtype dtype, const hnv_options &o);
void init_plan_shape(hnv_plan *p, const std::vector<LevelShape> &shape, int d, hnv_dtype dtype,
                     const hnv_options &o);
void carve(hnv_plan *p, const std::vector<LevelShape> &shape, char *base);

// Forward-sweep launch geometry of a level (blocks per panel and finalize blocks).
void forward_geometry(const hnv_plan *p, const LevelPlan &L, int64_t *main_blocks, int64_t *fin_blocks);

// Device arrays of a candidate-scoring plan (carved from the caller's workspace)
struct ScorePlan {
    const int32_t *idx = nullptr;
    const Item *small = nullptr;
    int32_t n_small = 0;
    const Item *chunks = nullptr;
    int32_t n_chunks = 0;
    const Split *splits = nullptr;
    int32_t n_splits = 0;
    float *partials = nullptr;
};

constexpr int kScoreChunk = 512;     // members per wavefront work item of the scoring kernel

// Device-side pieces implemented in hnv_kernels.hip
hnv_status dev_recompute_reciprocals(hnv_plan *p, int level, void *stream);
// Fills both sides' small_ids / small_cids of a level of a host-built plan
// from its work items and neighbour arrays (the device-built plan fills them
// as it writes its work items).
hnv_status dev_fill_inline_ids(hnv_plan *p, int level, hipStream_t s);
hnv_status dev_check(const char *what);
hnv_status dev_score(const ScorePlan &sp, const void *z, hnv_dtype dtype, int d, int op, float *out,
                     hipStream_t s);

}  // namespace hnv

// A candidate-scoring plan: the device arrays above plus the sizes.
struct hnv_score_plan {
    hnv::ScorePlan sp;
    int64_t n_cand = 0, z_rows = 0;
    int d = 0;
    hnv_dtype dtype = HNV_F32;
};

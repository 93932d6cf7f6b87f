// Plan construction on the GPU from device-resident levels (the output of
// the GPU coarsening), producing the same plan as hnv_plan_create builds on
// the host, array for array:
//   side 0 (hyperedge rows): the member lists as given;
//   side 1 (node rows): each node's hyperedges in ascending id, from a stable
//     radix sort of the incidences by node;
//   projection row map, composed indices, inverse map (a stable sort of the
//     fine rows by coarse row);
//   degree tiers: rows of at most small_max neighbours ordered by degree
//     descending then row (a stable sort on small_max - degree), longer rows
//     cut into chunks laid out in row order and stably sorted longest first,
//     split rows with consecutive partial slots, side 0 before side 1;
//   weights and the FP64 reciprocals as for a host-built plan.
// The workspace is sized from the level sizes alone, with the work-list
// arrays at their upper bounds; the build's temporaries live in the plan's
// scratch embedding when it is large enough, else after the plan.
#include <hip/hip_runtime.h>

#include "hnv_prim.h"

#include <algorithm>
#include <climits>
#include <string>
#include <vector>

#include "hnv_internal.h"
#include "hnv_level_check.h"

namespace hnv {
namespace {

// ---------------------------------------------------------------------------
// kernels
// ---------------------------------------------------------------------------

// Map checks.  Flag bits: 4 node map range, 5 hyperedge map range, 6 a
// removed hyperedge without members, 7 (full) a removed hyperedge whose
// members lie in different coarse nodes.
__global__ __launch_bounds__(kThreads) void k_check_node_map(const int32_t *__restrict__ node_rep, int64_t n_nodes,
                                                             int64_t n_nodes_c, int *__restrict__ flag)
{
    const int64_t v = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (v < n_nodes && (node_rep[v] < 0 || node_rep[v] >= n_nodes_c))
        atomicOr(flag, 1 << 4);
}

// Runs after the level's own checks in the same stream and does nothing
// when they found bad offsets or member ids (level_flag bits 0 and 1), so
// every member it follows is in range.
__global__ __launch_bounds__(kThreads) void k_check_edge_map(const int32_t *__restrict__ ptr,
                                                             const int32_t *__restrict__ idx,
                                                             const int32_t *__restrict__ node_rep,
                                                             const int32_t *__restrict__ edge_rep, int64_t n_nodes,
                                                             int64_t n_edges, int64_t n_edges_c, int full,
                                                             const int *__restrict__ level_flag,
                                                             int *__restrict__ flag)
{
    const int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (e >= n_edges || (*level_flag & 3))
        return;
    const int32_t r = edge_rep[e];
    int bad = 0;
    if (r < -1 || r >= n_edges_c) {
        bad = 1 << 5;
    } else if (r == -1) {
        const int32_t a = ptr[e], b = ptr[e + 1];
        if (b == a) {
            bad = 1 << 6;
        } else if (full) {
            const int32_t first = node_rep[idx[a]];
            for (int32_t j = a + 1; j < b; ++j)
                if (node_rep[idx[j]] != first)
                    bad = 1 << 7;
        }
    }
    if (bad)
        atomicOr(flag, bad);
}

// A level without hyperedges: its offsets are the single 0 and it has no
// incidences (flag bit 0 otherwise).
__global__ void k_check_no_edges(const int32_t *__restrict__ ptr, int64_t nnz, int *__restrict__ flag)
{
    if (threadIdx.x == 0 && blockIdx.x == 0 && (ptr[0] != 0 || nnz != 0))
        atomicOr(flag, 1);
}

// One pass of a stable counting sort of (key, value) pairs by the digit
// (key >> shift) & mask, which is below n_bins <= kBinsMax: per-tile counts
// of every digit, an exclusive scan of the counts laid out digit-major
// (digit b of tile t at b * n_tiles + t), and a scatter in which each tile
// places its elements in input order.  The degree tiers of both sides need
// one pass (2 (small_max + 3) keys), the wavefront tier's chunk keys one pass
// while both sides' keys (2 chunk) fit in kBinsMax, else one per 10 bits;
// the result equals a stable radix sort's.  The number of pairs is n_max, or
// *n_dev when that is given (the grid is sized for n_max).  The values may
// be absent (null); a one-pass sort can also write each input element's
// sorted position (pos_out).
constexpr int kBinsMax = 1024;
constexpr int kBinBits = 10;   // digit width of the multi-pass form
constexpr int kBinRounds = 16;
constexpr int kBinTile = kThreads * kBinRounds;
constexpr int kBinWaves = kThreads / kWave;

__device__ inline int64_t pairs_of(int64_t n_max, const int64_t *n_dev)
{
    return n_dev ? min(n_max, *n_dev) : n_max;
}

__global__ __launch_bounds__(kThreads) void k_bin_count(const uint32_t *__restrict__ key, int64_t n_max,
                                                        const int64_t *__restrict__ n_dev, int shift, uint32_t mask,
                                                        int n_bins, int64_t n_tiles, int32_t *__restrict__ counts)
{
    __shared__ int32_t h[kBinsMax];
    for (int b = threadIdx.x; b < n_bins; b += kThreads)
        h[b] = 0;
    __syncthreads();
    const int64_t n = pairs_of(n_max, n_dev);
    const int64_t base = (int64_t)blockIdx.x * kBinTile;
    for (int k = 0; k < kBinRounds; ++k) {
        const int64_t i = base + (int64_t)k * kThreads + threadIdx.x;
        if (i < n)
            atomicAdd(&h[(key[i] >> shift) & mask], 1);
    }
    __syncthreads();
    for (int b = threadIdx.x; b < n_bins; b += kThreads)
        counts[(int64_t)b * n_tiles + blockIdx.x] = h[b];
}

// The lanes of the wavefront that hold the same key (active lanes only):
// one ballot per key bit.  Every lane of the wavefront must call it.
__device__ inline uint64_t same_key_lanes(uint32_t key, int bits, bool active)
{
    uint64_t m = __ballot(active);
    for (int b = 0; b < bits; ++b) {
        const bool one = (key >> b) & 1u;
        const uint64_t ones = __ballot(active && one);
        m &= one ? ones : ~ones;
    }
    return m;
}

// Round k of a tile places elements base + k * kThreads + [0, kThreads):
// an element goes to the next free position of its key, after the elements
// of the same key in lower lanes of its wavefront and in lower wavefronts.
__global__ __launch_bounds__(kThreads) void k_bin_scatter(const uint32_t *__restrict__ key,
                                                          const int32_t *__restrict__ val, int64_t n_max,
                                                          const int64_t *__restrict__ n_dev, int shift,
                                                          uint32_t mask, int n_bins, int bits, int64_t n_tiles,
                                                          const int32_t *__restrict__ offs,
                                                          uint32_t *__restrict__ key_out,
                                                          int32_t *__restrict__ val_out,
                                                          int32_t *__restrict__ pos_out)
{
    __shared__ int32_t next[kBinsMax];
    __shared__ int32_t wcount[kBinWaves][kBinsMax];
    for (int b = threadIdx.x; b < n_bins; b += kThreads) {
        next[b] = offs[(int64_t)b * n_tiles + blockIdx.x];
        for (int w = 0; w < kBinWaves; ++w)
            wcount[w][b] = 0;
    }
    __syncthreads();
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (kWave - lane));
    const int64_t n = pairs_of(n_max, n_dev);
    const int64_t base = (int64_t)blockIdx.x * kBinTile;
    for (int k = 0; k < kBinRounds && base + (int64_t)k * kThreads < n; ++k) {   // uniform over the block
        const int64_t i = base + (int64_t)k * kThreads + threadIdx.x;
        const bool act = i < n;
        const uint32_t kv = act ? key[i] : 0u;
        const uint32_t dg = (kv >> shift) & mask;
        const uint64_t peers = same_key_lanes(dg, bits, act);
        const int rank = __popcll(peers & below);
        if (act && rank == 0)
            wcount[wave][dg] = __popcll(peers);
        __syncthreads();
        if (act) {
            int32_t pos = next[dg] + rank;
            for (int w = 0; w < wave; ++w)
                pos += wcount[w][dg];
            key_out[pos] = kv;
            if (val_out)
                val_out[pos] = val[i];
            if (pos_out)
                pos_out[i] = pos;
        }
        __syncthreads();
        for (int b = threadIdx.x; b < n_bins; b += kThreads) {
            int32_t add = 0;
            for (int w = 0; w < kBinWaves; ++w) {
                add += wcount[w][b];
                wcount[w][b] = 0;
            }
            next[b] += add;
        }
        __syncthreads();
    }
}

// A level's build runs to its end even when its checks failed, so that the
// plan needs a single synchronisation: the kernels below that would follow
// the level's offsets, ids or map entries read the check flags first (the
// level's word and the map's) and then write an empty but well-formed
// result instead (zero offsets, zero ids, zero degrees).  Every later
// kernel stays in bounds on those.
__device__ inline bool level_failed(const int *bad) { return bad && (bad[0] | bad[1]) != 0; }

// CSR offsets from keys sorted ascending (keys in [0, n_keys)): ptr[v] is
// the first position whose key is >= v, for v in [0, n_keys].  Thread j
// (0 <= j <= n) writes the offsets of the keys in (keys[j-1], keys[j]],
// with keys[-1] = -1 and keys[n] = n_keys, so every entry is written once
// and keys missing from the list (rows without entries) get empty ranges.
__global__ __launch_bounds__(kThreads) void k_offsets_sorted(const uint32_t *__restrict__ keys, int64_t n,
                                                             int64_t n_keys, const int *__restrict__ bad,
                                                             int32_t *__restrict__ ptr)
{
    const int64_t j = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (j > n)
        return;
    if (level_failed(bad)) {   // the n + 1 threads clear the n_keys + 1 entries
        for (int64_t v = j; v <= n_keys; v += n + 1)
            ptr[v] = 0;
        return;
    }
    const int64_t lo = (j == 0) ? -1 : (int64_t)keys[j - 1];
    const int64_t hi = (j == n) ? n_keys : (int64_t)keys[j];
    for (int64_t v = lo + 1; v <= hi; ++v)
        ptr[v] = (int32_t)j;
}

__global__ __launch_bounds__(kThreads) void k_iota(int64_t n, int32_t *__restrict__ out)
{
    const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (i < n)
        out[i] = (int32_t)i;
}

__global__ __launch_bounds__(kThreads) void k_fill_f32(float *__restrict__ p, int64_t n, float v)
{
    const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (i < n)
        p[i] = v;
}

// projection row map: node v -> rep(v); kept hyperedge -> n_nodes_c + rep(e);
// removed hyperedge -> the coarse node its members were merged into
__global__ __launch_bounds__(kThreads) void k_rowmap(const int32_t *__restrict__ ptr, const int32_t *__restrict__ idx,
                                                     const int32_t *__restrict__ node_rep,
                                                     const int32_t *__restrict__ edge_rep, int64_t n_nodes,
                                                     int64_t n_edges, int64_t n_nodes_c, const int *__restrict__ bad,
                                                     int32_t *__restrict__ rowmap)
{
    const int64_t u = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (u >= n_nodes + n_edges)
        return;
    if (level_failed(bad)) {
        rowmap[u] = 0;
        return;
    }
    if (u < n_nodes) {
        rowmap[u] = node_rep[u];
        return;
    }
    const int64_t e = u - n_nodes;
    const int32_t r = edge_rep[e];
    rowmap[u] = (r >= 0) ? (int32_t)(n_nodes_c + r) : node_rep[idx[ptr[e]]];
}

// Side 0's neighbour arrays: the member lists as given, and with a coarser
// level each member's coarse row (a node's row maps to rep(v), so
// cidx = node_rep[idx]; 0 when the level failed its checks).
__global__ __launch_bounds__(kThreads) void k_side0_idx(const int32_t *__restrict__ edge_idx,
                                                        const int32_t *__restrict__ node_rep, int64_t nnz,
                                                        const int *__restrict__ bad, int32_t *__restrict__ idx,
                                                        int32_t *__restrict__ cidx)
{
    const int64_t j = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (j >= nnz)
        return;
    const int32_t v = edge_idx[j];
    idx[j] = v;
    if (cidx)
        cidx[j] = level_failed(bad) ? 0 : node_rep[v];
}

// Side 1's neighbour arrays from the hyperedge of each incidence in node
// order: the hyperedge's Z row n_nodes + e, and with a coarser level its
// coarse row rowmap[n_nodes + e] (0 when the level failed its checks).
__global__ __launch_bounds__(kThreads) void k_side1_idx(const int32_t *__restrict__ csc_e, int64_t nnz,
                                                        int32_t n_nodes, const int32_t *__restrict__ rowmap,
                                                        const int *__restrict__ bad, int32_t *__restrict__ idx,
                                                        int32_t *__restrict__ cidx)
{
    const int64_t j = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (j >= nnz)
        return;
    const int32_t u = csc_e[j] + n_nodes;
    idx[j] = u;
    if (cidx)
        cidx[j] = level_failed(bad) ? 0 : rowmap[u];
}

// A row's wavefront-tier counts: its chunks, whether it is split, its
// partial slots.  One exclusive scan of them (componentwise sums) gives each
// row's first chunk item, split-row entry and partial slot.
struct TierCount {
    int32_t pieces, split, slots;
};
struct TierCountPlus {
    __host__ __device__ TierCount operator()(const TierCount &x, const TierCount &y) const
    {
        return TierCount{x.pieces + y.pieces, x.split + y.split, x.slots + y.slots};
    }
};

// The degree tiers of up to two sides are built together, over one array of
// entries: side k's rows take entries [off, off + n_rows), side 1 starting
// past side 0 on a 256-byte boundary, and the entries in between are
// padding.  Each kernel below handles every entry of both sides in one
// launch.  A stable sort of the entries on a key that puts side 0's keys
// below side 1's leaves each side's rows in its own entries, so one counting
// pass and one scan serve both sides; partial slots run on from side 0 into
// side 1, chunk items and split rows restart per side.
struct TierSide {
    const int32_t *ptr;      // [n_rows + 1] the side's offsets
    int32_t n_rows;
    int32_t off;             // first entry of the side's rows
    const int32_t *rowmap;   // projection row map (Z row row_base + r), or null
    int32_t row_base;
    const int32_t *idx, *cidx;   // the side's neighbour arrays (cidx may be null)
    Item *small;
    InlineIds *ids, *cids;   // may be null
    Item *chunks;
    Split *splits;
};
struct TierSides {
    TierSide s[2];
    int32_t n;       // sides (1 or 2)
    int64_t total;   // entries: s[n - 1].off + s[n - 1].n_rows
};

// The side of entry p (its row there is p - off; a row >= n_rows is
// padding), for p = blockIdx.x * kThreads + threadIdx.x.  Side 1 starts on a
// multiple of kTierAlign = 64 entries and a wavefront covers 64 consecutive
// entries from a multiple of 64, so every wavefront lies in one side: the
// side is taken wave-uniform, and the side's pointers then come from scalar
// loads.
__device__ inline int side_of(const TierSides &T, int64_t p)
{
    const int64_t p0 = p & ~(int64_t)(kWave - 1);
    return __builtin_amdgcn_readfirstlane((T.n == 2 && p0 >= T.s[1].off) ? 1 : 0);
}

// Tier sort key of a side's row: small_max - degree for the lane-group tier,
// small_max + 1 for longer rows, small_max + 2 for padding, plus the side
// times small_max + 3.
__device__ inline uint32_t tier_key_base(int sd, int small_max) { return (uint32_t)sd * (uint32_t)(small_max + 3); }

__global__ __launch_bounds__(kThreads) void k_tier_keys(TierSides T, int small_max, int chunk,
                                                        const int *__restrict__ bad, uint32_t *__restrict__ key,
                                                        TierCount *__restrict__ tc)
{
    const int64_t p = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (p >= T.total)
        return;
    const int sd = side_of(T, p);
    const TierSide &S = T.s[sd];
    const int64_t r = p - S.off;
    const uint32_t kb = tier_key_base(sd, small_max);
    if (r >= S.n_rows) {
        key[p] = kb + (uint32_t)(small_max + 2);
        tc[p] = TierCount{0, 0, 0};
        return;
    }
    const int32_t deg = level_failed(bad) ? 0 : S.ptr[r + 1] - S.ptr[r];
    const bool small = deg <= small_max;
    const int32_t pc = small ? 0 : (deg + chunk - 1) / chunk;
    key[p] = kb + (small ? (uint32_t)(small_max - deg) : (uint32_t)(small_max + 1));
    tc[p] = TierCount{pc, pc > 1 ? 1 : 0, pc > 1 ? pc : 0};
}

// the sums of the tier counts over entries [0, p) from the exclusive scan
__device__ inline TierCount counts_before(const TierCount *tc, const TierCount *tpos, int64_t p)
{
    if (p == 0)
        return TierCount{0, 0, 0};
    const TierCount a = tpos[p - 1], b = tc[p - 1];
    return TierCount{a.pieces + b.pieces, a.split + b.split, a.slots + b.slots};
}

// counts[4 * side + 0..3]: small rows, chunks, split rows, partial slots of
// the side (small rows from the sorted keys, the rest from the scan); and
// n_chunks: both sides' chunks.  Thread k handles side k.
__global__ void k_tier_counts(const uint32_t *__restrict__ sorted_key, const TierCount *__restrict__ tc,
                              const TierCount *__restrict__ tpos, TierSides T, int small_max,
                              int64_t *__restrict__ counts, int64_t *__restrict__ n_chunks)
{
    const int sd = threadIdx.x;
    if (blockIdx.x != 0 || sd >= T.n)
        return;
    const TierSide &S = T.s[sd];
    // sorted ascending: the side's small rows first; binary search for its
    // first longer row
    const uint32_t last_small = tier_key_base(sd, small_max) + (uint32_t)small_max;
    int64_t lo = S.off, hi = (int64_t)S.off + S.n_rows;
    while (lo < hi) {
        const int64_t mid = (lo + hi) / 2;
        if (sorted_key[mid] <= last_small)
            lo = mid + 1;
        else
            hi = mid;
    }
    const TierCount a = counts_before(tc, tpos, S.off), b = counts_before(tc, tpos, (int64_t)S.off + S.n_rows);
    int64_t *c = counts + 4 * sd;
    c[0] = lo - S.off;
    c[1] = (int64_t)b.pieces - a.pieces;
    c[2] = (int64_t)b.split - a.split;
    c[3] = (int64_t)b.slots - a.slots;
    if (sd == T.n - 1)
        *n_chunks = b.pieces;
}

// lane-group tier items, one thread per row in row order (so that the
// offsets and neighbour ids are read in order): the tier sort's position of
// the row's entry, less its side's first entry, is the row's item when it is
// below the side's count of small rows.  aux = the coarse row the row's own
// value is projected from (0 at the coarsest level).  With `ids`, also each
// item's first kInlineIds neighbour ids from idx (and from cidx into
// `cids`), 0 past the row's degree, and all 0 when the level failed its
// checks (its offsets may then point anywhere).
__global__ __launch_bounds__(kThreads) void k_small_items(TierSides T, const int32_t *__restrict__ pos,
                                                          const int64_t *__restrict__ counts,
                                                          const int *__restrict__ bad)
{
    const int64_t p = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (p >= T.total)
        return;
    const int sd = side_of(T, p);
    const TierSide &S = T.s[sd];
    const int32_t r = (int32_t)(p - S.off);
    if (r >= S.n_rows)
        return;
    const int64_t i = (int64_t)pos[p] - S.off;
    if (i >= counts[4 * sd])
        return;
    const int32_t a = S.ptr[r], len = S.ptr[r + 1] - a;
    S.small[i] = Item{r, a, len, S.rowmap ? S.rowmap[S.row_base + r] : 0};
    if (!S.ids)
        return;
    InlineIds x{}, c{};
    if (!level_failed(bad)) {
#pragma unroll
        for (int k = 0; k < kInlineIds; ++k) {
            if (k < len) {
                x.id[k] = S.idx[a + k];
                if (S.cids)
                    c.id[k] = S.cidx[a + k];
            }
        }
    }
    S.ids[i] = x;
    if (S.cids)
        S.cids[i] = c;
}

// wavefront tier items of both sides in entry order (pieces of a row in
// order), with the sort key side * chunk + chunk - len (a stable ascending
// sort keeps the sides apart and puts each side's longest first)
__global__ __launch_bounds__(kThreads) void k_chunk_items(TierSides T, int chunk, const TierCount *__restrict__ tc,
                                                          const TierCount *__restrict__ tpos,
                                                          Item *__restrict__ items, uint32_t *__restrict__ key,
                                                          int32_t *__restrict__ id)
{
    const int64_t p = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (p >= T.total)
        return;
    const int32_t pc = tc[p].pieces;
    if (pc == 0)
        return;
    const int sd = side_of(T, p);
    const TierSide &S = T.s[sd];
    const int32_t r = (int32_t)(p - S.off);
    const TierCount at = tpos[p];
    for (int32_t k = 0; k < pc; ++k) {
        const int32_t pos = at.pieces + k;
        const int32_t s = S.ptr[r] + k * chunk;
        const int32_t len = min(chunk, S.ptr[r + 1] - s);
        items[pos] = Item{r, s, len, pc == 1 ? -1 : at.slots + k};
        key[pos] = (uint32_t)(sd * chunk + chunk - len);
        id[pos] = pos;
    }
}

// the sorted chunk items into each side's list (side 0's come first)
__global__ __launch_bounds__(kThreads) void k_gather_items(TierSides T, const Item *__restrict__ in,
                                                           const int32_t *__restrict__ order,
                                                           const int64_t *__restrict__ counts,
                                                           const int64_t *__restrict__ n)
{
    const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (i >= *n)
        return;
    const int64_t c0 = counts[1];
    if (T.n == 2 && i >= c0)
        T.s[1].chunks[i - c0] = in[order[i]];
    else
        T.s[0].chunks[i] = in[order[i]];
}

__global__ __launch_bounds__(kThreads) void k_split_items(TierSides T, const TierCount *__restrict__ tc,
                                                          const TierCount *__restrict__ tpos,
                                                          const int64_t *__restrict__ counts)
{
    const int64_t p = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (p >= T.total || tc[p].pieces <= 1)
        return;
    const int sd = side_of(T, p);
    const TierSide &S = T.s[sd];
    const int32_t r = (int32_t)(p - S.off);
    const TierCount at = tpos[p];
    const int64_t first = sd == 0 ? 0 : counts[2];   // side 1's entries follow side 0's split rows
    S.splits[at.split - first] = Split{r, at.slots, tc[p].pieces, S.ptr[r + 1] - S.ptr[r]};
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------

// Work-list bounds from the sizes alone (see the tiering rules above): rows
// longer than small_max number at most nnz / (small_max + 1), each has at
// most degree / chunk + 1 pieces, and only rows longer than chunk split.
LevelShape bound_shape(const hnv_level_dev &lv, const hnv_level_dev *coarse, int small_max, int chunk)
{
    LevelShape sh;
    sh.nV = lv.n_nodes;
    sh.nE = lv.n_edges;
    sh.nnz = lv.nnz;
    sh.rows = sh.nV + sh.nE;
    sh.has_coarse = coarse != nullptr;
    sh.rows_c = coarse ? coarse->n_nodes + coarse->n_edges : 0;
    sh.unit_w = lv.edge_w == nullptr;
    auto cap = [](int64_t v) { return (int32_t)std::min<int64_t>(v, INT_MAX); };
    int64_t slots = 0;
    for (int s = 0; s < 2; ++s) {
        const int64_t n_rows = s == 0 ? sh.nE : sh.nV;
        sh.n_small[s] = cap(n_rows);
        sh.n_chunks[s] = cap(std::min<int64_t>(sh.nnz / chunk + sh.nnz / (small_max + 1) + 1, sh.nnz + 1));
        sh.n_splits[s] = cap(sh.nnz / (chunk + 1) + 1);
        slots += 2 * (sh.nnz / chunk) + 1;
    }
    sh.n_slots = cap(slots);
    return sh;
}

// The per-entry arrays of the degree tiers (both sides' entries).
struct TierArrays {
    int32_t *row_ids;       // 0, 1, 2, ..: the values of the inverse map's sort
    TierCount *tc, *tpos;   // per-entry tier counts and their exclusive scan
    uint32_t *key_a, *key_b;
    int32_t *pos;           // each entry's position in tier order
};

// Temporaries of one level's build, carved from `base` (nullptr: sizing).
// The tier arrays hold tier_entries(rows) entries: side 0's rows from 0,
// side 1's from side1_offset(n_edges).
struct Scratch {
    int32_t *inc_edge, *csc_e, *keys_out, *ids_a, *ids_b, *bin_counts, *bin_offs;
    uint32_t *ckey_a, *ckey_b;
    TierArrays tier;
    Item *items;
    int *flag;
    int64_t *counts;     // [side][small rows, chunks, split rows, partial slots]
    int64_t *n_chunks;   // both sides' chunk items
    void *temp;
    size_t temp_bytes, total;
};

constexpr int64_t kTierAlign = 64;   // side 1 starts on a 256-byte boundary and a wavefront boundary
static_assert(kTierAlign % kWave == 0, "a wavefront of tier entries must lie in one side");
int64_t side1_offset(int64_t n_edges) { return (n_edges + 1 + kTierAlign - 1) / kTierAlign * kTierAlign; }
int64_t tier_entries(int64_t rows) { return rows + 2 + kTierAlign; }

// entries of the key-count arrays of a bin sort of up to `rows` pairs
int64_t bin_cap(int64_t rows, int n_bins) { return (int64_t)n_bins * (rows / kBinTile + 1); }

hnv_status cub_sizes(int64_t nnz, int64_t rows, int64_t n_chunks, int64_t bins, size_t &bytes)
{
    size_t t[6] = {0, 0, 0, 0, 0, 0};
    const int n = (int)std::max<int64_t>(std::max(nnz, rows) + 1, 1);
    hipError_t e = prim_sort_pairs(nullptr, t[0], (uint32_t *)nullptr, (uint32_t *)nullptr,
                                                      (int32_t *)nullptr, (int32_t *)nullptr, n, 0, 32);
    if (e == hipSuccess)
        e = prim_exclusive_sum(nullptr, t[1], (int32_t *)nullptr, (int32_t *)nullptr, n);
    if (e == hipSuccess)
        e = prim_sort_pairs(nullptr, t[3], (uint32_t *)nullptr, (uint32_t *)nullptr,
                                               (int32_t *)nullptr, (int32_t *)nullptr,
                                               (int)std::max<int64_t>(n_chunks, 1), 0, 32);
    if (e == hipSuccess)
        e = prim_exclusive_sum(nullptr, t[4], (int32_t *)nullptr, (int32_t *)nullptr, (int)bins);
    if (e == hipSuccess)
        e = prim_exclusive_scan(nullptr, t[5], (TierCount *)nullptr, (TierCount *)nullptr, TierCount{0, 0, 0},
                                (int)tier_entries(rows), TierCountPlus());
    if (e != hipSuccess)
        return fail(HNV_EDEVICE, std::string("sort / scan storage query (needs a visible GPU): ") +
                                     hipGetErrorString(e));
    bytes = *std::max_element(t, t + 6);
    return HNV_OK;
}

// n_chunks: the chunk items of both sides together; tier_bins: the keys of
// the degree-tier sort
hnv_status scratch_layout(int64_t nnz, int64_t rows, int64_t n_chunks, int tier_bins, char *base, Scratch &S)
{
    size_t off = 0;
    auto take = [&](size_t bytes) -> char * {
        off = (off + 255) & ~size_t(255);
        char *p = base ? base + off : nullptr;
        off += std::max<size_t>(bytes, 8);
        return p;
    };
    const size_t n4 = 4 * (size_t)std::max(nnz, rows + 1);
    S.inc_edge = (int32_t *)take(4 * nnz);
    S.csc_e = (int32_t *)take(n4);
    S.keys_out = (int32_t *)take(n4);
    const size_t t4 = 4 * (size_t)tier_entries(rows);
    S.tier.row_ids = (int32_t *)take(t4);
    S.tier.tc = (TierCount *)take(3 * t4);
    S.tier.tpos = (TierCount *)take(3 * t4);
    S.tier.key_a = (uint32_t *)take(t4);
    S.tier.key_b = (uint32_t *)take(t4);
    S.tier.pos = (int32_t *)take(t4);
    const int64_t bins = std::max(bin_cap(tier_entries(rows), tier_bins), bin_cap(n_chunks, kBinsMax));
    S.bin_counts = (int32_t *)take(4 * bins);
    S.bin_offs = (int32_t *)take(4 * bins);
    S.ckey_a = (uint32_t *)take(4 * n_chunks);
    S.ckey_b = (uint32_t *)take(4 * n_chunks);
    S.ids_a = (int32_t *)take(4 * n_chunks);
    S.ids_b = (int32_t *)take(4 * n_chunks);
    S.items = (Item *)take(sizeof(Item) * n_chunks);
    S.flag = (int *)take(16);
    S.counts = (int64_t *)take(8 * 8);
    S.n_chunks = (int64_t *)take(8);
    if (hnv_status st = cub_sizes(nnz, rows, n_chunks, bins, S.temp_bytes); st != HNV_OK)
        return st;
    S.temp = take(S.temp_bytes);
    S.total = (off + 255) & ~size_t(255);
    return HNV_OK;
}

// What the build leaves on the device per level, read back once at its end:
// the check flags (the level's word, the map's word) and the tier counts of
// both sides (small rows, chunks, split rows, partial slots).  Kept ahead of
// the per-level temporaries.
struct LevelMeta {
    int32_t flags[4];
    int32_t pad[4];
    int64_t counts[8];
};
size_t meta_bytes(int n_levels) { return ((size_t)n_levels * sizeof(LevelMeta) + 255) & ~size_t(255); }

// plan layout and build-scratch size for these levels
hnv_status device_layout(const hnv_level_dev *levels, int n_levels, int d, hnv_dtype dtype, const hnv_options &o,
                         hnv_plan *p, std::vector<LevelShape> &bounds, size_t &scratch_bytes, bool &scratch_in_zbuf,
                         size_t &total)
{
    bounds.assign(n_levels, LevelShape{});
    std::vector<LevelShape> sizes(n_levels);
    for (int l = 0; l < n_levels; ++l) {
        sizes[l].nV = levels[l].n_nodes;
        sizes[l].nE = levels[l].n_edges;
        sizes[l].nnz = levels[l].nnz;
        sizes[l].unit_w = levels[l].edge_w == nullptr;
    }
    init_plan_shape(p, sizes, d, dtype, o);
    scratch_bytes = 0;
    for (int l = 0; l < n_levels; ++l) {
        bounds[l] = bound_shape(levels[l], l + 1 < n_levels ? &levels[l + 1] : nullptr, p->small_max, o.chunk);
        Scratch S{};
        const int64_t nch = (int64_t)bounds[l].n_chunks[0] + bounds[l].n_chunks[1];
        if (hnv_status st = scratch_layout(bounds[l].nnz, bounds[l].rows, nch, 2 * (p->small_max + 3), nullptr, S);
            st != HNV_OK)
            return st;
        scratch_bytes = std::max(scratch_bytes, S.total);
    }
    scratch_bytes += meta_bytes(n_levels);
    carve(p, bounds, nullptr);
    const size_t zbuf_bytes = (size_t)p->lv[0].rows * p->d * ((dtype == HNV_BF16) ? 2 : 4);
    scratch_in_zbuf = scratch_bytes <= zbuf_bytes;
    total = p->ws_bytes + (scratch_in_zbuf ? 0 : scratch_bytes);
    return HNV_OK;
}

hnv_status check_levels(const hnv_level_dev *levels, const hnv_map *maps, int n_levels)
{
    if (!levels || n_levels < 1)
        return fail(HNV_EINVAL, "need at least one level");
    if (n_levels > 1 && !maps)
        return fail(HNV_EINVAL, "maps is NULL with more than one level");
    for (int l = 0; l < n_levels; ++l) {
        const hnv_level_dev &L = levels[l];
        if (L.n_nodes < 0 || L.n_edges < 0 || L.nnz < 0 || !L.edge_ptr || (L.nnz > 0 && !L.edge_idx))
            return fail(HNV_EINVAL, "level " + std::to_string(l) + ": bad sizes or NULL arrays");
        if (L.n_edges == 0 && L.nnz != 0)
            return fail(HNV_EINVAL, "level " + std::to_string(l) + ": incidences without hyperedges");
        if (L.n_nodes + L.n_edges >= INT_MAX || L.nnz >= INT_MAX)
            return fail(HNV_EUNSUPPORTED, "level " + std::to_string(l) + ": rows and nnz must be below 2^31");
        if (L.n_nodes + L.n_edges > levels[0].n_nodes + levels[0].n_edges)
            return fail(HNV_EUNSUPPORTED, "level " + std::to_string(l) +
                                              " has more rows than level 0 (iterates live in buffers of its size)");
        if (l + 1 < n_levels && ((L.n_nodes > 0 && !maps[l].node_rep) || (L.n_edges > 0 && !maps[l].edge_rep)))
            return fail(HNV_EINVAL, "map " + std::to_string(l) + " has a NULL array");
    }
    return HNV_OK;
}

hnv_status read_back(void *dst, const void *src, size_t n, hipStream_t s)
{
    hipError_t e = hipMemcpyAsync(dst, src, n, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess)
        e = hipStreamSynchronize(s);
    return e == hipSuccess ? HNV_OK : fail(HNV_EDEVICE, std::string("read-back: ") + hipGetErrorString(e));
}

hnv_status copy_d2d(void *dst, const void *src, size_t n, hipStream_t s)
{
    if (n == 0)
        return HNV_OK;
    hipError_t e = hipMemcpyAsync(dst, src, n, hipMemcpyDeviceToDevice, s);
    return e == hipSuccess ? HNV_OK : fail(HNV_EDEVICE, std::string("hipMemcpyAsync: ") + hipGetErrorString(e));
}

// S.inc_edge[j] = the hyperedge of incidence j
hnv_status incidence_edges(const int32_t *ptr, int64_t nE, int64_t nnz, Scratch &S, hipStream_t s)
{
    k_fill<<<grid_for(nnz), kThreads, 0, s>>>(S.inc_edge, nnz, 0);
    k_inc_edge<<<grid_for(nE), kThreads, 0, s>>>(ptr, nE, nnz, S.inc_edge);
    return dev_check("incidence map");
}

// Checks of level l and (with a coarser level) of map l, launched without
// waiting: flags[0] gets the level's bits, flags[1] the map's.  The map's
// member-following check does nothing unless the level's offsets and member
// ids passed, so every kernel stays in bounds on any input.
hnv_status launch_checks(const hnv_level_dev &L, const hnv_level_dev *C, const hnv_map *m, bool full, Scratch &S,
                         int *flags, hipStream_t s)
{
    const int64_t nV = L.n_nodes, nE = L.n_edges, nnz = L.nnz;
    if (nE > 0) {
        k_check_edges<<<grid_for(nE), kThreads, 0, s>>>(L.edge_ptr, L.edge_w, nE, nnz, full ? 1 : 0, flags);
        if (nnz > 0) {
            if (hnv_status st = incidence_edges(L.edge_ptr, nE, nnz, S, s); st != HNV_OK)
                return st;
            k_check_members<<<grid_for(nnz), kThreads, 0, s>>>(L.edge_ptr, L.edge_idx, S.inc_edge, nV, nE, nnz,
                                                              full ? 1 : 0, flags);
        }
    } else {
        k_check_no_edges<<<1, 64, 0, s>>>(L.edge_ptr, nnz, flags);
    }
    if (C) {
        if (nV > 0)
            k_check_node_map<<<grid_for(nV), kThreads, 0, s>>>(m->node_rep, nV, C->n_nodes, flags + 1);
        if (nE > 0)
            k_check_edge_map<<<grid_for(nE), kThreads, 0, s>>>(L.edge_ptr, L.edge_idx, m->node_rep, m->edge_rep, nV,
                                                               nE, C->n_edges, full ? 1 : 0, flags, flags + 1);
    }
    return dev_check("level checks");
}

// The error for level l's flags (HNV_OK when there is none), level before map.
hnv_status report_checks(int l, const int *flags, bool full)
{
    const int bad = flags[0], mbad = flags[1];
    const std::string lv = "level " + std::to_string(l) + ": ";
    if (bad & 1)
        return fail(HNV_EINVAL, lv + "edge_ptr must start at 0, never decrease and end at nnz" +
                                    (full ? ", and no hyperedge may be empty" : ""));
    if (bad & 2)
        return fail(HNV_ERANGE, lv + "a member id is outside [0, n_nodes)");
    if (bad & 4)
        return fail(HNV_EUNSORTED, lv + "member lists must be strictly ascending");
    if (bad & 8)
        return fail(HNV_EINVAL, lv + "weights must be finite and > 0");
    const std::string mp = "map " + std::to_string(l) + ": ";
    if (mbad & (1 << 4))
        return fail(HNV_ERANGE, mp + "node_rep out of range");
    if (mbad & (1 << 5))
        return fail(HNV_ERANGE, mp + "edge_rep out of range");
    if (mbad & (1 << 6))
        return fail(HNV_ERANGE, mp + "a removed hyperedge has no members");
    if (mbad & (1 << 7))
        return fail(HNV_ERANGE, mp + "a removed hyperedge has members in different coarse nodes");
    return HNV_OK;
}

// Stable sort of the pairs (ka, va) by key (every key below key_limit) with
// the counting passes above: n_max pairs, or *n_dev of them.  The sorted
// pairs end in (kb, vb) after an odd number of passes, else in (ka, va);
// `in_b` tells which.  va and vb may both be null (keys only).  pos_out (one
// pass only): pos_out[i] = the sorted position of input pair i.
hnv_status bin_sort(uint32_t *ka, int32_t *va, uint32_t *kb, int32_t *vb, int64_t n_max, const int64_t *n_dev,
                    int64_t key_limit, Scratch &S, hipStream_t s, bool &in_b, int32_t *pos_out = nullptr)
{
    in_b = false;
    if (n_max == 0)
        return HNV_OK;
    const int64_t tiles = (n_max + kBinTile - 1) / kBinTile;
    const bool one = key_limit <= kBinsMax;
    const int passes = one ? 1 : (bits_for(key_limit) + kBinBits - 1) / kBinBits;
    const int n_bins = one ? (int)key_limit : kBinsMax;
    if (pos_out && !one)
        return fail(HNV_EUNSUPPORTED, "sorted positions from a multi-pass counting sort");
    const uint32_t mask = one ? 0xffffffffu : (uint32_t)(kBinsMax - 1);
    uint32_t *kin = ka, *kout = kb;
    int32_t *vin = va, *vout = vb;
    for (int pass = 0; pass < passes; ++pass) {
        const int shift = pass * kBinBits;
        k_bin_count<<<(unsigned)tiles, kThreads, 0, s>>>(kin, n_max, n_dev, shift, mask, n_bins, tiles, S.bin_counts);
        size_t tb = S.temp_bytes;
        if (prim_exclusive_sum(S.temp, tb, S.bin_counts, S.bin_offs, tiles * n_bins, s) != hipSuccess)
            return fail(HNV_EDEVICE, "scan of a counting sort's digit counts");
        k_bin_scatter<<<(unsigned)tiles, kThreads, 0, s>>>(kin, vin, n_max, n_dev, shift, mask, n_bins,
                                                           bits_for(n_bins), tiles, S.bin_offs, kout, vout, pos_out);
        std::swap(kin, kout);
        std::swap(vin, vout);
        in_b = !in_b;
    }
    return dev_check("counting sort");
}

// The tier keys, sort and scan of the sides T (one or two); counts[4 * side
// + 0..3] and S.n_chunks on the device.  `bad`: the level's check flags
// (null: checked already).
hnv_status tier_scan(const TierSides &T, int small_max, int chunk, const int *bad, Scratch &S, int64_t *counts,
                     hipStream_t s)
{
    if (T.total == 0) {
        k_fill<<<1, kThreads, 0, s>>>(reinterpret_cast<int32_t *>(counts), 16, 0);
        k_fill<<<1, kThreads, 0, s>>>(reinterpret_cast<int32_t *>(S.n_chunks), 2, 0);
        return dev_check("tier counts");
    }
    const int64_t n_keys = (int64_t)T.n * (small_max + 3);
    if (n_keys > kBinsMax)
        return fail(HNV_EUNSUPPORTED, "small_max above the tier sort's key range");
    const TierArrays &A = S.tier;
    k_tier_keys<<<grid_for(T.total), kThreads, 0, s>>>(T, small_max, chunk, bad, A.key_a, A.tc);
    // the lane-group tier order of both sides: one counting pass, which
    // gives each entry's position in that order
    bool in_b = false;
    if (hnv_status st = bin_sort(A.key_a, nullptr, A.key_b, nullptr, T.total, nullptr, n_keys, S, s, in_b, A.pos);
        st != HNV_OK)
        return st;
    size_t tb = S.temp_bytes;
    if (prim_exclusive_scan(S.temp, tb, A.tc, A.tpos, TierCount{0, 0, 0}, (int)T.total, TierCountPlus(), s) !=
        hipSuccess)
        return fail(HNV_EDEVICE, "scan of the tier counts");
    k_tier_counts<<<1, 64, 0, s>>>(in_b ? A.key_b : A.key_a, A.tc, A.tpos, T, small_max, counts, S.n_chunks);
    return dev_check("tier keys");
}

// The work lists of the sides T after tier_scan, from the counts it left on
// the device without reading them: grids cover the bounds (max_chunks
// wavefront-tier items of both sides) and the kernels stop at the counts.
hnv_status tier_emit(const TierSides &T, int chunk, int64_t max_chunks, const int *bad, Scratch &S,
                     const int64_t *counts, hipStream_t s)
{
    if (T.total == 0)
        return HNV_OK;
    const TierArrays &A = S.tier;
    k_small_items<<<grid_for(T.total), kThreads, 0, s>>>(T, A.pos, counts, bad);
    if (max_chunks > 0) {
        k_chunk_items<<<grid_for(T.total), kThreads, 0, s>>>(T, chunk, A.tc, A.tpos, S.items, S.ckey_a, S.ids_a);
        // each side's longest first: a stable sort on side * chunk + chunk - len
        bool in_b = false;
        if (hnv_status st = bin_sort(S.ckey_a, S.ids_a, S.ckey_b, S.ids_b, max_chunks, S.n_chunks,
                                     (int64_t)T.n * chunk, S, s, in_b);
            st != HNV_OK)
            return st;
        k_gather_items<<<grid_for(max_chunks), kThreads, 0, s>>>(T, S.items, in_b ? S.ids_b : S.ids_a, counts,
                                                                 S.n_chunks);
    }
    k_split_items<<<grid_for(T.total), kThreads, 0, s>>>(T, A.tc, A.tpos, counts);
    return dev_check("work lists");
}

// One side's part of a tier build (its rows at entries from `off`).
TierSide tier_side(const DevSide &D, int64_t n_rows, int64_t off, const int32_t *rowmap)
{
    TierSide t{};
    t.ptr = D.ptr;
    t.n_rows = (int32_t)n_rows;
    t.off = (int32_t)off;
    t.rowmap = rowmap;
    t.row_base = D.row_base;
    t.idx = D.idx;
    t.cidx = D.cidx;
    t.small = const_cast<Item *>(D.small);
    t.ids = const_cast<InlineIds *>(D.small_ids);
    t.cids = const_cast<InlineIds *>(D.small_cids);
    t.chunks = const_cast<Item *>(D.chunks);
    t.splits = const_cast<Split *>(D.splits);
    return t;
}

// Level l of a plan, enqueued without waiting: its checks were launched
// before (their flags in M.flags gate the kernels that follow offsets and
// ids), and the tier counts it leaves in M.counts are read with every other
// level's once the whole build is enqueued (finish_level).
hnv_status build_level(hnv_plan *p, const hnv_level_dev *levels, const hnv_map *maps, int n_levels, int l,
                       LevelMeta *M, Scratch &S, hipStream_t s)
{
    const int *bad = M->flags;
    const hnv_level_dev &lv = levels[l];
    const hnv_level_dev *C = (l + 1 < n_levels) ? &levels[l + 1] : nullptr;
    const hnv_map *m = C ? &maps[l] : nullptr;
    LevelPlan &L = p->lv[l];
    const int64_t nV = lv.n_nodes, nE = lv.n_edges, nnz = lv.nnz;
    const int sm = p->small_max, chunk = p->opts.chunk;
    DevSide &S0 = L.side[0], &S1 = L.side[1];
    hnv_status st;
    // projection row map (first: the composed indices below read it)
    if (C)
        k_rowmap<<<grid_for(nV + nE), kThreads, 0, s>>>(lv.edge_ptr, lv.edge_idx, m->node_rep, m->edge_rep, nV, nE,
                                                        C->n_nodes, bad, L.rowmap);
    // side 0: the member lists as given, and their coarse rows
    if ((st = copy_d2d((void *)S0.ptr, lv.edge_ptr, 4 * (nE + 1), s)) != HNV_OK)
        return st;
    if (nnz > 0)
        k_side0_idx<<<grid_for(nnz), kThreads, 0, s>>>(lv.edge_idx, C ? m->node_rep : nullptr, nnz, bad,
                                                       const_cast<int32_t *>(S0.idx),
                                                       C ? const_cast<int32_t *>(S0.cidx) : nullptr);
    // side 1: node -> hyperedges in ascending id (stable sort of incidences
    // by node; the offsets come from the sorted node ids)
    size_t tb = S.temp_bytes;
    if (nnz > 0) {
        // the values: the hyperedge of each incidence, which the level's
        // checks left in S.inc_edge (a level with incidences has hyperedges)
        if (prim_sort_pairs(S.temp, tb, reinterpret_cast<const uint32_t *>(lv.edge_idx),
                                               reinterpret_cast<uint32_t *>(S.keys_out), S.inc_edge, S.csc_e,
                                               (int)nnz, 0, bits_for(nV), s) != hipSuccess)
            return fail(HNV_EDEVICE, "sort of incidences by node");
        k_side1_idx<<<grid_for(nnz), kThreads, 0, s>>>(S.csc_e, nnz, (int32_t)nV, C ? L.rowmap : nullptr, bad,
                                                       const_cast<int32_t *>(S1.idx),
                                                       C ? const_cast<int32_t *>(S1.cidx) : nullptr);
    }
    k_offsets_sorted<<<grid_for(nnz + 1), kThreads, 0, s>>>(reinterpret_cast<const uint32_t *>(S.keys_out), nnz, nV,
                                                            bad, const_cast<int32_t *>(S1.ptr));
    // inverse map
    if (C) {
        const int64_t rows = nV + nE, rows_c = L.rows_coarse;
        if (rows > 0) {
            k_iota<<<grid_for(rows), kThreads, 0, s>>>(rows, S.tier.row_ids);
            tb = S.temp_bytes;
            if (prim_sort_pairs(S.temp, tb, reinterpret_cast<const uint32_t *>(L.rowmap),
                                                   reinterpret_cast<uint32_t *>(S.keys_out), S.tier.row_ids, L.inv_idx,
                                                   (int)rows, 0, bits_for(rows_c), s) != hipSuccess)
                return fail(HNV_EDEVICE, "sort of the inverse map");
        }
        k_offsets_sorted<<<grid_for(rows + 1), kThreads, 0, s>>>(reinterpret_cast<const uint32_t *>(S.keys_out),
                                                                 rows, rows_c, bad, L.inv_ptr);
    }
    if ((st = dev_check("plan arrays")) != HNV_OK)
        return st;
    // degree tiers of both sides together (partial slots continue from side
    // 0 into side 1); the sizes of the work lists stay on the device until
    // the build ends.  D.n_* still hold the bounds the workspace was carved
    // for.
    TierSides TS{};
    TS.n = 2;
    TS.s[0] = tier_side(S0, nE, 0, C ? L.rowmap : nullptr);
    TS.s[1] = tier_side(S1, nV, side1_offset(nE), C ? L.rowmap : nullptr);
    TS.total = side1_offset(nE) + nV;
    if ((st = tier_scan(TS, sm, chunk, bad, S, M->counts, s)) != HNV_OK ||
        (st = tier_emit(TS, chunk, (int64_t)S0.n_chunks + S1.n_chunks, bad, S, M->counts, s)) != HNV_OK)
        return st;
    // weights and reciprocals
    if (lv.edge_w) {
        if ((st = copy_d2d(L.w, lv.edge_w, 4 * nE, s)) != HNV_OK)
            return st;
    } else if (nE > 0) {
        k_fill_f32<<<grid_for(nE), kThreads, 0, s>>>(L.w, nE, 1.0f);
    }
    if ((st = dev_check("weights")) != HNV_OK)
        return st;
    return dev_recompute_reciprocals(p, l, s);
}

// Level l's work-list sizes from the counts read back after the build
// (counts: this level's LevelMeta::counts), checked against the bounds the
// workspace was carved for.
hnv_status finish_level(hnv_plan *p, int l, const int64_t *counts)
{
    LevelPlan &L = p->lv[l];
    for (int sd = 0; sd < 2; ++sd) {
        const int64_t *cnt = counts + 4 * sd;
        DevSide &D = L.side[sd];
        if (cnt[0] > D.n_small || cnt[1] > D.n_chunks || cnt[2] > D.n_splits)
            return fail(HNV_EDEVICE, "work lists exceed their bounds");
        D.n_small = (int32_t)cnt[0];
        D.n_chunks = (int32_t)cnt[1];
        D.n_splits = (int32_t)cnt[2];
        L.n_small[sd] = D.n_small;
        L.n_chunks[sd] = D.n_chunks;
        L.n_splits[sd] = D.n_splits;
    }
    const int64_t slots = counts[3] + counts[7];
    if (slots > p->max_slots)
        return fail(HNV_EDEVICE, "partial slots exceed their bound");
    L.n_slots = (int32_t)slots;
    return HNV_OK;
}

// Candidate-scoring plan from device arrays: the candidates are the rows of
// one side (offsets cand_ptr, members cand_idx), tiered exactly as the host
// score plan tiers them (small_max = kIdxRegs lanes' worth of the scoring
// lane group, kScoreChunk members per wavefront item).
struct ScoreDevLayout {
    size_t off_idx = 0, off_small = 0, off_chunks = 0, off_splits = 0, off_part = 0, off_scratch = 0;
    int32_t n_small = 0, n_chunks = 0, n_splits = 0, n_slots = 0;
    int small_max = 0;
    size_t scratch_bytes = 0, total = 0;
};

hnv_status score_dev_layout(int64_t n_cand, int64_t n_members, int d, hnv_dtype dtype, ScoreDevLayout &L)
{
    if (n_cand < 0 || n_members < 0)
        return fail(HNV_EINVAL, "negative size");
    if (d < 8 || d > 512 || d % 8 != 0)
        return fail(HNV_EUNSUPPORTED, "d must be a multiple of 8 in [8, 512]");
    if (dtype != HNV_F32 && dtype != HNV_BF16)
        return fail(HNV_EINVAL, "unknown dtype");
    if (n_cand >= INT_MAX || n_members >= INT_MAX)
        return fail(HNV_EUNSUPPORTED, "candidates and members must be below 2^31");
    int G = 1, E = 8;
    lane_layout(d, dtype == HNV_BF16 ? 2 : 4, &G, &E);
    L.small_max = kIdxRegs * G;
    auto cap = [](int64_t v) { return (int32_t)std::min<int64_t>(std::max<int64_t>(v, 1), INT_MAX); };
    L.n_small = cap(n_cand);
    L.n_chunks = cap(std::min<int64_t>(n_members / kScoreChunk + n_members / (L.small_max + 1) + 1, n_members + 1));
    L.n_splits = cap(n_members / (kScoreChunk + 1) + 1);
    L.n_slots = cap(2 * (n_members / kScoreChunk) + 1);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        off = (off + 255) & ~size_t(255);
        const size_t p = off;
        off += std::max<size_t>(bytes, 8);
        return p;
    };
    L.off_idx = take(4 * (size_t)n_members);
    L.off_small = take(sizeof(Item) * (size_t)L.n_small);
    L.off_chunks = take(sizeof(Item) * (size_t)L.n_chunks);
    L.off_splits = take(sizeof(Split) * (size_t)L.n_splits);
    L.off_part = take(sizeof(float) * (size_t)L.n_slots * (2 * d + 8));
    Scratch S{};
    if (hnv_status st = scratch_layout(n_members, n_cand, L.n_chunks, L.small_max + 3, nullptr, S); st != HNV_OK)
        return st;
    L.scratch_bytes = S.total;
    L.off_scratch = take(L.scratch_bytes);
    L.total = (off + 255) & ~size_t(255);
    return HNV_OK;
}

}  // namespace
}  // namespace hnv

using namespace hnv;

extern "C" hnv_status hnv_plan_workspace_bytes_device(const hnv_level_dev *levels, const hnv_map *maps,
                                                      int n_levels, int d, hnv_dtype dtype,
                                                      const hnv_options *opts, size_t *bytes)
{
    clear_error();
    if (!bytes)
        return fail(HNV_EINVAL, "bytes is NULL");
    hnv_options o;
    resolve_options(opts, d, dtype, &o);
    hnv_status st = check_plan_options(d, dtype, o);
    if (st == HNV_OK)
        st = check_levels(levels, maps, n_levels);
    if (st != HNV_OK)
        return st;
    try {
        hnv_plan p;
        std::vector<LevelShape> bounds;
        size_t scratch = 0, total = 0;
        bool in_zbuf = false;
        if ((st = device_layout(levels, n_levels, d, dtype, o, &p, bounds, scratch, in_zbuf, total)) != HNV_OK)
            return st;
        *bytes = total;
        return HNV_OK;
    } catch (const std::bad_alloc &) {
        return fail(HNV_ENOMEM, "host allocation failed in hnv_plan_workspace_bytes_device");
    }
}

extern "C" hnv_status hnv_plan_create_device(const hnv_level_dev *levels, const hnv_map *maps, int n_levels, int d,
                                             hnv_dtype dtype, const hnv_options *opts, int validate_inputs,
                                             void *workspace, size_t ws_bytes, void *stream, hnv_plan **out)
{
    clear_error();
    if (!out)
        return fail(HNV_EINVAL, "out is NULL");
    *out = nullptr;
    hnv_options o;
    resolve_options(opts, d, dtype, &o);
    hnv_status st = check_plan_options(d, dtype, o);
    if (st == HNV_OK)
        st = check_levels(levels, maps, n_levels);
    if (st != HNV_OK)
        return st;
    if (!workspace || (reinterpret_cast<uintptr_t>(workspace) & 255) != 0)
        return fail(HNV_EWORKSPACE, "workspace must be non-NULL and 256-byte aligned");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    hnv_plan *p = nullptr;
    try {
        p = new hnv_plan;
        std::vector<LevelShape> bounds;
        size_t scratch_bytes = 0, total = 0;
        bool in_zbuf = false;
        if ((st = device_layout(levels, n_levels, d, dtype, o, p, bounds, scratch_bytes, in_zbuf, total)) != HNV_OK) {
            delete p;
            return st;
        }
        if (total > ws_bytes) {
            delete p;
            return fail(HNV_EWORKSPACE, "workspace of " + std::to_string(ws_bytes) + " bytes, need " +
                                            std::to_string(total));
        }
        char *base = static_cast<char *>(workspace);
        carve(p, bounds, base);
        char *scratch_base = in_zbuf ? static_cast<char *>(p->zbuf) : base + p->ws_bytes;
        LevelMeta *meta = reinterpret_cast<LevelMeta *>(scratch_base);
        char *level_base = scratch_base + meta_bytes(n_levels);
        // Each level's checks, then its build, all enqueued without waiting
        // (the build's kernels that follow offsets and ids are gated on the
        // check flags); then the one synchronisation of the build: every
        // level's flags and tier counts read together.
        const bool full = validate_inputs != 0;
        const int64_t meta_words = (int64_t)n_levels * (int64_t)sizeof(LevelMeta) / 4;
        k_fill<<<grid_for(meta_words), kThreads, 0, s>>>(reinterpret_cast<int32_t *>(meta), meta_words, 0);
        for (int l = 0; l < n_levels && st == HNV_OK; ++l) {
            Scratch S{};
            const int64_t nch = (int64_t)bounds[l].n_chunks[0] + bounds[l].n_chunks[1];
            const hnv_level_dev *C = l + 1 < n_levels ? &levels[l + 1] : nullptr;
            if ((st = scratch_layout(bounds[l].nnz, bounds[l].rows, nch, 2 * (p->small_max + 3), level_base, S)) ==
                    HNV_OK &&
                (st = launch_checks(levels[l], C, C ? &maps[l] : nullptr, full, S, meta[l].flags, s)) == HNV_OK)
                st = build_level(p, levels, maps, n_levels, l, &meta[l], S, s);
        }
        std::vector<LevelMeta> h(n_levels);
        if (st == HNV_OK)
            st = read_back(h.data(), meta, h.size() * sizeof(LevelMeta), s);
        for (int l = 0; l < n_levels && st == HNV_OK; ++l)
            st = report_checks(l, h[l].flags, full);
        for (int l = 0; l < n_levels && st == HNV_OK; ++l)
            st = finish_level(p, l, h[l].counts);
        if (st == HNV_OK)
            p->ws_bytes = total;
        if (st != HNV_OK) {
            delete p;
            return st;
        }
    } catch (const std::bad_alloc &) {
        delete p;
        return fail(HNV_ENOMEM, "host allocation failed in hnv_plan_create_device");
    }
    *out = p;
    return HNV_OK;
}

extern "C" hnv_status hnv_score_workspace_bytes_device(int64_t n_cand, int64_t n_members, int d, hnv_dtype dtype,
                                                      size_t *bytes)
{
    clear_error();
    if (!bytes)
        return fail(HNV_EINVAL, "bytes is NULL");
    ScoreDevLayout L;
    hnv_status st = score_dev_layout(n_cand, n_members, d, dtype, L);
    if (st == HNV_OK)
        *bytes = L.total;
    return st;
}

extern "C" hnv_status hnv_score_plan_create_device(const int32_t *cand_ptr, const int32_t *cand_idx, int64_t n_cand,
                                                   int64_t n_members, int64_t z_rows, int d, hnv_dtype dtype,
                                                   void *workspace, size_t ws_bytes, void *stream,
                                                   hnv_score_plan **out)
{
    clear_error();
    if (!out)
        return fail(HNV_EINVAL, "out is NULL");
    *out = nullptr;
    if (z_rows < 0 || !cand_ptr || (n_members > 0 && !cand_idx))
        return fail(HNV_EINVAL, "bad arguments");
    if (!workspace || (reinterpret_cast<uintptr_t>(workspace) & 255))
        return fail(HNV_EWORKSPACE, "workspace must be non-NULL and 256-byte aligned");
    ScoreDevLayout L;
    hnv_status st = score_dev_layout(n_cand, n_members, d, dtype, L);
    if (st != HNV_OK)
        return st;
    if (L.total > ws_bytes)
        return fail(HNV_EWORKSPACE, "workspace of " + std::to_string(ws_bytes) + " bytes, need " +
                                        std::to_string(L.total));
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    char *base = static_cast<char *>(workspace);
    Scratch S{};
    if ((st = scratch_layout(n_members, n_cand, L.n_chunks, L.small_max + 3, base + L.off_scratch, S)) != HNV_OK)
        return st;
    // checks: offsets (start 0, never decrease, end at n_members) and member
    // ids in [0, z_rows); empty candidates are allowed (their rows are NaN)
    k_fill<<<1, kThreads, 0, s>>>(S.flag, 4, 0);
    if (n_cand > 0)
        k_check_edges<<<grid_for(n_cand), kThreads, 0, s>>>(cand_ptr, nullptr, n_cand, n_members, 0, S.flag);
    if (n_members > 0)
        k_check_members<<<grid_for(n_members), kThreads, 0, s>>>(cand_ptr, cand_idx, nullptr, z_rows, n_cand,
                                                                n_members, 0, S.flag);
    if ((st = dev_check("candidate checks")) != HNV_OK)
        return st;
    int bad = 0;
    if ((st = read_back(&bad, S.flag, sizeof(int), s)) != HNV_OK)
        return st;
    if (n_cand == 0) {
        int32_t p0 = 0;
        if ((st = read_back(&p0, cand_ptr, 4, s)) != HNV_OK)
            return st;
        if (p0 != 0 || n_members != 0)
            bad |= 1;
    }
    if (bad & 1)
        return fail(HNV_EINVAL, "cand_ptr must start at 0, never decrease and end at n_members");
    if (bad & 2)
        return fail(HNV_ERANGE, "a member id is outside [0, z_rows)");
    // members, then the work lists as the host score plan lays them out
    if ((st = copy_d2d(base + L.off_idx, cand_idx, 4 * (size_t)n_members, s)) != HNV_OK)
        return st;
    int64_t cnt[4] = {0, 0, 0, 0};
    DevSide D{};
    D.small = reinterpret_cast<const Item *>(base + L.off_small);
    D.chunks = reinterpret_cast<const Item *>(base + L.off_chunks);
    D.splits = reinterpret_cast<const Split *>(base + L.off_splits);
    if (n_cand > 0) {
        D.ptr = cand_ptr;
        TierSides TS{};
        TS.n = 1;
        TS.s[0] = tier_side(D, n_cand, 0, nullptr);
        TS.total = n_cand;
        if ((st = tier_scan(TS, L.small_max, kScoreChunk, nullptr, S, S.counts, s)) != HNV_OK ||
            (st = tier_emit(TS, kScoreChunk, L.n_chunks, nullptr, S, S.counts, s)) != HNV_OK ||
            (st = read_back(cnt, S.counts, sizeof(cnt), s)) != HNV_OK)
            return st;
        if (cnt[0] > L.n_small || cnt[1] > L.n_chunks || cnt[2] > L.n_splits || cnt[3] > L.n_slots)
            return fail(HNV_EDEVICE, "work lists exceed their bounds");
    }
    hipError_t e = hipStreamSynchronize(s);
    if (e != hipSuccess)
        return fail(HNV_EDEVICE, std::string("hipStreamSynchronize: ") + hipGetErrorString(e));
    try {
        auto *plan = new hnv_score_plan;
        plan->n_cand = n_cand;
        plan->z_rows = z_rows;
        plan->d = d;
        plan->dtype = dtype;
        plan->sp.idx = reinterpret_cast<const int32_t *>(base + L.off_idx);
        plan->sp.small = D.small;
        plan->sp.n_small = (int32_t)cnt[0];
        plan->sp.chunks = D.chunks;
        plan->sp.n_chunks = (int32_t)cnt[1];
        plan->sp.splits = D.splits;
        plan->sp.n_splits = (int32_t)cnt[2];
        plan->sp.partials = reinterpret_cast<float *>(base + L.off_part);
        *out = plan;
    } catch (const std::bad_alloc &) {
        return fail(HNV_ENOMEM, "host allocation failed in hnv_score_plan_create_device");
    }
    return HNV_OK;
}

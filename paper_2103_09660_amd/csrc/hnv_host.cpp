// Host side of the HyperNetVec refinement library: error plumbing, input
// validation, featureless coarsening (Section 3.1, Algorithm 1), and the
// plan: star-expansion adjacency in both directions, degree-tiered work
// lists, projection row maps and their inverse, all carved out of the
// caller's device workspace.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <limits>
#include <memory>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "hnv_internal.h"

namespace hnv {

static thread_local std::string g_error;

hnv_status fail(hnv_status st, const std::string &msg)
{
    g_error = msg;
    return st;
}

void clear_error() { g_error.clear(); }

int next_pow2(int x)
{
    int p = 1;
    while (p < x)
        p <<= 1;
    return p;
}

int64_t blocks_for(int64_t items, int64_t per_block) { return (items + per_block - 1) / per_block; }

void lane_layout(int cols, int elem, int *lanes, int *elems_per_lane)
{
    // FP32 slices of 128 columns or more take 32 B per lane so that a
    // wavefront still covers four rows; narrower ones, and BF16, 16 B.
    int epl = 16 / elem;
    if (elem == 4 && cols / epl > 16)
        epl = 8;
    *elems_per_lane = epl;
    *lanes = next_pow2((cols + epl - 1) / epl);
}

static constexpr int64_t kMaxI32 = std::numeric_limits<int32_t>::max();
static constexpr int kDefaultSmallMax = 64;
static constexpr int kDefaultChunk = 512;

// ---------------------------------------------------------------------------
// host parallelism
// ---------------------------------------------------------------------------

// Threads for host loops: OMP_NUM_THREADS if set, else the hardware count.
static int host_threads()
{
    int t = 0;
    if (const char *e = std::getenv("OMP_NUM_THREADS"))
        t = std::atoi(e);
    if (t <= 0)
        t = (int)std::thread::hardware_concurrency();
    return std::max(1, std::min(t, 64));
}

// f(begin, end) over [0, n) in contiguous static chunks.  Every loop run this
// way writes disjoint outputs (or commutative atomic counts), so results do
// not depend on the thread count.
template <class F>
static void parallel_for(int64_t n, F f, int64_t grain = 1 << 15)
{
    const int T = (int)std::max<int64_t>(1, std::min<int64_t>(host_threads(), n / grain));
    if (T <= 1) {
        f((int64_t)0, n);
        return;
    }
    std::vector<std::thread> pool;
    pool.reserve(T);
    for (int t = 0; t < T; ++t) {
        const int64_t b = n * t / T, e = n * (t + 1) / T;
        pool.emplace_back([=, &f] { f(b, e); });
    }
    for (auto &th : pool)
        th.join();
}

// ---------------------------------------------------------------------------
// validation
// ---------------------------------------------------------------------------

// One hyperedge's checks; the message names the first violation.
static hnv_status check_edge(const hnv_level *lv, int64_t e, bool full)
{
    const int64_t a = lv->edge_ptr[e], b = lv->edge_ptr[e + 1];
    if (b < a || b > lv->nnz)
        return fail(HNV_EINVAL, "edge_ptr decreases at hyperedge " + std::to_string(e));
    if (full && b == a)
        return fail(HNV_EINVAL, "hyperedge " + std::to_string(e) + " is empty");
    for (int64_t j = a; j < b; ++j) {
        const int32_t v = lv->edge_idx[j];
        if (v < 0 || v >= lv->n_nodes)
            return fail(HNV_ERANGE, "member " + std::to_string(v) + " of hyperedge " + std::to_string(e) +
                                        " outside [0, n_nodes)");
        if (full && j > a && lv->edge_idx[j - 1] >= v)
            return fail(HNV_EUNSORTED, "members of hyperedge " + std::to_string(e) + " are not strictly ascending");
    }
    if (full && lv->edge_w) {
        const float w = lv->edge_w[e];
        if (!(w > 0.0f) || !std::isfinite(w))
            return fail(HNV_EINVAL, "weight of hyperedge " + std::to_string(e) + " is not finite and > 0");
    }
    return HNV_OK;
}

static bool edge_ok(const hnv_level *lv, int64_t e, bool full)
{
    const int64_t a = lv->edge_ptr[e], b = lv->edge_ptr[e + 1];
    if (b < a || b > lv->nnz || (full && b == a))
        return false;
    for (int64_t j = a; j < b; ++j) {
        const int32_t v = lv->edge_idx[j];
        if (v < 0 || v >= lv->n_nodes || (full && j > a && lv->edge_idx[j - 1] >= v))
            return false;
    }
    return !(full && lv->edge_w && (!(lv->edge_w[e] > 0.0f) || !std::isfinite(lv->edge_w[e])));
}

// A CSC given with the level must be the exact transpose of the CSR: offsets
// from 0 to nnz that never decrease, and, walking the hyperedges in
// ascending id, every member v's next unread CSC entry is that hyperedge.
// Each entry is then read exactly once, so the lists hold precisely the
// hyperedges of each node in ascending order.  Needs the CSR checked first.
static hnv_status check_csc(const hnv_level *lv)
{
    if (!lv->node_ptr && !lv->node_idx)
        return HNV_OK;
    if (!lv->node_ptr || (!lv->node_idx && lv->nnz > 0))
        return fail(HNV_EINVAL, "node_ptr and node_idx must both be given or both be NULL");
    const int64_t nV = lv->n_nodes;
    if (lv->node_ptr[0] != 0 || lv->node_ptr[nV] != lv->nnz)
        return fail(HNV_EINVAL, "node_ptr must start at 0 and end at nnz");
    for (int64_t v = 0; v < nV; ++v)
        if (lv->node_ptr[v + 1] < lv->node_ptr[v])
            return fail(HNV_EINVAL, "node_ptr decreases at node " + std::to_string(v));
    std::vector<int64_t> next(lv->node_ptr, lv->node_ptr + nV);
    for (int64_t e = 0; e < lv->n_edges; ++e)
        for (int64_t j = lv->edge_ptr[e]; j < lv->edge_ptr[e + 1]; ++j) {
            const int32_t v = lv->edge_idx[j];
            if (next[v] >= lv->node_ptr[v + 1] || lv->node_idx[next[v]] != e)
                return fail(HNV_EINVAL, "node_idx is not the transpose of edge_idx (node " + std::to_string(v) +
                                            ", hyperedge " + std::to_string(e) + ")");
            ++next[v];
        }
    return HNV_OK;
}

// full = false checks only what memory safety needs (offsets and index
// ranges); full = true also checks ordering, emptiness and weights.  The
// offsets are checked first, then the hyperedges in parallel ranges; the
// error reported is the one of the lowest failing hyperedge.  A CSC given
// with the level is always checked (the kernels trust it).
static hnv_status validate(const hnv_level *lv, bool full = true)
{
    if (!lv)
        return fail(HNV_EINVAL, "level is NULL");
    if (lv->n_nodes < 0 || lv->n_edges < 0 || lv->nnz < 0)
        return fail(HNV_EINVAL, "negative size");
    if (lv->n_nodes + lv->n_edges >= kMaxI32 || lv->nnz >= kMaxI32)
        return fail(HNV_EUNSUPPORTED, "rows and nnz must be below 2^31");
    if (!lv->edge_ptr || (lv->nnz > 0 && !lv->edge_idx))
        return fail(HNV_EINVAL, "edge_ptr / edge_idx is NULL");
    if (lv->edge_ptr[0] != 0 || lv->edge_ptr[lv->n_edges] != lv->nnz)
        return fail(HNV_EINVAL, "edge_ptr must start at 0 and end at nnz");
    // a hyperedge's members are read only once every earlier offset is known
    // not to decrease, so no read leaves [0, nnz)
    for (int64_t e = 0; e < lv->n_edges; ++e)
        if (lv->edge_ptr[e + 1] < lv->edge_ptr[e] || lv->edge_ptr[e + 1] > lv->nnz)
            return fail(HNV_EINVAL, "edge_ptr decreases at hyperedge " + std::to_string(e));
    std::atomic<int64_t> first_bad{std::numeric_limits<int64_t>::max()};
    parallel_for(lv->n_edges, [&](int64_t eb, int64_t ee) {
        for (int64_t e = eb; e < ee; ++e)
            if (!edge_ok(lv, e, full)) {
                int64_t cur = first_bad.load();
                while (e < cur && !first_bad.compare_exchange_weak(cur, e)) {
                }
                return;
            }
    }, 1 << 14);
    const int64_t e = first_bad.load();
    if (e != std::numeric_limits<int64_t>::max())
        return check_edge(lv, e, full);
    return check_csc(lv);
}

// ---------------------------------------------------------------------------
// coarsening
// ---------------------------------------------------------------------------

// Per-(range, node) incidence counts: the hyperedges are cut into T
// contiguous ranges of about equal incidence count and thread t counts its
// range's incidences per node.  Returns the cut points; cnt[t * nV + v]
// becomes the offset of range t's first incidence of v within v's list, and
// nptr the node offsets.  Integer counts, so the result does not depend on
// the thread count.
static std::vector<int64_t> count_by_node(const hnv_level *lv, std::vector<int32_t> &cnt, std::vector<int32_t> &nptr)
{
    const int64_t nV = lv->n_nodes, nE = lv->n_edges, nnz = lv->nnz;
    const int T = (int)std::max<int64_t>(1, std::min<int64_t>(host_threads(), nnz / (1 << 16)));
    std::vector<int64_t> cut(T + 1, nE);
    cut[0] = 0;
    for (int t = 1; t < T; ++t)
        cut[t] = std::upper_bound(lv->edge_ptr, lv->edge_ptr + nE + 1, nnz * t / T) - lv->edge_ptr - 1;
    cnt.assign((size_t)T * nV, 0);
    parallel_for(T, [&](int64_t tb, int64_t te) {
        for (int64_t t = tb; t < te; ++t) {
            int32_t *c = cnt.data() + t * nV;
            for (int64_t j = lv->edge_ptr[cut[t]]; j < lv->edge_ptr[cut[t + 1]]; ++j)
                ++c[lv->edge_idx[j]];
        }
    }, 1);
    nptr.assign(nV + 1, 0);
    parallel_for(nV, [&](int64_t vb, int64_t ve) {
        for (int64_t v = vb; v < ve; ++v) {
            int32_t run = 0;
            for (int t = 0; t < T; ++t) {
                const int32_t c = cnt[(size_t)t * nV + v];
                cnt[(size_t)t * nV + v] = run;
                run += c;
            }
            nptr[v + 1] = run;
        }
    });
    for (int64_t v = 0; v < nV; ++v)
        nptr[v + 1] += nptr[v];
    return cut;
}

// node -> incident hyperedges, each list in ascending hyperedge id: after
// count_by_node, thread t fills its range's slots.  Ranges are in hyperedge
// order, so every list comes out ascending without atomics or sorting,
// whatever the thread count.
static void incidence_by_node(const hnv_level *lv, std::vector<int32_t> &nptr, std::vector<int32_t> &nedge)
{
    std::vector<int32_t> cnt;
    const std::vector<int64_t> cut = count_by_node(lv, cnt, nptr);
    const int T = (int)cut.size() - 1;
    const int64_t nV = lv->n_nodes;
    nedge.resize(lv->nnz);
    parallel_for(T, [&](int64_t tb, int64_t te) {
        for (int64_t t = tb; t < te; ++t) {
            int32_t *c = cnt.data() + t * nV;
            for (int64_t e = cut[t]; e < cut[t + 1]; ++e)
                for (int64_t j = lv->edge_ptr[e]; j < lv->edge_ptr[e + 1]; ++j) {
                    const int32_t v = lv->edge_idx[j];
                    nedge[nptr[v] + c[v]++] = (int32_t)e;
                }
        }
    }, 1);
}

static hnv_status coarsen(const hnv_level *lv, int32_t *node_rep, int32_t *edge_rep, int64_t *c_ptr,
                          int32_t *c_idx, float *c_w, int64_t *c_nodes, int64_t *c_edges, int64_t *c_nnz)
{
    const int64_t nV = lv->n_nodes, nE = lv->n_edges;
    std::vector<int32_t> nptr, nedge;
    incidence_by_node(lv, nptr, nedge);

    // Assignment key of a hyperedge: larger weight wins, then fewer members,
    // then the lower id.  choice[v] = -1 for a node without hyperedges.
    auto wt = [&](int32_t e) { return lv->edge_w ? lv->edge_w[e] : 1.0f; };
    auto size = [&](int32_t e) { return lv->edge_ptr[e + 1] - lv->edge_ptr[e]; };
    std::vector<int32_t> choice(nV, -1);
    parallel_for(nV, [&](int64_t vb, int64_t ve) {
        for (int64_t v = vb; v < ve; ++v) {
            int32_t best = -1;
            for (int32_t j = nptr[v]; j < nptr[v + 1]; ++j) {
                const int32_t e = nedge[j];
                if (best < 0) {
                    best = e;
                    continue;
                }
                const float we = wt(e), wb = wt(best);
                const int64_t se = size(e), sb = size(best);
                if (we > wb || (we == wb && (se < sb || (se == sb && e < best))))
                    best = e;
            }
            choice[v] = best;
        }
    });

    // Coarse node numbering: first appearance of a group in ascending v.
    std::vector<int32_t> group_of_edge(nE, -1);
    std::vector<int64_t> chosen_count(nE, 0);
    int32_t n_groups = 0;
    for (int64_t v = 0; v < nV; ++v) {
        const int32_t e = choice[v];
        if (e < 0) {
            node_rep[v] = n_groups++;
            continue;
        }
        if (group_of_edge[e] < 0)
            group_of_edge[e] = n_groups++;
        node_rep[v] = group_of_edge[e];
        ++chosen_count[e];
    }

    // A hyperedge is removed when every member chose it (count == size).
    int32_t kept = 0;
    for (int64_t e = 0; e < nE; ++e)
        edge_rep[e] = (chosen_count[e] == size((int32_t)e)) ? -1 : kept++;

    // Coarse member sets through rep(), ascending, repeats collapsed: map and
    // sort every kept row in place in a scratch copy, count its distinct
    // members, then lay the rows out in order.
    std::vector<int32_t> mapped(lv->nnz);
    std::vector<int64_t> distinct(nE, 0);
    parallel_for(nE, [&](int64_t eb, int64_t ee) {
        for (int64_t e = eb; e < ee; ++e) {
            if (edge_rep[e] < 0)
                continue;
            const int64_t a = lv->edge_ptr[e], b = lv->edge_ptr[e + 1];
            for (int64_t j = a; j < b; ++j)
                mapped[j] = node_rep[lv->edge_idx[j]];
            std::sort(mapped.begin() + a, mapped.begin() + b);
            distinct[e] = std::unique(mapped.begin() + a, mapped.begin() + b) - (mapped.begin() + a);
        }
    }, 1 << 12);
    c_ptr[0] = 0;
    for (int64_t e = 0; e < nE; ++e)
        if (edge_rep[e] >= 0)
            c_ptr[edge_rep[e] + 1] = c_ptr[edge_rep[e]] + distinct[e];
    parallel_for(nE, [&](int64_t eb, int64_t ee) {
        for (int64_t e = eb; e < ee; ++e) {
            if (edge_rep[e] < 0)
                continue;
            std::copy(mapped.begin() + lv->edge_ptr[e], mapped.begin() + lv->edge_ptr[e] + distinct[e],
                      c_idx + c_ptr[edge_rep[e]]);
            if (c_w)
                c_w[edge_rep[e]] = wt((int32_t)e);
        }
    }, 1 << 12);
    *c_nodes = n_groups;
    *c_edges = kept;
    *c_nnz = c_ptr[kept];
    return HNV_OK;
}

// ---------------------------------------------------------------------------
// plan construction
// ---------------------------------------------------------------------------

struct HostTier {
    std::vector<Item> small;
    std::vector<Item> chunks;
    std::vector<Split> splits;
};

// Rows with at most small_max neighbours: ordered by degree (descending,
// then row) so that the rows sharing a wavefront have equal trip counts.
// Longer rows: cut into chunks of at most `chunk` neighbours; a row of more
// than one chunk gets consecutive partial slots.  Chunks are ordered longest
// first so the heaviest work starts earliest.
static void tier_side(const int32_t *ptr, int32_t n_rows, int small_max, int chunk, int32_t *slot_base,
                      HostTier &t)
{
    std::vector<int32_t> count(small_max + 2, 0);
    int64_t n_small = 0;
    for (int32_t r = 0; r < n_rows; ++r) {
        const int32_t deg = ptr[r + 1] - ptr[r];
        if (deg <= small_max) {
            ++count[small_max - deg + 1];
            ++n_small;
        }
    }
    for (int k = 0; k <= small_max; ++k)
        count[k + 1] += count[k];
    t.small.assign(n_small, Item{0, 0, 0, 0});
    t.chunks.clear();
    t.splits.clear();
    for (int32_t r = 0; r < n_rows; ++r) {
        const int32_t deg = ptr[r + 1] - ptr[r];
        if (deg <= small_max) {
            t.small[count[small_max - deg]++] = Item{r, ptr[r], deg, 0};
            continue;
        }
        const int32_t pieces = (deg + chunk - 1) / chunk;
        if (pieces == 1) {
            t.chunks.push_back(Item{r, ptr[r], deg, -1});
            continue;
        }
        t.splits.push_back(Split{r, *slot_base, pieces, deg});
        for (int32_t k = 0; k < pieces; ++k) {
            const int32_t s = ptr[r] + k * chunk;
            t.chunks.push_back(Item{r, s, std::min(chunk, ptr[r + 1] - s), *slot_base + k});
        }
        *slot_base += pieces;
    }
    std::stable_sort(t.chunks.begin(), t.chunks.end(), [](const Item &a, const Item &b) { return a.len > b.len; });
}

struct HostLevel {
    int64_t nV = 0, nE = 0, nnz = 0, rows = 0, rows_c = 0;
    bool has_coarse = false;
    std::vector<int32_t> ptr[2], idx[2], cidx[2];
    HostTier tier[2];
    int32_t n_slots = 0;
    std::vector<int32_t> rowmap, inv_ptr, inv_idx;
};

void resolve_options(const hnv_options *in, int d, hnv_dtype dtype, hnv_options *out)
{
    hnv_options o{};
    if (in)
        o = *in;
    // Rows wider than 256 bytes run in passes of 256-byte column slices (64
    // FP32 or 128 BF16 columns): 16 lanes per slice keep four rows per
    // wavefront, measured faster than wider slices at fewer rows per
    // wavefront despite reading the indices once per pass.
    if (o.panel_cols <= 0) {
        const int pc = (dtype == HNV_F32) ? 64 : 128;
        o.panel_cols = (d > pc && d % pc == 0) ? pc : d;
    }
    if (o.small_max <= 0)
        o.small_max = kDefaultSmallMax;
    if (o.chunk <= 0)
        o.chunk = kDefaultChunk;
    *out = o;
}

hnv_status check_plan_options(int d, hnv_dtype dtype, const hnv_options &o)
{
    if (d < 8 || d > 512 || d % 8 != 0)
        return fail(HNV_EUNSUPPORTED, "d must be a multiple of 8 in [8, 512]");
    if (dtype != HNV_F32 && dtype != HNV_BF16)
        return fail(HNV_EINVAL, "unknown dtype");
    if (o.panel_cols % 8 != 0 || d % o.panel_cols != 0)
        return fail(HNV_EUNSUPPORTED, "panel_cols must be a multiple of 8 dividing d");
    if (o.small_max > 4096 || o.chunk > (1 << 20))
        return fail(HNV_EUNSUPPORTED, "small_max <= 4096 and chunk <= 2^20");
    if (o.order != HNV_ORDER_JACOBI && o.order != HNV_ORDER_EDGE_FIRST)
        return fail(HNV_EINVAL, "unknown sweep order");
    return HNV_OK;
}

static hnv_status check_shape(const hnv_level *levels, const hnv_map *maps, int n_levels, int d,
                              hnv_dtype dtype, const hnv_options &o)
{
    if (!levels || n_levels < 1)
        return fail(HNV_EINVAL, "need at least one level");
    if (n_levels > 1 && !maps)
        return fail(HNV_EINVAL, "maps is NULL with more than one level");
    if (hnv_status st = check_plan_options(d, dtype, o); st != HNV_OK)
        return st;
    for (int l = 0; l < n_levels; ++l) {
        const hnv_level &L = levels[l];
        if (L.n_nodes < 0 || L.n_edges < 0 || L.nnz < 0 || !L.edge_ptr || (L.nnz > 0 && !L.edge_idx))
            return fail(HNV_EINVAL, "level " + std::to_string(l) + ": bad sizes or NULL arrays");
        if (L.n_nodes + L.n_edges >= kMaxI32 || L.nnz >= kMaxI32)
            return fail(HNV_EUNSUPPORTED, "level " + std::to_string(l) + ": rows and nnz must be below 2^31");
        if (L.n_nodes + L.n_edges > levels[0].n_nodes + levels[0].n_edges)
            return fail(HNV_EUNSUPPORTED, "level " + std::to_string(l) +
                                              " has more rows than level 0 (iterates live in buffers of its size)");
        if (l + 1 < n_levels && (!maps[l].node_rep || (L.n_edges > 0 && !maps[l].edge_rep)))
            return fail(HNV_EINVAL, "map " + std::to_string(l) + " has a NULL array");
        // a caller's CSC: its offsets size the node side before the full
        // transpose check, so they are checked here
        if (L.node_ptr || L.node_idx) {
            if (!L.node_ptr || (!L.node_idx && L.nnz > 0))
                return fail(HNV_EINVAL, "level " + std::to_string(l) + ": node_ptr and node_idx must both be given "
                                                                           "or both be NULL");
            if (L.node_ptr[0] != 0 || L.node_ptr[L.n_nodes] != L.nnz)
                return fail(HNV_EINVAL, "level " + std::to_string(l) + ": node_ptr must start at 0 and end at nnz");
            for (int64_t v = 0; v < L.n_nodes; ++v)
                if (L.node_ptr[v + 1] < L.node_ptr[v])
                    return fail(HNV_EINVAL, "level " + std::to_string(l) + ": node_ptr decreases at node " +
                                                std::to_string(v));
        }
    }
    return HNV_OK;
}

static hnv_status check_map(const hnv_level &f, const hnv_level &c, const hnv_map &m, int l, bool full)
{
    for (int64_t v = 0; v < f.n_nodes; ++v)
        if (m.node_rep[v] < 0 || m.node_rep[v] >= c.n_nodes)
            return fail(HNV_ERANGE, "map " + std::to_string(l) + ": node_rep[" + std::to_string(v) + "] out of range");
    for (int64_t e = 0; e < f.n_edges; ++e) {
        const int32_t r = m.edge_rep[e];
        if (r < -1 || r >= c.n_edges)
            return fail(HNV_ERANGE, "map " + std::to_string(l) + ": edge_rep[" + std::to_string(e) + "] out of range");
        if (r == -1 && f.edge_ptr[e + 1] == f.edge_ptr[e])
            return fail(HNV_ERANGE, "map " + std::to_string(l) + ": removed hyperedge " + std::to_string(e) +
                                        " has no members");
        if (full && r == -1) {
            const int32_t first = m.node_rep[f.edge_idx[f.edge_ptr[e]]];
            for (int64_t j = f.edge_ptr[e]; j < f.edge_ptr[e + 1]; ++j)
                if (m.node_rep[f.edge_idx[j]] != first)
                    return fail(HNV_ERANGE, "map " + std::to_string(l) + ": removed hyperedge " + std::to_string(e) +
                                                " has members in different coarse nodes");
        }
    }
    return HNV_OK;
}

// Builds the host arrays of one level (with_arrays = false: only what the
// workspace size needs).
static void build_level(const hnv_level *levels, const hnv_map *maps, int n_levels, int l, const hnv_options &o,
                        int small_max, bool with_arrays, HostLevel &h)
{
    const hnv_level &L = levels[l];
    h.nV = L.n_nodes;
    h.nE = L.n_edges;
    h.nnz = L.nnz;
    h.rows = h.nV + h.nE;
    h.has_coarse = (l + 1 < n_levels);
    h.rows_c = h.has_coarse ? levels[l + 1].n_nodes + levels[l + 1].n_edges : 0;

    // side 0: hyperedge rows -> member nodes (Z row = node id)
    h.ptr[0].resize(h.nE + 1);
    for (int64_t e = 0; e <= h.nE; ++e)
        h.ptr[0][e] = (int32_t)L.edge_ptr[e];
    // side 1: node rows -> incident hyperedges (Z row = n_nodes + e), the
    // caller's CSC (checked to be the transpose) or derived from the CSR
    if (L.node_ptr) {
        h.ptr[1].resize(h.nV + 1);
        for (int64_t v = 0; v <= h.nV; ++v)
            h.ptr[1][v] = (int32_t)L.node_ptr[v];
        if (with_arrays)
            h.idx[1].assign(L.node_idx, L.node_idx + h.nnz);
    } else if (with_arrays) {
        incidence_by_node(&L, h.ptr[1], h.idx[1]);
    } else {
        std::vector<int32_t> cnt;
        count_by_node(&L, cnt, h.ptr[1]);
    }

    int32_t slots = 0;
    tier_side(h.ptr[0].data(), (int32_t)h.nE, small_max, o.chunk, &slots, h.tier[0]);
    tier_side(h.ptr[1].data(), (int32_t)h.nV, small_max, o.chunk, &slots, h.tier[1]);
    h.n_slots = slots;
    if (!with_arrays)
        return;

    h.idx[0].assign(L.edge_idx, L.edge_idx + h.nnz);
    parallel_for(h.nnz, [&](int64_t b, int64_t e) {
        for (int64_t j = b; j < e; ++j)
            h.idx[1][j] += (int32_t)h.nV;
    });
    if (!h.has_coarse)
        return;

    // Projection row map: node v -> rep(v); kept hyperedge -> rep(e);
    // removed hyperedge -> the coarse node its members were merged into.
    const hnv_map &m = maps[l];
    const int64_t nVc = levels[l + 1].n_nodes;
    h.rowmap.resize(h.rows);
    for (int64_t v = 0; v < h.nV; ++v)
        h.rowmap[v] = m.node_rep[v];
    for (int64_t e = 0; e < h.nE; ++e) {
        const int32_t r = m.edge_rep[e];
        h.rowmap[h.nV + e] = (r >= 0) ? (int32_t)(nVc + r) : m.node_rep[L.edge_idx[L.edge_ptr[e]]];
    }
    for (int s = 0; s < 2; ++s) {
        h.cidx[s].resize(h.nnz);
        parallel_for(h.nnz, [&](int64_t b, int64_t e) {
            for (int64_t j = b; j < e; ++j)
                h.cidx[s][j] = h.rowmap[h.idx[s][j]];
        });
        // lane-group items carry the coarse row their own value comes from
        const int64_t base = (s == 0) ? h.nV : 0;
        for (auto &it : h.tier[s].small)
            it.aux = h.rowmap[base + it.row];
    }
    // inverse map: fine rows of each coarse row, ascending
    h.inv_ptr.assign(h.rows_c + 1, 0);
    for (int64_t u = 0; u < h.rows; ++u)
        ++h.inv_ptr[h.rowmap[u] + 1];
    for (int64_t r = 0; r < h.rows_c; ++r)
        h.inv_ptr[r + 1] += h.inv_ptr[r];
    h.inv_idx.resize(h.rows);
    std::vector<int32_t> cursor(h.inv_ptr.begin(), h.inv_ptr.end() - 1);
    for (int64_t u = 0; u < h.rows; ++u)
        h.inv_idx[cursor[h.rowmap[u]]++] = (int32_t)u;
}

struct Carver {
    char *base;
    size_t off = 0;
    template <class T>
    T *take(int64_t count)
    {
        off = (off + 255) & ~size_t(255);
        T *p = base ? reinterpret_cast<T *>(base + off) : nullptr;
        off += size_t(std::max<int64_t>(count, 1)) * sizeof(T);
        return p;
    }
};

void forward_geometry(const hnv_plan *p, const LevelPlan &L, int64_t *main_blocks, int64_t *fin_blocks)
{
    const int64_t rows_per_block = kRowsPerGroup * kBlock / p->g_fwd;
    int64_t per_panel = 0;
    for (int s = 0; s < 2; ++s)
        per_panel += blocks_for(L.n_chunks[s], kWavesPerBlock) + blocks_for(L.n_small[s], rows_per_block);
    int64_t fin = 0;
    for (int s = 0; s < 2; ++s)
        fin += blocks_for(L.n_splits[s], kWavesPerBlock);
    *main_blocks = per_panel * p->panels;
    *fin_blocks = fin * p->panels;
}

static LevelShape shape_of(const HostLevel &h, bool unit_w)
{
    LevelShape sh;
    sh.nV = h.nV;
    sh.nE = h.nE;
    sh.nnz = h.nnz;
    sh.rows = h.rows;
    sh.rows_c = h.rows_c;
    sh.has_coarse = h.has_coarse;
    sh.unit_w = unit_w;
    for (int s = 0; s < 2; ++s) {
        sh.n_small[s] = (int32_t)h.tier[s].small.size();
        sh.n_chunks[s] = (int32_t)h.tier[s].chunks.size();
        sh.n_splits[s] = (int32_t)h.tier[s].splits.size();
    }
    sh.n_slots = h.n_slots;
    return sh;
}

// Lays out the workspace (base == nullptr: sizing only) and fills the
// plan's device pointers and work-list counts.
void carve(hnv_plan *p, const std::vector<LevelShape> &shape, char *base)
{
    Carver c{base};
    const size_t elem = (p->dtype == HNV_BF16) ? 2 : 4;
    int64_t max_nodes = 1;
    p->max_slots = 1;
    p->max_resid_blocks = 1;
    for (int l = 0; l < p->n_levels; ++l) {
        const LevelShape &h = shape[l];
        LevelPlan &L = p->lv[l];
        for (int s = 0; s < 2; ++s) {
            DevSide &S = L.side[s];
            S.n_rows = (int32_t)(s == 0 ? h.nE : h.nV);
            S.row_base = (int32_t)(s == 0 ? h.nV : 0);
            S.ptr = c.take<int32_t>(S.n_rows + 1);
            S.idx = c.take<int32_t>(h.nnz);
            S.cidx = h.has_coarse ? c.take<int32_t>(h.nnz) : nullptr;
            S.wn = (s == 1) ? c.take<float>(h.nnz) : nullptr;
            S.sn = c.take<float>(h.nnz);
            S.n_small = h.n_small[s];
            S.n_chunks = h.n_chunks[s];
            S.n_splits = h.n_splits[s];
            S.small = c.take<Item>(S.n_small);
            S.small_ids = c.take<InlineIds>(S.n_small);
            S.small_cids = h.has_coarse ? c.take<InlineIds>(S.n_small) : nullptr;
            S.chunks = c.take<Item>(S.n_chunks);
            S.splits = c.take<Split>(S.n_splits);
            L.n_small[s] = S.n_small;
            L.n_chunks[s] = S.n_chunks;
            L.n_splits[s] = S.n_splits;
        }
        L.r = c.take<float>(h.rows);
        L.w = c.take<float>(h.nE);
        if (h.has_coarse) {
            L.rowmap = c.take<int32_t>(h.rows);
            L.inv_ptr = c.take<int32_t>(h.rows_c + 1);
            L.inv_idx = c.take<int32_t>(h.rows);
        }
        L.n_slots = h.n_slots;
        max_nodes = std::max(max_nodes, h.nV);
        p->max_slots = std::max<int64_t>(p->max_slots, h.n_slots);
        int64_t mb = 0, fb = 0;
        forward_geometry(p, L, &mb, &fb);
        p->max_resid_blocks = std::max(p->max_resid_blocks, mb + fb);
    }
    p->zbuf = c.take<char>(p->lv[0].rows * p->d * (int64_t)elem);
    p->partials = c.take<float>(p->max_slots * p->pstride);
    p->resid_part = c.take<double>(kResidBatch * p->max_resid_blocks);
    p->resid_stage_len = blocks_for(p->max_resid_blocks, kBlock * 8) + 1;
    p->resid_stage = c.take<double>(2 * kResidBatch * p->resid_stage_len);
    p->cscratch = c.take<float>(max_nodes);
    p->resid_tmp = c.take<double>(1);
    p->ctl = c.take<SweepCtl>(1);
    p->ctl_flags = c.take<int32_t>(2 * (int64_t)p->n_levels);
    p->ws_bytes = (c.off + 255) & ~size_t(255);
}

void init_plan_shape(hnv_plan *p, const std::vector<LevelShape> &shape, int d, hnv_dtype dtype,
                     const hnv_options &o)
{
    const int n_levels = (int)shape.size();
    p->n_levels = n_levels;
    p->d = d;
    p->dtype = dtype;
    p->opts = o;
    p->dp = o.panel_cols;
    p->panels = d / o.panel_cols;
    const int elem = (dtype == HNV_BF16) ? 2 : 4;
    lane_layout(p->dp, elem, &p->g_fwd, &p->epl_fwd);
    lane_layout(d, elem, &p->g_full, &p->epl_full);
    p->small_max = std::min(o.small_max, kIdxRegs * p->g_fwd);
    p->pstride = d + 8;
    p->lv.assign(n_levels, LevelPlan{});
    for (int l = 0; l < n_levels; ++l) {
        LevelPlan &L = p->lv[l];
        L.n_nodes = shape[l].nV;
        L.n_edges = shape[l].nE;
        L.nnz = shape[l].nnz;
        L.rows = L.n_nodes + L.n_edges;
        L.has_coarse = (l + 1 < n_levels);
        L.rows_coarse = L.has_coarse ? shape[l + 1].nV + shape[l + 1].nE : 0;
        L.unit_w = shape[l].unit_w;
    }
}

// Sizes of host levels (work-list counts unknown yet).
static std::vector<LevelShape> sizes_of(const hnv_level *levels, int n_levels)
{
    std::vector<LevelShape> sh(n_levels);
    for (int l = 0; l < n_levels; ++l) {
        sh[l].nV = levels[l].n_nodes;
        sh[l].nE = levels[l].n_edges;
        sh[l].nnz = levels[l].nnz;
        sh[l].rows = sh[l].nV + sh[l].nE;
        sh[l].has_coarse = (l + 1 < n_levels);
        sh[l].rows_c = sh[l].has_coarse ? levels[l + 1].n_nodes + levels[l + 1].n_edges : 0;
        sh[l].unit_w = (levels[l].edge_w == nullptr);
    }
    return sh;
}

}  // namespace hnv

using namespace hnv;

// ---------------------------------------------------------------------------
// C ABI (host-only calls)
// ---------------------------------------------------------------------------

extern "C" int hnv_abi_version(void) { return HNV_ABI_VERSION; }

extern "C" const char *hnv_last_error(void) { return g_error.c_str(); }

extern "C" hnv_status hnv_validate_level(const hnv_level *level)
{
    clear_error();
    return validate(level);
}

extern "C" hnv_status hnv_coarsen_level(const hnv_level *fine, int32_t *node_rep, int32_t *edge_rep,
                                        int64_t *c_edge_ptr, int32_t *c_edge_idx, float *c_edge_w,
                                        int64_t *c_n_nodes, int64_t *c_n_edges, int64_t *c_nnz)
{
    clear_error();
    hnv_status st = validate(fine);
    if (st != HNV_OK)
        return st;
    if ((fine->n_nodes > 0 && !node_rep) || (fine->n_edges > 0 && !edge_rep) || !c_edge_ptr ||
        (fine->nnz > 0 && !c_edge_idx) || !c_n_nodes || !c_n_edges || !c_nnz)
        return fail(HNV_EINVAL, "an output array is NULL");
    try {
        return coarsen(fine, node_rep, edge_rep, c_edge_ptr, c_edge_idx, c_edge_w, c_n_nodes, c_n_edges, c_nnz);
    } catch (const std::bad_alloc &) {
        return fail(HNV_ENOMEM, "host allocation failed in hnv_coarsen_level");
    }
}

extern "C" hnv_status hnv_plan_workspace_bytes(const hnv_level *levels, const hnv_map *maps, int n_levels, int d,
                                               hnv_dtype dtype, const hnv_options *opts, size_t *bytes)
{
    clear_error();
    if (!bytes)
        return fail(HNV_EINVAL, "bytes is NULL");
    hnv_options o;
    resolve_options(opts, d, dtype, &o);
    hnv_status st = check_shape(levels, maps, n_levels, d, dtype, o);
    if (st != HNV_OK)
        return st;
    try {
        hnv_plan p;
        std::vector<LevelShape> sh = sizes_of(levels, n_levels);
        init_plan_shape(&p, sh, d, dtype, o);
        for (int l = 0; l < n_levels; ++l) {
            HostLevel h;
            build_level(levels, maps, n_levels, l, o, p.small_max, false, h);
            sh[l] = shape_of(h, sh[l].unit_w);
        }
        carve(&p, sh, nullptr);
        *bytes = p.ws_bytes;
        return HNV_OK;
    } catch (const std::bad_alloc &) {
        return fail(HNV_ENOMEM, "host allocation failed in hnv_plan_workspace_bytes");
    }
}

static hnv_status upload(void *dst, const void *src, size_t bytes, hipStream_t s)
{
    if (bytes == 0)
        return HNV_OK;
    hipError_t e = hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, s);
    if (e != hipSuccess)
        return fail(HNV_EDEVICE, std::string("hipMemcpyAsync: ") + hipGetErrorString(e));
    return HNV_OK;
}

extern "C" hnv_status hnv_plan_create(const hnv_level *levels, const hnv_map *maps, int n_levels, int d,
                                      hnv_dtype dtype, const hnv_options *opts, int validate_inputs,
                                      void *workspace, size_t ws_bytes, void *stream, hnv_plan **out)
{
    clear_error();
    if (!out)
        return fail(HNV_EINVAL, "out is NULL");
    *out = nullptr;
    hnv_options o;
    resolve_options(opts, d, dtype, &o);
    hnv_status st = check_shape(levels, maps, n_levels, d, dtype, o);
    if (st != HNV_OK)
        return st;
    if (!workspace || (reinterpret_cast<uintptr_t>(workspace) & 255) != 0)
        return fail(HNV_EWORKSPACE, "workspace must be non-NULL and 256-byte aligned");
    // Offsets, index ranges and map ranges are always checked (the kernels
    // trust them); validate_inputs adds ordering, emptiness and weights.
    for (int l = 0; l < n_levels; ++l) {
        st = validate(&levels[l], validate_inputs != 0);
        if (st != HNV_OK)
            return fail(st, "level " + std::to_string(l) + ": " + g_error);
        if (l + 1 < n_levels) {
            st = check_map(levels[l], levels[l + 1], maps[l], l, validate_inputs != 0);
            if (st != HNV_OK)
                return st;
        }
    }
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    hnv_plan *p = nullptr;
    try {
        p = new hnv_plan;
        std::vector<LevelShape> sh = sizes_of(levels, n_levels);
        init_plan_shape(p, sh, d, dtype, o);
        // sizing pass (work-list counts only), then carve for real
        {
            for (int l = 0; l < n_levels; ++l) {
                HostLevel h;
                build_level(levels, maps, n_levels, l, o, p->small_max, false, h);
                sh[l] = shape_of(h, sh[l].unit_w);
            }
            carve(p, sh, nullptr);
            if (p->ws_bytes > ws_bytes) {
                const size_t need = p->ws_bytes;
                delete p;
                return fail(HNV_EWORKSPACE, "workspace of " + std::to_string(ws_bytes) + " bytes, need " +
                                                std::to_string(need));
            }
            carve(p, sh, reinterpret_cast<char *>(workspace));
        }
        // one level at a time: build host arrays, upload, wait, free
        for (int l = 0; l < n_levels; ++l) {
            HostLevel h;
            build_level(levels, maps, n_levels, l, o, p->small_max, true, h);
            LevelPlan &L = p->lv[l];
            for (int sd = 0; sd < 2; ++sd) {
                DevSide &S = L.side[sd];
                if ((st = upload((void *)S.ptr, h.ptr[sd].data(), h.ptr[sd].size() * 4, s)) != HNV_OK ||
                    (st = upload((void *)S.idx, h.idx[sd].data(), h.idx[sd].size() * 4, s)) != HNV_OK ||
                    (S.cidx && (st = upload((void *)S.cidx, h.cidx[sd].data(), h.cidx[sd].size() * 4, s)) != HNV_OK) ||
                    (st = upload((void *)S.small, h.tier[sd].small.data(), h.tier[sd].small.size() * sizeof(Item), s)) != HNV_OK ||
                    (st = upload((void *)S.chunks, h.tier[sd].chunks.data(), h.tier[sd].chunks.size() * sizeof(Item), s)) != HNV_OK ||
                    (st = upload((void *)S.splits, h.tier[sd].splits.data(), h.tier[sd].splits.size() * sizeof(Split), s)) != HNV_OK)
                    break;
            }
            if (st == HNV_OK && L.has_coarse) {
                if ((st = upload(L.rowmap, h.rowmap.data(), h.rowmap.size() * 4, s)) == HNV_OK &&
                    (st = upload(L.inv_ptr, h.inv_ptr.data(), h.inv_ptr.size() * 4, s)) == HNV_OK)
                    st = upload(L.inv_idx, h.inv_idx.data(), h.inv_idx.size() * 4, s);
            }
            std::vector<float> w(L.n_edges, 1.0f);
            if (st == HNV_OK && levels[l].edge_w)
                std::copy(levels[l].edge_w, levels[l].edge_w + L.n_edges, w.begin());
            if (st == HNV_OK)
                st = upload(L.w, w.data(), w.size() * 4, s);
            if (st == HNV_OK) {
                hipError_t e = hipStreamSynchronize(s);
                if (e != hipSuccess)
                    st = fail(HNV_EDEVICE, std::string("hipStreamSynchronize: ") + hipGetErrorString(e));
            }
            if (st == HNV_OK)
                st = dev_recompute_reciprocals(p, l, stream);
            if (st == HNV_OK)
                st = dev_fill_inline_ids(p, l, s);
            if (st != HNV_OK) {
                delete p;
                return st;
            }
        }
        hipError_t e = hipStreamSynchronize(s);
        if (e != hipSuccess) {
            delete p;
            return fail(HNV_EDEVICE, std::string("hipStreamSynchronize: ") + hipGetErrorString(e));
        }
    } catch (const std::bad_alloc &) {
        delete p;
        return fail(HNV_ENOMEM, "host allocation failed in hnv_plan_create");
    }
    *out = p;
    return HNV_OK;
}

extern "C" hnv_status hnv_plan_destroy(hnv_plan *plan)
{
    clear_error();
    delete plan;
    return HNV_OK;
}

extern "C" hnv_status hnv_plan_level_info(const hnv_plan *plan, int level, int64_t *n_nodes, int64_t *n_edges,
                                          int64_t *nnz)
{
    clear_error();
    if (!plan || level < 0 || level >= plan->n_levels)
        return fail(HNV_EINVAL, "bad plan or level");
    const LevelPlan &L = plan->lv[level];
    if (n_nodes)
        *n_nodes = L.n_nodes;
    if (n_edges)
        *n_edges = L.n_edges;
    if (nnz)
        *nnz = L.nnz;
    return HNV_OK;
}

// ---------------------------------------------------------------------------
// hyperedge-prediction features: host plan
// ---------------------------------------------------------------------------

namespace hnv {


struct ScoreLayout {
    HostTier tier;
    int32_t slots = 0;
    size_t bytes = 0;
    size_t off_idx = 0, off_small = 0, off_chunks = 0, off_splits = 0, off_part = 0;
};

static hnv_status score_layout(const int64_t *cand_ptr, int64_t n_cand, int d, hnv_dtype dtype, ScoreLayout &L)
{
    if (n_cand < 0 || (n_cand > 0 && !cand_ptr))
        return fail(HNV_EINVAL, "bad candidate arrays");
    if (d < 8 || d > 512 || d % 8 != 0)
        return fail(HNV_EUNSUPPORTED, "d must be a multiple of 8 in [8, 512]");
    if (dtype != HNV_F32 && dtype != HNV_BF16)
        return fail(HNV_EINVAL, "unknown dtype");
    if (n_cand >= kMaxI32)
        return fail(HNV_EUNSUPPORTED, "too many candidates");
    if (n_cand == 0) {
        L.bytes = 256;
        return HNV_OK;
    }
    if (cand_ptr[0] != 0)
        return fail(HNV_EINVAL, "cand_ptr must start at 0");
    for (int64_t c = 0; c < n_cand; ++c)
        if (cand_ptr[c + 1] < cand_ptr[c])
            return fail(HNV_EINVAL, "cand_ptr decreases at candidate " + std::to_string(c));
    const int64_t nnz = cand_ptr[n_cand];
    if (nnz >= kMaxI32)
        return fail(HNV_EUNSUPPORTED, "at most 2^31 - 1 members");
    std::vector<int32_t> ptr32(n_cand + 1);
    for (int64_t c = 0; c <= n_cand; ++c)
        ptr32[c] = (int32_t)cand_ptr[c];
    int G = 1, E = 8;
    lane_layout(d, dtype == HNV_BF16 ? 2 : 4, &G, &E);
    tier_side(ptr32.data(), (int32_t)n_cand, kIdxRegs * G, kScoreChunk, &L.slots, L.tier);
    Carver c{nullptr};
    c.take<int32_t>(nnz);
    L.off_idx = 0;
    c.take<Item>((int64_t)L.tier.small.size());
    L.off_small = (c.off - std::max<size_t>(L.tier.small.size(), 1) * sizeof(Item));
    c.take<Item>((int64_t)L.tier.chunks.size());
    L.off_chunks = (c.off - std::max<size_t>(L.tier.chunks.size(), 1) * sizeof(Item));
    c.take<Split>((int64_t)L.tier.splits.size());
    L.off_splits = (c.off - std::max<size_t>(L.tier.splits.size(), 1) * sizeof(Split));
    c.take<float>((int64_t)std::max<int32_t>(L.slots, 1) * (2 * d + 8));
    L.off_part = (c.off - (size_t)std::max<int32_t>(L.slots, 1) * (2 * d + 8) * sizeof(float));
    L.bytes = (c.off + 255) & ~size_t(255);
    return HNV_OK;
}

}  // namespace hnv

extern "C" hnv_status hnv_score_workspace_bytes(const int64_t *cand_ptr, int64_t n_cand, int d, hnv_dtype dtype,
                                                size_t *bytes)
{
    clear_error();
    if (!bytes)
        return fail(HNV_EINVAL, "bytes is NULL");
    try {
        ScoreLayout L;
        hnv_status st = score_layout(cand_ptr, n_cand, d, dtype, L);
        if (st == HNV_OK)
            *bytes = L.bytes;
        return st;
    } catch (const std::bad_alloc &) {
        return fail(HNV_ENOMEM, "host allocation failed in hnv_score_workspace_bytes");
    }
}

extern "C" hnv_status hnv_score_plan_create(const int64_t *cand_ptr, const int32_t *cand_idx, int64_t n_cand,
                                            int64_t z_rows, int d, hnv_dtype dtype, void *workspace,
                                            size_t ws_bytes, void *stream, hnv_score_plan **out)
{
    clear_error();
    if (!out)
        return fail(HNV_EINVAL, "out is NULL");
    *out = nullptr;
    if (z_rows < 0 || (n_cand > 0 && !workspace))
        return fail(HNV_EINVAL, "bad arguments");
    if (reinterpret_cast<uintptr_t>(workspace) & 255)
        return fail(HNV_EWORKSPACE, "workspace must be 256-byte aligned");
    try {
        ScoreLayout L;
        hnv_status st = score_layout(cand_ptr, n_cand, d, dtype, L);
        if (st != HNV_OK)
            return st;
        if (n_cand > 0 && L.bytes > ws_bytes)
            return fail(HNV_EWORKSPACE, "workspace of " + std::to_string(ws_bytes) + " bytes, need " +
                                            std::to_string(L.bytes));
        const int64_t nnz = n_cand > 0 ? cand_ptr[n_cand] : 0;
        if (nnz > 0 && !cand_idx)
            return fail(HNV_EINVAL, "cand_idx is NULL");
        for (int64_t j = 0; j < nnz; ++j)
            if (cand_idx[j] < 0 || cand_idx[j] >= z_rows)
                return fail(HNV_ERANGE, "member id " + std::to_string(cand_idx[j]) + " outside [0, z_rows)");
        auto *plan = new hnv_score_plan;
        plan->n_cand = n_cand;
        plan->z_rows = z_rows;
        plan->d = d;
        plan->dtype = dtype;
        if (n_cand > 0) {
            char *base = static_cast<char *>(workspace);
            hipStream_t s = reinterpret_cast<hipStream_t>(stream);
            auto up = [&](size_t off, const void *src, size_t n) -> hnv_status {
                if (n == 0)
                    return HNV_OK;
                hipError_t e = hipMemcpyAsync(base + off, src, n, hipMemcpyHostToDevice, s);
                return e == hipSuccess ? HNV_OK
                                       : fail(HNV_EDEVICE, std::string("hipMemcpyAsync: ") + hipGetErrorString(e));
            };
            if ((st = up(L.off_idx, cand_idx, (size_t)nnz * 4)) == HNV_OK &&
                (st = up(L.off_small, L.tier.small.data(), L.tier.small.size() * sizeof(Item))) == HNV_OK &&
                (st = up(L.off_chunks, L.tier.chunks.data(), L.tier.chunks.size() * sizeof(Item))) == HNV_OK &&
                (st = up(L.off_splits, L.tier.splits.data(), L.tier.splits.size() * sizeof(Split))) == HNV_OK) {
                hipError_t e = hipStreamSynchronize(s);
                if (e != hipSuccess)
                    st = fail(HNV_EDEVICE, std::string("hipStreamSynchronize: ") + hipGetErrorString(e));
            }
            if (st != HNV_OK) {
                delete plan;
                return st;
            }
            plan->sp.idx = reinterpret_cast<const int32_t *>(base + L.off_idx);
            plan->sp.small = reinterpret_cast<const Item *>(base + L.off_small);
            plan->sp.n_small = (int32_t)L.tier.small.size();
            plan->sp.chunks = reinterpret_cast<const Item *>(base + L.off_chunks);
            plan->sp.n_chunks = (int32_t)L.tier.chunks.size();
            plan->sp.splits = reinterpret_cast<const Split *>(base + L.off_splits);
            plan->sp.n_splits = (int32_t)L.tier.splits.size();
            plan->sp.partials = reinterpret_cast<float *>(base + L.off_part);
        }
        *out = plan;
        return HNV_OK;
    } catch (const std::bad_alloc &) {
        return fail(HNV_ENOMEM, "host allocation failed in hnv_score_plan_create");
    }
}

extern "C" hnv_status hnv_score_plan_destroy(hnv_score_plan *plan)
{
    clear_error();
    delete plan;
    return HNV_OK;
}

extern "C" hnv_status hnv_score_candidates(hnv_score_plan *plan, const void *z, int op, float *out, void *stream)
{
    clear_error();
    if (!plan)
        return fail(HNV_EINVAL, "plan is NULL");
    if (op < HNV_SCORE_VARIANCE || op > HNV_SCORE_MAX)
        return fail(HNV_EINVAL, "unknown statistic");
    if (plan->n_cand == 0)
        return HNV_OK;
    if (!z || !out)
        return fail(HNV_EINVAL, "NULL argument");
    if ((reinterpret_cast<uintptr_t>(z) & 15) || (reinterpret_cast<uintptr_t>(out) & 15))
        return fail(HNV_EINVAL, "z and out must be 16-byte aligned");
    return dev_score(plan->sp, z, plan->dtype, plan->d, op, out, reinterpret_cast<hipStream_t>(stream));
}

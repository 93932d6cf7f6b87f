// Coarsening of one level on the GPU (Section 3.1, Algorithm 1).  The
// featureless form has the same reading as the host coarsening in
// hnv_host.cpp and the same maps bit for bit:
//   1. every hyperedge gets a rank in the order (weight descending, size
//      ascending, id ascending): a stable radix sort of a 64-bit key
//      (inverted weight bits, size) over the ids;
//   2. a node's choice c(v) is its incident hyperedge of least rank: an
//      atomic minimum, which does not depend on the order of the updates;
//   3. a group's coarse id follows its smallest node: a node starts a group
//      if it has no hyperedge or is the smallest node that chose c(v); an
//      exclusive scan over those flags numbers the groups in node order;
//   4. a hyperedge is removed iff every member chose it (a count per
//      hyperedge); a scan numbers the kept ones in order;
//   5. the coarse member sets: every member mapped through rep(), a
//      segmented sort per hyperedge, the first of each run of equal values
//      flagged, one scan over the flags for positions and offsets.
// Incidence-parallel steps find their hyperedge through inc_edge (a max-scan
// of each hyperedge's id placed at its first incidence), so no thread walks a
// whole hyperedge.
// Integer work only (the key compares FP32 weights through their bit
// patterns, which order like the values for positive finite floats).
//
// With node features (bag-of-words counts), step 2 instead takes, per node,
// the hyperedge of largest cosine between the hyperedge feature (the mean of
// its members' rows) and the node's row, equal scores going to the least
// rank of step 1; the coarse node's row is the sum of its fine nodes' rows.
// The member sums, the dot products and the squared norms are exact
// integers, and the score d|d|/|s_e|^2 is one IEEE FP64 product and one
// quotient, so the choice does not depend on summation order.
#include <hip/hip_runtime.h>

#include "hnv_prim.h"

#include <climits>
#include <string>

#include "hnv_grid.h"
#include "hnv_internal.h"
#include "hnv_level_check.h"

namespace hnv {
namespace {

// Sort key of hyperedge e: the complemented weight bits above the size, which
// takes size_bits bits (a size is at most n_nodes), so that an ascending
// stable sort gives weight descending, size ascending, id ascending.
__global__ __launch_bounds__(kThreads) void k_keys(const int32_t *__restrict__ ptr, const float *__restrict__ w,
                                                   int64_t n_edges, int size_bits, uint64_t *__restrict__ keys,
                                                   int32_t *__restrict__ ids)
{
    const int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (e >= n_edges)
        return;
    const uint32_t wb = __float_as_uint(w ? w[e] : 1.0f);
    const uint32_t size = (uint32_t)(ptr[e + 1] - ptr[e]);
    keys[e] = ((uint64_t)(~wb) << size_bits) | size;
    ids[e] = (int32_t)e;
}

// rank[order[i]] = i, and the per-hyperedge and per-node accumulators of
// the choice step set to their start values (first INT_MAX, count 0, best
// INT_MAX)
__global__ __launch_bounds__(kThreads) void k_rank(const int32_t *__restrict__ order, int64_t n_edges,
                                                   int64_t n_nodes, int32_t *__restrict__ rank,
                                                   int32_t *__restrict__ first, int32_t *__restrict__ count,
                                                   int32_t *__restrict__ best)
{
    const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (i < n_edges) {
        rank[order[i]] = (int32_t)i;
        first[i] = INT_MAX;
        count[i] = 0;
    }
    if (i < n_nodes)
        best[i] = INT_MAX;
}

// no long member lists yet: the count and both bound arrays cleared
__global__ __launch_bounds__(kThreads) void k_clear_big(int32_t *__restrict__ n_big, int32_t *__restrict__ begin,
                                                        int32_t *__restrict__ end, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (i == 0)
        *n_big = 0;
    if (i < n)
        begin[i] = end[i] = 0;
}

// best[v] = least rank over the hyperedges containing v, one incidence per
// thread
__global__ __launch_bounds__(kThreads) void k_best(const int32_t *__restrict__ idx,
                                                   const int32_t *__restrict__ inc_edge,
                                                   const int32_t *__restrict__ rank, int64_t nnz,
                                                   int32_t *__restrict__ best, const int *__restrict__ bad)
{
    if (*bad)   // the step's input failed its checks
        return;
    const int64_t j = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (j >= nnz)
        return;
    // The minimum only decreases, so any value read earlier (even a stale
    // cached one) bounds the final one from above: a rank not below it
    // cannot win and needs no atomic.
    const int32_t v = idx[j], r = rank[inc_edge[j]];
    if (r < best[v])
        atomicMin(best + v, r);
}

// The same minima without global atomics, for large levels: the incidences'
// (node, rank) pairs are partitioned by the node's high bits (one stable radix
// pass, node >> shift), then one workgroup per bucket of 2^shift nodes takes
// the minima in LDS and writes the bucket's best[] once.
constexpr int kBucketShiftMax = 13;   // 8192 nodes, 32 KB of LDS per bucket
constexpr int kBucketThreads = 1024;

bool bucketed_best(int64_t n_nodes, int64_t nnz) { return nnz >= (int64_t(1) << 20) && bits_for(n_nodes) > 8; }

int bucket_shift(int64_t n_nodes) { return std::min(bits_for(n_nodes) - 8, kBucketShiftMax); }

int64_t bucket_count(int64_t n_nodes) { return ((n_nodes - 1) >> bucket_shift(n_nodes)) + 1; }

// the hyperedge rank of every incidence
__global__ __launch_bounds__(kThreads) void k_inc_rank(const int32_t *__restrict__ inc_edge,
                                                       const int32_t *__restrict__ rank, int64_t nnz,
                                                       int32_t *__restrict__ out)
{
    const int64_t j = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (j < nnz)
        out[j] = rank[inc_edge[j]];
}

// start[b] = the first position of bucket b in node ids sorted on their bits
// from `shift` up (b in [0, n_buckets]; start[n_buckets] = n)
__global__ __launch_bounds__(kThreads) void k_bucket_starts(const uint32_t *__restrict__ keys, int64_t n,
                                                            int shift, int64_t n_buckets,
                                                            int64_t *__restrict__ start)
{
    const int64_t b = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (b > n_buckets)
        return;
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        const int64_t mid = (lo + hi) / 2;
        if ((int64_t)(keys[mid] >> shift) < b)
            lo = mid + 1;
        else
            hi = mid;
    }
    start[b] = lo;
}

__global__ __launch_bounds__(kBucketThreads) void k_bucket_min(const uint32_t *__restrict__ keys,
                                                               const int32_t *__restrict__ vals,
                                                               const int64_t *__restrict__ start, int shift,
                                                               int64_t n_nodes, int32_t *__restrict__ best,
                                                               const int *__restrict__ bad)
{
    if (*bad)   // the step's input failed its checks
        return;
    __shared__ int32_t m[1 << kBucketShiftMax];
    const int span = 1 << shift;
    const int64_t base = (int64_t)blockIdx.x << shift;
    for (int t = threadIdx.x; t < span; t += kBucketThreads)
        m[t] = INT_MAX;
    __syncthreads();
    const int64_t a = start[blockIdx.x], b = start[blockIdx.x + 1];
    for (int64_t i = a + threadIdx.x; i < b; i += kBucketThreads)
        atomicMin(&m[(int64_t)keys[i] - base], vals[i]);
    __syncthreads();
    for (int t = threadIdx.x; t < span && base + t < n_nodes; t += kBucketThreads)
        best[base + t] = m[t];
}

// choice, then per hyperedge: smallest node that chose it, and how many did
__global__ __launch_bounds__(kThreads) void k_choice(const int32_t *__restrict__ best,
                                                     const int32_t *__restrict__ order, int64_t n_nodes,
                                                     int32_t *__restrict__ choice, int32_t *__restrict__ first,
                                                     int32_t *__restrict__ count)
{
    const int64_t v = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (v >= n_nodes)
        return;
    const int32_t b = best[v];
    const int32_t c = (b == INT_MAX) ? -1 : order[b];
    choice[v] = c;
    if (c >= 0) {
        atomicMin(first + c, (int32_t)v);
        atomicAdd(count + c, 1);
    }
}

__global__ __launch_bounds__(kThreads) void k_group_flags(const int32_t *__restrict__ choice,
                                                          const int32_t *__restrict__ first, int64_t n_nodes,
                                                          int32_t *__restrict__ flag)
{
    const int64_t v = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (v >= n_nodes)
        return;
    const int32_t c = choice[v];
    flag[v] = (c < 0 || first[c] == (int32_t)v) ? 1 : 0;
}

__global__ __launch_bounds__(kThreads) void k_node_rep(const int32_t *__restrict__ choice,
                                                       const int32_t *__restrict__ first,
                                                       const int32_t *__restrict__ gid, int64_t n_nodes,
                                                       int32_t *__restrict__ node_rep, const int *__restrict__ bad)
{
    if (*bad)   // the step's input failed its checks
        return;
    const int64_t v = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (v >= n_nodes)
        return;
    const int32_t c = choice[v];
    node_rep[v] = (c < 0) ? gid[v] : gid[first[c]];
}

__global__ __launch_bounds__(kThreads) void k_kept_flags(const int32_t *__restrict__ ptr,
                                                         const int32_t *__restrict__ count, int64_t n_edges,
                                                         int32_t *__restrict__ kept)
{
    const int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (e < n_edges)
        kept[e] = (count[e] != ptr[e + 1] - ptr[e]) ? 1 : 0;
}

__global__ __launch_bounds__(kThreads) void k_map(const int32_t *__restrict__ idx,
                                                  const int32_t *__restrict__ node_rep, int64_t nnz,
                                                  int32_t *__restrict__ mapped, const int *__restrict__ bad)
{
    if (*bad)   // the step's input failed its checks
        return;
    const int64_t j = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (j < nnz)
        mapped[j] = node_rep[idx[j]];
}

// ---------------------------------------------------------------------------
// Coarse member lists sorted per hyperedge.  A library segmented sort spends
// most of its time on per-segment overhead when, as here, most segments hold
// two to four keys.  So: lists of at most kSortThread members are sorted by
// one thread in registers (a network of 8, or of 16 above 8 members); lists
// of at most kSortWave members by one wavefront (a bitonic network over 64
// lanes x up to 16 registers); the few longer ones go to the library's
// segmented sort.  Each list's result is the same whatever order the lists
// are taken in.
// ---------------------------------------------------------------------------

constexpr int kSortThread = 16;
constexpr int kSortWave = 1024;

// Appends the lanes with `pred` to a list through one atomic per wavefront;
// returns each such lane's slot (-1 for the others).  Every lane of the
// wavefront must call it.
__device__ __forceinline__ int32_t wave_append(int32_t *counter, bool pred)
{
    const uint64_t m = __ballot(pred);
    if (m == 0)
        return -1;
    const int lane = threadIdx.x & (kWave - 1);
    const int leader = __ffsll((long long)m) - 1;
    int32_t base = 0;
    if (lane == leader)
        base = atomicAdd(counter, (int32_t)__popcll(m));
    base = __shfl(base, leader, kWave);
    return pred ? base + (int32_t)__popcll(m & ((1ull << lane) - 1ull)) : -1;
}

// Bitonic sorting network over the N registers of one thread (N a power of
// two; every index is a compile-time constant).
template <int N>
__device__ __forceinline__ void thread_bitonic(int32_t (&v)[N])
{
#pragma unroll
    for (int k = 2; k <= N; k <<= 1) {
#pragma unroll
        for (int j = k >> 1; j > 0; j >>= 1) {
#pragma unroll
            for (int i = 0; i < N; ++i) {
                const int l = i ^ j;
                if (l > i) {
                    const int32_t a = v[i], b = v[l];
                    const bool up = (i & k) == 0;
                    v[i] = up ? min(a, b) : max(a, b);
                    v[l] = up ? max(a, b) : min(a, b);
                }
            }
        }
    }
}

// One thread per hyperedge: a list of at most 8 members is sorted here with
// Batcher's odd-even merge network of 19 comparators, one of 9 to
// kSortThread members with a bitonic network of 16 (INT_MAX padding); one of
// more than kSortWave members is appended to the library sort's segment
// list (a few per level, so one atomic per wavefront that has any is
// cheap).  The lists in between are left to k_sort_wave.
__global__ __launch_bounds__(kThreads) void k_sort_short(const int32_t *__restrict__ ptr,
                                                         const int32_t *__restrict__ mapped, int64_t n_edges,
                                                         int32_t *__restrict__ sorted, int32_t *__restrict__ big_begin,
                                                         int32_t *__restrict__ big_end, int32_t *__restrict__ n_big,
                                                         const int *__restrict__ bad)
{
    if (*bad)   // the step's input failed its checks
        return;
    const int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    int32_t s = 0, n = 0;
    if (e < n_edges) {
        s = ptr[e];
        n = ptr[e + 1] - s;
    }
    if (e < n_edges && n > 8 && n <= kSortThread) {
        int32_t v[16];
#pragma unroll
        for (int i = 0; i < 16; ++i)
            v[i] = (i < n) ? mapped[s + i] : INT_MAX;
        thread_bitonic<16>(v);
#pragma unroll
        for (int i = 0; i < 16; ++i)
            if (i < n)
                sorted[s + i] = v[i];
    }
    if (e < n_edges && n <= 8) {
        int32_t v[8];
#pragma unroll
        for (int i = 0; i < 8; ++i)
            v[i] = (i < n) ? mapped[s + i] : INT_MAX;
        constexpr int net[19][2] = {{0, 1}, {2, 3}, {4, 5}, {6, 7}, {0, 2}, {1, 3}, {4, 6}, {5, 7}, {1, 2}, {5, 6},
                                    {0, 4}, {3, 7}, {1, 5}, {2, 6}, {1, 4}, {3, 6}, {2, 4}, {3, 5}, {3, 4}};
#pragma unroll
        for (int c = 0; c < 19; ++c) {
            const int32_t a = v[net[c][0]], b = v[net[c][1]];
            v[net[c][0]] = min(a, b);
            v[net[c][1]] = max(a, b);
        }
#pragma unroll
        for (int i = 0; i < 8; ++i)
            if (i < n)
                sorted[s + i] = v[i];
    }
    const bool is_big = e < n_edges && n > kSortWave;
    const int32_t b = wave_append(n_big, is_big);
    if (is_big) {
        big_begin[b] = s;
        big_end[b] = s + n;
    }
}

// Bitonic sorting network over 64 K keys held as v[r] in lane `lane`, key
// index r * 64 + lane: partners at distance j < 64 are in other lanes of the
// same register (exchanged by shuffles), at j >= 64 in other registers of
// the same lane.  All loop bounds are compile-time, so every register index
// is a constant.
template <int K>
__device__ __forceinline__ void wave_bitonic(int32_t (&v)[K], int lane)
{
    constexpr int LOGN = (K == 1) ? 6 : (K == 2) ? 7 : (K == 4) ? 8 : (K == 8) ? 9 : 10;
#pragma unroll
    for (int lk = 1; lk <= LOGN; ++lk) {
        const int k = 1 << lk;
#pragma unroll
        for (int lj = lk - 1; lj >= 0; --lj) {
            const int j = 1 << lj;
            if (j >= kWave) {
                const int rj = j / kWave;
#pragma unroll
                for (int r = 0; r < K; ++r) {
                    if (r & rj)
                        continue;
                    const bool asc = ((r * kWave) & k) == 0;   // k > 64: the direction is the register's
                    const int32_t a = v[r], b = v[r | rj];
                    v[r] = asc ? min(a, b) : max(a, b);
                    v[r | rj] = asc ? max(a, b) : min(a, b);
                }
            } else {
#pragma unroll
                for (int r = 0; r < K; ++r) {
                    const bool asc = ((r * kWave + lane) & k) == 0;
                    const int32_t y = __shfl_xor(v[r], j, kWave);
                    const bool keep_min = ((lane & j) == 0) == asc;
                    v[r] = keep_min ? min(v[r], y) : max(v[r], y);
                }
            }
        }
    }
}

template <int K>
__device__ __forceinline__ void wave_sort(const int32_t *__restrict__ in, int32_t *__restrict__ out, int n, int lane)
{
    int32_t v[K];
#pragma unroll
    for (int r = 0; r < K; ++r) {
        const int i = r * kWave + lane;
        v[r] = (i < n) ? in[i] : INT_MAX;
    }
    wave_bitonic<K>(v, lane);
#pragma unroll
    for (int r = 0; r < K; ++r) {
        const int i = r * kWave + lane;
        if (i < n)
            out[i] = v[r];
    }
}

// The lists of more than kSortThread and at most kSortWave members: each
// wavefront takes a window of 64 consecutive hyperedges (one per lane),
// finds those lists by a ballot, and sorts them one after the other with
// all 64 lanes.  No list of work, no atomics.
__global__ __launch_bounds__(kThreads) void k_sort_wave(const int32_t *__restrict__ ptr,
                                                        const int32_t *__restrict__ mapped, int64_t n_edges,
                                                        int32_t *__restrict__ sorted, const int *__restrict__ bad)
{
    if (*bad)   // the step's input failed its checks
        return;
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t window = ((int64_t)blockIdx.x * kThreads + threadIdx.x) / kWave;
    const int64_t e = window * kWave + lane;
    int32_t s = 0, n = 0;
    if (e < n_edges) {
        s = ptr[e];
        n = ptr[e + 1] - s;
    }
    uint64_t todo = __ballot(n > kSortThread && n <= kSortWave);
    while (todo) {
        const int src = __ffsll((long long)todo) - 1;
        todo &= todo - 1;
        const int32_t ss = __shfl(s, src, kWave), nn = __shfl(n, src, kWave);
        if (nn <= 64)
            wave_sort<1>(mapped + ss, sorted + ss, nn, lane);
        else if (nn <= 128)
            wave_sort<2>(mapped + ss, sorted + ss, nn, lane);
        else if (nn <= 256)
            wave_sort<4>(mapped + ss, sorted + ss, nn, lane);
        else if (nn <= 512)
            wave_sort<8>(mapped + ss, sorted + ss, nn, lane);
        else
            wave_sort<16>(mapped + ss, sorted + ss, nn, lane);
    }
}

// dflag[j] = 1 where sorted[j] starts a new distinct value inside a kept
// hyperedge's sorted mapped members
__global__ __launch_bounds__(kThreads) void k_distinct(const int32_t *__restrict__ ptr,
                                                       const int32_t *__restrict__ sorted,
                                                       const int32_t *__restrict__ inc_edge,
                                                       const int32_t *__restrict__ kept, int64_t nnz,
                                                       int32_t *__restrict__ dflag, const int *__restrict__ bad)
{
    if (*bad)   // the step's input failed its checks
        return;
    const int64_t j = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (j >= nnz)
        return;
    const int32_t e = inc_edge[j];
    dflag[j] = (kept[e] && (j == ptr[e] || sorted[j] != sorted[j - 1])) ? 1 : 0;
}

// coarse members: the flagged values at their scanned positions
__global__ __launch_bounds__(kThreads) void k_emit_members(const int32_t *__restrict__ sorted,
                                                           const int32_t *__restrict__ dflag,
                                                           const int32_t *__restrict__ dpos, int64_t nnz,
                                                           int32_t *__restrict__ c_idx, const int *__restrict__ bad)
{
    if (*bad)   // the step's input failed its checks
        return;
    const int64_t j = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (j < nnz && dflag[j])
        c_idx[dpos[j]] = sorted[j];
}

// per hyperedge: edge_rep, coarse offset (the scanned position of its first
// incidence, which is always flagged when kept) and weight
__global__ __launch_bounds__(kThreads) void k_emit_edges(const int32_t *__restrict__ ptr,
                                                         const int32_t *__restrict__ kept,
                                                         const int32_t *__restrict__ krank,
                                                         const int32_t *__restrict__ dpos,
                                                         const float *__restrict__ w, int64_t n_edges,
                                                         int32_t *__restrict__ edge_rep, int32_t *__restrict__ c_ptr,
                                                         float *__restrict__ c_w, const int *__restrict__ bad)
{
    if (*bad)   // the step's input failed its checks
        return;
    const int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (e >= n_edges)
        return;
    if (!kept[e]) {
        edge_rep[e] = -1;
        return;
    }
    const int32_t r = krank[e];
    edge_rep[e] = r;
    c_ptr[r] = dpos[ptr[e]];
    if (c_w)
        c_w[r] = w ? w[e] : 1.0f;
}

// sizes[0..2] = coarse nodes, kept hyperedges, coarse incidences; closes c_ptr
__global__ void k_sizes(const int32_t *__restrict__ gflag, const int32_t *__restrict__ gid, int64_t n_nodes,
                        const int32_t *__restrict__ kept, const int32_t *__restrict__ krank, int64_t n_edges,
                        const int32_t *__restrict__ dflag, const int32_t *__restrict__ dpos, int64_t nnz,
                        int32_t *__restrict__ c_ptr, int64_t *__restrict__ sizes, const int *__restrict__ bad)
{
    if (*bad)   // the step's input failed its checks
        return;
    if (threadIdx.x != 0 || blockIdx.x != 0)
        return;
    const int64_t nv = n_nodes ? (int64_t)gid[n_nodes - 1] + gflag[n_nodes - 1] : 0;
    const int64_t ne = n_edges ? (int64_t)krank[n_edges - 1] + kept[n_edges - 1] : 0;
    const int64_t nz = nnz ? (int64_t)dpos[nnz - 1] + dflag[nnz - 1] : 0;
    sizes[0] = nv;
    sizes[1] = ne;
    sizes[2] = nz;
    c_ptr[ne] = (int32_t)nz;
}

// ---------------------------------------------------------------------------
// feature-based assignment (bag-of-words counts, int32 [rows x k], k % 4 == 0)
// ---------------------------------------------------------------------------

// counts must be >= 0 (flag bit 4) and their total below 2^31 (checked on
// the host from `total`); with that bound every sum, product and dot below
// fits its integer type exactly
__global__ __launch_bounds__(kThreads) void k_fcheck(const int4 *__restrict__ x, int64_t n4, int *__restrict__ flag,
                                                     unsigned long long *__restrict__ total)
{
    __shared__ unsigned long long part[kThreads / kWave];
    unsigned long long sum = 0;
    int neg = 0;
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n4; i += (int64_t)gridDim.x * kThreads) {
        const int4 v = x[i];
        neg |= (v.x | v.y | v.z | v.w) < 0;
        sum += (unsigned long long)(uint32_t)v.x + (uint32_t)v.y + (uint32_t)v.z + (uint32_t)v.w;
    }
    for (int o = kWave / 2; o > 0; o >>= 1)
        sum += __shfl_xor(sum, o);
    if ((threadIdx.x & (kWave - 1)) == 0)
        part[threadIdx.x / kWave] = sum;
    if (neg)
        atomicOr(flag, 16);
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long b = 0;
        for (int w = 0; w < kThreads / kWave; ++w)
            b += part[w];
        atomicAdd(total, b);
    }
}

// Members handled together by one wavefront in the feature kernels: their
// row loads are independent, so this many rows are in flight per lane
// (fewer for wide rows held in registers, to keep the register count down).
template <int NC>
constexpr int members_in_flight()
{
    return (NC == 0 || NC <= 2) ? 4 : 8 / NC;
}

// A feature row of k counts is read by one wavefront as NC passes of 256
// counts (4 per lane, 16 B); NC is a compile-time bound (k <= 256 NC) so the
// per-lane pieces of a row live in registers.  NC = 0: any k, one pass at a
// time (wide rows).
template <int NC>
struct RowPieces {
    int4 p[NC];
    __device__ void zero()
    {
#pragma unroll
        for (int i = 0; i < NC; ++i)
            p[i] = make_int4(0, 0, 0, 0);
    }
    __device__ void load(const int32_t *row, int lane, int k)
    {
#pragma unroll
        for (int i = 0; i < NC; ++i) {
            const int c = lane * 4 + i * kWave * 4;
            p[i] = (c < k) ? *reinterpret_cast<const int4 *>(row + c) : make_int4(0, 0, 0, 0);
        }
    }
    __device__ void add(const RowPieces &o)
    {
#pragma unroll
        for (int i = 0; i < NC; ++i) {
            p[i].x += o.p[i].x;
            p[i].y += o.p[i].y;
            p[i].z += o.p[i].z;
            p[i].w += o.p[i].w;
        }
    }
    __device__ int64_t dot(const RowPieces &o) const
    {
        int64_t d = 0;
#pragma unroll
        for (int i = 0; i < NC; ++i)
            d += (int64_t)p[i].x * o.p[i].x + (int64_t)p[i].y * o.p[i].y + (int64_t)p[i].z * o.p[i].z +
                 (int64_t)p[i].w * o.p[i].w;
        return d;
    }
    __device__ void store(int32_t *row, int lane, int k) const
    {
#pragma unroll
        for (int i = 0; i < NC; ++i) {
            const int c = lane * 4 + i * kWave * 4;
            if (c < k)
                *reinterpret_cast<int4 *>(row + c) = p[i];
        }
    }
};

__device__ inline int64_t wave_sum(int64_t v)
{
    for (int o = kWave / 2; o > 0; o >>= 1)
        v += __shfl_xor(v, o);
    return v;
}

// out[r] = sum of the rows x[idx[j]], j in [ptr[r], ptr[r+1]), for r below
// *limit (all rows if limit is NULL); one wavefront per row.  SQ: also
// sq[r] = |out[r]|^2 (int64).  Integer sums: the order of the additions
// does not change the result.
template <bool SQ, int NC>
__global__ __launch_bounds__(kThreads) void k_rowsum(const int32_t *__restrict__ ptr, const int32_t *__restrict__ idx,
                                                     const int32_t *__restrict__ x, int k, int64_t n_rows,
                                                     const int64_t *__restrict__ limit, int32_t *__restrict__ out,
                                                     int64_t *__restrict__ sq)
{
    constexpr int U = members_in_flight<NC>();
    const int64_t r = linear_block() * (kThreads / kWave) + threadIdx.x / kWave;
    const int lane = threadIdx.x & (kWave - 1);
    if (r >= n_rows || (limit && r >= *limit))
        return;
    const int32_t a = ptr[r], b = ptr[r + 1];
    if constexpr (NC > 0) {
        RowPieces<NC> acc;
        acc.zero();
        int32_t j = a;
        for (; j + U <= b; j += U) {
            RowPieces<NC> m[U];
#pragma unroll
            for (int u = 0; u < U; ++u)
                m[u].load(x + (int64_t)idx[j + u] * k, lane, k);
#pragma unroll
            for (int u = 0; u < U; ++u)
                acc.add(m[u]);
        }
        for (; j < b; ++j) {
            RowPieces<NC> m;
            m.load(x + (int64_t)idx[j] * k, lane, k);
            acc.add(m);
        }
        acc.store(out + r * k, lane, k);
        if (SQ) {
            const int64_t q = wave_sum(acc.dot(acc));
            if (lane == 0)
                sq[r] = q;
        }
    } else {
        int64_t q = 0;
        for (int c = lane * 4; c < k; c += kWave * 4) {
            int4 acc = make_int4(0, 0, 0, 0);
            for (int32_t j = a; j < b; ++j) {
                const int4 v = *reinterpret_cast<const int4 *>(x + (int64_t)idx[j] * k + c);
                acc.x += v.x;
                acc.y += v.y;
                acc.z += v.z;
                acc.w += v.w;
            }
            *reinterpret_cast<int4 *>(out + r * k + c) = acc;
            if (SQ)
                q += (int64_t)acc.x * acc.x + (int64_t)acc.y * acc.y + (int64_t)acc.z * acc.z +
                     (int64_t)acc.w * acc.w;
        }
        if (SQ) {
            q = wave_sum(q);
            if (lane == 0)
                sq[r] = q;
        }
    }
}

// IEEE FP64 cosine score d|d| / |s_e|^2 (0 when s_e = 0); d and |s_e|^2 are
// exact integers, the product and the quotient are each rounded once
__device__ inline double cosine_score(int64_t d, int64_t s2)
{
    if (s2 == 0)
        return 0.0;
    const double dd = (double)d;
    const double num = dd * fabs(dd);
    return num / (double)s2;
}

// order-preserving map of a double onto unsigned 64-bit integers
__device__ inline unsigned long long ordered_bits(double q)
{
    const unsigned long long b = (unsigned long long)__double_as_longlong(q);
    return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}

// per incidence (e, v): q = cosine score of e for v, kept in CSR order;
// bestq[v] = max over v's incidences (atomic max: order-independent).
// One wavefront takes 64 consecutive incidences, whatever their hyperedges:
// lane l loads incidence l's node, hyperedge and |s_e|^2, the wavefront then
// walks the 64 in steps of score_batch (rows broadcast by __shfl, the next
// step's rows loaded before this step's reduction), and at the end lane l
// finishes incidence l.
template <int NC>
constexpr int score_batch()
{
    return (NC == 0 || NC == 1) ? 4 : NC == 2 ? 2 : 1;
}

template <int NC>
__global__ __launch_bounds__(kThreads) void k_qscore(const int32_t *__restrict__ idx,
                                                     const int32_t *__restrict__ inc_edge,
                                                     const int32_t *__restrict__ s, const int64_t *__restrict__ s2,
                                                     const int32_t *__restrict__ x, int k, int64_t nnz,
                                                     double *__restrict__ q, unsigned long long *__restrict__ bestq)
{
    constexpr int U = score_batch<NC>();
    static_assert(kWave % U == 0, "a step must divide the wavefront");
    const int64_t j0 = ((int64_t)blockIdx.x * (kThreads / kWave) + threadIdx.x / kWave) * kWave;
    const int lane = threadIdx.x & (kWave - 1);
    if (j0 >= nnz)
        return;
    const int n = (int)std::min<int64_t>(kWave, nnz - j0);
    const int32_t my_v = lane < n ? idx[j0 + lane] : 0;
    const int32_t my_e = lane < n ? inc_edge[j0 + lane] : 0;
    const int64_t my_s2 = lane < n ? s2[my_e] : 0;
    int64_t mine = 0;
    if constexpr (NC > 0) {
        RowPieces<NC> f[U], m[U];
        auto load_step = [&](int t) {
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int32_t v = __shfl(my_v, t + u), e = __shfl(my_e, t + u);
                if (t + u < n) {
                    f[u].load(s + (int64_t)e * k, lane, k);
                    m[u].load(x + (int64_t)v * k, lane, k);
                } else {
                    f[u].zero();
                    m[u].zero();
                }
            }
        };
        load_step(0);
        for (int t = 0; t < n; t += U) {
            int64_t d[U];
#pragma unroll
            for (int u = 0; u < U; ++u)
                d[u] = f[u].dot(m[u]);
            if (t + U < n)
                load_step(t + U);
            for (int o = kWave / 2; o > 0; o >>= 1) {
#pragma unroll
                for (int u = 0; u < U; ++u)
                    d[u] += __shfl_xor(d[u], o);
            }
#pragma unroll
            for (int u = 0; u < U; ++u)
                if (lane == t + u)
                    mine = d[u];
        }
    } else {
        for (int t = 0; t < n; ++t) {
            const int32_t v = __shfl(my_v, t), e = __shfl(my_e, t);
            int64_t d = 0;
            for (int c = lane * 4; c < k; c += kWave * 4) {
                const int4 fc = *reinterpret_cast<const int4 *>(s + (int64_t)e * k + c);
                const int4 mc = *reinterpret_cast<const int4 *>(x + (int64_t)v * k + c);
                d += (int64_t)fc.x * mc.x + (int64_t)fc.y * mc.y + (int64_t)fc.z * mc.z + (int64_t)fc.w * mc.w;
            }
            d = wave_sum(d);
            if (lane == t)
                mine = d;
        }
    }
    if (lane < n) {
        const double sc = cosine_score(mine, my_s2);
        q[j0 + lane] = sc;
        const unsigned long long ob = ordered_bits(sc);
        if (ob > bestq[my_v])   // an earlier read bounds the maximum from below
            atomicMax(bestq + my_v, ob);
    }
}

// The register bound NC for a feature width k (0: wider than 2048).
inline int pieces_for(int k) { return k <= 256 ? 1 : k <= 512 ? 2 : k <= 1024 ? 4 : k <= 2048 ? 8 : 0; }

template <int NC>
void launch_edge_features(dim3 grid, hipStream_t st, const int32_t *ptr, const int32_t *idx,
                          const int32_t *inc_edge, const int32_t *x, int k, int64_t n_edges, int64_t nnz,
                          int32_t *fsum, int64_t *fsq, double *q, unsigned long long *bestq)
{
    k_rowsum<true, NC><<<grid, kThreads, 0, st>>>(ptr, idx, x, k, n_edges, nullptr, fsum, fsq);
    const int64_t waves = (nnz + kWave - 1) / kWave;
    const unsigned sgrid = (unsigned)((waves + kThreads / kWave - 1) / (kThreads / kWave));
    k_qscore<NC><<<sgrid, kThreads, 0, st>>>(idx, inc_edge, fsum, fsq, x, k, nnz, q, bestq);
}

template <int NC>
void launch_group_sums(dim3 grid, hipStream_t st, const int32_t *gptr, const int32_t *gnodes, const int32_t *x,
                       int k, int64_t n_rows, const int64_t *limit, int32_t *out)
{
    k_rowsum<false, NC><<<grid, kThreads, 0, st>>>(gptr, gnodes, x, k, n_rows, limit, out, nullptr);
}

// best[v] = least rank among v's hyperedges whose score equals bestq[v]
__global__ __launch_bounds__(kThreads) void k_best_feat(const int32_t *__restrict__ idx,
                                                        const int32_t *__restrict__ inc_edge,
                                                        const int32_t *__restrict__ rank,
                                                        const double *__restrict__ q,
                                                        const unsigned long long *__restrict__ bestq, int64_t nnz,
                                                        int32_t *__restrict__ best)
{
    const int64_t j = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (j >= nnz)
        return;
    const int32_t v = idx[j];
    if (ordered_bits(q[j]) == bestq[v]) {
        const int32_t r = rank[inc_edge[j]];
        if (r < best[v])   // an earlier read bounds the minimum from above
            atomicMin(best + v, r);
    }
}

// coarse-node member lists: count, then place (the order inside a group is
// free; the sums over it are exact integers)
__global__ __launch_bounds__(kThreads) void k_group_count(const int32_t *__restrict__ node_rep, int64_t n_nodes,
                                                          int32_t *__restrict__ gcount)
{
    const int64_t v = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (v < n_nodes)
        atomicAdd(gcount + node_rep[v], 1);
}

__global__ __launch_bounds__(kThreads) void k_group_fill(const int32_t *__restrict__ node_rep,
                                                         const int32_t *__restrict__ gptr, int64_t n_nodes,
                                                         int32_t *__restrict__ gcur, int32_t *__restrict__ gnodes)
{
    const int64_t v = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (v >= n_nodes)
        return;
    const int32_t g = node_rep[v];
    gnodes[gptr[g] + atomicAdd(gcur + g, 1)] = (int32_t)v;
}

// Member lists longer than kSortWave that one level can hold.
int64_t max_big_lists(int64_t nnz) { return nnz / (kSortWave + 1) + 1; }

// Temporary storage of the two sorts for the given key widths in bits (the
// segmented sort over at most max_big_lists segments).
hnv_status sort_storage(int64_t nE, int64_t nnz, int key_bits, int member_bits, size_t &t_keys, size_t &t_members)
{
    t_keys = t_members = 0;
    hipError_t e = prim_sort_pairs(nullptr, t_keys, (uint64_t *)nullptr, (uint64_t *)nullptr,
                                                      (int32_t *)nullptr, (int32_t *)nullptr,
                                                      (int)std::max<int64_t>(nE, 1), 0, key_bits);
    if (e == hipSuccess)
        e = prim_segmented_sort_keys(nullptr, t_members, (uint32_t *)nullptr, (uint32_t *)nullptr,
                                                       (int)std::max<int64_t>(nnz, 1), max_big_lists(nnz),
                                                       (int32_t *)nullptr, (int32_t *)nullptr, 0, member_bits);
    if (e != hipSuccess)
        return fail(HNV_EDEVICE, std::string("sort storage query (needs a visible GPU): ") + hipGetErrorString(e));
    return HNV_OK;
}

struct CoarsenLayout {
    size_t keys_in, keys_out, ids_in, order, rank, best, choice, first, count, gflag, gid, kept, krank, mapped,
        sorted, inc_edge, dflag, dpos, sizes, flag, big_begin, big_end, sort_counts, bstart;
    // feature path (k > 0)
    size_t fsum, fsq, q, bestq, gcount, gptr, gcur, gnodes;
    size_t temp, temp_bytes, total;
};

hnv_status layout(int64_t nV, int64_t nE, int64_t nnz, int k, CoarsenLayout &L)
{
    size_t off = 0;
    auto take = [&](size_t bytes) {
        off = (off + 255) & ~size_t(255);
        const size_t p = off;
        off += std::max<size_t>(bytes, 8);
        return p;
    };
    L.keys_in = take(8 * nE);
    L.keys_out = take(8 * nE);
    L.ids_in = take(4 * nE);
    L.order = take(4 * nE);
    L.rank = take(4 * nE);
    L.best = take(4 * nV);
    L.choice = take(4 * nV);
    L.first = take(4 * nE);
    L.count = take(4 * nE);
    L.gflag = take(4 * nV);
    L.gid = take(4 * nV);
    L.kept = take(4 * nE);
    L.krank = take(4 * nE);
    L.mapped = take(4 * nnz);
    L.sorted = take(4 * nnz);
    L.inc_edge = take(4 * nnz);
    L.dflag = take(4 * nnz);
    L.dpos = take(4 * nnz);
    // the check word (int flags, pad, uint64 feature total) and the coarse
    // sizes (3 x int64) side by side: one read-back takes both
    L.flag = take(16 + 8 * 4);
    L.sizes = L.flag + 16;
    L.big_begin = take(4 * max_big_lists(nnz));
    L.big_end = take(4 * max_big_lists(nnz));
    L.sort_counts = take(8);
    L.bstart = take(8 * (size_t)(std::max<int64_t>(nV >> kBucketShiftMax, 256) + 2));
    L.fsum = L.fsq = L.q = L.bestq = L.gcount = L.gptr = L.gcur = L.gnodes = 0;
    if (k > 0) {
        L.fsum = take(4 * (size_t)nE * k);
        L.fsq = take(8 * nE);
        L.q = take(8 * nnz);
        L.bestq = take(8 * nV);
        L.gcount = take(4 * (nV + 1));
        L.gptr = take(4 * (nV + 1));
        L.gcur = take(4 * nV);
        L.gnodes = take(4 * nV);
    }
    size_t t1 = 0, t2 = 0, t3 = 0, t4 = 0;
    if (hnv_status st = sort_storage(nE, nnz, 64, 32, t1, t4); st != HNV_OK)
        return st;
    hipError_t e = prim_exclusive_sum(nullptr, t2, (int32_t *)nullptr, (int32_t *)nullptr,
                                                    (int)std::max<int64_t>(nV + 1, 1));
    if (e == hipSuccess)
        e = prim_exclusive_sum(nullptr, t3, (int32_t *)nullptr, (int32_t *)nullptr,
                                             (int)std::max<int64_t>(std::max(nE, nnz), 1));
    size_t t6 = 0;
    if (e == hipSuccess && bucketed_best(nV, nnz))
        e = prim_sort_pairs(nullptr, t6, (uint32_t *)nullptr, (uint32_t *)nullptr, (int32_t *)nullptr,
                            (int32_t *)nullptr, nnz, bucket_shift(nV), bits_for(nV));
    if (e != hipSuccess)
        return fail(HNV_EDEVICE, std::string("scan storage query (needs a visible GPU): ") + hipGetErrorString(e));
    L.temp_bytes = std::max(std::max(std::max(t1, t2), std::max(t3, t4)), t6);
    L.temp = take(L.temp_bytes);
    L.total = (off + 255) & ~size_t(255);
    return HNV_OK;
}

hnv_status check_sizes(int64_t n_nodes, int64_t n_edges, int64_t nnz, int k)
{
    if (n_nodes < 0 || n_edges < 0 || nnz < 0 || k < 0)
        return fail(HNV_EINVAL, "negative size");
    if (n_nodes >= INT_MAX || n_edges >= INT_MAX || nnz >= INT_MAX)
        return fail(HNV_EUNSUPPORTED, "sizes must be below 2^31");
    if (k % 4 != 0 || k > (1 << 16) || (int64_t)n_edges * k >= INT64_MAX / 8)
        return fail(HNV_EUNSUPPORTED, "feature width k must be a multiple of 4 up to 65536");
    return HNV_OK;
}

// One coarsening step; featureless when x is NULL (k = 0), else on the
// cosine of bag-of-words features with X' summed into c_x.
hnv_status coarsen_device(int64_t n_nodes, int64_t n_edges, int64_t nnz, const int32_t *edge_ptr,
                          const int32_t *edge_idx, const float *edge_w, const int32_t *x, int k, int32_t *node_rep,
                          int32_t *edge_rep, int32_t *c_edge_ptr, int32_t *c_edge_idx, float *c_edge_w,
                          int32_t *c_x, int64_t *c_sizes, void *workspace, size_t ws_bytes, void *stream)
{
    clear_error();
    hnv_status st = check_sizes(n_nodes, n_edges, nnz, k);
    if (st != HNV_OK)
        return st;
    if (!c_sizes || !edge_ptr || !c_edge_ptr || (nnz > 0 && (!edge_idx || !c_edge_idx)) ||
        (n_nodes > 0 && !node_rep) || (n_edges > 0 && !edge_rep))
        return fail(HNV_EINVAL, "a required pointer is NULL");
    const bool feat = k > 0;
    if (feat && n_nodes > 0 && (!x || !c_x))
        return fail(HNV_EINVAL, "features: x and c_x are required");
    if (feat && ((reinterpret_cast<uintptr_t>(x) | reinterpret_cast<uintptr_t>(c_x)) & 15))
        return fail(HNV_EINVAL, "features: x and c_x must be 16-byte aligned");
    if (!workspace || (reinterpret_cast<uintptr_t>(workspace) & 255))
        return fail(HNV_EWORKSPACE, "workspace must be non-NULL and 256-byte aligned");
    CoarsenLayout L;
    if ((st = layout(n_nodes, n_edges, nnz, k, L)) != HNV_OK)
        return st;
    if (L.total > ws_bytes)
        return fail(HNV_EWORKSPACE, "workspace of " + std::to_string(ws_bytes) + " bytes, need " +
                                        std::to_string(L.total));
    char *base = static_cast<char *>(workspace);
    auto at = [&](size_t off) { return reinterpret_cast<int32_t *>(base + off); };
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const int nV = (int)n_nodes, nE = (int)n_edges, nz = (int)nnz;
    auto sync_read = [&](void *dst, const void *src, size_t n) -> hnv_status {
        hipError_t e = hipMemcpyAsync(dst, src, n, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess)
            e = hipStreamSynchronize(s);
        return e == hipSuccess ? HNV_OK : fail(HNV_EDEVICE, std::string("read-back: ") + hipGetErrorString(e));
    };

    // 0. input check (every later kernel trusts offsets, member ids, counts)
    int *flag = reinterpret_cast<int *>(base + L.flag);
    unsigned long long *total = reinterpret_cast<unsigned long long *>(base + L.flag + 8);
    k_fill<<<1, kThreads, 0, s>>>(flag, 4, 0);
    int32_t *inc_edge = at(L.inc_edge), *dflag = at(L.dflag), *dpos = at(L.dpos);
    if (nE > 0) {
        k_check_edges<<<grid_for(nE), kThreads, 0, s>>>(edge_ptr, edge_w, n_edges, nnz, 1, flag);
        if (nz > 0) {
            k_fill<<<grid_for(nz), kThreads, 0, s>>>(inc_edge, nnz, 0);
            k_inc_edge<<<grid_for(nE), kThreads, 0, s>>>(edge_ptr, n_edges, nnz, inc_edge);
            k_check_members<<<grid_for(nz), kThreads, 0, s>>>(edge_ptr, edge_idx, inc_edge, n_nodes, n_edges, nnz, 1,
                                                              flag);
        }
    }
    if (feat && nV > 0) {
        const int64_t n4 = (int64_t)nV * k / 4;
        k_fcheck<<<(unsigned)std::min<int64_t>(grid_for(n4), 2048), kThreads, 0, s>>>(
            reinterpret_cast<const int4 *>(x), n4, flag, total);
    }
    if ((st = dev_check("coarsening input check")) != HNV_OK)
        return st;
    // The checks' result: read here on the feature path; on the featureless
    // path with the coarse sizes at the end (every kernel there that follows
    // offsets or member ids, or writes an output, first reads the check
    // word and does nothing when it is set).
    struct {
        int bad, pad;
        unsigned long long total;
    } chk{};
    auto report = [&]() -> hnv_status {
        if (nE == 0) {
            int32_t p0 = 0;
            if (hnv_status r = sync_read(&p0, edge_ptr, 4); r != HNV_OK)
                return r;
            if (p0 != 0 || nz != 0)
                chk.bad |= 1;
        }
        if (chk.bad & 1)
            return fail(HNV_EINVAL, "edge_ptr: offsets must start at 0, increase, end at nnz, no empty hyperedge");
        if (chk.bad & 2)
            return fail(HNV_ERANGE, "a member id is outside [0, n_nodes)");
        if (chk.bad & 4)
            return fail(HNV_EUNSORTED, "member lists must be strictly ascending");
        if (chk.bad & 8)
            return fail(HNV_EINVAL, "weights must be finite and > 0");
        if ((chk.bad & 16) || chk.total >= (1ull << 31))
            return fail(HNV_EINVAL, "features must be counts >= 0 with a total below 2^31");
        return HNV_OK;
    };
    if (feat) {
        if ((st = sync_read(&chk, flag, sizeof(chk))) != HNV_OK || (st = report()) != HNV_OK)
            return st;
    }

    int32_t *order = at(L.order), *rank = at(L.rank), *best = at(L.best), *choice = at(L.choice);
    int32_t *first = at(L.first), *count = at(L.count), *gflag = at(L.gflag), *gid = at(L.gid);
    int32_t *kept = at(L.kept), *krank = at(L.krank), *mapped = at(L.mapped), *sorted = at(L.sorted);
    int64_t *sizes = reinterpret_cast<int64_t *>(base + L.sizes);
    void *temp = base + L.temp;
    size_t tb = L.temp_bytes;
    // Without weights every key's weight part is the same: sort the size bits
    // only.  Coarse member ids are below n_nodes.
    const int size_bits = bits_for(n_nodes + 1);
    const int key_bits = edge_w ? 32 + size_bits : size_bits, member_bits = bits_for(n_nodes);
    {
        size_t need_keys = 0, need_members = 0;
        if ((st = sort_storage(n_edges, nnz, key_bits, member_bits, need_keys, need_members)) != HNV_OK)
            return st;
        if (need_keys > L.temp_bytes || need_members > L.temp_bytes)
            return fail(HNV_EDEVICE, "sort storage exceeds the queried size");
    }
    if (nE > 0) {
        // 1. ranks in the order (weight descending, size ascending, id ascending)
        uint64_t *kin = reinterpret_cast<uint64_t *>(base + L.keys_in);
        uint64_t *kout = reinterpret_cast<uint64_t *>(base + L.keys_out);
        k_keys<<<grid_for(nE), kThreads, 0, s>>>(edge_ptr, edge_w, n_edges, size_bits, kin, at(L.ids_in));
        if (prim_sort_pairs(temp, tb, kin, kout, at(L.ids_in), order, nE, 0, key_bits, s) != hipSuccess)
            return fail(HNV_EDEVICE, "radix sort of hyperedge keys");
    }
    if (nE > 0 || nV > 0)
        k_rank<<<grid_for(std::max(nE, nV)), kThreads, 0, s>>>(order, n_edges, n_nodes, rank, first, count, best);
    if (nV > 0) {
        // 2. choices: the least rank, or (features) the least rank among the
        // hyperedges of best cosine score
        if (nE > 0 && !feat) {
            if (bucketed_best(n_nodes, nnz)) {
                // (mapped, sorted and dflag are free until step 5)
                int32_t *pr = mapped, *pr_sorted = dflag;
                uint32_t *nodes_sorted = reinterpret_cast<uint32_t *>(sorted);
                const int shift = bucket_shift(n_nodes);
                const int64_t nb = bucket_count(n_nodes);
                int64_t *bstart = reinterpret_cast<int64_t *>(base + L.bstart);
                k_inc_rank<<<grid_for(nz), kThreads, 0, s>>>(inc_edge, rank, nnz, pr);
                tb = L.temp_bytes;
                if (prim_sort_pairs(temp, tb, reinterpret_cast<const uint32_t *>(edge_idx), nodes_sorted, pr,
                                    pr_sorted, nz, shift, bits_for(n_nodes), s) != hipSuccess)
                    return fail(HNV_EDEVICE, "partition of incidences by node");
                k_bucket_starts<<<grid_for(nb + 1), kThreads, 0, s>>>(nodes_sorted, nnz, shift, nb, bstart);
                k_bucket_min<<<(unsigned)nb, kBucketThreads, 0, s>>>(nodes_sorted, pr_sorted, bstart, shift, n_nodes,
                                                                     best, flag);
            } else {
                k_best<<<grid_for(nz), kThreads, 0, s>>>(edge_idx, inc_edge, rank, nnz, best, flag);
            }
        }
        if (nE > 0 && feat) {
            int32_t *fsum = at(L.fsum);
            int64_t *fsq = reinterpret_cast<int64_t *>(base + L.fsq);
            double *q = reinterpret_cast<double *>(base + L.q);
            unsigned long long *bestq = reinterpret_cast<unsigned long long *>(base + L.bestq);
            const dim3 wave_grid = fold_grid((n_edges + kThreads / kWave - 1) / (kThreads / kWave));
            k_fill<<<grid_for(2 * (int64_t)nV), kThreads, 0, s>>>(reinterpret_cast<int32_t *>(bestq),
                                                                   2 * (int64_t)nV, 0);
            switch (pieces_for(k)) {
            case 1: launch_edge_features<1>(wave_grid, s, edge_ptr, edge_idx, inc_edge, x, k, n_edges, nnz, fsum, fsq, q, bestq); break;
            case 2: launch_edge_features<2>(wave_grid, s, edge_ptr, edge_idx, inc_edge, x, k, n_edges, nnz, fsum, fsq, q, bestq); break;
            case 4: launch_edge_features<4>(wave_grid, s, edge_ptr, edge_idx, inc_edge, x, k, n_edges, nnz, fsum, fsq, q, bestq); break;
            case 8: launch_edge_features<8>(wave_grid, s, edge_ptr, edge_idx, inc_edge, x, k, n_edges, nnz, fsum, fsq, q, bestq); break;
            default: launch_edge_features<0>(wave_grid, s, edge_ptr, edge_idx, inc_edge, x, k, n_edges, nnz, fsum, fsq, q, bestq);
            }
            k_best_feat<<<grid_for(nz), kThreads, 0, s>>>(edge_idx, inc_edge, rank, q, bestq, nnz, best);
        }
        k_choice<<<grid_for(nV), kThreads, 0, s>>>(best, order, n_nodes, choice, first, count);
        // 3. group numbering by smallest node
        k_group_flags<<<grid_for(nV), kThreads, 0, s>>>(choice, first, n_nodes, gflag);
        tb = L.temp_bytes;
        if (prim_exclusive_sum(temp, tb, gflag, gid, nV, s) != hipSuccess)
            return fail(HNV_EDEVICE, "scan of group flags");
        k_node_rep<<<grid_for(nV), kThreads, 0, s>>>(choice, first, gid, n_nodes, node_rep, flag);
    }
    if (nE > 0) {
        // 4. removed hyperedges
        k_kept_flags<<<grid_for(nE), kThreads, 0, s>>>(edge_ptr, count, n_edges, kept);
        tb = L.temp_bytes;
        if (prim_exclusive_sum(temp, tb, kept, krank, nE, s) != hipSuccess)
            return fail(HNV_EDEVICE, "scan of kept flags");
        // 5. coarse member sets: every hyperedge's mapped members sorted (short
        // lists by a thread, medium ones by a wavefront, long ones by the
        // library's segmented sort over a list of them)
        if (nz > 0) {
            k_map<<<grid_for(nz), kThreads, 0, s>>>(edge_idx, node_rep, nnz, mapped, flag);
            int32_t *big_begin = at(L.big_begin), *big_end = at(L.big_end), *n_big_dev = at(L.sort_counts);
            const int64_t n_big = max_big_lists(nnz);
            k_clear_big<<<grid_for(n_big), kThreads, 0, s>>>(n_big_dev, big_begin, big_end, n_big);
            k_sort_short<<<grid_for(nE), kThreads, 0, s>>>(edge_ptr, mapped, n_edges, sorted, big_begin, big_end,
                                                            n_big_dev, flag);
            if (nnz > kSortThread)
                k_sort_wave<<<grid_for(nE), kThreads, 0, s>>>(edge_ptr, mapped, n_edges, sorted, flag);
            if (nnz > kSortWave) {
                tb = L.temp_bytes;
                // non-negative ids: sorted as unsigned so only the low bits count;
                // unused segments are empty
                if (prim_segmented_sort_keys(temp, tb, reinterpret_cast<const uint32_t *>(mapped),
                                             reinterpret_cast<uint32_t *>(sorted), nz, n_big, big_begin, big_end, 0,
                                             member_bits, s) != hipSuccess)
                    return fail(HNV_EDEVICE, "segmented sort of long coarse member lists");
            }
        }
        k_distinct<<<grid_for(nz), kThreads, 0, s>>>(edge_ptr, sorted, inc_edge, kept, nnz, dflag, flag);
        tb = L.temp_bytes;
        if (prim_exclusive_sum(temp, tb, dflag, dpos, nz, s) != hipSuccess)
            return fail(HNV_EDEVICE, "scan of coarse members");
        k_emit_members<<<grid_for(nz), kThreads, 0, s>>>(sorted, dflag, dpos, nnz, c_edge_idx, flag);
        k_emit_edges<<<grid_for(nE), kThreads, 0, s>>>(edge_ptr, kept, krank, dpos, edge_w, n_edges, edge_rep,
                                                       c_edge_ptr, c_edge_w, flag);
    }
    k_sizes<<<1, 64, 0, s>>>(gflag, gid, n_nodes, kept, krank, n_edges, dflag, dpos, nnz, c_edge_ptr, sizes, flag);
    if (feat && nV > 0) {
        // 6. X': each coarse node's row is the sum of its fine nodes' rows
        int32_t *gcount = at(L.gcount), *gptr = at(L.gptr), *gcur = at(L.gcur), *gnodes = at(L.gnodes);
        k_fill<<<grid_for(nV + 1), kThreads, 0, s>>>(gcount, n_nodes + 1, 0);
        k_fill<<<grid_for(nV), kThreads, 0, s>>>(gcur, n_nodes, 0);
        k_group_count<<<grid_for(nV), kThreads, 0, s>>>(node_rep, n_nodes, gcount);
        tb = L.temp_bytes;
        if (prim_exclusive_sum(temp, tb, gcount, gptr, nV + 1, s) != hipSuccess)
            return fail(HNV_EDEVICE, "scan of group sizes");
        k_group_fill<<<grid_for(nV), kThreads, 0, s>>>(node_rep, gptr, n_nodes, gcur, gnodes);
        const dim3 wave_grid = fold_grid((n_nodes + kThreads / kWave - 1) / (kThreads / kWave));
        switch (pieces_for(k)) {
        case 1: launch_group_sums<1>(wave_grid, s, gptr, gnodes, x, k, n_nodes, sizes, c_x); break;
        case 2: launch_group_sums<2>(wave_grid, s, gptr, gnodes, x, k, n_nodes, sizes, c_x); break;
        case 4: launch_group_sums<4>(wave_grid, s, gptr, gnodes, x, k, n_nodes, sizes, c_x); break;
        case 8: launch_group_sums<8>(wave_grid, s, gptr, gnodes, x, k, n_nodes, sizes, c_x); break;
        default: launch_group_sums<0>(wave_grid, s, gptr, gnodes, x, k, n_nodes, sizes, c_x);
        }
    }
    if ((st = dev_check("coarsening kernels")) != HNV_OK)
        return st;
    if (feat)
        return sync_read(c_sizes, sizes, 3 * sizeof(int64_t));
    struct {
        int bad, pad;
        unsigned long long total;
        int64_t sizes[3];
    } back{};
    static_assert(sizeof(back) == 16 + 3 * sizeof(int64_t), "check word and sizes are read as one block");
    if ((st = sync_read(&back, flag, sizeof(back))) != HNV_OK)
        return st;
    chk.bad = back.bad;
    chk.total = back.total;
    if ((st = report()) != HNV_OK)
        return st;
    std::memcpy(c_sizes, back.sizes, sizeof(back.sizes));
    return HNV_OK;
}

}  // namespace
}  // namespace hnv

using namespace hnv;

extern "C" hnv_status hnv_coarsen_workspace_bytes(int64_t n_nodes, int64_t n_edges, int64_t nnz, size_t *bytes)
{
    return hnv_coarsen_features_workspace_bytes(n_nodes, n_edges, nnz, 0, bytes);
}

extern "C" hnv_status hnv_coarsen_features_workspace_bytes(int64_t n_nodes, int64_t n_edges, int64_t nnz, int k,
                                                           size_t *bytes)
{
    clear_error();
    if (!bytes)
        return fail(HNV_EINVAL, "bytes is NULL");
    hnv_status st = check_sizes(n_nodes, n_edges, nnz, k);
    if (st != HNV_OK)
        return st;
    CoarsenLayout L;
    if ((st = layout(n_nodes, n_edges, nnz, k, L)) == HNV_OK)
        *bytes = L.total;
    return st;
}

extern "C" hnv_status hnv_coarsen_level_device(int64_t n_nodes, int64_t n_edges, int64_t nnz,
                                               const int32_t *edge_ptr, const int32_t *edge_idx,
                                               const float *edge_w, int32_t *node_rep, int32_t *edge_rep,
                                               int32_t *c_edge_ptr, int32_t *c_edge_idx, float *c_edge_w,
                                               int64_t *c_sizes, void *workspace, size_t ws_bytes, void *stream)
{
    return coarsen_device(n_nodes, n_edges, nnz, edge_ptr, edge_idx, edge_w, nullptr, 0, node_rep, edge_rep,
                          c_edge_ptr, c_edge_idx, c_edge_w, nullptr, c_sizes, workspace, ws_bytes, stream);
}

extern "C" hnv_status hnv_coarsen_level_features_device(int64_t n_nodes, int64_t n_edges, int64_t nnz,
                                                        const int32_t *edge_ptr, const int32_t *edge_idx,
                                                        const float *edge_w, const int32_t *x, int k,
                                                        int32_t *node_rep, int32_t *edge_rep, int32_t *c_edge_ptr,
                                                        int32_t *c_edge_idx, float *c_edge_w, int32_t *c_x,
                                                        int64_t *c_sizes, void *workspace, size_t ws_bytes,
                                                        void *stream)
{
    if (k <= 0) {
        clear_error();
        return fail(HNV_EUNSUPPORTED, "feature width k must be a multiple of 4 up to 65536");
    }
    return coarsen_device(n_nodes, n_edges, nnz, edge_ptr, edge_idx, edge_w, x, k, node_rep, edge_rep, c_edge_ptr,
                          c_edge_idx, c_edge_w, c_x, c_sizes, workspace, ws_bytes, stream);
}

// Featureless coarsening of one level on the GPU (Section 3.1, Algorithm 1),
// with the same reading as the host coarsening in hnv_host.cpp and the same
// maps bit for bit:
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
//      segmented sort per hyperedge, distinct values counted, a scan for the
//      coarse offsets, then the distinct values copied.
// Integer work only (the key compares FP32 weights through their bit
// patterns, which order like the values for positive finite floats).
#include <hip/hip_runtime.h>

#include <hipcub/hipcub.hpp>

#include <climits>
#include <string>

#include "hnv_internal.h"

namespace hnv {
namespace {

constexpr int kThreads = 256;

inline unsigned grid_for(int64_t n) { return (unsigned)((n + kThreads - 1) / kThreads); }

// input check: bit 0 offsets, bit 1 member range, bit 2 member order, bit 3 weights
__global__ __launch_bounds__(kThreads) void k_check(const int32_t *__restrict__ ptr, const int32_t *__restrict__ idx,
                                                    const float *__restrict__ w, int64_t n_nodes, int64_t n_edges,
                                                    int64_t nnz, int *__restrict__ flag)
{
    const int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (e >= n_edges)
        return;
    const int64_t a = ptr[e], b = ptr[e + 1];
    int bad = 0;
    if (a < 0 || b < a || b > nnz || (e == 0 && a != 0) || (e == n_edges - 1 && b != nnz) || a == b)
        bad |= 1;
    if (!(bad & 1)) {
        for (int64_t j = a; j < b; ++j) {
            const int32_t v = idx[j];
            if (v < 0 || v >= n_nodes)
                bad |= 2;
            else if (j > a && idx[j - 1] >= v)
                bad |= 4;
        }
    }
    if (w && !(w[e] > 0.0f && w[e] < INFINITY))
        bad |= 8;
    if (bad)
        atomicOr(flag, bad);
}

__global__ __launch_bounds__(kThreads) void k_fill(int32_t *__restrict__ p, int64_t n, int32_t v)
{
    const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (i < n)
        p[i] = v;
}

__global__ __launch_bounds__(kThreads) void k_keys(const int32_t *__restrict__ ptr, const float *__restrict__ w,
                                                   int64_t n_edges, uint64_t *__restrict__ keys,
                                                   int32_t *__restrict__ ids)
{
    const int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (e >= n_edges)
        return;
    const uint32_t wb = __float_as_uint(w ? w[e] : 1.0f);
    const uint32_t size = (uint32_t)(ptr[e + 1] - ptr[e]);
    keys[e] = ((uint64_t)(~wb) << 32) | size;
    ids[e] = (int32_t)e;
}

__global__ __launch_bounds__(kThreads) void k_rank(const int32_t *__restrict__ order, int64_t n_edges,
                                                   int32_t *__restrict__ rank)
{
    const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (i < n_edges)
        rank[order[i]] = (int32_t)i;
}

// best[v] = least rank over the hyperedges containing v
__global__ __launch_bounds__(kThreads) void k_best(const int32_t *__restrict__ ptr, const int32_t *__restrict__ idx,
                                                   const int32_t *__restrict__ rank, int64_t n_edges,
                                                   int32_t *__restrict__ best)
{
    const int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (e >= n_edges)
        return;
    const int32_t r = rank[e];
    for (int32_t j = ptr[e]; j < ptr[e + 1]; ++j)
        atomicMin(best + idx[j], r);
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
                                                       int32_t *__restrict__ node_rep)
{
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
                                                  int32_t *__restrict__ mapped)
{
    const int64_t j = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (j < nnz)
        mapped[j] = node_rep[idx[j]];
}

// distinct values of each kept hyperedge's sorted mapped members
__global__ __launch_bounds__(kThreads) void k_distinct(const int32_t *__restrict__ ptr,
                                                       const int32_t *__restrict__ sorted,
                                                       const int32_t *__restrict__ kept, int64_t n_edges,
                                                       int32_t *__restrict__ dcount)
{
    const int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (e >= n_edges)
        return;
    int32_t n = 0;
    if (kept[e]) {
        for (int32_t j = ptr[e]; j < ptr[e + 1]; ++j)
            n += (j == ptr[e] || sorted[j] != sorted[j - 1]) ? 1 : 0;
    }
    dcount[e] = n;
}

__global__ __launch_bounds__(kThreads) void k_emit(const int32_t *__restrict__ ptr,
                                                   const int32_t *__restrict__ sorted,
                                                   const int32_t *__restrict__ kept,
                                                   const int32_t *__restrict__ krank,
                                                   const int32_t *__restrict__ cstart, const float *__restrict__ w,
                                                   int64_t n_edges, int32_t *__restrict__ edge_rep,
                                                   int32_t *__restrict__ c_ptr, int32_t *__restrict__ c_idx,
                                                   float *__restrict__ c_w)
{
    const int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (e >= n_edges)
        return;
    if (!kept[e]) {
        edge_rep[e] = -1;
        return;
    }
    const int32_t r = krank[e];
    edge_rep[e] = r;
    c_ptr[r] = cstart[e];
    if (c_w)
        c_w[r] = w ? w[e] : 1.0f;
    int32_t pos = cstart[e];
    for (int32_t j = ptr[e]; j < ptr[e + 1]; ++j)
        if (j == ptr[e] || sorted[j] != sorted[j - 1])
            c_idx[pos++] = sorted[j];
}

// sizes[0..2] = coarse nodes, kept hyperedges, coarse incidences; closes c_ptr
__global__ void k_sizes(const int32_t *__restrict__ gflag, const int32_t *__restrict__ gid, int64_t n_nodes,
                        const int32_t *__restrict__ kept, const int32_t *__restrict__ krank,
                        const int32_t *__restrict__ dcount, const int32_t *__restrict__ cstart, int64_t n_edges,
                        int32_t *__restrict__ c_ptr, int64_t *__restrict__ sizes)
{
    if (threadIdx.x != 0 || blockIdx.x != 0)
        return;
    const int64_t nv = n_nodes ? (int64_t)gid[n_nodes - 1] + gflag[n_nodes - 1] : 0;
    const int64_t ne = n_edges ? (int64_t)krank[n_edges - 1] + kept[n_edges - 1] : 0;
    const int64_t nz = n_edges ? (int64_t)cstart[n_edges - 1] + dcount[n_edges - 1] : 0;
    sizes[0] = nv;
    sizes[1] = ne;
    sizes[2] = nz;
    c_ptr[ne] = (int32_t)nz;
}

// Temporary storage of the two sorts for the given key widths in bits.
hnv_status sort_storage(int64_t nE, int64_t nnz, int key_bits, int member_bits, size_t &t_keys, size_t &t_members)
{
    t_keys = t_members = 0;
    hipError_t e = hipcub::DeviceRadixSort::SortPairs(nullptr, t_keys, (uint64_t *)nullptr, (uint64_t *)nullptr,
                                                      (int32_t *)nullptr, (int32_t *)nullptr,
                                                      (int)std::max<int64_t>(nE, 1), 0, key_bits);
    if (e == hipSuccess)
        e = hipcub::DeviceSegmentedRadixSort::SortKeys(nullptr, t_members, (uint32_t *)nullptr, (uint32_t *)nullptr,
                                                       (int)std::max<int64_t>(nnz, 1), (int)std::max<int64_t>(nE, 1),
                                                       (int32_t *)nullptr, (int32_t *)nullptr, 0, member_bits);
    if (e != hipSuccess)
        return fail(HNV_EDEVICE, std::string("sort storage query (needs a visible GPU): ") + hipGetErrorString(e));
    return HNV_OK;
}

// Bits that hold every value in [0, n).
int bits_for(int64_t n)
{
    int b = 1;
    while (b < 32 && (int64_t(1) << b) < n)
        ++b;
    return b;
}

struct CoarsenLayout {
    size_t keys_in, keys_out, ids_in, order, rank, best, choice, first, count, gflag, gid, kept, krank, mapped,
        sorted, dcount, cstart, sizes, flag, temp, temp_bytes, total;
};

hnv_status layout(int64_t nV, int64_t nE, int64_t nnz, CoarsenLayout &L)
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
    L.dcount = take(4 * nE);
    L.cstart = take(4 * nE);
    L.sizes = take(8 * 4);
    L.flag = take(8);
    size_t t1 = 0, t2 = 0, t3 = 0, t4 = 0;
    if (hnv_status st = sort_storage(nE, nnz, 64, 32, t1, t4); st != HNV_OK)
        return st;
    hipError_t e = hipcub::DeviceScan::ExclusiveSum(nullptr, t2, (int32_t *)nullptr, (int32_t *)nullptr,
                                                    (int)std::max<int64_t>(nV, 1));
    if (e == hipSuccess)
        e = hipcub::DeviceScan::ExclusiveSum(nullptr, t3, (int32_t *)nullptr, (int32_t *)nullptr,
                                             (int)std::max<int64_t>(nE, 1));
    if (e != hipSuccess)
        return fail(HNV_EDEVICE, std::string("scan storage query (needs a visible GPU): ") + hipGetErrorString(e));
    L.temp_bytes = std::max(std::max(t1, t2), std::max(t3, t4));
    L.temp = take(L.temp_bytes);
    L.total = (off + 255) & ~size_t(255);
    return HNV_OK;
}

}  // namespace
}  // namespace hnv

using namespace hnv;

extern "C" hnv_status hnv_coarsen_workspace_bytes(int64_t n_nodes, int64_t n_edges, int64_t nnz, size_t *bytes)
{
    clear_error();
    if (!bytes || n_nodes < 0 || n_edges < 0 || nnz < 0)
        return fail(HNV_EINVAL, "bad arguments");
    if (n_nodes >= INT_MAX || n_edges >= INT_MAX || nnz >= INT_MAX)
        return fail(HNV_EUNSUPPORTED, "sizes must be below 2^31");
    CoarsenLayout L;
    hnv_status st = layout(n_nodes, n_edges, nnz, L);
    if (st == HNV_OK)
        *bytes = L.total;
    return st;
}

extern "C" hnv_status hnv_coarsen_level_device(int64_t n_nodes, int64_t n_edges, int64_t nnz,
                                               const int32_t *edge_ptr, const int32_t *edge_idx,
                                               const float *edge_w, int32_t *node_rep, int32_t *edge_rep,
                                               int32_t *c_edge_ptr, int32_t *c_edge_idx, float *c_edge_w,
                                               int64_t *c_sizes, void *workspace, size_t ws_bytes, void *stream)
{
    clear_error();
    if (n_nodes < 0 || n_edges < 0 || nnz < 0 || !c_sizes || !edge_ptr || !c_edge_ptr ||
        (nnz > 0 && (!edge_idx || !c_edge_idx)) || (n_nodes > 0 && !node_rep) || (n_edges > 0 && !edge_rep))
        return fail(HNV_EINVAL, "bad arguments");
    if (n_nodes >= INT_MAX || n_edges >= INT_MAX || nnz >= INT_MAX)
        return fail(HNV_EUNSUPPORTED, "sizes must be below 2^31");
    if (!workspace || (reinterpret_cast<uintptr_t>(workspace) & 255))
        return fail(HNV_EWORKSPACE, "workspace must be non-NULL and 256-byte aligned");
    CoarsenLayout L;
    hnv_status st = layout(n_nodes, n_edges, nnz, L);
    if (st != HNV_OK)
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

    // 0. input check (every later kernel trusts offsets and member ids)
    int *flag = reinterpret_cast<int *>(base + L.flag);
    k_fill<<<1, kThreads, 0, s>>>(flag, 1, 0);
    if (nE > 0)
        k_check<<<grid_for(nE), kThreads, 0, s>>>(edge_ptr, edge_idx, edge_w, n_nodes, n_edges, nnz, flag);
    if ((st = dev_check("coarsening input check")) != HNV_OK)
        return st;
    int bad = 0;
    if (nE == 0) {
        int32_t p0 = 0;
        if ((st = sync_read(&p0, edge_ptr, 4)) != HNV_OK)
            return st;
        if (p0 != 0 || nz != 0)
            bad |= 1;
    } else if ((st = sync_read(&bad, flag, sizeof(int))) != HNV_OK) {
        return st;
    }
    if (bad & 1)
        return fail(HNV_EINVAL, "edge_ptr: offsets must start at 0, increase, end at nnz, no empty hyperedge");
    if (bad & 2)
        return fail(HNV_ERANGE, "a member id is outside [0, n_nodes)");
    if (bad & 4)
        return fail(HNV_EUNSORTED, "member lists must be strictly ascending");
    if (bad & 8)
        return fail(HNV_EINVAL, "weights must be finite and > 0");

    int32_t *order = at(L.order), *rank = at(L.rank), *best = at(L.best), *choice = at(L.choice);
    int32_t *first = at(L.first), *count = at(L.count), *gflag = at(L.gflag), *gid = at(L.gid);
    int32_t *kept = at(L.kept), *krank = at(L.krank), *mapped = at(L.mapped), *sorted = at(L.sorted);
    int32_t *dcount = at(L.dcount), *cstart = at(L.cstart);
    void *temp = base + L.temp;
    size_t tb = L.temp_bytes;
    // Without weights the upper half of every key is the same: sort the size
    // half only.  Coarse member ids are below n_nodes.
    const int key_bits = edge_w ? 64 : 32, member_bits = bits_for(n_nodes);
    {
        size_t need_keys = 0, need_members = 0;
        if ((st = sort_storage(n_edges, nnz, key_bits, member_bits, need_keys, need_members)) != HNV_OK)
            return st;
        if (need_keys > L.temp_bytes || need_members > L.temp_bytes)
            return fail(HNV_EDEVICE, "sort storage exceeds the queried size");
    }
    if (nE > 0) {
        // 1. ranks
        uint64_t *kin = reinterpret_cast<uint64_t *>(base + L.keys_in);
        uint64_t *kout = reinterpret_cast<uint64_t *>(base + L.keys_out);
        k_keys<<<grid_for(nE), kThreads, 0, s>>>(edge_ptr, edge_w, n_edges, kin, at(L.ids_in));
        if (hipcub::DeviceRadixSort::SortPairs(temp, tb, kin, kout, at(L.ids_in), order, nE, 0, key_bits, s) != hipSuccess)
            return fail(HNV_EDEVICE, "radix sort of hyperedge keys");
        k_rank<<<grid_for(nE), kThreads, 0, s>>>(order, n_edges, rank);
        k_fill<<<grid_for(nE), kThreads, 0, s>>>(first, n_edges, INT_MAX);
        k_fill<<<grid_for(nE), kThreads, 0, s>>>(count, n_edges, 0);
    }
    if (nV > 0) {
        // 2. choices
        k_fill<<<grid_for(nV), kThreads, 0, s>>>(best, n_nodes, INT_MAX);
        if (nE > 0)
            k_best<<<grid_for(nE), kThreads, 0, s>>>(edge_ptr, edge_idx, rank, n_edges, best);
        k_choice<<<grid_for(nV), kThreads, 0, s>>>(best, order, n_nodes, choice, first, count);
        // 3. group numbering by smallest node
        k_group_flags<<<grid_for(nV), kThreads, 0, s>>>(choice, first, n_nodes, gflag);
        tb = L.temp_bytes;
        if (hipcub::DeviceScan::ExclusiveSum(temp, tb, gflag, gid, nV, s) != hipSuccess)
            return fail(HNV_EDEVICE, "scan of group flags");
        k_node_rep<<<grid_for(nV), kThreads, 0, s>>>(choice, first, gid, n_nodes, node_rep);
    }
    if (nE > 0) {
        // 4. removed hyperedges
        k_kept_flags<<<grid_for(nE), kThreads, 0, s>>>(edge_ptr, count, n_edges, kept);
        tb = L.temp_bytes;
        if (hipcub::DeviceScan::ExclusiveSum(temp, tb, kept, krank, nE, s) != hipSuccess)
            return fail(HNV_EDEVICE, "scan of kept flags");
        // 5. coarse member sets
        if (nz > 0) {
            k_map<<<grid_for(nz), kThreads, 0, s>>>(edge_idx, node_rep, nnz, mapped);
            tb = L.temp_bytes;
            // non-negative ids: sorted as unsigned so only the low bits count
            if (hipcub::DeviceSegmentedRadixSort::SortKeys(temp, tb, reinterpret_cast<const uint32_t *>(mapped),
                                                           reinterpret_cast<uint32_t *>(sorted), nz, nE, edge_ptr,
                                                           edge_ptr + 1, 0, member_bits, s) != hipSuccess)
                return fail(HNV_EDEVICE, "segmented sort of coarse members");
        }
        k_distinct<<<grid_for(nE), kThreads, 0, s>>>(edge_ptr, sorted, kept, n_edges, dcount);
        tb = L.temp_bytes;
        if (hipcub::DeviceScan::ExclusiveSum(temp, tb, dcount, cstart, nE, s) != hipSuccess)
            return fail(HNV_EDEVICE, "scan of coarse sizes");
        k_emit<<<grid_for(nE), kThreads, 0, s>>>(edge_ptr, sorted, kept, krank, cstart, edge_w, n_edges, edge_rep,
                                                 c_edge_ptr, c_edge_idx, c_edge_w);
    }
    int64_t *sizes = reinterpret_cast<int64_t *>(base + L.sizes);
    k_sizes<<<1, 64, 0, s>>>(gflag, gid, n_nodes, kept, krank, dcount, cstart, n_edges, c_edge_ptr, sizes);
    if ((st = dev_check("coarsening kernels")) != HNV_OK)
        return st;
    return sync_read(c_sizes, sizes, 3 * sizeof(int64_t));
}

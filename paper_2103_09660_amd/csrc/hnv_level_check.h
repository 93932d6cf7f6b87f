// Device-side checks of a level given as device arrays (int32 offsets), and
// small helpers shared by the GPU coarsening and the device-built plan.
// Included by the .hip sources only; every symbol has internal linkage.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace hnv {
namespace {

constexpr int kThreads = 256;

inline unsigned grid_for(int64_t n) { return (unsigned)((n + kThreads - 1) / kThreads); }

// Bits that hold every value in [0, n).
inline int bits_for(int64_t n)
{
    int b = 1;
    while (b < 32 && (int64_t(1) << b) < n)
        ++b;
    return b;
}

__global__ __launch_bounds__(kThreads) void k_fill(int32_t *__restrict__ p, int64_t n, int32_t v)
{
    const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (i < n)
        p[i] = v;
}

// Flag bits of the checks: 0 offsets, 1 member range, 2 member order,
// 3 weights.  Per hyperedge: offsets (start at 0, end at nnz, never
// decrease, stay in [0, nnz]); with `full` also no empty hyperedge and
// weights finite and > 0.
__global__ __launch_bounds__(kThreads) void k_check_edges(const int32_t *__restrict__ ptr,
                                                          const float *__restrict__ w, int64_t n_edges,
                                                          int64_t nnz, int full, int *__restrict__ flag)
{
    const int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (e >= n_edges)
        return;
    const int64_t a = ptr[e], b = ptr[e + 1];
    int bad = 0;
    if (a < 0 || b < a || b > nnz || (e == 0 && a != 0) || (e == n_edges - 1 && b != nnz) || (full && a == b))
        bad |= 1;
    if (full && w && !(w[e] > 0.0f && w[e] < INFINITY))
        bad |= 8;
    if (bad)
        atomicOr(flag, bad);
}

// inc_edge[j] = the hyperedge of incidence j, written by the hyperedges over
// a zero fill (the caller's): a hyperedge of at most kIncSmall members by its
// own thread, longer ones by the whole wavefront in turn, found with a ballot.
// Offsets are clamped to [0, nnz] (bad ones are reported by k_check_edges), so
// every write stays in the array and every value is a hyperedge id.
constexpr int kIncSmall = 32;

__global__ __launch_bounds__(kThreads) void k_inc_edge(const int32_t *__restrict__ ptr, int64_t n_edges,
                                                       int64_t nnz, int32_t *__restrict__ inc_edge)
{
    const int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    int32_t a = 0, b = 0;
    if (e < n_edges) {
        a = (int32_t)max<int64_t>(ptr[e], 0);
        b = (int32_t)min<int64_t>(ptr[e + 1], nnz);
    }
    const bool big = b - a > kIncSmall;
    if (!big)
        for (int32_t j = a; j < b; ++j)
            inc_edge[j] = (int32_t)e;
    uint64_t m = __ballot(big);   // every lane reaches this
    const int lane = threadIdx.x % 64;
    while (m) {
        const int l = __ffsll((unsigned long long)m) - 1;
        m &= m - 1;
        const int32_t la = __shfl(a, l, 64), lb = __shfl(b, l, 64), le = __shfl((int32_t)e, l, 64);
        for (int32_t j = la + lane; j < lb; j += 64)
            inc_edge[j] = le;
    }
}

// Member range per incidence; with `full` also strictly ascending members
// (inc_edge is only meaningful when the offsets are valid; every read stays
// in bounds either way).
__global__ __launch_bounds__(kThreads) void k_check_members(const int32_t *__restrict__ ptr,
                                                            const int32_t *__restrict__ idx,
                                                            const int32_t *__restrict__ inc_edge, int64_t n_nodes,
                                                            int64_t n_edges, int64_t nnz, int full,
                                                            int *__restrict__ flag)
{
    const int64_t j = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (j >= nnz)
        return;
    const int32_t v = idx[j];
    int bad = 0;
    if (v < 0 || v >= n_nodes) {
        bad = 2;
    } else if (full && j > 0) {
        const int32_t e = inc_edge[j];
        if (e >= 0 && e < n_edges && j > ptr[e] && idx[j - 1] >= v)
            bad = 4;
    }
    if (bad)
        atomicOr(flag, bad);
}

}  // namespace
}  // namespace hnv

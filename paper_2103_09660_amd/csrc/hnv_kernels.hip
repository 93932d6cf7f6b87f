// HIP kernels (gfx950) of the HyperNetVec refinement library and the C ABI
// calls that launch them.
//
// The refinement sweep (Section 3.3, Algorithm 2) is a sparse x dense gather
// over the star expansion H* (Section 1.1): every row of H* relaxes towards
// the weighted mean of its neighbours' rows.  It has no dense contraction, so
// it is bound by memory traffic and latency, and the kernels are built around
// them rather than around matrix cores:
//   - a row slice of Z is read by a group of G lanes, each moving 16 bytes
//     (8 BF16 or 4 FP32 elements), so every gathered row is one coalesced
//     access and a wavefront covers 64/G rows at once;
//   - rows are tiered by neighbour count on the host.  Rows with few
//     neighbours get one lane group each (same-degree rows share a
//     wavefront); longer rows get a whole wavefront per chunk of neighbours,
//     the 64/G groups taking interleaved neighbours and being combined by a
//     cross-lane butterfly; rows longer than one chunk are split over several
//     wavefronts whose FP32 partial sums a finalize pass adds in slot order;
//   - latency is hidden by keeping the dependent-load chain short: a work
//     item carries the row, its first neighbour and its degree (and, for the
//     first sweep of a level, the coarser row it is projected from); a lane
//     preloads its share of the row's neighbour indices, the row's own value
//     is fetched before the neighbours, and four neighbour rows are in
//     flight per lane, masked at the row's end (deeper unrolling costs
//     registers, and measured slower: occupancy matters more here);
//   - the first sweep of a level reads the coarser level's rows through the
//     projection row map (fused projection + sweep);
//   - no atomics: every sum has a fixed order, so results are bitwise
//     reproducible run to run;
//   - the per-sweep residual is reduced in FP64 (per block, then a single
//     fixed-order pass), as are the reciprocals of the row weight sums.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <string>

#include "hnv_grid.h"
#include "hnv_internal.h"

#define HNV_DEV __device__ __forceinline__

namespace hnv {

typedef uint16_t bf16_t;

#ifndef HNV_UNROLL
#define HNV_UNROLL 4
#endif
constexpr int kUnroll = HNV_UNROLL;   // neighbour rows in flight per lane (4 keeps 8 waves per SIMD)

// ---------------------------------------------------------------------------
// storage: one lane's slice of a row, EPL consecutive elements
// ---------------------------------------------------------------------------

HNV_DEV float bf_lo(uint32_t x) { return __uint_as_float(x << 16); }
HNV_DEV float bf_hi(uint32_t x) { return __uint_as_float(x & 0xffff0000u); }

// FP32 -> BF16 bits, round to nearest even; NaN stays NaN.
HNV_DEV uint32_t to_bf16(float f)
{
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u)
        return (u >> 16) | 0x40u;
    u += 0x7fffu + ((u >> 16) & 1u);
    return u >> 16;
}

template <typename T, int EPL>
struct Slice;

template <>
struct Slice<float, 4> {
    struct Raw {
        float4 a;
    };
    static HNV_DEV Raw load(const float *p) { return Raw{*reinterpret_cast<const float4 *>(p)}; }
    static HNV_DEV void unpack(const Raw &r, float (&v)[4])
    {
        v[0] = r.a.x; v[1] = r.a.y; v[2] = r.a.z; v[3] = r.a.w;
    }
    // stores v and leaves in v the values as stored
    static HNV_DEV void store(float *p, float (&v)[4])
    {
        *reinterpret_cast<float4 *>(p) = make_float4(v[0], v[1], v[2], v[3]);
    }
};

template <>
struct Slice<float, 8> {
    struct Raw {
        float4 a, b;
    };
    static HNV_DEV Raw load(const float *p)
    {
        return Raw{reinterpret_cast<const float4 *>(p)[0], reinterpret_cast<const float4 *>(p)[1]};
    }
    static HNV_DEV void unpack(const Raw &r, float (&v)[8])
    {
        v[0] = r.a.x; v[1] = r.a.y; v[2] = r.a.z; v[3] = r.a.w;
        v[4] = r.b.x; v[5] = r.b.y; v[6] = r.b.z; v[7] = r.b.w;
    }
    static HNV_DEV void store(float *p, float (&v)[8])
    {
        reinterpret_cast<float4 *>(p)[0] = make_float4(v[0], v[1], v[2], v[3]);
        reinterpret_cast<float4 *>(p)[1] = make_float4(v[4], v[5], v[6], v[7]);
    }
};

template <>
struct Slice<bf16_t, 8> {
    struct Raw {
        uint4 q;
    };
    static HNV_DEV Raw load(const bf16_t *p) { return Raw{*reinterpret_cast<const uint4 *>(p)}; }
    static HNV_DEV void unpack(const Raw &r, float (&v)[8])
    {
        v[0] = bf_lo(r.q.x); v[1] = bf_hi(r.q.x); v[2] = bf_lo(r.q.y); v[3] = bf_hi(r.q.y);
        v[4] = bf_lo(r.q.z); v[5] = bf_hi(r.q.z); v[6] = bf_lo(r.q.w); v[7] = bf_hi(r.q.w);
    }
    static HNV_DEV void store(bf16_t *p, float (&v)[8])
    {
        uint32_t h[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            h[i] = to_bf16(v[i]);
            v[i] = __uint_as_float(h[i] << 16);
        }
        uint4 q;
        q.x = h[0] | (h[1] << 16);
        q.y = h[2] | (h[3] << 16);
        q.z = h[4] | (h[5] << 16);
        q.w = h[6] | (h[7] << 16);
        *reinterpret_cast<uint4 *>(p) = q;
    }
};

template <int N>
HNV_DEV void zero(float (&a)[N])
{
#pragma unroll
    for (int i = 0; i < N; ++i)
        a[i] = 0.0f;
}

// acc += s * row (SCALE) or acc += row
template <bool SCALE, typename T, int EPL>
HNV_DEV void accumulate(float (&acc)[EPL], float s, const typename Slice<T, EPL>::Raw &raw)
{
    float v[EPL];
    Slice<T, EPL>::unpack(raw, v);
#pragma unroll
    for (int i = 0; i < EPL; ++i)
        acc[i] = SCALE ? fmaf(s, v[i], acc[i]) : acc[i] + v[i];
}

// ---------------------------------------------------------------------------
// kernel arguments
// ---------------------------------------------------------------------------

enum Mode : int {
    kFwd = 0,       // forward sweep
    kAdjNode = 1,   // reverse sweep, node rows
    kAdjEdge = 2,   // reverse sweep, hyperedge rows, summing the per-node scalars of their members
    kAdjEdgeNoSum = 3,   // reverse sweep, hyperedge rows, without that sum
};

struct GatherArgs {
    DevSide side[2];
    int32_t nb_chunk[2];      // blocks of the wavefront tier per side (per panel)
    int32_t nb_small[2];      // blocks of the lane-group tier per side (per panel)
    int32_t nb_split[2];      // finalize blocks per side (per panel)
    int32_t blocks_per_panel;
    int32_t dp;               // columns per panel
    int64_t ld;               // row stride (elements) = d
    float omega;
    const float *r;           // [rows] reciprocal row weight sum
    const float *w;           // [n_edges] hyperedge weights
    const int32_t *rowmap;    // fused projection: row map to the coarser level
    const void *src;          // gathered matrix (Z^{i-1}, the coarser Z if fused, or G)
    void *dst;                // output matrix
    const void *yprev;        // reverse: sweep input y
    const void *zcur;         // reverse: sweep output z
    float *cvec;              // reverse: per-node scalar (written on node rows, read on hyperedge rows)
    void *dst2;               // reverse, edge-first order: hyperedge rows' dL/de' (read by the node launch)
    int32_t wgrad;            // reverse: weight gradient 0 none, 1 in one sweep (cvec = c), 2 split (cvec += omega c)
    float *dw;                // reverse: dL/dw accumulator or null
    float *partials;          // split-row partial sums
    int32_t pstride;
    double *resid;            // per-block residual partials or null
    int32_t resid_offset;     // first partial index of this launch
    const void *self_src;     // forward: matrix a row's own value is read from
    int32_t self_mapped;      // forward: own value read through the projection row map
    SweepCtl *ctl;            // early-stop refinement: the matrices and the stop flag come from here
    int32_t ctl_level;        // level of the sweep (its stop flag)
    int32_t ctl_src_next;     // gathered rows from ctl->next (the node half of an edge-first sweep)
    int64_t n_blocks;         // blocks of this launch (the grid may hold padding blocks past them)
};

// The matrices one launch reads and writes.  Fixed ones come from the
// arguments; in an early-stop refinement they are known on the device only:
// the own rows and (Jacobi) the gathered rows are the latest iterate, the
// output is the other buffer.  (Kept apart from GatherArgs, which the
// kernels index by side at run time and so must not copy.)
struct Mats {
    const void *src, *self;
    void *dst;
};

template <bool CTL>
HNV_DEV Mats mats_of(const GatherArgs &a)
{
    if constexpr (CTL) {
        const SweepCtl *c = a.ctl;
        return Mats{a.ctl_src_next ? c->next : c->cur, c->cur, c->next};
    } else {
        return Mats{a.src, a.self_src, a.dst};
    }
}

// ---------------------------------------------------------------------------
// gathers
// ---------------------------------------------------------------------------

// One lane group (G lanes) gathers one row of degree deg <= kIdxRegs * G:
// acc = sum_j s_j * src[nb_j] in neighbour order; csum (per lane, partial) =
// sum of c[nb_j] over the lane's own neighbours.  Lane gl preloads the
// indices of positions gl, gl + G, gl + 2G, gl + 3G; the neighbour rows are
// fetched kUnroll at a time, masked at the row's end.
template <typename T, int EPL, int G, bool SCALE, bool SCALAR>
HNV_DEV void gather_group(const int32_t *__restrict__ nb, const float *__restrict__ sc,
                          const float *__restrict__ cvec, int start, int deg, const T *__restrict__ src, int64_t ld,
                          int col, bool col_ok, int gl, int gbase, int my_id, float (&acc)[EPL], float &csum)
{
    using S = Slice<T, EPL>;
    // With at least kInlineIds lanes per group, lane gl < kInlineIds holds
    // neighbour gl's id from the work item (my_id), so the first neighbours
    // are gathered without waiting for the index list.
    constexpr bool kInl = G >= kInlineIds;
    int ix[kIdxRegs];
    float sv[kIdxRegs];
#pragma unroll
    for (int r = 0; r < kIdxRegs; ++r) {
        const int p = gl + r * G;
        ix[r] = 0;
        sv[r] = 1.0f;
        if (p < deg) {
            ix[r] = (kInl && p < kInlineIds) ? my_id : nb[start + p];
            if (SCALE)
                sv[r] = sc[start + p];
        }
    }
    if (SCALAR) {
#pragma unroll
        for (int r = 0; r < kIdxRegs; ++r)
            if (gl + r * G < deg)
                csum += cvec[ix[r]];
    }
    int j0 = 0;
    if (kInl) {   // neighbours 0 .. kInlineIds-1 (the first position of lanes 0 .. kInlineIds-1)
        typename S::Raw raw[kInlineIds];
        float s[kInlineIds];
#pragma unroll
        for (int k = 0; k < kInlineIds; ++k) {
            const int v = __shfl(my_id, gbase + k, kWave);
            s[k] = SCALE ? __shfl(sv[0], gbase + k, kWave) : 1.0f;
            if (k < deg && col_ok)
                raw[k] = S::load(src + (int64_t)v * ld + col);
        }
        if (col_ok) {
#pragma unroll
            for (int k = 0; k < kInlineIds; ++k)
                if (k < deg)
                    accumulate<SCALE, T, EPL>(acc, s[k], raw[k]);
        }
        j0 = kInlineIds;
    }
    for (int j = j0; j < deg; j += kUnroll) {
        typename S::Raw raw[kUnroll];
        float s[kUnroll];
        bool ok[kUnroll];
#pragma unroll
        for (int k = 0; k < kUnroll; ++k) {
            const int q = j + k;
            const int r = q / G;
            const int xr = (r == 0) ? ix[0] : (r == 1) ? ix[1] : (r == 2) ? ix[2] : ix[3];
            const float sr = (r == 0) ? sv[0] : (r == 1) ? sv[1] : (r == 2) ? sv[2] : sv[3];
            const int lane_src = gbase + (q & (G - 1));
            ok[k] = q < deg;
            const int v = __shfl(xr, lane_src, kWave);
            s[k] = SCALE ? __shfl(sr, lane_src, kWave) : 1.0f;
            if (ok[k] && col_ok)
                raw[k] = S::load(src + (int64_t)v * ld + col);
        }
        if (col_ok) {
#pragma unroll
            for (int k = 0; k < kUnroll; ++k)
                if (ok[k])
                    accumulate<SCALE, T, EPL>(acc, s[k], raw[k]);
        }
    }
}

// A whole wavefront gathers `len` neighbours: group g takes neighbours
// g, g + Q, g + 2Q, ... (Q = 64 / G), then the Q group sums are added with an
// xor butterfly (every lane ends with the same, order-fixed total).  The
// indices of the next 64 neighbours are fetched while the current ones are
// gathered.
template <typename T, int EPL, int G, bool SCALE, bool SCALAR>
HNV_DEV void gather_wave(const int32_t *__restrict__ nb, const float *__restrict__ sc,
                         const float *__restrict__ cvec, int start, int len, const T *__restrict__ src, int64_t ld,
                         int col, bool col_ok, int lane, int g, float (&acc)[EPL], float &csum)
{
    using S = Slice<T, EPL>;
    constexpr int Q = kWave / G;
    int my_nb = 0;
    float my_s = 1.0f;
    if (lane < len) {
        my_nb = nb[start + lane];
        if (SCALE)
            my_s = sc[start + lane];
    }
    for (int b = 0; b < len; b += kWave) {
        const int pn = b + kWave + lane;
        int nx_nb = 0;
        float nx_s = 1.0f;
        if (pn < len) {
            nx_nb = nb[start + pn];
            if (SCALE)
                nx_s = sc[start + pn];
        }
        if (SCALAR && b + lane < len)
            csum += cvec[my_nb];
        const int n = min(kWave, len - b);
        for (int t = 0; t < n; t += kUnroll * Q) {
            typename S::Raw raw[kUnroll];
            float s[kUnroll];
            bool ok[kUnroll];
#pragma unroll
            for (int k = 0; k < kUnroll; ++k) {
                const int q = t + k * Q + g;
                ok[k] = q < n;
                const int v = __shfl(my_nb, q & (kWave - 1), kWave);
                s[k] = SCALE ? __shfl(my_s, q & (kWave - 1), kWave) : 1.0f;
                if (ok[k] && col_ok)
                    raw[k] = S::load(src + (int64_t)v * ld + col);
            }
            if (col_ok) {
#pragma unroll
                for (int k = 0; k < kUnroll; ++k)
                    if (ok[k])
                        accumulate<SCALE, T, EPL>(acc, s[k], raw[k]);
            }
        }
        my_nb = nx_nb;
        my_s = nx_s;
    }
#pragma unroll
    for (int off = G; off < kWave; off <<= 1)
#pragma unroll
        for (int i = 0; i < EPL; ++i)
            acc[i] += __shfl_xor(acc[i], off, kWave);
    if (SCALAR) {
#pragma unroll
        for (int off = 1; off < kWave; off <<= 1)
            csum += __shfl_xor(csum, off, kWave);
    }
}

// sum over the G lanes of a group (xor butterfly inside the group)
template <int G>
HNV_DEV float group_sum(float x)
{
#pragma unroll
    for (int off = 1; off < G; off <<= 1)
        x += __shfl_xor(x, off, kWave);
    return x;
}

// ---------------------------------------------------------------------------
// row epilogues
// ---------------------------------------------------------------------------

// A row's own slices, fetched before its neighbours so that their latency
// overlaps the gather: forward, the row's previous value (or the coarser
// row it is projected from); reverse, its cotangent g and, for rows with
// neighbours, the sweep's input y (and, on node rows, its output z).  On
// the hyperedge rows of an edge-first reverse sweep, y is the sweep's
// output row e' (the caller passes z as yprev).
template <typename T, int EPL>
struct Own {
    typename Slice<T, EPL>::Raw x, y, z;
    float rs;     // the row's scalar factor: r_u (forward, node rows) or w_e (hyperedge rows)
    float prev;   // the accumulator the row adds to: dL/dw_e (hyperedge rows) or c_v (split node rows)
};

template <typename T, int EPL, int MODE>
HNV_DEV void load_own(Own<T, EPL> &o, const GatherArgs &a, const Mats &m, int row, int64_t zrow, int64_t srow,
                      int deg, int col)
{
    using S = Slice<T, EPL>;
    o.x = S::load(static_cast<const T *>(m.self) + srow * a.ld + col);
    // The epilogue's scalars are fetched here too: issued after the gather
    // they would add a dependent memory round trip to every row.  (Each row
    // is finished by one lane group, so no other wave of the launch writes
    // the accumulator in between.)
    if (MODE == kFwd) {
        if (deg > 0)
            o.rs = a.r[zrow];
    } else if (MODE == kAdjNode) {
        if (deg > 0 && a.wgrad != 0)
            o.rs = a.r[zrow];
        if (a.wgrad == 2)
            o.prev = a.cvec[row];
    } else {
        if (deg > 0) {
            o.rs = a.w[row];
            if (a.dw)
                o.prev = a.dw[row];
        }
    }
    // the sweep's input and output rows serve the weight gradient only
    if (MODE != kFwd && deg > 0 && a.wgrad != 0) {
        o.y = S::load(static_cast<const T *>(a.yprev) + zrow * a.ld + col);
        if (MODE == kAdjNode)
            o.z = S::load(static_cast<const T *>(a.zcur) + zrow * a.ld + col);
    }
}

// Forward: z'_u = (1 - omega) z_u + omega r_u acc (rows with neighbours),
// z'_u = z_u otherwise.  Returns the row's contribution to ||z' - z||^2.
template <typename T, int EPL>
HNV_DEV double epilogue_fwd(const GatherArgs &a, void *dst, int zrow, int deg, int col, bool col_ok,
                            float (&acc)[EPL],
                            const Own<T, EPL> &own)
{
    if (!col_ok)
        return 0.0;
    float z[EPL], o[EPL];
    Slice<T, EPL>::unpack(own.x, z);
    if (deg > 0) {
        const float keep = 1.0f - a.omega;
        const float mix = a.omega * own.rs;
#pragma unroll
        for (int i = 0; i < EPL; ++i)
            o[i] = fmaf(mix, acc[i], keep * z[i]);
    } else {
#pragma unroll
        for (int i = 0; i < EPL; ++i)
            o[i] = z[i];
    }
    Slice<T, EPL>::store(static_cast<T *>(dst) + (int64_t)zrow * a.ld + col, o);
    double r2 = 0.0;
    if (a.resid) {
#pragma unroll
        for (int i = 0; i < EPL; ++i) {
            const double dd = (double)o[i] - (double)z[i];
            r2 += dd * dd;
        }
    }
    return r2;
}

// Reverse, node row v (side 1): g'_v = (1-omega) g_v + omega acc where acc =
// sum_e g_e / |e|; c_v = <g_v, zt_v> / S_v with zt_v = (z_v - (1-omega) y_v) / omega
// (stored, added times omega, or not formed: a.wgrad = 1, 2, 0).
template <typename T, int EPL, int G>
HNV_DEV void epilogue_adj_node(const GatherArgs &a, int row, int deg, int col, bool col_ok, float (&acc)[EPL],
                               const Own<T, EPL> &own, bool writer)
{
    using S = Slice<T, EPL>;
    const int64_t zrow = row;  // node rows start at Z row 0
    float dot = 0.0f;
    if (col_ok) {
        float g[EPL], o[EPL];
        S::unpack(own.x, g);
        if (deg > 0) {
            float y[EPL], z[EPL];
            S::unpack(own.y, y);
            S::unpack(own.z, z);
            const float keep = 1.0f - a.omega;
            const float inv_om = 1.0f / a.omega;
#pragma unroll
            for (int i = 0; i < EPL; ++i) {
                o[i] = fmaf(a.omega, acc[i], keep * g[i]);
                const float zt = (z[i] - keep * y[i]) * inv_om;
                dot = fmaf(g[i], zt, dot);
            }
        } else {
#pragma unroll
            for (int i = 0; i < EPL; ++i)
                o[i] = g[i];
        }
        if (writer)
            S::store(static_cast<T *>(a.dst) + zrow * a.ld + col, o);
    }
    dot = group_sum<G>(dot);
    if (writer && (threadIdx.x % G) == 0 && a.wgrad != 0) {
        const float c = (deg > 0) ? own.rs * dot : 0.0f;
        if (a.wgrad == 1)
            a.cvec[row] = c;
        else
            a.cvec[row] = own.prev + a.omega * c;
    }
}

// Reverse, hyperedge row e (side 0): g'_e = (1-omega) g_e + omega w_e acc with
// acc = sum_v g_v / S_v; dL/dw_e += omega (<acc, y_e> - sum_v c_v).
// Edge-first order (a.dst2 != null): the node half runs last forward, so
// its reverse comes first: ge_e = g_e + omega w_e acc is dL/de'_e, stored to
// dst2 for the node launch, and g'_e = (1-omega) ge_e; y_e is then e'_e.
template <typename T, int EPL, int G>
HNV_DEV void epilogue_adj_edge(const GatherArgs &a, int row, int deg, int col, bool col_ok, float (&acc)[EPL],
                               float csum, const Own<T, EPL> &own, bool writer)
{
    using S = Slice<T, EPL>;
    const int64_t zrow = (int64_t)a.side[0].row_base + row;
    float dot = 0.0f;
    if (col_ok) {
        float g[EPL], o[EPL];
        S::unpack(own.x, g);
        if (deg > 0) {
            float y[EPL];
            S::unpack(own.y, y);
            const float keep = 1.0f - a.omega;
            const float mix = a.omega * own.rs;
            if (a.dst2) {
                float ge[EPL];
#pragma unroll
                for (int i = 0; i < EPL; ++i) {
                    ge[i] = fmaf(mix, acc[i], g[i]);
                    o[i] = keep * ge[i];
                    dot = fmaf(acc[i], y[i], dot);
                }
                if (writer)
                    S::store(static_cast<T *>(a.dst2) + zrow * a.ld + col, ge);
            } else {
#pragma unroll
                for (int i = 0; i < EPL; ++i) {
                    o[i] = fmaf(mix, acc[i], keep * g[i]);
                    dot = fmaf(acc[i], y[i], dot);
                }
            }
        } else {
#pragma unroll
            for (int i = 0; i < EPL; ++i)
                o[i] = g[i];
            if (writer && a.dst2)
                S::store(static_cast<T *>(a.dst2) + zrow * a.ld + col, o);
        }
        if (writer)
            S::store(static_cast<T *>(a.dst) + zrow * a.ld + col, o);
    }
    dot = group_sum<G>(dot);
    if (writer && a.dw && deg > 0 && (threadIdx.x % G) == 0)
        a.dw[row] = own.prev + a.omega * (dot - csum);
}

// ---------------------------------------------------------------------------
// block-level residual reduction (FP64, fixed order)
// ---------------------------------------------------------------------------

HNV_DEV void block_resid(const GatherArgs &a, double r2, int64_t lb)
{
    if (!a.resid)
        return;
    __shared__ double wsum[kWavesPerBlock];
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1)
        r2 += __shfl_xor(r2, off, kWave);
    const int wave = threadIdx.x / kWave;
    if ((threadIdx.x % kWave) == 0)
        wsum[wave] = r2;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int i = 0; i < kWavesPerBlock; ++i)
            s += wsum[i];
        a.resid[a.resid_offset + lb] = s;
    }
}

// ---------------------------------------------------------------------------
// main kernel: wavefront tier + lane-group tier of both sides, all panels
// ---------------------------------------------------------------------------

template <typename T, int EPL, int G, int MODE, bool FUSED, bool CTL>
__global__ __launch_bounds__(kBlock) void k_gather(GatherArgs a)
{
    const int64_t lb = linear_block();
    if (lb >= a.n_blocks)
        return;
    if constexpr (CTL) {
        if (a.ctl->stop[a.ctl_level])   // the level has converged: this sweep does nothing
            return;
    }
    const Mats mats = mats_of<CTL>(a);
    int b = (int)lb;
    const int panel = b / a.blocks_per_panel;
    b -= panel * a.blocks_per_panel;
    const int lane = threadIdx.x % kWave;
    const int wave = threadIdx.x / kWave;
    const int g = lane / G;
    const int gl = lane % G;
    const int col = panel * a.dp + gl * EPL;
    const bool col_ok = gl * EPL < a.dp;
    const T *src = static_cast<const T *>(mats.src);
    float acc[EPL];
    zero(acc);
    float csum = 0.0f;
    double r2 = 0.0;

    // which tier / side does this block serve?  (uniform over the block)
    int side, tier = 0;  // tier 0: wavefront, 1: lane group
    if (b < a.nb_chunk[0]) {
        side = 0;
    } else if ((b -= a.nb_chunk[0]) < a.nb_chunk[1]) {
        side = 1;
    } else if ((b -= a.nb_chunk[1]) < a.nb_small[0]) {
        side = 0;
        tier = 1;
    } else {
        b -= a.nb_small[0];
        side = 1;
        tier = 1;
    }
    const DevSide &Sd = a.side[side];
    constexpr bool kScalar = (MODE == kAdjEdge);
    const bool use_scale = (MODE != kFwd) || (side == 1 && Sd.wn != nullptr);
    const float *sc = (MODE == kFwd) ? Sd.wn : Sd.sn;
    const int32_t *nb = FUSED ? Sd.cidx : Sd.idx;

    // In reverse mode only one side is active per launch.
    if ((MODE == kAdjNode && side != 1) || ((MODE == kAdjEdge || MODE == kAdjEdgeNoSum) && side != 0))
        return;

    if (tier == 0) {
        const int item = b * kWavesPerBlock + wave;
        if (item < Sd.n_chunks) {   // uniform over the wavefront
            const Item c = Sd.chunks[item];
            const int zrow = Sd.row_base + c.row;
            const bool whole = c.aux < 0;
            Own<T, EPL> self{};
            if (whole && col_ok) {
                const int64_t srow =
                    (MODE == kFwd && (FUSED || a.self_mapped)) ? (int64_t)a.rowmap[zrow] : (int64_t)zrow;
                load_own<T, EPL, MODE>(self, a, mats, c.row, zrow, srow, c.len, col);
            }
            if (use_scale)
                gather_wave<T, EPL, G, true, kScalar>(nb, sc, a.cvec, c.start, c.len, src, a.ld, col, col_ok, lane, g,
                                                      acc, csum);
            else
                gather_wave<T, EPL, G, false, kScalar>(nb, sc, a.cvec, c.start, c.len, src, a.ld, col, col_ok, lane,
                                                       g, acc, csum);
            if (!whole) {
                if (g == 0 && col_ok) {
                    float *pp = a.partials + (int64_t)c.aux * a.pstride + col;
#pragma unroll
                    for (int i = 0; i < EPL; i += 4)
                        *reinterpret_cast<float4 *>(pp + i) = make_float4(acc[i], acc[i + 1], acc[i + 2], acc[i + 3]);
                    if (kScalar && gl == 0)
                        a.partials[(int64_t)c.aux * a.pstride + a.ld] = csum;
                }
            } else if (MODE == kFwd) {
                if (g == 0)
                    r2 = epilogue_fwd<T, EPL>(a, mats.dst, zrow, c.len, col, col_ok, acc, self);
            } else if (MODE == kAdjNode) {
                epilogue_adj_node<T, EPL, G>(a, c.row, c.len, col, col_ok, acc, self, g == 0);
            } else {
                epilogue_adj_edge<T, EPL, G>(a, c.row, c.len, col, col_ok, acc, csum, self, g == 0);
            }
        }
    } else {
        for (int rr = 0; rr < kRowsPerGroup; ++rr) {
            const int item = (b * kRowsPerGroup + rr) * (kBlock / G) + (int)(threadIdx.x / G);
            const bool valid = item < Sd.n_small;
            Item it{0, 0, 0, 0};
            int my_id = 0;   // lane gl < kInlineIds: the row's neighbour gl, loaded with the item
            if (valid) {
                it = Sd.small[item];
                if (gl < kInlineIds && G >= kInlineIds)
                    my_id = (FUSED ? Sd.small_cids : Sd.small_ids)[item].id[gl];
            }
            const int zrow = Sd.row_base + it.row;
            Own<T, EPL> self{};
            if (valid && col_ok) {
                const int64_t srow = (MODE == kFwd && (FUSED || a.self_mapped)) ? (int64_t)it.aux : (int64_t)zrow;
                load_own<T, EPL, MODE>(self, a, mats, it.row, zrow, srow, it.len, col);
            }
            if (rr > 0) {
                zero(acc);
                csum = 0.0f;
            }
            if (use_scale)
                gather_group<T, EPL, G, true, kScalar>(nb, sc, a.cvec, it.start, it.len, src, a.ld, col, col_ok, gl,
                                                       g * G, my_id, acc, csum);
            else
                gather_group<T, EPL, G, false, kScalar>(nb, sc, a.cvec, it.start, it.len, src, a.ld, col, col_ok, gl,
                                                        g * G, my_id, acc, csum);
            if (MODE == kFwd) {
                if (valid)
                    r2 += epilogue_fwd<T, EPL>(a, mats.dst, zrow, it.len, col, col_ok, acc, self);
            } else if (MODE == kAdjNode) {
                epilogue_adj_node<T, EPL, G>(a, it.row, it.len, col, col_ok, acc, self, valid);
            } else {
                csum = group_sum<G>(csum);
                epilogue_adj_edge<T, EPL, G>(a, it.row, it.len, col, col_ok, acc, csum, self, valid);
            }
        }
    }
    if (MODE == kFwd)
        block_resid(a, r2, lb);
}

// Finalize rows that were split over several wavefronts: one wavefront per
// row adds the row's partial slots in slot order (group g takes slots
// g, g+Q, ...; groups combined by the xor butterfly), then applies the
// row's epilogue.
template <typename T, int EPL, int G, int MODE, bool FUSED, bool CTL>
__global__ __launch_bounds__(kBlock) void k_finalize(GatherArgs a)
{
    const int64_t lb = linear_block();
    if (lb >= a.n_blocks)
        return;
    if constexpr (CTL) {
        if (a.ctl->stop[a.ctl_level])
            return;
    }
    const Mats mats = mats_of<CTL>(a);
    constexpr int Q = kWave / G;
    int b = (int)lb;
    const int per_panel = a.nb_split[0] + a.nb_split[1];
    const int panel = b / per_panel;
    b -= panel * per_panel;
    const int lane = threadIdx.x % kWave;
    const int wave = threadIdx.x / kWave;
    const int g = lane / G;
    const int gl = lane % G;
    const int col = panel * a.dp + gl * EPL;
    const bool col_ok = gl * EPL < a.dp;
    int side = 0;
    if (b >= a.nb_split[0]) {
        b -= a.nb_split[0];
        side = 1;
    }
    const DevSide &Sd = a.side[side];
    const int item = b * kWavesPerBlock + wave;
    float acc[EPL];
    zero(acc);
    float csum = 0.0f;
    double r2 = 0.0;
    const bool active = item < Sd.n_splits && !((MODE == kAdjNode && side != 1) ||
                                                ((MODE == kAdjEdge || MODE == kAdjEdgeNoSum) && side != 0));
    if (active) {   // uniform over the wavefront
        const Split sp = Sd.splits[item];
        const int zrow = Sd.row_base + sp.row;
        Own<T, EPL> self{};
        if (col_ok) {
            const int64_t srow =
                (MODE == kFwd && (FUSED || a.self_mapped)) ? (int64_t)a.rowmap[zrow] : (int64_t)zrow;
            load_own<T, EPL, MODE>(self, a, mats, sp.row, zrow, srow, sp.deg, col);
        }
        for (int k = g; k < sp.n_slots; k += Q) {
            const float *pp = a.partials + (int64_t)(sp.first_slot + k) * a.pstride;
            if (col_ok) {
#pragma unroll
                for (int i = 0; i < EPL; i += 4) {
                    const float4 x = *reinterpret_cast<const float4 *>(pp + col + i);
                    acc[i] += x.x;
                    acc[i + 1] += x.y;
                    acc[i + 2] += x.z;
                    acc[i + 3] += x.w;
                }
            }
            if (MODE == kAdjEdge && gl == 0)
                csum += pp[a.ld];
        }
#pragma unroll
        for (int off = G; off < kWave; off <<= 1) {
#pragma unroll
            for (int i = 0; i < EPL; ++i)
                acc[i] += __shfl_xor(acc[i], off, kWave);
            if (MODE == kAdjEdge)
                csum += __shfl_xor(csum, off, kWave);
        }
        if (MODE == kFwd) {
            if (g == 0)
                r2 = epilogue_fwd<T, EPL>(a, mats.dst, zrow, sp.deg, col, col_ok, acc, self);
        } else if (MODE == kAdjNode) {
            epilogue_adj_node<T, EPL, G>(a, sp.row, sp.deg, col, col_ok, acc, self, g == 0);
        } else {
            epilogue_adj_edge<T, EPL, G>(a, sp.row, sp.deg, col, col_ok, acc, csum, self, g == 0);
        }
    }
    if (MODE == kFwd)
        block_resid(a, r2, lb);
}

// Residual reduction, one stage: block b sums partials [b*2048, (b+1)*2048)
// (each thread eight strided loads, all in flight at once, added in a fixed
// order, then a tree over the block) and writes one value; the last stage
// (a single block) writes the square root.  In an early-stop refinement
// (ctl != null) nothing runs once the level has stopped, and the last stage
// instead stores the residual at the next packed position, counts the
// sweep, raises the level's stop flag if the residual is <= tol, and makes
// the sweep's output the latest iterate.  Several sweeps' reductions run
// side by side along blockIdx.y, sweep y reading part + y * part_stride and
// writing out + y * out_stride (each in the order one sweep alone takes).
constexpr int kResidPer = kBlock * 8;
__global__ __launch_bounds__(kBlock) void k_resid_stage(const double *__restrict__ part, int64_t n,
                                                        int64_t part_stride, double *__restrict__ out,
                                                        int64_t out_stride, int final_sqrt, SweepCtl *ctl, int level)
{
    if (ctl && ctl->stop[level])
        return;
    part += (int64_t)blockIdx.y * part_stride;
    out += (int64_t)blockIdx.y * out_stride;
    __shared__ double s[kBlock];
    const int64_t base = (int64_t)blockIdx.x * kResidPer + threadIdx.x;
    double x[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const int64_t i = base + (int64_t)k * kBlock;
        x[k] = (i < n) ? part[i] : 0.0;
    }
    s[threadIdx.x] = ((x[0] + x[1]) + (x[2] + x[3])) + ((x[4] + x[5]) + (x[6] + x[7]));
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            s[threadIdx.x] += s[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        if (!final_sqrt) {
            out[blockIdx.x] = s[0];
        } else if (!ctl) {
            out[0] = sqrt(s[0]);
        } else {
            const double r = sqrt(s[0]);
            (ctl->res ? ctl->res + ctl->n_res : ctl->res_tmp)[0] = r;
            ctl->n_res += 1;
            ctl->done[level] += 1;
            if (r <= ctl->tol)
                ctl->stop[level] = 1;
            void *w = ctl->next;
            ctl->cur = w;
            ctl->next = (w == ctl->buf[0]) ? ctl->buf[1] : ctl->buf[0];
        }
    }
}

// Sets up an early-stop refinement (one block): the first operation reads
// z_in and writes first_out; stop flags and sweep counts start at zero.
__global__ __launch_bounds__(kBlock) void k_ctl_init(SweepCtl *ctl, int32_t *flags, int n_levels, const void *z_in,
                                                     void *first_out, void *buf0, void *buf1, double *res,
                                                     double *res_tmp, double tol)
{
    for (int i = threadIdx.x; i < 2 * n_levels; i += kBlock)
        flags[i] = 0;
    if (threadIdx.x == 0) {
        ctl->cur = z_in;
        ctl->next = first_out;
        ctl->buf[0] = buf0;
        ctl->buf[1] = buf1;
        ctl->res = res;
        ctl->res_tmp = res_tmp;
        ctl->stop = flags;
        ctl->done = flags + n_levels;
        ctl->tol = tol;
        ctl->n_res = 0;
    }
}

// After a projection (which always runs): its output is the latest iterate.
__global__ void k_ctl_advance(SweepCtl *ctl)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        void *w = ctl->next;
        ctl->cur = w;
        ctl->next = (w == ctl->buf[0]) ? ctl->buf[1] : ctl->buf[0];
    }
}

// Second half of a split weight gradient: dw[e] -= scale * (sum of node_acc
// over the members of e).  16 lanes per hyperedge, each summing a strided
// share in member order, combined by a fixed butterfly (reproducible).
__global__ __launch_bounds__(kBlock) void k_wgrad_finish(const int32_t *__restrict__ ptr,
                                                         const int32_t *__restrict__ idx,
                                                         const float *__restrict__ node_acc, float *__restrict__ dw,
                                                         int64_t n_edges, float scale)
{
    constexpr int GW = 16;
    const int64_t e = (linear_block() * kBlock + threadIdx.x) / GW;
    const int gl = threadIdx.x % GW;
    int32_t a0 = 0, a1 = 0;
    if (e < n_edges) {   // whole lane groups share e
        a0 = ptr[e];
        a1 = ptr[e + 1];
    }
    float sum = 0.0f;
    for (int32_t j = a0 + gl; j < a1; j += GW)
        sum += node_acc[idx[j]];
#pragma unroll
    for (int off = 1; off < GW; off <<= 1)
        sum += __shfl_xor(sum, off, kWave);
    if (e < n_edges && gl == 0)
        dw[e] -= scale * sum;
}

// Copies the latest iterate to out (n16 16-byte words) unless it is there.
__global__ __launch_bounds__(kBlock) void k_ctl_result(const SweepCtl *ctl, void *out, int64_t n16)
{
    const uint4 *src = static_cast<const uint4 *>(ctl->cur);
    if (src == out)
        return;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n16; i += (int64_t)gridDim.x * kBlock)
        static_cast<uint4 *>(out)[i] = src[i];
}

// ---------------------------------------------------------------------------
// projection and its reverse
// ---------------------------------------------------------------------------

// z_fine[u] = z_coarse[rowmap[u]], one lane slice per thread
template <typename T, int EPL>
__global__ __launch_bounds__(kBlock) void k_project(const T *__restrict__ zc, T *__restrict__ zf, const int32_t *__restrict__ rowmap,
                                                    int64_t rows, int d, const SweepCtl *ctl)
{
    using S = Slice<T, EPL>;
    if (ctl) {   // early-stop refinement: the matrices come from the control block
        zc = static_cast<const T *>(ctl->cur);
        zf = static_cast<T *>(ctl->next);
    }
    const int per_row = d / EPL;
    const int64_t t = linear_block() * kBlock + threadIdx.x;
    if (t >= rows * per_row)
        return;
    const int64_t u = t / per_row;
    const int c = (int)(t - u * per_row) * EPL;
    float v[EPL];
    S::unpack(S::load(zc + (int64_t)rowmap[u] * d + c), v);
    S::store(zf + u * d + c, v);
}

// g_coarse[r] = sum of g_fine[u] over rowmap(u) = r, ascending u.  One
// wavefront per coarse row (gather_wave over the inverse map).
template <typename T, int EPL, int G>
__global__ __launch_bounds__(kBlock) void k_project_adj(const T *__restrict__ gf, T *__restrict__ gc,
                                                        const int32_t *__restrict__ inv_ptr,
                                                        const int32_t *__restrict__ inv_idx, int64_t rows_c, int d)
{
    const int64_t r = linear_block() * kWavesPerBlock + threadIdx.x / kWave;
    const int lane = threadIdx.x % kWave;
    const int g = lane / G, gl = lane % G;
    const int col = gl * EPL;
    const bool col_ok = col < d;
    if (r >= rows_c)
        return;  // uniform per wavefront
    float acc[EPL];
    zero(acc);
    float cs = 0.0f;
    const int start = inv_ptr[r], len = inv_ptr[r + 1] - start;
    gather_wave<T, EPL, G, false, false>(inv_idx, nullptr, nullptr, start, len, gf, d, col, col_ok, lane, g, acc, cs);
    if (g == 0 && col_ok)
        Slice<T, EPL>::store(gc + r * d + col, acc);
}

// ---------------------------------------------------------------------------
// hyperedge-prediction features
// ---------------------------------------------------------------------------

// Running statistic of one lane's column slice: count, and per column the
// mean and sum of squared deviations (Welford), or the min / max.
template <int EPL>
struct Stat {
    float n;
    float m[EPL], q[EPL];
};

template <int EPL>
HNV_DEV void stat_init(Stat<EPL> &s, int op)
{
    s.n = 0.0f;
#pragma unroll
    for (int i = 0; i < EPL; ++i) {
        s.m[i] = (op == HNV_SCORE_MIN) ? INFINITY : (op == HNV_SCORE_MAX) ? -INFINITY : 0.0f;
        s.q[i] = 0.0f;
    }
}

template <int EPL>
HNV_DEV void stat_add(Stat<EPL> &s, const float (&x)[EPL], int op)
{
    s.n += 1.0f;
    const float inv = 1.0f / s.n;
#pragma unroll
    for (int i = 0; i < EPL; ++i) {
        if (op == HNV_SCORE_MIN) {
            s.m[i] = fminf(s.m[i], x[i]);
        } else if (op == HNV_SCORE_MAX) {
            s.m[i] = fmaxf(s.m[i], x[i]);
        } else {
            const float delta = x[i] - s.m[i];
            s.m[i] = fmaf(delta, inv, s.m[i]);
            if (op == HNV_SCORE_VARIANCE)
                s.q[i] = fmaf(delta, x[i] - s.m[i], s.q[i]);
        }
    }
}

// a <- combination of a (earlier members) and b (later members): Chan et
// al.'s pairwise update for mean / squared deviations, or min / max.
template <int EPL>
HNV_DEV void stat_merge(Stat<EPL> &a, float bn, const float (&bm)[EPL], const float (&bq)[EPL], int op)
{
    const float n = a.n + bn;
    if (bn == 0.0f)
        return;
    const float fb = bn / n, cross = a.n * bn / n;
#pragma unroll
    for (int i = 0; i < EPL; ++i) {
        if (op == HNV_SCORE_MIN) {
            a.m[i] = fminf(a.m[i], bm[i]);
        } else if (op == HNV_SCORE_MAX) {
            a.m[i] = fmaxf(a.m[i], bm[i]);
        } else if (a.n == 0.0f) {
            a.m[i] = bm[i];
            a.q[i] = bq[i];
        } else {
            const float delta = bm[i] - a.m[i];
            a.m[i] = fmaf(delta, fb, a.m[i]);
            if (op == HNV_SCORE_VARIANCE)
                a.q[i] = a.q[i] + bq[i] + delta * delta * cross;
        }
    }
    a.n = n;
}

// Combine the Q lane groups of a wavefront, lower group first at every
// level of the tree, so that both partners of a step compute the same value
// and the order is fixed.
template <int EPL, int G>
HNV_DEV void stat_wave_combine(Stat<EPL> &s, int g, int op)
{
#pragma unroll
    for (int off = G; off < kWave; off <<= 1) {
        float pn = __shfl_xor(s.n, off, kWave);
        float pm[EPL], pq[EPL];
#pragma unroll
        for (int i = 0; i < EPL; ++i) {
            pm[i] = __shfl_xor(s.m[i], off, kWave);
            pq[i] = __shfl_xor(s.q[i], off, kWave);
        }
        const bool low = ((g * G) & off) == 0;
        if (low) {
            stat_merge(s, pn, pm, pq, op);
        } else {
            Stat<EPL> t;
            t.n = pn;
#pragma unroll
            for (int i = 0; i < EPL; ++i) {
                t.m[i] = pm[i];
                t.q[i] = pq[i];
            }
            stat_merge(t, s.n, s.m, s.q, op);
            s = t;
        }
    }
}

template <int EPL>
HNV_DEV void stat_write(float *po, const Stat<EPL> &s, int op)
{
    float o[EPL];
#pragma unroll
    for (int i = 0; i < EPL; ++i)
        o[i] = (s.n == 0.0f) ? NAN : (op == HNV_SCORE_VARIANCE) ? s.q[i] / s.n : s.m[i];
#pragma unroll
    for (int i = 0; i < EPL; i += 4)
        *reinterpret_cast<float4 *>(po + i) = make_float4(o[i], o[i + 1], o[i + 2], o[i + 3]);
}

struct ScoreArgs {
    const Item *small;        // candidates of at most kIdxRegs * G members, largest first
    int32_t n_small;
    const Item *chunks;       // wavefront work items (aux = partial slot or -1)
    int32_t n_chunks;
    const Split *splits;      // candidates split over several chunks
    int32_t n_splits;
    int32_t nb_chunk, nb_small;
    const int32_t *idx;       // member node ids
    const void *z;
    int64_t ld;
    int op;
    float *out;
    float *partials;          // [slots x pstride]: mean [d], squared deviations [d], count
    int32_t pstride;
};

// OP (HNV_SCORE_*) is a template parameter so that each statistic keeps
// only the registers it needs.
template <typename T, int EPL, int G, int OP>
__global__ __launch_bounds__(kBlock) void k_score(ScoreArgs a)
{
    using S = Slice<T, EPL>;
    constexpr int Q = kWave / G;
    const int lane = threadIdx.x % kWave;
    const int g = lane / G, gl = lane % G;
    const int col = gl * EPL;
    const bool col_ok = col < a.ld;
    const T *z = static_cast<const T *>(a.z);
    Stat<EPL> st;
    stat_init(st, OP);
    const int64_t lb = linear_block();
    if (lb >= (int64_t)a.nb_chunk + a.nb_small)
        return;
    int b = (int)lb;
    if (b < a.nb_chunk) {
        const int item = b * kWavesPerBlock + (int)(threadIdx.x / kWave);
        if (item >= a.n_chunks)
            return;   // uniform over the wavefront
        const Item c = a.chunks[item];
        for (int base = 0; base < c.len; base += kWave) {
            const int my = (base + lane < c.len) ? a.idx[c.start + base + lane] : 0;
            const int n = min(kWave, c.len - base);
            for (int t = 0; t < n; t += 4 * Q) {
                typename S::Raw raw[4];
                bool ok[4];
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const int q = t + k * Q + g;
                    ok[k] = q < n;
                    const int v = __shfl(my, q & (kWave - 1), kWave);
                    if (ok[k] && col_ok)
                        raw[k] = S::load(z + (int64_t)v * a.ld + col);
                }
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    if (!ok[k])
                        continue;
                    float x[EPL];
                    if (col_ok)
                        S::unpack(raw[k], x);
                    else
                        zero(x);
                    stat_add(st, x, OP);
                }
            }
        }
        stat_wave_combine<EPL, G>(st, g, OP);
        if (g != 0 || !col_ok)
            return;
        if (c.aux < 0) {
            stat_write(a.out + (int64_t)c.row * a.ld + col, st, OP);
        } else {
            float *pp = a.partials + (int64_t)c.aux * a.pstride;
#pragma unroll
            for (int i = 0; i < EPL; ++i) {
                pp[col + i] = st.m[i];
                pp[a.ld + col + i] = st.q[i];
            }
            if (gl == 0)
                pp[2 * a.ld] = st.n;
        }
        return;
    }
    b -= a.nb_chunk;
    const int item = b * (kBlock / G) + (int)(threadIdx.x / G);
    const bool valid = item < a.n_small;
    Item it{0, 0, 0, 0};
    if (valid)
        it = a.small[item];
    int ix[kIdxRegs];
#pragma unroll
    for (int r = 0; r < kIdxRegs; ++r) {
        const int p = gl + r * G;
        ix[r] = (p < it.len) ? a.idx[it.start + p] : 0;
    }
    for (int j = 0; j < it.len; j += 4) {
        typename S::Raw raw[4];
        bool ok[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int q = j + k;
            const int r = q / G;
            const int xr = (r == 0) ? ix[0] : (r == 1) ? ix[1] : (r == 2) ? ix[2] : ix[3];
            ok[k] = q < it.len;
            const int v = __shfl(xr, g * G + (q & (G - 1)), kWave);
            if (ok[k] && col_ok)
                raw[k] = S::load(z + (int64_t)v * a.ld + col);
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            if (!ok[k])
                continue;
            float x[EPL];
            if (col_ok)
                S::unpack(raw[k], x);
            else
                zero(x);
            stat_add(st, x, OP);
        }
    }
    if (valid && col_ok)
        stat_write(a.out + (int64_t)it.row * a.ld + col, st, OP);
}

// Candidates split over several chunks: one wavefront merges the chunk
// partials in slot order (group g takes slots g, g+Q, ..., then the groups
// are combined lower first).
template <int EPL, int G, int OP>
__global__ __launch_bounds__(kBlock) void k_score_final(ScoreArgs a)
{
    constexpr int Q = kWave / G;
    const int64_t item = linear_block() * kWavesPerBlock + (int)(threadIdx.x / kWave);
    if (item >= a.n_splits)
        return;   // uniform over the wavefront
    const int lane = threadIdx.x % kWave;
    const int g = lane / G, gl = lane % G;
    const int col = gl * EPL;
    const bool col_ok = col < a.ld;
    const Split sp = a.splits[item];
    Stat<EPL> st;
    stat_init(st, OP);
    for (int k = g; k < sp.n_slots; k += Q) {
        const float *pp = a.partials + (int64_t)(sp.first_slot + k) * a.pstride;
        float bm[EPL], bq[EPL];
#pragma unroll
        for (int i = 0; i < EPL; ++i) {
            bm[i] = col_ok ? pp[col + i] : 0.0f;
            bq[i] = col_ok ? pp[a.ld + col + i] : 0.0f;
        }
        stat_merge(st, pp[2 * a.ld], bm, bq, OP);
    }
    stat_wave_combine<EPL, G>(st, g, OP);
    if (g == 0 && col_ok)
        stat_write(a.out + (int64_t)sp.row * a.ld + col, st, OP);
}

// ---------------------------------------------------------------------------
// reciprocals (FP64) and per-star-edge scale arrays
// ---------------------------------------------------------------------------

// node v: S_v = sum_{e ∋ v} w_e in FP64, r_v = 1 / S_v (0 without
// hyperedges).  A group of kRecipLanes lanes per node: lane i adds the
// positions i, i + 16, i + 32, ... in that order (four loads in flight),
// then a fixed butterfly over the group.
constexpr int kRecipLanes = 16;
__global__ __launch_bounds__(kBlock) void k_recip_nodes(const int32_t *__restrict__ ptr,
                                                        const int32_t *__restrict__ idx,
                                                        const float *__restrict__ w, int64_t n_nodes,
                                                        int64_t row_base_edges, float *__restrict__ r)
{
    const int64_t v = (linear_block() * kBlock + threadIdx.x) / kRecipLanes;
    const int gl = threadIdx.x % kRecipLanes;
    double s = 0.0;
    if (v < n_nodes) {
        const int32_t end = ptr[v + 1];
        int32_t j = ptr[v] + gl;
        for (; j + 3 * kRecipLanes < end; j += 4 * kRecipLanes) {
            const float w0 = w[idx[j] - row_base_edges], w1 = w[idx[j + kRecipLanes] - row_base_edges];
            const float w2 = w[idx[j + 2 * kRecipLanes] - row_base_edges];
            const float w3 = w[idx[j + 3 * kRecipLanes] - row_base_edges];
            s += (double)w0;
            s += (double)w1;
            s += (double)w2;
            s += (double)w3;
        }
        for (; j < end; j += kRecipLanes)
            s += (double)w[idx[j] - row_base_edges];
    }
#pragma unroll
    for (int off = 1; off < kRecipLanes; off <<= 1)
        s += __shfl_xor(s, off, kWave);
    if (v < n_nodes && gl == 0)
        r[v] = (s > 0.0) ? (float)(1.0 / s) : 0.0f;
}

// node v with unit weights: S_v is v's degree (the FP64 sum of that many
// ones, exactly), so r_v = 1 / degree without reading the hyperedge ids
__global__ __launch_bounds__(kBlock) void k_recip_nodes_unit(const int32_t *__restrict__ ptr, int64_t n_nodes,
                                                             float *__restrict__ r)
{
    const int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (v >= n_nodes)
        return;
    const int deg = ptr[v + 1] - ptr[v];
    r[v] = (deg > 0) ? (float)(1.0 / (double)deg) : 0.0f;
}

// hyperedge e: r_e = 1 / |e| (its weight cancels in its own mean)
__global__ __launch_bounds__(kBlock) void k_recip_edges(const int32_t *__restrict__ ptr, int64_t n_edges,
                                                        int64_t n_nodes, float *__restrict__ r)
{
    const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (e >= n_edges)
        return;
    const int deg = ptr[e + 1] - ptr[e];
    r[n_nodes + e] = (deg > 0) ? (float)(1.0 / (double)deg) : 0.0f;
}

// per star edge of the node side (neighbour = hyperedge e): its weight w_e,
// which the forward sweep multiplies by (not needed for unit weights)
__global__ __launch_bounds__(kBlock) void k_fill_weights(const int32_t *__restrict__ idx_node_side,
                                                         const float *__restrict__ w, int64_t nnz, int64_t n_nodes,
                                                         float *__restrict__ wn)
{
    const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (j < nnz)
        wn[j] = w[idx_node_side[j] - n_nodes];
}

// per star edge, the reverse sweep's scale, the reciprocal row sum of the
// neighbour: node side (neighbour = hyperedge e) r_e, hyperedge side
// (neighbour = node v) r_v
__global__ __launch_bounds__(kBlock) void k_fill_reverse_scales(const int32_t *__restrict__ idx_node_side,
                                                                const int32_t *__restrict__ idx_edge_side,
                                                                const float *__restrict__ r, int64_t nnz,
                                                                float *__restrict__ sn_node_side,
                                                                float *__restrict__ sn_edge_side)
{
    const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (j >= nnz)
        return;
    sn_node_side[j] = r[idx_node_side[j]];
    sn_edge_side[j] = r[idx_edge_side[j]];
}

__global__ __launch_bounds__(kBlock) void k_exp(const float *__restrict__ theta, float *__restrict__ w,
                                                float *__restrict__ w_out, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n)
        return;
    const float x = expf(theta[i]);
    w[i] = x;
    if (w_out)
        w_out[i] = x;
}

__global__ __launch_bounds__(kBlock) void k_mul(const float *__restrict__ a, const float *__restrict__ b,
                                                float *__restrict__ out, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n)
        out[i] = a[i] * b[i];
}

__global__ __launch_bounds__(kBlock) void k_cast_f32_bf16(const float *__restrict__ src, bf16_t *__restrict__ dst,
                                                          int64_t n)
{
    const int64_t i = linear_block() * kBlock + threadIdx.x;
    if (i < n)
        dst[i] = (bf16_t)to_bf16(src[i]);
}

__global__ __launch_bounds__(kBlock) void k_cast_bf16_f32(const bf16_t *__restrict__ src, float *__restrict__ dst,
                                                          int64_t n)
{
    const int64_t i = linear_block() * kBlock + threadIdx.x;
    if (i < n)
        dst[i] = __uint_as_float((uint32_t)src[i] << 16);
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------

hnv_status dev_check(const char *what)
{
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return fail(HNV_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
    return HNV_OK;
}

static inline unsigned grid1d(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

hnv_status dev_recompute_reciprocals(hnv_plan *p, int level, void *stream)
{
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    LevelPlan &L = p->lv[level];
    if (L.n_nodes > 0 && L.unit_w)
        k_recip_nodes_unit<<<grid1d(L.n_nodes, kBlock), kBlock, 0, s>>>(L.side[1].ptr, L.n_nodes, L.r);
    else if (L.n_nodes > 0)
        k_recip_nodes<<<fold_grid(blocks_for(L.n_nodes, kBlock / kRecipLanes)), kBlock, 0, s>>>(
            L.side[1].ptr, L.side[1].idx, L.w, L.n_nodes, L.n_nodes, L.r);
    if (L.n_edges > 0)
        k_recip_edges<<<grid1d(L.n_edges, kBlock), kBlock, 0, s>>>(L.side[0].ptr, L.n_edges, L.n_nodes, L.r);
    if (L.nnz > 0 && !L.unit_w)
        k_fill_weights<<<grid1d(L.nnz, kBlock), kBlock, 0, s>>>(L.side[1].idx, L.w, L.nnz, L.n_nodes, L.side[1].wn);
    L.scales_ready = false;   // the reverse sweep refills them from these reciprocals
    return dev_check("reciprocal kernels");
}

// small_ids[i] (and small_cids[i]) = the first kInlineIds neighbour ids of
// lane-group item i from idx (cidx), 0 past the row's degree.
__global__ __launch_bounds__(kBlock) void k_inline_ids(const Item *__restrict__ small, int64_t n,
                                                       const int32_t *__restrict__ idx,
                                                       const int32_t *__restrict__ cidx,
                                                       InlineIds *__restrict__ ids, InlineIds *__restrict__ cids)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n)
        return;
    const Item it = small[i];
    InlineIds a{}, c{};
#pragma unroll
    for (int k = 0; k < kInlineIds; ++k) {
        if (k < it.len) {
            a.id[k] = idx[it.start + k];
            if (cids)
                c.id[k] = cidx[it.start + k];
        }
    }
    ids[i] = a;
    if (cids)
        cids[i] = c;
}

hnv_status dev_fill_inline_ids(hnv_plan *p, int level, hipStream_t s)
{
    LevelPlan &L = p->lv[level];
    for (int sd = 0; sd < 2; ++sd) {
        const DevSide &D = L.side[sd];
        if (D.n_small > 0)
            k_inline_ids<<<grid1d(D.n_small, kBlock), kBlock, 0, s>>>(D.small, D.n_small, D.idx, D.cidx,
                                                                    const_cast<InlineIds *>(D.small_ids),
                                                                    const_cast<InlineIds *>(D.small_cids));
    }
    return dev_check("inline neighbour ids");
}

// The reverse sweep's per-star-edge scales of a level, filled from the
// current reciprocals before the first reverse sweep after a weight change
// (forward sweeps never read them).  While the stream is being captured the
// fill goes into the graph and is not taken as done.
static hnv_status ensure_reverse_scales(hnv_plan *p, int level, hipStream_t s)
{
    LevelPlan &L = p->lv[level];
    if (L.scales_ready)
        return HNV_OK;
    if (L.nnz > 0)
        k_fill_reverse_scales<<<grid1d(L.nnz, kBlock), kBlock, 0, s>>>(L.side[1].idx, L.side[0].idx, L.r, L.nnz,
                                                                       L.side[1].sn, L.side[0].sn);
    hnv_status st = dev_check("reverse-mode scales");
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    if (st == HNV_OK && hipStreamIsCapturing(s, &cap) == hipSuccess && cap == hipStreamCaptureStatusNone)
        L.scales_ready = true;
    return st;
}

static GatherArgs base_args(hnv_plan *p, LevelPlan &L, int G, int dp)
{
    GatherArgs a{};
    a.side[0] = L.side[0];
    a.side[1] = L.side[1];
    if (L.unit_w)
        a.side[1].wn = nullptr;  // unit weights: skip the per-edge multiply
    const int rows_per_block = kRowsPerGroup * kBlock / G;
    int32_t per_panel = 0;
    for (int s = 0; s < 2; ++s) {
        a.nb_chunk[s] = (int32_t)blocks_for(L.n_chunks[s], kWavesPerBlock);
        a.nb_small[s] = (int32_t)blocks_for(L.n_small[s], rows_per_block);
        a.nb_split[s] = (int32_t)blocks_for(L.n_splits[s], kWavesPerBlock);
        per_panel += a.nb_chunk[s] + a.nb_small[s];
    }
    a.blocks_per_panel = per_panel;
    a.dp = dp;
    a.ld = p->d;
    a.r = L.r;
    a.w = L.w;
    a.rowmap = L.rowmap;
    a.partials = p->partials;
    a.pstride = p->pstride;
    a.self_mapped = 0;
    return a;
}

// Restricts a launch to one side (the reverse sweep runs its two sides as
// two dependent launches).
static GatherArgs only_side(GatherArgs a, int side)
{
    const int other = 1 - side;
    a.nb_chunk[other] = a.nb_small[other] = a.nb_split[other] = 0;
    a.blocks_per_panel = a.nb_chunk[side] + a.nb_small[side];
    return a;
}

// Events bracketing one main-kernel launch when the plan is profiling.
struct ProfScope {
    hnv_plan *p;
    hipStream_t s;
    int kind, level;
    hipEvent_t b = nullptr, e = nullptr;
    hipEvent_t take()
    {
        if (!p->ev_pool.empty()) {
            hipEvent_t ev = reinterpret_cast<hipEvent_t>(p->ev_pool.back());
            p->ev_pool.pop_back();
            return ev;
        }
        hipEvent_t ev = nullptr;
        return hipEventCreate(&ev) == hipSuccess ? ev : nullptr;
    }
    void begin()
    {
        if (!p || !p->profiling)
            return;
        b = take();
        e = take();
        if (b && e)
            (void)hipEventRecord(b, s);
    }
    void end()
    {
        if (!b || !e)
            return;
        (void)hipEventRecord(e, s);
        p->prof.push_back(hnv_plan::ProfRecord{kind, level, b, e});
    }
};

template <typename T, int EPL, int G, int MODE, bool FUSED, bool CTL>
static void launch_pair(const GatherArgs &a, int panels, hipStream_t s, ProfScope *ps)
{
    const int64_t main_blocks = (int64_t)a.blocks_per_panel * panels;
    if (ps)
        ps->begin();
    if (main_blocks) {
        GatherArgs m = a;
        m.n_blocks = main_blocks;
        k_gather<T, EPL, G, MODE, FUSED, CTL><<<fold_grid(main_blocks), kBlock, 0, s>>>(m);
    }
    if (ps)
        ps->end();
    const int64_t fin_blocks = (int64_t)(a.nb_split[0] + a.nb_split[1]) * panels;
    if (fin_blocks) {
        GatherArgs f = a;
        f.resid_offset = a.resid_offset + (int32_t)main_blocks;
        f.n_blocks = fin_blocks;
        k_finalize<T, EPL, G, MODE, FUSED, CTL><<<fold_grid(fin_blocks), kBlock, 0, s>>>(f);
    }
}

// Instantiated lane layouts: BF16 always 8 elements per lane; FP32 4 per
// lane, or 8 for full-width rows of 128 columns or more (G = 16 .. 64).
template <typename T, int MODE, bool FUSED, bool CTL = false>
static hnv_status dispatch_g(int G, int EPL, const GatherArgs &a, int panels, hipStream_t s, ProfScope *ps)
{
    constexpr int E = 16 / (int)sizeof(T);
    if (EPL == E) {
        switch (G) {
        case 1: launch_pair<T, E, 1, MODE, FUSED, CTL>(a, panels, s, ps); break;
        case 2: launch_pair<T, E, 2, MODE, FUSED, CTL>(a, panels, s, ps); break;
        case 4: launch_pair<T, E, 4, MODE, FUSED, CTL>(a, panels, s, ps); break;
        case 8: launch_pair<T, E, 8, MODE, FUSED, CTL>(a, panels, s, ps); break;
        case 16: launch_pair<T, E, 16, MODE, FUSED, CTL>(a, panels, s, ps); break;
        case 32: launch_pair<T, E, 32, MODE, FUSED, CTL>(a, panels, s, ps); break;
        case 64: launch_pair<T, E, 64, MODE, FUSED, CTL>(a, panels, s, ps); break;
        default: return fail(HNV_EUNSUPPORTED, "lane group width");
        }
    } else if (E == 4 && EPL == 8) {
        switch (G) {
        case 16: launch_pair<T, 8, 16, MODE, FUSED, CTL>(a, panels, s, ps); break;
        case 32: launch_pair<T, 8, 32, MODE, FUSED, CTL>(a, panels, s, ps); break;
        case 64: launch_pair<T, 8, 64, MODE, FUSED, CTL>(a, panels, s, ps); break;
        default: return fail(HNV_EUNSUPPORTED, "lane group width");
        }
    } else {
        return fail(HNV_EUNSUPPORTED, "lane layout");
    }
    return dev_check("sweep kernels");
}

template <typename T>
static hnv_status dispatch_fwd(hnv_plan *p, bool fused, const GatherArgs &a, hipStream_t s, ProfScope *ps)
{
    if (a.ctl)
        return fused ? dispatch_g<T, kFwd, true, true>(p->g_fwd, p->epl_fwd, a, p->panels, s, ps)
                     : dispatch_g<T, kFwd, false, true>(p->g_fwd, p->epl_fwd, a, p->panels, s, ps);
    return fused ? dispatch_g<T, kFwd, true>(p->g_fwd, p->epl_fwd, a, p->panels, s, ps)
                 : dispatch_g<T, kFwd, false>(p->g_fwd, p->epl_fwd, a, p->panels, s, ps);
}

// Scratch of one forward sweep: the FP32 partial sums of rows split over
// several wavefronts, and the per-block FP64 residual partials with the two
// buffers of their reduction stages.  Every entry is written before it is
// read within the sweep, so nothing needs clearing.
struct SweepScratch {
    float *partials;
    double *resid_part;
    double *resid_stage;        // [2 x resid_stage_len]
    int64_t resid_stage_len;
};

static SweepScratch plan_scratch(const hnv_plan *p)
{
    return SweepScratch{p->partials, p->resid_part, p->resid_stage, p->resid_stage_len};
}

// The residuals of `batch` sweeps of one level (batch 1: a single sweep, the
// only form with ctl) from their per-block partials: n partials per sweep,
// sweep y's at part + y * part_stride; sweep y's residual goes to out[y].
// The stage sums alternate between two halves of sc.resid_stage, each
// batch x resid_stage_len long (a single sweep's scratch holds batch 1).
static hnv_status reduce_resid(const double *part, int64_t n, int batch, int64_t part_stride, double *out,
                               const SweepScratch &sc, SweepCtl *ctl, int level, hipStream_t s)
{
    const double *in = part;
    int64_t stride = part_stride;
    int which = 0;
    while (n > kResidPer) {
        const int64_t nb = blocks_for(n, kResidPer);
        double *o = sc.resid_stage + (int64_t)which * batch * sc.resid_stage_len;
        k_resid_stage<<<dim3((unsigned)nb, (unsigned)batch), kBlock, 0, s>>>(in, n, stride, o, sc.resid_stage_len, 0,
                                                                            ctl, level);
        in = o;
        stride = sc.resid_stage_len;
        n = nb;
        which ^= 1;
    }
    k_resid_stage<<<dim3(1, (unsigned)batch), kBlock, 0, s>>>(in, n, stride, out, 1, 1, ctl, level);
    return dev_check("residual kernels");
}

// One forward sweep of `level` (src -> dst); fused reads the coarser level.
// Jacobi: both sides in one launch, every row reading src.  Edge-first:
// hyperedge rows first (from src), then node rows, whose neighbours are the
// new hyperedge rows in dst and whose own value still comes from src.  With
// ctl (an early-stop refinement) src and dst come from the control block and
// the residual stage decides on the device whether the level goes on.  The
// scratch is the plan's workspace unless `scr` names other memory.  With
// resid_slot >= 0 (a fixed-count refinement) the sweep only leaves its
// per-block partials in that slot of the plan's residual scratch, for
// reduce_resid to reduce with the level's next sweeps.
static hnv_status run_sweep(hnv_plan *p, int level, const void *src, void *dst, float omega, bool fused,
                            double *resid_out, hipStream_t s, SweepCtl *ctl = nullptr,
                            const SweepScratch *scr = nullptr, int resid_slot = -1)
{
    LevelPlan &L = p->lv[level];
    const SweepScratch sc = scr ? *scr : plan_scratch(p);
    GatherArgs a = base_args(p, L, p->g_fwd, p->dp);
    a.partials = sc.partials;
    a.omega = omega;
    a.src = src;
    a.self_src = src;
    a.dst = dst;
    a.ctl = ctl;
    a.ctl_level = level;
    a.ctl_src_next = 0;
    a.resid = (resid_out || ctl) ? sc.resid_part : nullptr;
    if (resid_slot >= 0)
        a.resid = sc.resid_part + (int64_t)resid_slot * p->max_resid_blocks;
    a.resid_offset = 0;
    const bool bf = p->dtype == HNV_BF16;
    hnv_status st;
    if (p->opts.order == HNV_ORDER_JACOBI) {
        ProfScope ps{p, s, fused ? HNV_PROF_FUSED : HNV_PROF_SWEEP, level};
        st = bf ? dispatch_fwd<bf16_t>(p, fused, a, s, &ps) : dispatch_fwd<float>(p, fused, a, s, &ps);
    } else {
        GatherArgs e = only_side(a, 0);
        ProfScope pe{p, s, fused ? HNV_PROF_FUSED : HNV_PROF_SWEEP, level};
        st = bf ? dispatch_fwd<bf16_t>(p, fused, e, s, &pe) : dispatch_fwd<float>(p, fused, e, s, &pe);
        if (st != HNV_OK)
            return st;
        GatherArgs n = only_side(a, 1);
        n.src = dst;                      // neighbours: the hyperedge rows just written
        n.ctl_src_next = 1;
        n.self_mapped = fused ? 1 : 0;    // own value: from the coarser level in a fused sweep
        n.resid_offset = (int32_t)((e.blocks_per_panel + e.nb_split[0]) * p->panels);
        ProfScope pn{p, s, HNV_PROF_SWEEP, level};
        st = bf ? dispatch_fwd<bf16_t>(p, false, n, s, &pn) : dispatch_fwd<float>(p, false, n, s, &pn);
    }
    if (st != HNV_OK)
        return st;
    if (resid_slot < 0 && (resid_out || ctl)) {
        int64_t mb = 0, fb = 0;
        forward_geometry(p, L, &mb, &fb);
        return reduce_resid(sc.resid_part, mb + fb, 1, 0, resid_out, sc, ctl, level, s);
    }
    return HNV_OK;
}

// The projection onto `level` (zc -> zf); with ctl (an early-stop
// refinement) the matrices come from the control block, which then takes
// the projection's output as the latest iterate.
static hnv_status run_project(hnv_plan *p, int level, const void *zc, void *zf, hipStream_t s,
                              SweepCtl *ctl = nullptr)
{
    LevelPlan &L = p->lv[level];
    const int E = p->epl_full;
    const int64_t threads = L.rows * (p->d / E);
    if (threads > 0) {
        const dim3 grid = fold_grid(blocks_for(threads, kBlock));
        if (p->dtype == HNV_F32) {
            if (E == 4)
                k_project<float, 4><<<grid, kBlock, 0, s>>>(static_cast<const float *>(zc),
                                                            static_cast<float *>(zf), L.rowmap, L.rows, p->d, ctl);
            else
                k_project<float, 8><<<grid, kBlock, 0, s>>>(static_cast<const float *>(zc),
                                                            static_cast<float *>(zf), L.rowmap, L.rows, p->d, ctl);
        } else {
            k_project<bf16_t, 8><<<grid, kBlock, 0, s>>>(static_cast<const bf16_t *>(zc),
                                                         static_cast<bf16_t *>(zf), L.rowmap, L.rows, p->d, ctl);
        }
    }
    if (ctl)
        k_ctl_advance<<<1, 1, 0, s>>>(ctl);
    return dev_check("projection kernel");
}

static size_t elem_bytes(const hnv_plan *p) { return p->dtype == HNV_BF16 ? 2 : 4; }

static hnv_status check_level(const hnv_plan *p, int level)
{
    if (!p)
        return fail(HNV_EINVAL, "plan is NULL");
    if (level < 0 || level >= p->n_levels)
        return fail(HNV_EINVAL, "level " + std::to_string(level) + " out of range");
    return HNV_OK;
}

static bool aligned16(const void *q) { return (reinterpret_cast<uintptr_t>(q) & 15) == 0; }

}  // namespace hnv

using namespace hnv;

// ---------------------------------------------------------------------------
// C ABI (device calls)
// ---------------------------------------------------------------------------

extern "C" hnv_status hnv_set_edge_weights(hnv_plan *plan, int level, const float *w_dev, void *stream)
{
    clear_error();
    hnv_status st = check_level(plan, level);
    if (st != HNV_OK)
        return st;
    if (!w_dev && plan->lv[level].n_edges > 0)
        return fail(HNV_EINVAL, "w_dev is NULL");
    LevelPlan &L = plan->lv[level];
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    if (L.n_edges > 0) {
        hipError_t e = hipMemcpyAsync(L.w, w_dev, L.n_edges * sizeof(float), hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess)
            return fail(HNV_EDEVICE, std::string("hipMemcpyAsync: ") + hipGetErrorString(e));
    }
    L.unit_w = false;
    return dev_recompute_reciprocals(plan, level, stream);
}

extern "C" hnv_status hnv_set_edge_logweights(hnv_plan *plan, int level, const float *theta_dev, float *w_out_dev,
                                              void *stream)
{
    clear_error();
    hnv_status st = check_level(plan, level);
    if (st != HNV_OK)
        return st;
    LevelPlan &L = plan->lv[level];
    if (!theta_dev && L.n_edges > 0)
        return fail(HNV_EINVAL, "theta_dev is NULL");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    if (L.n_edges > 0)
        k_exp<<<grid1d(L.n_edges, kBlock), kBlock, 0, s>>>(theta_dev, L.w, w_out_dev, L.n_edges);
    if ((st = dev_check("exp kernel")) != HNV_OK)
        return st;
    L.unit_w = false;
    return dev_recompute_reciprocals(plan, level, stream);
}

extern "C" hnv_status hnv_logweight_grad(hnv_plan *plan, int level, const float *dw, float *dtheta, void *stream)
{
    clear_error();
    hnv_status st = check_level(plan, level);
    if (st != HNV_OK)
        return st;
    LevelPlan &L = plan->lv[level];
    if ((!dw || !dtheta) && L.n_edges > 0)
        return fail(HNV_EINVAL, "dw / dtheta is NULL");
    if (L.n_edges > 0)
        k_mul<<<grid1d(L.n_edges, kBlock), kBlock, 0, reinterpret_cast<hipStream_t>(stream)>>>(L.w, dw, dtheta,
                                                                                               L.n_edges);
    return dev_check("log-weight gradient kernel");
}

extern "C" hnv_status hnv_sweep(hnv_plan *plan, int level, const void *z_in, void *z_out, float omega,
                                int from_coarse, double *resid_dev, void *stream)
{
    clear_error();
    hnv_status st = check_level(plan, level);
    if (st != HNV_OK)
        return st;
    if (!z_in || !z_out)
        return fail(HNV_EINVAL, "z_in / z_out is NULL");
    if (z_in == z_out && (plan->opts.order != HNV_ORDER_EDGE_FIRST || from_coarse))
        return fail(HNV_EINVAL, "z_in and z_out may alias only for an edge-first sweep within a level");
    if (!aligned16(z_in) || !aligned16(z_out))
        return fail(HNV_EINVAL, "z_in / z_out must be 16-byte aligned");
    if (!(omega >= 0.0f && omega <= 1.0f))
        return fail(HNV_EINVAL, "omega must be in [0, 1]");
    if (from_coarse && !plan->lv[level].has_coarse)
        return fail(HNV_EINVAL, "from_coarse at the coarsest level");
    return run_sweep(plan, level, z_in, z_out, omega, from_coarse != 0, resid_dev,
                     reinterpret_cast<hipStream_t>(stream));
}

// ---------------------------------------------------------------------------
// the forward sweep for callers that cannot allocate: its scratch lives in a
// static device array instead of the plan's workspace
// ---------------------------------------------------------------------------

static __device__ __align__(256) unsigned char scratch[HNV_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices];   // per device: the address of `scratch` there (null until looked up)
}  // namespace

// The device address of `scratch` on the current device, looked up once per
// device with that device current.  The array's name is a host-side stand-in
// for the symbol; only this address may reach a kernel.
static hnv_status scratch_address(void **out)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return fail(HNV_EDEVICE, std::string("hipGetDevice: ") + hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices)
        return fail(HNV_EUNSUPPORTED, "device index beyond the static scratch table");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(HNV_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") +
                                         (e != hipSuccess ? hipGetErrorString(e) : "null address"));
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return HNV_OK;
}

static int64_t align256(int64_t x) { return (x + 255) & ~int64_t(255); }

extern "C" hnv_status hnv_sweep_noalloc(hnv_plan *plan, int level, const void *z_in, void *z_out, float omega,
                                        int from_coarse, double *resid_dev, void *stream)
{
    clear_error();
    hnv_status st = check_level(plan, level);
    if (st != HNV_OK)
        return st;
    if (!z_in || !z_out)
        return fail(HNV_EINVAL, "z_in / z_out is NULL");
    if (z_in == z_out && (plan->opts.order != HNV_ORDER_EDGE_FIRST || from_coarse))
        return fail(HNV_EINVAL, "z_in and z_out may alias only for an edge-first sweep within a level");
    if (!aligned16(z_in) || !aligned16(z_out))
        return fail(HNV_EINVAL, "z_in / z_out must be 16-byte aligned");
    if (!(omega >= 0.0f && omega <= 1.0f))
        return fail(HNV_EINVAL, "omega must be in [0, 1]");
    if (from_coarse && !plan->lv[level].has_coarse)
        return fail(HNV_EINVAL, "from_coarse at the coarsest level");
    // the level's scratch, laid out in the static array: residual partials
    // and stages (only with a residual), then the split-row partial slots
    const LevelPlan &L = plan->lv[level];
    int64_t mb = 0, fb = 0;
    forward_geometry(plan, L, &mb, &fb);
    const int64_t n_part = resid_dev ? mb + fb : 0;
    const int64_t stage_len = resid_dev ? blocks_for(n_part, kResidPer) + 1 : 0;
    const int64_t off_stage = align256(n_part * (int64_t)sizeof(double));
    const int64_t off_slots = off_stage + align256(2 * stage_len * (int64_t)sizeof(double));
    const int64_t need = off_slots + (int64_t)L.n_slots * plan->pstride * (int64_t)sizeof(float);
    if (need > (int64_t)HNV_NOALLOC_SCRATCH_BYTES)
        return fail(HNV_EUNSUPPORTED, "level " + std::to_string(level) + " needs " + std::to_string(need) +
                                          " bytes of sweep scratch, more than the static " +
                                          std::to_string((int64_t)HNV_NOALLOC_SCRATCH_BYTES));
    void *base = nullptr;
    if ((st = scratch_address(&base)) != HNV_OK)
        return st;
    char *b = static_cast<char *>(base);
    const SweepScratch sc{reinterpret_cast<float *>(b + off_slots), reinterpret_cast<double *>(b),
                          reinterpret_cast<double *>(b + off_stage), stage_len};
    return run_sweep(plan, level, z_in, z_out, omega, from_coarse != 0, resid_dev,
                     reinterpret_cast<hipStream_t>(stream), nullptr, &sc);
}

extern "C" hnv_status hnv_project(hnv_plan *plan, int level, const void *z_coarse, void *z_fine, void *stream)
{
    clear_error();
    hnv_status st = check_level(plan, level);
    if (st != HNV_OK)
        return st;
    if (!plan->lv[level].has_coarse)
        return fail(HNV_EINVAL, "no coarser level to project from");
    if (!z_coarse || !z_fine || !aligned16(z_coarse) || !aligned16(z_fine))
        return fail(HNV_EINVAL, "z_coarse / z_fine NULL or not 16-byte aligned");
    return run_project(plan, level, z_coarse, z_fine, reinterpret_cast<hipStream_t>(stream));
}

// Refinement with the epsilon rule (Section 3.3), decided on the device:
// each sweep's residual stage compares its change with tol and raises the
// level's stop flag, after which that level's remaining sweeps return at
// once.  The operations read and write the matrices the control block
// names, so where the iterate ends up is known on the device only; a last
// kernel copies it to z_finest if it is not there already.  Sweeps are
// enqueued in batches of 1, 2, 4, .. kMaxStopBatch per level, and the host
// reads the level's flag between batches only to stop enqueueing launches
// that would do nothing: O(log K) waits per level instead of one per sweep.
// While the stream is being captured into a graph every sweep is enqueued
// and nothing waits for the host.
constexpr int kMaxStopBatch = 16;

static hnv_status refine_early_stop(hnv_plan *plan, const void *z_coarsest, void *z_finest,
                                    const int32_t *sweeps_per_level, float omega, double tol,
                                    double *residuals_dev, int32_t *sweeps_done, hipStream_t s, void *first_out)
{
    const int Lc = plan->n_levels - 1;
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cap) != hipSuccess)
        return fail(HNV_EDEVICE, "hipStreamIsCapturing failed");
    const bool capturing = cap != hipStreamCaptureStatusNone;
    if (capturing && sweeps_done)
        return fail(HNV_EINVAL, "sweeps_done must be NULL while the stream is being captured");
    k_ctl_init<<<1, kBlock, 0, s>>>(plan->ctl, plan->ctl_flags, plan->n_levels, z_coarsest, first_out, z_finest,
                                    plan->zbuf, residuals_dev, plan->resid_tmp, tol);
    hnv_status st = dev_check("early-stop set-up");
    for (int l = Lc; l >= 0 && st == HNV_OK; --l) {
        const int K = sweeps_per_level[l];
        if (K == 0 && l < Lc)
            st = run_project(plan, l, nullptr, nullptr, s, plan->ctl);
        int k = 0, batch = 1;
        while (k < K && st == HNV_OK) {
            for (const int end = std::min(K, k + batch); k < end && st == HNV_OK; ++k)
                st = run_sweep(plan, l, nullptr, nullptr, omega, k == 0 && l < Lc, nullptr, s, plan->ctl);
            if (st != HNV_OK || k >= K)
                break;
            if (capturing) {   // no waits in a graph: the rest of the level at once
                batch = K;
                continue;
            }
            int32_t stopped = 0;
            hipError_t e = hipMemcpyAsync(&stopped, plan->ctl_flags + l, sizeof(int32_t), hipMemcpyDeviceToHost, s);
            if (e == hipSuccess)
                e = hipStreamSynchronize(s);
            if (e != hipSuccess)
                return fail(HNV_EDEVICE, std::string("stop-flag read-back: ") + hipGetErrorString(e));
            if (stopped)
                break;
            batch = std::min(2 * batch, kMaxStopBatch);
        }
    }
    if (st != HNV_OK)
        return st;
    const int64_t n16 = plan->lv[0].rows * plan->d * (int64_t)elem_bytes(plan) / 16;
    if (n16 > 0)
        k_ctl_result<<<grid1d(std::min<int64_t>(n16, 2048LL * kBlock), kBlock), kBlock, 0, s>>>(plan->ctl, z_finest,
                                                                                                 n16);
    if ((st = dev_check("result copy")) != HNV_OK)
        return st;
    if (sweeps_done) {
        hipError_t e = hipMemcpyAsync(sweeps_done, plan->ctl_flags + plan->n_levels,
                                      sizeof(int32_t) * plan->n_levels, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess)
            e = hipStreamSynchronize(s);
        if (e != hipSuccess)
            return fail(HNV_EDEVICE, std::string("sweep-count read-back: ") + hipGetErrorString(e));
    }
    return HNV_OK;
}

extern "C" hnv_status hnv_refine(hnv_plan *plan, const void *z_coarsest, void *z_finest,
                                 const int32_t *sweeps_per_level, float omega, double tol, double *residuals_dev,
                                 int32_t *sweeps_done, void *stream)
{
    clear_error();
    if (!plan)
        return fail(HNV_EINVAL, "plan is NULL");
    if (!z_coarsest || !z_finest || z_coarsest == z_finest || !sweeps_per_level)
        return fail(HNV_EINVAL, "z_coarsest / z_finest / sweeps_per_level NULL or aliased");
    if (!aligned16(z_coarsest) || !aligned16(z_finest))
        return fail(HNV_EINVAL, "embeddings must be 16-byte aligned");
    if (!(omega >= 0.0f && omega <= 1.0f))
        return fail(HNV_EINVAL, "omega must be in [0, 1]");
    const int Lc = plan->n_levels - 1;
    for (int l = 0; l <= Lc; ++l)
        if (sweeps_per_level[l] < 0)
            return fail(HNV_EINVAL, "negative sweep count");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const size_t eb = elem_bytes(plan);

    // Operations in order: per level (coarsest first) the sweeps, or a bare
    // projection when a finer level has no sweeps.  Writes alternate between
    // z_finest and the scratch buffer.
    int64_t n_ops = 0;
    for (int l = Lc; l >= 0; --l)
        n_ops += (sweeps_per_level[l] > 0) ? sweeps_per_level[l] : (l < Lc ? 1 : 0);
    if (n_ops == 0) {
        hipError_t e = hipMemcpyAsync(z_finest, z_coarsest, plan->lv[0].rows * plan->d * eb,
                                      hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess)
            return fail(HNV_EDEVICE, std::string("hipMemcpyAsync: ") + hipGetErrorString(e));
        if (sweeps_done)
            for (int l = 0; l <= Lc; ++l)
                sweeps_done[l] = 0;
        return HNV_OK;
    }
    void *bufs[2] = {z_finest, plan->zbuf};
    if (tol > 0)
        return refine_early_stop(plan, z_coarsest, z_finest, sweeps_per_level, omega, tol, residuals_dev,
                                 sweeps_done, s, bufs[(n_ops - 1) % 2]);
    int64_t op = 0;
    const void *cur = z_coarsest;
    // the alternation is counted back from the last operation, which writes z_finest
    auto target = [&](int64_t k) { return bufs[(n_ops - 1 - k) % 2]; };
    int64_t resid_k = 0;
    hnv_status st = HNV_OK;
    for (int l = Lc; l >= 0; --l) {
        const int K = sweeps_per_level[l];
        if (K == 0 && l < Lc) {
            void *out = target(op++);
            if ((st = run_project(plan, l, cur, out, s)) != HNV_OK)
                return st;
            cur = out;
        }
        // the level's residuals reduced kResidBatch sweeps at a time
        int64_t mb = 0, fb = 0;
        forward_geometry(plan, plan->lv[l], &mb, &fb);
        int pending = 0;
        for (int k = 0; k < K; ++k) {
            void *out = target(op++);
            const bool fused = (k == 0 && l < Lc);
            if ((st = run_sweep(plan, l, cur, out, omega, fused, nullptr, s, nullptr, nullptr,
                                residuals_dev ? pending : -1)) != HNV_OK)
                return st;
            ++resid_k;
            cur = out;
            if (residuals_dev && (++pending == kResidBatch || k + 1 == K)) {
                if ((st = reduce_resid(plan->resid_part, mb + fb, pending, plan->max_resid_blocks,
                                       residuals_dev + resid_k - pending, plan_scratch(plan), nullptr, l, s)) !=
                    HNV_OK)
                    return st;
                pending = 0;
            }
        }
        if (sweeps_done)
            sweeps_done[l] = K;
    }
    return HNV_OK;
}

// One reverse sweep of `level`.  wgrad: 0 no weight gradient (the sweep's
// input and output rows are not read), 1 the whole gradient into dw in this
// sweep, 2 split: node rows add omega times their scalar to node_acc,
// hyperedge rows add only their own term to dw.
//
// Jacobi order: node rows first (they produce the per-node scalars), then
// hyperedge rows, which with wgrad = 1 sum the scalars of their members.
// Edge-first order: the forward node half read the new hyperedge rows, so
// the hyperedge rows go first, writing dL/de' to the plan's scratch
// embedding; the node rows then gather it.  There the per-node scalars come
// last, so wgrad = 1 runs as the split form over one sweep: the scalars go
// to the plan's per-node scratch and a finish pass subtracts omega times
// their member sums.
static hnv_status run_adjoint(hnv_plan *plan, int level, const void *g_in, void *g_out, const void *z_prev,
                              const void *z_cur, float *dw, float *node_acc, float omega, int wgrad, hipStream_t s)
{
    LevelPlan &L = plan->lv[level];
    if (hnv_status st = ensure_reverse_scales(plan, level, s); st != HNV_OK)
        return st;
    const int G = plan->g_full, E = plan->epl_full;
    const bool edge_first = plan->opts.order == HNV_ORDER_EDGE_FIRST;
    GatherArgs a = base_args(plan, L, G, plan->d);
    a.omega = omega;
    a.src = g_in;
    a.self_src = g_in;
    a.dst = g_out;
    a.yprev = z_prev;
    a.zcur = z_cur;
    a.cvec = (wgrad == 2) ? node_acc : plan->cscratch;
    a.dw = (wgrad == 0) ? nullptr : dw;
    a.wgrad = wgrad;
    a.resid = nullptr;
    GatherArgs an = only_side(a, 1), ae = only_side(a, 0);
    ProfScope pn{plan, s, HNV_PROF_ADJ_NODE, level}, pe{plan, s, HNV_PROF_ADJ_EDGE, level};
    hnv_status st;
    if (edge_first) {
        ae.dst2 = plan->zbuf;
        ae.yprev = z_cur;     // the dot of the weight gradient takes e'_e
        an.src = plan->zbuf;  // node rows gather dL/de'
        const bool whole = (wgrad == 1);
        if (whole)
            an.wgrad = 1;     // store the scalars (plain, not times omega)
        if (plan->dtype == HNV_F32) {
            if ((st = dispatch_g<float, kAdjEdgeNoSum, false>(G, E, ae, 1, s, &pe)) != HNV_OK)
                return st;
            st = dispatch_g<float, kAdjNode, false>(G, E, an, 1, s, &pn);
        } else {
            if ((st = dispatch_g<bf16_t, kAdjEdgeNoSum, false>(G, E, ae, 1, s, &pe)) != HNV_OK)
                return st;
            st = dispatch_g<bf16_t, kAdjNode, false>(G, E, an, 1, s, &pn);
        }
        if (st != HNV_OK || !whole || L.n_edges == 0)
            return st;
        const int64_t threads = L.n_edges * 16;
        k_wgrad_finish<<<fold_grid(blocks_for(threads, kBlock)), kBlock, 0, s>>>(
            L.side[0].ptr, L.side[0].idx, plan->cscratch, dw, L.n_edges, omega);
        return dev_check("weight-gradient finish");
    }
    if (plan->dtype == HNV_F32) {
        if ((st = dispatch_g<float, kAdjNode, false>(G, E, an, 1, s, &pn)) != HNV_OK)
            return st;
        st = (wgrad == 1) ? dispatch_g<float, kAdjEdge, false>(G, E, ae, 1, s, &pe)
                          : dispatch_g<float, kAdjEdgeNoSum, false>(G, E, ae, 1, s, &pe);
    } else {
        if ((st = dispatch_g<bf16_t, kAdjNode, false>(G, E, an, 1, s, &pn)) != HNV_OK)
            return st;
        st = (wgrad == 1) ? dispatch_g<bf16_t, kAdjEdge, false>(G, E, ae, 1, s, &pe)
                          : dispatch_g<bf16_t, kAdjEdgeNoSum, false>(G, E, ae, 1, s, &pe);
    }
    return st;
}

static hnv_status check_adjoint_args(hnv_plan *plan, int level, const void *g_in, void *g_out, const void *z_prev,
                                     const void *z_cur, float omega)
{
    hnv_status st = check_level(plan, level);
    if (st != HNV_OK)
        return st;
    if (!g_in || !g_out || !z_prev || !z_cur || g_in == g_out)
        return fail(HNV_EINVAL, "NULL or aliased matrices");
    if (!aligned16(g_in) || !aligned16(g_out) || !aligned16(z_prev) || !aligned16(z_cur))
        return fail(HNV_EINVAL, "matrices must be 16-byte aligned");
    if (!(omega > 0.0f && omega <= 1.0f))
        return fail(HNV_EINVAL, "omega must be in (0, 1] for the reverse sweep");
    return HNV_OK;
}

extern "C" hnv_status hnv_sweep_adjoint(hnv_plan *plan, int level, const void *g_in, void *g_out,
                                        const void *z_prev, const void *z_cur, float *dw_accum, float omega,
                                        void *stream)
{
    clear_error();
    hnv_status st = check_adjoint_args(plan, level, g_in, g_out, z_prev, z_cur, omega);
    if (st != HNV_OK)
        return st;
    return run_adjoint(plan, level, g_in, g_out, z_prev, z_cur, dw_accum, nullptr, omega, dw_accum ? 1 : 0,
                       reinterpret_cast<hipStream_t>(stream));
}

extern "C" hnv_status hnv_sweep_adjoint_split(hnv_plan *plan, int level, const void *g_in, void *g_out,
                                              const void *z_prev, const void *z_cur, float *dw_accum,
                                              float *node_accum, float omega, void *stream)
{
    clear_error();
    hnv_status st = check_adjoint_args(plan, level, g_in, g_out, z_prev, z_cur, omega);
    if (st != HNV_OK)
        return st;
    const LevelPlan &L = plan->lv[level];
    if ((!dw_accum && L.n_edges > 0) || (!node_accum && L.n_nodes > 0))
        return fail(HNV_EINVAL, "dw_accum / node_accum is NULL");
    return run_adjoint(plan, level, g_in, g_out, z_prev, z_cur, dw_accum, node_accum, omega, 2,
                       reinterpret_cast<hipStream_t>(stream));
}

extern "C" hnv_status hnv_weight_grad_finish(hnv_plan *plan, int level, const float *node_accum, float *dw_accum,
                                             void *stream)
{
    clear_error();
    hnv_status st = check_level(plan, level);
    if (st != HNV_OK)
        return st;
    const LevelPlan &L = plan->lv[level];
    if (L.n_edges == 0)
        return HNV_OK;
    if (!dw_accum || (!node_accum && L.n_nodes > 0))
        return fail(HNV_EINVAL, "dw_accum / node_accum is NULL");
    const int64_t threads = L.n_edges * 16;
    k_wgrad_finish<<<fold_grid(blocks_for(threads, kBlock)), kBlock, 0, reinterpret_cast<hipStream_t>(stream)>>>(
        L.side[0].ptr, L.side[0].idx, node_accum, dw_accum, L.n_edges, 1.0f);
    return dev_check("weight-gradient finish");
}

extern "C" hnv_status hnv_project_adjoint(hnv_plan *plan, int level, const void *g_fine, void *g_coarse,
                                          void *stream)
{
    clear_error();
    hnv_status st = check_level(plan, level);
    if (st != HNV_OK)
        return st;
    LevelPlan &L = plan->lv[level];
    if (!L.has_coarse)
        return fail(HNV_EINVAL, "no coarser level");
    if (!g_fine || !g_coarse || !aligned16(g_fine) || !aligned16(g_coarse))
        return fail(HNV_EINVAL, "g_fine / g_coarse NULL or not 16-byte aligned");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const int G = plan->g_full, E = plan->epl_full;
    const int64_t n_blocks = blocks_for(L.rows_coarse, kWavesPerBlock);
    if (n_blocks == 0)
        return HNV_OK;
    const dim3 blocks = fold_grid(n_blocks);
#define HNV_PADJ(TT, EE, GG)                                                                                     \
    k_project_adj<TT, EE, GG><<<blocks, kBlock, 0, s>>>(static_cast<const TT *>(g_fine), static_cast<TT *>(g_coarse), \
                                                        L.inv_ptr, L.inv_idx, L.rows_coarse, plan->d)
#define HNV_PADJ_G(TT, EE)                                                                                       \
    switch (G) {                                                                                                 \
    case 1: HNV_PADJ(TT, EE, 1); break;                                                                          \
    case 2: HNV_PADJ(TT, EE, 2); break;                                                                          \
    case 4: HNV_PADJ(TT, EE, 4); break;                                                                          \
    case 8: HNV_PADJ(TT, EE, 8); break;                                                                          \
    case 16: HNV_PADJ(TT, EE, 16); break;                                                                        \
    case 32: HNV_PADJ(TT, EE, 32); break;                                                                        \
    default: HNV_PADJ(TT, EE, 64); break;                                                                        \
    }
    if (plan->dtype == HNV_F32) {
        if (E == 4) {
            HNV_PADJ_G(float, 4)
        } else if (G == 16) {
            HNV_PADJ(float, 8, 16);
        } else if (G == 32) {
            HNV_PADJ(float, 8, 32);
        } else {
            HNV_PADJ(float, 8, 64);
        }
    } else {
        HNV_PADJ_G(bf16_t, 8)
    }
#undef HNV_PADJ_G
#undef HNV_PADJ
    return dev_check("projection reverse kernel");
}

extern "C" hnv_status hnv_cast(const void *src, hnv_dtype src_dtype, void *dst, hnv_dtype dst_dtype, int64_t n,
                               void *stream)
{
    clear_error();
    if (n < 0 || (n > 0 && (!src || !dst)))
        return fail(HNV_EINVAL, "bad cast arguments");
    if (n == 0)
        return HNV_OK;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    if (src_dtype == HNV_F32 && dst_dtype == HNV_BF16)
        k_cast_f32_bf16<<<fold_grid(blocks_for(n, kBlock)), kBlock, 0, s>>>(static_cast<const float *>(src),
                                                                            static_cast<bf16_t *>(dst), n);
    else if (src_dtype == HNV_BF16 && dst_dtype == HNV_F32)
        k_cast_bf16_f32<<<fold_grid(blocks_for(n, kBlock)), kBlock, 0, s>>>(static_cast<const bf16_t *>(src),
                                                                            static_cast<float *>(dst), n);
    else if (src_dtype == dst_dtype) {
        hipError_t e = hipMemcpyAsync(dst, src, n * (src_dtype == HNV_BF16 ? 2 : 4), hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess)
            return fail(HNV_EDEVICE, std::string("hipMemcpyAsync: ") + hipGetErrorString(e));
        return HNV_OK;
    } else
        return fail(HNV_EINVAL, "unknown dtype");
    return dev_check("cast kernel");
}

extern "C" hnv_status hnv_plan_set_profiling(hnv_plan *plan, int enable)
{
    clear_error();
    if (!plan)
        return fail(HNV_EINVAL, "plan is NULL");
    if (!enable) {
        for (auto &r : plan->prof) {
            plan->ev_pool.push_back(r.ev_begin);
            plan->ev_pool.push_back(r.ev_end);
        }
        plan->prof.clear();
    }
    plan->profiling = enable != 0;
    return HNV_OK;
}

extern "C" hnv_status hnv_plan_profile_read(hnv_plan *plan, int kind, int level, int64_t *launches,
                                            double *total_ms)
{
    clear_error();
    if (!plan || !launches || !total_ms)
        return fail(HNV_EINVAL, "NULL argument");
    int64_t n = 0;
    double ms = 0.0;
    for (auto &r : plan->prof) {
        if (r.kind != kind || (level >= 0 && r.level != level))
            continue;
        hipEvent_t e = reinterpret_cast<hipEvent_t>(r.ev_end);
        hipError_t err = hipEventSynchronize(e);
        float t = 0.0f;
        if (err == hipSuccess)
            err = hipEventElapsedTime(&t, reinterpret_cast<hipEvent_t>(r.ev_begin), e);
        if (err != hipSuccess)
            return fail(HNV_EDEVICE, std::string("event timing: ") + hipGetErrorString(err));
        ++n;
        ms += t;
    }
    *launches = n;
    *total_ms = ms;
    return HNV_OK;
}

hnv_plan::~hnv_plan()
{
    for (auto &r : prof) {
        (void)hipEventDestroy(reinterpret_cast<hipEvent_t>(r.ev_begin));
        (void)hipEventDestroy(reinterpret_cast<hipEvent_t>(r.ev_end));
    }
    for (void *ev : ev_pool)
        (void)hipEventDestroy(reinterpret_cast<hipEvent_t>(ev));
}

namespace hnv {
// Launches the scoring kernels on a plan that hnv_host.cpp built and
// uploaded (see hnv_score_candidates there).
template <typename T, int EPL, int G, int OP>
static void launch_score(const ScoreArgs &a, int64_t grid, int64_t fgrid, hipStream_t s)
{
    if (grid)
        k_score<T, EPL, G, OP><<<fold_grid(grid), kBlock, 0, s>>>(a);
    if (fgrid)
        k_score_final<EPL, G, OP><<<fold_grid(fgrid), kBlock, 0, s>>>(a);
}

hnv_status dev_score(const ScorePlan &sp, const void *z, hnv_dtype dtype, int d, int op, float *out,
                     hipStream_t s)
{
    int G = 1, E = 8;
    lane_layout(d, dtype == HNV_BF16 ? 2 : 4, &G, &E);
    ScoreArgs a{};
    a.small = sp.small;
    a.n_small = sp.n_small;
    a.chunks = sp.chunks;
    a.n_chunks = sp.n_chunks;
    a.splits = sp.splits;
    a.n_splits = sp.n_splits;
    a.nb_chunk = (int32_t)blocks_for(sp.n_chunks, kWavesPerBlock);
    a.nb_small = (int32_t)blocks_for(sp.n_small, kBlock / G);
    a.idx = sp.idx;
    a.z = z;
    a.ld = d;
    a.op = op;
    a.out = out;
    a.partials = sp.partials;
    a.pstride = 2 * d + 8;
    const int64_t grid = (int64_t)a.nb_chunk + a.nb_small;
    const int64_t fgrid = blocks_for(sp.n_splits, kWavesPerBlock);
#define HNV_SCORE(TT, EE, GG)                                                   \
    do {                                                                        \
        switch (op) {                                                           \
        case HNV_SCORE_VARIANCE: launch_score<TT, EE, GG, HNV_SCORE_VARIANCE>(a, grid, fgrid, s); break; \
        case HNV_SCORE_MEAN: launch_score<TT, EE, GG, HNV_SCORE_MEAN>(a, grid, fgrid, s); break;         \
        case HNV_SCORE_MIN: launch_score<TT, EE, GG, HNV_SCORE_MIN>(a, grid, fgrid, s); break;           \
        default: launch_score<TT, EE, GG, HNV_SCORE_MAX>(a, grid, fgrid, s); break;                      \
        }                                                                       \
    } while (0)
#define HNV_SCORE_G(TT, EE)                                                     \
    switch (G) {                                                                \
    case 1: HNV_SCORE(TT, EE, 1); break;                                        \
    case 2: HNV_SCORE(TT, EE, 2); break;                                        \
    case 4: HNV_SCORE(TT, EE, 4); break;                                        \
    case 8: HNV_SCORE(TT, EE, 8); break;                                        \
    case 16: HNV_SCORE(TT, EE, 16); break;                                      \
    case 32: HNV_SCORE(TT, EE, 32); break;                                      \
    default: HNV_SCORE(TT, EE, 64); break;                                      \
    }
    if (dtype == HNV_BF16) {
        HNV_SCORE_G(bf16_t, 8)
    } else if (E == 4) {
        HNV_SCORE_G(float, 4)
    } else if (G == 16) {
        HNV_SCORE(float, 8, 16);
    } else if (G == 32) {
        HNV_SCORE(float, 8, 32);
    } else {
        HNV_SCORE(float, 8, 64);
    }
#undef HNV_SCORE_G
#undef HNV_SCORE
    return dev_check("candidate scoring kernels");
}
}  // namespace hnv

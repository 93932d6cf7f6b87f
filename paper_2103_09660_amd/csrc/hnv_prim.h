// Library sort and scan primitives of the GPU coarsening and the device plan
// builder, called straight from rocPRIM.  Each takes rocPRIM's two-phase
// form: with temp == nullptr it only writes the temporary storage it needs
// to `bytes`; otherwise it enqueues the work on `s`.  The radix sorts are
// stable (least significant digit first), which the callers rely on for
// their tie orders.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>

#include <rocprim/device/device_radix_sort.hpp>
#include <rocprim/device/device_scan.hpp>
#include <rocprim/device/device_segmented_radix_sort.hpp>
#include <rocprim/functional.hpp>

namespace hnv {

// The radix sorts take the one-sweep (digit-at-a-time) path from 2^16 pairs
// on: for the hundreds of thousands of hyperedges of a coarse level it is
// fewer launches than the merge path rocPRIM picks by default below 2^20.
// The one-sweep passes take 9-bit digits over workgroups of 1024 threads x 8
// pairs: measured on MI355X against rocPRIM's default for this target (8-bit
// digits, 1024 x 16), 22% faster on 13.1M pairs with 21-bit keys, 7% on 3.5M
// with 22-bit keys, 21-31% on 0.4M-1.5M; the result does not depend on the
// configuration (a stable sort).
using SortConfig = rocprim::radix_sort_config<
    rocprim::default_config, rocprim::default_config,
    rocprim::radix_sort_onesweep_config<rocprim::kernel_config<1024, 16>, rocprim::kernel_config<1024, 8>, 9,
                                        rocprim::block_radix_rank_algorithm::match>,
    size_t(1) << 16>;

// (key, value) pairs by key bits [begin_bit, end_bit), stable.
template <typename K, typename V>
inline hipError_t prim_sort_pairs(void *temp, size_t &bytes, const K *keys_in, K *keys_out, const V *vals_in,
                                  V *vals_out, int64_t n, int begin_bit, int end_bit, hipStream_t s = 0)
{
    return rocprim::radix_sort_pairs<SortConfig>(temp, bytes, keys_in, keys_out, vals_in, vals_out, (size_t)n,
                                                 (unsigned)begin_bit, (unsigned)end_bit, s);
}

// The segmented sort takes one workgroup per segment and never splits the
// segments by size: the split that rocPRIM's default configuration makes
// from 64 segments on reads the split's counts back to the host, a wait in
// the middle of the caller's work.  The callers pass only long segments
// (and empty ones, which end at once).
using SegSortConfig = rocprim::segmented_radix_sort_config<8, rocprim::kernel_config<256, 16>,
                                                           rocprim::DisabledWarpSortConfig, false>;

// Keys of each segment [begin[i], end[i]) sorted independently, stable.
template <typename K, typename O>
inline hipError_t prim_segmented_sort_keys(void *temp, size_t &bytes, const K *keys_in, K *keys_out, int64_t n,
                                           int64_t segments, O begin, O end, int begin_bit, int end_bit,
                                           hipStream_t s = 0)
{
    return rocprim::segmented_radix_sort_keys<SegSortConfig>(temp, bytes, keys_in, keys_out, (unsigned)n,
                                                             (unsigned)segments, begin, end, (unsigned)begin_bit,
                                                             (unsigned)end_bit, s);
}

// The scans take workgroups of 256 threads x 32 items of 4 bytes (x 12 of
// larger types): rocPRIM has no tuned scan configuration for this target and
// falls back to 256 x 16, which measured on MI355X 30% slower on 13.1M int32
// sums (59 against 42 us) and on 3.3M sums of three int32 (48 against 33 us).
template <typename T>
using ScanConfig = rocprim::scan_config<256, sizeof(T) <= 4 ? 32 : 12, rocprim::block_load_method::block_load_transpose,
                                        rocprim::block_store_method::block_store_transpose,
                                        rocprim::block_scan_algorithm::using_warp_scan>;

// out[i] = in[0] + .. + in[i-1], out[0] = 0.
template <typename T>
inline hipError_t prim_exclusive_sum(void *temp, size_t &bytes, const T *in, T *out, int64_t n, hipStream_t s = 0)
{
    return rocprim::exclusive_scan<ScanConfig<T>>(temp, bytes, in, out, T(0), (size_t)n, rocprim::plus<T>(), s);
}

// out[i] = in[0] op .. op in[i-1], out[0] = init, for an associative op.
template <typename T, typename Op>
inline hipError_t prim_exclusive_scan(void *temp, size_t &bytes, const T *in, T *out, T init, int64_t n, Op op,
                                      hipStream_t s = 0)
{
    return rocprim::exclusive_scan<ScanConfig<T>>(temp, bytes, in, out, init, (size_t)n, op, s);
}

}  // namespace hnv

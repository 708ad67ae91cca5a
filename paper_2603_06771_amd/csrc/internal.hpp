// Internal (C++) launch helpers shared between translation units of the
// library.  Not part of the C ABI.
#pragma once

#include "common.hpp"

namespace sfc {

// ---- frame + codes (encode.hip)
// bbox_ws: 8 ints of device scratch
int launch_frame(const float *xyz, int64_t n, int curve, int bits, sfc_frame *frame, int *bbox_ws,
                 hipStream_t s);
// keys[i] = code of point i; if iota != nullptr also iota[i] = i
int launch_encode(const float *xyz, int64_t n, const sfc_frame *frame, uint64_t *keys, uint32_t *iota,
                  hipStream_t s);

// ---- device-wide exclusive scan (scan.hip)
size_t scan_ws_bytes(int64_t n);
// out[i] = sum_{j<i} in[j]; if write_total, out[n] = sum of all
int scan_u32_to_u32(const uint32_t *in, int64_t n, uint32_t *out, bool write_total, void *ws, hipStream_t s);
int scan_u32_to_u64(const uint32_t *in, int64_t n, uint64_t *out, bool write_total, void *ws, hipStream_t s);

// ---- LSD radix sort of (u64 key, u32 value) pairs (sort.hip), stable.
size_t radix_ws_bytes(int64_t n);
// Sorts on bits [0, key_bits).  Data ping-pongs between (keys, vals) and
// (keys_alt, vals_alt); *in_alt tells where the result ended up.
// If n_dev is not null the element count is read from the device and the
// host n is only an upper bound used to size the grids.  With seg_start
// (nseg + 1 ascending starts, nseg > 1) further passes order the pairs stably
// by the segment holding each value.
int radix_sort_pairs(uint64_t *keys, uint32_t *vals, uint64_t *keys_alt, uint32_t *vals_alt, int64_t n,
                     const int64_t *n_dev, int key_bits, void *ws, hipStream_t s, bool *in_alt,
                     const int64_t *seg_start = nullptr, int nseg = 0);

// ---- octree build (build.hip)
int64_t internal_upper_bound(int64_t n, uint32_t leaf_size, int bits);
size_t tree_layout(int64_t n, uint32_t leaf_size, int bits, void *mem, sfc_octree *t);
// one layout for a batch: shared point arrays, then every cloud's tree arrays;
// fills clouds[c].tree when mem is not null
size_t batch_layout(int B, sfc_cloud *clouds, void *mem);
// copies a host cloud table into device memory on stream s (kernel arguments,
// so no host buffer has to outlive the call)
int upload_clouds(const sfc_cloud *host, int B, sfc_cloud *dev, hipStream_t s);

}  // namespace sfc

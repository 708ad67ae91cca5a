// Section 4, reorder step 2: stable LSD radix sort of (63-bit code, index)
// pairs, 8-bit digits.  Since the input values are the original indices in
// ascending order and every pass is stable, equal codes end up ordered by
// original index.
//
// Per pass:
//   k_radix_hist    : digit histogram of each 4096-key tile (LDS atomics),
//                     stored digit-major: hist[d * tiles + tile]
//   scan            : exclusive scan of hist -> first output slot of every
//                     (digit, tile)
//   k_radix_scatter : each wave ranks its keys inside 64-key chunks with a
//                     match-by-ballot over the 8 digit bits, per-wave digit
//                     counters in LDS give the stable rank inside the tile,
//                     and each key goes to slot + rank.
// Batches: after the code passes, optional passes keyed by the segment (cloud)
// of each value, found by binary search of the value in the segment starts,
// leave every segment contiguous and internally ordered by (code, index).
// Roofline: per pass 8 B (hist) + 12 B in + 12 B out per key, HBM bound.
#include "internal.hpp"

namespace sfc {

namespace {
constexpr int kRadixBlock = 256;
constexpr int kRadixWaves = kRadixBlock / kWave;
constexpr int kRadixItems = 16;                      // chunks of 64 keys per wave
constexpr int kRadixTile = kRadixBlock * kRadixItems; // 4096 keys

// digit of a (key, value) pair: bits [shift, shift + 8) of the key, or of the
// segment index of the value (last c < nseg with seg[c] <= value)
template <bool kSeg>
__device__ __forceinline__ uint32_t digit_of(uint64_t key, uint32_t val, int shift, const int64_t *seg, int nseg) {
    if (!kSeg) return static_cast<uint32_t>(key >> shift) & 0xFFu;
    int lo = 0, hi = nseg - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (seg[mid] <= static_cast<int64_t>(val))
            lo = mid;
        else
            hi = mid - 1;
    }
    return static_cast<uint32_t>(lo >> shift) & 0xFFu;
}
}  // namespace

template <bool kSeg>
__global__ __launch_bounds__(kRadixBlock) void k_radix_hist(const uint64_t *__restrict__ keys,
                                                            const uint32_t *__restrict__ vals, int64_t n,
                                                            const int64_t *__restrict__ n_dev, int shift,
                                                            const int64_t *__restrict__ seg, int nseg,
                                                            uint32_t *__restrict__ hist, int64_t tiles) {
    __shared__ uint32_t s_cnt[256];
    if (n_dev) n = *n_dev;
    s_cnt[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = static_cast<int64_t>(blockIdx.x) * kRadixTile;
#pragma unroll 4
    for (int i = 0; i < kRadixItems; ++i) {
        const int64_t j = base + static_cast<int64_t>(i) * kRadixBlock + threadIdx.x;
        if (j < n) atomicAdd(&s_cnt[digit_of<kSeg>(kSeg ? 0ull : keys[j], kSeg ? vals[j] : 0u, shift, seg, nseg)], 1u);
    }
    __syncthreads();
    hist[static_cast<int64_t>(threadIdx.x) * tiles + blockIdx.x] = s_cnt[threadIdx.x];
}

template <bool kSeg>
__global__ __launch_bounds__(kRadixBlock) void k_radix_scatter(const uint64_t *__restrict__ kin,
                                                               const uint32_t *__restrict__ vin,
                                                               uint64_t *__restrict__ kout,
                                                               uint32_t *__restrict__ vout, int64_t n,
                                                               const int64_t *__restrict__ n_dev, int shift,
                                                               const int64_t *__restrict__ seg, int nseg,
                                                               const uint32_t *__restrict__ offs, int64_t tiles) {
    __shared__ uint32_t s_wcnt[kRadixWaves][256];
    if (n_dev) n = *n_dev;
    if (static_cast<int64_t>(blockIdx.x) * kRadixTile >= n) return;
    __shared__ uint32_t s_goff[256];
    const int lane = lane_id(), wave = threadIdx.x / kWave;
    for (int w = 0; w < kRadixWaves; ++w) s_wcnt[w][threadIdx.x] = 0;
    s_goff[threadIdx.x] = offs[static_cast<int64_t>(threadIdx.x) * tiles + blockIdx.x];
    __syncthreads();

    const int64_t base = static_cast<int64_t>(blockIdx.x) * kRadixTile + static_cast<int64_t>(wave) * (kRadixItems * kWave);
    uint64_t key[kRadixItems];
    uint32_t val[kRadixItems];
    uint32_t rank[kRadixItems];
    uint32_t dig[kRadixItems];
#pragma unroll
    for (int c = 0; c < kRadixItems; ++c) {
        const int64_t j = base + c * kWave + lane;
        const bool valid = j < n;
        key[c] = valid ? kin[j] : 0ull;
        val[c] = valid ? vin[j] : 0u;
        const uint32_t d = digit_of<kSeg>(key[c], val[c], shift, seg, nseg);
        dig[c] = d;
        uint64_t peers = ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const bool bit = (d >> b) & 1u;
            const uint64_t m = ballot(bit);
            peers &= bit ? m : ~m;
        }
        const uint32_t before = rank_below(peers);
        const uint32_t old = s_wcnt[wave][d];
        rank[c] = old + before;
        // the lowest lane of each digit group advances the counter after the
        // whole wave has read it
        __builtin_amdgcn_wave_barrier();
        if (valid && before == 0) s_wcnt[wave][d] = old + static_cast<uint32_t>(__popcll(peers));
        __builtin_amdgcn_wave_barrier();
    }
    __syncthreads();
    // exclusive prefix of the per-wave counts, per digit
    {
        uint32_t run = 0;
        for (int w = 0; w < kRadixWaves; ++w) {
            const uint32_t t = s_wcnt[w][threadIdx.x];
            s_wcnt[w][threadIdx.x] = run;
            run += t;
        }
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < kRadixItems; ++c) {
        const int64_t j = base + c * kWave + lane;
        if (j < n) {
            const uint32_t d = dig[c];
            const int64_t pos = static_cast<int64_t>(s_goff[d]) + s_wcnt[wave][d] + rank[c];
            kout[pos] = key[c];
            vout[pos] = val[c];
        }
    }
}

size_t radix_ws_bytes(int64_t n) {
    const int64_t tiles = n > 0 ? (n + kRadixTile - 1) / kRadixTile : 1;
    const int64_t h = 256 * tiles;
    Carver c(nullptr);
    c.take<uint32_t>(h);      // hist
    c.take<uint32_t>(h + 1);  // offsets
    c.take<char>(scan_ws_bytes(h));
    return c.bytes();
}

int radix_sort_pairs(uint64_t *keys, uint32_t *vals, uint64_t *keys_alt, uint32_t *vals_alt, int64_t n,
                     const int64_t *n_dev, int key_bits, void *ws, hipStream_t s, bool *in_alt,
                     const int64_t *seg_start, int nseg) {
    *in_alt = false;
    if (n <= 1 && !n_dev) return SFC_OK;
    if (n < 1) n = 1;
    const int64_t tiles = (n + kRadixTile - 1) / kRadixTile;
    const int64_t h = 256 * tiles;
    Carver c(ws);
    uint32_t *hist = c.take<uint32_t>(h);
    uint32_t *offs = c.take<uint32_t>(h + 1);
    void *scan_ws = c.take<char>(scan_ws_bytes(h));
    uint64_t *ki = keys, *ko = keys_alt;
    uint32_t *vi = vals, *vo = vals_alt;
    int seg_bits = 0;
    if (seg_start && nseg > 1)
        while ((int64_t(1) << seg_bits) < nseg) seg_bits += 8;
    const int kb = (key_bits + 7) / 8 * 8;  // bits covered by the code passes
    for (int shift = 0; shift < kb + seg_bits; shift += 8) {
        const bool by_seg = shift >= kb;
        const int sh = by_seg ? shift - kb : shift;
        const unsigned g = static_cast<unsigned>(tiles);
        if (by_seg)
            k_radix_hist<true><<<g, kRadixBlock, 0, s>>>(ki, vi, n, n_dev, sh, seg_start, nseg, hist, tiles);
        else
            k_radix_hist<false><<<g, kRadixBlock, 0, s>>>(ki, vi, n, n_dev, sh, nullptr, 0, hist, tiles);
        SFC_LAUNCH_CHECK("k_radix_hist");
        int rc = scan_u32_to_u32(hist, h, offs, false, scan_ws, s);
        if (rc) return rc;
        if (by_seg)
            k_radix_scatter<true><<<g, kRadixBlock, 0, s>>>(ki, vi, ko, vo, n, n_dev, sh, seg_start, nseg, offs, tiles);
        else
            k_radix_scatter<false><<<g, kRadixBlock, 0, s>>>(ki, vi, ko, vo, n, n_dev, sh, nullptr, 0, offs, tiles);
        SFC_LAUNCH_CHECK("k_radix_scatter");
        uint64_t *tk = ki;
        ki = ko;
        ko = tk;
        uint32_t *tv = vi;
        vi = vo;
        vo = tv;
        *in_alt = !*in_alt;
    }
    return SFC_OK;
}

}  // namespace sfc

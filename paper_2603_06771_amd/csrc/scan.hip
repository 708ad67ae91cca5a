// Device-wide exclusive prefix sum of uint32 counts (reduce-then-scan, each
// count read twice and each offset written once):
//   k_scan_reduce : each block sums a tile of kScanTile counts
//   k_scan_sums   : one block scans the tile totals (exclusive, grand total last)
//   k_scan_down   : each block scans its tile again, from its tile's offset,
//                   and writes the offsets; the grand total goes to out[n]
// Used for CSR row offsets, radix-sort digit offsets and node emission.  The
// input and output may be the same array (every item is read before the
// thread that reads it writes it).
#include "internal.hpp"

namespace sfc {

namespace {
constexpr int kScanBlock = 256;
constexpr int kScanItems = 16;
constexpr int kScanTile = kScanBlock * kScanItems;

template <typename T>
__device__ T block_exclusive_sum(T v, T *s_wave, T *total) {
    const int lane = lane_id(), wave = threadIdx.x / kWave;
    const T incl = wave_inclusive_sum(v);
    if (lane == kWave - 1) s_wave[wave] = incl;
    __syncthreads();
    T wave_off = 0, all = 0;
    for (int w = 0; w < kScanBlock / kWave; ++w) {
        const T t = s_wave[w];
        if (w < wave) wave_off += t;
        all += t;
    }
    __syncthreads();
    *total = all;
    return wave_off + incl - v;
}

// thread t of a block holds items [base + t * kScanItems, ... + kScanItems)
__device__ __forceinline__ int64_t item_base(int64_t block) {
    return block * kScanTile + static_cast<int64_t>(threadIdx.x) * kScanItems;
}
}  // namespace

template <typename T>
__global__ __launch_bounds__(kScanBlock) void k_scan_reduce(const uint32_t *__restrict__ in, int64_t n,
                                                            T *__restrict__ sums) {
    __shared__ T s_wave[kScanBlock / kWave];
    const int64_t base = item_base(blockIdx.x);
    T thread_sum = 0;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) thread_sum += (base + i < n) ? static_cast<T>(in[base + i]) : T(0);
    T total;
    block_exclusive_sum<T>(thread_sum, s_wave, &total);
    if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

template <typename T>
__global__ __launch_bounds__(kScanBlock) void k_scan_sums(T *sums, int64_t nb) {
    __shared__ T s_wave[kScanBlock / kWave];
    T carry = 0;
    for (int64_t base = 0; base < nb; base += kScanBlock) {
        const int64_t i = base + threadIdx.x;
        const T v = i < nb ? sums[i] : T(0);
        T total;
        const T ex = block_exclusive_sum<T>(v, s_wave, &total);
        if (i < nb) sums[i] = carry + ex;
        carry += total;
    }
    if (threadIdx.x == 0) sums[nb] = carry;
}

template <typename T>
__global__ __launch_bounds__(kScanBlock) void k_scan_down(const uint32_t *in, int64_t n, T *out,
                                                          const T *__restrict__ sums, int64_t nb, int write_total) {
    __shared__ T s_wave[kScanBlock / kWave];
    const int64_t base = item_base(blockIdx.x);
    T v[kScanItems];
    T thread_sum = 0;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        v[i] = (base + i < n) ? static_cast<T>(in[base + i]) : T(0);
        thread_sum += v[i];
    }
    T total;
    T run = sums[blockIdx.x] + block_exclusive_sum<T>(thread_sum, s_wave, &total);
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        if (base + i < n) out[base + i] = run;
        run += v[i];
    }
    if (write_total && blockIdx.x == 0 && threadIdx.x == 0) out[n] = sums[nb];
}

size_t scan_ws_bytes(int64_t n) {
    const int64_t nb = (n + kScanTile - 1) / kScanTile + 1;
    return align_up(static_cast<size_t>(nb + 1) * sizeof(uint64_t), 256);
}

template <typename T>
static int scan_impl(const uint32_t *in, int64_t n, T *out, bool write_total, void *ws, hipStream_t s) {
    const int64_t nb = n > 0 ? (n + kScanTile - 1) / kScanTile : 0;
    T *sums = static_cast<T *>(ws);
    if (nb > 0) {
        k_scan_reduce<T><<<static_cast<unsigned>(nb), kScanBlock, 0, s>>>(in, n, sums);
        SFC_LAUNCH_CHECK("k_scan_reduce");
    }
    k_scan_sums<T><<<1, kScanBlock, 0, s>>>(sums, nb);
    SFC_LAUNCH_CHECK("k_scan_sums");
    k_scan_down<T><<<static_cast<unsigned>(nb > 0 ? nb : 1), kScanBlock, 0, s>>>(in, n, out, sums, nb,
                                                                                   write_total ? 1 : 0);
    SFC_LAUNCH_CHECK("k_scan_down");
    return SFC_OK;
}

int scan_u32_to_u32(const uint32_t *in, int64_t n, uint32_t *out, bool write_total, void *ws, hipStream_t s) {
    return scan_impl<uint32_t>(in, n, out, write_total, ws, s);
}
int scan_u32_to_u64(const uint32_t *in, int64_t n, uint64_t *out, bool write_total, void *ws, hipStream_t s) {
    return scan_impl<uint64_t>(in, n, out, write_total, ws, s);
}

}  // namespace sfc

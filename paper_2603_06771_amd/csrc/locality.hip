// Section 5.2: the kNN locality histogram of a stored order, and its
// moments, skewness and quartiles.
//
//   k_inverse_perm   : pos[perm[i]] = i (stored position of every point)
//   k_locality_count : one thread per (query, neighbour) pair, d = |row - pos|;
//                      d below kLocalBins is counted in an LDS histogram per
//                      block (the small distances are the hot bins), larger d
//                      with a global atomic
//   k_moments_*      : fp64 sums over the bins in a fixed order (per-thread
//                      runs, fixed-shape wave and block reductions, block
//                      partials summed by one thread), so the statistics are
//                      the same bits on every run
//   quartiles        : exclusive scan of the histogram, then a binary search
// Roofline: the counting pass reads 4 B (index) + a 4-B gather per pair and
// is bound by the histogram atomics; the moment passes stream 4 B per bin.
#include <cmath>

#include "internal.hpp"

namespace sfc {

namespace {

constexpr int kLocalBins = 2048;
constexpr int kMomBlock = 256;
constexpr int kMomPerThread = 16;
constexpr int64_t kMomTile = static_cast<int64_t>(kMomBlock) * kMomPerThread;

__device__ __forceinline__ double block_sum_f64(double v, double *red) {
    for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o);
    const int w = threadIdx.x / kWave;
    __syncthreads();
    if (lane_id() == 0) red[w] = v;
    __syncthreads();
    double t = 0.0;
    for (int i = 0; i < kMomBlock / kWave; ++i) t += red[i];
    return t;
}

}  // namespace

__global__ __launch_bounds__(256) void k_inverse_perm(const uint32_t *__restrict__ perm, int64_t n,
                                                      uint32_t *__restrict__ pos) {
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride)
        pos[perm[i]] = static_cast<uint32_t>(i);
}

__global__ __launch_bounds__(256) void k_fill_zero(uint32_t *__restrict__ a, int64_t n) {
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride) a[i] = 0u;
}

__global__ __launch_bounds__(256) void k_locality_count(const uint32_t *__restrict__ rows, int64_t nq,
                                                        const uint32_t *__restrict__ idx, int k, int kstride,
                                                        const uint32_t *__restrict__ pos, int64_t n,
                                                        uint32_t *__restrict__ hist) {
    __shared__ uint32_t s_h[kLocalBins];
    for (int i = threadIdx.x; i < kLocalBins; i += blockDim.x) s_h[i] = 0u;
    __syncthreads();
    const int64_t pairs = nq * k;
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    for (int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; e < pairs; e += stride) {
        const int64_t r = e / k;
        const int t = static_cast<int>(e - r * k);
        const uint32_t j = idx[r * kstride + t];
        if (j >= n) continue;  // padding (k beyond the cloud)
        const int64_t i = rows ? static_cast<int64_t>(rows[r]) : r;
        if (i >= n) continue;  // not a stored position
        const int64_t pj = pos[j];
        const int64_t d = i > pj ? i - pj : pj - i;
        if (d < kLocalBins)
            atomicAdd(&s_h[d], 1u);
        else
            atomicAdd(&hist[d], 1u);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < kLocalBins && i < n; i += blockDim.x)
        if (s_h[i]) atomicAdd(&hist[i], s_h[i]);
}

// pass 1: per block, the total and the sum of d over its bins
__global__ __launch_bounds__(kMomBlock) void k_moments_1(const uint32_t *__restrict__ hist, int64_t n,
                                                         double *__restrict__ part) {
    __shared__ double red[kMomBlock / kWave];
    const int64_t b0 = static_cast<int64_t>(blockIdx.x) * kMomTile + static_cast<int64_t>(threadIdx.x) * kMomPerThread;
    double c = 0.0, s = 0.0;
    for (int t = 0; t < kMomPerThread; ++t) {
        const int64_t d = b0 + t;
        if (d < n) {
            const double h = static_cast<double>(hist[d]);
            c += h;
            s += h * static_cast<double>(d);
        }
    }
    c = block_sum_f64(c, red);
    s = block_sum_f64(s, red);
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = c;
        part[2 * blockIdx.x + 1] = s;
    }
}

__global__ void k_moments_mean(const double *__restrict__ part, int64_t nb, double *__restrict__ stats) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double c = 0.0, s = 0.0;
    for (int64_t b = 0; b < nb; ++b) {
        c += part[2 * b];
        s += part[2 * b + 1];
    }
    stats[0] = c;
    stats[1] = c > 0.0 ? s / c : 0.0;
}

// pass 2: second and third central moments about the mean
__global__ __launch_bounds__(kMomBlock) void k_moments_2(const uint32_t *__restrict__ hist, int64_t n,
                                                         const double *__restrict__ stats, double *__restrict__ part) {
    __shared__ double red[kMomBlock / kWave];
    const double mean = stats[1];
    const int64_t b0 = static_cast<int64_t>(blockIdx.x) * kMomTile + static_cast<int64_t>(threadIdx.x) * kMomPerThread;
    double m2 = 0.0, m3 = 0.0;
    for (int t = 0; t < kMomPerThread; ++t) {
        const int64_t d = b0 + t;
        if (d < n) {
            const double h = static_cast<double>(hist[d]);
            const double x = static_cast<double>(d) - mean;
            m2 += h * (x * x);
            m3 += h * (x * x * x);
        }
    }
    m2 = block_sum_f64(m2, red);
    m3 = block_sum_f64(m3, red);
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = m2;
        part[2 * blockIdx.x + 1] = m3;
    }
}

// standard deviation, skewness, quartiles and largest d from the exclusive
// prefix sums off[d] = sum of hist below d (off[n] = total)
__global__ void k_moments_final(const double *__restrict__ part, int64_t nb, const uint64_t *__restrict__ off,
                                int64_t n, double *__restrict__ stats) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double m2 = 0.0, m3 = 0.0;
    for (int64_t b = 0; b < nb; ++b) {
        m2 += part[2 * b];
        m3 += part[2 * b + 1];
    }
    const double c = stats[0];
    double sd = 0.0, g1 = 0.0;
    if (c > 0.0) {
        sd = sqrt(m2 / c);
        if (sd > 0.0) g1 = (m3 / c) / (sd * sd * sd);
    }
    stats[2] = sd;
    stats[3] = g1;
    const uint64_t total = off[n];
    // smallest d with off[d + 1] >= target
    for (int q = 1; q <= 4; ++q) {
        const uint64_t target = q < 4 ? (q * total + 3) / 4 : total;
        int64_t lo = 0, hi = n > 0 ? n - 1 : 0;
        while (lo < hi) {
            const int64_t mid = (lo + hi) >> 1;
            if (off[mid + 1] >= target)
                hi = mid;
            else
                lo = mid + 1;
        }
        stats[3 + q] = total > 0 ? static_cast<double>(lo) : 0.0;
    }
}

namespace {

struct LocalityWs {
    uint32_t *pos;
    double *part;
    uint64_t *off;
    void *scan;
};

size_t carve_locality_ws(int64_t n, void *mem, LocalityWs *w) {
    const int64_t nb = (n + kMomTile - 1) / kMomTile + 1;
    Carver c(mem);
    LocalityWs x;
    x.pos = c.take<uint32_t>(n > 0 ? n : 1);
    x.part = c.take<double>(2 * nb);
    x.off = c.take<uint64_t>(n + 1);
    x.scan = c.take<char>(scan_ws_bytes(n));
    if (w) *w = x;
    return c.bytes();
}

}  // namespace

}  // namespace sfc

extern "C" int knn_locality(const sfc_octree *tree, const uint32_t *rows, int64_t nq, const uint32_t *idx, int k,
                            int kstride, uint32_t *hist, double *stats, void *ws, size_t *ws_bytes, void *stream) {
    using namespace sfc;
    if (!ws_bytes || !tree || !tree->perm || tree->n < 1 || nq < 0 || k < 1 || kstride < k || !hist || !stats ||
        (nq > 0 && !idx) || (!rows && nq > tree->n)) {
        set_error("knn_locality: invalid argument");
        return SFC_EINVAL;
    }
    if (nq * static_cast<int64_t>(k) > 0xFFFFFFFFll) {
        set_error("knn_locality: more than 2^32 - 1 pairs");
        return SFC_ENOTSUP;
    }
    const int64_t n = tree->n;
    const size_t need = carve_locality_ws(n, nullptr, nullptr);
    if (!ws) {
        *ws_bytes = need;
        return SFC_OK;
    }
    if (*ws_bytes < need || (reinterpret_cast<uintptr_t>(ws) & 255u)) {
        set_error("knn_locality: workspace needs %zu bytes, 256-aligned", need);
        return SFC_EWORKSPACE;
    }
    LocalityWs w;
    carve_locality_ws(n, ws, &w);
    hipStream_t s = static_cast<hipStream_t>(stream);
    k_inverse_perm<<<grid_for(n, 256, 8192), 256, 0, s>>>(tree->perm, n, w.pos);
    SFC_LAUNCH_CHECK("k_inverse_perm");
    k_fill_zero<<<grid_for(n, 256, 8192), 256, 0, s>>>(hist, n);
    SFC_LAUNCH_CHECK("k_fill_zero");
    if (nq > 0) {
        k_locality_count<<<grid_for(nq * k, 256, 4096), 256, 0, s>>>(rows, nq, idx, k, kstride, w.pos, n, hist);
        SFC_LAUNCH_CHECK("k_locality_count");
    }
    const int64_t nb = (n + kMomTile - 1) / kMomTile;
    k_moments_1<<<static_cast<unsigned>(nb), kMomBlock, 0, s>>>(hist, n, w.part);
    SFC_LAUNCH_CHECK("k_moments_1");
    k_moments_mean<<<1, 64, 0, s>>>(w.part, nb, stats);
    SFC_LAUNCH_CHECK("k_moments_mean");
    k_moments_2<<<static_cast<unsigned>(nb), kMomBlock, 0, s>>>(hist, n, stats, w.part);
    SFC_LAUNCH_CHECK("k_moments_2");
    const int rc = scan_u32_to_u64(hist, n, w.off, true, w.scan, s);
    if (rc) return rc;
    k_moments_final<<<1, 64, 0, s>>>(w.part, nb, w.off, n, stats);
    SFC_LAUNCH_CHECK("k_moments_final");
    return SFC_OK;
}

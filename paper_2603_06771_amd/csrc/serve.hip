// Serving helper: assembles query batches from point ids (a request names
// points of a resident cloud).  One thread per query point; reads are
// gathers from the cloud, writes are coalesced.
#include "internal.hpp"

namespace sfc {

__global__ __launch_bounds__(256) void k_gather_points(const float *__restrict__ xyz, int64_t n_points,
                                                       const uint32_t *__restrict__ rows, int64_t n,
                                                       float *__restrict__ out) {
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride) {
        const int64_t r = rows[i];
        float x = __uint_as_float(0x7FC00000u), y = x, z = x;
        if (r < n_points) {
            x = xyz[3 * r];
            y = xyz[3 * r + 1];
            z = xyz[3 * r + 2];
        }
        out[3 * i] = x;
        out[3 * i + 1] = y;
        out[3 * i + 2] = z;
    }
}

}  // namespace sfc

extern "C" int gather_points(const float *xyz, int64_t n_points, const uint32_t *rows, int64_t n, float *out,
                             void *stream) {
    using namespace sfc;
    if (n < 0 || n_points < 0 || (n > 0 && (!rows || !out || (n_points > 0 && !xyz)))) {
        set_error("gather_points: invalid argument");
        return SFC_EINVAL;
    }
    if (n == 0) return SFC_OK;
    k_gather_points<<<grid_for(n, 256, 1 << 14), 256, 0, static_cast<hipStream_t>(stream)>>>(xyz, n_points, rows, n,
                                                                                            out);
    SFC_LAUNCH_CHECK("k_gather_points");
    return SFC_OK;
}

// Section 4, steps 1-2 and reorder step 1: frame of the cloud and the code of
// every point.
//
//   k_bbox_init / k_bbox : exact per-axis min and max (order-free, so any
//                          reduction tree gives the same bits); one wave
//                          reduction per wave, one integer atomic per wave
//   k_frame              : E = largest fp32 side, scale = 2^L / E (one thread,
//                          correctly rounded division)
//   k_encode             : cells and Morton / Hilbert code per point
//
// Roofline: k_encode streams 12 B in and 8 B out per point (HBM bound);
// k_bbox reads 12 B per point.
#include <cstdarg>
#include <cstdio>

#include "codes.hpp"
#include "internal.hpp"

namespace sfc {

__global__ void k_bbox_init(int *bb) {
    if (threadIdx.x < 3) {
        bb[threadIdx.x] = ordered_int(INFINITY);
        bb[3 + threadIdx.x] = ordered_int(-INFINITY);
    }
}

__global__ __launch_bounds__(256) void k_bbox(const float *__restrict__ xyz, int64_t n, int *bb) {
    float mn[3] = {INFINITY, INFINITY, INFINITY};
    float mx[3] = {-INFINITY, -INFINITY, -INFINITY};
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride) {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const float v = xyz[3 * i + a];
            mn[a] = fminf(mn[a], v);
            mx[a] = fmaxf(mx[a], v);
        }
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        mn[a] = wave_min(mn[a]);
        mx[a] = wave_max(mx[a]);
    }
    if (lane_id() == 0) {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            atomicMin(bb + a, ordered_int(mn[a]));
            atomicMax(bb + 3 + a, ordered_int(mx[a]));
        }
    }
}

__global__ void k_frame(const int *bb, int64_t n, int curve, int bits, sfc_frame *frame) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    float lo[3], E = 0.0f;
    for (int a = 0; a < 3; ++a) {
        lo[a] = ordered_float(bb[a]);
        const float hi = ordered_float(bb[3 + a]);
        if (n > 0) {
            const float side = fsub(hi, lo[a]);
            if (side > E) E = side;
        }
    }
    if (n == 0) lo[0] = lo[1] = lo[2] = 0.0f;
    if (!(E > 0.0f)) E = 1.0f;
    sfc_frame f;
    f.lo[0] = lo[0];
    f.lo[1] = lo[1];
    f.lo[2] = lo[2];
    f.scale = __fdiv_rn(static_cast<float>(1u << bits), E);
    f.bits = bits;
    f.curve = curve;
    *frame = f;
}

__global__ __launch_bounds__(256) void k_encode(const float *__restrict__ xyz, int64_t n,
                                                const sfc_frame *__restrict__ frame,
                                                uint64_t *__restrict__ keys, uint32_t *__restrict__ iota) {
    const sfc_frame f = *frame;
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride) {
        keys[i] = point_key(xyz[3 * i], xyz[3 * i + 1], xyz[3 * i + 2], f);
        if (iota) iota[i] = static_cast<uint32_t>(i);
    }
}

int launch_frame(const float *xyz, int64_t n, int curve, int bits, sfc_frame *frame, int *bb,
                 hipStream_t s) {
    k_bbox_init<<<1, 64, 0, s>>>(bb);
    SFC_LAUNCH_CHECK("k_bbox_init");
    if (n > 0) {
        k_bbox<<<grid_for(n, 256, 2048), 256, 0, s>>>(xyz, n, bb);
        SFC_LAUNCH_CHECK("k_bbox");
    }
    k_frame<<<1, 64, 0, s>>>(bb, n, curve, bits, frame);
    SFC_LAUNCH_CHECK("k_frame");
    return SFC_OK;
}

int launch_encode(const float *xyz, int64_t n, const sfc_frame *frame, uint64_t *keys, uint32_t *iota,
                  hipStream_t s) {
    if (n == 0) return SFC_OK;
    k_encode<<<grid_for(n, 256, 1 << 16), 256, 0, s>>>(xyz, n, frame, keys, iota);
    SFC_LAUNCH_CHECK("k_encode");
    return SFC_OK;
}

// ------------------------------------------------------------ error state
static thread_local char g_err[512] = "";

void set_error(const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
}

int hip_fail(hipError_t e, const char *what) {
    set_error("%s: %s", what, hipGetErrorString(e));
    return SFC_EHIP;
}

}  // namespace sfc

extern "C" const char *sfc_last_error(void) { return sfc::g_err; }

extern "C" const char *sfc_version(void) { return "sfcoct 0.1 gfx950"; }

extern "C" int encode_sfc(const float *xyz, int64_t n, int curve, int bits, sfc_frame *frame, uint64_t *keys,
                          void *ws, size_t *ws_bytes, void *stream) {
    using namespace sfc;
    if (!ws_bytes) {
        set_error("encode_sfc: ws_bytes is NULL");
        return SFC_EINVAL;
    }
    const size_t need = 256;
    if (!ws) {
        *ws_bytes = need;
        return SFC_OK;
    }
    if (*ws_bytes < need || (reinterpret_cast<uintptr_t>(ws) & 255u)) {
        set_error("encode_sfc: workspace needs %zu bytes, 256-aligned", need);
        return SFC_EWORKSPACE;
    }
    if (n < 0 || n > 0xFFFFFFFFll || (n > 0 && (!xyz || !keys)) || !frame || bits < 1 || bits > 21 ||
        (curve != SFC_MORTON && curve != SFC_HILBERT)) {
        set_error("encode_sfc: invalid argument (n=%lld bits=%d curve=%d)", (long long)n, bits, curve);
        return SFC_EINVAL;
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    int rc = launch_frame(xyz, n, curve, bits, frame, static_cast<int *>(ws), s);
    if (rc) return rc;
    return launch_encode(xyz, n, frame, keys, nullptr, s);
}

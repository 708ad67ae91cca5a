// Shared device/host helpers of the gfx950 library (wave64 primitives, fp32
// operations with explicit rounding, launch checks).  Device code is built
// with -ffp-contract=off and the *_rn intrinsics below, so every fp32
// expression is evaluated exactly as written.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/sfcoct.h"

namespace sfc {

constexpr int kWave = 64;

// ---------------------------------------------------------------- host side
void set_error(const char *fmt, ...);
int hip_fail(hipError_t e, const char *what);

#define SFC_LAUNCH_CHECK(what)                                       \
    do {                                                             \
        hipError_t _e = hipGetLastError();                           \
        if (_e != hipSuccess) return ::sfc::hip_fail(_e, what);      \
    } while (0)

#define SFC_HIP_TRY(call)                                            \
    do {                                                             \
        hipError_t _e = (call);                                      \
        if (_e != hipSuccess) return ::sfc::hip_fail(_e, #call);     \
    } while (0)

inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Sequential carving of one caller buffer into aligned sub-arrays.
struct Carver {
    char *base;
    size_t off = 0;
    explicit Carver(void *b) : base(static_cast<char *>(b)) {}
    template <typename T>
    T *take(size_t count) {
        off = align_up(off, 256);
        T *p = base ? reinterpret_cast<T *>(base + off) : nullptr;
        off += count * sizeof(T);
        return p;
    }
    size_t bytes() const { return align_up(off, 256); }
};

inline int grid_for(int64_t n, int block, int cap = 1 << 20) {
    int64_t g = (n + block - 1) / block;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return static_cast<int>(g);
}

// -------------------------------------------------------------- device side
__device__ __forceinline__ int lane_id() { return __lane_id(); }

// the lane mask of p (the builtin on the i1 value: no round trip through a
// vector register)
__device__ __forceinline__ uint64_t ballot(bool p) { return __builtin_amdgcn_ballot_w64(p); }

// Orders the LDS accesses of a workgroup made of a single wave: LDS writes of
// any lane before the call are seen by LDS reads of every lane after it.  A
// wave's LDS instructions execute in issue order, so no wait instruction is
// needed; the wavefront-scope fences keep the compiler from moving memory
// accesses across the call.  Unlike a workgroup barrier, it does not wait for
// the wave's outstanding global stores.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// number of set bits of m below this lane
__device__ __forceinline__ uint32_t rank_below(uint64_t m) {
    return __builtin_amdgcn_mbcnt_hi(static_cast<uint32_t>(m >> 32),
                                     __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(m), 0u));
}

__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

// readlane of unsigned values (the builtin returns int: widen through uint32_t,
// never through int, or the value is sign-extended)
__device__ __forceinline__ uint32_t readlane_u32(uint32_t v, int l) {
    return static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(v), l));
}
__device__ __forceinline__ uint64_t readlane_u64(uint64_t v, int l) {
    return (static_cast<uint64_t>(readlane_u32(static_cast<uint32_t>(v >> 32), l)) << 32) |
           static_cast<uint64_t>(readlane_u32(static_cast<uint32_t>(v), l));
}

// v_writelane: lane l (wave-uniform) of `old` takes the wave-uniform value v,
// the other lanes keep theirs.  The compiler has the intrinsic but no builtin
// for it, so it is bound by its LLVM name (the compiler still schedules it
// and resolves its hazards; no inline assembly).
__device__ int sfc_llvm_writelane_i32(int v, int l, int old) __asm("llvm.amdgcn.writelane.i32");
__device__ __forceinline__ uint32_t writelane_u32(uint32_t v, int l, uint32_t old) {
    return static_cast<uint32_t>(sfc_llvm_writelane_i32(static_cast<int>(v), l, static_cast<int>(old)));
}

__device__ __forceinline__ float wave_min(float v) {
    for (int o = 32; o > 0; o >>= 1) v = fminf(v, __shfl_xor(v, o));
    return v;
}
__device__ __forceinline__ float wave_max(float v) {
    for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o));
    return v;
}

// Wave-uniform min / max / sum without LDS: DPP exchanges inside rows of 16
// lanes (quad permutes, row rotations), then the four row results are read
// with readlane.  Every lane of the wave must be active.
template <int CTRL>
__device__ __forceinline__ int dpp_i(int v) {
    return __builtin_amdgcn_update_dpp(v, v, CTRL, 0xF, 0xF, false);
}
template <int CTRL>
__device__ __forceinline__ float dpp_f(float v) {
    return __int_as_float(dpp_i<CTRL>(__float_as_int(v)));
}
__device__ __forceinline__ float wave_min_u(float v) {
    v = fminf(v, dpp_f<0xB1>(v));   // quad_perm [1,0,3,2]
    v = fminf(v, dpp_f<0x4E>(v));   // quad_perm [2,3,0,1]
    v = fminf(v, dpp_f<0x124>(v));  // row_ror:4
    v = fminf(v, dpp_f<0x128>(v));  // row_ror:8
    const int x = __float_as_int(v);
    return fminf(fminf(__int_as_float(__builtin_amdgcn_readlane(x, 0)), __int_as_float(__builtin_amdgcn_readlane(x, 16))),
                 fminf(__int_as_float(__builtin_amdgcn_readlane(x, 32)), __int_as_float(__builtin_amdgcn_readlane(x, 48))));
}
__device__ __forceinline__ float wave_max_u(float v) {
    v = fmaxf(v, dpp_f<0xB1>(v));
    v = fmaxf(v, dpp_f<0x4E>(v));
    v = fmaxf(v, dpp_f<0x124>(v));
    v = fmaxf(v, dpp_f<0x128>(v));
    const int x = __float_as_int(v);
    return fmaxf(fmaxf(__int_as_float(__builtin_amdgcn_readlane(x, 0)), __int_as_float(__builtin_amdgcn_readlane(x, 16))),
                 fmaxf(__int_as_float(__builtin_amdgcn_readlane(x, 32)), __int_as_float(__builtin_amdgcn_readlane(x, 48))));
}
__device__ __forceinline__ float wave_sum_f(float v) {
    v += dpp_f<0xB1>(v);
    v += dpp_f<0x4E>(v);
    v += dpp_f<0x124>(v);
    v += dpp_f<0x128>(v);
    const int x = __float_as_int(v);
    return (__int_as_float(__builtin_amdgcn_readlane(x, 0)) + __int_as_float(__builtin_amdgcn_readlane(x, 16))) +
           (__int_as_float(__builtin_amdgcn_readlane(x, 32)) + __int_as_float(__builtin_amdgcn_readlane(x, 48)));
}
__device__ __forceinline__ uint32_t wave_sum_u(uint32_t v) {
    int x = static_cast<int>(v);
    x += dpp_i<0xB1>(x);
    x += dpp_i<0x4E>(x);
    x += dpp_i<0x124>(x);
    x += dpp_i<0x128>(x);
    const uint32_t u = static_cast<uint32_t>(x);
    return readlane_u32(u, 0) + readlane_u32(u, 16) + readlane_u32(u, 32) + readlane_u32(u, 48);
}

template <typename T>
__device__ __forceinline__ T wave_inclusive_sum(T v) {
    const int l = lane_id();
    for (int o = 1; o < kWave; o <<= 1) {
        T y = __shfl_up(v, o);
        if (l >= o) v += y;
    }
    return v;
}

// fp32 operations with round-to-nearest-even and no contraction
__device__ __forceinline__ float fsub(float a, float b) { return __fsub_rn(a, b); }
__device__ __forceinline__ float fadd(float a, float b) { return __fadd_rn(a, b); }
__device__ __forceinline__ float fmul(float a, float b) { return __fmul_rn(a, b); }

// order-preserving int image of a float, for integer atomics on floats
__device__ __forceinline__ int ordered_int(float f) {
    int i = __float_as_int(f);
    return i >= 0 ? i : (i ^ 0x7FFFFFFF);
}
__device__ __forceinline__ float ordered_float(int i) {
    return __int_as_float(i >= 0 ? i : (i ^ 0x7FFFFFFF));
}

// 8 XCDs take workgroups round robin; give each XCD a contiguous range of
// work items so that neighbouring items share that XCD's L2.
__device__ __forceinline__ int64_t xcd_item(int64_t block, int64_t grid) {
    const int64_t per = (grid + 7) / 8;
    return (block & 7) * per + (block >> 3);
}
inline int64_t xcd_grid(int64_t items) { return ((items + 7) / 8) * 8; }

}  // namespace sfc

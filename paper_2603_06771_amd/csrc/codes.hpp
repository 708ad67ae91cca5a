// Cell discretisation and space-filling-curve codes (device side).
//
// Section 4, steps 1-2: cell = floor((x - lo) * scale) per axis, clamped to
// the grid.  Section 4.1: Morton code = bit interleave, x most significant in
// each triple.  Section 4.2: Hilbert code, J. Skilling's transposed-index
// construction ("Programming the Hilbert curve", AIP Conf. Proc. 707, 2004):
// per level, from the coarsest, the lower bits are reflected or exchanged
// between axes, then a Gray code is applied and the three words are
// interleaved like a Morton code.
#pragma once

#include "common.hpp"

namespace sfc {

__device__ __forceinline__ uint32_t cell_of(float x, float lo, float s, uint32_t ncell) {
    const float u = fmul(fsub(x, lo), s);
    if (u >= static_cast<float>(ncell)) return ncell - 1u;
    if (u > 0.0f) return static_cast<uint32_t>(u);  // truncation is floor here
    return 0u;                                       // below the box, or NaN
}

// spread the low 21 bits of v to every third bit (bit i -> bit 3i)
__device__ __forceinline__ uint64_t spread3(uint32_t v) {
    uint64_t x = v & 0x1fffffull;
    x = (x | (x << 32)) & 0x001f00000000ffffull;
    x = (x | (x << 16)) & 0x001f0000ff0000ffull;
    x = (x | (x << 8)) & 0x100f00f00f00f00full;
    x = (x | (x << 4)) & 0x10c30c30c30c30c3ull;
    x = (x | (x << 2)) & 0x1249249249249249ull;
    return x;
}

__device__ __forceinline__ uint64_t morton_key(uint32_t x, uint32_t y, uint32_t z) {
    return (spread3(x) << 2) | (spread3(y) << 1) | spread3(z);
}

__device__ __forceinline__ uint64_t hilbert_key(uint32_t x, uint32_t y, uint32_t z, int bits) {
    for (int b = bits - 1; b >= 1; --b) {
        const uint32_t low = (1u << b) - 1u;
        // x: its own bit set -> reflect its lower bits (an exchange with itself is a no-op)
        x ^= low & (0u - ((x >> b) & 1u));
        // y: bit set -> reflect x's lower bits, else exchange lower bits of x and y
        {
            const uint32_t set = 0u - ((y >> b) & 1u);
            const uint32_t t = (x ^ y) & low & ~set;
            x ^= (low & set) | t;
            y ^= t;
        }
        // z: same with z
        {
            const uint32_t set = 0u - ((z >> b) & 1u);
            const uint32_t t = (x ^ z) & low & ~set;
            x ^= (low & set) | t;
            z ^= t;
        }
    }
    // Gray code: y ^= x, z ^= y, then every word takes the parity of the bits
    // of z strictly above each position
    y ^= x;
    z ^= y;
    uint32_t t = z >> 1;
    t ^= t >> 1;
    t ^= t >> 2;
    t ^= t >> 4;
    t ^= t >> 8;
    t ^= t >> 16;
    x ^= t;
    y ^= t;
    z ^= t;
    return morton_key(x, y, z);
}

__device__ __forceinline__ uint64_t point_key(float px, float py, float pz, const sfc_frame &f) {
    const uint32_t ncell = 1u << f.bits;
    const uint32_t cx = cell_of(px, f.lo[0], f.scale, ncell);
    const uint32_t cy = cell_of(py, f.lo[1], f.scale, ncell);
    const uint32_t cz = cell_of(pz, f.lo[2], f.scale, ncell);
    return f.curve == SFC_HILBERT ? hilbert_key(cx, cy, cz, f.bits) : morton_key(cx, cy, cz);
}

}  // namespace sfc

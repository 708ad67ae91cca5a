// Sections 4 and 5.1: frame, codes, sort, reorder and the complete linear
// octree, for a batch of independent clouds (one cloud is a batch of one).
//
// The paper refines the leaves array {0, 8^L} by repeated binary-search
// counting until no range holds more than N_max points.  On the GPU the same
// tree is derived in one pass from the sorted codes:
//
//  * A node (prefix P at level l) holds more than N points iff some window of
//    N + 1 consecutive sorted codes shares P.  With cw[t] = levels shared by
//    codes t and t + N and ca[t] = levels shared by codes t - 1 and t, the
//    internal (split) nodes whose first point is t are exactly the levels
//    ca[t] < l <= min(cw[t], L - 1).  Emitting them in order of t gives all
//    internal nodes in depth-first pre-order, with no search and no iteration.
//  * A stable counting pass by (cloud, level) turns the list into
//    breadth-first order; the children of the r-th internal node of level l
//    are then the 8 consecutive nodes 8r .. 8r + 7 of level l + 1 (the octree
//    is complete).
//  * Every node gets its code, its point range (internalRanges) by binary
//    search, its child link, and leaves get their tight point box and their
//    position p in the paper's leaves / counts arrays:
//      p = (sum of the leaf's octal digits)
//          + 7 * #(internal nodes that end before the leaf starts),
//    since every left sibling subtree with i internal nodes holds 7i + 1 leaves.
//  * Internal boxes are unions of the 8 child boxes, one launch per level,
//    deepest first.
//
// Batches: point kernels run on blocks of kChunk points that never straddle
// two clouds (a block finds its cloud in the table of first blocks), so every
// block has one frame, one curve and one threshold.  The sort runs on all
// points at once and ends with one stable pass by cloud, which leaves every
// cloud contiguous and ordered by (code, index).  Internal nodes of all clouds
// live in one list; per-cloud level counts locate each cloud's part.
// Roofline: the O(n) passes stream HBM; the sort dominates (8 + 1 passes of
// 8 + 24 B per point); tree kernels are latency / launch bound.
#include <algorithm>
#include <vector>

#include "codes.hpp"
#include "internal.hpp"

namespace sfc {

namespace {

constexpr int kChunk = 2048;   // points per block in point kernels
constexpr int kLevels = 24;    // level slots (levels 0..21 used)

struct CloudMeta {
    uint32_t lvl_cnt[kLevels];      // internal nodes per level
    uint32_t lvl_int_off[kLevels];  // global breadth-first index of each level's first internal node
    int64_t node_off[kLevels];      // first local node index of each level; node_off[L+1] = n_nodes
    int64_t int_base;               // global index of the cloud's first internal node
    int64_t n_internal;
    int64_t n_nodes;
};

__device__ __forceinline__ int shared_levels(uint64_t a, uint64_t b, int bits) {
    if (a == b) return bits;
    const int h = 63 - __clzll(static_cast<long long>(a ^ b));  // highest differing bit
    return bits - 1 - h / 3;
}

template <typename T>
__device__ __forceinline__ int64_t lower_bound_dev(const T *a, int64_t n, T v) {
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (a[mid] < v)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo;
}

// index i of the last entry with a[i] <= v (a ascending, a[0] <= v)
template <typename T>
__device__ __forceinline__ int last_le(const T *a, int n, T v) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (a[mid] <= v)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

// Batch-wide device tables (in the workspace).
struct Tables {
    sfc_cloud *cl;        // [B] cloud table
    uint32_t *blk;        // [B+1] first point block of each cloud
    int64_t *start;       // [B+1] first point of each cloud (start[B] = total)
    CloudMeta *meta;      // [B]
    int64_t *node_base;   // [B+1] first flattened node of each cloud
    uint32_t *lvlpref;    // [kLevels][B+1] per level: internal nodes of earlier clouds
    float *part;          // [blocks][6] per point block: min xyz, max xyz
};

struct TableChunk {
    sfc_cloud c[16];
};

}  // namespace

// ------------------------------------------------------------------ tables
__global__ void k_write_table(TableChunk chunk, int first, int count, sfc_cloud *cl) {
    const int i = threadIdx.x;
    if (i < count) cl[first + i] = chunk.c[i];
}

__global__ void k_batch_prefix(const sfc_cloud *__restrict__ cl, int B, uint32_t *blk, int64_t *start) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    uint32_t b = 0;
    int64_t s = 0;
    for (int c = 0; c < B; ++c) {
        blk[c] = b;
        start[c] = cl[c].offset;
        b += static_cast<uint32_t>((cl[c].n + kChunk - 1) / kChunk);
        s = cl[c].offset + cl[c].n;
    }
    blk[B] = b;
    start[B] = s;
}

// block -> (cloud, [p0, p1)) for point kernels
struct BlockRange {
    int c;
    int64_t p0, p1;
};
__device__ __forceinline__ BlockRange block_range(const uint32_t *__restrict__ blk, const sfc_cloud *__restrict__ cl,
                                                  int B, uint32_t b) {
    BlockRange r;
    r.c = last_le<uint32_t>(blk, B, b);
    while (r.c + 1 < B && blk[r.c + 1] <= b) ++r.c;  // skip empty clouds
    const sfc_cloud &C = cl[r.c];
    r.p0 = C.offset + static_cast<int64_t>(b - blk[r.c]) * kChunk;
    r.p1 = min(r.p0 + static_cast<int64_t>(kChunk), C.offset + C.n);
    return r;
}

// ------------------------------------------------------------------ frame
__global__ void k_meta_init(CloudMeta *meta, int B) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= B) return;
    for (int l = 0; l < kLevels; ++l) meta[c].lvl_cnt[l] = 0;
}

// per point block: exact min / max of its points (order-free, so any
// reduction tree gives the same bits)
__global__ __launch_bounds__(256) void k_bbox_b(const float *__restrict__ xyz, Tables T, int B) {
    __shared__ float s_red[6][4];
    const BlockRange br = block_range(T.blk, T.cl, B, blockIdx.x);
    float mn[3] = {INFINITY, INFINITY, INFINITY}, mx[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int64_t i = br.p0 + threadIdx.x; i < br.p1; i += blockDim.x) {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const float v = xyz[3 * i + a];
            mn[a] = fminf(mn[a], v);
            mx[a] = fmaxf(mx[a], v);
        }
    }
    const int w = threadIdx.x / kWave;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const float lo = wave_min_u(mn[a]), hi = wave_max_u(mx[a]);
        if (lane_id() == 0) {
            s_red[a][w] = lo;
            s_red[3 + a][w] = hi;
        }
    }
    __syncthreads();
    if (threadIdx.x < 6) {
        const int a = threadIdx.x;
        float v = s_red[a][0];
        for (int j = 1; j < 4; ++j) v = a < 3 ? fminf(v, s_red[a][j]) : fmaxf(v, s_red[a][j]);
        T.part[6ll * blockIdx.x + a] = v;
    }
}

// Section 4, step 1: one wave per cloud reduces its block boxes; E is the
// largest fp32 side, scale = 2^L / E (correctly rounded division)
__global__ __launch_bounds__(64) void k_frame_b(Tables T, int B) {
    const int c = blockIdx.x;
    if (c >= B) return;
    const sfc_cloud &C = T.cl[c];
    float mn[3] = {INFINITY, INFINITY, INFINITY}, mx[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (uint32_t b = T.blk[c] + threadIdx.x; b < T.blk[c + 1]; b += kWave) {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            mn[a] = fminf(mn[a], T.part[6ll * b + a]);
            mx[a] = fmaxf(mx[a], T.part[6ll * b + 3 + a]);
        }
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        mn[a] = wave_min_u(mn[a]);
        mx[a] = wave_max_u(mx[a]);
    }
    if (threadIdx.x != 0) return;
    float lo[3], E = 0.0f;
    for (int a = 0; a < 3; ++a) {
        lo[a] = mn[a];
        const float hi = mx[a];
        if (C.n > 0) {
            const float side = fsub(hi, lo[a]);
            if (side > E) E = side;
        }
    }
    if (C.n == 0) lo[0] = lo[1] = lo[2] = 0.0f;
    if (!(E > 0.0f)) E = 1.0f;
    sfc_frame f;
    f.lo[0] = lo[0];
    f.lo[1] = lo[1];
    f.lo[2] = lo[2];
    f.scale = __fdiv_rn(static_cast<float>(1u << C.bits), E);
    f.bits = C.bits;
    f.curve = C.curve;
    *C.tree.frame = f;
}

// codes of every point (global arrays), iota of global indices
__global__ __launch_bounds__(256) void k_encode_b(const float *__restrict__ xyz, Tables T, int B,
                                                  uint64_t *__restrict__ keys, uint32_t *__restrict__ iota) {
    const BlockRange br = block_range(T.blk, T.cl, B, blockIdx.x);
    const sfc_frame f = *T.cl[br.c].tree.frame;
    for (int64_t i = br.p0 + threadIdx.x; i < br.p1; i += blockDim.x) {
        keys[i] = point_key(xyz[3 * i], xyz[3 * i + 1], xyz[3 * i + 2], f);
        iota[i] = static_cast<uint32_t>(i);
    }
}

// sorted cloud {x, y, z, local index} and local permutation
__global__ __launch_bounds__(256) void k_gather_b(const float *__restrict__ xyz, Tables T, int B,
                                                  uint32_t *__restrict__ perm, float4 *__restrict__ pts) {
    const BlockRange br = block_range(T.blk, T.cl, B, blockIdx.x);
    const uint32_t base = static_cast<uint32_t>(T.cl[br.c].offset);
    for (int64_t i = br.p0 + threadIdx.x; i < br.p1; i += blockDim.x) {
        const uint32_t o = perm[i];  // global original index
        const uint32_t loc = o - base;
        pts[i] = make_float4(xyz[3ll * o], xyz[3ll * o + 1], xyz[3ll * o + 2], __uint_as_float(loc));
        perm[i] = loc;
    }
}

// ------------------------------------------------------------------ octree
__global__ __launch_bounds__(256) void k_gen_count_b(const uint64_t *__restrict__ keys, Tables T, int B,
                                                     uint32_t *__restrict__ gen) {
    const BlockRange br = block_range(T.blk, T.cl, B, blockIdx.x);
    const sfc_cloud &C = T.cl[br.c];
    const int64_t s = C.offset, e = C.offset + C.n;
    const int64_t N = C.leaf_size;
    const int bits = C.bits;
    for (int64_t t = br.p0 + threadIdx.x; t < br.p1; t += blockDim.x) {
        const uint64_t k = keys[t];
        const int cw = (t + N < e) ? shared_levels(k, keys[t + N], bits) : -1;
        const int ca = (t > s) ? shared_levels(keys[t - 1], k, bits) : -1;
        const int top = min(cw, bits - 1);
        gen[t] = top > ca ? static_cast<uint32_t>(top - ca) : 0u;
    }
}

__global__ __launch_bounds__(256) void k_emit_b(const uint64_t *__restrict__ keys, Tables T, int B,
                                                const uint32_t *__restrict__ goff, uint64_t *__restrict__ ipre_prefix,
                                                uint64_t *__restrict__ ipre_start, uint64_t *__restrict__ lvkey,
                                                uint32_t *__restrict__ iota) {
    __shared__ uint32_t s_cnt[kLevels];
    if (threadIdx.x < kLevels) s_cnt[threadIdx.x] = 0;
    __syncthreads();
    const BlockRange br = block_range(T.blk, T.cl, B, blockIdx.x);
    const sfc_cloud &C = T.cl[br.c];
    const int64_t s = C.offset, e = C.offset + C.n;
    const int64_t N = C.leaf_size;
    const int bits = C.bits;
    for (int64_t t = br.p0 + threadIdx.x; t < br.p1; t += blockDim.x) {
        const uint64_t k = keys[t];
        const int cw = (t + N < e) ? shared_levels(k, keys[t + N], bits) : -1;
        const int ca = (t > s) ? shared_levels(keys[t - 1], k, bits) : -1;
        const int top = min(cw, bits - 1);
        uint32_t idx = goff[t];
        for (int l = ca + 1; l <= top; ++l, ++idx) {
            const int shift = 3 * (bits - l);
            const uint64_t prefix = k >> shift;
            ipre_prefix[idx] = prefix;
            ipre_start[idx] = prefix << shift;
            lvkey[idx] = static_cast<uint64_t>(br.c) * 32u + static_cast<uint64_t>(l);
            iota[idx] = idx;
            atomicAdd(&s_cnt[l], 1u);
        }
    }
    __syncthreads();
    if (threadIdx.x < kLevels && s_cnt[threadIdx.x]) atomicAdd(&T.meta[br.c].lvl_cnt[threadIdx.x], s_cnt[threadIdx.x]);
}

// per cloud: level offsets, counts, info; then (one thread) batch prefixes
__global__ void k_level_meta_b(const uint32_t *__restrict__ goff, Tables T, int B, int64_t *n_internal_total) {
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    int64_t nodes = 0;
    for (int c = 0; c < B; ++c) {
        const sfc_cloud &C = T.cl[c];
        CloudMeta &m = T.meta[c];
        const int bits = C.bits;
        const int64_t ib = goff[C.offset];
        const int64_t ni = static_cast<int64_t>(goff[C.offset + C.n]) - ib;
        uint32_t run = static_cast<uint32_t>(ib);
        int deepest = -1;
        for (int l = 0; l < kLevels; ++l) {
            m.lvl_int_off[l] = run;
            if (l <= bits) {
                run += m.lvl_cnt[l];
                if (m.lvl_cnt[l]) deepest = l;
            }
        }
        m.node_off[0] = 0;
        m.node_off[1] = 1;
        for (int l = 1; l + 1 < kLevels; ++l)
            m.node_off[l + 1] = m.node_off[l] + (l <= bits ? 8ll * m.lvl_cnt[l - 1] : 0ll);
        m.int_base = ib;
        m.n_internal = ni;
        m.n_nodes = 1 + 8 * ni;
        T.node_base[c] = nodes;
        nodes += m.n_nodes;
        sfc_tree_info *info = C.tree.info;
        info->n_points = C.n;
        info->n_internal = ni;
        info->n_leaves = 7 * ni + 1;
        info->n_nodes = 1 + 8 * ni;
        info->depth = deepest + 1;
        info->status = (static_cast<int64_t>(run) - ib == ni) ? 0 : 1;
        for (int l = 0; l < 23; ++l) info->level_nodes_off[l] = m.node_off[l <= bits + 1 ? l : bits + 1];
        for (int l = 0; l < kLevels; ++l) T.lvlpref[l * (B + 1) + c] = 0;
    }
    T.node_base[B] = nodes;
    for (int l = 0; l < kLevels; ++l) {
        uint32_t run = 0;
        for (int c = 0; c < B; ++c) {
            T.lvlpref[l * (B + 1) + c] = run;
            run += T.meta[c].lvl_cnt[l];
        }
        T.lvlpref[l * (B + 1) + B] = run;
    }
    *n_internal_total = B > 0 ? static_cast<int64_t>(goff[T.start[B]]) : 0;
}

__global__ __launch_bounds__(256) void k_bfs_prefix(const uint64_t *__restrict__ ipre_prefix,
                                                    const uint32_t *__restrict__ order,
                                                    const int64_t *__restrict__ ni_total,
                                                    uint64_t *__restrict__ ibfs_prefix) {
    const int64_t ni = *ni_total;
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    for (int64_t k = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; k < ni; k += stride)
        ibfs_prefix[k] = ipre_prefix[order[k]];
}

// cloud holding global breadth-first internal index k
__device__ __forceinline__ int cloud_of_internal(const CloudMeta *meta, int B, int64_t k) {
    int lo = 0, hi = B - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (meta[mid].int_base <= k)
            lo = mid;
        else
            hi = mid - 1;
    }
    while (lo + 1 < B && meta[lo + 1].int_base <= k) ++lo;
    return lo;
}

__global__ __launch_bounds__(256) void k_internal_node_index_b(const uint64_t *__restrict__ ibfs_prefix, Tables T,
                                                               int B, const int64_t *__restrict__ ni_total,
                                                               int32_t *__restrict__ int_node) {
    const int64_t ni = *ni_total;
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    for (int64_t k = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; k < ni; k += stride) {
        const int c = cloud_of_internal(T.meta, B, k);
        const CloudMeta &m = T.meta[c];
        const int bits = T.cl[c].bits;
        int l = 0;
        while (l + 1 < bits && static_cast<int64_t>(m.lvl_int_off[l + 1]) <= k) ++l;
        if (l == 0) {
            int_node[k] = 0;
            continue;
        }
        const uint64_t prefix = ibfs_prefix[k];
        const int64_t pr = lower_bound_dev<uint64_t>(ibfs_prefix + m.lvl_int_off[l - 1], m.lvl_cnt[l - 1], prefix >> 3);
        int_node[k] = static_cast<int32_t>(m.node_off[l] + 8 * pr + static_cast<int64_t>(prefix & 7u));
    }
}

__global__ __launch_bounds__(256) void k_nodes_b(Tables T, int B, const uint64_t *__restrict__ ibfs_prefix,
                                                 const uint64_t *__restrict__ ipre_start) {
    const int64_t total = T.node_base[B];
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    for (int64_t j = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; j < total; j += stride) {
        const int c = last_le<int64_t>(T.node_base, B, j);
        int cc = c;
        while (cc + 1 < B && T.node_base[cc + 1] <= j) ++cc;
        const sfc_cloud &C = T.cl[cc];
        const CloudMeta &m = T.meta[cc];
        const int bits = C.bits;
        const int64_t jl = j - T.node_base[cc];
        const int64_t ni = m.n_internal;
        int l = 0;
        while (l < bits && m.node_off[l + 1] <= jl) ++l;
        const int64_t s = jl - m.node_off[l];
        uint64_t prefix = 0;
        if (l > 0) prefix = (ibfs_prefix[m.lvl_int_off[l - 1] + s / 8] << 3) | static_cast<uint64_t>(s & 7);
        const int shift = 3 * (bits - l);
        const uint64_t start = prefix << shift;
        const uint64_t stop = start + (1ull << shift);
        const uint64_t *keys = C.tree.keys;
        const int64_t b = lower_bound_dev<uint64_t>(keys, C.n, start);
        const int64_t e = lower_bound_dev<uint64_t>(keys, C.n, stop);
        int32_t ch = -1;
        if (l < bits) {
            const uint32_t off = m.lvl_int_off[l], cnt = m.lvl_cnt[l];
            const int64_t r = lower_bound_dev<uint64_t>(ibfs_prefix + off, cnt, prefix);
            if (r < cnt && ibfs_prefix[off + r] == prefix) ch = static_cast<int32_t>(m.node_off[l + 1] + 8 * r);
        }
        C.tree.child[jl] = ch;
        C.tree.node_key[jl] = start;
        C.tree.node_level[jl] = static_cast<uint8_t>(l);
        sfc_node nd;
        nd.begin = static_cast<uint32_t>(b);
        nd.end = static_cast<uint32_t>(e);
        nd.lo[0] = nd.lo[1] = nd.lo[2] = INFINITY;
        nd.hi[0] = nd.hi[1] = nd.hi[2] = -INFINITY;
        if (ch < 0) {
            const float4 *pts = reinterpret_cast<const float4 *>(C.tree.points);
            for (int64_t p = b; p < e; ++p) {
                const float4 q = pts[p];
                nd.lo[0] = fminf(nd.lo[0], q.x);
                nd.lo[1] = fminf(nd.lo[1], q.y);
                nd.lo[2] = fminf(nd.lo[2], q.z);
                nd.hi[0] = fmaxf(nd.hi[0], q.x);
                nd.hi[1] = fmaxf(nd.hi[1], q.y);
                nd.hi[2] = fmaxf(nd.hi[2], q.z);
            }
            // position among the leaves in code order
            const uint64_t m0 = 0x1249249249249249ull;
            const int64_t digit_sum = __popcll(prefix & m0) + 2 * __popcll(prefix & (m0 << 1)) +
                                      4 * __popcll(prefix & (m0 << 2));
            const int zeros = prefix == 0 ? l : (__ffsll(static_cast<long long>(prefix)) - 1) / 3;
            const int64_t before = lower_bound_dev<uint64_t>(ipre_start + m.int_base, ni, start) - (l - zeros);
            const int64_t rank = digit_sum + 7 * before;
            if (rank >= 0 && rank <= 7 * ni) {
                C.tree.leaves[rank] = start;
                C.tree.counts[rank] = static_cast<uint32_t>(e - b);
            }
        }
        C.tree.nodes[jl] = nd;
        if (jl == 0) C.tree.leaves[7 * ni + 1] = 1ull << (3 * bits);
    }
}

__global__ __launch_bounds__(256) void k_internal_boxes_b(Tables T, int B, int level,
                                                          const int32_t *__restrict__ int_node) {
    const uint32_t *pref = T.lvlpref + level * (B + 1);
    const int64_t cnt = pref[B];
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < cnt; i += stride) {
        int c = last_le<uint32_t>(pref, B, static_cast<uint32_t>(i));
        while (c + 1 < B && pref[c + 1] <= i) ++c;
        const CloudMeta &m = T.meta[c];
        const sfc_octree &t = T.cl[c].tree;
        const int32_t j = int_node[m.lvl_int_off[level] + (i - pref[c])];
        const int32_t ch = t.child[j];
        sfc_node nd = t.nodes[j];
        for (int k = 0; k < 8; ++k) {
            const sfc_node cn = t.nodes[ch + k];
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                nd.lo[a] = fminf(nd.lo[a], cn.lo[a]);
                nd.hi[a] = fmaxf(nd.hi[a], cn.hi[a]);
            }
        }
        t.nodes[j] = nd;
    }
}

// ----------------------------------------------------------- sizes, layout
int64_t internal_upper_bound(int64_t n, uint32_t leaf_size, int bits) {
    // internal nodes of one level are disjoint and each holds > leaf_size points
    const int64_t per_level = n / (static_cast<int64_t>(leaf_size) + 1);
    int64_t total = 0, pow8 = 1;
    for (int l = 0; l < bits; ++l) {
        total += pow8 < per_level ? pow8 : per_level;
        if (pow8 < (int64_t(1) << 40)) pow8 *= 8;
    }
    return total;
}

// Shared point arrays first, then each cloud's frame, info and node arrays.
size_t batch_layout(int B, sfc_cloud *cl, void *mem) {
    int64_t total = 0;
    for (int c = 0; c < B; ++c) total = std::max<int64_t>(total, cl[c].offset + cl[c].n);
    Carver cv(mem);
    float *points = cv.take<float>(4 * static_cast<size_t>(total));
    uint64_t *keys = cv.take<uint64_t>(total);
    uint32_t *perm = cv.take<uint32_t>(total);
    for (int c = 0; c < B; ++c) {
        sfc_octree &t = cl[c].tree;
        const int64_t ni = internal_upper_bound(cl[c].n, cl[c].leaf_size, cl[c].bits);
        const int64_t nl = 7 * ni + 1, nn = 8 * ni + 1;
        t.frame = cv.take<sfc_frame>(1);
        t.info = cv.take<sfc_tree_info>(1);
        t.leaves = cv.take<uint64_t>(nl + 1);
        t.counts = cv.take<uint32_t>(nl);
        t.nodes = cv.take<sfc_node>(nn);
        t.child = cv.take<int32_t>(nn);
        t.node_key = cv.take<uint64_t>(nn);
        t.node_level = cv.take<uint8_t>(nn);
        t.points = points ? points + 4 * cl[c].offset : nullptr;
        t.keys = keys ? keys + cl[c].offset : nullptr;
        t.perm = perm ? perm + cl[c].offset : nullptr;
        t.n = cl[c].n;
        t.max_nodes = nn;
        t.max_leaves = nl;
        t.bits = cl[c].bits;
        t.curve = cl[c].curve;
        t.leaf_size = cl[c].leaf_size;
        t.reserved = 0;
    }
    return cv.bytes();
}

size_t tree_layout(int64_t n, uint32_t leaf_size, int bits, void *mem, sfc_octree *t) {
    sfc_cloud c{};
    c.offset = 0;
    c.n = n;
    c.leaf_size = leaf_size;
    c.bits = bits;
    const size_t b = batch_layout(1, &c, mem);
    if (t) *t = c.tree;
    return b;
}

namespace {

struct BuildWs {
    Tables T;
    int64_t *ni_total;
    uint64_t *keys_alt;
    uint32_t *vals_alt;
    void *radix_ws;
    uint32_t *gen;
    uint32_t *goff;
    void *scan_ws;
    uint64_t *ipre_prefix, *ipre_start, *lvkey, *lvkey_alt, *ibfs_prefix;
    uint32_t *iota, *iota_alt;
    int32_t *int_node;
    void *radix_ws_int;
};

struct BatchSizes {
    int64_t n = 0;    // points
    int64_t ni = 0;   // internal-node bound
    int64_t blocks = 0;
    int max_bits = 1;
};

BatchSizes batch_sizes(int B, const sfc_cloud *cl) {
    BatchSizes s;
    for (int c = 0; c < B; ++c) {
        s.n = std::max<int64_t>(s.n, cl[c].offset + cl[c].n);
        s.ni += internal_upper_bound(cl[c].n, cl[c].leaf_size, cl[c].bits);
        s.blocks += (cl[c].n + kChunk - 1) / kChunk;
        s.max_bits = std::max(s.max_bits, cl[c].bits);
    }
    return s;
}

size_t carve_build_ws(int B, const BatchSizes &s, void *mem, BuildWs *w) {
    const int64_t n = s.n > 0 ? s.n : 1, nic = s.ni > 0 ? s.ni : 1;
    Carver c(mem);
    BuildWs x;
    x.T.cl = c.take<sfc_cloud>(B);
    x.T.blk = c.take<uint32_t>(B + 1);
    x.T.start = c.take<int64_t>(B + 1);
    x.T.meta = c.take<CloudMeta>(B);
    x.T.node_base = c.take<int64_t>(B + 1);
    x.T.lvlpref = c.take<uint32_t>(static_cast<size_t>(kLevels) * (B + 1));
    x.T.part = c.take<float>(6 * static_cast<size_t>(s.blocks > 0 ? s.blocks : 1));
    x.ni_total = c.take<int64_t>(1);
    x.keys_alt = c.take<uint64_t>(n);
    x.vals_alt = c.take<uint32_t>(n);
    x.radix_ws = c.take<char>(radix_ws_bytes(n));
    x.gen = c.take<uint32_t>(n);
    x.goff = c.take<uint32_t>(n + 1);
    x.scan_ws = c.take<char>(scan_ws_bytes(n));
    x.ipre_prefix = c.take<uint64_t>(nic);
    x.ipre_start = c.take<uint64_t>(nic);
    x.lvkey = c.take<uint64_t>(nic);
    x.lvkey_alt = c.take<uint64_t>(nic);
    x.ibfs_prefix = c.take<uint64_t>(nic);
    x.iota = c.take<uint32_t>(nic);
    x.iota_alt = c.take<uint32_t>(nic);
    x.int_node = c.take<int32_t>(nic);
    x.radix_ws_int = c.take<char>(radix_ws_bytes(nic));
    if (w) *w = x;
    return c.bytes();
}

}  // namespace

// Writes the host cloud table into device memory with kernel launches (the
// table travels as kernel arguments: no host buffer has to outlive the call).
int upload_clouds(const sfc_cloud *host, int B, sfc_cloud *dev, hipStream_t s) {
    for (int first = 0; first < B; first += 16) {
        TableChunk ch;
        const int cnt = std::min(16, B - first);
        for (int i = 0; i < cnt; ++i) ch.c[i] = host[first + i];
        k_write_table<<<1, 64, 0, s>>>(ch, first, cnt, dev);
        SFC_LAUNCH_CHECK("k_write_table");
    }
    return SFC_OK;
}

static int build_batch_impl(const float *xyz, int B, const sfc_cloud *cl, const BatchSizes &sz, BuildWs &w,
                            hipStream_t s) {
    int rc = upload_clouds(cl, B, w.T.cl, s);
    if (rc) return rc;
    k_batch_prefix<<<1, 64, 0, s>>>(w.T.cl, B, w.T.blk, w.T.start);
    SFC_LAUNCH_CHECK("k_batch_prefix");
    k_meta_init<<<grid_for(B, 64), 64, 0, s>>>(w.T.meta, B);
    SFC_LAUNCH_CHECK("k_meta_init");
    const unsigned blocks = static_cast<unsigned>(std::max<int64_t>(sz.blocks, 1));
    // the shared arrays of the batch (identical for every cloud's view)
    uint64_t *keys = cl[0].tree.keys - cl[0].offset;
    uint32_t *perm = cl[0].tree.perm - cl[0].offset;
    float4 *pts = reinterpret_cast<float4 *>(cl[0].tree.points - 4 * cl[0].offset);
    const int64_t n = sz.n;
    if (sz.blocks > 0) {
        // Section 4: frames and codes
        k_bbox_b<<<blocks, 256, 0, s>>>(xyz, w.T, B);
        SFC_LAUNCH_CHECK("k_bbox_b");
    }
    k_frame_b<<<B, 64, 0, s>>>(w.T, B);
    SFC_LAUNCH_CHECK("k_frame_b");
    if (sz.blocks > 0) {
        k_encode_b<<<blocks, 256, 0, s>>>(xyz, w.T, B, keys, perm);
        SFC_LAUNCH_CHECK("k_encode_b");
        // Section 4, reorder step 2: sort by code, then stably by cloud
        bool in_alt = false;
        rc = radix_sort_pairs(keys, perm, w.keys_alt, w.vals_alt, n, nullptr, 3 * sz.max_bits, w.radix_ws, s, &in_alt,
                              w.T.start, B);
        if (rc) return rc;
        if (in_alt) {
            SFC_HIP_TRY(hipMemcpyAsync(keys, w.keys_alt, sizeof(uint64_t) * n, hipMemcpyDeviceToDevice, s));
            SFC_HIP_TRY(hipMemcpyAsync(perm, w.vals_alt, sizeof(uint32_t) * n, hipMemcpyDeviceToDevice, s));
        }
        k_gather_b<<<blocks, 256, 0, s>>>(xyz, w.T, B, perm, pts);
        SFC_LAUNCH_CHECK("k_gather_b");
        // Section 5.1: internal nodes in pre-order
        k_gen_count_b<<<blocks, 256, 0, s>>>(keys, w.T, B, w.gen);
        SFC_LAUNCH_CHECK("k_gen_count_b");
    }
    rc = scan_u32_to_u32(w.gen, n, w.goff, true, w.scan_ws, s);
    if (rc) return rc;
    if (sz.blocks > 0) {
        k_emit_b<<<blocks, 256, 0, s>>>(keys, w.T, B, w.goff, w.ipre_prefix, w.ipre_start, w.lvkey, w.iota);
        SFC_LAUNCH_CHECK("k_emit_b");
    }
    k_level_meta_b<<<1, 64, 0, s>>>(w.goff, w.T, B, w.ni_total);
    SFC_LAUNCH_CHECK("k_level_meta_b");
    // breadth-first order: stable sort of the pre-order list by (cloud, level)
    const int64_t ni_ub = sz.ni;
    if (ni_ub > 0) {
        int key_bits = 8;
        while ((int64_t(1) << key_bits) < static_cast<int64_t>(B) * 32) key_bits += 8;
        bool in_alt = false;
        rc = radix_sort_pairs(w.lvkey, w.iota, w.lvkey_alt, w.iota_alt, ni_ub, w.ni_total, key_bits, w.radix_ws_int,
                              s, &in_alt);
        if (rc) return rc;
        const uint32_t *order = in_alt ? w.iota_alt : w.iota;
        k_bfs_prefix<<<grid_for(ni_ub, 256, 4096), 256, 0, s>>>(w.ipre_prefix, order, w.ni_total, w.ibfs_prefix);
        SFC_LAUNCH_CHECK("k_bfs_prefix");
        k_internal_node_index_b<<<grid_for(ni_ub, 256, 4096), 256, 0, s>>>(w.ibfs_prefix, w.T, B, w.ni_total,
                                                                            w.int_node);
        SFC_LAUNCH_CHECK("k_internal_node_index_b");
    }
    const int64_t nn_ub = 8 * ni_ub + B;
    k_nodes_b<<<grid_for(nn_ub, 256, 8192), 256, 0, s>>>(w.T, B, w.ibfs_prefix, w.ipre_start);
    SFC_LAUNCH_CHECK("k_nodes_b");
    int64_t per_level = 0;
    for (int c = 0; c < B; ++c) per_level += cl[c].n / (static_cast<int64_t>(cl[c].leaf_size) + 1);
    for (int l = sz.max_bits - 1; l >= 0; --l) {
        int64_t ub = per_level;
        if (3 * l <= 40 && (static_cast<int64_t>(B) << (3 * l)) < ub) ub = static_cast<int64_t>(B) << (3 * l);
        if (ub <= 0) continue;
        k_internal_boxes_b<<<grid_for(ub, 256, 2048), 256, 0, s>>>(w.T, B, l, w.int_node);
        SFC_LAUNCH_CHECK("k_internal_boxes_b");
    }
    return SFC_OK;
}

static bool clouds_valid(int B, const sfc_cloud *cl) {
    if (B < 1 || B > (1 << 16) || !cl) return false;
    int64_t expect = 0;
    for (int c = 0; c < B; ++c) {
        const sfc_cloud &C = cl[c];
        if (C.n < 0 || C.n > 0xFFFFFFFFll || C.offset != expect || C.leaf_size < 1 || C.bits < 1 || C.bits > 21 ||
            (C.curve != SFC_MORTON && C.curve != SFC_HILBERT))
            return false;
        expect += C.n;
        if (8 * internal_upper_bound(C.n, C.leaf_size, C.bits) + 1 > 0x7FFFFFFFll) return false;
    }
    return expect <= 0xFFFFFFFFll;
}

// The layout of batch_layout with the actual counts of every tree (nodes
// and leaves from its sfc_tree_info) instead of the upper bounds: shared
// point arrays first, then each cloud's frame, info and node arrays.
static size_t compact_layout(int B, const sfc_cloud *src, const sfc_tree_info *info, sfc_cloud *dst, void *mem) {
    int64_t total = 0;
    for (int c = 0; c < B; ++c) total = std::max<int64_t>(total, src[c].offset + src[c].n);
    Carver cv(mem);
    float *points = cv.take<float>(4 * static_cast<size_t>(total));
    uint64_t *keys = cv.take<uint64_t>(total);
    uint32_t *perm = cv.take<uint32_t>(total);
    for (int c = 0; c < B; ++c) {
        const int64_t nl = info[c].n_leaves, nn = info[c].n_nodes;
        sfc_octree t = src[c].tree;
        t.frame = cv.take<sfc_frame>(1);
        t.info = cv.take<sfc_tree_info>(1);
        t.leaves = cv.take<uint64_t>(nl + 1);
        t.counts = cv.take<uint32_t>(nl);
        t.nodes = cv.take<sfc_node>(nn);
        t.child = cv.take<int32_t>(nn);
        t.node_key = cv.take<uint64_t>(nn);
        t.node_level = cv.take<uint8_t>(nn);
        t.points = points ? points + 4 * src[c].offset : nullptr;
        t.keys = keys ? keys + src[c].offset : nullptr;
        t.perm = perm ? perm + src[c].offset : nullptr;
        t.max_nodes = nn;
        t.max_leaves = nl;
        if (dst) {
            dst[c] = src[c];
            dst[c].tree = t;
        }
    }
    return cv.bytes();
}

}  // namespace sfc

extern "C" int octree_batch_compact(int B, const sfc_cloud *clouds, void *dst_mem, size_t *bytes, sfc_cloud *out,
                                    void *stream) {
    using namespace sfc;
    if (!bytes || !clouds_valid(B, clouds) || (dst_mem && !out)) {
        set_error("octree_batch_compact: invalid argument");
        return SFC_EINVAL;
    }
    for (int c = 0; c < B; ++c)
        if (!clouds[c].tree.info || !clouds[c].tree.nodes || !clouds[c].tree.keys ||
            clouds[c].tree.keys - clouds[c].offset != clouds[0].tree.keys - clouds[0].offset) {
            set_error("octree_batch_compact: trees not laid out by octree_batch_layout");
            return SFC_EINVAL;
        }
    hipStream_t s = static_cast<hipStream_t>(stream);
    // the actual counts (the host waits for the build on the stream)
    std::vector<sfc_tree_info> info(B);
    for (int c = 0; c < B; ++c)
        SFC_HIP_TRY(hipMemcpyAsync(&info[c], clouds[c].tree.info, sizeof(sfc_tree_info), hipMemcpyDeviceToHost, s));
    SFC_HIP_TRY(hipStreamSynchronize(s));
    for (int c = 0; c < B; ++c)
        if (info[c].status != 0 || info[c].n_nodes < 1 || info[c].n_nodes > clouds[c].tree.max_nodes ||
            info[c].n_leaves < 1 || info[c].n_leaves > clouds[c].tree.max_leaves) {
            set_error("octree_batch_compact: cloud %d: its tree is not built (status %d, %lld nodes)", c,
                      info[c].status, static_cast<long long>(info[c].n_nodes));
            return SFC_EINVAL;
        }
    const size_t need = compact_layout(B, clouds, info.data(), nullptr, nullptr);
    if (!dst_mem) {
        *bytes = need;
        return SFC_OK;
    }
    if (*bytes < need || (reinterpret_cast<uintptr_t>(dst_mem) & 255u)) {
        set_error("octree_batch_compact: destination needs %zu bytes, 256-aligned", need);
        return SFC_EINVAL;
    }
    compact_layout(B, clouds, info.data(), out, dst_mem);
    int64_t total = 0;
    for (int c = 0; c < B; ++c) total = std::max<int64_t>(total, clouds[c].offset + clouds[c].n);
    auto copy = [&](void *d, const void *src, size_t n) -> int {
        if (n == 0) return SFC_OK;
        SFC_HIP_TRY(hipMemcpyAsync(d, src, n, hipMemcpyDeviceToDevice, s));
        return SFC_OK;
    };
    const sfc_octree &a0 = clouds[0].tree, &b0 = out[0].tree;
    const int64_t o0 = clouds[0].offset;
    int rc = copy(b0.points - 4 * o0, a0.points - 4 * o0, 16 * static_cast<size_t>(total));
    if (!rc) rc = copy(b0.keys - o0, a0.keys - o0, 8 * static_cast<size_t>(total));
    if (!rc) rc = copy(b0.perm - o0, a0.perm - o0, 4 * static_cast<size_t>(total));
    for (int c = 0; c < B && !rc; ++c) {
        const sfc_octree &a = clouds[c].tree, &b = out[c].tree;
        const size_t nl = static_cast<size_t>(info[c].n_leaves), nn = static_cast<size_t>(info[c].n_nodes);
        rc = copy(b.frame, a.frame, sizeof(sfc_frame));
        if (!rc) rc = copy(b.info, a.info, sizeof(sfc_tree_info));
        if (!rc) rc = copy(b.leaves, a.leaves, 8 * (nl + 1));
        if (!rc) rc = copy(b.counts, a.counts, 4 * nl);
        if (!rc) rc = copy(b.nodes, a.nodes, sizeof(sfc_node) * nn);
        if (!rc) rc = copy(b.child, a.child, 4 * nn);
        if (!rc) rc = copy(b.node_key, a.node_key, 8 * nn);
        if (!rc) rc = copy(b.node_level, a.node_level, nn);
    }
    return rc;
}

extern "C" int octree_bytes(int64_t n, uint32_t leaf_size, int bits, size_t *bytes) {
    using namespace sfc;
    if (!bytes || n < 0 || n > 0xFFFFFFFFll || leaf_size < 1 || bits < 1 || bits > 21) {
        set_error("octree_bytes: invalid argument");
        return SFC_EINVAL;
    }
    if (8 * internal_upper_bound(n, leaf_size, bits) + 1 > 0x7FFFFFFFll) {
        set_error("octree_bytes: node bound exceeds 2^31 - 1; raise leaf_size");
        return SFC_ENOTSUP;
    }
    *bytes = tree_layout(n, leaf_size, bits, nullptr, nullptr);
    return SFC_OK;
}

extern "C" int octree_batch_layout(int B, sfc_cloud *clouds, void *tree_mem, size_t *bytes) {
    using namespace sfc;
    if (!bytes || !clouds_valid(B, clouds)) {
        set_error("octree_batch_layout: invalid batch (offsets must be the running sum of sizes)");
        return SFC_EINVAL;
    }
    if (!tree_mem) {
        std::vector<sfc_cloud> tmp(clouds, clouds + B);
        *bytes = batch_layout(B, tmp.data(), nullptr);
        return SFC_OK;
    }
    if (reinterpret_cast<uintptr_t>(tree_mem) & 255u) {
        set_error("octree_batch_layout: tree memory must be 256-byte aligned");
        return SFC_EINVAL;
    }
    *bytes = batch_layout(B, clouds, tree_mem);
    return SFC_OK;
}

extern "C" int build_linear_octree_batched(const float *xyz, int B, const sfc_cloud *clouds, void *ws,
                                           size_t *ws_bytes, void *stream) {
    using namespace sfc;
    if (!ws_bytes || !clouds_valid(B, clouds)) {
        set_error("build_linear_octree_batched: invalid batch");
        return SFC_EINVAL;
    }
    const BatchSizes sz = batch_sizes(B, clouds);
    const size_t need = carve_build_ws(B, sz, nullptr, nullptr);
    if (!ws) {
        *ws_bytes = need;
        return SFC_OK;
    }
    if (*ws_bytes < need || (reinterpret_cast<uintptr_t>(ws) & 255u)) {
        set_error("build_linear_octree_batched: workspace needs %zu bytes, 256-aligned", need);
        return SFC_EWORKSPACE;
    }
    for (int c = 0; c < B; ++c)
        if (!clouds[c].tree.nodes || !clouds[c].tree.frame || !clouds[c].tree.keys ||
            clouds[c].tree.keys - clouds[c].offset != clouds[0].tree.keys - clouds[0].offset ||
            (sz.n > 0 && !xyz)) {
            set_error("build_linear_octree_batched: trees not laid out by octree_batch_layout");
            return SFC_EINVAL;
        }
    BuildWs w;
    carve_build_ws(B, sz, ws, &w);
    return build_batch_impl(xyz, B, clouds, sz, w, static_cast<hipStream_t>(stream));
}

extern "C" int build_linear_octree(const float *xyz, int64_t n, int curve, int bits, uint32_t leaf_size,
                                   void *tree_mem, size_t tree_bytes, sfc_octree *tree_out, void *ws,
                                   size_t *ws_bytes, void *stream) {
    using namespace sfc;
    sfc_cloud c{};
    c.offset = 0;
    c.n = n;
    c.curve = curve;
    c.bits = bits;
    c.leaf_size = leaf_size;
    if (!ws_bytes || !clouds_valid(1, &c)) {
        set_error("build_linear_octree: invalid argument (n=%lld bits=%d curve=%d leaf_size=%u)", (long long)n, bits,
                  curve, leaf_size);
        return (n >= 0 && leaf_size >= 1 && bits >= 1 && bits <= 21 && (curve == SFC_MORTON || curve == SFC_HILBERT) &&
                8 * internal_upper_bound(n, leaf_size, bits) + 1 > 0x7FFFFFFFll)
                   ? SFC_ENOTSUP
                   : SFC_EINVAL;
    }
    const BatchSizes sz = batch_sizes(1, &c);
    const size_t need = carve_build_ws(1, sz, nullptr, nullptr);
    if (!ws) {
        *ws_bytes = need;
        return SFC_OK;
    }
    if (*ws_bytes < need || (reinterpret_cast<uintptr_t>(ws) & 255u)) {
        set_error("build_linear_octree: workspace needs %zu bytes, 256-aligned", need);
        return SFC_EWORKSPACE;
    }
    const size_t tneed = tree_layout(n, leaf_size, bits, nullptr, nullptr);
    if (!tree_mem || !tree_out || tree_bytes < tneed || (reinterpret_cast<uintptr_t>(tree_mem) & 255u) ||
        (n > 0 && !xyz)) {
        set_error("build_linear_octree: tree memory needs %zu bytes, 256-aligned", tneed);
        return SFC_EINVAL;
    }
    batch_layout(1, &c, tree_mem);
    BuildWs w;
    carve_build_ws(1, sz, ws, &w);
    const int rc = build_batch_impl(xyz, 1, &c, sz, w, static_cast<hipStream_t>(stream));
    if (rc == SFC_OK) *tree_out = c.tree;
    return rc;
}

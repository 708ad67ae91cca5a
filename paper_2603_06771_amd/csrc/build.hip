// Section 5.1: the complete linear octree over the sorted codes.
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
//  * A stable counting pass by level turns the list into breadth-first order;
//    the children of the r-th internal node of level l are then the 8
//    consecutive nodes 8r .. 8r + 7 of level l + 1 (the octree is complete).
//  * Every node gets its code, its point range (internalRanges) by binary
//    search, its child link, and leaves get their tight point box and their
//    position p in the paper's leaves / counts arrays:
//      p = (sum of the leaf's octal digits)
//          + 7 * #(internal nodes that end before the leaf starts),
//    since every left sibling subtree with i internal nodes holds 7i + 1 leaves.
//  * Internal boxes are unions of the 8 child boxes, one launch per level,
//    deepest first.
// Roofline: all kernels are O(n) streams or O(nodes * log) searches; the build
// is bound by the radix sort (HBM) and by launch latency on small clouds.
#include "internal.hpp"

namespace sfc {

namespace {

struct LevelMeta {
    uint32_t lvl_cnt[32];      // internal nodes per level
    uint32_t lvl_int_off[33];  // first breadth-first internal index per level
    int64_t node_off[34];      // first node index per level; node_off[L+1] = n_nodes
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

}  // namespace

__global__ __launch_bounds__(256) void k_gather(const float *__restrict__ xyz, const uint32_t *__restrict__ perm,
                                                int64_t n, float4 *__restrict__ pts) {
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride) {
        const uint32_t o = perm[i];
        pts[i] = make_float4(xyz[3ll * o], xyz[3ll * o + 1], xyz[3ll * o + 2], __uint_as_float(o));
    }
}

__global__ void k_meta_init(LevelMeta *m) {
    for (int i = threadIdx.x; i < 32; i += blockDim.x) m->lvl_cnt[i] = 0;
}

__global__ __launch_bounds__(256) void k_gen_count(const uint64_t *__restrict__ keys, int64_t n, uint32_t N, int bits,
                                                   uint32_t *__restrict__ gen) {
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    for (int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; t < n; t += stride) {
        const uint64_t k = keys[t];
        const int cw = (t + N < n) ? shared_levels(k, keys[t + N], bits) : -1;
        const int ca = (t > 0) ? shared_levels(keys[t - 1], k, bits) : -1;
        const int top = min(cw, bits - 1);
        gen[t] = top > ca ? static_cast<uint32_t>(top - ca) : 0u;
    }
}

__global__ __launch_bounds__(256) void k_emit_internal(const uint64_t *__restrict__ keys, int64_t n, uint32_t N,
                                                       int bits, const uint32_t *__restrict__ goff,
                                                       uint64_t *__restrict__ ipre_prefix,
                                                       uint64_t *__restrict__ ipre_start, uint64_t *__restrict__ lvkey,
                                                       uint32_t *__restrict__ iota, LevelMeta *meta) {
    __shared__ uint32_t s_cnt[32];
    if (threadIdx.x < 32) s_cnt[threadIdx.x] = 0;
    __syncthreads();
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    for (int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; t < n; t += stride) {
        const uint64_t k = keys[t];
        const int cw = (t + N < n) ? shared_levels(k, keys[t + N], bits) : -1;
        const int ca = (t > 0) ? shared_levels(keys[t - 1], k, bits) : -1;
        const int top = min(cw, bits - 1);
        uint32_t idx = goff[t];
        for (int l = ca + 1; l <= top; ++l, ++idx) {
            const int shift = 3 * (bits - l);
            const uint64_t prefix = k >> shift;
            ipre_prefix[idx] = prefix;
            ipre_start[idx] = prefix << shift;
            lvkey[idx] = static_cast<uint64_t>(l);
            iota[idx] = idx;
            atomicAdd(&s_cnt[l], 1u);
        }
    }
    __syncthreads();
    if (threadIdx.x < 32 && s_cnt[threadIdx.x]) atomicAdd(&meta->lvl_cnt[threadIdx.x], s_cnt[threadIdx.x]);
}

__global__ void k_level_meta(const uint32_t *__restrict__ goff, int64_t n, int bits, LevelMeta *meta,
                             sfc_tree_info *info) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const int64_t ni = goff[n];
    uint32_t run = 0;
    int deepest = -1;
    for (int l = 0; l <= bits; ++l) {
        meta->lvl_int_off[l] = run;
        run += meta->lvl_cnt[l];
        if (meta->lvl_cnt[l]) deepest = l;
    }
    meta->lvl_int_off[bits + 1] = run;
    meta->node_off[0] = 0;
    meta->node_off[1] = 1;
    for (int l = 1; l <= bits; ++l) meta->node_off[l + 1] = meta->node_off[l] + 8ll * meta->lvl_cnt[l - 1];
    meta->n_internal = ni;
    meta->n_nodes = 1 + 8 * ni;
    info->n_points = n;
    info->n_internal = ni;
    info->n_leaves = 7 * ni + 1;
    info->n_nodes = 1 + 8 * ni;
    info->depth = deepest + 1;
    info->status = (static_cast<int64_t>(run) == ni) ? 0 : 1;
    for (int l = 0; l < 23; ++l) info->level_nodes_off[l] = l <= bits + 1 ? meta->node_off[l] : meta->node_off[bits + 1];
}

__global__ __launch_bounds__(256) void k_bfs_prefix(const uint64_t *__restrict__ ipre_prefix,
                                                    const uint32_t *__restrict__ order, const LevelMeta *meta,
                                                    uint64_t *__restrict__ ibfs_prefix) {
    const int64_t ni = meta->n_internal;
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    for (int64_t k = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; k < ni; k += stride)
        ibfs_prefix[k] = ipre_prefix[order[k]];
}

__global__ __launch_bounds__(256) void k_internal_node_index(const uint64_t *__restrict__ ibfs_prefix,
                                                             const LevelMeta *__restrict__ meta, int bits,
                                                             int32_t *__restrict__ int_node) {
    const int64_t ni = meta->n_internal;
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    for (int64_t k = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; k < ni; k += stride) {
        int l = 0;
        while (l + 1 < bits && static_cast<int64_t>(meta->lvl_int_off[l + 1]) <= k) ++l;
        if (l == 0) {
            int_node[k] = 0;
            continue;
        }
        const uint64_t prefix = ibfs_prefix[k];
        const uint32_t poff = meta->lvl_int_off[l - 1];
        const int64_t pr = lower_bound_dev<uint64_t>(ibfs_prefix + poff, meta->lvl_cnt[l - 1], prefix >> 3);
        int_node[k] = static_cast<int32_t>(meta->node_off[l] + 8 * pr + static_cast<int64_t>(prefix & 7u));
    }
}

__global__ __launch_bounds__(256) void k_nodes(const uint64_t *__restrict__ keys, const float4 *__restrict__ pts,
                                               int64_t n, int bits, const LevelMeta *__restrict__ meta,
                                               const uint64_t *__restrict__ ibfs_prefix,
                                               const uint64_t *__restrict__ ipre_start, sfc_node *__restrict__ nodes,
                                               int32_t *__restrict__ child, uint64_t *__restrict__ node_key,
                                               uint8_t *__restrict__ node_level, uint64_t *__restrict__ leaves,
                                               uint32_t *__restrict__ counts) {
    const int64_t nn = meta->n_nodes;
    const int64_t ni = meta->n_internal;
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    for (int64_t j = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; j < nn; j += stride) {
        int l = 0;
        while (l < bits && meta->node_off[l + 1] <= j) ++l;
        const int64_t s = j - meta->node_off[l];
        uint64_t prefix = 0;
        if (l > 0) prefix = (ibfs_prefix[meta->lvl_int_off[l - 1] + s / 8] << 3) | static_cast<uint64_t>(s & 7);
        const int shift = 3 * (bits - l);
        const uint64_t start = prefix << shift;
        const uint64_t stop = start + (1ull << shift);
        const int64_t b = lower_bound_dev<uint64_t>(keys, n, start);
        const int64_t e = lower_bound_dev<uint64_t>(keys, n, stop);
        int32_t c = -1;
        if (l < bits) {
            const uint32_t off = meta->lvl_int_off[l], cnt = meta->lvl_cnt[l];
            const int64_t r = lower_bound_dev<uint64_t>(ibfs_prefix + off, cnt, prefix);
            if (r < cnt && ibfs_prefix[off + r] == prefix) c = static_cast<int32_t>(meta->node_off[l + 1] + 8 * r);
        }
        child[j] = c;
        node_key[j] = start;
        node_level[j] = static_cast<uint8_t>(l);
        sfc_node nd;
        nd.begin = static_cast<uint32_t>(b);
        nd.end = static_cast<uint32_t>(e);
        nd.lo[0] = nd.lo[1] = nd.lo[2] = INFINITY;
        nd.hi[0] = nd.hi[1] = nd.hi[2] = -INFINITY;
        if (c < 0) {
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
            const int64_t before = lower_bound_dev<uint64_t>(ipre_start, ni, start) - (l - zeros);
            const int64_t rank = digit_sum + 7 * before;
            if (rank >= 0 && rank <= 7 * ni) {
                leaves[rank] = start;
                counts[rank] = static_cast<uint32_t>(e - b);
            }
        }
        nodes[j] = nd;
        if (j == 0) leaves[7 * ni + 1] = 1ull << (3 * bits);
    }
}

__global__ __launch_bounds__(256) void k_internal_boxes(const LevelMeta *__restrict__ meta, int level,
                                                        const int32_t *__restrict__ int_node,
                                                        const int32_t *__restrict__ child, sfc_node *nodes) {
    const int64_t off = meta->lvl_int_off[level], cnt = meta->lvl_cnt[level];
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    for (int64_t k = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; k < cnt; k += stride) {
        const int32_t j = int_node[off + k];
        const int32_t c = child[j];
        sfc_node nd = nodes[j];
        for (int i = 0; i < 8; ++i) {
            const sfc_node ch = nodes[c + i];
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                nd.lo[a] = fminf(nd.lo[a], ch.lo[a]);
                nd.hi[a] = fmaxf(nd.hi[a], ch.hi[a]);
            }
        }
        nodes[j] = nd;
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

size_t tree_layout(int64_t n, uint32_t leaf_size, int bits, void *mem, sfc_octree *t) {
    const int64_t ni = internal_upper_bound(n, leaf_size, bits);
    const int64_t nl = 7 * ni + 1, nn = 8 * ni + 1;
    Carver c(mem);
    sfc_frame *frame = c.take<sfc_frame>(1);
    sfc_tree_info *info = c.take<sfc_tree_info>(1);
    float *points = c.take<float>(4 * static_cast<size_t>(n));
    uint64_t *keys = c.take<uint64_t>(n);
    uint32_t *perm = c.take<uint32_t>(n);
    uint64_t *leaves = c.take<uint64_t>(nl + 1);
    uint32_t *counts = c.take<uint32_t>(nl);
    sfc_node *nodes = c.take<sfc_node>(nn);
    int32_t *child = c.take<int32_t>(nn);
    uint64_t *node_key = c.take<uint64_t>(nn);
    uint8_t *node_level = c.take<uint8_t>(nn);
    if (t) {
        t->n = n;
        t->max_nodes = nn;
        t->max_leaves = nl;
        t->bits = bits;
        t->leaf_size = leaf_size;
        t->reserved = 0;
        t->frame = frame;
        t->info = info;
        t->points = points;
        t->keys = keys;
        t->perm = perm;
        t->leaves = leaves;
        t->counts = counts;
        t->nodes = nodes;
        t->child = child;
        t->node_key = node_key;
        t->node_level = node_level;
    }
    return c.bytes();
}

namespace {
struct BuildWs {
    int *bbox;
    uint64_t *keys_alt;
    uint32_t *vals_alt;
    void *radix_ws;
    uint32_t *gen;
    uint32_t *goff;
    void *scan_ws;
    LevelMeta *meta;
    uint64_t *ipre_prefix, *ipre_start, *lvkey, *lvkey_alt, *ibfs_prefix;
    uint32_t *iota, *iota_alt;
    int32_t *int_node;
    void *radix_ws_int;
};

size_t carve_build_ws(int64_t n, uint32_t leaf_size, int bits, void *mem, BuildWs *w) {
    const int64_t ni = internal_upper_bound(n, leaf_size, bits);
    const int64_t nic = ni > 0 ? ni : 1;
    Carver c(mem);
    BuildWs x;
    x.bbox = c.take<int>(8);
    x.keys_alt = c.take<uint64_t>(n);
    x.vals_alt = c.take<uint32_t>(n);
    x.radix_ws = c.take<char>(radix_ws_bytes(n));
    x.gen = c.take<uint32_t>(n);
    x.goff = c.take<uint32_t>(n + 1);
    x.scan_ws = c.take<char>(scan_ws_bytes(n));
    x.meta = c.take<LevelMeta>(1);
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

size_t build_ws_bytes(int64_t n, uint32_t leaf_size, int bits) { return carve_build_ws(n, leaf_size, bits, nullptr, nullptr); }

static int build_impl(const float *xyz, int64_t n, int curve, int bits, uint32_t N, sfc_octree *t, BuildWs &w,
                      hipStream_t s) {
    int rc;
    // Section 4: frame, codes (straight into the tree's key array), iota
    rc = launch_frame(xyz, n, curve, bits, t->frame, w.bbox, s);
    if (rc) return rc;
    rc = launch_encode(xyz, n, t->frame, t->keys, t->perm, s);
    if (rc) return rc;
    // Section 4, reorder step 2: sort (code, index)
    bool in_alt = false;
    rc = radix_sort_pairs(t->keys, t->perm, w.keys_alt, w.vals_alt, n, nullptr, 3 * bits, w.radix_ws, s, &in_alt);
    if (rc) return rc;
    if (in_alt && n > 0) {
        SFC_HIP_TRY(hipMemcpyAsync(t->keys, w.keys_alt, sizeof(uint64_t) * n, hipMemcpyDeviceToDevice, s));
        SFC_HIP_TRY(hipMemcpyAsync(t->perm, w.vals_alt, sizeof(uint32_t) * n, hipMemcpyDeviceToDevice, s));
    }
    float4 *pts = reinterpret_cast<float4 *>(t->points);
    if (n > 0) {
        k_gather<<<grid_for(n, 256, 1 << 16), 256, 0, s>>>(xyz, t->perm, n, pts);
        SFC_LAUNCH_CHECK("k_gather");
    }
    // Section 5.1: internal nodes in pre-order
    k_meta_init<<<1, 64, 0, s>>>(w.meta);
    SFC_LAUNCH_CHECK("k_meta_init");
    if (n > 0) {
        k_gen_count<<<grid_for(n, 256, 1 << 16), 256, 0, s>>>(t->keys, n, N, bits, w.gen);
        SFC_LAUNCH_CHECK("k_gen_count");
    }
    rc = scan_u32_to_u32(w.gen, n, w.goff, true, w.scan_ws, s);
    if (rc) return rc;
    if (n > 0) {
        k_emit_internal<<<grid_for(n, 256, 1 << 16), 256, 0, s>>>(t->keys, n, N, bits, w.goff, w.ipre_prefix,
                                                                  w.ipre_start, w.lvkey, w.iota, w.meta);
        SFC_LAUNCH_CHECK("k_emit_internal");
    }
    k_level_meta<<<1, 64, 0, s>>>(w.goff, n, bits, w.meta, t->info);
    SFC_LAUNCH_CHECK("k_level_meta");
    // breadth-first order: stable sort of the pre-order list by level
    const int64_t ni_ub = internal_upper_bound(n, N, bits);
    const uint32_t *order = w.iota;
    if (ni_ub > 0) {
        rc = radix_sort_pairs(w.lvkey, w.iota, w.lvkey_alt, w.iota_alt, ni_ub, &w.meta->n_internal, 8, w.radix_ws_int,
                              s, &in_alt);
        if (rc) return rc;
        order = in_alt ? w.iota_alt : w.iota;
        k_bfs_prefix<<<grid_for(ni_ub, 256, 4096), 256, 0, s>>>(w.ipre_prefix, order, w.meta, w.ibfs_prefix);
        SFC_LAUNCH_CHECK("k_bfs_prefix");
        k_internal_node_index<<<grid_for(ni_ub, 256, 4096), 256, 0, s>>>(w.ibfs_prefix, w.meta, bits, w.int_node);
        SFC_LAUNCH_CHECK("k_internal_node_index");
    }
    const int64_t nn_ub = 8 * ni_ub + 1;
    k_nodes<<<grid_for(nn_ub, 256, 8192), 256, 0, s>>>(t->keys, pts, n, bits, w.meta, w.ibfs_prefix, w.ipre_start,
                                                         t->nodes, t->child, t->node_key, t->node_level, t->leaves,
                                                         t->counts);
    SFC_LAUNCH_CHECK("k_nodes");
    const int64_t per_level = n / (static_cast<int64_t>(N) + 1);
    for (int l = bits - 1; l >= 0; --l) {
        int64_t ub = per_level;
        if (l < 21 && (int64_t(1) << (3 * l)) < ub) ub = int64_t(1) << (3 * l);
        if (ub <= 0) continue;
        k_internal_boxes<<<grid_for(ub, 256, 2048), 256, 0, s>>>(w.meta, l, w.int_node, t->child, t->nodes);
        SFC_LAUNCH_CHECK("k_internal_boxes");
    }
    return SFC_OK;
}

}  // namespace sfc

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

extern "C" int build_linear_octree(const float *xyz, int64_t n, int curve, int bits, uint32_t leaf_size,
                                   void *tree_mem, size_t tree_bytes, sfc_octree *tree_out, void *ws,
                                   size_t *ws_bytes, void *stream) {
    using namespace sfc;
    if (!ws_bytes || n < 0 || n > 0xFFFFFFFFll || leaf_size < 1 || bits < 1 || bits > 21 ||
        (curve != SFC_MORTON && curve != SFC_HILBERT)) {
        set_error("build_linear_octree: invalid argument (n=%lld bits=%d curve=%d leaf_size=%u)", (long long)n, bits,
                  curve, leaf_size);
        return SFC_EINVAL;
    }
    if (8 * internal_upper_bound(n, leaf_size, bits) + 1 > 0x7FFFFFFFll) {
        set_error("build_linear_octree: node bound exceeds 2^31 - 1; raise leaf_size");
        return SFC_ENOTSUP;
    }
    const size_t need = build_ws_bytes(n, leaf_size, bits);
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
    sfc_octree t;
    tree_layout(n, leaf_size, bits, tree_mem, &t);
    t.curve = curve;
    BuildWs w;
    carve_build_ws(n, leaf_size, bits, ws, &w);
    const int rc = build_impl(xyz, n, curve, bits, leaf_size, &t, w, static_cast<hipStream_t>(stream));
    if (rc == SFC_OK) *tree_out = t;
    return rc;
}

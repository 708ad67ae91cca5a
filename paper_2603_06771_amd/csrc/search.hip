// Section 3.2 fixed-radius search with the pruning of Section 5.1
// (neighboursPrune), and Section 3.3 k-nearest-neighbour search, on the
// linear octree.
//
// GPU mapping (one wave = one workgroup):
//  * A group is 64 consecutive queries; for cloud queries these are 64
//    consecutive points of the curve, so their union is compact.  Lane i owns
//    query i of the group.
//  * Traversal: the wave walks the tree from the root with an LDS stack, 64
//    nodes per step (one per lane).  A node is kept when it may hold a
//    neighbour of SOME query of the group (its box against the group's box
//    with the kernel's norm); kept leaves become candidates.
//  * Sweep: the candidates' points are staged in LDS (coalesced loads), then
//    every candidate is classified per query against the node's tight box:
//    disjoint (skip), contained (all its points are neighbours: Section 5.1
//    step 1a) or partial (test point by point: step 2).  The point loop reads
//    LDS with a wave-uniform address (broadcast) and each lane tests its own
//    query.
//  * Exactness: boxes are the tight fp32 boxes of the node's points.  fp32
//    subtraction, product and sum are monotone, so a box corner bounds every
//    point's fp32 expression from the same side; the shortcuts therefore give
//    bit-identical sets to testing every point.
//  * Count pass writes per-query counts; fill pass writes the original
//    indices: each lane appends to its own LDS row and full rows are flushed
//    to HBM as one coalesced 64-lane store.
//  * k-NN: lane-owned top-k of (d2, index) keys in registers (descending,
//    so the current k-th is always register 0), seeded with an upper bound
//    of the k-th distance taken from the query's k curve neighbours.
// Roofline: the fill pass is bound by HBM writes of the indices for large
// neighbourhoods and by VALU (candidate tests) for small ones.
#include <cmath>

#include "codes.hpp"
#include "internal.hpp"

namespace sfc {

namespace {

constexpr int kStack = 1024;
constexpr int kCand = 128;
constexpr int kStage = 512;
constexpr int kRowCap = 64;
constexpr int kChunk = 32;

template <int KERNEL>
__device__ __forceinline__ bool point_hit(const float4 &p, float qx, float qy, float qz, float r, float r2) {
    const float dx = fsub(p.x, qx), dy = fsub(p.y, qy);
    if constexpr (KERNEL == SFC_SPHERE) {
        const float dz = fsub(p.z, qz);
        return fadd(fadd(fmul(dx, dx), fmul(dy, dy)), fmul(dz, dz)) < r2;
    } else if constexpr (KERNEL == SFC_CIRCLE) {
        return fadd(fmul(dx, dx), fmul(dy, dy)) < r2;
    } else if constexpr (KERNEL == SFC_CUBE) {
        const float dz = fsub(p.z, qz);
        return fabsf(dx) < r && fabsf(dy) < r && fabsf(dz) < r;
    } else {
        return fabsf(dx) < r && fabsf(dy) < r;
    }
}

__device__ __forceinline__ float dist2(const float4 &p, float qx, float qy, float qz) {
    const float dx = fsub(p.x, qx), dy = fsub(p.y, qy), dz = fsub(p.z, qz);
    return fadd(fadd(fmul(dx, dx), fmul(dy, dy)), fmul(dz, dz));
}

// nearest and farthest |fp32 difference| between the query coordinate and a
// coordinate of the box [lo, hi]
__device__ __forceinline__ void axis_range(float lo, float hi, float q, float &nr, float &fr) {
    const float dlo = fsub(lo, q), dhi = fsub(hi, q);
    nr = dlo > 0.0f ? dlo : (dhi < 0.0f ? -dhi : 0.0f);
    fr = fmaxf(fabsf(dlo), fabsf(dhi));
}

// 0: no point of the box is a neighbour; 1: every point is; 2: test points
template <int KERNEL>
__device__ __forceinline__ int classify(const sfc_node &b, float qx, float qy, float qz, float r, float r2) {
    float nx, fx, ny, fy;
    axis_range(b.lo[0], b.hi[0], qx, nx, fx);
    axis_range(b.lo[1], b.hi[1], qy, ny, fy);
    if constexpr (KERNEL == SFC_SPHERE || KERNEL == SFC_CUBE) {
        float nz, fz;
        axis_range(b.lo[2], b.hi[2], qz, nz, fz);
        if constexpr (KERNEL == SFC_SPHERE) {
            const float near2 = fadd(fadd(fmul(nx, nx), fmul(ny, ny)), fmul(nz, nz));
            if (!(near2 < r2)) return 0;
            const float far2 = fadd(fadd(fmul(fx, fx), fmul(fy, fy)), fmul(fz, fz));
            return far2 < r2 ? 1 : 2;
        } else {
            if (!(nx < r && ny < r && nz < r)) return 0;
            return (fx < r && fy < r && fz < r) ? 1 : 2;
        }
    } else if constexpr (KERNEL == SFC_CIRCLE) {
        const float near2 = fadd(fmul(nx, nx), fmul(ny, ny));
        if (!(near2 < r2)) return 0;
        const float far2 = fadd(fmul(fx, fx), fmul(fy, fy));
        return far2 < r2 ? 1 : 2;
    } else {
        if (!(nx < r && ny < r)) return 0;
        return (fx < r && fy < r) ? 1 : 2;
    }
}

// per-axis fp32 gap between the node box and the group box (0 if they overlap)
__device__ __forceinline__ float gap(float lo, float hi, float glo, float ghi) {
    return fmaxf(fmaxf(fsub(lo, ghi), fsub(glo, hi)), 0.0f);
}

// may the node hold a neighbour of some query inside the group box?
template <int KERNEL>
__device__ __forceinline__ bool group_may_hit(const sfc_node &b, const float *glo, const float *ghi, float r,
                                              float r2) {
    const float gx = gap(b.lo[0], b.hi[0], glo[0], ghi[0]);
    const float gy = gap(b.lo[1], b.hi[1], glo[1], ghi[1]);
    if constexpr (KERNEL == SFC_SPHERE) {
        const float gz = gap(b.lo[2], b.hi[2], glo[2], ghi[2]);
        return fadd(fadd(fmul(gx, gx), fmul(gy, gy)), fmul(gz, gz)) < r2;
    } else if constexpr (KERNEL == SFC_CIRCLE) {
        return fadd(fmul(gx, gx), fmul(gy, gy)) < r2;
    } else if constexpr (KERNEL == SFC_CUBE) {
        const float gz = gap(b.lo[2], b.hi[2], glo[2], ghi[2]);
        return gx < r && gy < r && gz < r;
    } else {
        return gx < r && gy < r;
    }
}

struct Query {
    float x, y, z;
    bool valid;
};

__device__ __forceinline__ Query load_query(const float *queries, const float4 *pts, int64_t row, int64_t nq) {
    Query q{0.0f, 0.0f, 0.0f, row < nq};
    if (q.valid) {
        if (queries) {
            q.x = queries[3 * row];
            q.y = queries[3 * row + 1];
            q.z = queries[3 * row + 2];
        } else {
            const float4 p = pts[row];
            q.x = p.x;
            q.y = p.y;
            q.z = p.z;
        }
    }
    return q;
}

__device__ __forceinline__ void group_box(const Query &q, float *glo, float *ghi) {
    glo[0] = wave_min(q.valid ? q.x : INFINITY);
    glo[1] = wave_min(q.valid ? q.y : INFINITY);
    glo[2] = wave_min(q.valid ? q.z : INFINITY);
    ghi[0] = wave_max(q.valid ? q.x : -INFINITY);
    ghi[1] = wave_max(q.valid ? q.y : -INFINITY);
    ghi[2] = wave_max(q.valid ? q.z : -INFINITY);
}

// Shared LDS of one wave: traversal stack, candidate nodes, staged points.
struct WaveLds {
    int stack[kStack];
    sfc_node cand[kCand];
    float4 pts[kStage];
    uint32_t cstart[65];
};

// Walks the tree; each time the candidate list fills up (or the walk ends)
// calls sweep(ncand).  ACCEPT(node) decides whether the wave keeps a node.
template <typename Accept, typename Sweep>
__device__ __forceinline__ void traverse(WaveLds &L, const sfc_node *__restrict__ nodes,
                                         const int32_t *__restrict__ child, Accept accept, Sweep sweep) {
    const int lane = lane_id();
    if (lane == 0) L.stack[0] = 0;
    int sp = 1, ncand = 0;
    __syncthreads();
    while (sp > 0) {
        int take = (kStack - sp) / 7;
        if (take > kWave) take = kWave;
        if (take > sp) take = sp;
        if (take < 1) take = 1;
        const int node = lane < take ? L.stack[sp - take + lane] : -1;
        sp -= take;
        __syncthreads();
        sfc_node nd;
        int32_t ch = -1;
        bool keep = false;
        if (node >= 0) {
            nd = nodes[node];
            ch = child[node];
            keep = nd.end > nd.begin && accept(nd);
        }
        const bool internal = keep && ch >= 0;
        const uint64_t m_int = ballot(internal);
        int allow = (kStack - sp) / 8;
        const int n_int = __popcll(m_int);
        if (allow > n_int) allow = n_int;
        const int rk = static_cast<int>(rank_below(m_int));
        const bool push = internal && rk < allow;
        if (push) {
#pragma unroll
            for (int c = 0; c < 8; ++c) L.stack[sp + 8 * rk + c] = ch + c;
        }
        sp += 8 * allow;
        const bool cand = keep && !push;  // leaves, and internal nodes that found no stack room
        const uint64_t m_c = ballot(cand);
        if (cand) L.cand[ncand + rank_below(m_c)] = nd;
        ncand += __popcll(m_c);
        __syncthreads();
        if (ncand > kCand - kWave || (sp == 0 && ncand > 0)) {
            sweep(ncand);
            ncand = 0;
        }
    }
}

// Stages candidates [c0, c0 + nb) (their points, total <= kStage) into L.pts;
// L.cstart[i] is the first staged slot of candidate c0 + i.
__device__ __forceinline__ void stage_points(WaveLds &L, const float4 *__restrict__ pts, int c0, int nb,
                                             uint32_t total) {
    const int lane = lane_id();
    for (uint32_t p = lane; p < total; p += kWave) {
        int lo = 0, hi = nb - 1;  // last candidate whose start <= p
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (L.cstart[mid] <= p)
                lo = mid;
            else
                hi = mid - 1;
        }
        L.pts[p] = pts[L.cand[c0 + lo].begin + (p - L.cstart[lo])];
    }
    __syncthreads();
}

// Batches the candidate list into stageable groups and calls
// visit(node, staged_points, count) for every candidate.  A candidate larger
// than the staging area is visited in slices.
template <typename Visit>
__device__ __forceinline__ void sweep_candidates(WaveLds &L, const float4 *__restrict__ pts, int ncand, Visit visit) {
    const int lane = lane_id();
    int c0 = 0;
    while (c0 < ncand) {
        const int m = min(kWave, ncand - c0);
        uint32_t sz = 0;
        if (lane < m) sz = L.cand[c0 + lane].end - L.cand[c0 + lane].begin;
        const uint32_t incl = wave_inclusive_sum(sz);
        const int nb = __popcll(ballot(lane < m && incl <= static_cast<uint32_t>(kStage)));
        if (nb == 0) {
            // one candidate bigger than the staging area: slice it
            const sfc_node nd = L.cand[c0];
            for (uint32_t s0 = nd.begin; s0 < nd.end; s0 += kStage) {
                const uint32_t len = min(static_cast<uint32_t>(kStage), nd.end - s0);
                __syncthreads();
                for (uint32_t p = lane; p < len; p += kWave) L.pts[p] = pts[s0 + p];
                __syncthreads();
                sfc_node part = nd;
                part.begin = s0;
                part.end = s0 + len;
                visit(part, L.pts, len);
            }
            __syncthreads();
            c0 += 1;
            continue;
        }
        if (lane < nb) L.cstart[lane] = incl - sz;
        const uint32_t total = __shfl(incl, nb - 1);
        __syncthreads();
        stage_points(L, pts, c0, nb, total);
        for (int o = 0; o < nb; ++o) {
            const sfc_node nd = L.cand[c0 + o];
            visit(nd, L.pts + L.cstart[o], nd.end - nd.begin);
        }
        __syncthreads();
        c0 += nb;
    }
}

struct RadiusArgs {
    const sfc_node *nodes;
    const int32_t *child;
    const float4 *pts;
    const float *queries;
    int64_t nq;
    int64_t groups;
    float r;
    uint32_t flags;
    uint32_t *counts;
    const uint64_t *offsets;
    uint32_t *indices;
    uint64_t capacity;
};

}  // namespace

template <int KERNEL>
__global__ __launch_bounds__(64) void k_radius_count(RadiusArgs a) {
    __shared__ WaveLds L;
    const int64_t g = xcd_item(blockIdx.x, gridDim.x);
    if (g >= a.groups) return;
    const int64_t row = g * kWave + lane_id();
    const Query q = load_query(a.queries, a.pts, row, a.nq);
    float glo[3], ghi[3];
    group_box(q, glo, ghi);
    const float r = a.r, r2 = fmul(r, r);
    const bool prune = !(a.flags & SFC_NO_PRUNE);
    uint32_t cnt = 0;
    auto accept = [&](const sfc_node &nd) { return group_may_hit<KERNEL>(nd, glo, ghi, r, r2); };
    auto visit = [&](const sfc_node &nd, const float4 *sp, uint32_t len) {
        int cls = q.valid ? classify<KERNEL>(nd, q.x, q.y, q.z, r, r2) : 0;
        if (cls == 1 && !prune) cls = 2;
        if (cls == 1) cnt += len;
        if (ballot(cls == 2)) {
            const bool test = cls == 2;
            for (uint32_t j = 0; j < len; ++j) cnt += (test && point_hit<KERNEL>(sp[j], q.x, q.y, q.z, r, r2)) ? 1u : 0u;
        }
    };
    auto sweep = [&](int ncand) { sweep_candidates(L, a.pts, ncand, visit); };
    traverse(L, a.nodes, a.child, accept, sweep);
    if (q.valid) a.counts[row] = cnt;
}

template <int KERNEL>
__global__ __launch_bounds__(64) void k_radius_fill(RadiusArgs a) {
    __shared__ WaveLds L;
    __shared__ uint32_t s_rows[kWave * (kRowCap + 1)];
    const int64_t g = xcd_item(blockIdx.x, gridDim.x);
    if (g >= a.groups) return;
    if (a.offsets[a.nq] > a.capacity) return;  // caller's buffer too small: write nothing
    const int lane = lane_id();
    const int64_t row = g * kWave + lane;
    const Query q = load_query(a.queries, a.pts, row, a.nq);
    float glo[3], ghi[3];
    group_box(q, glo, ghi);
    const float r = a.r, r2 = fmul(r, r);
    const bool prune = !(a.flags & SFC_NO_PRUNE);
    uint64_t gpos = q.valid ? a.offsets[row] : 0;
    const uint64_t gend = q.valid ? a.offsets[row + 1] : 0;  // never write past the counted row
    int nb = 0;
    uint32_t *myrow = s_rows + lane * (kRowCap + 1);
    uint32_t *out = a.indices;

    // write out every row holding more than `limit` staged entries
    auto flush = [&](int limit) {
        uint64_t m = ballot(nb > limit);
        while (m) {
            const int l = __ffsll(static_cast<long long>(m)) - 1;
            m &= m - 1;
            const int cl = __shfl(nb, l);
            const uint64_t base = __shfl(gpos, l);
            const uint64_t end = __shfl(gend, l);
            if (lane < cl && base + lane < end) out[base + lane] = s_rows[l * (kRowCap + 1) + lane];
            if (lane == l) {
                gpos += static_cast<uint64_t>(nb);
                nb = 0;
            }
        }
    };
    auto accept = [&](const sfc_node &nd) { return group_may_hit<KERNEL>(nd, glo, ghi, r, r2); };
    auto visit = [&](const sfc_node &nd, const float4 *sp, uint32_t len) {
        int cls = q.valid ? classify<KERNEL>(nd, q.x, q.y, q.z, r, r2) : 0;
        if (cls == 1 && !prune) cls = 2;
        if (!ballot(cls != 0)) return;
        for (uint32_t j0 = 0; j0 < len; j0 += kChunk) {
            const uint32_t jn = min(len - j0, static_cast<uint32_t>(kChunk));
            flush(kRowCap - static_cast<int>(jn));
            for (uint32_t j = j0; j < j0 + jn; ++j) {
                const float4 p = sp[j];
                const bool h = cls == 1 || (cls == 2 && point_hit<KERNEL>(p, q.x, q.y, q.z, r, r2));
                if (h) myrow[nb++] = __float_as_uint(p.w);
            }
        }
    };
    auto sweep = [&](int ncand) { sweep_candidates(L, a.pts, ncand, visit); };
    traverse(L, a.nodes, a.child, accept, sweep);
    flush(0);
}

__global__ void k_zero_rows(uint32_t *counts, uint64_t *offsets, int64_t nq) {
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i <= nq; i += stride) {
        if (i < nq && counts) counts[i] = 0;
        offsets[i] = 0;
    }
}

// ------------------------------------------------------------------ k-NN
namespace {

struct KnnArgs {
    const sfc_node *nodes;
    const int32_t *child;
    const float4 *pts;
    const uint64_t *keys;
    const sfc_frame *frame;
    int64_t n;
    const float *queries;
    int64_t nq;
    int64_t groups;
    int k;
    uint32_t *idx;
    float *d2;
};

constexpr int64_t kPad = static_cast<int64_t>((0x7F800000ull << 32) | 0xFFFFFFFFull);  // (+inf, no index)

__device__ __forceinline__ int64_t pack(float d, uint32_t i) {
    return static_cast<int64_t>((static_cast<uint64_t>(__float_as_uint(d)) << 32) | i);
}

template <typename T>
__device__ __forceinline__ int64_t lower_bound_keys(const T *a, int64_t n, T v) {
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

template <int KMAX>
__global__ __launch_bounds__(64) void k_knn(KnnArgs a) {
    __shared__ WaveLds L;
    const int64_t g = xcd_item(blockIdx.x, gridDim.x);
    if (g >= a.groups) return;
    const int lane = lane_id();
    const int64_t row = g * kWave + lane;
    const Query q = load_query(a.queries, a.pts, row, a.nq);
    const int k = a.k;

    // upper bound of the k-th distance: the farthest of the k curve neighbours
    float tau = INFINITY;
    if (q.valid && a.n >= k) {
        int64_t pos = row;
        if (a.queries) pos = lower_bound_keys<uint64_t>(a.keys, a.n, point_key(q.x, q.y, q.z, *a.frame));
        int64_t s = pos - k / 2;
        if (s > a.n - k) s = a.n - k;
        if (s < 0) s = 0;
        tau = 0.0f;
        for (int i = 0; i < k; ++i) tau = fmaxf(tau, dist2(a.pts[s + i], q.x, q.y, q.z));
    }
    float glo[3], ghi[3];
    group_box(q, glo, ghi);
    const float R2 = wave_max(q.valid ? tau : 0.0f);
    const float R2open = R2 < INFINITY ? nextafterf(R2, INFINITY) : INFINITY;

    int64_t best[KMAX];
#pragma unroll
    for (int i = 0; i < KMAX; ++i) best[i] = i < k ? kPad : int64_t(-1);

    auto accept = [&](const sfc_node &nd) { return group_may_hit<SFC_SPHERE>(nd, glo, ghi, 0.0f, R2open); };
    auto visit = [&](const sfc_node &nd, const float4 *sp, uint32_t len) {
        float thr = tau;
        const float kth = __uint_as_float(static_cast<uint32_t>(static_cast<uint64_t>(best[0]) >> 32));
        if (kth < thr) thr = kth;
        bool live = false;
        if (q.valid) {
            float nx, fx, ny, fy, nz, fz;
            axis_range(nd.lo[0], nd.hi[0], q.x, nx, fx);
            axis_range(nd.lo[1], nd.hi[1], q.y, ny, fy);
            axis_range(nd.lo[2], nd.hi[2], q.z, nz, fz);
            const float near2 = fadd(fadd(fmul(nx, nx), fmul(ny, ny)), fmul(nz, nz));
            live = !(near2 > thr);  // equality kept: an equal d2 with a smaller index may enter
        }
        if (!ballot(live)) return;
        for (uint32_t j = 0; j < len; ++j) {
            const float4 p = sp[j];
            const float d = dist2(p, q.x, q.y, q.z);
            const int64_t x = pack(d, __float_as_uint(p.w));
            if (live && d <= tau && x < best[0]) {
#pragma unroll
                for (int i = 0; i < KMAX; ++i) {
                    const int64_t nxt = (i + 1 < KMAX) ? best[i + 1] : int64_t(-1);
                    best[i] = nxt > x ? nxt : (best[i] > x ? x : best[i]);
                }
            }
        }
    };
    auto sweep = [&](int ncand) { sweep_candidates(L, a.pts, ncand, visit); };
    traverse(L, a.nodes, a.child, accept, sweep);
    if (q.valid) {
        uint32_t *oi = a.idx + row * k;
        float *od = a.d2 + row * k;
#pragma unroll
        for (int i = 0; i < KMAX; ++i) {
            if (i < k) {
                const uint64_t v = static_cast<uint64_t>(best[i]);
                oi[k - 1 - i] = static_cast<uint32_t>(v);
                od[k - 1 - i] = __uint_as_float(static_cast<uint32_t>(v >> 32));
            }
        }
    }
}

}  // namespace sfc

// -------------------------------------------------------------- C ABI
using namespace sfc;

static bool tree_ok(const sfc_octree *t) {
    return t && t->nodes && t->child && t->points && t->keys && t->frame && t->n >= 0;
}

extern "C" int radius_search(const sfc_octree *tree, const float *queries, int64_t nq, int kernel, float r,
                             uint32_t *counts, uint64_t *offsets, uint32_t *indices, uint64_t capacity,
                             uint32_t flags, void *ws, size_t *ws_bytes, void *stream) {
    if (!ws_bytes || !tree_ok(tree) || kernel < 0 || kernel > 3 || nq < 0 || !offsets || !counts ||
        (!queries && nq != tree->n) || std::isnan(r) || std::isinf(r)) {
        set_error("radius_search: invalid argument");
        return SFC_EINVAL;
    }
    const size_t need = scan_ws_bytes(nq);
    if (!ws) {
        *ws_bytes = need;
        return SFC_OK;
    }
    if (*ws_bytes < need || (reinterpret_cast<uintptr_t>(ws) & 255u)) {
        set_error("radius_search: workspace needs %zu bytes, 256-aligned", need);
        return SFC_EWORKSPACE;
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (nq == 0 || !(r > 0.0f)) {
        if (!(flags & SFC_REUSE_COUNTS)) {
            k_zero_rows<<<grid_for(nq + 1, 256, 4096), 256, 0, s>>>(counts, offsets, nq);
            SFC_LAUNCH_CHECK("k_zero_rows");
        }
        return SFC_OK;
    }
    RadiusArgs a;
    a.nodes = tree->nodes;
    a.child = tree->child;
    a.pts = reinterpret_cast<const float4 *>(tree->points);
    a.queries = queries;
    a.nq = nq;
    a.groups = (nq + kWave - 1) / kWave;
    a.r = r;
    a.flags = flags;
    a.counts = counts;
    a.offsets = offsets;
    a.indices = indices;
    a.capacity = capacity;
    const unsigned grid = static_cast<unsigned>(xcd_grid(a.groups));
    if (!(flags & SFC_REUSE_COUNTS)) {
        switch (kernel) {
        case SFC_SPHERE: k_radius_count<SFC_SPHERE><<<grid, 64, 0, s>>>(a); break;
        case SFC_CIRCLE: k_radius_count<SFC_CIRCLE><<<grid, 64, 0, s>>>(a); break;
        case SFC_CUBE: k_radius_count<SFC_CUBE><<<grid, 64, 0, s>>>(a); break;
        default: k_radius_count<SFC_SQUARE><<<grid, 64, 0, s>>>(a); break;
        }
        SFC_LAUNCH_CHECK("k_radius_count");
        const int rc = scan_u32_to_u64(counts, nq, offsets, true, ws, s);
        if (rc) return rc;
    }
    if (indices) {
        switch (kernel) {
        case SFC_SPHERE: k_radius_fill<SFC_SPHERE><<<grid, 64, 0, s>>>(a); break;
        case SFC_CIRCLE: k_radius_fill<SFC_CIRCLE><<<grid, 64, 0, s>>>(a); break;
        case SFC_CUBE: k_radius_fill<SFC_CUBE><<<grid, 64, 0, s>>>(a); break;
        default: k_radius_fill<SFC_SQUARE><<<grid, 64, 0, s>>>(a); break;
        }
        SFC_LAUNCH_CHECK("k_radius_fill");
    }
    return SFC_OK;
}

extern "C" int knn_search(const sfc_octree *tree, const float *queries, int64_t nq, int k, uint32_t *idx, float *d2,
                          void *ws, size_t *ws_bytes, void *stream) {
    if (!ws_bytes || !tree_ok(tree) || nq < 0 || k < 1 || (!queries && nq != tree->n) || (nq > 0 && (!idx || !d2))) {
        set_error("knn_search: invalid argument");
        return SFC_EINVAL;
    }
    if (k > 32) {
        set_error("knn_search: k = %d above 32 is not supported", k);
        return SFC_ENOTSUP;
    }
    const size_t need = 256;
    if (!ws) {
        *ws_bytes = need;
        return SFC_OK;
    }
    if (*ws_bytes < need) {
        set_error("knn_search: workspace needs %zu bytes", need);
        return SFC_EWORKSPACE;
    }
    if (nq == 0) return SFC_OK;
    hipStream_t s = static_cast<hipStream_t>(stream);
    KnnArgs a;
    a.nodes = tree->nodes;
    a.child = tree->child;
    a.pts = reinterpret_cast<const float4 *>(tree->points);
    a.keys = tree->keys;
    a.frame = tree->frame;
    a.n = tree->n;
    a.queries = queries;
    a.nq = nq;
    a.groups = (nq + kWave - 1) / kWave;
    a.k = k;
    a.idx = idx;
    a.d2 = d2;
    const unsigned grid = static_cast<unsigned>(xcd_grid(a.groups));
    if (k <= 8)
        k_knn<8><<<grid, 64, 0, s>>>(a);
    else if (k <= 16)
        k_knn<16><<<grid, 64, 0, s>>>(a);
    else
        k_knn<32><<<grid, 64, 0, s>>>(a);
    SFC_LAUNCH_CHECK("k_knn");
    return SFC_OK;
}

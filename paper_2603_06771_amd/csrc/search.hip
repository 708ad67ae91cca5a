// Section 3.2 fixed-radius search with the pruning of Section 5.1
// (neighboursPrune), and Section 3.3 k-nearest-neighbour search, on the
// linear octree.
//
// GPU mapping (one wave = one workgroup, so LDS is ordered with
// wavefront-scope fences, never a workgroup barrier):
//  * A group is 64 consecutive queries; for cloud queries these are 64
//    consecutive points of the curve, so their union is compact.  Lane i owns
//    query i of the group.  The group is cut into segments where consecutive
//    queries jump apart; the segment boxes drive every shortcut below.
//  * Traversal: the wave walks the tree with an LDS stack, 64 nodes per step
//    (one per lane), from the root or, for cloud queries, from the deepest
//    node whose cell holds the group's whole reach.  A node is kept when it
//    may hold a neighbour of SOME query (its box against the segment boxes
//    with the kernel's norm); kept leaves become candidates.
//  * Sweep: candidates are classified (lane = candidate) against each
//    segment box: disjoint (skip), contained for every query of the segment
//    (counted without touching the points: Section 5.1 step 1a) or partial.
//    Points of partial candidates are staged in LDS (coalesced loads, points
//    no segment can reach dropped, carried over between candidate batches),
//    then every lane tests its own query against every staged point with a
//    wave-uniform LDS address (broadcast; step 2).
//  * Exactness: boxes are the tight fp32 boxes of the node's points.  fp32
//    subtraction, product and sum are monotone, so a box corner bounds every
//    point's fp32 expression from the same side; the shortcuts therefore give
//    bit-identical sets to testing every point.
//  * Count pass writes per-query counts; fill pass writes the original
//    indices: each lane appends the slots of its hits among the staged points
//    to its own LDS row (one byte each), and rows are flushed to HBM with
//    coalesced half-wave stores when they fill up and at the end of every
//    staging round.
//  * Recorded hits (optional): the count pass also stores, per group, every
//    staged point that hits some lane (its index and the 64-bit mask of the
//    lanes it hits, in staging order); the fill then writes the rows from
//    these records without traversal or distance tests, in the same order.
//  * k-NN: lane-owned top-k (k <= 64) of (d2, index) keys in registers
//    (descending, so the current k-th is always register 0), seeded with an
//    upper bound of the k-th distance taken from the query's curve
//    neighbours; larger k takes one query per wave with an LDS buffer.
// Roofline: the fill pass is bound by HBM writes of the indices for large
// neighbourhoods and by VALU (candidate tests) for small ones.
#include <algorithm>
#include <cmath>
#include <cstddef>
#include <cstring>
#include <mutex>
#include <type_traits>
#include <unordered_map>
#include <utility>
#include <vector>

#include "codes.hpp"
#include "internal.hpp"

namespace sfc {

namespace {

// Tile parameters (overridable at build time for tuning sweeps).
#ifndef SFC_STACK
#define SFC_STACK 256
#endif
#ifndef SFC_CAND
#define SFC_CAND 128
#endif
#ifndef SFC_STAGE
#define SFC_STAGE 128
#endif
#ifndef SFC_ROWCAP
#define SFC_ROWCAP 32
#endif
#ifndef SFC_REC_BATCH
#define SFC_REC_BATCH 4
#endif
#ifndef SFC_REC_LONG_MEAN
#define SFC_REC_LONG_MEAN 64
#endif
#ifndef SFC_REC_CAP
#define SFC_REC_CAP 4096
#endif
#ifndef SFC_CHUNK
#define SFC_CHUNK 16
#endif
#ifndef SFC_REC_ROWBLK
#define SFC_REC_ROWBLK 20
#endif
constexpr int kStack = SFC_STACK;     // traversal stack entries
constexpr int kCand = SFC_CAND;       // candidate nodes held before a sweep
constexpr int kStage = SFC_STAGE;     // points staged per round
constexpr int kRowCap = SFC_ROWCAP;   // fill: staged output entries per query
constexpr int kChunk = SFC_CHUNK;     // fill: points swept between flush checks
constexpr int kSegMax = 8;            // query segments per wave
constexpr float kJumpSteps = 5.0f;    // radius search: segment cut distance in mean curve steps (at least)
constexpr int kRecCap = SFC_REC_CAP;  // recorded hits per group of 64 queries
constexpr uint32_t kRecOverflow = 0xFFFFFFFFu;        // rec_n: the group's records did not fit (or it was deferred)
constexpr uint32_t kRecLongRows = 0x40000000u;        // rec_n flag: the group takes the long-row fill
constexpr uint32_t kRecLongMean = SFC_REC_LONG_MEAN;  // mean row length from which a group takes it
static_assert(kRecCap < static_cast<int>(kRecLongRows), "record count and form flag share rec_n");
static_assert(kChunk <= kRowCap && kRowCap <= 32 && kCand >= 2 * 64 && kStage % 4 == 0 && kStage >= 64 && kStage <= 256,
              "tile parameters");

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
        return (fabsf(dx) < r) & (fabsf(dy) < r) & (fabsf(dz) < r);
    } else {
        return (fabsf(dx) < r) & (fabsf(dy) < r);
    }
}

// point_hit as a lane mask, taken straight from the comparisons (ordered
// less-than, as `<` is), so a caller that needs the mask of the wave's hits
// gets it without turning every lane's result into a 0/1 value first.  Every
// lane of the wave must be active.
template <int KERNEL>
__device__ __forceinline__ uint64_t hit_mask(const float4 &p, float qx, float qy, float qz, float r, float r2) {
    constexpr int kOlt = 4;  // the ordered less-than predicate of the compare intrinsic
    const float dx = fsub(p.x, qx), dy = fsub(p.y, qy);
    if constexpr (KERNEL == SFC_SPHERE) {
        const float dz = fsub(p.z, qz);
        return __builtin_amdgcn_fcmpf(fadd(fadd(fmul(dx, dx), fmul(dy, dy)), fmul(dz, dz)), r2, kOlt);
    } else if constexpr (KERNEL == SFC_CIRCLE) {
        return __builtin_amdgcn_fcmpf(fadd(fmul(dx, dx), fmul(dy, dy)), r2, kOlt);
    } else if constexpr (KERNEL == SFC_CUBE) {
        const float dz = fsub(p.z, qz);
        return __builtin_amdgcn_fcmpf(fabsf(dx), r, kOlt) & __builtin_amdgcn_fcmpf(fabsf(dy), r, kOlt) &
               __builtin_amdgcn_fcmpf(fabsf(dz), r, kOlt);
    } else {
        return __builtin_amdgcn_fcmpf(fabsf(dx), r, kOlt) & __builtin_amdgcn_fcmpf(fabsf(dy), r, kOlt);
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
            if (!((nx < r) & (ny < r) & (nz < r))) return 0;
            return ((fx < r) & (fy < r) & (fz < r)) ? 1 : 2;
        }
    } else if constexpr (KERNEL == SFC_CIRCLE) {
        const float near2 = fadd(fmul(nx, nx), fmul(ny, ny));
        if (!(near2 < r2)) return 0;
        const float far2 = fadd(fmul(fx, fx), fmul(fy, fy));
        return far2 < r2 ? 1 : 2;
    } else {
        if (!((nx < r) & (ny < r))) return 0;
        return ((fx < r) & (fy < r)) ? 1 : 2;
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
        return (gx < r) & (gy < r) & (gz < r);
    } else {
        return (gx < r) & (gy < r);
    }
}

struct Query {
    float x, y, z;
    bool valid;
};

// Shared LDS of one wave: traversal stack, candidate nodes, staged points.
struct WaveLds {
    static constexpr int kPts = kStage;
    int stack[kStack];
    int cand[kCand];         // candidate nodes (indices)
    uint32_t cbeg[kCand];    // their point ranges
    uint32_t cend[kCand];
    sfc_node cnode[kCand];   // and the nodes themselves (per-lane pruning reads them in turn)
    float4 pts[kStage];
    uint8_t owner[kStage];   // candidate (within the batch) of each staged point
    uint32_t cincl[kWave];   // inclusive prefix of staged sizes of the batch
    float seg[kSegMax][6];   // boxes of the query segments
};

// Splits the wave's 64 queries into at most kSegMax runs of consecutive
// queries, cutting where two consecutive queries are more than `jump` apart
// (the largest such steps first).  A space-filling curve visits empty space
// between occupied regions, so consecutive points can be far apart; one box
// over such a group would cover the whole gap.  With step_factor > 0 the
// cut distance grows towards step_factor times the group's mean step (the
// point spacing along the curve), up to twice `jump`, so groups whose
// radius is small next to the spacing are not cut into pieces whose extra
// box tests cost more than the gaps save.  Writes the run boxes to L.seg
// and returns their number.
template <typename Lds>
__device__ __forceinline__ int make_segments(Lds &L, const Query &q, float jump, int *sid_out,
                                             float step_factor = 0.0f) {
    const int lane = lane_id();
    const float px = __shfl_up(q.x, 1), py = __shfl_up(q.y, 1), pz = __shfl_up(q.z, 1);
    const int pv = __shfl_up(q.valid ? 1 : 0, 1);
    float step = 0.0f;
    const bool has = lane > 0 && q.valid && pv;
    if (has) step = fmaxf(fabsf(q.x - px), fmaxf(fabsf(q.y - py), fabsf(q.z - pz)));
    if (step_factor > 0.0f) {
        const int ns = __popcll(ballot(has));
        if (ns > 0) jump = fmaxf(jump, fminf(2.0f * jump, step_factor * wave_sum_f(step) / static_cast<float>(ns)));
    }
    const bool brk = step > jump;
    uint64_t bm = ballot(brk);
    if (__popcll(bm) > kSegMax - 1) {
        uint64_t keep = 0;
        float sv = brk ? step : -1.0f;
        for (int i = 0; i < kSegMax - 1; ++i) {
            const float m = wave_max_u(sv);
            const uint64_t w = ballot(brk && sv == m);
            const int l = __ffsll(static_cast<long long>(w)) - 1;
            keep |= 1ull << l;
            if (lane == l) sv = -1.0f;
        }
        bm = keep;
    }
    const int sid = __popcll(bm & ((2ull << lane) - 1ull));
    const int nseg = __popcll(bm) + 1;
    for (int s = 0; s < nseg; ++s) {
        const bool in = q.valid && sid == s;
        const float b0 = wave_min_u(in ? q.x : INFINITY), b1 = wave_min_u(in ? q.y : INFINITY);
        const float b2 = wave_min_u(in ? q.z : INFINITY), b3 = wave_max_u(in ? q.x : -INFINITY);
        const float b4 = wave_max_u(in ? q.y : -INFINITY), b5 = wave_max_u(in ? q.z : -INFINITY);
        if (lane == 0) {
            L.seg[s][0] = b0;
            L.seg[s][1] = b1;
            L.seg[s][2] = b2;
            L.seg[s][3] = b3;
            L.seg[s][4] = b4;
            L.seg[s][5] = b5;
        }
    }
    wave_sync();
    if (sid_out) *sid_out = sid;
    return nseg;
}

template <int KERNEL, typename Lds>
__device__ __forceinline__ bool segments_may_hit(const Lds &L, int nseg, const sfc_node &nd, float r, float r2) {
    bool hit = false;
    for (int s = 0; s < nseg; ++s) hit = hit || group_may_hit<KERNEL>(nd, &L.seg[s][0], &L.seg[s][3], r, r2);
    return hit;
}

// does the LDS layout keep the candidates' ends?
template <typename T, typename = void>
struct HasEnds : std::false_type {};
template <typename T>
struct HasEnds<T, std::void_t<decltype(std::declval<T &>().cend)>> : std::true_type {};

// Walks the tree below node `start` (the root by default); each time the
// candidate list fills up (or the walk ends) calls sweep(ncand).
// accept(node) decides whether the wave keeps a node.
template <typename Lds, typename Accept, typename Sweep>
__device__ __forceinline__ void traverse(Lds &L, const sfc_node *__restrict__ nodes,
                                         const int32_t *__restrict__ child, Accept accept, Sweep sweep,
                                         int start = 0) {
    const int lane = lane_id();
    if (lane == 0) L.stack[0] = start;
    int sp = 1, ncand = 0;
    wave_sync();
    while (sp > 0) {
        int take = (kStack - sp) / 7;
        if (take > kWave) take = kWave;
        if (take > sp) take = sp;
        if (take < 1) take = 1;
        const int node = lane < take ? L.stack[sp - take + lane] : -1;
        sp -= take;
        wave_sync();
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
        if (cand) {
            const int at = ncand + static_cast<int>(rank_below(m_c));
            L.cand[at] = node;
            L.cbeg[at] = nd.begin;
            if constexpr (HasEnds<Lds>::value) L.cend[at] = nd.end;
            if constexpr (std::is_same<Lds, WaveLds>::value) L.cnode[at] = nd;
        }
        ncand += __popcll(m_c);
        wave_sync();
        if (ncand > kCand - kWave || (sp == 0 && ncand > 0)) {
            sweep(ncand);
            ncand = 0;
        }
    }
}

__device__ __forceinline__ uint64_t wave_or(uint64_t v) {
    uint32_t lo = static_cast<uint32_t>(v), hi = static_cast<uint32_t>(v >> 32);
    for (int o = 32; o > 0; o >>= 1) {
        lo |= __shfl_xor(lo, o);
        hi |= __shfl_xor(hi, o);
    }
    return (static_cast<uint64_t>(static_cast<uint32_t>(__builtin_amdgcn_readfirstlane(hi))) << 32) |
           static_cast<uint64_t>(static_cast<uint32_t>(__builtin_amdgcn_readfirstlane(lo)));
}

// Stages the points of the batch candidates [c0, c0 + m) selected by `need`
// (bit i: candidate c0 + i), in candidate order, up to kStage points per
// round, and for every round calls body(count): L.pts[0..count) are the
// points and L.owner[] their candidate within the batch.  Points for which
// keep(point) is false are dropped while staging (lane = point).
template <typename Keep, typename Body>
__device__ __forceinline__ void stage_rounds(WaveLds &L, const float4 *__restrict__ pts, int c0, int m, uint64_t need,
                                             Keep keep, Body body) {
    const int lane = lane_id();
    uint32_t sz = 0;
    if (lane < m && ((need >> lane) & 1ull)) sz = L.cend[c0 + lane] - L.cbeg[c0 + lane];
    const uint32_t incl = wave_inclusive_sum(sz);
    L.cincl[lane] = incl;
    const uint32_t total = __builtin_amdgcn_readfirstlane(__shfl(incl, kWave - 1));
    wave_sync();
    uint32_t kept = 0;  // the same in every lane
    for (uint32_t base = 0; base < total; base += kWave) {
        const uint32_t p = base + lane;
        bool k = false;
        float4 v;
        int lo = 0;
        if (p < total) {
            int hi = m - 1;  // first candidate whose inclusive end exceeds p
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (L.cincl[mid] > p)
                    hi = mid;
                else
                    lo = mid + 1;
            }
            const uint32_t first = lo > 0 ? L.cincl[lo - 1] : 0u;
            v = pts[L.cbeg[c0 + lo] + (p - first)];
            k = keep(v);
        }
        const uint64_t km = ballot(k);
        if (k) {
            const uint32_t at = kept + rank_below(km);
            L.pts[at] = v;
            L.owner[at] = static_cast<uint8_t>(lo);
        }
        kept += static_cast<uint32_t>(__popcll(km));
        if (kept > static_cast<uint32_t>(WaveLds::kPts - kWave) || (base + kWave >= total && kept > 0)) {
            wave_sync();
            body(kept);
            wave_sync();
            kept = 0;
        }
    }
}

// One cloud of a search launch (a table of these, or one in the kernel
// arguments).  Rows of the cloud are global rows q_offset .. q_offset + nq - 1;
// its groups of 64 rows are global groups g0 .. g0 + ceil(nq / 64) - 1.
struct SearchCloud {
    const sfc_node *nodes;
    const int32_t *child;
    const float4 *pts;
    const uint32_t *perm;
    const uint64_t *keys;
    const sfc_frame *frame;
    int64_t n;
    int64_t q_offset;
    int64_t nq;
    int64_t g0;
    int64_t rg0;    // its groups' record regions start here (regions exist only for recording clouds)
    float r;
    int32_t kernel;
    int32_t k;
    int32_t stage;  // radius search: points staged per round (64, 128, 256)
    int32_t rec;    // radius search: the cloud's hits are recorded (SFC_RECORD_HITS or the cloud's choice)
};
// The host hashes table entries byte for byte up to `rec` (the records'
// provenance tag): no padding may lie in between, since its bytes are
// indeterminate and would make two identical calls hash differently.
constexpr size_t kCloudHashBytes = offsetof(SearchCloud, rec) + sizeof(int32_t);
static_assert(offsetof(SearchCloud, r) == 6 * sizeof(void *) + 5 * sizeof(int64_t) &&
                  kCloudHashBytes == offsetof(SearchCloud, r) + 5 * sizeof(int32_t),
              "SearchCloud has no padding before its end");

struct SearchArgs {
    SearchCloud one;          // the cloud when tab is null
    const SearchCloud *tab;   // [B] in device memory
    int B;
    int64_t groups;           // groups of all clouds
    const float *queries;     // global rows (3 floats each), or null: each cloud's own sorted points
    const uint32_t *qperm;    // with queries: global row of every curve-sorted query position, or null
    int64_t nq_total;
    uint32_t flags;
    uint32_t *counts;
    const uint64_t *offsets;
    uint32_t *indices;
    uint64_t capacity;
    int kstride;
    uint32_t *idx;
    float *d2;
    uint32_t *spread;         // [groups] groups left to the one-query-per-wave kernels
    uint32_t *nspread;        // their number
    uint32_t *rcounts;        // range form: ranges per row
    const uint64_t *roffsets; // their row starts
    uint32_t *ranges;         // (begin, end) pairs of sorted positions
    uint64_t rcapacity;       // pairs the ranges buffer holds
    // recorded hits (SFC_RECORD_HITS): per global group, kRecCap slots of
    // (original index, mask of the group's queries it is a neighbour of)
    uint32_t *rec_idx;
    uint64_t *rec_mask;
    uint32_t *rec_n;          // records of each group; kRecOverflow: did not fit
    // provenance of the records: the recording count stamps (tag0, tag1) into
    // rec_tag; a fill uses the records only if rec_tag holds its own pair
    // (the number the host gave the workspace's last count call, and a hash
    // of the call's arguments), else it searches again
    uint64_t *rec_tag;
    uint64_t tag0, tag1;
    uint32_t fill_scan;       // k_radius_fill: every group recorded, kFillScan groups per wave
};

// Query of a lane (position lr in its cloud's rows) and the global row its
// results go to.  External queries are taken in curve order through qperm,
// so a wave's 64 queries are close in space whatever the caller's order.
__device__ __forceinline__ Query lane_query(const SearchArgs &a, const SearchCloud &C, int64_t lr, int64_t *row) {
    Query q{0.0f, 0.0f, 0.0f, lr < C.nq};
    int64_t g = C.q_offset + lr;
    if (q.valid) {
        if (a.queries) {
            if (a.qperm) g = a.qperm[g];
            q.x = a.queries[3 * g];
            q.y = a.queries[3 * g + 1];
            q.z = a.queries[3 * g + 2];
        } else {
            const float4 p = C.pts[lr];
            q.x = p.x;
            q.y = p.y;
            q.z = p.z;
        }
    }
    *row = g;
    return q;
}

// the cloud owning global group g: the last table entry with g0 <= g (clouds
// without rows own no group, so the search skips them)
__device__ __forceinline__ SearchCloud group_cloud(const SearchArgs &a, int64_t g) {
    if (!a.tab) return a.one;
    int lo = 0, hi = a.B - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (a.tab[mid].g0 <= g)
            lo = mid;
        else
            hi = mid - 1;
    }
    return a.tab[lo];
}

// Radius search.  Every candidate node is classified against the box of
// every query segment (exactly, by the monotonicity argument): disjoint from
// every query of the segment, contained for every one of them, or mixed.
// Nodes that are mixed for some segment are staged in LDS and swept: every
// lane tests its own query against every staged point (a lane for which the
// node is contained gets "true" for each of its points, by the same
// argument, so no per-lane bookkeeping is needed).  Nodes contained for a
// segment and mixed for none are counted without touching their points.
//
// STAGE (points staged per round: 64, 128 or 256) is the search's tile: a
// larger round amortises the per-round work (and, in the search fill, the
// row flushes every round ends with) over more points, a smaller one needs
// less LDS, so more waves stay resident.  It is chosen per cloud at run time
// (the autotuner picks it per group of clouds); results do not depend on it.
template <int STAGE>
struct RadLdsT {
    static constexpr int kPts = STAGE;
    int stack[kStack];
    int cand[kCand];         // candidate nodes (indices)
    uint32_t cbeg[kCand];    // their first points
    float4 pts[STAGE];
    union {
        uint32_t clen[kWave];   // sizes of the batch candidates (read before staging starts)
        uint32_t cincl[kWave];  // inclusive prefix of staged sizes of the batch
    };
    float seg[kSegMax][6];
};

using RadLds = RadLdsT<kStage>;

template <int STAGE>
struct FillLdsT : RadLdsT<STAGE> {
    uint8_t rows[kWave * (kRowCap + 1)];   // per-query output staging: staged-point slots
    uint64_t fpos[kWave];                  // rows being flushed, by list entry: global position
    uint32_t fmeta[kWave];                 // and lane | entries that fit the row's slot << 8
};
using FillLds = FillLdsT<kStage>;

// the range form also keeps the candidates' ends and records the candidate
// of every staged point
struct StructLds : FillLds {
    uint32_t cend[kCand];
    uint8_t owner[kStage];
};

// largest |fp32 difference| between a coordinate of [lo, hi] and one of [glo, ghi]
__device__ __forceinline__ float far_gap(float lo, float hi, float glo, float ghi) {
    return fmaxf(fabsf(fsub(lo, ghi)), fabsf(fsub(hi, glo)));
}

// 0: no point of the node is a neighbour of any query in the box [glo, ghi];
// 1: every point is a neighbour of every such query; 2: mixed.
template <int KERNEL>
__device__ __forceinline__ int classify_box(const sfc_node &b, const float *glo, const float *ghi, float r,
                                            float r2) {
    if (!group_may_hit<KERNEL>(b, glo, ghi, r, r2)) return 0;
    const float fx = far_gap(b.lo[0], b.hi[0], glo[0], ghi[0]);
    const float fy = far_gap(b.lo[1], b.hi[1], glo[1], ghi[1]);
    if constexpr (KERNEL == SFC_SPHERE) {
        const float fz = far_gap(b.lo[2], b.hi[2], glo[2], ghi[2]);
        return fadd(fadd(fmul(fx, fx), fmul(fy, fy)), fmul(fz, fz)) < r2 ? 1 : 2;
    } else if constexpr (KERNEL == SFC_CIRCLE) {
        return fadd(fmul(fx, fx), fmul(fy, fy)) < r2 ? 1 : 2;
    } else if constexpr (KERNEL == SFC_CUBE) {
        const float fz = far_gap(b.lo[2], b.hi[2], glo[2], ghi[2]);
        return ((fx < r) & (fy < r) & (fz < r)) ? 1 : 2;
    } else {
        return ((fx < r) & (fy < r)) ? 1 : 2;
    }
}

// Classifies the batch candidates [c0, c0 + m) (lane = candidate) against
// every segment box.  Stores the candidate sizes in L.clen and returns the
// lane's own; *mixed / *touched: candidates mixed / not disjoint for some
// segment; *full: candidates contained for the calling lane's segment.
template <int KERNEL, typename Lds>
__device__ __forceinline__ uint32_t classify_segments(Lds &L, const sfc_node *__restrict__ nodes, int c0, int m,
                                                      int nseg, int sid, float r, float r2, bool prune,
                                                      uint64_t *mixed, uint64_t *touched, uint64_t *full) {
    const int lane = lane_id();
    const bool have = lane < m;
    sfc_node nd;
    if (have) nd = nodes[L.cand[c0 + lane]];
    const uint32_t len = have ? nd.end - nd.begin : 0u;
    L.clen[lane] = len;
    uint64_t mx = 0, tc = 0, fm = 0;
    for (int s = 0; s < nseg; ++s) {
        int cls = have ? classify_box<KERNEL>(nd, &L.seg[s][0], &L.seg[s][3], r, r2) : 0;
        if (cls == 1 && !prune) cls = 2;
        mx |= ballot(cls == 2);
        tc |= ballot(cls != 0);
        const uint64_t f = ballot(cls == 1);
        if (sid == s) fm = f;
    }
    *mixed = mx;
    *touched = tc;
    *full = fm;
    wave_sync();
    return len;
}

// Stages the points of the batch candidates [c0, c0 + m) selected by `need`
// (bit i: candidate c0 + i), in candidate order, and calls body(count) with
// L.pts[0..count) filled (and, with OWNER, L.owner[] the candidate of each
// point within the batch), up to kStage points per round.  Points that no
// query of any segment can reach are dropped while staging (lane = point,
// the conservative gap test of the segment boxes, exact by the monotonicity
// argument): a point outside every grown segment box is a neighbour of none
// of the wave's queries, so only the sweep's work changes, never a result.
//
// With `carry`, the staged points stay for the next batch: body runs only
// when the buffer is full, *carry holds the count in and out, and the caller
// sweeps what is left after its last batch (bodies that do not depend on the
// batch; fuller rounds mean fewer round ends).
template <int KERNEL, bool OWNER = false, typename Lds, typename Body>
__device__ __forceinline__ void stage_union(Lds &L, const float4 *__restrict__ pts, int c0, int m, uint64_t need,
                                            uint32_t len, int nseg, float r, float r2, Body body,
                                            uint32_t *carry = nullptr) {
    const int lane = lane_id();
    const uint32_t incl = wave_inclusive_sum(((need >> lane) & 1ull) ? len : 0u);
    L.cincl[lane] = incl;
    const uint32_t total = __builtin_amdgcn_readfirstlane(__shfl(incl, kWave - 1));
    wave_sync();
    uint32_t kept = carry ? *carry : 0u;  // points staged for the next round (the same in every lane)
    for (uint32_t base = 0; base < total; base += kWave) {
        const uint32_t p = base + lane;
        bool keep = false;
        float4 v;
        int lo = 0;
        if (p < total) {
            int hi = m - 1;  // first candidate whose inclusive end exceeds p
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (L.cincl[mid] > p)
                    hi = mid;
                else
                    lo = mid + 1;
            }
            const uint32_t first = lo > 0 ? L.cincl[lo - 1] : 0u;
            v = pts[L.cbeg[c0 + lo] + (p - first)];
            sfc_node b;
            b.lo[0] = b.hi[0] = v.x;
            b.lo[1] = b.hi[1] = v.y;
            b.lo[2] = b.hi[2] = v.z;
            keep = segments_may_hit<KERNEL>(L, nseg, b, r, r2);
        }
        const uint64_t km = ballot(keep);
        if (keep) {
            L.pts[kept + rank_below(km)] = v;
            if constexpr (OWNER) L.owner[kept + rank_below(km)] = static_cast<uint8_t>(lo);
        }
        kept += static_cast<uint32_t>(__popcll(km));
        if (kept > static_cast<uint32_t>(Lds::kPts - kWave) || (!carry && base + kWave >= total && kept > 0)) {
            wave_sync();
            body(kept);
            wave_sync();
            kept = 0;
        }
    }
    if (carry) *carry = kept;
}

// A wave's queries are "spread" when the region every lane sweeps in the
// group scheme (the segment boxes grown by r) is much larger than the
// queries' own neighbourhoods together (nvalid cubes or squares of side 2r):
// most of each lane's tests would then be other queries' work.  Such a wave
// serves its queries one after another instead, all lanes on one query
// (lane = candidate point).  Only the cost model uses these products, never
// a result.
// `factor` weighs the group scheme's per-point cost against the one-query
// scheme's (k-NN group sweeps pay a register top-k insertion per point).
template <typename Lds>
__device__ __forceinline__ bool spread_group(const Lds &L, int nseg, float r, int nvalid, float factor = 1.0f) {
    const float d = 2.0f * r;
    float sweep = 0.0f;
    for (int s = 0; s < nseg; ++s) sweep += (L.seg[s][3] - L.seg[s][0] + d) * (L.seg[s][4] - L.seg[s][1] + d);
    return sweep > factor * static_cast<float>(nvalid) * d * d;
}

// Only external queries can be spread: a cloud's own points taken in curve
// order are dense (64 consecutive curve points are close, apart from the few
// jumps the segments already split off).
__device__ __forceinline__ bool may_defer(const SearchArgs &a) { return a.spread && a.queries; }

// hands group g to the one-query-per-wave kernel
__device__ __forceinline__ void defer_group(const SearchArgs &a, int64_t g) {
    if (lane_id() == 0) a.spread[atomicAdd(a.nspread, 1u)] = static_cast<uint32_t>(g);
}

// Walks the tree for the single query (qx, qy, qz); per batch of candidates
// calls full(mask) with the candidates that are contained (all points are
// neighbours) and sweep(n) for every staged round of the points of the mixed
// ones.  Classification against the one-point box is the exact per-query
// test (the box gap and far-corner distances equal those of the point).
template <int KERNEL, typename Lds, typename Full, typename Sweep>
__device__ __forceinline__ void walk_one(Lds &L, const SearchCloud &C, float qx, float qy, float qz, float r, float r2,
                                         bool prune, Full full, Sweep sweep) {
    if (lane_id() == 0) {
        L.seg[0][0] = qx;
        L.seg[0][1] = qy;
        L.seg[0][2] = qz;
        L.seg[0][3] = qx;
        L.seg[0][4] = qy;
        L.seg[0][5] = qz;
    }
    wave_sync();
    auto accept = [&](const sfc_node &nd) { return segments_may_hit<KERNEL>(L, 1, nd, r, r2); };
    auto batches = [&](int ncand) {
        for (int c0 = 0; c0 < ncand; c0 += kWave) {
            const int m = min(kWave, ncand - c0);
            uint64_t mixed, touched, fm;
            const uint32_t len = classify_segments<KERNEL>(L, C.nodes, c0, m, 1, 0, r, r2, prune, &mixed, &touched, &fm);
            full(c0, fm & ~mixed, len);
            if (mixed) stage_union<KERNEL>(L, C.pts, c0, m, mixed, len, 1, r, r2, sweep);
        }
    };
    traverse(L, C.nodes, C.child, accept, batches);
}

template <int KERNEL>
__device__ __forceinline__ uint32_t count_one(RadLds &L, const SearchCloud &C, float qx, float qy, float qz, float r,
                                              float r2, bool prune) {
    const int lane = lane_id();
    uint32_t cnt = 0;  // the same in every lane
    walk_one<KERNEL>(
        L, C, qx, qy, qz, r, r2, prune,
        [&](int, uint64_t fm, uint32_t len) { cnt += wave_sum_u(((fm >> lane) & 1ull) ? len : 0u); },
        [&](uint32_t n) {
            for (uint32_t t0 = 0; t0 < n; t0 += kWave) {
                const uint32_t t = t0 + lane;
                const bool h = t < n && point_hit<KERNEL>(L.pts[t < n ? t : 0], qx, qy, qz, r, r2);
                cnt += static_cast<uint32_t>(__popcll(ballot(h)));
            }
        });
    return cnt;
}

// The deepest node whose cell holds every point that may be a neighbour of
// the wave's queries, so the walk can start there instead of at the root.
// The reach is the union of the segment boxes grown by r (and widened by a
// few ulps of the coordinates against rounding); for the 2D kernels its z
// range is the cloud's whole extent.  The cell discretisation of the codes
// is monotone, so every such point lies in the cells between those of the
// reach's corners, i.e. inside the deepest cell that holds both; the walk
// down to it follows the digits of any code inside it (a query's own code:
// the queries lie in the reach, also in z for the 2D kernels, whose z range
// takes in the queries' too), internal nodes having all 8 children in digit
// order.
template <int KERNEL, typename Lds>
__device__ __forceinline__ int start_node(const Lds &L, const SearchArgs &a, const SearchCloud &C, int nseg, float r,
                                          const Query &q, int64_t lr) {
    if (C.n <= 0 || a.queries) return 0;  // external queries: no code at hand, start at the root
    float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int s = 0; s < nseg; ++s) {
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            lo[d] = fminf(lo[d], L.seg[s][d]);
            hi[d] = fmaxf(hi[d], L.seg[s][3 + d]);
        }
    }
    const sfc_frame f = *C.frame;
    const uint32_t ncell = 1u << f.bits;
    int span = 0;  // bits in which the corner cells differ, over the axes
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        float rl = lo[d], rh = hi[d], g = r;
        if ((KERNEL == SFC_CIRCLE || KERNEL == SFC_SQUARE) && d == 2) {
            rl = fminf(rl, C.nodes[0].lo[2]);
            rh = fmaxf(rh, C.nodes[0].hi[2]);
            g = 0.0f;
        }
        const float e = (fabsf(rl) + fabsf(rh) + g) * 1e-6f;
        const uint32_t c0 = cell_of(rl - g - e, f.lo[d], f.scale, ncell);
        const uint32_t c1 = cell_of(rh + g + e, f.lo[d], f.scale, ncell);
        const uint32_t x = c0 ^ c1;
        const int b = x ? 32 - __clz(static_cast<int>(x)) : 0;
        span = b > span ? b : span;
    }
    const int l = f.bits - span;  // level of the cell holding the reach
    if (l <= 0 || !(lo[0] <= hi[0])) return 0;
    // a code inside that cell: the first valid lane's query
    const int first = __ffsll(static_cast<long long>(ballot(q.valid))) - 1;
    if (first < 0) return 0;
    const uint64_t key = readlane_u64(C.keys[lr < C.n ? lr : 0], first);
    int node = 0;
    for (int d = 1; d <= l; ++d) {
        const int c = C.child[node];
        if (c < 0) break;
        node = c + static_cast<int>((key >> (3 * (f.bits - d))) & 7u);
    }
    return node;
}

// Shader-clock time of the count's phases per wave, in the statistics build
// only (elsewhere every call compiles to nothing): [0] segments, [1] start
// node, [2] walk (traversal alone), [3] classification, [4] staging (without
// the tests), [5] tests, [6] the rest (the last tests and the epilogue).
struct PhaseClock {
#ifdef SFC_SWEEP_STATS
    unsigned long long t[7] = {};
    unsigned long long tests_before_tail = 0;
    __device__ __forceinline__ static unsigned long long now() { return __builtin_amdgcn_s_memtime(); }
    __device__ __forceinline__ void add(int i, unsigned long long t0) { t[i] += now() - t0; }
    __device__ __forceinline__ void mark_tail() { tests_before_tail = t[5]; }
    // the walk's time holds the sweeps', a sweep's holds its classification
    // and tests, and the tail's its last tests: take each nested phase out
    __device__ __forceinline__ void nest() {
        const unsigned long long tail_tests = t[5] - tests_before_tail;
        t[6] -= tail_tests;
        t[2] -= t[4];
        t[4] -= t[3] + tests_before_tail;
    }
#else
    __device__ __forceinline__ static unsigned long long now() { return 0ull; }
    __device__ __forceinline__ void add(int, unsigned long long) {}
    __device__ __forceinline__ void mark_tail() {}
#endif
};

#ifdef SFC_SWEEP_STATS
// Sweep statistics of the count kernels (a separate build, libsfcoct_stats.so:
// the search itself is unchanged), summed over every group since the last
// reset: [0] point tests (staged points swept x the group's valid queries),
// [1] neighbours found, [2] groups, [3] staged points swept; [4..7] the same
// for recording groups only; [8..14] the phase clocks (PhaseClock), [15]
// the whole body's clock.
__device__ unsigned long long g_sweep_stats[16];

__device__ __forceinline__ void sweep_clock_add(const PhaseClock &pc, unsigned long long total) {
    if (lane_id() != 0) return;
    for (int i = 0; i < 7; ++i) atomicAdd(g_sweep_stats + 8 + i, pc.t[i]);
    atomicAdd(g_sweep_stats + 15, total);
}

__device__ __forceinline__ void sweep_stats_add(uint32_t swept, int nvalid, uint32_t hits, bool rec) {
    if (lane_id() != 0) return;
    unsigned long long *s = g_sweep_stats + (rec ? 4 : 0);
    atomicAdd(s + 0, static_cast<unsigned long long>(swept) * static_cast<unsigned long long>(nvalid));
    atomicAdd(s + 1, static_cast<unsigned long long>(hits));
    atomicAdd(s + 2, 1ull);
    atomicAdd(s + 3, static_cast<unsigned long long>(swept));
}
#endif

// With REC (SFC_RECORD_HITS) the wave also records, per staged point that
// is a neighbour of at least one of its queries, the point's original index
// and the mask of those queries, in staging order, into the group's region
// of the workspace: k_radius_fill_rec and k_radius_fill_rows then write the
// rows from the records alone.  Every touched node is staged and tested (a
// contained node is not counted from its size), so the records hold every
// neighbour in the order k_radius_fill would write them.  A group whose records do not fit kRecCap,
// or that is deferred, is marked kRecOverflow and left to k_radius_fill.
template <int KERNEL, bool REC, int STAGE>
__device__ __forceinline__ void radius_count_body(RadLdsT<STAGE> &L, const SearchArgs &a, const SearchCloud &C,
                                                  int64_t lg) {
    const int lane = lane_id();
    const int64_t lr = lg * kWave + lane;  // position within the cloud's rows
    int64_t row;
    const Query q = lane_query(a, C, lr, &row);
    const float r = C.r, r2 = fmul(r, r);
    const bool prune = !(a.flags & SFC_NO_PRUNE);
    const int64_t gg = lg + C.g0;  // global group
    uint32_t cnt = 0;
    int sid = 0;
    PhaseClock pc;
    const unsigned long long t_begin = PhaseClock::now();
    const int nseg = r > 0.0f ? make_segments(L, q, 2.0f * r, &sid, kJumpSteps) : 0;
    if (r > 0.0f && may_defer(a) && spread_group(L, nseg, r, __popcll(ballot(q.valid)))) {
        if constexpr (REC) {
            if (lane == 0) a.rec_n[gg] = kRecOverflow;
        }
        defer_group(a, gg);
        return;
    }
    pc.add(0, t_begin);
    uint32_t nrec = 0;  // records of the group so far (may pass kRecCap: then none is kept)
    uint32_t swept = 0;  // staged points every lane tested (the sweep statistics)
    if (r > 0.0f) {
        // every lane tests its query against the staged points
        auto body = [&](uint32_t n_) {
            const unsigned long long t_body = PhaseClock::now();
            const uint32_t n = __builtin_amdgcn_readfirstlane(n_);
            swept += n;
            uint32_t t = 0;
            for (; t + 4 <= n; t += 4) {
                const float4 p0 = L.pts[t], p1 = L.pts[t + 1], p2 = L.pts[t + 2], p3 = L.pts[t + 3];
                cnt += point_hit<KERNEL>(p0, q.x, q.y, q.z, r, r2) ? 1u : 0u;
                cnt += point_hit<KERNEL>(p1, q.x, q.y, q.z, r, r2) ? 1u : 0u;
                cnt += point_hit<KERNEL>(p2, q.x, q.y, q.z, r, r2) ? 1u : 0u;
                cnt += point_hit<KERNEL>(p3, q.x, q.y, q.z, r, r2) ? 1u : 0u;
            }
            for (; t < n; ++t) cnt += point_hit<KERNEL>(L.pts[t], q.x, q.y, q.z, r, r2) ? 1u : 0u;
            pc.add(5, t_body);
        };
        // recording: lane j of (mlo, mhi) takes the query mask of staged point
        // t0 + j; per 64 points the ones with a neighbour are compacted and
        // stored (lane = record: coalesced)
        const float qx = q.valid ? q.x : INFINITY, qy = q.valid ? q.y : INFINITY, qz = q.valid ? q.z : INFINITY;
        uint32_t *const ridx = a.rec_idx + (C.rg0 + lg) * kRecCap;
        uint64_t *const rmask = a.rec_mask + (C.rg0 + lg) * kRecCap;
        auto body_rec = [&](uint32_t n_) {
            const unsigned long long t_body = PhaseClock::now();
            const uint32_t n = __builtin_amdgcn_readfirstlane(n_);
            swept += n;
            for (uint32_t t0 = 0; t0 < n; t0 += kWave) {
                const uint32_t te = min(n, t0 + kWave);
                uint32_t mlo = 0, mhi = 0;
                uint32_t t = t0;
                auto test = [&](uint32_t u) {
                    // the hit mask straight from the comparison; the lane's own
                    // bit of it counts (no 0/1 value in a vector register)
                    const uint64_t m = hit_mask<KERNEL>(L.pts[u], qx, qy, qz, r, r2);
                    cnt += __builtin_amdgcn_inverse_ballot_w64(m) ? 1u : 0u;
                    const int at = static_cast<int>(u - t0);
                    mlo = writelane_u32(static_cast<uint32_t>(m), at, mlo);
                    mhi = writelane_u32(static_cast<uint32_t>(m >> 32), at, mhi);
                };
                for (; t + 4 <= te; t += 4) {
                    test(t);
                    test(t + 1);
                    test(t + 2);
                    test(t + 3);
                }
                for (; t < te; ++t) test(t);
                const bool keep = static_cast<uint32_t>(lane) < te - t0 && (mlo | mhi) != 0u;
                const uint64_t km = ballot(keep);
                const uint32_t at = nrec + static_cast<uint32_t>(rank_below(km));
                if (keep && at < static_cast<uint32_t>(kRecCap)) {
                    ridx[at] = __float_as_uint(L.pts[t0 + lane].w);
                    rmask[at] = (static_cast<uint64_t>(mhi) << 32) | mlo;
                }
                nrec += static_cast<uint32_t>(__popcll(km));
            }
            pc.add(5, t_body);
        };
        uint32_t staged = 0;  // points staged and not yet swept, across candidate batches
        // Once the records overflow the group is left to the search fill, so
        // the rest of the walk counts as the plain count does (contained
        // nodes from their sizes); points already staged are tested either way.
        auto recording = [&]() { return REC && nrec <= static_cast<uint32_t>(kRecCap); };
        auto accept = [&](const sfc_node &nd) { return segments_may_hit<KERNEL>(L, nseg, nd, r, r2); };
        auto sweep = [&](int ncand) {
            const unsigned long long t_sweep = PhaseClock::now();
            for (int c0 = 0; c0 < ncand; c0 += kWave) {
                const int m = min(kWave, ncand - c0);
                uint64_t mixed, touched, full;
                const unsigned long long t_cls = PhaseClock::now();
                const uint32_t len =
                    classify_segments<KERNEL>(L, C.nodes, c0, m, nseg, sid, r, r2, prune, &mixed, &touched, &full);
                pc.add(3, t_cls);
                if (recording()) {
                    if (!touched) continue;
                    stage_union<KERNEL>(L, C.pts, c0, m, touched, len, nseg, r, r2, body_rec, &staged);
                } else {
                    // contained for my segment and not swept: count the whole node
                    for (uint64_t b = full & ~mixed; b; b &= b - 1)
                        cnt += L.clen[__ffsll(static_cast<long long>(b)) - 1];
                    if (!mixed) continue;
                    stage_union<KERNEL>(L, C.pts, c0, m, mixed, len, nseg, r, r2, body, &staged);
                }
            }
            pc.add(4, t_sweep);  // the sweep's whole time; classification and tests are taken out below
        };
        const unsigned long long t_start = PhaseClock::now();
        const int start = start_node<KERNEL>(L, a, C, nseg, r, q, lr);
        pc.add(1, t_start);
        const unsigned long long t_walk = PhaseClock::now();
        traverse(L, C.nodes, C.child, accept, sweep, start);
        pc.add(2, t_walk);  // the walk's whole time; the sweeps are taken out below
        pc.mark_tail();
        const unsigned long long t_tail = PhaseClock::now();
        if (staged) {
            wave_sync();
            if (recording())
                body_rec(staged);
            else
                body(staged);
        }
        pc.add(6, t_tail);
    }
    if (q.valid) a.counts[row] = cnt;
#ifdef SFC_SWEEP_STATS
    sweep_stats_add(swept, __popcll(ballot(q.valid)), wave_sum_u(q.valid ? cnt : 0u), REC);
    pc.nest();
    sweep_clock_add(pc, PhaseClock::now() - t_begin);
#else
    (void)swept;
#endif
    if constexpr (REC) {
        // groups whose rows average kRecLongMean entries or more take the long-row form
        const uint32_t hits = __shfl(wave_inclusive_sum(q.valid ? cnt : 0u), kWave - 1);
        const uint32_t nvalid = static_cast<uint32_t>(__popcll(ballot(q.valid)));
        const uint32_t form = hits >= kRecLongMean * nvalid ? kRecLongRows : 0u;
        if (lane == 0) a.rec_n[gg] = nrec <= static_cast<uint32_t>(kRecCap) ? (nrec | form) : kRecOverflow;
    }
}

// Writing the rows of a group from its records (SFC_RECORD_HITS): no
// traversal and no distance test.  Two forms, chosen per group by the count
// pass from the group's mean row length, each a kernel of its own (so each
// keeps its own register and LDS footprint):
//  - short rows (k_radius_fill_rec): per record, every lane whose bit is set
//    appends a one-byte slot into the current batch of up to 256 records to
//    its LDS row; rows are written out (two rows per step, one per half wave)
//    once they could overflow and after every batch;
//  - long rows (k_radius_fill_rows): the rows are written one query after
//    another straight from the records held in registers (below).
constexpr int kRecBatch = SFC_REC_BATCH;         // short rows: chunks of 64 records per load round trip and slot table
static_assert(kRecBatch >= 1 && kRecBatch <= 4, "record fill shapes");

// Rows being written out are listed compactly: entry i holds the row's
// output position and its lane and counts packed in one word, so a writing
// lane fetches everything about its row with two independent LDS reads.
struct RecLds {
    uint8_t rows[kWave * (kRowCap + 1)];
    uint64_t fpos[kWave];   // by list entry: output position
    uint32_t fmeta[kWave];  // by list entry: lane | entries to write << 8
    uint32_t pidx[kRecBatch * kWave];  // original indices of the batch's records (slot = position in the batch)
};

__device__ __forceinline__ void radius_fill_rec_body(RecLds &L, const SearchArgs &a, const SearchCloud &C,
                                                     int64_t lg, uint32_t n) {
    const int lane = lane_id();
    const int64_t lr = lg * kWave + lane;
    int64_t row;
    const Query q = lane_query(a, C, lr, &row);
    const int64_t orow = q.valid ? row : 0;
    const uint64_t o0 = a.offsets[orow], o1 = a.offsets[orow + 1];
    uint64_t gpos = q.valid ? o0 : 0ull;
    const uint64_t gend = q.valid ? o1 : 0ull;
    uint64_t left = gend > gpos ? gend - gpos : 0ull;
    uint32_t nb = 0;
    uint8_t *myrow = L.rows + lane * (kRowCap + 1);
    uint32_t *out = a.indices;
    const int half = lane >> 5, hl = lane & 31;
    auto flush = [&](uint32_t limit) {
        const bool go = nb > limit;
        const uint64_t fm = ballot(go);
        if (!fm) return;
        const int nf = __popcll(fm);
        if (go) {
            const uint32_t i = rank_below(fm);
            L.fpos[i] = gpos;
            L.fmeta[i] = static_cast<uint32_t>(lane) | (static_cast<uint32_t>(left < nb ? left : nb) << 8);
        }
        wave_sync();
        for (int i0 = 0; i0 < nf; i0 += 2) {
            const int i = i0 + half;
            if (i < nf) {
                const uint32_t meta = L.fmeta[i];
                const uint64_t pos = L.fpos[i];
                const uint32_t slot = L.rows[(meta & 0xFFu) * (kRowCap + 1) + hl];  // hl < kRowCap + 1
                if (static_cast<uint32_t>(hl) < (meta >> 8)) out[pos + hl] = L.pidx[slot];
            }
        }
        if (go) {
            gpos += nb;
            left -= left < nb ? left : nb;
            nb = 0;
        }
        wave_sync();
    };
    const uint32_t *ridx = a.rec_idx + (C.rg0 + lg) * kRecCap;
    const uint64_t *rmask = a.rec_mask + (C.rg0 + lg) * kRecCap;
    // kRecBatch chunks of 64 records per round trip (lane = record of each chunk)
    for (uint32_t b0 = 0; b0 < n; b0 += kRecBatch * kWave) {
        uint32_t bpi[kRecBatch], blo[kRecBatch], bhi[kRecBatch];
#pragma unroll
        for (int u = 0; u < kRecBatch; ++u) {
            const uint32_t k = b0 + u * kWave + lane;
            const bool have = k < n;
            const uint64_t pm = have ? rmask[k] : 0ull;
            bpi[u] = have ? ridx[k] : 0u;
            blo[u] = static_cast<uint32_t>(pm);
            bhi[u] = static_cast<uint32_t>(pm >> 32);
        }
        // the previous batch's rows were written (and read) already
#pragma unroll
        for (int u = 0; u < kRecBatch; ++u) L.pidx[u * kWave + lane] = bpi[u];
#pragma unroll
        for (int u = 0; u < kRecBatch; ++u) {
            const uint32_t c0 = b0 + u * kWave;
            if (c0 >= n) break;
            const uint32_t m = min(n - c0, static_cast<uint32_t>(kWave));
            const uint32_t lo = blo[u], hi = bhi[u];
            for (uint32_t j0 = 0; j0 < m; j0 += kChunk) {
                flush(kRowCap - kChunk);
                const uint32_t je = min(m, j0 + kChunk);
                uint8_t *w = myrow + nb;
                auto append = [&](uint32_t j) {
                    const uint64_t mk = (static_cast<uint64_t>(readlane_u32(hi, static_cast<int>(j))) << 32) |
                                        readlane_u32(lo, static_cast<int>(j));
                    *w = static_cast<uint8_t>(u * kWave + j);
                    w += static_cast<uint32_t>(mk >> lane) & 1u;
                };
                if (je - j0 == static_cast<uint32_t>(kChunk)) {
#pragma unroll
                    for (int v = 0; v < kChunk; ++v) append(j0 + v);
                } else {
                    for (uint32_t j = j0; j < je; ++j) append(j);
                }
                nb = static_cast<uint32_t>(w - myrow);
            }
        }
        flush(0);  // the rows point into this batch's records
    }
}

// Long rows, written one query after another: the wave holds up to kRowBlk
// chunks of 64 records in registers (lane = record; 20 chunks cover the
// records of nearly every long-row group, so the wave loads nothing after its
// first store: on this GPU a wait for a load also waits for every store
// issued before it).  For each query the lanes whose record mask holds its
// bit put their original index at the row's next positions (each lane's
// rank among them from mbcnt, which also adds the entries already written).
// A group of a cloud's own points has its rows consecutive in the output, so
// the pieces fill one region in order: they go to an LDS ring written out
// 256 entries at a time with 16-byte stores; other groups store each piece
// straight to its row.
constexpr int kRowBlk = SFC_REC_ROWBLK;
static_assert(kRowBlk >= 1 && kRowBlk <= 32, "record chunks held per pass");

// The queries of `qm` against NCH chunks of records: word[u] / pi[u] hold
// chunk u's mask words (the low ones for queries 0-31, the high ones for
// 32-63) and original indices.  start / len / done: per lane, its row's first
// output position, length and entries written so far.
template <int NCH>
__device__ __forceinline__ void rows_queries(uint64_t qm, const uint32_t (&word)[kRowBlk],
                                             const uint32_t (&pi)[kRowBlk], uint64_t start, uint32_t len,
                                             uint32_t &done, uint32_t *__restrict__ out) {
    for (; qm; qm &= qm - 1) {
        const int j = __builtin_amdgcn_readfirstlane(__ffsll(static_cast<long long>(qm)) - 1);
        const uint32_t rl = readlane_u32(len, j);
        const uint32_t w = readlane_u32(done, j);
        const uint32_t bit = 1u << (j & 31);
        uint64_t m[NCH];
        uint32_t tot = 0;
#pragma unroll
        for (int u = 0; u < NCH; ++u) {
            m[u] = ballot((word[u] & bit) != 0u);
            tot += static_cast<uint32_t>(__popcll(m[u]));
        }
        uint32_t *const row = out + readlane_u64(start, j);
        const bool whole = w + tot <= rl;  // always, when the offsets come from this count
        uint32_t at = w;
#pragma unroll
        for (int u = 0; u < NCH; ++u) {
            const uint32_t pos = at + rank_below(m[u]);
            // a shorter row (offsets not from this count) takes the first of its entries
            if (__builtin_amdgcn_inverse_ballot_w64(m[u]) && (whole || pos < rl)) row[pos] = pi[u];
            at += static_cast<uint32_t>(__popcll(m[u]));
        }
        done = writelane_u32(w + tot, j, done);
    }
}

// the chunk count as a template argument (no per-chunk checks in the loops)
template <int NCH = kRowBlk>
__device__ __forceinline__ void rows_block(int nch, uint64_t rows, const uint32_t (&lo)[kRowBlk],
                                           const uint32_t (&hi)[kRowBlk], const uint32_t (&pi)[kRowBlk],
                                           uint64_t start, uint32_t len, uint32_t &done, uint32_t *out) {
    if constexpr (NCH > 1) {
        if (nch < NCH) {
            rows_block<NCH - 1>(nch, rows, lo, hi, pi, start, len, done, out);
            return;
        }
    }
    rows_queries<NCH>(rows & 0xFFFFFFFFull, lo, pi, start, len, done, out);
    rows_queries<NCH>(rows & ~0xFFFFFFFFull, hi, pi, start, len, done, out);
}

// Staged long rows, for a group whose records fit one block and whose rows
// are consecutive in lane order (then its output is one region [r0, r1),
// written strictly in order): pieces go to an LDS ring of kRowRing entries
// (entry g of the output at g mod kRowRing) and every 256 entries are written
// out as one 16-byte store per lane, so the wave issues a quarter of the
// stores at whole cache lines.  Before a query's pieces fewer than 256
// entries wait in the ring and a query adds at most one entry per record.
// A query whose entries fit the rest of the ring (in a group of at most
// kRowRing - 256 records, every query) writes all its pieces and then writes
// out the full blocks; a longer one writes out the full blocks after each
// piece of at most 64 entries, so the ring never overwrites what it still
// holds.
#ifndef SFC_ROW_RING
#define SFC_ROW_RING 1024
#endif
constexpr uint32_t kRowRing = SFC_ROW_RING;
static_assert((kRowRing & (kRowRing - 1)) == 0 && kRowRing >= 512, "row ring size");
struct RowStage {
    uint32_t *buf;  // LDS, kRowRing entries, 16-byte aligned
    uint32_t *out;  // the output indices, 16-byte aligned
    uint64_t r0, r1, base;  // base: the next entry to write out (a multiple of 4)
};

// Writes out entries [st.base, st.base + 256) that lie in [r0, r1).
__device__ __forceinline__ void stage_flush(RowStage &st) {
    const int lane = lane_id();
    const uint64_t g0 = st.base + 4u * static_cast<uint32_t>(lane);
    wave_sync();
    const uint4 v = *reinterpret_cast<const uint4 *>(st.buf + (static_cast<uint32_t>(g0) & (kRowRing - 1)));
    wave_sync();
    if (g0 >= st.r0 && g0 + 4 <= st.r1) {
        *reinterpret_cast<uint4 *>(st.out + g0) = v;
    } else {
        const uint32_t e[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int i = 0; i < 4; ++i)
            if (g0 + i >= st.r0 && g0 + i < st.r1) st.out[g0 + i] = e[i];
    }
    st.base += 256;
}

template <int NCH>
__device__ __forceinline__ void rows_queries_staged(uint64_t qm, const uint32_t (&word)[kRowBlk],
                                                    const uint32_t (&pi)[kRowBlk], uint64_t start, uint32_t len,
                                                    RowStage &st) {
    // NCH chunks hold at most 64 NCH records: with at most kRowRing - 256,
    // every query's entries fit the ring
    constexpr bool FIT = NCH * kWave + 256 <= static_cast<int>(kRowRing);
    for (; qm; qm &= qm - 1) {
        const int j = __builtin_amdgcn_readfirstlane(__ffsll(static_cast<long long>(qm)) - 1);
        const uint32_t rl = readlane_u32(len, j);
        const uint64_t s0 = readlane_u64(start, j);
        const uint32_t bit = 1u << (j & 31);
        // rows between (longer than their records) are skipped over
        while (s0 >= st.base + 256) stage_flush(st);
        uint64_t m[NCH];
        uint32_t tot = 0;
#pragma unroll
        for (int u = 0; u < NCH; ++u) {
            m[u] = ballot((word[u] & bit) != 0u);
            tot += static_cast<uint32_t>(__popcll(m[u]));
        }
        // the row's whole (always, when the offsets come from this count) and it fits the ring
        if (tot <= rl && (FIT || static_cast<uint32_t>(s0 - st.base) + tot <= kRowRing)) {
            uint32_t at = static_cast<uint32_t>(s0);  // ring positions wrap, so the low word suffices
#pragma unroll
            for (int u = 0; u < NCH; ++u) {
                const uint32_t pos = __builtin_amdgcn_mbcnt_hi(static_cast<uint32_t>(m[u] >> 32),
                                                               __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(m[u]), at));
                if (__builtin_amdgcn_inverse_ballot_w64(m[u])) st.buf[pos & (kRowRing - 1)] = pi[u];
                at += static_cast<uint32_t>(__popcll(m[u]));
            }
        } else {  // piece by piece; a shorter row takes the first of its entries
            uint32_t at = 0;
#pragma unroll
            for (int u = 0; u < NCH; ++u) {
                const uint32_t pos = __builtin_amdgcn_mbcnt_hi(static_cast<uint32_t>(m[u] >> 32),
                                                               __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(m[u]), at));
                if (__builtin_amdgcn_inverse_ballot_w64(m[u]) && pos < rl)
                    st.buf[(static_cast<uint32_t>(s0) + pos) & (kRowRing - 1)] = pi[u];
                at += static_cast<uint32_t>(__popcll(m[u]));
                if constexpr (!FIT) {
                    const uint64_t front = s0 + min(at, rl);
                    while (front >= st.base + 256) stage_flush(st);
                }
            }
        }
        const uint64_t front = s0 + min(tot, rl);
        while (front >= st.base + 256) stage_flush(st);
    }
}

template <int NCH = kRowBlk>
__device__ __forceinline__ void rows_block_staged(int nch, uint64_t rows, const uint32_t (&lo)[kRowBlk],
                                                  const uint32_t (&hi)[kRowBlk], const uint32_t (&pi)[kRowBlk],
                                                  uint64_t start, uint32_t len, RowStage &st) {
    if constexpr (NCH > 1) {
        if (nch < NCH) {
            rows_block_staged<NCH - 1>(nch, rows, lo, hi, pi, start, len, st);
            return;
        }
    }
    rows_queries_staged<NCH>(rows & 0xFFFFFFFFull, lo, pi, start, len, st);
    rows_queries_staged<NCH>(rows & ~0xFFFFFFFFull, hi, pi, start, len, st);
}

__device__ __forceinline__ void radius_fill_rows_body(const SearchArgs &a, const SearchCloud &C, int64_t lg,
                                                      uint32_t n, uint32_t *stage_buf) {
    const int lane = lane_id();
    const int64_t lr = lg * kWave + lane;
    int64_t row;
    const Query q = lane_query(a, C, lr, &row);
    const int64_t orow = q.valid ? row : 0;
    const uint64_t o0 = a.offsets[orow], o1 = a.offsets[orow + 1];
    const uint64_t start = q.valid ? o0 : 0ull;
    // counts are 32-bit, so a row's length is too
    const uint32_t len = q.valid && o1 > o0 ? static_cast<uint32_t>(o1 - o0) : 0u;
    uint32_t done = 0;  // entries of the lane's row written so far
    const uint64_t rows = ballot(len > 0);
    const uint32_t *ridx = a.rec_idx + (C.rg0 + lg) * kRecCap;
    const uint64_t *rmask = a.rec_mask + (C.rg0 + lg) * kRecCap;
    // one block, rows consecutive in lane order, output 16-byte aligned: staged
    const int64_t row0 = readlane_u64(static_cast<uint64_t>(row), 0);
    const bool consecutive = ballot(q.valid && row != row0 + lane) == 0ull;
    if (n <= static_cast<uint32_t>(kRowBlk * kWave) && consecutive &&
        (reinterpret_cast<uintptr_t>(a.indices) & 15u) == 0 && rows) {
        uint32_t pi[kRowBlk], lo[kRowBlk], hi[kRowBlk];
#pragma unroll
        for (int u = 0; u < kRowBlk; ++u) {
            const uint32_t k = u * kWave + lane;
            const bool have = k < n;
            const uint64_t pm = have ? rmask[k] : 0ull;
            pi[u] = have ? ridx[k] : 0u;
            lo[u] = static_cast<uint32_t>(pm);
            hi[u] = static_cast<uint32_t>(pm >> 32);
        }
        RowStage st;
        st.buf = stage_buf;
        st.out = a.indices;
        const int last = 63 - __clzll(static_cast<long long>(ballot(q.valid)));
        st.r0 = readlane_u64(start, 0);
        st.r1 = readlane_u64(start + len, last);
        st.base = st.r0 & ~3ull;
        const int nch = static_cast<int>(min((n + kWave - 1) / kWave, static_cast<uint32_t>(kRowBlk)));
        rows_block_staged(nch, rows, lo, hi, pi, start, len, st);
        while (st.base < st.r1) stage_flush(st);
        return;
    }
    // otherwise each piece is stored straight to its row
    for (uint32_t b0 = 0; b0 < n; b0 += kRowBlk * kWave) {
        uint32_t pi[kRowBlk], lo[kRowBlk], hi[kRowBlk];
#pragma unroll
        for (int u = 0; u < kRowBlk; ++u) {
            const uint32_t k = b0 + u * kWave + lane;
            const bool have = k < n;
            const uint64_t pm = have ? rmask[k] : 0ull;
            pi[u] = have ? ridx[k] : 0u;
            lo[u] = static_cast<uint32_t>(pm);
            hi[u] = static_cast<uint32_t>(pm >> 32);
        }
        const int nch = static_cast<int>(min((n - b0 + kWave - 1) / kWave, static_cast<uint32_t>(kRowBlk)));
        rows_block(nch, rows, lo, hi, pi, start, len, done, a.indices);
    }
}

// One query's row [pos, end): contained candidates are copied from the
// permutation (their points in sorted order), points of mixed ones are tested
// with lane = point and compacted with ballot; both give coalesced stores.
template <int KERNEL>
__device__ __forceinline__ void fill_one(RadLds &L, const SearchCloud &C, float qx, float qy, float qz, float r,
                                         float r2, bool prune, uint64_t pos, uint64_t end, uint32_t *out) {
    const int lane = lane_id();
    walk_one<KERNEL>(
        L, C, qx, qy, qz, r, r2, prune,
        [&](int c0, uint64_t fm, uint32_t) {
            for (uint64_t b = fm; b; b &= b - 1) {
                const int j = __ffsll(static_cast<long long>(b)) - 1;
                const uint32_t beg = L.cbeg[c0 + j], len = L.clen[j];
                for (uint32_t t0 = 0; t0 < len; t0 += kWave) {
                    const uint32_t t = t0 + lane;
                    if (t < len && pos + t < end) out[pos + t] = C.perm[beg + t];
                }
                pos += len;
            }
        },
        [&](uint32_t n) {
            for (uint32_t t0 = 0; t0 < n; t0 += kWave) {
                const uint32_t t = t0 + lane;
                const float4 p = L.pts[t < n ? t : 0];
                const bool h = t < n && point_hit<KERNEL>(p, qx, qy, qz, r, r2);
                const uint64_t m = ballot(h);
                const uint64_t at = pos + rank_below(m);
                if (h && at < end) out[at] = __float_as_uint(p.w);
                pos += static_cast<uint64_t>(__popcll(m));
            }
        });
}

template <int KERNEL, int STAGE>
__device__ __forceinline__ void radius_fill_body(FillLdsT<STAGE> &L, const SearchArgs &a, const SearchCloud &C,
                                                 int64_t lg) {
    const int lane = lane_id();
    const int64_t lr = lg * kWave + lane;
    int64_t row;
    const Query q = lane_query(a, C, lr, &row);
    const float r = C.r, r2 = fmul(r, r);
    if (!(r > 0.0f)) return;  // empty rows
    const bool prune = !(a.flags & SFC_NO_PRUNE);
    int sid = 0;
    const int nseg = make_segments(L, q, 2.0f * r, &sid, kJumpSteps);
    // an invalid lane owns an empty row and never appends
    // loaded by every lane (a lane without a query reads row 0 and drops it),
    // so the wait for the loads is not left inside a branch
    const int64_t orow = q.valid ? row : 0;
    const uint64_t o0 = a.offsets[orow], o1 = a.offsets[orow + 1];
    uint64_t gpos = q.valid ? o0 : 0ull;
    const uint64_t gend = q.valid ? o1 : 0ull;
    uint64_t left = gend > gpos ? gend - gpos : 0ull;  // entries the row can still take
    if (may_defer(a) && spread_group(L, nseg, r, __popcll(ballot(q.valid)))) {
        defer_group(a, lg + C.g0);
        return;
    }
    uint32_t nb = 0;
    uint8_t *myrow = L.rows + lane * (kRowCap + 1);
    uint32_t *out = a.indices;
    // a lane without a query tests against a point at infinity: it never
    // hits (finite points), so its row stays empty
    const float qx = q.valid ? q.x : INFINITY, qy = q.valid ? q.y : INFINITY, qz = q.valid ? q.z : INFINITY;
    const int half = lane >> 5, hl = lane & 31;

    // Writes out every row holding more than `limit` entries, two rows per
    // step (one per half wave, 32 consecutive slots each: coalesced stores).
    // Each flushed row publishes its cursor in LDS (clamped to the row's end,
    // so a row never spills into its neighbour) and joins a compact list.
    auto flush = [&](uint32_t limit) {
        const bool go = nb > limit;
        const uint64_t fm = ballot(go);
        if (!fm) return;
        const int nf = __popcll(fm);
        if (go) {
            const uint32_t i = rank_below(fm);
            L.fpos[i] = gpos;
            L.fmeta[i] = static_cast<uint32_t>(lane) | (static_cast<uint32_t>(left < nb ? left : nb) << 8);
        }
        wave_sync();
        for (int i0 = 0; i0 < nf; i0 += 2) {
            const int i = i0 + half;
            if (i < nf) {
                const uint32_t meta = L.fmeta[i];
                const uint64_t pos = L.fpos[i];
                const uint32_t slot = L.rows[(meta & 0xFFu) * (kRowCap + 1) + hl];  // hl < kRowCap + 1
                if (static_cast<uint32_t>(hl) < (meta >> 8)) out[pos + hl] = __float_as_uint(L.pts[slot].w);
            }
        }
        if (go) {
            gpos += nb;
            left -= left < nb ? left : nb;
            nb = 0;
        }
        wave_sync();
    };
    // every lane tests its query against the staged points and appends the
    // slots of its hits to its row
    auto body = [&](uint32_t n_) {
        const uint32_t n = __builtin_amdgcn_readfirstlane(n_);
        for (uint32_t t0 = 0; t0 < n; t0 += kChunk) {
            flush(kRowCap - kChunk);
            const uint32_t te = min(n, t0 + kChunk);
            uint32_t t = t0;
            uint8_t *w = myrow + nb;  // next free slot
            for (; t + 4 <= te; t += 4) {
                const float4 p0 = L.pts[t], p1 = L.pts[t + 1], p2 = L.pts[t + 2], p3 = L.pts[t + 3];
                const bool h0 = point_hit<KERNEL>(p0, qx, qy, qz, r, r2);
                const bool h1 = point_hit<KERNEL>(p1, qx, qy, qz, r, r2);
                const bool h2 = point_hit<KERNEL>(p2, qx, qy, qz, r, r2);
                const bool h3 = point_hit<KERNEL>(p3, qx, qy, qz, r, r2);
                // each slot is overwritten unless it holds a hit
                *w = static_cast<uint8_t>(t + 0);
                w += h0;
                *w = static_cast<uint8_t>(t + 1);
                w += h1;
                *w = static_cast<uint8_t>(t + 2);
                w += h2;
                *w = static_cast<uint8_t>(t + 3);
                w += h3;
            }
            for (; t < te; ++t) {
                const bool h = point_hit<KERNEL>(L.pts[t], qx, qy, qz, r, r2);
                *w = static_cast<uint8_t>(t);
                w += h;
            }
            nb = static_cast<uint32_t>(w - myrow);
        }
        flush(0);  // the rows point into this round's staged points
    };
    uint32_t staged = 0;  // points staged and not yet swept, across candidate batches
    auto accept = [&](const sfc_node &nd) { return segments_may_hit<KERNEL>(L, nseg, nd, r, r2); };
    auto sweep = [&](int ncand) {
        for (int c0 = 0; c0 < ncand; c0 += kWave) {
            const int m = min(kWave, ncand - c0);
            uint64_t mixed, touched, full;
            const uint32_t len = classify_segments<KERNEL>(L, C.nodes, c0, m, nseg, sid, r, r2, prune, &mixed, &touched, &full);
            if (!touched) continue;
            stage_union<KERNEL>(L, C.pts, c0, m, touched, len, nseg, r, r2, body, &staged);
        }
    };
    traverse(L, C.nodes, C.child, accept, sweep, start_node<KERNEL>(L, a, C, nseg, r, q, lr));
    if (staged) {
        wave_sync();
        body(staged);
    }
    flush(0);
}

// ------------------------------------------------------- range output
// The paper's neighboursStruct form (Section 5.1): per query, the ranges of
// sorted positions of the nodes that lie entirely inside its neighbourhood,
// and the individual points of the nodes it overlaps only partly.  Nodes are
// classified per lane (the lane's own query against each candidate node,
// exact by the monotonicity argument); the points of a node that is
// contained for a lane are not tested for that lane, so ranges and points
// are disjoint and their union is the radius_search set.
template <int KERNEL>
__device__ __forceinline__ void struct_body(StructLds &L, const SearchArgs &a, const SearchCloud &C, int64_t lg,
                                            bool fill) {
    const int lane = lane_id();
    const int64_t lr = lg * kWave + lane;
    int64_t row;
    const Query q = lane_query(a, C, lr, &row);
    const float r = C.r, r2 = fmul(r, r);
    const bool prune = !(a.flags & SFC_NO_PRUNE);
    uint32_t nr = 0, np = 0;
    if (r > 0.0f) {
        int sid = 0;
        const int nseg = make_segments(L, q, 2.0f * r, &sid, kJumpSteps);
        uint64_t rpos = 0, rend = 0, gpos = 0, gend = 0;
        if (fill && q.valid) {
            rpos = a.roffsets[row];
            rend = a.roffsets[row + 1];
            gpos = a.offsets[row];
            gend = a.offsets[row + 1];
        }
        uint32_t nb = 0;
        uint8_t *myrow = L.rows + lane * (kRowCap + 1);
        const int half = lane >> 5, hl = lane & 31;
        auto flush = [&](uint32_t limit) {
            const bool go = nb > limit;
            const uint64_t fm = ballot(go);
            if (!fm) return;
            const int nf = __popcll(fm);
            if (go) {
                const uint64_t room = gend > gpos ? gend - gpos : 0ull;
                const uint32_t i = rank_below(fm);
                L.fpos[i] = gpos;
                L.fmeta[i] = static_cast<uint32_t>(lane) | (static_cast<uint32_t>(room < nb ? room : nb) << 8);
            }
            wave_sync();
            for (int i = half; i < nf; i += 2) {
                const uint32_t meta = L.fmeta[i];
                const uint64_t pos = L.fpos[i];
                const uint32_t slot = L.rows[(meta & 0xFFu) * (kRowCap + 1) + hl];  // hl < kRowCap + 1
                if (static_cast<uint32_t>(hl) < (meta >> 8)) a.indices[pos + hl] = __float_as_uint(L.pts[slot].w);
            }
            if (go) {
                gpos += nb;
                nb = 0;
            }
            wave_sync();
        };
        auto accept = [&](const sfc_node &nd) { return segments_may_hit<KERNEL>(L, nseg, nd, r, r2); };
        auto sweep = [&](int ncand) {
            for (int c0 = 0; c0 < ncand; c0 += kWave) {
                const int m = min(kWave, ncand - c0);
                const uint32_t len = lane < m ? L.cend[c0 + lane] - L.cbeg[c0 + lane] : 0u;
                uint64_t full = 0, mixed = 0;
                for (int i = 0; i < m; ++i) {
                    const sfc_node nd = C.nodes[__builtin_amdgcn_readfirstlane(L.cand[c0 + i])];
                    int cls = q.valid ? classify<KERNEL>(nd, q.x, q.y, q.z, r, r2) : 0;
                    if (cls == 1 && !prune) cls = 2;
                    full |= static_cast<uint64_t>(cls == 1) << i;
                    mixed |= static_cast<uint64_t>(cls == 2) << i;
                }
                if (!fill) {
                    nr += static_cast<uint32_t>(__popcll(full));
                } else {
                    for (int i = 0; i < m; ++i) {
                        if ((full >> i) & 1ull) {
                            if (rpos < rend) {
                                a.ranges[2 * rpos] = L.cbeg[c0 + i];
                                a.ranges[2 * rpos + 1] = L.cend[c0 + i];
                            }
                            ++rpos;
                        }
                    }
                }
                const uint64_t need = wave_or(mixed);
                if (!need) continue;
                stage_union<KERNEL, true>(L, C.pts, c0, m, need, len, nseg, r, r2, [&](uint32_t n) {
                    if (!fill) {
                        for (uint32_t t = 0; t < n; ++t)
                            np += (point_hit<KERNEL>(L.pts[t], q.x, q.y, q.z, r, r2) && ((mixed >> L.owner[t]) & 1ull))
                                      ? 1u : 0u;
                        return;
                    }
                    for (uint32_t t0 = 0; t0 < n; t0 += kChunk) {
                        flush(kRowCap - kChunk);
                        const uint32_t te = min(n, t0 + kChunk);
                        for (uint32_t t = t0; t < te; ++t) {
                            const bool h = point_hit<KERNEL>(L.pts[t], q.x, q.y, q.z, r, r2) &
                                           (((mixed >> L.owner[t]) & 1ull) != 0);
                            myrow[nb] = static_cast<uint8_t>(t);
                            nb += h ? 1u : 0u;
                        }
                    }
                    flush(0);
                });
            }
        };
        traverse(L, C.nodes, C.child, accept, sweep);
    }
    if (!fill && q.valid) {
        a.rcounts[row] = nr;
        a.counts[row] = np;
    }
}

}  // namespace

__global__ __launch_bounds__(64) void k_struct_count(SearchArgs a) {
    __shared__ StructLds L;
    const int64_t g = xcd_item(blockIdx.x, gridDim.x);
    if (g >= a.groups) return;
    const SearchCloud C = group_cloud(a, g);
    const int64_t lg = g - C.g0;
    switch (C.kernel) {
    case SFC_SPHERE: struct_body<SFC_SPHERE>(L, a, C, lg, false); break;
    case SFC_CIRCLE: struct_body<SFC_CIRCLE>(L, a, C, lg, false); break;
    case SFC_CUBE: struct_body<SFC_CUBE>(L, a, C, lg, false); break;
    default: struct_body<SFC_SQUARE>(L, a, C, lg, false); break;
    }
}

__global__ __launch_bounds__(64) void k_struct_fill(SearchArgs a) {
    __shared__ StructLds L;
    const int64_t g = xcd_item(blockIdx.x, gridDim.x);
    if (g >= a.groups) return;
    // either buffer too small: write nothing
    if (a.offsets[a.nq_total] > a.capacity || a.roffsets[a.nq_total] > a.rcapacity) return;
    const SearchCloud C = group_cloud(a, g);
    const int64_t lg = g - C.g0;
    switch (C.kernel) {
    case SFC_SPHERE: struct_body<SFC_SPHERE>(L, a, C, lg, true); break;
    case SFC_CIRCLE: struct_body<SFC_CIRCLE>(L, a, C, lg, true); break;
    case SFC_CUBE: struct_body<SFC_CUBE>(L, a, C, lg, true); break;
    default: struct_body<SFC_SQUARE>(L, a, C, lg, true); break;
    }
}

namespace {

// The record state the count kernel wrote, read through the device-coherent
// vector path (uniform addresses would otherwise go through the scalar data
// cache, which is only as fresh as its last invalidation).
template <typename T>
__device__ __forceinline__ T coherent_load(const T *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// do the workspace's records come from the count call this fill follows?
__device__ __forceinline__ bool records_valid(const SearchArgs &a) {
    if (!a.rec_tag) return false;
    const uint64_t t0 = coherent_load(a.rec_tag), t1 = coherent_load(a.rec_tag + 1);  // both loads in flight
    return t0 == a.tag0 && t1 == a.tag1;
}

}  // namespace

// The count and search-fill kernels come in one kernel per staging tile (a
// kernel holding every tile's body would need the registers of the largest
// one in every cloud); the host launches those of the tiles its clouds use,
// each serving the groups of its own tile's clouds, with the tile's layout
// in the launch's dynamic LDS.
extern __shared__ __align__(16) unsigned char g_radius_lds[];

// a cloud's staging tile (64, 128 or 256 points; anything else is 128)
__device__ __forceinline__ int tile_of(const SearchCloud &C) {
    return C.stage == 64 ? 64 : C.stage == 256 ? 256 : 128;
}

template <bool REC, int STAGE>
__device__ __forceinline__ void radius_count_tile(const SearchArgs &a, const SearchCloud &C, int64_t lg) {
    RadLdsT<STAGE> &L = *reinterpret_cast<RadLdsT<STAGE> *>(g_radius_lds);
    switch (C.kernel) {
    case SFC_SPHERE: radius_count_body<SFC_SPHERE, REC, STAGE>(L, a, C, lg); break;
    case SFC_CIRCLE: radius_count_body<SFC_CIRCLE, REC, STAGE>(L, a, C, lg); break;
    case SFC_CUBE: radius_count_body<SFC_CUBE, REC, STAGE>(L, a, C, lg); break;
    default: radius_count_body<SFC_SQUARE, REC, STAGE>(L, a, C, lg); break;
    }
}

// One wave per group of 64 queries of one cloud of the kernel's tile; the
// cloud's kernel selects the (wave-uniform) body.
template <int STAGE>
__device__ __forceinline__ void radius_count_kernel(const SearchArgs &a) {
    const int64_t g = xcd_item(blockIdx.x, gridDim.x);
    if (g >= a.groups) return;
    const SearchCloud C = group_cloud(a, g);
    if (tile_of(C) != STAGE) return;
    radius_count_tile<false, STAGE>(a, C, g - C.g0);
}

// the count that also records the hits of every group of the recording
// clouds (SFC_RECORD_HITS, or the cloud's own choice in a batch); groups of
// the other clouds are counted plainly and left to k_radius_fill
template <int STAGE>
__device__ __forceinline__ void radius_count_rec_kernel(const SearchArgs &a) {
    const int64_t g = xcd_item(blockIdx.x, gridDim.x);
    if (g >= a.groups) return;
    if (g == 0 && lane_id() == 0) {  // the records' provenance (read by the fills, which run after this kernel)
        a.rec_tag[0] = a.tag0;
        a.rec_tag[1] = a.tag1;
    }
    const SearchCloud C = group_cloud(a, g);
    if (tile_of(C) != STAGE) return;
    if (C.rec) {
        radius_count_tile<true, STAGE>(a, C, g - C.g0);
    } else {
        if (lane_id() == 0) a.rec_n[g] = kRecOverflow;
        radius_count_tile<false, STAGE>(a, C, g - C.g0);
    }
}

// the default tile's kernels, then those of the 64- and 256-point tiles
__global__ __launch_bounds__(64) void k_radius_count(SearchArgs a) { radius_count_kernel<128>(a); }
__global__ __launch_bounds__(64) void k_radius_count_t64(SearchArgs a) { radius_count_kernel<64>(a); }
__global__ __launch_bounds__(64) void k_radius_count_t256(SearchArgs a) { radius_count_kernel<256>(a); }
__global__ __launch_bounds__(64) void k_radius_count_rec(SearchArgs a) { radius_count_rec_kernel<128>(a); }
__global__ __launch_bounds__(64) void k_radius_count_rec_t64(SearchArgs a) { radius_count_rec_kernel<64>(a); }
__global__ __launch_bounds__(64) void k_radius_count_rec_t256(SearchArgs a) { radius_count_rec_kernel<256>(a); }

// Rows of the recorded groups that took the short-row form; the long-row
// groups are k_radius_fill_rows' and those whose records did not fit
// k_radius_fill's.  One wave per group, as in the count: a wave that took
// several groups in turn would wait, before each next group's loads, for
// every store of the previous one.
__global__ __launch_bounds__(64) void k_radius_fill_rec(SearchArgs a) {
    const int64_t g = xcd_item(blockIdx.x, gridDim.x);
    if (g >= a.groups) return;
    if (!records_valid(a)) return;  // no records of this count (rec_n may be null): k_radius_fill searches every group
    const uint32_t v = __builtin_amdgcn_readfirstlane(coherent_load(a.rec_n + g));
    if (v == kRecOverflow || (v & kRecLongRows)) return;
    if (a.offsets[a.nq_total] > a.capacity) return;  // caller's buffer too small: write nothing
    const SearchCloud C = group_cloud(a, g);
    if (!(C.r > 0.0f)) return;  // empty rows
    radius_fill_rec_body(*reinterpret_cast<RecLds *>(g_radius_lds), a, C, g - C.g0,
                         min(v, static_cast<uint32_t>(kRecCap)));
}

// Rows of the recorded groups that took the long-row form.
__global__ __launch_bounds__(64) void k_radius_fill_rows(SearchArgs a) {
    const int64_t g = xcd_item(blockIdx.x, gridDim.x);
    if (g >= a.groups) return;
    if (!records_valid(a)) return;
    const uint32_t v = __builtin_amdgcn_readfirstlane(coherent_load(a.rec_n + g));
    if (v == kRecOverflow || !(v & kRecLongRows)) return;
    if (a.offsets[a.nq_total] > a.capacity) return;
    const SearchCloud C = group_cloud(a, g);
    if (!(C.r > 0.0f)) return;
    __shared__ __align__(16) uint32_t stage_buf[kRowRing];
    radius_fill_rows_body(a, C, g - C.g0, min(v & ~kRecLongRows, static_cast<uint32_t>(kRecCap)), stage_buf);
}

template <int STAGE>
__device__ __forceinline__ void radius_fill_tile(const SearchArgs &a, const SearchCloud &C, int64_t lg) {
    FillLdsT<STAGE> &L = *reinterpret_cast<FillLdsT<STAGE> *>(g_radius_lds);
    switch (C.kernel) {
    case SFC_SPHERE: radius_fill_body<SFC_SPHERE, STAGE>(L, a, C, lg); break;
    case SFC_CIRCLE: radius_fill_body<SFC_CIRCLE, STAGE>(L, a, C, lg); break;
    case SFC_CUBE: radius_fill_body<SFC_CUBE, STAGE>(L, a, C, lg); break;
    default: radius_fill_body<SFC_SQUARE, STAGE>(L, a, C, lg); break;
    }
}

// group g, if its cloud has the kernel's tile
template <int STAGE>
__device__ __forceinline__ void radius_fill_group(const SearchArgs &a, int64_t g) {
    const SearchCloud C = group_cloud(a, g);
    if (tile_of(C) != STAGE) return;
    radius_fill_tile<STAGE>(a, C, g - C.g0);
}

// One wave per group; or, when every cloud of the launch records its hits
// (a.fill_scan), one wave per kFillScan groups that picks out the groups
// whose records overflowed and serves them in turn: a search with none costs
// an eighth of the waves, one where all overflow at most 8 groups in a row
// per wave.
constexpr int kFillScan = 8;

template <int STAGE>
__device__ __forceinline__ void radius_fill_kernel(const SearchArgs &a) {
    if (a.fill_scan) {
        const int64_t g0 = xcd_item(blockIdx.x, gridDim.x) * kFillScan;
        if (g0 >= a.groups) return;
        if (a.offsets[a.nq_total] > a.capacity) return;
        const bool valid = records_valid(a);  // else every group is searched
        const int64_t g = g0 + lane_id();
        const bool need = lane_id() < kFillScan && g < a.groups &&
                          (!valid || coherent_load(a.rec_n + g) == kRecOverflow);
        for (uint64_t m = ballot(need); m; m &= m - 1)
            radius_fill_group<STAGE>(a, g0 + __builtin_amdgcn_readfirstlane(__ffsll(static_cast<long long>(m)) - 1));
        return;
    }
    const int64_t g = xcd_item(blockIdx.x, gridDim.x);
    if (g >= a.groups) return;
    if (a.offsets[a.nq_total] > a.capacity) return;  // caller's buffer too small: write nothing
    if (a.rec_n && records_valid(a) && coherent_load(a.rec_n + g) != kRecOverflow) return;  // written from its records
    radius_fill_group<STAGE>(a, g);
}

__global__ __launch_bounds__(64) void k_radius_fill(SearchArgs a) { radius_fill_kernel<128>(a); }
__global__ __launch_bounds__(64) void k_radius_fill_t64(SearchArgs a) { radius_fill_kernel<64>(a); }
__global__ __launch_bounds__(64) void k_radius_fill_t256(SearchArgs a) { radius_fill_kernel<256>(a); }

// Deferred (spread) groups: one wave per query, grid-stride over the list.
__global__ __launch_bounds__(64) void k_radius_count_spread(SearchArgs a) {
    __shared__ RadLds L;
    const int64_t total = static_cast<int64_t>(*a.nspread) * kWave;
    for (int64_t j = xcd_item(blockIdx.x, gridDim.x); j < total; j += gridDim.x) {
        const int64_t g = a.spread[j / kWave];
        const SearchCloud C = group_cloud(a, g);
        const int64_t lr = (g - C.g0) * kWave + (j % kWave);
        if (lr >= C.nq) continue;
        int64_t row;
        const Query q = lane_query(a, C, lr, &row);
        const float r = C.r, r2 = fmul(r, r);
        const bool prune = !(a.flags & SFC_NO_PRUNE);
        uint32_t c;
        switch (C.kernel) {
        case SFC_SPHERE: c = count_one<SFC_SPHERE>(L, C, q.x, q.y, q.z, r, r2, prune); break;
        case SFC_CIRCLE: c = count_one<SFC_CIRCLE>(L, C, q.x, q.y, q.z, r, r2, prune); break;
        case SFC_CUBE: c = count_one<SFC_CUBE>(L, C, q.x, q.y, q.z, r, r2, prune); break;
        default: c = count_one<SFC_SQUARE>(L, C, q.x, q.y, q.z, r, r2, prune); break;
        }
        if (lane_id() == 0) a.counts[row] = c;
    }
}

__global__ __launch_bounds__(64) void k_radius_fill_spread(SearchArgs a) {
    __shared__ RadLds L;
    if (a.offsets[a.nq_total] > a.capacity) return;
    const int64_t total = static_cast<int64_t>(*a.nspread) * kWave;
    for (int64_t j = xcd_item(blockIdx.x, gridDim.x); j < total; j += gridDim.x) {
        const int64_t g = a.spread[j / kWave];
        const SearchCloud C = group_cloud(a, g);
        const int64_t lr = (g - C.g0) * kWave + (j % kWave);
        if (lr >= C.nq) continue;
        int64_t row;
        const Query q = lane_query(a, C, lr, &row);
        const float r = C.r, r2 = fmul(r, r);
        const bool prune = !(a.flags & SFC_NO_PRUNE);
        const uint64_t pos = a.offsets[row], end = a.offsets[row + 1];
        switch (C.kernel) {
        case SFC_SPHERE: fill_one<SFC_SPHERE>(L, C, q.x, q.y, q.z, r, r2, prune, pos, end, a.indices); break;
        case SFC_CIRCLE: fill_one<SFC_CIRCLE>(L, C, q.x, q.y, q.z, r, r2, prune, pos, end, a.indices); break;
        case SFC_CUBE: fill_one<SFC_CUBE>(L, C, q.x, q.y, q.z, r, r2, prune, pos, end, a.indices); break;
        default: fill_one<SFC_SQUARE>(L, C, q.x, q.y, q.z, r, r2, prune, pos, end, a.indices); break;
        }
    }
}

__global__ void k_reset_spread(uint32_t *nspread) {
    if (threadIdx.x == 0) *nspread = 0;
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

// Minimum and maximum of two k-NN keys viewed as doubles.  Keys are never
// NaNs, so no operand needs quietening first.
__device__ __forceinline__ double key_min(double a, double b) {
    double r;
    asm("v_min_f64 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
    return r;
}
__device__ __forceinline__ double key_max(double a, double b) {
    double r;
    asm("v_max_f64 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
    return r;
}
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

// tau: the largest d2 over a window of at least k consecutive curve points
// is an upper bound of the k-th distance; take the best of 5 windows sliding
// over the 8 blocks of kb = ceil(k/4) points around the query's curve
// position (at a jump of the curve one window lies on the query's side).
// lr is the query's position in the cloud for cloud queries.
__device__ __forceinline__ float curve_tau(const SearchArgs &a, const SearchCloud &C, const Query &q, int64_t lr,
                                           int k) {
    const int64_t n = C.n;
    float tau = INFINITY;
    if (n >= k) {
        int64_t pos = lr;
        if (a.queries) pos = lower_bound_keys<uint64_t>(C.keys, n, point_key(q.x, q.y, q.z, *C.frame));
        const int kb = (k + 3) / 4;
        if (n >= 8 * kb) {
            int64_t s0 = pos - 4 * kb;
            if (s0 > n - 8 * kb) s0 = n - 8 * kb;
            if (s0 < 0) s0 = 0;
            float blk[8];
#pragma unroll
            for (int b = 0; b < 8; ++b) {
                float m = 0.0f;
                for (int i = 0; i < kb; ++i) m = fmaxf(m, dist2(C.pts[s0 + b * kb + i], q.x, q.y, q.z));
                blk[b] = m;
            }
#pragma unroll
            for (int w = 0; w < 5; ++w)
                tau = fminf(tau, fmaxf(fmaxf(blk[w], blk[w + 1]), fmaxf(blk[w + 2], blk[w + 3])));
        } else {
            int64_t s = pos - k / 2;
            if (s > n - k) s = n - k;
            if (s < 0) s = 0;
            tau = 0.0f;
            for (int i = 0; i < k; ++i) tau = fmaxf(tau, dist2(C.pts[s + i], q.x, q.y, q.z));
        }
    }
    return tau;
}

}  // namespace

// k-NN in at most two exact rounds per wave.
//  * tau_l (per lane) bounds the k-th distance from above: the largest d2 over
//    the query's k curve neighbours.
//  * Round 1 searches every active query out to R1 = the median of tau over
//    the wave and inserts points with d2 <= R1.  A lane is done when tau_l <=
//    R1 or its list is full with k-th d2 <= R1: every point that can still
//    belong to its answer was within R1 and has been seen.
//  * Round 2 serves the remaining lanes, each segment with its own radius (the
//    largest tau of its lanes), inserting only points with d2 > R1 (those with
//    d2 <= R1 were all seen in round 1), so no point is inserted twice.
// Candidate nodes are pruned per lane only on near2 > bound (equality kept:
// an equal d2 with a smaller index may still enter).
template <int KMAX>
__global__ __launch_bounds__(64) void k_knn(SearchArgs a) {
    __shared__ WaveLds L;
    __shared__ float s_segr2[kSegMax];
    const int64_t g = xcd_item(blockIdx.x, gridDim.x);
    if (g >= a.groups) return;
    const SearchCloud C = group_cloud(a, g);
    const int lane = lane_id();
    const int64_t lr = (g - C.g0) * kWave + lane;
    int64_t row;
    const Query q = lane_query(a, C, lr, &row);
    const int k = C.k;

    const float tau = q.valid ? curve_tau(a, C, q, lr, k) : INFINITY;
    // R1: median of tau over the valid lanes (bisection on the order-preserving
    // bit pattern of non-negative floats)
    const int nvalid = __popcll(ballot(q.valid));
    const uint32_t tb = q.valid ? __float_as_uint(tau) : 0xFFFFFFFFu;
    uint32_t lo = 0u, hi = 0x7F800000u;  // +inf
    const int want = (nvalid + 1) / 2;
    while (lo < hi) {
        const uint32_t mid = lo + (hi - lo) / 2;
        if (__popcll(ballot(tb <= mid)) >= want)
            hi = mid;
        else
            lo = mid + 1;
    }
    const float R1 = __uint_as_float(lo);
    if (may_defer(a) && R1 > 0.0f && R1 < INFINITY) {
        const int nseg0 = make_segments(L, q, 2.0f * sqrtf(R1), nullptr);
        if (spread_group(L, nseg0, sqrtf(R1), nvalid, 0.25f)) {
            defer_group(a, g);
            return;
        }
    }

    // Entries past k hold 0, the smallest key, so they never move up.  Keys
    // are non-negative and below the bit pattern of +inf as a double (d2 <=
    // +inf as a float keeps the top 12 bits at most 0x7F8), so as IEEE doubles
    // they order exactly as the integers do and the insertion compares them
    // with one 64-bit float min or max each (denormal doubles, the keys with
    // d2 = 0, are preserved in this build).
    // No key is a NaN, so the min and max are issued directly: the compiler's
    // fmin/fmax would first quieten every operand with one more 64-bit op.
    double best[KMAX];
#pragma unroll
    for (int i = 0; i < KMAX; ++i) best[i] = __longlong_as_double(i < k ? kPad : int64_t(0));
    auto kth_of = [&]() { return __uint_as_float(static_cast<uint32_t>(static_cast<uint64_t>(__double_as_longlong(best[0])) >> 32)); };

    bool active = q.valid;
    float lo2 = -1.0f;  // points with d2 <= lo2 were handled by an earlier round
    for (int round = 0; round < 2; ++round) {
        if (!ballot(active)) break;
        const float bound = round == 0 ? fminf(R1, tau) : tau;  // per lane, inclusive
        Query qa = q;
        qa.valid = active;
        const float bmax = wave_max_u(active ? bound : 0.0f);
        const int nseg = make_segments(L, qa, bmax < INFINITY ? 2.0f * sqrtf(bmax) : INFINITY, nullptr);
        // per-segment radius: the largest bound of its lanes (recomputed from
        // the segment boxes written by make_segments)
        for (int sg = 0; sg < nseg; ++sg) {
            const bool in = active && q.x >= L.seg[sg][0] && q.x <= L.seg[sg][3] && q.y >= L.seg[sg][1] &&
                            q.y <= L.seg[sg][4] && q.z >= L.seg[sg][2] && q.z <= L.seg[sg][5];
            const float m = wave_max_u(in ? bound : 0.0f);
            if (lane == 0) s_segr2[sg] = m < INFINITY ? nextafterf(m, INFINITY) : INFINITY;
        }
        wave_sync();
        auto accept = [&](const sfc_node &nd) {
            bool hit = false;
            for (int sg = 0; sg < nseg; ++sg)
                hit = hit || group_may_hit<SFC_SPHERE>(nd, &L.seg[sg][0], &L.seg[sg][3], 0.0f, s_segr2[sg]);
            return hit;
        };
        auto sweep = [&](int ncand) {
            for (int c0 = 0; c0 < ncand; c0 += kWave) {
                const int m = min(kWave, ncand - c0);
                float thr = bound;
                const float kth = kth_of();
                if (kth < thr) thr = kth;
                uint64_t lm = 0;
                if (active) {
                    for (int i = 0; i < m; ++i) {
                        const sfc_node nd = L.cnode[c0 + i];
                        float nx, fx, ny, fy, nz, fz;
                        axis_range(nd.lo[0], nd.hi[0], q.x, nx, fx);
                        axis_range(nd.lo[1], nd.hi[1], q.y, ny, fy);
                        axis_range(nd.lo[2], nd.hi[2], q.z, nz, fz);
                        const float near2 = fadd(fadd(fmul(nx, nx), fmul(ny, ny)), fmul(nz, nz));
                        const float far2 = fadd(fadd(fmul(fx, fx), fmul(fy, fy)), fmul(fz, fz));
                        // equality kept: an equal d2 with a smaller index may still enter
                        if (!(near2 > thr) && far2 > lo2) lm |= 1ull << i;
                    }
                }
                const uint64_t need = wave_or(lm);
                if (!need) continue;
                // a point farther from a segment box than the segment's bound
                // is beyond the bound of each of its lanes (gap test, exact)
                auto reach = [&](const float4 &v) {
                    sfc_node b;
                    b.lo[0] = b.hi[0] = v.x;
                    b.lo[1] = b.hi[1] = v.y;
                    b.lo[2] = b.hi[2] = v.z;
                    bool hit = false;
                    for (int sg = 0; sg < nseg; ++sg)
                        hit = hit || group_may_hit<SFC_SPHERE>(b, &L.seg[sg][0], &L.seg[sg][3], 0.0f, s_segr2[sg]);
                    return hit;
                };
                stage_rounds(L, C.pts, c0, m, need, reach, [&](uint32_t cnt) {
                    for (uint32_t t = 0; t < cnt; ++t) {
                        const float4 p = L.pts[t];
                        const uint32_t o = L.owner[t];
                        const float d = dist2(p, q.x, q.y, q.z);
                        const int64_t x = pack(d, __float_as_uint(p.w));
                        const double xd = __longlong_as_double(x);
                        if (((lm >> o) & 1ull) && d > lo2 && d <= bound && xd < best[0]) {
                            // the list (descending) without its largest key, x
                            // inserted: entry i becomes max(best[i + 1], min(best[i], x))
#pragma unroll
                            for (int i = 0; i < KMAX; ++i) {
                                const double lo = key_min(best[i], xd);
                                best[i] = i + 1 < KMAX ? key_max(best[i + 1], lo) : lo;
                            }
                        }
                    }
                });
            }
        };
        // short lists start below the root (the reach: the segment boxes grown
        // by the largest segment bound); for long lists the extra registers
        // cost more occupancy than the skipped levels save
        int start = 0;
        if constexpr (KMAX <= 16) {
            float smax = 0.0f;
            for (int sg = 0; sg < nseg; ++sg) smax = fmaxf(smax, s_segr2[sg]);
            if (smax < INFINITY) start = start_node<SFC_SPHERE>(L, a, C, nseg, sqrtf(smax), qa, lr);
        }
        traverse(L, C.nodes, C.child, accept, sweep, start);
        // done: the answer lies within the radius already searched
        const float kth = kth_of();
        if (round == 0) active = active && !(tau <= R1 || kth <= R1);
        else active = false;
        lo2 = R1;
    }
    if (q.valid) {
        uint32_t *oi = a.idx + row * a.kstride;
        float *od = a.d2 + row * a.kstride;
#pragma unroll
        for (int i = 0; i < KMAX; ++i) {
            if (i < k) {
                const uint64_t v = static_cast<uint64_t>(__double_as_longlong(best[i]));
                oi[k - 1 - i] = static_cast<uint32_t>(v);
                od[k - 1 - i] = __uint_as_float(static_cast<uint32_t>(v >> 32));
            }
        }
        for (int i = k; i < a.kstride; ++i) {
            oi[i] = 0xFFFFFFFFu;
            od[i] = INFINITY;
        }
    }
}

// ---------------------------------------------------- k-NN of spread groups
namespace {

constexpr int kKnnRegK = 64;        // largest k of the register (group) kernel
constexpr int kKnnBuf = 256;        // candidate keys held per query (k <= kKnnRegK)
constexpr int kKnnBufLarge = 1024;  // the same for k up to kKnnMaxK
constexpr int kKnnMaxK = 512;

template <int BUF>
struct KnnOneLds : RadLds {
    int64_t buf[BUF];
};

// Keeps the k smallest of the cnt keys in L.buf (keys are distinct: the
// index is part of them); returns the k-th smallest.  The k-th key is found
// by bisection on the key value (counting keys <= mid over the wave).
template <int BUF>
__device__ __forceinline__ int64_t keep_k_smallest(KnnOneLds<BUF> &L, int &cnt, int k) {
    const int lane = lane_id();
    int64_t v[BUF / kWave];
#pragma unroll
    for (int i = 0; i < BUF / kWave; ++i) {
        const int e = lane + i * kWave;
        v[i] = e < cnt ? L.buf[e] : INT64_MAX;
    }
    int64_t lo = 0, hi = INT64_MAX;
    while (lo < hi) {
        const int64_t mid = lo + (hi - lo) / 2;
        uint32_t c = 0;
#pragma unroll
        for (int i = 0; i < BUF / kWave; ++i) c += v[i] <= mid ? 1u : 0u;
        if (static_cast<int>(wave_sum_u(c)) >= k)
            hi = mid;
        else
            lo = mid + 1;
    }
    wave_sync();
    int at = 0;
#pragma unroll
    for (int i = 0; i < BUF / kWave; ++i) {
        const bool keep = v[i] <= lo;
        const uint64_t m = ballot(keep);
        if (keep) L.buf[at + static_cast<int>(rank_below(m))] = v[i];
        at += __popcll(m);
    }
    wave_sync();
    cnt = at;
    return lo;
}

// k-NN of one query with the whole wave (lane = candidate point): every
// point with d2 <= tau is a candidate (tau bounds the k-th distance), the
// buffer is cut back to the k best when it fills, and the final k are ranked
// by counting, for each kept key, the kept keys below it.
template <int BUF>
__device__ __forceinline__ void knn_one(KnnOneLds<BUF> &L, const SearchCloud &C, const Query &q, int k, float tau,
                                        uint32_t *oi, float *od, int kstride) {
    const int lane = lane_id();
    int cnt = 0;
    float bound = tau;  // inclusive
    const float r2 = tau < INFINITY ? nextafterf(tau, INFINITY) : INFINITY;
    walk_one<SFC_SPHERE>(
        L, C, q.x, q.y, q.z, tau < INFINITY ? sqrtf(r2) : INFINITY, r2, false, [](int, uint64_t, uint32_t) {},
        [&](uint32_t n) {
            for (uint32_t t0 = 0; t0 < n; t0 += kWave) {
                if (cnt + kWave > BUF) {
                    const int64_t kth = keep_k_smallest(L, cnt, k);
                    bound = __uint_as_float(static_cast<uint32_t>(static_cast<uint64_t>(kth) >> 32));
                }
                const uint32_t t = t0 + lane;
                const float4 p = L.pts[t < n ? t : 0];
                const float d = dist2(p, q.x, q.y, q.z);
                const bool h = t < n && d <= bound;
                const uint64_t m = ballot(h);
                if (h) L.buf[cnt + static_cast<int>(rank_below(m))] = pack(d, __float_as_uint(p.w));
                cnt += __popcll(m);
            }
            wave_sync();
        });
    // more keys than lanes (or than k) are cut back to the k best first
    if (cnt > (k < kWave ? kWave : k)) keep_k_smallest(L, cnt, k);
    const int have = cnt < k ? cnt : k;
    for (int e0 = 0; e0 < cnt; e0 += kWave) {
        const int e = e0 + lane;
        const int64_t mine = e < cnt ? L.buf[e] : INT64_MAX;
        int rank = 0;
        for (int j = 0; j < cnt; ++j) rank += L.buf[j] < mine ? 1 : 0;
        if (e < cnt && rank < k) {
            oi[rank] = static_cast<uint32_t>(static_cast<uint64_t>(mine));
            od[rank] = __uint_as_float(static_cast<uint32_t>(static_cast<uint64_t>(mine) >> 32));
        }
    }
    for (int i = have + lane; i < kstride; i += kWave) {
        oi[i] = 0xFFFFFFFFu;
        od[i] = INFINITY;
    }
    wave_sync();
}

// tau for one query with the whole wave: the k-th smallest d2 over the
// min(n, max(64, 2k)) curve points around the query's curve position (lane j
// takes points j, j + 64, ...), a bound of the k-th distance
template <int PER>
__device__ __forceinline__ float window_tau(const SearchArgs &a, const SearchCloud &C, const Query &q, int64_t lr,
                                            int k) {
    if (C.n < k) return INFINITY;
    int64_t want = 2 * static_cast<int64_t>(k);
    if (want < kWave) want = kWave;
    if (want > static_cast<int64_t>(PER) * kWave) want = static_cast<int64_t>(PER) * kWave;
    const int64_t w = C.n < want ? C.n : want;
    int64_t pos = lr;
    if (a.queries) pos = lower_bound_keys<uint64_t>(C.keys, C.n, point_key(q.x, q.y, q.z, *C.frame));
    int64_t s0 = pos - w / 2;
    if (s0 > C.n - w) s0 = C.n - w;
    if (s0 < 0) s0 = 0;
    const int lane = lane_id();
    uint32_t db[PER];
#pragma unroll
    for (int i = 0; i < PER; ++i) {
        const int64_t j = lane + static_cast<int64_t>(i) * kWave;
        db[i] = j < w ? __float_as_uint(dist2(C.pts[s0 + j], q.x, q.y, q.z)) : 0xFFFFFFFFu;
    }
    uint32_t lo = 0u, hi = 0x7F800000u;
    while (lo < hi) {
        const uint32_t mid = lo + (hi - lo) / 2;
        uint32_t c = 0;
#pragma unroll
        for (int i = 0; i < PER; ++i) c += db[i] <= mid ? 1u : 0u;
        if (static_cast<int>(wave_sum_u(c)) >= k)
            hi = mid;
        else
            lo = mid + 1;
    }
    return __uint_as_float(lo);
}

}  // namespace

// Deferred (spread) k-NN groups: one query per wave.
__global__ __launch_bounds__(64) void k_knn_spread(SearchArgs a) {
    __shared__ KnnOneLds<kKnnBuf> L;
    const int64_t total = static_cast<int64_t>(*a.nspread) * kWave;
    for (int64_t j = xcd_item(blockIdx.x, gridDim.x); j < total; j += gridDim.x) {
        const int64_t g = a.spread[j / kWave];
        const SearchCloud C = group_cloud(a, g);
        const int64_t lr = (g - C.g0) * kWave + (j % kWave);
        if (lr >= C.nq) continue;
        int64_t row;
        const Query q = lane_query(a, C, lr, &row);
        const float tau = window_tau<2 * kKnnRegK / kWave>(a, C, q, lr, C.k);
        knn_one(L, C, q, C.k, tau, a.idx + row * a.kstride, a.d2 + row * a.kstride, a.kstride);
    }
}

// k above what the registers of the group kernel hold: every query with
// the one-query-per-wave scheme.
__global__ __launch_bounds__(64) void k_knn_large(SearchArgs a) {
    __shared__ KnnOneLds<kKnnBufLarge> L;
    const int64_t total = a.groups * kWave;
    for (int64_t j = xcd_item(blockIdx.x, gridDim.x); j < total; j += gridDim.x) {
        const int64_t g = j / kWave;
        const SearchCloud C = group_cloud(a, g);
        const int64_t lr = (g - C.g0) * kWave + (j % kWave);
        if (lr >= C.nq) continue;
        int64_t row;
        const Query q = lane_query(a, C, lr, &row);
        const float tau = window_tau<2 * kKnnMaxK / kWave>(a, C, q, lr, C.k);
        knn_one(L, C, q, C.k, tau, a.idx + row * a.kstride, a.d2 + row * a.kstride, a.kstride);
    }
}

constexpr int kQueryKeyBits = 30;

// External queries in curve order: the code of every query in its cloud's
// frame (same grid of one wave per 64 rows as the searches) ...
__global__ __launch_bounds__(64) void k_query_keys(SearchArgs a, uint64_t *__restrict__ keys,
                                                   uint32_t *__restrict__ perm) {
    const int64_t g = xcd_item(blockIdx.x, gridDim.x);
    if (g >= a.groups) return;
    const SearchCloud C = group_cloud(a, g);
    const int64_t lr = (g - C.g0) * kWave + lane_id();
    if (lr >= C.nq) return;
    const int64_t row = C.q_offset + lr;
    // the leading 30 bits of the code (10 levels: cells of 2^-10 of the
    // frame) order the queries well enough and need 4 sort passes, not 8
    const sfc_frame f = *C.frame;
    const int drop = 3 * f.bits > kQueryKeyBits ? 3 * f.bits - kQueryKeyBits : 0;
    keys[row] = point_key(a.queries[3 * row], a.queries[3 * row + 1], a.queries[3 * row + 2], f) >> drop;
    perm[row] = static_cast<uint32_t>(row);
}

// ... and the first row of every cloud (segments of the sort)
__global__ void k_entry_starts(SearchArgs a, int64_t *starts) {
    for (int c = threadIdx.x; c <= a.B; c += blockDim.x) starts[c] = c < a.B ? a.tab[c].q_offset : a.nq_total;
}

}  // namespace sfc

// -------------------------------------------------------------- C ABI
using namespace sfc;

namespace {

bool tree_ok(const sfc_octree *t) {
    return t && t->nodes && t->child && t->points && t->keys && t->frame && t->n >= 0;
}

SearchCloud cloud_entry(const sfc_octree &t, int64_t q_offset, int64_t nq, int64_t g0, int kernel, float r, int k) {
    SearchCloud c;
    c.nodes = t.nodes;
    c.child = t.child;
    c.pts = reinterpret_cast<const float4 *>(t.points);
    c.perm = t.perm;
    c.keys = t.keys;
    c.frame = t.frame;
    c.n = t.n;
    c.q_offset = q_offset;
    c.nq = nq;
    c.g0 = g0;
    c.r = r;
    c.kernel = kernel;
    c.k = k;
    c.stage = kStage;
    c.rec = 0;
    c.rg0 = 0;
    return c;
}

// Validates a batch for search and builds its host table; returns the total
// group count, or -1 (error set) if the batch is malformed.
int64_t search_table(const char *who, int B, const sfc_cloud *clouds, const float *queries, int64_t nq_total,
                     bool knn, int kstride, std::vector<SearchCloud> &tab, uint32_t flags = 0,
                     int64_t *rec_groups = nullptr) {
    if (B < 1 || B > (1 << 20) || !clouds || nq_total < 0) {
        set_error("%s: invalid batch", who);
        return -1;
    }
    tab.resize(B);
    int64_t rows = 0, g = 0, rg = 0;
    for (int c = 0; c < B; ++c) {
        const sfc_cloud &C = clouds[c];
        const bool kernel_ok = knn ? (C.k >= 1 && C.k <= kstride) : (C.kernel >= 0 && C.kernel <= 3);
        if (!tree_ok(&C.tree) || C.nq < 0 || C.q_offset != rows || !kernel_ok || std::isnan(C.r) ||
            std::isinf(C.r) || (!queries && (C.nq != C.tree.n || C.q_offset != C.offset))) {
            set_error("%s: cloud %d: invalid (rows must be consecutive; cloud queries need nq == n and "
                      "q_offset == offset)", who, c);
            return -1;
        }
        if (!knn && C.stage != 0 && C.stage != 64 && C.stage != 128 && C.stage != 256) {
            set_error("%s: cloud %d: stage %u is not 0, 64, 128 or 256", who, c, C.stage);
            return -1;
        }
        tab[c] = cloud_entry(C.tree, C.q_offset, C.nq, g, C.kernel, C.r, C.k);
        if (!knn) {
            tab[c].stage = C.stage ? static_cast<int32_t>(C.stage) : kStage;
            tab[c].rec = ((flags & SFC_RECORD_HITS) || C.record) ? 1 : 0;
            tab[c].rg0 = rg;
            if (tab[c].rec) rg += (C.nq + kWave - 1) / kWave;
        }
        rows += C.nq;
        g += (C.nq + kWave - 1) / kWave;
    }
    if (rec_groups) *rec_groups = rg;
    if (rows != nq_total) {
        set_error("%s: nq_total %lld differs from the sum of the clouds' nq (%lld)", who, (long long)nq_total,
                  (long long)rows);
        return -1;
    }
    return g;
}

// table entries per upload launch (kernel arguments stay under 4 KiB)
constexpr int kTabChunk = 32;
struct TabChunk {
    SearchCloud c[kTabChunk];
};

}  // namespace

__global__ void k_write_search_table(TabChunk chunk, int first, int count, SearchCloud *tab) {
    const int i = threadIdx.x;
    if (i < count) tab[first + i] = chunk.c[i];
}

namespace {

int upload_table(const std::vector<SearchCloud> &tab, SearchCloud *dev, hipStream_t s) {
    const int B = static_cast<int>(tab.size());
    for (int first = 0; first < B; first += kTabChunk) {
        TabChunk ch;
        const int cnt = std::min(kTabChunk, B - first);
        for (int i = 0; i < cnt; ++i) ch.c[i] = tab[first + i];
        k_write_search_table<<<1, 64, 0, s>>>(ch, first, cnt, dev);
        SFC_LAUNCH_CHECK("k_write_search_table");
    }
    return SFC_OK;
}

// workspace: [table][scan scratch]
// Workspace: [table][scan scratch][query order: keys, perm, their copies,
// sort scratch, cloud starts].
struct SearchWs {
    SearchCloud *tab = nullptr;
    void *scan = nullptr;
    uint64_t *keys = nullptr, *keys_alt = nullptr;
    uint32_t *perm = nullptr, *perm_alt = nullptr;
    void *radix = nullptr;
    int64_t *starts = nullptr;
    uint32_t *spread = nullptr;
    uint32_t *nspread = nullptr;
    uint32_t *rec_idx = nullptr;
    uint64_t *rec_mask = nullptr;
    uint32_t *rec_n = nullptr;
    uint64_t *rec_tag = nullptr;
};

bool wants_order(const float *queries, int64_t nq_total, uint32_t flags) {
    return queries && !(flags & SFC_QUERIES_ORDERED) && nq_total > kWave;
}

// rec_groups: record regions (groups of the recording clouds); 0: no records
size_t carve_search_ws(int B, int64_t nq_total, bool scan, bool order, void *mem, SearchWs *w,
                       int64_t rec_groups = 0) {
    Carver c(mem);
    SearchWs x;
    if (B > 1) x.tab = c.take<SearchCloud>(B);
    if (scan) x.scan = c.take<char>(scan_ws_bytes(nq_total));
    // groups: at most one per 64 rows of each cloud, so <= nq / 64 + B
    x.spread = c.take<uint32_t>(nq_total / kWave + B + 1);
    x.nspread = c.take<uint32_t>(1);
    if (order) {
        x.keys = c.take<uint64_t>(nq_total);
        x.keys_alt = c.take<uint64_t>(nq_total);
        x.perm = c.take<uint32_t>(nq_total);
        x.perm_alt = c.take<uint32_t>(nq_total);
        x.radix = c.take<char>(radix_ws_bytes(nq_total));
        x.starts = c.take<int64_t>(B + 1);
    }
    if (rec_groups > 0) {
        const int64_t groups = nq_total / kWave + B + 1;
        x.rec_idx = c.take<uint32_t>(rec_groups * kRecCap);
        x.rec_mask = c.take<uint64_t>(rec_groups * kRecCap);
        x.rec_n = c.take<uint32_t>(groups);
        x.rec_tag = c.take<uint64_t>(2);
    }
    c.take<char>(256);
    if (w) *w = x;
    return c.bytes();
}

size_t search_ws_bytes(int B, int64_t nq_total, bool scan, bool order = false, int64_t rec_groups = 0) {
    return carve_search_ws(B, nq_total, scan, order, nullptr, nullptr, rec_groups);
}

// record regions a launch needs: the groups of its recording clouds
int64_t record_groups(const std::vector<SearchCloud> &tab) {
    int64_t rg = 0;
    for (const SearchCloud &c : tab)
        if (c.rec) rg += (c.nq + kWave - 1) / kWave;
    return rg;
}

// dynamic LDS of the count and search-fill kernels: the layout of the
// largest staging tile among the launch's clouds
// dynamic LDS of the count and search-fill kernels of one staging tile
size_t radius_lds_bytes(int tile, bool fill) {
    if (tile == 256) return fill ? sizeof(FillLdsT<256>) : sizeof(RadLdsT<256>);
    if (tile == 64) return fill ? sizeof(FillLdsT<64>) : sizeof(RadLdsT<64>);
    return fill ? sizeof(FillLdsT<128>) : sizeof(RadLdsT<128>);
}

// the staging tiles the clouds use (the host's reading of each cloud's tile
// is the device's tile_of)
std::vector<int> radius_tiles(const std::vector<SearchCloud> &tab) {
    bool has[3] = {false, false, false};
    for (const SearchCloud &c : tab) has[c.stage == 64 ? 0 : c.stage == 256 ? 2 : 1] = true;
    std::vector<int> out;
    if (has[1]) out.push_back(128);
    if (has[0]) out.push_back(64);
    if (has[2]) out.push_back(256);
    return out;
}

// Sorts the external queries of every cloud by their code (stable, so equal
// codes keep the caller's order) and points a.qperm at the result.
int order_queries(SearchArgs &a, const SearchWs &w, hipStream_t s) {
    const unsigned grid = static_cast<unsigned>(xcd_grid(a.groups));
    k_query_keys<<<grid, 64, 0, s>>>(a, w.keys, w.perm);
    SFC_LAUNCH_CHECK("k_query_keys");
    if (a.B > 1) {
        k_entry_starts<<<1, 256, 0, s>>>(a, w.starts);
        SFC_LAUNCH_CHECK("k_entry_starts");
    }
    bool in_alt = false;
    const int rc = radix_sort_pairs(w.keys, w.perm, w.keys_alt, w.perm_alt, a.nq_total, nullptr, kQueryKeyBits,
                                    w.radix, s, &in_alt, a.B > 1 ? w.starts : nullptr, a.B);
    if (rc) return rc;
    a.qperm = in_alt ? w.perm_alt : w.perm;
    return SFC_OK;
}

// Provenance of recorded hits.  Every count call on a workspace gets a new
// number (0 when it records nothing); a recording count stamps the number
// and a hash of its arguments into the workspace, and a fill that reuses the
// counts (SFC_REUSE_COUNTS) expects the pair of the last count call on the
// same workspace address with its own arguments.  A fill after a count that
// did not record, on another workspace or with other arguments finds a
// different pair and searches instead of reading the records.
std::mutex g_tag_mu;
std::unordered_map<uintptr_t, uint64_t> g_tag_last;  // workspace address -> number of its last count call
uint64_t g_tag_next = 1;

uint64_t fnv1a(uint64_t h, const void *p, size_t n) {
    const unsigned char *b = static_cast<const unsigned char *>(p);
    for (size_t i = 0; i < n; ++i) {
        h ^= b[i];
        h *= 0x100000001b3ull;
    }
    return h;
}

void record_provenance(SearchArgs &a, const std::vector<SearchCloud> &tab, void *ws, uint64_t *tag, bool record) {
    uint64_t h = 0xcbf29ce484222325ull;
    for (const SearchCloud &c : tab) h = fnv1a(h, &c, kCloudHashBytes);
    const uintptr_t ptrs[4] = {reinterpret_cast<uintptr_t>(a.queries), reinterpret_cast<uintptr_t>(a.counts),
                               reinterpret_cast<uintptr_t>(a.offsets), static_cast<uintptr_t>(a.nq_total)};
    h = fnv1a(h, ptrs, sizeof ptrs);
    const uint32_t nf = a.flags & SFC_NO_PRUNE;
    h = fnv1a(h, &nf, sizeof nf);
    std::lock_guard<std::mutex> lock(g_tag_mu);
    uint64_t &last = g_tag_last[reinterpret_cast<uintptr_t>(ws)];
    if (!(a.flags & SFC_REUSE_COUNTS)) last = record ? g_tag_next++ : 0;
    a.tag0 = last;
    a.tag1 = h;
    if (!record || last == 0) {
        a.rec_tag = nullptr;  // no records to read: every group is searched
        a.rec_n = nullptr;
    } else {
        a.rec_tag = tag;
    }
}

int radius_launch(SearchArgs &a, const std::vector<SearchCloud> &tab, int64_t groups, uint32_t *counts,
                  void *ws, hipStream_t s) {
    const int B = static_cast<int>(tab.size());
    const bool order = wants_order(a.queries, a.nq_total, a.flags);
    const int64_t rec_groups = record_groups(tab);
    const bool record = rec_groups > 0;
    SearchWs w;
    carve_search_ws(B, a.nq_total, true, order, ws, &w, rec_groups);
    if (record) {
        a.rec_idx = w.rec_idx;
        a.rec_mask = w.rec_mask;
        a.rec_n = w.rec_n;
    }
    record_provenance(a, tab, ws, w.rec_tag, record);
    SearchCloud *dtab = w.tab;
    void *scan_ws = w.scan;
    a.one = tab[0];
    a.tab = dtab;
    a.B = B;
    a.groups = groups;
    if (dtab) {
        const int rc = upload_table(tab, dtab, s);
        if (rc) return rc;
    }
    if (order && groups > 0) {
        const int rc = order_queries(a, w, s);
        if (rc) return rc;
    }
    const unsigned grid = static_cast<unsigned>(xcd_grid(groups > 0 ? groups : 1));
    // spread groups: up to 64 waves each, grid-stride over the deferred list
    const unsigned sgrid = static_cast<unsigned>(xcd_grid(std::min<int64_t>(groups * kWave, 1 << 16)));
    a.spread = w.spread;
    a.nspread = w.nspread;
    if (!(a.flags & SFC_REUSE_COUNTS)) {
        if (groups > 0) {
            if (a.queries) {
                k_reset_spread<<<1, 64, 0, s>>>(a.nspread);
                SFC_LAUNCH_CHECK("k_reset_spread");
            }
            for (const int tile : radius_tiles(tab)) {
                const size_t lds = radius_lds_bytes(tile, false);
                if (record) {
                    if (tile == 64)
                        k_radius_count_rec_t64<<<grid, 64, lds, s>>>(a);
                    else if (tile == 256)
                        k_radius_count_rec_t256<<<grid, 64, lds, s>>>(a);
                    else
                        k_radius_count_rec<<<grid, 64, lds, s>>>(a);
                    SFC_LAUNCH_CHECK("k_radius_count_rec");
                } else {
                    if (tile == 64)
                        k_radius_count_t64<<<grid, 64, lds, s>>>(a);
                    else if (tile == 256)
                        k_radius_count_t256<<<grid, 64, lds, s>>>(a);
                    else
                        k_radius_count<<<grid, 64, lds, s>>>(a);
                    SFC_LAUNCH_CHECK("k_radius_count");
                }
            }
            if (a.queries) {  // only external queries are ever deferred
                k_radius_count_spread<<<sgrid, 64, 0, s>>>(a);
                SFC_LAUNCH_CHECK("k_radius_count_spread");
            }
        }
        const int rc = scan_u32_to_u64(counts, a.nq_total, const_cast<uint64_t *>(a.offsets), true, scan_ws, s);
        if (rc) return rc;
    }
    if (a.indices && groups > 0) {
        if (a.queries) {
            k_reset_spread<<<1, 64, 0, s>>>(a.nspread);
            SFC_LAUNCH_CHECK("k_reset_spread");
        }
        if (record) {
            k_radius_fill_rec<<<grid, 64, sizeof(RecLds), s>>>(a);
            SFC_LAUNCH_CHECK("k_radius_fill_rec");
            k_radius_fill_rows<<<grid, 64, 0, s>>>(a);
            SFC_LAUNCH_CHECK("k_radius_fill_rows");
        }
        // every group recorded: the search fill only looks for overflowed ones
        a.fill_scan = record && rec_groups == groups ? 1u : 0u;
        const unsigned fgrid =
            a.fill_scan ? static_cast<unsigned>(xcd_grid((groups + kFillScan - 1) / kFillScan)) : grid;
        for (const int tile : radius_tiles(tab)) {
            const size_t lds = radius_lds_bytes(tile, true);
            if (tile == 64)
                k_radius_fill_t64<<<fgrid, 64, lds, s>>>(a);
            else if (tile == 256)
                k_radius_fill_t256<<<fgrid, 64, lds, s>>>(a);
            else
                k_radius_fill<<<fgrid, 64, lds, s>>>(a);
            SFC_LAUNCH_CHECK("k_radius_fill");
        }
        if (a.queries) {
            k_radius_fill_spread<<<sgrid, 64, 0, s>>>(a);
            SFC_LAUNCH_CHECK("k_radius_fill_spread");
        }
    }
    return SFC_OK;
}

int knn_launch(SearchArgs &a, const std::vector<SearchCloud> &tab, int64_t groups, int kmax, void *ws,
               hipStream_t s) {
    const int B = static_cast<int>(tab.size());
    const bool order = wants_order(a.queries, a.nq_total, 0);
    SearchWs w;
    carve_search_ws(B, a.nq_total, false, order, ws, &w);
    SearchCloud *dtab = w.tab;
    a.one = tab[0];
    a.tab = dtab;
    a.B = B;
    a.groups = groups;
    if (groups == 0) return SFC_OK;
    if (dtab) {
        const int rc = upload_table(tab, dtab, s);
        if (rc) return rc;
    }
    if (order) {
        const int rc = order_queries(a, w, s);
        if (rc) return rc;
    }
    const unsigned grid = static_cast<unsigned>(xcd_grid(groups));
    const unsigned qgrid = static_cast<unsigned>(xcd_grid(std::min<int64_t>(groups * kWave, 1 << 16)));
    if (kmax > kKnnRegK) {
        k_knn_large<<<qgrid, 64, 0, s>>>(a);
        SFC_LAUNCH_CHECK("k_knn_large");
        return SFC_OK;
    }
    a.spread = w.spread;
    a.nspread = w.nspread;
    k_reset_spread<<<1, 64, 0, s>>>(a.nspread);
    SFC_LAUNCH_CHECK("k_reset_spread");
    if (kmax <= 8)
        k_knn<8><<<grid, 64, 0, s>>>(a);
    else if (kmax <= 16)
        k_knn<16><<<grid, 64, 0, s>>>(a);
    else if (kmax <= 32)
        k_knn<32><<<grid, 64, 0, s>>>(a);
    else if (kmax <= 48)
        k_knn<48><<<grid, 64, 0, s>>>(a);
    else
        k_knn<64><<<grid, 64, 0, s>>>(a);
    SFC_LAUNCH_CHECK("k_knn");
    if (a.queries) {  // only external queries are ever deferred
        k_knn_spread<<<qgrid, 64, 0, s>>>(a);
        SFC_LAUNCH_CHECK("k_knn_spread");
    }
    return SFC_OK;
}

SearchArgs blank_args() {
    SearchArgs a;
    memset(&a, 0, sizeof a);
    return a;
}

}  // namespace

extern "C" int radius_search(const sfc_octree *tree, const float *queries, int64_t nq, int kernel, float r,
                             uint32_t *counts, uint64_t *offsets, uint32_t *indices, uint64_t capacity,
                             uint32_t flags, void *ws, size_t *ws_bytes, void *stream) {
    if (!ws_bytes || !tree_ok(tree) || kernel < 0 || kernel > 3 || nq < 0 || !offsets || !counts ||
        (!queries && nq != tree->n) || std::isnan(r) || std::isinf(r)) {
        set_error("radius_search: invalid argument");
        return SFC_EINVAL;
    }
    if ((flags & SFC_STAGE_MASK) == SFC_STAGE_MASK) {
        set_error("radius_search: flags select no staging tile");
        return SFC_EINVAL;
    }
    const size_t need = search_ws_bytes(1, nq, true, wants_order(queries, nq, flags),
                                        (flags & SFC_RECORD_HITS) ? (nq + kWave - 1) / kWave : 0);
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
    std::vector<SearchCloud> tab(1, cloud_entry(*tree, 0, nq, 0, kernel, r, 0));
    tab[0].stage = (flags & SFC_STAGE_64) ? 64 : ((flags & SFC_STAGE_256) ? 256 : kStage);
    tab[0].rec = (flags & SFC_RECORD_HITS) ? 1 : 0;
    SearchArgs a = blank_args();
    a.queries = queries;
    a.flags = flags;
    a.counts = counts;
    a.offsets = offsets;
    a.indices = indices;
    a.capacity = capacity;
    a.nq_total = nq;
    return radius_launch(a, tab, (nq + kWave - 1) / kWave, counts, ws, s);
}

extern "C" int radius_search_struct(const sfc_octree *tree, const float *queries, int64_t nq, int kernel, float r,
                                    uint32_t *rcounts, uint64_t *roffsets, uint32_t *ranges, uint64_t rcapacity,
                                    uint32_t *pcounts, uint64_t *poffsets, uint32_t *points, uint64_t pcapacity,
                                    uint32_t flags, void *ws, size_t *ws_bytes, void *stream) {
    if (!ws_bytes || !tree_ok(tree) || kernel < 0 || kernel > 3 || nq < 0 || !rcounts || !roffsets || !pcounts ||
        !poffsets || (!queries && nq != tree->n) || std::isnan(r) || std::isinf(r) ||
        (ranges == nullptr) != (points == nullptr)) {
        set_error("radius_search_struct: invalid argument");
        return SFC_EINVAL;
    }
    const bool order = wants_order(queries, nq, flags);
    // two scans: the second scratch follows the search workspace
    const size_t need = search_ws_bytes(1, nq, true, order) + align_up(scan_ws_bytes(nq), 256);
    if (!ws) {
        *ws_bytes = need;
        return SFC_OK;
    }
    if (*ws_bytes < need || (reinterpret_cast<uintptr_t>(ws) & 255u)) {
        set_error("radius_search_struct: workspace needs %zu bytes, 256-aligned", need);
        return SFC_EWORKSPACE;
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (nq == 0 || !(r > 0.0f)) {
        if (!(flags & SFC_REUSE_COUNTS)) {
            k_zero_rows<<<grid_for(nq + 1, 256, 4096), 256, 0, s>>>(rcounts, roffsets, nq);
            SFC_LAUNCH_CHECK("k_zero_rows");
            k_zero_rows<<<grid_for(nq + 1, 256, 4096), 256, 0, s>>>(pcounts, poffsets, nq);
            SFC_LAUNCH_CHECK("k_zero_rows");
        }
        return SFC_OK;
    }
    std::vector<SearchCloud> tab(1, cloud_entry(*tree, 0, nq, 0, kernel, r, 0));
    SearchArgs a = blank_args();
    a.queries = queries;
    a.flags = flags;
    a.counts = pcounts;
    a.offsets = poffsets;
    a.indices = points;
    a.capacity = pcapacity;
    a.rcounts = rcounts;
    a.roffsets = roffsets;
    a.ranges = ranges;
    a.rcapacity = rcapacity;
    a.nq_total = nq;
    SearchWs w;
    carve_search_ws(1, nq, true, order, ws, &w);
    void *scan2 = static_cast<char *>(ws) + search_ws_bytes(1, nq, true, order);
    a.one = tab[0];
    a.tab = nullptr;
    a.B = 1;
    a.groups = (nq + kWave - 1) / kWave;
    if (order) {
        const int rc = order_queries(a, w, s);
        if (rc) return rc;
    }
    const unsigned grid = static_cast<unsigned>(xcd_grid(a.groups));
    if (!(flags & SFC_REUSE_COUNTS)) {
        k_struct_count<<<grid, 64, 0, s>>>(a);
        SFC_LAUNCH_CHECK("k_struct_count");
        int rc = scan_u32_to_u64(rcounts, nq, roffsets, true, w.scan, s);
        if (rc) return rc;
        rc = scan_u32_to_u64(pcounts, nq, poffsets, true, scan2, s);
        if (rc) return rc;
    }
    if (ranges) {
        k_struct_fill<<<grid, 64, 0, s>>>(a);
        SFC_LAUNCH_CHECK("k_struct_fill");
    }
    return SFC_OK;
}

extern "C" int radius_search_batched(int B, const sfc_cloud *clouds, const float *queries, int64_t nq_total,
                                     uint32_t *counts, uint64_t *offsets, uint32_t *indices, uint64_t capacity,
                                     uint32_t flags, void *ws, size_t *ws_bytes, void *stream) {
    if (!ws_bytes || !offsets || !counts) {
        set_error("radius_search_batched: invalid argument");
        return SFC_EINVAL;
    }
    std::vector<SearchCloud> tab;
    int64_t rec_groups = 0;
    const int64_t groups =
        search_table("radius_search_batched", B, clouds, queries, nq_total, false, 0, tab, flags, &rec_groups);
    if (groups < 0) return SFC_EINVAL;
    const size_t need = search_ws_bytes(B, nq_total, true, wants_order(queries, nq_total, flags), rec_groups);
    if (!ws) {
        *ws_bytes = need;
        return SFC_OK;
    }
    if (*ws_bytes < need || (reinterpret_cast<uintptr_t>(ws) & 255u)) {
        set_error("radius_search_batched: workspace needs %zu bytes, 256-aligned", need);
        return SFC_EWORKSPACE;
    }
    SearchArgs a = blank_args();
    a.queries = queries;
    a.flags = flags;
    a.counts = counts;
    a.offsets = offsets;
    a.indices = indices;
    a.capacity = capacity;
    a.nq_total = nq_total;
    return radius_launch(a, tab, groups, counts, ws, static_cast<hipStream_t>(stream));
}

extern "C" int knn_search(const sfc_octree *tree, const float *queries, int64_t nq, int k, uint32_t *idx, float *d2,
                          void *ws, size_t *ws_bytes, void *stream) {
    if (!ws_bytes || !tree_ok(tree) || nq < 0 || k < 1 || (!queries && nq != tree->n) || (nq > 0 && (!idx || !d2))) {
        set_error("knn_search: invalid argument");
        return SFC_EINVAL;
    }
    if (k > kKnnMaxK) {
        set_error("knn_search: k = %d above %d is not supported", k, kKnnMaxK);
        return SFC_ENOTSUP;
    }
    const size_t need = search_ws_bytes(1, nq, false, wants_order(queries, nq, 0));
    if (!ws) {
        *ws_bytes = need;
        return SFC_OK;
    }
    if (*ws_bytes < need || (reinterpret_cast<uintptr_t>(ws) & 255u)) {
        set_error("knn_search: workspace needs %zu bytes, 256-aligned", need);
        return SFC_EWORKSPACE;
    }
    std::vector<SearchCloud> tab(1, cloud_entry(*tree, 0, nq, 0, SFC_SPHERE, 0.0f, k));
    SearchArgs a = blank_args();
    a.queries = queries;
    a.nq_total = nq;
    a.kstride = k;
    a.idx = idx;
    a.d2 = d2;
    return knn_launch(a, tab, (nq + kWave - 1) / kWave, k, ws, static_cast<hipStream_t>(stream));
}

extern "C" int knn_search_batched(int B, const sfc_cloud *clouds, const float *queries, int64_t nq_total, int kstride,
                                  uint32_t *idx, float *d2, void *ws, size_t *ws_bytes, void *stream) {
    if (!ws_bytes || kstride < 1 || (nq_total > 0 && (!idx || !d2))) {
        set_error("knn_search_batched: invalid argument");
        return SFC_EINVAL;
    }
    if (kstride > kKnnMaxK) {
        set_error("knn_search_batched: kstride = %d above %d is not supported", kstride, kKnnMaxK);
        return SFC_ENOTSUP;
    }
    std::vector<SearchCloud> tab;
    const int64_t groups = search_table("knn_search_batched", B, clouds, queries, nq_total, true, kstride, tab);
    if (groups < 0) return SFC_EINVAL;
    const size_t need = search_ws_bytes(B, nq_total, false, wants_order(queries, nq_total, 0));
    if (!ws) {
        *ws_bytes = need;
        return SFC_OK;
    }
    if (*ws_bytes < need || (reinterpret_cast<uintptr_t>(ws) & 255u)) {
        set_error("knn_search_batched: workspace needs %zu bytes, 256-aligned", need);
        return SFC_EWORKSPACE;
    }
    int kmax = 1;
    for (int c = 0; c < B; ++c) kmax = std::max(kmax, clouds[c].k);
    SearchArgs a = blank_args();
    a.queries = queries;
    a.nq_total = nq_total;
    a.kstride = kstride;
    a.idx = idx;
    a.d2 = d2;
    return knn_launch(a, tab, groups, kmax, ws, static_cast<hipStream_t>(stream));
}

extern "C" int radius_search_check(const uint64_t *offsets, int64_t nq, uint64_t capacity, uint64_t *total,
                                   void *stream) {
    if (!offsets || nq < 0 || !total) {
        set_error("radius_search_check: invalid argument");
        return SFC_EINVAL;
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    uint64_t t = 0;
    SFC_HIP_TRY(hipMemcpyAsync(&t, offsets + nq, sizeof t, hipMemcpyDeviceToHost, s));
    SFC_HIP_TRY(hipStreamSynchronize(s));
    *total = t;
    if (t > capacity) {
        set_error("radius_search_check: %llu neighbour indices exceed the capacity %llu; no index was written",
                  static_cast<unsigned long long>(t), static_cast<unsigned long long>(capacity));
        return SFC_ECAPACITY;
    }
    return SFC_OK;
}


// ---------------------------------------------------------------------------
// radius_search without a caller workspace: the workspace is a fixed device
// array of this library (one per GPU, held until the process ends), for
// callers that cannot allocate device memory.  Host code never passes the
// array's name to a kernel (in host code it is a stand-in, not a device
// address): the device address is looked up once per device and kept.
namespace {

constexpr size_t kScratchBytes = SFC_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kScratchDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch[kScratchDevices] = {};

// device address of the current device's scratch array (looked up on the
// first call on that device, with the device current)
int scratch_ptr(void **out) {
    int dev = -1;
    SFC_HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kScratchDevices) {
        set_error("radius_search_noalloc: device %d beyond the %d supported", dev, kScratchDevices);
        return SFC_ENOTSUP;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            set_error("radius_search_noalloc: hipGetSymbolAddress: %s", hipGetErrorString(e));
            return SFC_EHIP;
        }
        g_scratch[dev] = p;
    }
    *out = g_scratch[dev];
    return SFC_OK;
}

}  // namespace

extern "C" int radius_search_noalloc(const sfc_octree *tree, const float *queries, int64_t nq, int kernel, float r,
                                     uint32_t *counts, uint64_t *offsets, uint32_t *indices, uint64_t capacity,
                                     uint32_t flags, void *stream) {
    size_t need = 0;
    int rc = radius_search(tree, queries, nq, kernel, r, counts, offsets, indices, capacity, flags, nullptr, &need,
                           stream);
    if (rc) return rc;
    if (need > kScratchBytes) {
        set_error("radius_search_noalloc: the call needs %zu bytes of workspace, beyond the fixed %zu "
                  "(fewer external queries per call, or radius_search with a workspace)",
                  need, kScratchBytes);
        return SFC_EWORKSPACE;
    }
    void *ws = nullptr;
    rc = scratch_ptr(&ws);
    if (rc) return rc;
    size_t have = kScratchBytes;
    return radius_search(tree, queries, nq, kernel, r, counts, offsets, indices, capacity, flags, ws, &have, stream);
}

#ifdef SFC_SWEEP_STATS
// Copies the count kernels' sweep statistics (see g_sweep_stats) to out[16]
// and, with reset != 0, clears them; synchronizes the device.
extern "C" int sfc_sweep_stats(unsigned long long *out, int reset) {
    if (!out) {
        set_error("sfc_sweep_stats: null output");
        return SFC_EINVAL;
    }
    void *p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(sfc::g_sweep_stats));
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e == hipSuccess) e = hipMemcpy(out, p, sizeof(unsigned long long) * 16, hipMemcpyDeviceToHost);
    if (e == hipSuccess && reset) e = hipMemset(p, 0, sizeof(unsigned long long) * 16);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        set_error("sfc_sweep_stats: %s", hipGetErrorString(e));
        return SFC_EHIP;
    }
    return SFC_OK;
}
#endif

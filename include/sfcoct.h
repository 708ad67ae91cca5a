/*
 * sfcoct.h -- C ABI of the MI355X (gfx950) library for space-filling-curve
 * reordering, linear octrees and neighbourhood search in 3D point clouds,
 * after arXiv 2603.06771 ("Efficient Neighbourhood Search in 3D Point Clouds
 * Through Space-Filling Curves and Linear Octrees").
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - All array arguments are DEVICE pointers into caller-owned memory unless
 *   stated otherwise.  The library never allocates or frees device memory.
 * - Every call is asynchronous on `stream` (a hipStream_t passed as void*;
 *   NULL is the default stream) and performs no host synchronisation.
 * - Workspace protocol: a call that takes (ws, ws_bytes) with ws == NULL only
 *   stores the workspace size it needs in *ws_bytes (a host pointer) and runs
 *   nothing.  A call with ws != NULL and *ws_bytes below that size returns
 *   SFC_EWORKSPACE and runs nothing.  Workspace must be 256-byte aligned.
 *   Its contents are scratch and need no initialisation.
 * - Return codes are sfc_status values.  SFC_EINVAL and SFC_EWORKSPACE are
 *   returned before anything is enqueued, so no output is touched.
 *   SFC_EHIP reports a failed launch; sfc_last_error() gives the message.
 * - Coordinates are IEEE binary32 and must be finite.  Indices are uint32,
 *   so a cloud holds at most 2^32 - 1 points.
 * - Arithmetic contract: every fp32 expression is evaluated as written, with
 *   round-to-nearest-even, no fused multiply-add and denormals kept, so the
 *   results are bit-for-bit those of the definitions below.
 * - Calls on one stream are ordered; calls that share output buffers on
 *   different streams race and are the caller's responsibility.
 */
#ifndef SFCOCT_H
#define SFCOCT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SFC_OK = 0,
    SFC_EINVAL = -1,      /* bad argument (null pointer, size, enum) */
    SFC_EWORKSPACE = -2,  /* workspace too small or misaligned */
    SFC_ECAPACITY = -3,   /* radius_search_check: the neighbour total exceeds the capacity */
    SFC_EHIP = -4,        /* a HIP runtime call or kernel launch failed */
    SFC_ENOTSUP = -5      /* valid but unsupported request (e.g. k > 512) */
} sfc_status;

/* Space-filling curves of Section 4 (4.1 Morton, 4.2 Hilbert). */
typedef enum { SFC_MORTON = 0, SFC_HILBERT = 1 } sfc_curve;

/* Search kernels of Section 3.2 (Definition of a search kernel). */
typedef enum { SFC_SPHERE = 0, SFC_CIRCLE = 1, SFC_CUBE = 2, SFC_SQUARE = 3 } sfc_kernel;

/* Discretisation frame of Section 4, steps 1-2: cell_a = floor((x_a - lo_a) *
 * scale), clamped to [0, 2^bits - 1]; scale = 2^bits / E with E the largest
 * side of the cloud's bounding box (E = 1 for a degenerate or empty cloud). */
typedef struct sfc_frame {
    float lo[3];
    float scale;
    int32_t bits;   /* L, levels per axis, 1..21 */
    int32_t curve;  /* sfc_curve */
} sfc_frame;

/* Octree node record: the node's point range [begin, end) in sorted order
 * (the paper's internalRanges, Section 5.1) and the tight bounding box of its
 * points (lo = +inf, hi = -inf when the node is empty). 32 bytes. */
typedef struct sfc_node {
    float lo[3];
    uint32_t begin;
    float hi[3];
    uint32_t end;
} sfc_node;

/* Device-resident counts written by build_linear_octree. */
typedef struct sfc_tree_info {
    int64_t n_points;
    int64_t n_internal;
    int64_t n_leaves;   /* = 7 * n_internal + 1 (complete octree) */
    int64_t n_nodes;    /* = n_internal + n_leaves */
    int32_t depth;      /* deepest level holding a node */
    int32_t status;     /* 0 = ok */
    int64_t level_nodes_off[23]; /* first node index of each level (BFS order) */
} sfc_tree_info;

/* Non-owning view of a built octree; every pointer is a device address inside
 * the caller's tree memory.  Filled in by build_linear_octree (host struct).
 * Nodes are stored level by level (breadth first), ordered by code inside a
 * level; the 8 children of an internal node are consecutive. */
typedef struct sfc_octree {
    int64_t n;            /* points */
    int64_t max_nodes;    /* capacity of the node arrays */
    int64_t max_leaves;   /* capacity of leaves / counts */
    int32_t bits;
    int32_t curve;
    uint32_t leaf_size;   /* N_max of Section 5.1 */
    uint32_t reserved;
    sfc_frame *frame;     /* [1] frame used for the codes */
    float *points;        /* [4n] sorted cloud {x, y, z, bits(original index)} */
    uint64_t *keys;       /* [n] sorted codes */
    uint32_t *perm;       /* [n] original index of the i-th sorted point */
    uint64_t *leaves;     /* [n_leaves + 1] the paper's leaves array (codes) */
    uint32_t *counts;     /* [n_leaves] points per leaf */
    sfc_node *nodes;      /* [n_nodes] ranges and boxes, breadth-first */
    int32_t *child;       /* [n_nodes] index of the first child, -1 for a leaf */
    uint64_t *node_key;   /* [n_nodes] first code of the node */
    uint8_t *node_level;  /* [n_nodes] level (0 = root) */
    sfc_tree_info *info;  /* [1] actual counts */
} sfc_octree;

/* Section 4 (steps 1-2, 4.1, 4.2), reorder step 1: codes of every point.
 *   xyz    [3n] fp32, x y z interleaved, original order (device)
 *   curve  sfc_curve; bits = L in 1..21 (the paper uses 21, a 63-bit code)
 *   frame  [1] device output: the frame of the cloud
 *   keys   [n] device output: key[i] = C(cell(xyz[i])) < 8^bits
 * n == 0 is valid (frame lo = 0, scale = 2^bits). */
int encode_sfc(const float *xyz, int64_t n, int curve, int bits, sfc_frame *frame, uint64_t *keys,
               void *ws, size_t *ws_bytes, void *stream);

/* Bytes of tree memory build_linear_octree needs for n points and the given
 * leaf threshold (an upper bound on every array; host output). */
int octree_bytes(int64_t n, uint32_t leaf_size, int bits, size_t *bytes);

/* Sections 4 and 5.1: encode, sort ascending by code (ties by original
 * index), gather the sorted cloud, and build the complete linear octree in
 * which a node is split into its 8 octants iff it holds more than leaf_size
 * points and its level is below bits.  Computes leaves, counts, every node's
 * point range (internalRanges) and tight bounding box, and the child links.
 *   xyz        [3n] fp32 original cloud (device, read only)
 *   tree_mem   device memory of at least octree_bytes(n, leaf_size, bits)
 *   tree_out   host output: the view of the tree inside tree_mem
 * leaf_size >= 1.  Node counts are written to tree_out->info on the device. */
int build_linear_octree(const float *xyz, int64_t n, int curve, int bits, uint32_t leaf_size,
                        void *tree_mem, size_t tree_bytes, sfc_octree *tree_out, void *ws,
                        size_t *ws_bytes, void *stream);

/* Section 3.2 with the pruning of Section 5.1 (neighboursPrune): for every
 * query c and the chosen kernel, the set {j : pred(p_j, c, r)} of ORIGINAL
 * point indices, as CSR.  Predicates, with dx = p - c per axis in fp32:
 *   SPHERE (dx*dx + dy*dy) + dz*dz < r*r     CIRCLE dx*dx + dy*dy < r*r
 *   CUBE   |dx| < r, |dy| < r, |dz| < r      SQUARE |dx| < r, |dy| < r
 * r <= 0 gives empty rows; r must not be NaN or infinite.
 *   tree      built octree (host struct, device pointers)
 *   queries   [3nq] fp32 centres (device), or NULL: every cloud point is a
 *             query and row i is the point at sorted position i (nq == n)
 *   counts    [nq] output neighbour counts
 *   offsets   [nq+1] output exclusive prefix sums of counts (row starts)
 *   indices   [capacity] output neighbour lists, or NULL for counts only.
 *             Written only if offsets[nq] <= capacity (checked on the device);
 *             otherwise nothing is written and the caller retries with
 *             capacity >= offsets[nq].  Order inside a row is unspecified but
 *             deterministic.
 *   flags     bit 0 (SFC_REUSE_COUNTS): counts/offsets already hold the
 *             result of a count call with identical arguments; skip it.
 *             bit 1 (SFC_NO_PRUNE): no containment shortcut (neighboursLin).
 *             bit 2 (SFC_QUERIES_ORDERED): external queries are already in
 *             a spatially coherent order (e.g. along the curve); skip the
 *             internal reordering.  Without it, external queries are sorted
 *             by their code in the tree's frame inside the call (workspace
 *             grows by about 24 bytes per query); rows of the output always
 *             follow the caller's query order.
 *             bit 3 (SFC_RECORD_HITS): the count pass records, for every
 *             group of 64 queries, each tested point that is a neighbour of
 *             one of them (its index and the mask of those queries), and
 *             the fill writes the rows from these records instead of
 *             searching again; a group whose records do not fit (more than
 *             4096), and a group of far-apart external queries (served one
 *             query per wave), is filled by the search.  Rows come out in
 *             the same order as without the bit.  The workspace grows by
 *             about 48 KB per 64 queries.  With SFC_REUSE_COUNTS the
 *             records of the preceding count call on the same workspace are
 *             used, so both calls pass this bit, the same workspace and
 *             identical arguments.  The count stamps the records with a
 *             number the library gives each count call on a workspace
 *             address and a hash of the call's arguments; a fill that finds
 *             another stamp (the count did not record, ran on another
 *             workspace or with other arguments, or a later count call used
 *             the workspace) searches instead, so the result is the same
 *             with or without the bit.
 *             bits 4-5 (SFC_STAGE_64, SFC_STAGE_256): the search's staging
 *             tile, the points staged in LDS per sweep round: 64 or 256
 *             instead of 128 (both bits: SFC_EINVAL).  A larger round
 *             amortises per-round work over more points, a smaller one
 *             keeps more waves resident; results are identical for every
 *             tile.
 *
 * Capacity protocol: the indices are written only when the neighbour total
 * offsets[nq] fits `capacity`, which the kernels check on the device (no
 * host round trip).  The caller learns the outcome at its own sync point
 * from offsets[nq], or with radius_search_check below.
 */
#define SFC_REUSE_COUNTS 1u
#define SFC_NO_PRUNE 2u
#define SFC_QUERIES_ORDERED 4u
#define SFC_RECORD_HITS 8u
#define SFC_STAGE_64 16u
#define SFC_STAGE_256 32u
#define SFC_STAGE_MASK 48u
int radius_search(const sfc_octree *tree, const float *queries, int64_t nq, int kernel, float r,
                  uint32_t *counts, uint64_t *offsets, uint32_t *indices, uint64_t capacity,
                  uint32_t flags, void *ws, size_t *ws_bytes, void *stream);

/* The sync point of the capacity protocol (Section 5.1 output of
 * neighboursPrune as CSR): waits for `stream`, stores the neighbour total
 * offsets[nq] (offsets: the device array a radius_search or
 * radius_search_batched call on that stream wrote) in *total (a host
 * pointer) and returns SFC_ECAPACITY if it exceeds `capacity` (the indices
 * were then not written: call again with a buffer of at least *total
 * entries and SFC_REUSE_COUNTS), SFC_OK otherwise.  This call blocks the
 * host; it allocates nothing.  SFC_EHIP if the copy or the wait fails. */
int radius_search_check(const uint64_t *offsets, int64_t nq, uint64_t capacity, uint64_t *total, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc):
 * radius_search with the same arguments, results and capacity protocol,
 * but no workspace argument.  Its workspace is a fixed array of
 * SFC_NOALLOC_SCRATCH_BYTES bytes inside this library, one per GPU, taken
 * when the library is loaded and held until the process ends; the call
 * allocates nothing.  A call whose workspace (the size radius_search would
 * ask for) exceeds it returns SFC_EWORKSPACE and does nothing: 64 MiB covers
 * up to about a billion queries around a cloud's own points (queries ==
 * NULL) or already ordered (SFC_QUERIES_ORDERED), and about 2.6 million
 * external queries that the call sorts; SFC_RECORD_HITS takes about 48 KB
 * per 64 queries of it.  All calls on one GPU share the array, which
 * keeps the last call's contents: calls that overlap on one GPU (two
 * streams, two host threads) race and give undefined results; calls in
 * one stream are ordered and safe.  Arguments, layouts, ownership and the
 * other errors are those of radius_search. */
#define SFC_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int radius_search_noalloc(const sfc_octree *tree, const float *queries, int64_t nq, int kernel, float r,
                          uint32_t *counts, uint64_t *offsets, uint32_t *indices, uint64_t capacity,
                          uint32_t flags, void *stream);

/* Section 5.1, the neighboursStruct form of radius_search: the same
 * neighbour set per query, split into the ranges of sorted positions of the
 * octree nodes that lie entirely inside the neighbourhood and the individual
 * points of the nodes it overlaps only partly (original indices).  Ranges and
 * points of a row are disjoint; the range [b, e) stands for the points at
 * sorted positions b .. e - 1 (tree->perm gives their original indices).
 *   rcounts [nq], roffsets [nq+1]: ranges per row and their row starts
 *   ranges  [2 * rcapacity]: (begin, end) pairs, or NULL for counts only
 *   pcounts [nq], poffsets [nq+1], points [pcapacity]: the individual points
 *           (points must be NULL exactly when ranges is)
 * Both buffers are written only if both totals fit (checked on the device).
 * flags: SFC_REUSE_COUNTS, SFC_NO_PRUNE (no ranges: every point listed),
 * SFC_QUERIES_ORDERED, as for radius_search.  Queries are handled 64 at a time
 * (no one-query-per-wave path), so widely scattered queries are slower than
 * with radius_search. */
int radius_search_struct(const sfc_octree *tree, const float *queries, int64_t nq, int kernel, float r,
                         uint32_t *rcounts, uint64_t *roffsets, uint32_t *ranges, uint64_t rcapacity,
                         uint32_t *pcounts, uint64_t *poffsets, uint32_t *points, uint64_t pcapacity,
                         uint32_t flags, void *ws, size_t *ws_bytes, void *stream);

/* Section 3.3: the k nearest cloud points of every query, as the k smallest
 * pairs (d2, original index) in lexicographic order, ascending, where d2 is
 * the SPHERE expression above.  Ties in d2 are broken by the smaller index; a
 * query that is a cloud point finds itself at d2 = 0.  When k > n the missing
 * entries are (0xFFFFFFFF, +inf).
 *   queries  [3nq] fp32 (device) or NULL (every point, rows in sorted order);
 *            external queries are reordered along the curve inside the call
 *            (as radius_search without SFC_QUERIES_ORDERED)
 *   idx      [nq*k] output indices;  d2 [nq*k] output squared distances
 * 1 <= k <= 512 (SFC_ENOTSUP above).  k <= 64 keeps each query's list in
 * registers (64 queries per wave); larger k takes one query per wave with a
 * candidate buffer in LDS. */
int knn_search(const sfc_octree *tree, const float *queries, int64_t nq, int k, uint32_t *idx,
               float *d2, void *ws, size_t *ws_bytes, void *stream);

/* ------------------------------------------------------------------------
 * Batches of independent clouds (no counterpart in the paper: the paper
 * handles one cloud at a time; these run the same steps for many clouds in
 * the same launches).  The input is the concatenation of the clouds' points;
 * every kernel block works inside one cloud, so uneven sizes cost no padding.
 * ---------------------------------------------------------------------- */

/* One cloud of a batch: a HOST struct.  The library copies the table of B
 * entries to the device on the caller's stream (pinned host memory makes the
 * copy capturable in a graph). */
typedef struct sfc_cloud {
    int64_t offset;      /* first point of the cloud in the concatenated input */
    int64_t n;           /* points of the cloud */
    int32_t curve;       /* sfc_curve */
    int32_t bits;        /* 1..21 */
    uint32_t leaf_size;  /* N_max, >= 1 */
    int32_t kernel;      /* radius search: sfc_kernel */
    float r;             /* radius search: radius (r <= 0: empty rows) */
    int32_t k;           /* k-NN: 1..kstride (at most 512) */
    int64_t q_offset;    /* search: first row of the cloud in the concatenated queries */
    int64_t nq;          /* search: queries of the cloud (cloud queries: nq == n) */
    uint32_t stage;      /* radius search: staging tile, points per sweep round (64, 128, 256; 0: 128) */
    uint32_t record;     /* radius search: nonzero records the cloud's hits for the fill (as
                            SFC_RECORD_HITS does for every cloud; workspace only for such clouds) */
    sfc_octree tree;     /* filled by octree_batch_layout */
} sfc_cloud;

/* Lays out the trees of a batch in one block of tree memory: shared point /
 * code / permutation arrays (cloud c at [offset_c, offset_c + n_c)), then the
 * node arrays of every cloud (sized by the per-cloud bound of octree_bytes).
 * Reads offset, n, bits, leaf_size of each cloud (offsets must be the running
 * sum of the sizes); with tree_mem == NULL only *bytes is set, otherwise the
 * `tree` views are filled with device pointers into tree_mem. */
int octree_batch_layout(int B, sfc_cloud *clouds, void *tree_mem, size_t *bytes);

/* Sections 4 and 5.1 for every cloud of the batch (encode with the cloud's
 * own frame, stable sort by (cloud, code, index), reorder, build).  xyz holds
 * the concatenated clouds; indices stored in the trees are local to each cloud.
 * The trees must have been laid out by octree_batch_layout. */
int build_linear_octree_batched(const float *xyz, int B, const sfc_cloud *clouds, void *ws, size_t *ws_bytes,
                                void *stream);

/* Memory accounting of Section 7.5 (Tables 6-7: a linear octree costs a few
 * percent of the cloud): the trees of a batch built by
 * build_linear_octree_batched, copied into a block of exactly the memory
 * their actual node and leaf counts need, instead of the upper bounds that
 * octree_batch_layout reserves so the build never waits for the host (at
 * leaf size 64 the bound is about 24 times the actual internal nodes).
 * Waits for `stream` and reads every tree's sfc_tree_info (the host blocks).
 * With dst_mem == NULL only *bytes is set.  Otherwise dst_mem (device,
 * 256-byte aligned, at least *bytes, not overlapping the source) receives
 * the shared point, code and permutation arrays and every tree's frame,
 * info and node arrays, asynchronously on `stream`, and out[0..B) the same
 * descriptors as clouds with `tree` viewing dst_mem (max_nodes / max_leaves
 * = the actual counts).  The source memory can be freed once the copies
 * are done; searches on the copies give the same results.  SFC_EINVAL if a
 * tree was not built (or not laid out by octree_batch_layout). */
int octree_batch_compact(int B, const sfc_cloud *clouds, void *dst_mem, size_t *bytes, sfc_cloud *out,
                         void *stream);

/* Radius search for every cloud of the batch with its own kernel and radius,
 * in one launch per pass.  queries: concatenated per-cloud query blocks
 * (cloud c at rows [q_offset_c, q_offset_c + nq_c)), or NULL (each cloud's own
 * points, rows in the cloud's sorted order).  counts / offsets / indices form
 * ONE CSR over all nq_total rows (offsets[nq_total] = total), indices local to
 * each cloud.  Capacity and flags as for radius_search, except the staging
 * tile, which each cloud names itself (its `stage`; the flag bits are
 * ignored), and recorded hits, which SFC_RECORD_HITS turns on for every
 * cloud and a cloud's `record` for that cloud (the workspace holds records
 * for the recording clouds' groups only).  An autotuner can so choose leaf
 * size, tile and fill per cloud; every choice gives the same rows. */
int radius_search_batched(int B, const sfc_cloud *clouds, const float *queries, int64_t nq_total, uint32_t *counts,
                          uint64_t *offsets, uint32_t *indices, uint64_t capacity, uint32_t flags, void *ws,
                          size_t *ws_bytes, void *stream);

/* k-NN for every cloud of the batch with its own k (<= kstride <= 512): row q
 * occupies idx / d2 [q * kstride, (q + 1) * kstride); entries past the
 * cloud's k are (0xFFFFFFFF, +inf). */
int knn_search_batched(int B, const sfc_cloud *clouds, const float *queries, int64_t nq_total, int kstride,
                       uint32_t *idx, float *d2, void *ws, size_t *ws_bytes, void *stream);

/* Section 5.2: the kNN locality histogram of the tree's stored order.  For
 * the query stored at position rows[r] (rows == NULL: position r) and each of
 * its neighbours idx[r * kstride + t], t < k (original indices, as
 * knn_search returns them; entries >= n are padding and skipped), let
 * d = |rows[r] - pos| with pos the neighbour's stored position (the inverse of
 * tree->perm).  hist[d] (tree->n entries, u32, overwritten) counts the pairs.
 * stats (8 doubles, device) receives: total pairs, mean d, standard deviation,
 * Fisher-Pearson skewness G1 = E[((d - mean) / sd)^3], the quartiles Q1, Q2,
 * Q3 (smallest d whose cumulative count reaches 1/4, 1/2, 3/4 of the total)
 * and the largest d.  The statistics are summed in a fixed order (the same
 * bits on every run).  nq * k must stay below 2^32 (SFC_ENOTSUP). */
int knn_locality(const sfc_octree *tree, const uint32_t *rows, int64_t nq, const uint32_t *idx, int k, int kstride,
                 uint32_t *hist, double *stats, void *ws, size_t *ws_bytes, void *stream);

/* Serving helper (not an operation of the paper): assembles a query batch
 * from point ids.  out[3i .. 3i+2] = xyz[3 rows[i] .. 3 rows[i] + 2] for
 * i < n, where xyz holds n_points points (AoS, 3 floats each); a row id
 * >= n_points yields a NaN point (a query that matches nothing).  xyz, rows
 * and out are device arrays; out must not overlap xyz.  No workspace. */
int gather_points(const float *xyz, int64_t n_points, const uint32_t *rows, int64_t n, float *out, void *stream);

/* Message of the last SFC_EINVAL / SFC_EHIP on the calling thread. */
const char *sfc_last_error(void);

/* Library version string. */
const char *sfc_version(void);

#ifdef __cplusplus
}
#endif

#endif /* SFCOCT_H */

/*
 * oracle.c -- plain CPU reference for space-filling-curve reordering, the
 * linear octree and fixed-radius / k-nearest-neighbour search.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code, header or table with the GPU
 * library: every function here is written from the paper's definitions
 * (arXiv 2603.06771, "Efficient Neighbourhood Search in 3D Point Clouds
 * Through Space-Filling Curves and Linear Octrees"), as slowly and plainly as
 * the definition reads.
 *
 * Build: gcc -O2 -std=c11 -fPIC -shared -fopenmp -ffp-contract=off
 *        -fno-fast-math  (x86-64 SSE float arithmetic is IEEE binary32,
 *        round-to-nearest-even, and with contraction off every fp32
 *        expression below is evaluated exactly as written).
 *
 * Pins (what ties each function to something other than itself) are listed in
 * the test files; functions without a pin say so in their comment.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_MORTON 0
#define OR_HILBERT 1

#define OR_SPHERE 0
#define OR_CIRCLE 1
#define OR_CUBE 2
#define OR_SQUARE 3

/* ------------------------------------------------------------------------ */
/* Threads                                                                   */
/* ------------------------------------------------------------------------ */

void or_set_threads(int t)
{
#ifdef _OPENMP
    if (t > 0) omp_set_num_threads(t);
#else
    (void)t;
#endif
}

int or_get_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------------ */
/* Section 4, steps 1-2: frame of the cloud and discretisation.              */
/*                                                                           */
/* The bounding box is the exact per-axis min/max.  Scaling is isotropic     */
/* (one factor for all three axes, so that the octants are cubes): E is the   */
/* largest fp32 side length, s = 2^L / E in fp32.  A degenerate cloud        */
/* (E == 0, or no points) uses E = 1; an empty cloud uses lo = 0.            */
/* ------------------------------------------------------------------------ */

void or_frame(const float *xyz, int64_t n, int bits, float lo[3], float *scale)
{
    float mn[3] = {INFINITY, INFINITY, INFINITY};
    float mx[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int64_t i = 0; i < n; ++i) {
        for (int a = 0; a < 3; ++a) {
            float v = xyz[3 * i + a];
            if (v < mn[a]) mn[a] = v;
            if (v > mx[a]) mx[a] = v;
        }
    }
    float E = 0.0f;
    if (n == 0) {
        mn[0] = mn[1] = mn[2] = 0.0f;
    } else {
        for (int a = 0; a < 3; ++a) {
            float side = mx[a] - mn[a];
            if (side > E) E = side;
        }
    }
    if (!(E > 0.0f)) E = 1.0f;
    float cells = (float)(1u << bits);
    *scale = cells / E;
    lo[0] = mn[0];
    lo[1] = mn[1];
    lo[2] = mn[2];
}

/* Step 2: floor of the scaled coordinate.  A coordinate equal to the upper
 * corner maps to 2^L exactly and is clamped to the last cell (the box B is
 * half-open); a coordinate below the lower corner (a query outside the cloud)
 * or a NaN maps to cell 0. */
uint32_t or_cell(float x, float lo, float s, int bits)
{
    uint32_t ncell = 1u << bits;
    float d = x - lo;
    float u = d * s;
    if (u >= (float)ncell) return ncell - 1u;
    if (u > 0.0f) return (uint32_t)u; /* truncation == floor for u > 0 */
    return 0u;
}

/* ------------------------------------------------------------------------ */
/* Section 4.1: Morton code.  The bits of the three coordinates are          */
/* interleaved from the most significant level down, x first in each         */
/* triple, then y, then z.                                                   */
/* ------------------------------------------------------------------------ */

uint64_t or_morton_encode(uint32_t x, uint32_t y, uint32_t z, int bits)
{
    uint64_t key = 0;
    for (int level = 0; level < bits; ++level) {
        int b = bits - 1 - level;
        uint64_t triple = ((uint64_t)((x >> b) & 1u) << 2) |
                          ((uint64_t)((y >> b) & 1u) << 1) |
                          ((uint64_t)((z >> b) & 1u));
        key = (key << 3) | triple;
    }
    return key;
}

void or_morton_decode(uint64_t key, int bits, uint32_t out[3])
{
    uint32_t x = 0, y = 0, z = 0;
    for (int level = 0; level < bits; ++level) {
        int shift = 3 * (bits - 1 - level);
        uint32_t triple = (uint32_t)((key >> shift) & 7u);
        x = (x << 1) | ((triple >> 2) & 1u);
        y = (y << 1) | ((triple >> 1) & 1u);
        z = (z << 1) | (triple & 1u);
    }
    out[0] = x;
    out[1] = y;
    out[2] = z;
}

/* ------------------------------------------------------------------------ */
/* Section 4.2: Hilbert code.  The paper accepts any continuous 3D Hilbert    */
/* variant.  This is J. Skilling's construction ("Programming the Hilbert    */
/* curve", AIP Conf. Proc. 707, 381 (2004)): the coordinates are turned into */
/* the "transposed" Hilbert index by a per-level sequence of reflections and */
/* axis exchanges followed by a Gray code, and the index is the bit          */
/* interleave of the transposed words (first word most significant in each  */
/* triple).  The curve starts at the origin cell.                            */
/* ------------------------------------------------------------------------ */

static uint64_t interleave3(const uint32_t w[3], int bits)
{
    return or_morton_encode(w[0], w[1], w[2], bits);
}

uint64_t or_hilbert_encode(uint32_t x, uint32_t y, uint32_t z, int bits)
{
    uint32_t w[3] = {x, y, z};
    uint32_t top = 1u << (bits - 1);
    /* reflections / exchanges, from the coarsest level to the finest */
    for (uint32_t q = top; q > 1u; q >>= 1) {
        uint32_t low = q - 1u;
        for (int i = 0; i < 3; ++i) {
            if (w[i] & q) {
                w[0] ^= low; /* reflect the lower bits of the first word */
            } else {
                uint32_t t = (w[0] ^ w[i]) & low; /* exchange lower bits */
                w[0] ^= t;
                w[i] ^= t;
            }
        }
    }
    /* Gray encode */
    w[1] ^= w[0];
    w[2] ^= w[1];
    uint32_t flip = 0;
    for (uint32_t q = top; q > 1u; q >>= 1)
        if (w[2] & q) flip ^= q - 1u;
    w[0] ^= flip;
    w[1] ^= flip;
    w[2] ^= flip;
    return interleave3(w, bits);
}

void or_hilbert_decode(uint64_t key, int bits, uint32_t out[3])
{
    uint32_t w[3];
    or_morton_decode(key, bits, w);
    uint32_t limit = 2u << (bits - 1);
    /* Gray decode */
    uint32_t t = w[2] >> 1;
    w[2] ^= w[1];
    w[1] ^= w[0];
    w[0] ^= t;
    /* undo the reflections / exchanges, from the finest level up */
    for (uint32_t q = 2u; q != limit; q <<= 1) {
        uint32_t low = q - 1u;
        for (int i = 2; i >= 0; --i) {
            if (w[i] & q) {
                w[0] ^= low;
            } else {
                uint32_t s = (w[0] ^ w[i]) & low;
                w[0] ^= s;
                w[i] ^= s;
            }
        }
    }
    out[0] = w[0];
    out[1] = w[1];
    out[2] = w[2];
}

/* Section 4, reorder step 1: the code of every point. */
void or_encode(const float *xyz, int64_t n, int curve, int bits, float lo_out[3],
               float *scale_out, uint64_t *keys)
{
    float lo[3], s;
    or_frame(xyz, n, bits, lo, &s);
    for (int64_t i = 0; i < n; ++i) {
        uint32_t c[3];
        for (int a = 0; a < 3; ++a) c[a] = or_cell(xyz[3 * i + a], lo[a], s, bits);
        keys[i] = (curve == OR_HILBERT) ? or_hilbert_encode(c[0], c[1], c[2], bits)
                                        : or_morton_encode(c[0], c[1], c[2], bits);
    }
    lo_out[0] = lo[0];
    lo_out[1] = lo[1];
    lo_out[2] = lo[2];
    *scale_out = s;
}

/* ------------------------------------------------------------------------ */
/* Section 4, reorder step 2: ascending order of the codes.  Equal codes are */
/* ordered by original index, which makes the permutation unique.            */
/* ------------------------------------------------------------------------ */

typedef struct {
    uint64_t key;
    uint32_t idx;
} or_kv;

static int cmp_kv(const void *a, const void *b)
{
    const or_kv *x = (const or_kv *)a, *y = (const or_kv *)b;
    if (x->key != y->key) return x->key < y->key ? -1 : 1;
    if (x->idx != y->idx) return x->idx < y->idx ? -1 : 1;
    return 0;
}

void or_sort(const uint64_t *keys, int64_t n, uint64_t *keys_sorted, uint32_t *perm)
{
    or_kv *kv = (or_kv *)malloc(sizeof(or_kv) * (size_t)(n > 0 ? n : 1));
    for (int64_t i = 0; i < n; ++i) {
        kv[i].key = keys[i];
        kv[i].idx = (uint32_t)i;
    }
    qsort(kv, (size_t)n, sizeof(or_kv), cmp_kv);
    for (int64_t i = 0; i < n; ++i) {
        keys_sorted[i] = kv[i].key;
        perm[i] = kv[i].idx;
    }
    free(kv);
}

/* ------------------------------------------------------------------------ */
/* Section 5.1: the linear octree.                                           */
/*                                                                           */
/* leaves starts as {0, 8^L}.  The points of each range [leaves[i],          */
/* leaves[i+1]) are counted by binary search on the sorted codes; a range    */
/* holding more points than the threshold is replaced by its 8 equal parts;  */
/* this repeats until nothing changes.  A range of length 1 (level L) cannot */
/* be split and stays a leaf whatever its count.  The octree is complete:    */
/* all 8 parts are kept, empty or not.  counts[i] is the number of points of */
/* leaf i.  internalRanges, the [first, last) point range of every node, is  */
/* computed for leaves and internal nodes alike, together with the tight     */
/* bounding box of the node's points (+inf/-inf for an empty node).          */
/* ------------------------------------------------------------------------ */

static int64_t lower_bound_u64(const uint64_t *a, int64_t n, uint64_t v)
{
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (a[mid] < v)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo;
}

typedef struct {
    int64_t n_leaves;
    int64_t n_internal;
    int64_t n_nodes;
    uint64_t *leaves;   /* n_leaves + 1 boundaries */
    uint32_t *counts;   /* n_leaves */
    /* every node, sorted by (level, start code) */
    uint64_t *node_start;
    int32_t *node_level;
    int64_t *node_begin;
    int64_t *node_end;
    int64_t *node_child; /* index of the first child in this order, -1 for a leaf */
    float *node_box;     /* lo.x lo.y lo.z hi.x hi.y hi.z per node */
} or_tree;

typedef struct {
    uint64_t start;
    int32_t level;
    int32_t internal;
} or_node_tmp;

static int cmp_node(const void *a, const void *b)
{
    const or_node_tmp *x = (const or_node_tmp *)a, *y = (const or_node_tmp *)b;
    if (x->level != y->level) return x->level < y->level ? -1 : 1;
    if (x->start != y->start) return x->start < y->start ? -1 : 1;
    return 0;
}

void or_tree_free(or_tree *t)
{
    if (!t) return;
    free(t->leaves);
    free(t->counts);
    free(t->node_start);
    free(t->node_level);
    free(t->node_begin);
    free(t->node_end);
    free(t->node_child);
    free(t->node_box);
    free(t);
}

or_tree *or_build_tree(const float *xyz, const uint64_t *keys_sorted, const uint32_t *perm,
                       int64_t n, int bits, uint32_t max_leaf)
{
    const uint64_t end_all = (uint64_t)1 << (3 * bits); /* 8^L */

    /* the leaves array, refined until stable */
    int64_t nl = 1;
    uint64_t *leaves = (uint64_t *)malloc(sizeof(uint64_t) * 2);
    leaves[0] = 0;
    leaves[1] = end_all;

    /* internal nodes recorded as (start, length) when split */
    int64_t ni = 0, ni_cap = 64;
    uint64_t *int_start = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)ni_cap);
    uint64_t *int_len = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)ni_cap);

    int changed = 1;
    while (changed) {
        changed = 0;
        int64_t cap = nl * 8 + 1;
        uint64_t *next = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)cap);
        int64_t m = 0;
        for (int64_t i = 0; i < nl; ++i) {
            uint64_t a = leaves[i], b = leaves[i + 1];
            int64_t count = lower_bound_u64(keys_sorted, n, b) - lower_bound_u64(keys_sorted, n, a);
            uint64_t len = b - a;
            if ((uint64_t)count > (uint64_t)max_leaf && len > 1) {
                uint64_t part = len / 8;
                for (int c = 0; c < 8; ++c) next[m++] = a + (uint64_t)c * part;
                if (ni == ni_cap) {
                    ni_cap *= 2;
                    int_start = (uint64_t *)realloc(int_start, sizeof(uint64_t) * (size_t)ni_cap);
                    int_len = (uint64_t *)realloc(int_len, sizeof(uint64_t) * (size_t)ni_cap);
                }
                int_start[ni] = a;
                int_len[ni] = len;
                ++ni;
                changed = 1;
            } else {
                next[m++] = a;
            }
        }
        next[m] = end_all;
        free(leaves);
        leaves = next;
        nl = m;
    }

    or_tree *t = (or_tree *)calloc(1, sizeof(or_tree));
    t->n_leaves = nl;
    t->n_internal = ni;
    t->n_nodes = nl + ni;
    t->leaves = leaves;
    t->counts = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)nl);
    for (int64_t i = 0; i < nl; ++i)
        t->counts[i] = (uint32_t)(lower_bound_u64(keys_sorted, n, leaves[i + 1]) -
                                  lower_bound_u64(keys_sorted, n, leaves[i]));

    /* all nodes, ordered by (level, start) */
    int64_t nn = nl + ni;
    or_node_tmp *nodes = (or_node_tmp *)malloc(sizeof(or_node_tmp) * (size_t)nn);
    for (int64_t i = 0; i < nl; ++i) {
        uint64_t len = leaves[i + 1] - leaves[i];
        int level = bits;
        while (len > 1) {
            len >>= 3;
            --level;
        }
        nodes[i].start = leaves[i];
        nodes[i].level = level;
        nodes[i].internal = 0;
    }
    for (int64_t i = 0; i < ni; ++i) {
        uint64_t len = int_len[i];
        int level = bits;
        while (len > 1) {
            len >>= 3;
            --level;
        }
        nodes[nl + i].start = int_start[i];
        nodes[nl + i].level = level;
        nodes[nl + i].internal = 1;
    }
    free(int_start);
    free(int_len);
    qsort(nodes, (size_t)nn, sizeof(or_node_tmp), cmp_node);

    t->node_start = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)nn);
    t->node_level = (int32_t *)malloc(sizeof(int32_t) * (size_t)nn);
    t->node_begin = (int64_t *)malloc(sizeof(int64_t) * (size_t)nn);
    t->node_end = (int64_t *)malloc(sizeof(int64_t) * (size_t)nn);
    t->node_child = (int64_t *)malloc(sizeof(int64_t) * (size_t)nn);
    t->node_box = (float *)malloc(sizeof(float) * 6 * (size_t)nn);
    for (int64_t i = 0; i < nn; ++i) {
        uint64_t start = nodes[i].start;
        int level = nodes[i].level;
        uint64_t len = (uint64_t)1 << (3 * (bits - level));
        t->node_start[i] = start;
        t->node_level[i] = level;
        t->node_begin[i] = lower_bound_u64(keys_sorted, n, start);
        t->node_end[i] = lower_bound_u64(keys_sorted, n, start + len);
        /* first child: the node (level + 1, start), found by linear search */
        t->node_child[i] = -1;
        if (nodes[i].internal) {
            for (int64_t j = i + 1; j < nn; ++j)
                if (nodes[j].level == level + 1 && nodes[j].start == start) {
                    t->node_child[i] = j;
                    break;
                }
        }
        float *box = t->node_box + 6 * i;
        box[0] = box[1] = box[2] = INFINITY;
        box[3] = box[4] = box[5] = -INFINITY;
        for (int64_t p = t->node_begin[i]; p < t->node_end[i]; ++p) {
            const float *pt = xyz + 3 * (int64_t)perm[p];
            for (int a = 0; a < 3; ++a) {
                if (pt[a] < box[a]) box[a] = pt[a];
                if (pt[a] > box[3 + a]) box[3 + a] = pt[a];
            }
        }
    }
    free(nodes);
    return t;
}

/* ------------------------------------------------------------------------ */
/* Section 3.2: the four search kernels, as fp32 expressions with a fixed    */
/* evaluation order (no contraction): dx = p - c per axis,                   */
/*   Sphere: (dx*dx + dy*dy) + dz*dz < r*r                                   */
/*   Circle:  dx*dx + dy*dy          < r*r                                   */
/*   Cube:   |dx| < r and |dy| < r and |dz| < r                              */
/*   Square: |dx| < r and |dy| < r                                           */
/* A radius that is not positive gives the empty set (a norm is never below  */
/* it).                                                                      */
/* ------------------------------------------------------------------------ */

int or_kernel_test(int kernel, const float *p, const float *c, float r)
{
    if (!(r > 0.0f)) return 0;
    float dx = p[0] - c[0];
    float dy = p[1] - c[1];
    float dz = p[2] - c[2];
    float r2 = r * r;
    switch (kernel) {
    case OR_SPHERE: {
        float sx = dx * dx;
        float sy = dy * dy;
        float sz = dz * dz;
        float sxy = sx + sy;
        float s = sxy + sz;
        return s < r2;
    }
    case OR_CIRCLE: {
        float sx = dx * dx;
        float sy = dy * dy;
        float s = sx + sy;
        return s < r2;
    }
    case OR_CUBE:
        return fabsf(dx) < r && fabsf(dy) < r && fabsf(dz) < r;
    case OR_SQUARE:
        return fabsf(dx) < r && fabsf(dy) < r;
    default:
        return 0;
    }
}

/* Squared Euclidean distance in the Sphere expression order. */
float or_dist2(const float *p, const float *c)
{
    float dx = p[0] - c[0];
    float dy = p[1] - c[1];
    float dz = p[2] - c[2];
    float sx = dx * dx;
    float sy = dy * dy;
    float sz = dz * dz;
    float sxy = sx + sy;
    return sxy + sz;
}

/* ------------------------------------------------------------------------ */
/* Uniform grid (the oracle's own acceleration structure; it has nothing in  */
/* common with the octree).  Cells are cubes (or xy squares for the 2D       */
/* kernels) of side h, indexed by floor((p - lo) / h) in double precision.   */
/* Points are listed by (cell id, index).                                    */
/* ------------------------------------------------------------------------ */

typedef struct {
    int dims;      /* 3: cells over x,y,z; 2: cells over x,y (all z) */
    double h;
    double lo[3];
    int64_t nc[3]; /* cells per axis */
    int64_t n;
    const float *xyz;
    int64_t *id;     /* cell id of the i-th listed point */
    uint32_t *order; /* original index of the i-th listed point */
} or_grid;

typedef struct {
    int64_t id;
    uint32_t idx;
} or_cellpt;

static int cmp_cellpt(const void *a, const void *b)
{
    const or_cellpt *x = (const or_cellpt *)a, *y = (const or_cellpt *)b;
    if (x->id != y->id) return x->id < y->id ? -1 : 1;
    if (x->idx != y->idx) return x->idx < y->idx ? -1 : 1;
    return 0;
}

static int64_t grid_coord(const or_grid *g, double v, int a)
{
    return (int64_t)floor((v - g->lo[a]) / g->h);
}

static int64_t grid_id(const or_grid *g, const int64_t c[3])
{
    if (g->dims == 2) return c[0] * g->nc[1] + c[1];
    return (c[0] * g->nc[1] + c[1]) * g->nc[2] + c[2];
}

or_grid *or_grid_build(const float *xyz, int64_t n, double h, int dims)
{
    or_grid *g = (or_grid *)calloc(1, sizeof(or_grid));
    g->dims = dims;
    g->n = n;
    g->xyz = xyz;
    double mn[3] = {0, 0, 0}, mx[3] = {0, 0, 0};
    for (int64_t i = 0; i < n; ++i)
        for (int a = 0; a < 3; ++a) {
            double v = xyz[3 * i + a];
            if (i == 0 || v < mn[a]) mn[a] = v;
            if (i == 0 || v > mx[a]) mx[a] = v;
        }
    double ext = 0;
    for (int a = 0; a < 3; ++a)
        if (mx[a] - mn[a] > ext) ext = mx[a] - mn[a];
    /* keep the cell ids inside 64 bits: at most 2^20 cells per axis */
    double hmin = ext / 1048576.0;
    if (!(h > hmin)) h = hmin;
    if (!(h > 0)) h = 1.0;
    g->h = h;
    for (int a = 0; a < 3; ++a) {
        g->lo[a] = mn[a];
        g->nc[a] = (int64_t)floor((mx[a] - mn[a]) / h) + 1;
    }
    if (dims == 2) g->nc[2] = 1;
    or_cellpt *cp = (or_cellpt *)malloc(sizeof(or_cellpt) * (size_t)(n > 0 ? n : 1));
    for (int64_t i = 0; i < n; ++i) {
        int64_t c[3] = {0, 0, 0};
        for (int a = 0; a < dims; ++a) c[a] = grid_coord(g, xyz[3 * i + a], a);
        cp[i].id = grid_id(g, c);
        cp[i].idx = (uint32_t)i;
    }
    qsort(cp, (size_t)n, sizeof(or_cellpt), cmp_cellpt);
    g->id = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    g->order = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(n > 0 ? n : 1));
    for (int64_t i = 0; i < n; ++i) {
        g->id[i] = cp[i].id;
        g->order[i] = cp[i].idx;
    }
    free(cp);
    return g;
}

void or_grid_free(or_grid *g)
{
    if (!g) return;
    free(g->id);
    free(g->order);
    free(g);
}

static int64_t lower_bound_i64(const int64_t *a, int64_t n, int64_t v)
{
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (a[mid] < v)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo;
}

static int cmp_u32(const void *a, const void *b)
{
    uint32_t x = *(const uint32_t *)a, y = *(const uint32_t *)b;
    return x < y ? -1 : (x > y ? 1 : 0);
}

/* Visit every listed point whose cell lies within `ring` cells of the query's
 * cell on every gridded axis and apply the exact kernel predicate.  With
 * h >= r, ring = ceil(r/h) + 1 covers every point the predicate can accept
 * (the extra ring absorbs the rounding of the cell computation). */
static int64_t grid_radius_one(const or_grid *g, const float *c, int kernel, float r,
                               uint32_t *out)
{
    int64_t found = 0;
    if (!(r > 0.0f) || g->n == 0) return 0;
    int64_t ring = (int64_t)ceil((double)r / g->h) + 1;
    int64_t lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
    for (int a = 0; a < g->dims; ++a) {
        int64_t cq = grid_coord(g, c[a], a);
        lo[a] = cq - ring;
        hi[a] = cq + ring;
        if (lo[a] < 0) lo[a] = 0;
        if (hi[a] > g->nc[a] - 1) hi[a] = g->nc[a] - 1;
        if (lo[a] > hi[a]) return 0;
    }
    for (int64_t cx = lo[0]; cx <= hi[0]; ++cx)
        for (int64_t cy = lo[1]; cy <= hi[1]; ++cy) {
            /* cells (cx, cy, lo[2]..hi[2]) are consecutive ids */
            int64_t c0[3] = {cx, cy, lo[2]}, c1[3] = {cx, cy, hi[2]};
            int64_t b = lower_bound_i64(g->id, g->n, grid_id(g, c0));
            int64_t e = lower_bound_i64(g->id, g->n, grid_id(g, c1) + 1);
            for (int64_t k = b; k < e; ++k) {
                uint32_t j = g->order[k];
                if (or_kernel_test(kernel, g->xyz + 3 * (int64_t)j, c, r)) {
                    if (out) out[found] = j;
                    ++found;
                }
            }
        }
    return found;
}

/* Fixed-radius search, count pass: counts[q] = |N_kernel(P, c_q, r)|. */
void or_grid_radius_count(const or_grid *g, const float *q, int64_t nq, int kernel, float r,
                          uint32_t *counts)
{
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < nq; ++i) counts[i] = (uint32_t)grid_radius_one(g, q + 3 * i, kernel, r, NULL);
}

/* Fill pass: row q of the CSR, the neighbour indices in ascending order. */
void or_grid_radius_fill(const or_grid *g, const float *q, int64_t nq, int kernel, float r,
                         const int64_t *offsets, uint32_t *indices)
{
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < nq; ++i) {
        uint32_t *row = indices + offsets[i];
        int64_t m = grid_radius_one(g, q + 3 * i, kernel, r, row);
        qsort(row, (size_t)m, sizeof(uint32_t), cmp_u32);
    }
}

/* ------------------------------------------------------------------------ */
/* Section 3.3: k nearest neighbours.  The answer is the k smallest pairs    */
/* (d2, index) in lexicographic order, d2 being the Sphere expression, in    */
/* ascending order; the centre itself is included when it is a cloud point.  */
/* Missing entries (k > n) are (index 0xFFFFFFFF, d2 = +inf).                */
/*                                                                           */
/* Grid search: rings of cells around the query's cell are visited in order  */
/* of Chebyshev cell distance rho = 0, 1, 2, ...  After ring rho every       */
/* unvisited point is at least rho*h away, so the search stops once k        */
/* candidates are held and the k-th d2 is below (rho*h)^2 with a 2^-10       */
/* relative margin, or when every cell has been visited.                     */
/* ------------------------------------------------------------------------ */

static int pair_less(float da, uint32_t ia, float db, uint32_t ib)
{
    return da < db || (da == db && ia < ib);
}

/* insert (d, i) into the ascending list of size *m (capacity k) */
static void topk_insert(float *ds, uint32_t *is, int *m, int k, float d, uint32_t i)
{
    if (*m == k && !pair_less(d, i, ds[k - 1], is[k - 1])) return;
    int pos = (*m < k) ? *m : k - 1;
    while (pos > 0 && pair_less(d, i, ds[pos - 1], is[pos - 1])) {
        ds[pos] = ds[pos - 1];
        is[pos] = is[pos - 1];
        --pos;
    }
    ds[pos] = d;
    is[pos] = i;
    if (*m < k) ++*m;
}

static void grid_knn_one(const or_grid *g, const float *c, int k, uint32_t *oi, float *od)
{
    int m = 0;
    for (int t = 0; t < k; ++t) {
        od[t] = INFINITY;
        oi[t] = 0xFFFFFFFFu;
    }
    if (g->n == 0) return;
    int64_t cq[3];
    for (int a = 0; a < 3; ++a) cq[a] = grid_coord(g, c[a], a);
    int64_t maxring = 0;
    for (int a = 0; a < 3; ++a) {
        int64_t d0 = cq[a] < 0 ? -cq[a] : cq[a];
        int64_t d1 = (g->nc[a] - 1 - cq[a]);
        if (d1 < 0) d1 = -d1;
        if (d0 > maxring) maxring = d0;
        if (d1 > maxring) maxring = d1;
    }
    for (int64_t rho = 0; rho <= maxring; ++rho) {
        for (int64_t cx = cq[0] - rho; cx <= cq[0] + rho; ++cx) {
            if (cx < 0 || cx >= g->nc[0]) continue;
            for (int64_t cy = cq[1] - rho; cy <= cq[1] + rho; ++cy) {
                if (cy < 0 || cy >= g->nc[1]) continue;
                for (int64_t cz = cq[2] - rho; cz <= cq[2] + rho; ++cz) {
                    if (cz < 0 || cz >= g->nc[2]) continue;
                    int64_t ax = cx - cq[0], ay = cy - cq[1], az = cz - cq[2];
                    if (ax < 0) ax = -ax;
                    if (ay < 0) ay = -ay;
                    if (az < 0) az = -az;
                    int64_t cheb = ax > ay ? ax : ay;
                    if (az > cheb) cheb = az;
                    if (cheb != rho) continue; /* only the shell of this ring */
                    int64_t cc[3] = {cx, cy, cz};
                    int64_t id = grid_id(g, cc);
                    int64_t b = lower_bound_i64(g->id, g->n, id);
                    int64_t e = lower_bound_i64(g->id, g->n, id + 1);
                    for (int64_t s = b; s < e; ++s) {
                        uint32_t j = g->order[s];
                        float d = or_dist2(g->xyz + 3 * (int64_t)j, c);
                        topk_insert(od, oi, &m, k, d, j);
                    }
                }
            }
        }
        if (m == k) {
            double reach = (double)rho * g->h;
            double bound = reach * reach * (1.0 - 1.0 / 1024.0);
            if ((double)od[k - 1] < bound) break;
        }
    }
}

void or_grid_knn(const or_grid *g, const float *q, int64_t nq, int k, uint32_t *idx, float *d2)
{
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < nq; ++i) grid_knn_one(g, q + 3 * i, k, idx + i * (int64_t)k, d2 + i * (int64_t)k);
}

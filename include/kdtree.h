/*
 * kdtree.h -- C ABI of the MI355X k-d tree builder (libkdtree.so).
 *
 * The library builds k-d trees level by level (Chakravorty, Cleveland &
 * Wolfe, "Scalable k-d trees for distributed data", §2 and §4): on every
 * level each cell's points are split into subsets, per-subset statistics of
 * the cell's key coordinate are combined into a split value, and the cell
 * is stably partitioned into its two children.
 *
 * Problem statement (§2, §4): a data set X of n points in d dimensions; a
 * tree of cells obtained by recursive splits along one coordinate (the key)
 * at an (approximate) median.  The split values alone determine the tree
 * (§2); the leaves are cells of about equal count (§4).
 *
 * Conventions for every entry point
 *   - Points are fp32, structure of arrays: coordinate c of point i is at
 *     pts[c * ld + i].  All point, tree and workspace pointers are DEVICE
 *     pointers owned by the caller; the library never allocates, frees or
 *     keeps them.
 *   - Keys are compared through an order-preserving map of the fp32 bit
 *     pattern to uint32 (-0 folded onto +0).  Split values are stored in that
 *     key domain; descent is "key(x[dim]) <= split -> left child".
 *   - `stream` is a hipStream_t (NULL = the null stream).
 *   - KD_EINVAL and KD_ENOMEM mean nothing was enqueued.  KD_EDEVICE means
 *     a HIP call or launch failed part-way: work enqueued before the failure
 *     may still run, so synchronize the stream before reusing the buffers.
 *     Data-dependent errors (non-finite input, node capacity) are written to
 *     hdr->status on the device.
 *   - Calls on distinct streams with distinct workspaces may run
 *     concurrently.  The library's mutable global state is the process-wide
 *     launch-shape setting (kd_set_tuning, kd_autotune) and the fixed
 *     workspace of kd_build_noalloc (one per device).
 */
#ifndef KDTREE_H
#define KDTREE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t kd_status;
enum {
    KD_OK = 0,
    KD_EINVAL = 1,      /* bad argument (sizes, rules, null pointers)        */
    KD_ENOMEM = 2,      /* workspace smaller than kd_tree_bounds() asked for */
    KD_ENAN = 3,        /* (hdr->status) input holds NaN or +-Inf            */
    KD_ECAPACITY = 4,   /* (hdr->status) node arrays too small: retry larger */
    KD_EDEVICE = 5,     /* a HIP call or kernel launch failed                */
    KD_ECANCELLED = 6   /* request withdrawn by the caller (serving loop)    */
};

/* Key coordinate of a cell (§1): cyclic x, y, z, x, ... over the levels, or
 * the coordinate of largest variance within the cell.                      */
enum { KD_KEY_CYCLIC = 0, KD_KEY_MAXVAR = 1 };

/* Split rule.
 *   EXACT   lower median of the cell's keys (the canonical tree, §1, §2);
 *           per-subset digit histograms are added (reduce by +, App. C.2).
 *   FOURIER the paper's approximate median (§3.2, Eq. (1)-(2)) with p = 1
 *           on the cell's key: additive trigonometric moments of the scaled
 *           key, J odd harmonics, summed over subsets; the split is a sign
 *           change of the equal-count equation found by bisection.
 *   SUBSET  not from the paper: size-weighted mean (subset order) of the
 *           lower medians of the cell's subsets.                          */
enum { KD_SPLIT_EXACT = 0, KD_SPLIT_FOURIER = 1, KD_SPLIT_SUBSET = 2 };

/* kd_params.flags.  KD_FLAG_LEVEL_BY_LEVEL: small cells (at most 4096
 * points) are also split one level per pass, so every level of the build
 * streams through device memory, instead of each small cell's remaining
 * levels being finished on chip in one pass.  The tree is the same either
 * way; the flag exists to measure the plain per-level build.               */
enum { KD_FLAG_LEVEL_BY_LEVEL = 1 };

typedef struct kd_params {
    uint32_t leaf_size;        /* cells with > leaf_size points are split (>= 1)   */
    uint32_t max_depth;        /* cells at this depth stay leaves; 0 -> h + 10, at
                                * most 64, with h the depth of a balanced tree
                                * (leaf_size * 2^h >= n); kd_build enqueues
                                * that many levels                               */
    uint32_t num_subsets;      /* S: subsets per cell (1..4096)                     */
    uint32_t key_rule;         /* KD_KEY_*                                          */
    uint32_t split_rule;       /* KD_SPLIT_*                                        */
    uint32_t fourier_J;        /* harmonics for FOURIER (1..64)                     */
    const uint32_t *subset_pool; /* device, pool_entries x S uint32 cumulative
                                  * weights in units of 2^-32 (entry 0 unused);
                                  * NULL -> equal subsets floor(r*n_c/S)          */
    uint32_t pool_entries;
    uint32_t flags;            /* KD_FLAG_* (0: none)                               */
    uint64_t seed;             /* picks the pool row of each cell                   */
    uint64_t node_capacity;    /* 0 -> 4*ceil(n/leaf_size)+64                       */
} kd_params;

/* Device-side header, written by the build (read it after the stream syncs). */
typedef struct kd_header {
    uint32_t num_nodes;
    uint32_t num_leaves;
    uint32_t depth;            /* largest node depth (root = 0)                     */
    int32_t status;            /* KD_OK, KD_ENAN or KD_ECAPACITY                    */
    uint64_t point_levels;     /* sum of the sizes of all split cells               */
    uint32_t unsplittable;     /* cells kept as leaves because all keys were equal  */
    uint32_t oversize;         /* leaves with more than leaf_size points            */
} kd_header;

/* Output tree: DEVICE arrays owned by the caller, sized by kd_tree_bounds().
 * Node ids are breadth first: node 0 is the root; the children of the cells
 * split at depth l get the next ids, two per split cell, in position order.
 * Leaves are numbered in position order.                                     */
typedef struct kd_tree {
    uint32_t *perm;            /* [n]   original index of each position            */
    uint32_t *node_begin;      /* [cap] first position of the node's points        */
    uint32_t *node_end;        /* [cap] one past the last position                 */
    int32_t *node_child;       /* [cap] left child id (right = left+1), -1: leaf   */
    uint32_t *node_dim;        /* [cap] key coordinate of internal nodes           */
    uint32_t *node_split;      /* [cap] split in the key domain                    */
    float *node_split_f;       /* [cap] split decoded to fp32 (informational)      */
    uint32_t *node_leaf;       /* [cap] leaf index of leaves, 0xFFFFFFFF otherwise */
    uint32_t *leaf_node;       /* [cap] node id of each leaf                       */
    uint32_t *leaf_offsets;    /* [cap+1] first position of each leaf, then n      */
    kd_header *hdr;            /* [1]                                              */
    float *points_out;         /* optional [d][n] points in perm order, or NULL    */
    uint64_t node_capacity;    /* entries in the node arrays                        */
    uint64_t n;                /* points of the tree, and their dimension: kd_build */
    uint32_t d;                /* writes both; kd_build_batched callers fill them   */
    uint32_t reserved;         /* in (0 or the item's n and d); queries check them  */
} kd_tree;

/* Sizes to allocate for a build of n points in d dimensions (host only, no
 * device work).  The tree of §2 splits cells until they hold at most
 * leaf_size points (or reach the depth cap).  node_capacity: entries of
 * each node array, params->node_capacity if set, else 4 * ceil(n /
 * leaf_size) + 64, which holds any tree whose leaves average at least
 * half of leaf_size points (a tree that needs more reports
 * KD_ECAPACITY); workspace_bytes: device workspace for kd_build.  Returns
 * KD_EINVAL on bad parameters.                                             */
kd_status kd_tree_bounds(uint64_t n, uint32_t d, const kd_params *params,
                         uint64_t *node_capacity, uint64_t *workspace_bytes);

/* Build one tree (§4).  pts: device [d][ld] fp32, read only.  out: device
 * arrays of capacity out->node_capacity.  workspace: device, ws_bytes >=
 * kd_tree_bounds().  Stream-ordered: every level up to the depth cap is
 * enqueued on `stream` and the call returns without waiting for the device
 * (it blocks only if the stream's hardware queue is full); levels the tree
 * does not reach exit at once on the device.  Nothing on the host is read by
 * the device after the call returns, so the call can be captured in a graph.
 * Read the header and arrays after the stream has completed.               */
kd_status kd_build(const float *pts, uint64_t n, uint32_t d, uint64_t ld,
                   const kd_params *params, kd_tree *out, void *workspace,
                   uint64_t ws_bytes, void *stream);

/* For callers that cannot allocate device memory (code under graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): kd_build with the
 * library's own fixed workspace instead of a caller's.  The workspace is one
 * array of KD_NOALLOC_SCRATCH_BYTES per device, held by the library until
 * the process ends; the call allocates nothing.  Builds whose workspace
 * (kd_tree_bounds with out->node_capacity) is larger return KD_ENOMEM and
 * enqueue nothing.  Every call on a device uses the same array: calls whose
 * work overlaps on one device (other streams or threads) race and must be
 * ordered by the caller.  Otherwise as kd_build (stream-ordered).          */
#define KD_NOALLOC_SCRATCH_BYTES (64ull << 20)
kd_status kd_build_noalloc(const float *pts, uint64_t n, uint32_t d, uint64_t ld,
                           const kd_params *params, kd_tree *out, void *stream);

/* Optional instrumentation of one build: HIP events recorded on the build's
 * stream around every launch, summed per kernel class.  bytes are the
 * algorithmic bytes of the launches (points x bytes-per-point of the class:
 * select and count passes read the 4-byte key; scatters read and write d
 * columns and the permutation, 8d+8 bytes).                                */
enum {
    KD_PROF_INGEST = 0,      /* copy in, identity permutation, finiteness check  */
    KD_PROF_SELECT = 1,      /* large-cell radix-select histogram passes         */
    KD_PROF_PICK = 2,        /* per-cell digit pick / split solve                */
    KD_PROF_COUNT = 3,       /* large-cell per-tile left counts and tile scans   */
    KD_PROF_BIG_SCATTER = 4, /* large-cell stable partition-scatter              */
    KD_PROF_SMALL = 5,       /* small cells: select + partition in one kernel    */
    KD_PROF_EMIT = 6,        /* node records and next-level cells                */
    KD_PROF_OTHER = 7,       /* init, leaf numbering, header                     */
    KD_PROF_KINDS = 8
};
typedef struct kd_kernel_stat {
    double ms;
    uint64_t launches;
    uint64_t points;
    uint64_t bytes;
} kd_kernel_stat;
typedef struct kd_profile {
    kd_kernel_stat k[KD_PROF_KINDS];
    uint32_t levels;
    uint32_t reserved;
} kd_profile;

/* kd_build (§4) with per-kernel timing written to *prof (host struct,
 * zeroed by the call).  Same results as kd_build; for measurement only: it waits for
 * every level's totals so launch shapes and byte counts are exact, and
 * returns when the tree is complete.                                     */
kd_status kd_build_profiled(const float *pts, uint64_t n, uint32_t d, uint64_t ld,
                            const kd_params *params, kd_tree *out, void *workspace,
                            uint64_t ws_bytes, void *stream, kd_profile *prof);

/* One tree of a batch. */
typedef struct kd_batch_item {
    const float *pts;          /* device [d][ld] */
    uint64_t n;
    uint32_t d;
    uint32_t reserved;
    uint64_t ld;
    kd_tree out;
} kd_batch_item;

/* Workspace for kd_build_batched over the given items (host only): the sum
 * of what each item's tree of §2 needs, laid out for one shared level loop. */
kd_status kd_batch_bounds(uint32_t count, const kd_batch_item *items, const kd_params *params,
                          uint64_t *workspace_bytes);

/* Build `count` independent trees, each by the level-by-level construction
 * of §4, with one set of level launches over the union of their cells.
 * Every tree is bit-identical to kd_build on it (each tree keeps its own
 * depth cap).  Stream-ordered like kd_build.                               */
kd_status kd_build_batched(uint32_t count, const kd_batch_item *items, const kd_params *params,
                           void *workspace, uint64_t ws_bytes, void *stream);

/* Leaf of each query point by descent from the root (§2's cells).  q: device
 * [d][ldq] fp32; leaf_out: device [nq].  NaN query -> 0xFFFFFFFF.  d must
 * be the tree's dimension (tree->d), else KD_EINVAL and nothing enqueued.   */
kd_status kd_query_leaf(const kd_tree *tree, const float *q, uint64_t nq, uint32_t d,
                        uint64_t ldq, uint32_t *leaf_out, void *stream);

/* Queries that use a built tree (§1, §2: the cells of the tree answer
 * nearest-neighbour and range questions).  Both need the tree's points in
 * position order (tree->points_out, built with points_out set) and n, the
 * tree's point count.  Stream-ordered; KD_EINVAL for a missing array, an n
 * or d other than the tree's (tree->n, tree->d) or a bad size, and no work
 * is enqueued then.
 *
 * kd_query_knn: the k nearest points (1 <= k <= 64) of each query q (device
 * [d][ldq] fp32, nq queries) by squared Euclidean distance, computed in fp64
 * as the sum over coordinates in order of (x_c - q_c)^2 (NaN sums count as
 * +inf), ascending, ties to the smaller point index.  idx_out: device
 * [nq][k] original point indices; dist_out: device [nq][k] squared
 * distances.  Fewer than k points: the list ends with (0xFFFFFFFF, +inf); a
 * query with a NaN coordinate gets (0xFFFFFFFF, NaN) throughout.           */
kd_status kd_query_knn(const kd_tree *tree, uint64_t n, const float *q, uint64_t nq, uint32_t d,
                       uint64_t ldq, uint32_t k, uint32_t *idx_out, double *dist_out,
                       void *stream);

/* kd_query_box: for each box [lo, hi] (device [d][ldb] fp32 each, nb boxes,
 * inclusive in every coordinate, -0 equal to +0) the number of points inside
 * in count_out (device [nb]).  With ids_out (device), also their original
 * indices, in tree position order, written from offsets[i] (device [nb],
 * e.g. the exclusive prefix sum of the counts of a first call without
 * ids_out).  A box with a NaN bound holds nothing.                          */
kd_status kd_query_box(const kd_tree *tree, uint64_t n, const float *lo, const float *hi,
                       uint64_t nb, uint32_t d, uint64_t ldb, uint32_t *count_out,
                       const uint64_t *offsets, uint32_t *ids_out, void *stream);

/* The paper's global single-pass construction (§3.2, Eq. (1)-(2); App. C in
 * its basic form), for p <= 3 coordinates.  Points: device [p][ld] fp32,
 * assumed to lie in (0,1)^p (the paper's standing assumption; mapping data
 * there is the caller's choice).  Stream-ordered; KD_EINVAL (nothing
 * enqueued) for a null pointer, p outside 1..3, J outside 1..15, depth
 * outside 1..12, n == 0 or ld < n.
 *
 * kd_global_moments: ADDS to moments (device int64 [(2J+1)^p], first
 * coordinate slowest) the statistics sum_i prod_l q_{j_l}(x_il), where q_0 =
 * Q_p and q_{2j-1}, q_{2j} = rint(Q_p cos((2j-1)x)), rint(Q_p sin((2j-1)x))
 * (fp32, own series), Q_1 = 2^24, Q_2 = 2^15, Q_3 = 2^10.  The sums are exact,
 * so calls on any split of the data into subsets add up to the statistics of
 * the whole (the paper's map-reduce); zero moments before the first call.
 * Exact up to 2^32 points in total.                                        */
kd_status kd_global_moments(const float *pts, uint64_t n, uint32_t p, uint64_t ld, uint32_t J,
                            long long *moments, void *stream);

/* kd_global_solve: the 2^depth - 1 medians of a depth-`depth` tree from the
 * statistics alone: node i (heap order; children 2i+1 on the low side and
 * 2i+2) splits coordinate (level mod p) of its cell box (a, b) at the root of
 * Eq. (2), F(m) = sum_j D_j (g_j(a_t, m) - g_j(m, b_t)) with D the statistics
 * contracted with Lemma 3.1's g_j(a_l, b_l) of the other coordinates, found
 * by fp64 bisection from (a_t, b_t) (if F(a_t) >= 0 the median is a_t).
 * medians: device fp64 [2^depth - 1].                                      */
kd_status kd_global_solve(const long long *moments, uint32_t p, uint32_t J, uint32_t depth,
                          double *medians, void *stream);

/* kd_global_counts: points in each of the 2^depth leaf cells (descent: x_t
 * <= median goes to the low side); counts: device uint64 [2^depth],
 * overwritten.                                                             */
kd_status kd_global_counts(const float *pts, uint64_t n, uint32_t p, uint64_t ld,
                           const double *medians, uint32_t depth, unsigned long long *counts,
                           void *stream);

/* Launch shapes of the level kernels.  They change only how work is spread
 * over workgroups, never the result: every setting builds the same tree bit
 * for bit.  0 in a field means the default (2048 workgroups per digit pass,
 * one workgroup per tile of 4096 points for count and scatter, one
 * workgroup per bucket of small cells, a bucket holding about 4096
 * points).  A smaller grid takes tiles or buckets in turn.                 */
typedef struct kd_tuning {
    uint32_t hist_blocks;      /* workgroups of a large-cell digit pass            */
    uint32_t scatter_blocks;   /* workgroups of the large-cell count and scatter   */
    uint32_t small_blocks;     /* workgroups of the small-cell kernel              */
    uint32_t digit_bits;       /* EXACT large-cell digit width: 11 (three passes)
                                  or 8 (four); 0 = 11; anything else: KD_EINVAL  */
} kd_tuning;

/* Process-wide launch shapes and digit width used by kd_build and
 * kd_build_batched (host only).  Set them between builds, not while builds
 * run on other threads.  None of them changes the tree.  KD_EINVAL for a
 * digit width other than 0, 8 or 11.                                        */
kd_status kd_set_tuning(const kd_tuning *t);
kd_status kd_get_tuning(kd_tuning *t);

/* Time the build of the given input under a small set of launch shapes and
 * digit widths (one field at a time: digit-pass, scatter and small-cell
 * workgroup counts, then 11- or 8-bit digits; 3 timed builds each, on
 * `stream`), check that every
 * shape yields the same tree as the current one, keep the fastest with
 * kd_set_tuning and return it in *best.  Arguments as for kd_build; `out`
 * and `workspace` are overwritten.  Returns KD_EDEVICE if a shape gave a
 * different tree (which would be a library bug).                            */
kd_status kd_autotune(const float *pts, uint64_t n, uint32_t d, uint64_t ld,
                      const kd_params *params, kd_tree *out, void *workspace,
                      uint64_t ws_bytes, void *stream, kd_tuning *best);

const char *kd_status_string(kd_status s);
int kd_version(void);

#ifdef __cplusplus
}
#endif
#endif /* KDTREE_H */

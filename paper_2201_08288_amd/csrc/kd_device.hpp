// kd_device.hpp -- device-side building blocks of the MI355X k-d tree build:
// the order-preserving key map, wave64 / workgroup scans and reductions, and
// the per-level records shared by the kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kdtree.h"

namespace kd {

constexpr int NT = 256;              // threads per workgroup (4 wave64)
constexpr int WAVE = 64;
constexpr int NW = NT / WAVE;
constexpr int TILE = 4096;           // positions per tile on the large-cell path
constexpr int PER_THREAD = TILE / NT;
constexpr int SMALL_MAX = 4096;      // cells up to this size are done by one workgroup
constexpr int RBITS = 8;             // radix-select digit width inside one workgroup
constexpr int NBINS = 1 << RBITS;
constexpr int RPASSES = 32 / RBITS;
// large cells: device-wide passes of D-bit digits, most significant first
// (the last may be narrower).  D is a launch choice (kd_tuning.digit_bits):
// 11 (three passes) by default, or 8 (four passes, smaller histograms).
// Every cell's histogram has BIG_BINS_MAX bins of room.
constexpr int BIG_DIGIT_DEFAULT = 11;
constexpr int BIG_BINS_MAX = 1 << 11;
template <int D>
struct BigDigits {
    static_assert(D >= 8 && D <= 11, "histogram rows of 256 bins, at most BIG_BINS_MAX");
    static constexpr int PASSES = (32 + D - 1) / D;
    static constexpr int BINS = 1 << D;
    __host__ __device__ static constexpr int shift(int pass) {
        return 32 - D * (pass + 1) > 0 ? 32 - D * (pass + 1) : 0;
    }
    __host__ __device__ static constexpr int bits(int pass) { return 32 - D * pass - shift(pass); }
};
constexpr int MAX_SUBSETS = 4096;
constexpr int MAX_LEVELS = 128;
constexpr uint32_t NONE = 0xffffffffu;

// One active cell of the current level.  Cells of all trees of a build form
// one list ordered by (tree, begin).
struct Cell {
    uint32_t begin, end;  // positions in the tree's working buffers
    uint32_t node;        // node id in the tree
    uint32_t tile0;       // first tile on the large-cell path
    uint32_t big;         // index among the level's large cells, NONE if small
    uint32_t slot;        // max-variance statistics slot (parent-local index * 2 + side)
    uint32_t tree;
    uint32_t voff;        // small cells: points of the level's earlier small cells
};

// Per-cell state and result of one level.
struct CellRes {
    uint32_t dim;     // key coordinate
    uint32_t split;   // split key: key <= split goes left
    uint32_t nl;      // points going left
    uint32_t flags;   // RES_* bits
    uint32_t prefix;  // radix-select prefix found so far (large cells)
    uint32_t rank;    // rank still to find below the prefix
    uint32_t cand;    // candidate m of the split rule
    uint32_t lt;      // large cells, EXACT: keys below the selected prefix
    uint32_t le;      // ... and at or below the candidate once known
    uint32_t crec[2]; // record of each child made by the small-cell subtree kernel (REC_*), 0: none
};
constexpr uint32_t RES_SPLIT = 1u;       // the cell is split
constexpr uint32_t RES_LEFT_LEAF = 2u;   // the left child stops here
constexpr uint32_t RES_RIGHT_LEAF = 4u;  // the right child stops here

// A cell below the current level whose split the small-cell subtree kernel
// already found (REC_RESOLVED), or whose key coordinate it already chose.
// Child links hold REC_RESOLVED | (record index + 1); 0 means no record.
struct SubRec {
    uint32_t dim, split, nl, flags;
    uint32_t crec[2];
};
constexpr uint32_t REC_RESOLVED = 0x80000000u;
constexpr uint32_t REC_INDEX = 0x7fffffffu;

// One tile of a large cell, ready for the scatter (written once the cell's
// split is known): positions of the tile and of its left and right runs.
struct TileDesc {
    uint32_t tb, cnt;      // first position and size of the tile
    uint32_t lpos, rpos;   // first position of the tile's left / right run
    uint32_t split, flags; // the cell's split key and RES_* flags
    uint32_t dim, tree;
    uint32_t li, pad[3];   // the cell's index within its tree's level list
};

// Read-only description of one tree of the build (device memory).
struct TreeDesc {
    const uint32_t *pts;  // caller's points as float bits, [d][ld]
    uint64_t ld;
    uint32_t *cols[2];    // working copies, [d][n], by level parity
    uint32_t *perm[2];
    unsigned long long *stats[2];  // max-variance sums [slot][d][3], by level parity
    uint32_t *out_perm;
    uint32_t *pts_out;    // optional permuted points (float bits)
    uint32_t *node_begin, *node_end;
    int32_t *node_child;
    uint32_t *node_dim, *node_split;
    float *node_split_f;
    uint32_t *node_leaf, *leaf_node, *leaf_offsets;
    kd_header *hdr;
    uint64_t pbase;       // first bit of the tree's positions in the build's leaf-start bitmap
    uint64_t cap;
    uint32_t n, d;
    uint32_t max_depth;   // cells at this depth stay leaves
    uint32_t direct;      // the root is a large cell: level 0 reads pts, not cols[0]
};

// Column `dim` of the points a level reads: the caller's points ([d][ld])
// at level 0 of a tree whose root is a large cell, else the level's working
// copy ([d][n]).  Only large-cell kernels run at level 0 of such a tree.
template <class Desc>  // TreeDesc in any address space
__device__ __forceinline__ const uint32_t *level_col(const Desc &T, uint32_t level, uint32_t dim) {
    return level == 0 && T.direct ? T.pts + uint64_t(dim) * T.ld
                                  : T.cols[level & 1] + uint64_t(dim) * T.n;
}

// Mutable per-tree counters of the level loop (device memory).
struct TreeState {
    uint32_t num_nodes, nodes_base, split_base;
    int32_t status;
    uint32_t first[2], count[2];   // the tree's cells in the level list of each parity
    uint32_t maxabs;               // bits of max |x| (max-variance grid)
    uint32_t depth, unsplittable, oversize;
    unsigned long long point_levels;
    uint32_t depth_first[MAX_LEVELS + 2];  // first node id of each depth
};

// Totals of the level about to run (read back by the host).
struct LevelInfo {
    uint32_t num_cells, num_tiles, points, big_points;
    uint32_t num_big;
    uint32_t resolved;  // points of cells already resolved by the subtree kernel
    uint32_t pad[2];
};

// Pointers read from device-side descriptors are generic; accesses through
// these views compile to global (not flat) memory instructions.
#define KD_GLOBAL __attribute__((address_space(1)))
template <class T>
__device__ __forceinline__ KD_GLOBAL T *gp(T *p) {
    return (KD_GLOBAL T *)p;
}
template <class T>
__device__ __forceinline__ const KD_GLOBAL T *gp(const T *p) {
    return (const KD_GLOBAL T *)p;
}

// Read-only views for data no kernel writes while it runs (tree descriptors,
// the current level's cell list): loads become scalar when uniform.
#define KD_CONST __attribute__((address_space(4)))
template <class T>
__device__ __forceinline__ const KD_CONST T &cref(const T *p) {
    return *(const KD_CONST T *)p;
}

// Order-preserving map of an fp32 bit pattern onto uint32; -0 folds onto +0.
__device__ __forceinline__ uint32_t key_of_bits(uint32_t b) {
    b = (b == 0x80000000u) ? 0u : b;
    return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}
__device__ __forceinline__ uint32_t bits_of_key(uint32_t u) {
    return (u & 0x80000000u) ? (u & 0x7fffffffu) : ~u;
}

__device__ __forceinline__ int lane() { return threadIdx.x & (WAVE - 1); }
__device__ __forceinline__ int wave() { return threadIdx.x / WAVE; }


// Inclusive prefix sum over a wave64 with DPP moves (no LDS traffic): row
// shifts scan each row of 16 lanes, then the row broadcasts carry the totals
// of rows 0..2 into the rows after them.  Lane 63 holds the wave's total.
template <int CTRL, int ROWS>
__device__ __forceinline__ unsigned long long dpp_add64(unsigned long long x) {
    const uint32_t lo = __builtin_amdgcn_update_dpp(0u, uint32_t(x), CTRL, ROWS, 0xf, true);
    const uint32_t hi = __builtin_amdgcn_update_dpp(0u, uint32_t(x >> 32), CTRL, ROWS, 0xf, true);
    return x + ((unsigned long long)hi << 32 | lo);
}
__device__ __forceinline__ unsigned long long wave_scan64(unsigned long long x) {
    x = dpp_add64<0x111, 0xf>(x);  // row_shr:1
    x = dpp_add64<0x112, 0xf>(x);  // row_shr:2
    x = dpp_add64<0x114, 0xf>(x);  // row_shr:4
    x = dpp_add64<0x118, 0xf>(x);  // row_shr:8
    x = dpp_add64<0x142, 0xa>(x);  // row_bcast:15 into rows 1 and 3
    x = dpp_add64<0x143, 0xc>(x);  // row_bcast:31 into rows 2 and 3
    return x;
}

// The same inclusive prefix sum on 32 bits.  Call with every lane of the
// wave active.
template <int CTRL, int ROWS>
__device__ __forceinline__ uint32_t dpp_add32(uint32_t x) {
    return x + __builtin_amdgcn_update_dpp(0u, x, CTRL, ROWS, 0xf, true);
}
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t x) {
    x = dpp_add32<0x111, 0xf>(x);
    x = dpp_add32<0x112, 0xf>(x);
    x = dpp_add32<0x114, 0xf>(x);
    x = dpp_add32<0x118, 0xf>(x);
    x = dpp_add32<0x142, 0xa>(x);
    x = dpp_add32<0x143, 0xc>(x);
    return x;
}

// Reduction of 32-bit values over a wave64 with DPP moves, for an operation
// with identity `id` (lanes a move does not reach take the identity), in the
// pattern of wave_scan64; the result is lane 63's, returned to every lane.
template <class Op>
__device__ __forceinline__ uint32_t wave_reduce32(uint32_t x, uint32_t id, Op op) {
    x = op(x, uint32_t(__builtin_amdgcn_update_dpp(int(id), int(x), 0x111, 0xf, 0xf, false)));
    x = op(x, uint32_t(__builtin_amdgcn_update_dpp(int(id), int(x), 0x112, 0xf, 0xf, false)));
    x = op(x, uint32_t(__builtin_amdgcn_update_dpp(int(id), int(x), 0x114, 0xf, 0xf, false)));
    x = op(x, uint32_t(__builtin_amdgcn_update_dpp(int(id), int(x), 0x118, 0xf, 0xf, false)));
    x = op(x, uint32_t(__builtin_amdgcn_update_dpp(int(id), int(x), 0x142, 0xa, 0xf, false)));
    x = op(x, uint32_t(__builtin_amdgcn_update_dpp(int(id), int(x), 0x143, 0xc, 0xf, false)));
    return uint32_t(__builtin_amdgcn_readlane(int(x), WAVE - 1));
}

// Sum over a wave64, valid in every lane (DPP scan, then lane 63's total).
__device__ __forceinline__ unsigned long long wave_sum64(unsigned long long x) {
    x = wave_scan64(x);
    const uint32_t lo = __builtin_amdgcn_readlane(uint32_t(x), WAVE - 1);
    const uint32_t hi = __builtin_amdgcn_readlane(uint32_t(x >> 32), WAVE - 1);
    return (unsigned long long)hi << 32 | lo;
}

// Per-thread sums of the largest-variance grid values of one column:
// s1 = sum q, and sum q^2 kept as hi * 2^32 + lo (any split of the exact sum
// is allowed; only hi * 2^32 + lo is used).  Squares (each at most 2^60) are
// added into sq, which the caller folds into hi and lo after at most 8 adds,
// so nothing wraps.
struct VarSums {
    unsigned long long s1 = 0, hi = 0, lo = 0, sq = 0;
    __device__ __forceinline__ void fold() {
        hi += sq >> 32;
        lo += sq & 0xffffffffull;
        sq = 0;
    }
    __device__ __forceinline__ void add(int q) {
        const uint32_t a = uint32_t(q < 0 ? -q : q);
        s1 += (unsigned long long)(long long)q;
        sq += (unsigned long long)a * a;
    }
};

// Lane src's value in every lane (src the same in every lane).
__device__ __forceinline__ uint32_t wave_bcast(uint32_t x, int src) {
    return uint32_t(__builtin_amdgcn_readlane(int(x), src));
}

// Wave minimum and maximum, in every lane (every lane active).
__device__ __forceinline__ uint32_t wave_min(uint32_t x) {
    return wave_reduce32(x, ~0u, [](uint32_t a, uint32_t b) { return min(a, b); });
}

__device__ __forceinline__ uint32_t wave_max(uint32_t x) {
    return wave_reduce32(x, 0u, [](uint32_t a, uint32_t b) { return max(a, b); });
}

// Exclusive prefix of one value per thread over the workgroup.  sh must hold
// NW + 1 words.  Returns the prefix; *total gets the workgroup sum.  Ends
// with a barrier, so sh may be reused right after.
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t *sh, uint32_t *total) {
    uint32_t x = wave_incl_scan(v);
    if (lane() == WAVE - 1) sh[wave()] = x;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t s = 0;
        for (int i = 0; i < NW; i++) {
            uint32_t t = sh[i];
            sh[i] = s;
            s += t;
        }
        sh[NW] = s;
    }
    __syncthreads();
    uint32_t r = sh[wave()] + x - v;
    *total = sh[NW];
    __syncthreads();
    return r;
}

// Workgroup sums of N 64-bit values (results valid in every thread).
// sh: NW * N words of LDS.
template <int N>
__device__ __forceinline__ void block_sum64n(unsigned long long *v, unsigned long long *sh) {
#pragma unroll
    for (int k = 0; k < N; k++) {
        unsigned long long x = wave_sum64(v[k]);
        if (lane() == 0) sh[wave() * N + k] = x;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < N; k++) {
        unsigned long long s = 0;
        for (int w = 0; w < NW; w++) s += sh[w * N + k];
        v[k] = s;
    }
    __syncthreads();
}

// Workgroup min and max of one value per thread.
__device__ __forceinline__ void block_minmax(uint32_t &mn, uint32_t &mx, uint32_t *sh) {
    mn = wave_min(mn);
    mx = wave_max(mx);
    if (lane() == 0) {
        sh[wave()] = mn;
        sh[NW + wave()] = mx;
    }
    __syncthreads();
    mn = sh[0];
    mx = sh[NW];
    for (int w = 1; w < NW; w++) {
        mn = min(mn, sh[w]);
        mx = max(mx, sh[NW + w]);
    }
    __syncthreads();
}

// Tie rule shared by every split rule: given the candidate m and the counts
// lt = #{key < m}, le = #{key <= m} of a cell of n points, choose the
// closest-to-balanced non-empty split ("key <= m" wins ties), stored so that
// descent is key <= split.  Returns false when all keys are equal.
__device__ __forceinline__ bool tie_rule(uint32_t n, uint32_t lt, uint32_t le, uint32_t m,
                                         uint32_t *split, uint32_t *nl) {
    if (le < n && (unsigned long long)le + lt <= n) {
        *split = m;
        *nl = le;
        return true;
    }
    if (lt > 0) {
        *split = m - 1u;
        *nl = lt;
        return true;
    }
    return false;
}

// splitmix64 (Steele, Lea & Flood 2014).
__device__ __forceinline__ unsigned long long splitmix64(unsigned long long x) {
    unsigned long long z = x + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Fixed-point grid of the largest-variance key: shift = 30 - E where
// 2^(E-1) <= max|x| < 2^E (0 when all values are 0).
__device__ __forceinline__ int maxvar_shift(uint32_t maxabs_bits) {
    if (maxabs_bits == 0) return 0;
    const uint32_t eb = maxabs_bits >> 23;
    int E;
    if (eb > 0) {
        E = int(eb) - 126;
    } else {
        const uint32_t m = maxabs_bits & 0x7fffffu;
        E = (32 - __clz(m)) - 149;
    }
    return 30 - E;
}

// q = rint(x * 2^shift) on that grid (|q| <= 2^30).
__device__ __forceinline__ long long maxvar_q(uint32_t bits, int shift) {
    return (long long)(int)rintf(ldexpf(__uint_as_float(bits), shift));
}
__device__ __forceinline__ int maxvar_q32(uint32_t bits, int shift) {
    return (int)rintf(ldexpf(__uint_as_float(bits), shift));
}

}  // namespace kd

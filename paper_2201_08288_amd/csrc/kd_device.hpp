// kd_device.hpp -- device-side building blocks of the MI355X k-d tree build:
// the order-preserving key map, wave64 / workgroup scans and reductions, and
// the per-level data records shared by the kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace kd {

constexpr int NT = 256;              // threads per workgroup (4 wave64)
constexpr int WAVE = 64;
constexpr int NW = NT / WAVE;
constexpr int TILE = 4096;           // positions per tile on the large-cell path
constexpr int PER_THREAD = TILE / NT;
constexpr int SMALL_MAX = 4096;      // cells up to this size are done by one workgroup
constexpr int RBITS = 8;             // radix-select digit width
constexpr int NBINS = 1 << RBITS;
constexpr int RPASSES = 32 / RBITS;

// One active cell of the current level: positions [begin, end) of the
// working buffers, its node id, and the first tile it owns on the
// large-cell path (cells of <= SMALL_MAX points own no tile).
struct Cell {
    uint32_t begin, end, node, tile0;
};

// Per-cell state and result of one level.
struct CellRes {
    uint32_t dim;     // key coordinate
    uint32_t split;   // split key: key <= split goes left
    uint32_t nl;      // points going left
    uint32_t flags;   // RES_* bits
    uint32_t prefix;  // radix-select prefix found so far
    uint32_t rank;    // rank still to find below the prefix
    uint32_t lt;      // keys < candidate
    uint32_t le;      // keys <= candidate
};
constexpr uint32_t RES_SPLIT = 1u;       // the cell is split
constexpr uint32_t RES_LEFT_LEAF = 2u;   // the left child stops here
constexpr uint32_t RES_RIGHT_LEAF = 4u;  // the right child stops here

// Device-side counters of the level loop.
struct LevelInfo {
    uint32_t num_cells;    // active cells of the level about to run
    uint32_t num_tiles;    // tiles of its large cells
    uint32_t num_nodes;    // nodes created so far
    uint32_t nodes_base;   // num_nodes before the last emit
    int32_t status;        // KD_OK / KD_ENAN / KD_ECAPACITY
    uint32_t unsplittable;
    uint32_t oversize;
    uint32_t num_leaves;
    unsigned long long point_levels;
    uint32_t splits;       // cells split by the last level
    uint32_t points;       // points in the active cells of the level about to run
    uint32_t big_points;   // ... of which in large cells
    uint32_t pad[3];
};

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

// Inclusive prefix sum over a wave64.
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t x) {
    const int l = lane();
#pragma unroll
    for (int o = 1; o < WAVE; o <<= 1) {
        uint32_t y = __shfl_up(x, o, WAVE);
        if (l >= o) x += y;
    }
    return x;
}

__device__ __forceinline__ uint32_t wave_sum(uint32_t x) {
#pragma unroll
    for (int o = WAVE / 2; o > 0; o >>= 1) x += __shfl_xor(x, o, WAVE);
    return x;
}

__device__ __forceinline__ unsigned long long wave_sum64(unsigned long long x) {
#pragma unroll
    for (int o = WAVE / 2; o > 0; o >>= 1) x += __shfl_xor(x, o, WAVE);
    return x;
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

// Workgroup sum of a 64-bit value (result valid in every thread).
__device__ __forceinline__ unsigned long long block_sum64(unsigned long long v,
                                                          unsigned long long *sh) {
    v = wave_sum64(v);
    if (lane() == 0) sh[wave()] = v;
    __syncthreads();
    unsigned long long s = 0;
    for (int i = 0; i < NW; i++) s += sh[i];
    __syncthreads();
    return s;
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

}  // namespace kd

// kdtree.hip -- MI355X (gfx950) level-by-level k-d tree build behind the C ABI
// declared in include/kdtree.h.
//
// A build works on one or more trees at once.  The active cells of all trees
// at the current level form one list, ordered by (tree, position); every
// kernel below runs over that list, so a batch of trees shares each level's
// launches.  One level (§2: every cell is split along its key at an
// (approximate) median into the next level's cells):
//   a2  key choice: cyclic, or the coordinate of largest variance from exact
//       fixed-point sums accumulated by the previous level's scatter;
//   a4/a5 statistic and candidate, by split rule --
//       EXACT: radix select of the lower median; large cells (> SMALL_MAX
//         points) add per-tile digit histograms into the cell's histogram
//         (map per subset, reduce by +, App. C.2), small cells select in LDS;
//       FOURIER: min/max, int64 sums of quantized harmonics (§3.2 Eq. (1)),
//         fp64 solve of the equal-count equation (Eq. (2));
//       SUBSET: lower median of every subset, fp64 mean weighted by subset
//         size in subset order (not from the paper);
//   a6  counts below / at the candidate and the tie rule;
//   a7  stable partition-scatter of every column and the permutation;
//   a8  emit: breadth-first node records and the next level's cells.
// Children that stop being split are written straight to their final place
// in the output permutation (and the optional permuted points).
#include <hip/hip_runtime.h>
#include <rocprofiler-sdk-roctx/roctx.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <type_traits>
#include <vector>

#include "kdtree.h"
#include "kd_device.hpp"
#include "kd_fourier.hpp"
#include "kd_global.hpp"
#include "kd_query.hpp"
#include "kd_select.hpp"

using namespace kd;

static_assert(NBINS == NT, "one histogram bin per thread");
static_assert(PER_THREAD * NT == TILE && SMALL_MAX <= TILE, "tile shape");
static_assert(2 * FCHUNK <= NT, "moment chunk fits one workgroup");

namespace {

constexpr int EMIT_COUNTERS = 9;
constexpr int EMIT_STRIDE = 12;
constexpr uint32_t WAVE_CELL_MAX = 1024;  // small cells up to this size: one wave per cell
// emit counters: splits, active children, tiles, points, large-cell points,
// large cells, points of split cells, unsplittable cells

struct Ctx {
    TreeDesc *trees;
    TreeState *ts;
    uint32_t ntrees;
    Cell *cells[2];
    CellRes *res;
    uint32_t *big_list;
    uint32_t *tile_lt, *tile_le;
    uint32_t *tile_mm;  // EXACT: smallest and largest last digit of a tile's keys on the prefix
    uint32_t *tile_cell;
    TileDesc *tiles;
    uint32_t *hist;
    uint32_t *mm;
    long long *mom;
    uint32_t *bounds;
    uint32_t *med;
    uint32_t *pre;
    uint32_t *scan_tmp;
    uint32_t *bucket_first;  // small cells: first cell of each bucket of TILE numbers
    // SUBSET: subsets of more than SMALL_MAX points of the level's large cells
    // (seg_count[0] subsets, seg_count[1] histogram workgroups), each with its
    // first key and size; seg_blk: the (subset, part) of each workgroup
    uint32_t *seg_count, *seg_job, *seg_prefix, *seg_rank, *seg_hist, *seg_ns, *seg_blk;
    const uint32_t **seg_col;
    LevelInfo *info;  // totals of every level (MAX_LEVELS + 1)
    // leaf numbering: a bit per position of every tree at each leaf's first
    // position, and exclusive prefix counts of set bits per word (within a
    // scan block) and per scan block
    uint32_t *leafbits, *leafpre, *leafblk;
    // records of cells resolved ahead of their level by the subtree kernel
    uint32_t *cell_rec[2];  // per cell of the level list: its record link (REC_*), 0: none
    SubRec *subrec;
    uint32_t *rec_count;
    uint32_t rec_cap;
    // largest-variance key: each record's per-coordinate sums (S1, hi, lo),
    // stride recstats_stride * 3 words
    unsigned long long *recstats;
    uint32_t recstats_stride;
    uint32_t max_d;  // the largest dimension over the build's trees
    const uint32_t *pool;
    uint32_t pool_entries;
    unsigned long long seed;
    uint32_t leaf_size, key_rule, split_rule, J, S;
    TrigTables trig;
};

// ------------------------------------------------------------ kernels: setup

__global__ void k_fill_u32(uint32_t *p, uint64_t count, uint32_t v) {
    for (uint64_t i = blockIdx.x * uint64_t(NT) + threadIdx.x; i < count;
         i += uint64_t(gridDim.x) * NT)
        p[i] = v;
}

__global__ __launch_bounds__(NT) void k_init(Ctx c) {
    const uint32_t t = blockIdx.y;
    const KD_CONST TreeDesc &T = cref(&c.trees[t]);
    for (uint64_t i = blockIdx.x * uint64_t(NT) + threadIdx.x; i < T.cap;
         i += uint64_t(gridDim.x) * NT) {
        T.node_begin[i] = 0;
        T.node_end[i] = 0;
        T.node_child[i] = -1;
        T.node_dim[i] = 0;
        T.node_split[i] = 0;
        T.node_split_f[i] = 0.0f;
        T.node_leaf[i] = NONE;
    }
    if (blockIdx.x == 0) {
        TreeState &S = c.ts[t];
        for (int k = threadIdx.x; k < MAX_LEVELS + 2; k += NT) S.depth_first[k] = k == 1 ? 1u : 0u;
        if (c.key_rule == KD_KEY_MAXVAR)
            for (uint32_t k = threadIdx.x; k < 3 * T.d; k += NT) T.stats[0][k] = 0;
        if (threadIdx.x == 0) {
            S.num_nodes = 1;
            S.nodes_base = 0;
            S.split_base = 0;
            S.status = KD_OK;
            S.first[0] = S.first[1] = 0;
            S.count[0] = S.count[1] = 0;
            S.maxabs = 0;
            S.depth = 0;
            S.unsplittable = 0;
            S.oversize = 0;
            S.point_levels = 0;
            T.node_begin[0] = 0;
            T.node_end[0] = T.n;
        }
    }
}

// a1: reject NaN / Inf, identity permutation, max |x| for the
// largest-variance grid; copy the caller's points into working buffer 0
// (float bits) unless the root is a large cell, whose level 0 reads them in
// place.
__global__ __launch_bounds__(NT) void k_ingest(Ctx c) {
    const uint32_t t = blockIdx.z, col = blockIdx.y;
    const KD_CONST TreeDesc &T = cref(&c.trees[t]);
    if (col >= T.d) return;
    const KD_GLOBAL uint32_t *src = gp(T.pts + uint64_t(col) * T.ld);
    KD_GLOBAL uint32_t *dst = gp(T.cols[0] + uint64_t(col) * T.n);
    KD_GLOBAL uint32_t *perm = gp(T.perm[0]);
    const uint32_t n = T.n;
    const bool copy = !T.direct;  // a large root's level 0 reads the caller's points
    bool bad = false;
    uint32_t mx = 0;
    // sixteen loads per thread in flight (clamped indices, no branch)
    for (uint32_t i0 = blockIdx.x * NT * 16 + threadIdx.x; i0 < n; i0 += gridDim.x * NT * 16) {
        uint32_t b[16];
#pragma unroll
        for (int j = 0; j < 16; j++) b[j] = src[min(i0 + j * NT, n - 1)];
#pragma unroll
        for (int j = 0; j < 16; j++) {
            const uint32_t i = i0 + j * NT;
            const bool in = i < n;
            const bool nf = (b[j] & 0x7f800000u) == 0x7f800000u;
            bad |= in && nf;
            mx = in && !nf ? max(mx, b[j] & 0x7fffffffu) : mx;
        }
        if (copy || col == 0) {
#pragma unroll
            for (int j = 0; j < 16; j++) {
                const uint32_t i = i0 + j * NT;
                if (i < n) {
                    if (copy) dst[i] = b[j];
                    if (col == 0) perm[i] = i;
                }
            }
        }
    }
    if (__any(bad) && lane() == 0) atomicExch(&c.ts[t].status, int32_t(KD_ENAN));
    if (c.key_rule == KD_KEY_MAXVAR) {
        mx = wave_max(mx);
        if (lane() == 0 && mx) atomicMax(&c.ts[t].maxabs, mx);
    }
}

// Small cell `slot` holds the level's small-point numbers [voff, voff + n):
// for every bucket boundary b * TILE in (voff, voff + n], the first cell that
// starts at or after it is at slot + 1 or later.
__device__ __forceinline__ void mark_buckets(const Ctx &c, uint32_t voff, uint32_t n,
                                             uint32_t slot) {
    for (uint32_t b = voff / TILE + 1; uint64_t(b) * TILE <= uint64_t(voff) + n; b++)
        c.bucket_first[b] = slot + 1;
}

// Root cells of all trees whose root is split (one workgroup).
__global__ __launch_bounds__(NT) void k_roots(Ctx c) {
    __shared__ uint32_t sh[NW + 1];
    uint32_t base[5] = {0, 0, 0, 0, 0};  // cells, tiles, points, big points, big cells
    for (uint32_t t0 = 0; t0 < c.ntrees; t0 += NT) {
        const uint32_t t = t0 + threadIdx.x;
        uint32_t v[5] = {0, 0, 0, 0, 0};
        uint32_t n = 0;
        if (t < c.ntrees) {
            n = c.trees[t].n;
            const bool active =
                c.ts[t].status == KD_OK && n > c.leaf_size && c.trees[t].max_depth > 0;
            if (active) {
                const bool big = n > uint32_t(SMALL_MAX);
                v[0] = 1;
                v[1] = big ? (n + TILE - 1) / TILE : 0u;
                v[2] = n;
                v[3] = big ? n : 0u;
                v[4] = big ? 1u : 0u;
            }
        }
        uint32_t pre[5];
        for (int k = 0; k < 5; k++) {
            uint32_t tot;
            pre[k] = base[k] + block_excl_scan(v[k], sh, &tot);
            base[k] += tot;
        }
        if (t < c.ntrees) {
            TreeState &S = c.ts[t];
            S.first[0] = pre[0];
            S.count[0] = v[0];
            if (v[0]) {
                const uint32_t voff = pre[2] - pre[3];
                Cell cl{0u, n, 0u, pre[1], v[4] ? pre[4] : NONE, 0u, t, voff};
                c.cells[0][pre[0]] = cl;
                c.cell_rec[0][pre[0]] = 0;
                if (v[4]) c.big_list[pre[4]] = pre[0];
                else mark_buckets(c, voff, n, pre[0]);
            }
        }
    }
    if (threadIdx.x == 0) {
        LevelInfo in{};
        in.num_cells = base[0];
        in.num_tiles = base[1];
        in.points = base[2];
        in.big_points = base[3];
        in.num_big = base[4];
        c.info[0] = in;
        c.bucket_first[0] = 0;
    }
}

// Largest-variance sums of the root cells (slot 0 of parity 0).  Grid:
// (blocks over points, column, tree); eight values per thread per step.
__global__ __launch_bounds__(NT) void k_root_stats(Ctx c) {
    __shared__ unsigned long long sh[NW][3];
    const uint32_t t = blockIdx.z, col = blockIdx.y;
    const TreeState &S = c.ts[t];
    const KD_CONST TreeDesc &T = cref(&c.trees[t]);
    if (S.count[0] == 0 || col >= T.d) return;
    const int shift = maxvar_shift(S.maxabs);
    const KD_GLOBAL uint32_t *src = gp(level_col(T, 0, col));
    const uint32_t n = T.n;
    VarSums a;
    for (uint32_t i0 = blockIdx.x * NT * 8 + threadIdx.x; i0 < n; i0 += gridDim.x * NT * 8) {
        uint32_t v[8];
#pragma unroll
        for (int j = 0; j < 8; j++) {
            const uint32_t i = i0 + j * NT;
            v[j] = i < n ? src[i] : 0u;
        }
#pragma unroll
        for (int j = 0; j < 8; j++) a.add(i0 + j * NT < n ? maxvar_q32(v[j], shift) : 0);
        a.fold();
    }
    unsigned long long x[3] = {a.s1, a.hi, a.lo};
#pragma unroll
    for (int i = 0; i < 3; i++) x[i] = wave_scan64(x[i]);
    if (lane() == WAVE - 1)
        for (int i = 0; i < 3; i++) sh[wave()][i] = x[i];
    __syncthreads();
    if (threadIdx.x < 3) {
        unsigned long long v = 0;
        for (int w = 0; w < NW; w++) v += sh[w][threadIdx.x];
        atomicAdd(&T.stats[0][col * 3 + threadIdx.x], v);
    }
}

// Trees whose root is a leaf: everything goes straight to the outputs.
__global__ __launch_bounds__(NT) void k_copy_leafroots(Ctx c) {
    const uint32_t t = blockIdx.y;
    const TreeState &S = c.ts[t];
    if (S.count[0] != 0 || S.status != KD_OK) return;
    const KD_CONST TreeDesc &T = cref(&c.trees[t]);
    for (uint32_t i = blockIdx.x * NT + threadIdx.x; i < T.n; i += gridDim.x * NT) {
        T.out_perm[i] = i;
        if (T.pts_out)
            for (uint32_t k = 0; k < T.d; k++)
                T.pts_out[uint64_t(k) * T.n + i] = T.cols[0][uint64_t(k) * T.n + i];
    }
}

// ------------------------------------------------------------ kernels: per level

// a2 and per-level state: key coordinate, select start, zeroed accumulators.
__device__ __forceinline__ uint32_t find_tile_cell(const Cell *cells, uint32_t ncells, uint32_t t) {
    uint32_t lo = 0, hi = ncells;
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (cells[mid].tile0 <= t) lo = mid;
        else hi = mid;
    }
    return lo;
}

// Per cell: its key coordinate and target rank (or the split a subtree
// found ahead), and the large cells' accumulators cleared.  With map_tiles,
// also the cell of every tile of the level's large cells.
__global__ __launch_bounds__(NT) void k_level_init(Ctx c, uint32_t level, uint32_t map_tiles) {
    const uint32_t cur = level & 1, nxt = cur ^ 1;
    const uint32_t ncells = c.info[level].num_cells;
    for (uint32_t ci = blockIdx.x * NT + threadIdx.x; ci < ncells; ci += gridDim.x * NT) {
        const Cell cl = c.cells[cur][ci];
        const KD_CONST TreeDesc &T = cref(&c.trees[cl.tree]);
        CellRes r{};
        const uint32_t link = c.cell_rec[cur][ci];
        const SubRec R = link ? c.subrec[(link & REC_INDEX) - 1] : SubRec{};
        if (link & REC_RESOLVED) {
            // split already found by the subtree kernel
            r.dim = R.dim;
            r.split = R.split;
            r.nl = R.nl;
            r.flags = R.flags;
            r.crec[0] = R.crec[0];
            r.crec[1] = R.crec[1];
            c.res[ci] = r;
            continue;
        }
        if (link) {
            r.dim = R.dim;  // key coordinate chosen by the subtree kernel
        } else if (c.key_rule == KD_KEY_MAXVAR) {
            const unsigned long long *st = T.stats[cur] + uint64_t(cl.slot) * T.d * 3;
            const __int128 n_c = cl.end - cl.begin;
            __int128 best = -1;
            uint32_t bd = 0;
            for (uint32_t k0 = 0; k0 < T.d; k0 += 8) {
                // eight columns' sums requested at once
                unsigned long long x[8][3];
#pragma unroll
                for (int j = 0; j < 8; j++)
#pragma unroll
                    for (int i = 0; i < 3; i++) x[j][i] = st[3 * min(k0 + j, T.d - 1) + i];
#pragma unroll
                for (int j = 0; j < 8; j++) {
                    if (k0 + j >= T.d) break;
                    // S2 = hi * 2^32 + lo; a child's parts may be its parent's
                    // minus its sibling's, so each part is read as signed
                    const long long s1 = (long long)x[j][0];
                    const __int128 s2 = (__int128)(long long)x[j][1] * ((__int128)1 << 32) +
                                        (__int128)(long long)x[j][2];
                    const __int128 V = n_c * s2 - (__int128)s1 * (__int128)s1;
                    if (V > best) {
                        best = V;
                        bd = k0 + j;
                    }
                }
            }
            r.dim = bd;
        } else {
            r.dim = level % T.d;
        }
        r.rank = (cl.end - cl.begin - 1) / 2;
        c.res[ci] = r;
        if (cl.big != NONE) {
            if (c.split_rule == KD_SPLIT_FOURIER) {
                c.mm[2 * cl.big] = NONE;
                c.mm[2 * cl.big + 1] = 0;
                long long *m = c.mom + uint64_t(cl.big) * 2 * FOURIER_JMAX;
                for (int j = 0; j < 2 * FOURIER_JMAX; j++) m[j] = 0;
            }
            if (c.key_rule == KD_KEY_MAXVAR) {
                const uint32_t li = ci - c.ts[cl.tree].first[cur];
                unsigned long long *st = T.stats[nxt] + uint64_t(2 * li) * T.d * 3;
                for (uint32_t k = 0; k < 6 * T.d; k++) st[k] = 0;
            }
        }
    }
    if (map_tiles) {
        const uint32_t ntiles = c.info[level].num_tiles;
        for (uint32_t t = blockIdx.x * NT + threadIdx.x; t < ntiles; t += gridDim.x * NT)
            c.tile_cell[t] = find_tile_cell(c.cells[cur], ncells, t);
    }
}

// Tie rule and leaf flags once the candidate and its counts are known.
__device__ __forceinline__ void finish_cell(const Ctx &c, uint32_t level, uint32_t max_depth,
                                            uint32_t n_c, CellRes &r, uint32_t m, uint32_t lt,
                                            uint32_t le) {
    uint32_t split, nl;
    r.cand = m;
    if (tie_rule(n_c, lt, le, m, &split, &nl)) {
        r.split = split;
        r.nl = nl;
        const bool deep = level + 1 >= max_depth;
        r.flags = RES_SPLIT | ((nl <= c.leaf_size || deep) ? RES_LEFT_LEAF : 0u) |
                  ((n_c - nl <= c.leaf_size || deep) ? RES_RIGHT_LEAF : 0u);
    } else {
        // all keys equal: the cell stays a leaf and its points go to the outputs
        r.split = m;
        r.nl = n_c;
        r.flags = RES_LEFT_LEAF | RES_RIGHT_LEAF;
    }
}

// Largest-variance key, large cells: the child whose per-coordinate sums the
// scatter adds up (0 left, 1 right, -1 none).  When both children go on it
// is the smaller; k_big_derive then writes the other's sums as the parent's
// minus it (exact integers).
__device__ __forceinline__ int vsum_side(uint32_t flags, uint32_t nl, uint32_t n_c) {
    if (!(flags & RES_SPLIT)) return -1;
    const bool ll = flags & RES_LEFT_LEAF, rl = flags & RES_RIGHT_LEAF;
    if (ll && rl) return -1;
    if (ll) return 1;
    if (rl) return 0;
    return nl <= n_c - nl ? 0 : 1;
}

// LDS index of staged element i: one pad word per 32 keeps a thread's run of
// consecutive elements on distinct banks.
__device__ __forceinline__ uint32_t px(uint32_t i) { return i + (i >> 5); }
constexpr int PADDED = TILE + TILE / 32;

// Tile t of the level's large cells: its cell and position range.
struct TileView {
    uint32_t ci, tb, te;
    Cell cl;
};

__device__ __forceinline__ TileView tile_view(const Ctx &c, uint32_t cur, uint32_t ncells,
                                              uint32_t t, uint32_t *s_cell) {
    TileView v;
    v.ci = __builtin_amdgcn_readfirstlane(c.tile_cell[t]);  // uniform: scalar loads below
    v.cl = c.cells[cur][v.ci];
    v.tb = v.cl.begin + (t - v.cl.tile0) * TILE;
    v.te = min(v.tb + TILE, v.cl.end);
    return v;
}


// EXACT, large cells: digit histograms of a run of consecutive tiles in LDS,
// added into the cell's histogram whenever the run moves to another cell.
template <int D>
__global__ __launch_bounds__(NT, 8) void k_big_hist(Ctx c, uint32_t level, uint32_t pass) {
    using DG = BigDigits<D>;
    __shared__ uint32_t h[DG::BINS];
    __shared__ uint32_t s_cell;
    __shared__ uint32_t tsum[2][NW][3];  // last pass: per-wave tile summary, by tile parity
    const uint32_t cur = level & 1;
    const bool last = pass == DG::PASSES - 1;
    const uint32_t ncells = c.info[level].num_cells, ntiles = c.info[level].num_tiles;
    const int shift = DG::shift(pass);
    const uint32_t dmask = (1u << DG::bits(pass)) - 1u;
    const uint32_t pmask = pass == 0 ? 0u : (~0u << (shift + DG::bits(pass)));
    const uint32_t per = (ntiles + gridDim.x - 1) / gridDim.x;
    const uint32_t t0 = blockIdx.x * per, t1 = min(t0 + per, ntiles);
    for (int b = threadIdx.x; b < DG::BINS; b += NT) h[b] = 0;
    uint32_t big = NONE;
    for (uint32_t t = t0; t < t1; t++) {
        const TileView v = tile_view(c, cur, ncells, t, &s_cell);
        if (v.cl.big != big) {
            if (big != NONE) {
                uint32_t *gh = c.hist + uint64_t(big) * BIG_BINS_MAX;
                for (int b = threadIdx.x; b < DG::BINS; b += NT) {
                    if (h[b]) atomicAdd(&gh[b], h[b]);
                    h[b] = 0;
                }
            }
            big = v.cl.big;
            __syncthreads();
        }
        const CellRes r = c.res[v.ci];
        const KD_CONST TreeDesc &T = cref(&c.trees[v.cl.tree]);
        const KD_GLOBAL uint32_t *col = gp(level_col(T, level, r.dim));
        uint32_t u[PER_THREAD];
#pragma unroll
        for (int j = 0; j < PER_THREAD; j++) {
            const uint32_t i = v.tb + j * NT + threadIdx.x;
            // the index is clamped rather than the load made conditional: a
            // load under a condition was waited for before the next was
            // issued, one load in flight instead of sixteen
            u[j] = key_of_bits(col[min(i, v.te - 1)]);  // used only where i < v.te
        }
        // a thread's keys often share a digit (the leading digits of a cell):
        // one atomic per run of equal digits.  In the last pass the same loop
        // counts the tile's keys below the prefix and on it, and the
        // smallest and largest last digit of those on it: once the
        // candidate is known, the tile's counts around it follow without
        // rereading the keys unless its last digit falls strictly inside
        uint32_t run_bin = NONE, run_cnt = 0;
        uint32_t below = 0, on = 0, dmn = 0xffffu, dmx = 0;
#pragma unroll
        for (int j = 0; j < PER_THREAD; j++) {
            const uint32_t i = v.tb + j * NT + threadIdx.x;
            const uint32_t up = u[j] & pmask;
            if (i < v.te && up == r.prefix) {
                const uint32_t bin = (u[j] >> shift) & dmask;
                if (bin != run_bin) {
                    if (run_cnt) atomicAdd(&h[run_bin], run_cnt);
                    run_bin = bin;
                    run_cnt = 0;
                }
                run_cnt++;
                on++;
                dmn = min(dmn, bin);
                dmx = max(dmx, bin);
            }
            below += i < v.te && up < r.prefix;
        }
        if (run_cnt) atomicAdd(&h[run_bin], run_cnt);
        const uint32_t par = (t - t0) & 1u;
        if (last) {
            // both counts of a wave fit 16 bits: one sum of the pair
            const uint32_t pair = wave_reduce32(below | (on << 16), 0u,
                                                [](uint32_t a, uint32_t b) { return a + b; });
            dmn = wave_reduce32(dmn, 0xffffffffu, [](uint32_t a, uint32_t b) { return min(a, b); });
            dmx = wave_reduce32(dmx, 0u, [](uint32_t a, uint32_t b) { return max(a, b); });
            if (lane() == 0) {
                tsum[par][wave()][0] = pair & 0xffffu;
                tsum[par][wave()][1] = pair >> 16;
                tsum[par][wave()][2] = dmn | (dmx << 16);
            }
        }
        __syncthreads();
        if (last && threadIdx.x == 0) {
            uint32_t below = 0, on = 0, dmn = 0xffffu, dmx = 0;
            for (int w = 0; w < NW; w++) {
                below += tsum[par][w][0];
                on += tsum[par][w][1];
                dmn = min(dmn, tsum[par][w][2] & 0xffffu);
                dmx = max(dmx, tsum[par][w][2] >> 16);
            }
            c.tile_lt[t] = below;
            c.tile_le[t] = on;
            c.tile_mm[t] = dmn | (dmx << 16);
        }
    }
    if (big != NONE) {
        uint32_t *gh = c.hist + uint64_t(big) * BIG_BINS_MAX;
        for (int b = threadIdx.x; b < DG::BINS; b += NT)
            if (h[b]) atomicAdd(&gh[b], h[b]);
    }
}

// EXACT, large cells: pick the digit that holds the target rank (one wave
// per cell).  The histogram is read (and zeroed for the next pass) in rows of
// 256 bins, lane l holding bins 4l .. 4l+3 of each row, so that every load and
// store of the wave covers 1 KB; the rank is found row by row.  After the
// last pass the candidate is the lower median and lt / le are exact.
template <int D>
__global__ __launch_bounds__(NT) void k_big_pick(Ctx c, uint32_t level, uint32_t pass) {
    using DG = BigDigits<D>;
    constexpr int ROWS = DG::BINS / (4 * WAVE);
    static_assert(ROWS * 4 * WAVE == DG::BINS, "whole rows of bins");
    const int shift = DG::shift(pass);
    const uint32_t nbig = c.info[level].num_big;
    const int l = lane();
    for (uint32_t b = blockIdx.x * NW + wave(); b < nbig; b += gridDim.x * NW) {
        const uint32_t ci = c.big_list[b];
        CellRes r = c.res[ci];
        uint4 *gh = reinterpret_cast<uint4 *>(c.hist + uint64_t(b) * BIG_BINS_MAX);
        uint4 hv[ROWS];
#pragma unroll
        for (int q = 0; q < ROWS; q++) hv[q] = gh[q * WAVE + l];
#pragma unroll
        for (int q = 0; q < ROWS; q++) gh[q * WAVE + l] = make_uint4(0u, 0u, 0u, 0u);
        uint32_t base = 0, bin = 0, below = 0, cnt = 0;
#pragma unroll
        for (int q = 0; q < ROWS; q++) {
            const uint32_t v[4] = {hv[q].x, hv[q].y, hv[q].z, hv[q].w};
            const uint32_t local = v[0] + v[1] + v[2] + v[3];
            const uint32_t incl = wave_incl_scan(local);
            const uint32_t tot = wave_bcast(incl, WAVE - 1);
            if (base <= r.rank && r.rank < base + tot) {  // uniform: the rank's row
                const uint32_t ex = base + incl - local;
                const unsigned long long m = __ballot(ex <= r.rank && r.rank < ex + local);
                const int src = __builtin_ctzll(m);  // exactly one lane holds the rank
                uint32_t lb = 0, lbelow = ex, lcnt = 0;
                bool found = false;
#pragma unroll
                for (int j = 0; j < 4; j++) {
                    if (!found && r.rank < lbelow + v[j]) {
                        lb = uint32_t(q * 4 * WAVE + 4 * l + j);
                        lcnt = v[j];
                        found = true;
                    } else if (!found) {
                        lbelow += v[j];
                    }
                }
                bin = wave_bcast(lb, src);
                below = wave_bcast(lbelow, src);
                cnt = wave_bcast(lcnt, src);
            }
            base += tot;
        }
        if (l == 0) {
            r.prefix |= bin << shift;
            r.rank -= below;
            r.lt += below;  // keys below the selected digit
            if (pass == DG::PASSES - 1) {
                r.cand = r.prefix;
                r.le = r.lt + cnt;
            }
            c.res[ci] = r;
        }
    }
}

// FOURIER, large cells: smallest and largest key of every cell.  A
// workgroup takes a run of consecutive tiles (a tile's keys loaded at once),
// keeps its threads' extremes while the run stays in one cell and adds them
// into the cell's pair when it moves on.
__global__ __launch_bounds__(NT) void k_big_minmax(Ctx c, uint32_t level) {
    __shared__ uint32_t s_cell;
    __shared__ uint32_t sh[2 * NW];
    const uint32_t cur = level & 1;
    const uint32_t ncells = c.info[level].num_cells, ntiles = c.info[level].num_tiles;
    const uint32_t per = (ntiles + gridDim.x - 1) / gridDim.x;
    const uint32_t t0 = blockIdx.x * per, t1 = min(t0 + per, ntiles);
    uint32_t big = NONE, mn = NONE, mx = 0;
    auto flush = [&]() {
        block_minmax(mn, mx, sh);
        if (threadIdx.x == 0) {
            atomicMin(&c.mm[2 * big], mn);
            atomicMax(&c.mm[2 * big + 1], mx);
        }
        mn = NONE;
        mx = 0;
    };
    for (uint32_t t = t0; t < t1; t++) {
        const TileView v = tile_view(c, cur, ncells, t, &s_cell);
        if (v.cl.big != big) {
            if (big != NONE) flush();
            big = v.cl.big;
        }
        const CellRes r = c.res[v.ci];
        const KD_CONST TreeDesc &T = cref(&c.trees[v.cl.tree]);
        const KD_GLOBAL uint32_t *col = gp(level_col(T, level, r.dim));
        uint32_t u[PER_THREAD];
#pragma unroll
        for (int j = 0; j < PER_THREAD; j++) {
            const uint32_t i = v.tb + j * NT + threadIdx.x;
            u[j] = key_of_bits(col[min(i, v.te - 1)]);  // used only where i < v.te
        }
#pragma unroll
        for (int j = 0; j < PER_THREAD; j++) {
            const uint32_t i = v.tb + j * NT + threadIdx.x;
            if (i < v.te) {
                mn = min(mn, u[j]);
                mx = max(mx, u[j]);
            }
        }
    }
    if (big != NONE) flush();
}

// Sum one chunk of per-thread moment accumulators over the workgroup into
// dst[j0 + k] (cosines) and dst[FOURIER_JMAX + j0 + k] (sines), atomically
// when several workgroups share the cell.
__device__ __forceinline__ void reduce_moments(long long *acc, unsigned long long *sh64, int j0,
                                               int J, long long *dst, bool atomic) {
#pragma unroll
    for (int k = 0; k < 2 * FCHUNK; k++) {
        const unsigned long long x = wave_sum64((unsigned long long)acc[k]);
        if (lane() == 0) sh64[wave() * 2 * FCHUNK + k] = x;
    }
    __syncthreads();
    if (threadIdx.x < 2 * FCHUNK) {
        const int k = threadIdx.x, j = j0 + (k % FCHUNK);
        if (j < J) {
            unsigned long long s = 0;
            for (int w = 0; w < NW; w++) s += sh64[w * 2 * FCHUNK + k];
            long long *d = dst + (k < FCHUNK ? 0 : FOURIER_JMAX) + j;
            if (atomic) atomicAdd((unsigned long long *)d, s);
            else *d = (long long)s;
        }
    }
    __syncthreads();
}

// FOURIER, large cells: the map step (quantized harmonics summed per cell).
// A workgroup takes a run of consecutive tiles (a tile's keys loaded at
// once), keeps its threads' integer sums while the run stays in one cell and
// adds them into the cell's moments when it moves on.
__global__ __launch_bounds__(NT) void k_big_moments(Ctx c, uint32_t level) {
    __shared__ uint32_t s_cell;
    __shared__ unsigned long long sh64[NW * 2 * FCHUNK];
    const uint32_t cur = level & 1;
    const uint32_t ncells = c.info[level].num_cells, ntiles = c.info[level].num_tiles;
    const int J = int(c.J);
    const uint32_t per = (ntiles + gridDim.x - 1) / gridDim.x;
    const uint32_t t0 = blockIdx.x * per, t1 = min(t0 + per, ntiles);
    for (int j0 = 0; j0 < J; j0 += FCHUNK) {
        uint32_t big = NONE;
        long long acc[2 * FCHUNK];
#pragma unroll
        for (int k = 0; k < 2 * FCHUNK; k++) acc[k] = 0;
        for (uint32_t t = t0; t < t1; t++) {
            const TileView v = tile_view(c, cur, ncells, t, &s_cell);
            if (v.cl.big != big) {
                if (big != NONE) {
                    reduce_moments(acc, sh64, j0, J, c.mom + uint64_t(big) * 2 * FOURIER_JMAX, true);
#pragma unroll
                    for (int k = 0; k < 2 * FCHUNK; k++) acc[k] = 0;
                }
                big = v.cl.big;
            }
            const uint32_t lo = c.mm[2 * big], hi = c.mm[2 * big + 1];
            if (lo == hi) continue;  // all keys equal: no moments needed
            const CellRes r = c.res[v.ci];
            const KD_CONST TreeDesc &T = cref(&c.trees[v.cl.tree]);
            const KD_GLOBAL uint32_t *col = gp(level_col(T, level, r.dim));
            const int e = fourier_exponent(lo, hi);
            const double xmin = value_of_key(lo), scale = fourier_scale(e);
            uint32_t u[PER_THREAD];
#pragma unroll
            for (int j = 0; j < PER_THREAD; j++) {
                const uint32_t i = v.tb + j * NT + threadIdx.x;
                u[j] = key_of_bits(col[min(i, v.te - 1)]);  // used only where i < v.te
            }
            // a tile's sums per thread fit 32 bits (16 terms of at most 2^24)
            static_assert(PER_THREAD * (1ll << 24) < (1ll << 31), "per-tile sums fit int32");
            int a32[2 * FCHUNK];
#pragma unroll
            for (int k = 0; k < 2 * FCHUNK; k++) a32[k] = 0;
            for (int j = 0; j < PER_THREAD; j++)
                if (v.tb + j * NT + threadIdx.x < v.te)
                    fourier_terms(u[j], xmin, scale, J, j0, c.trig, a32);
#pragma unroll
            for (int k = 0; k < 2 * FCHUNK; k++) acc[k] += a32[k];
        }
        if (big != NONE) reduce_moments(acc, sh64, j0, J, c.mom + uint64_t(big) * 2 * FOURIER_JMAX, true);
    }
}

// FOURIER, large cells: solve Eq. (2) for the candidate (one wave per cell).
__global__ __launch_bounds__(NT) void k_big_fsolve(Ctx c, uint32_t level) {
    __shared__ __attribute__((aligned(16))) long long cf[NW][2 * FOURIER_JMAX];
    const uint32_t nbig = c.info[level].num_big;
    for (uint32_t b = blockIdx.x * NW + wave(); b < nbig; b += gridDim.x * NW) {
        const uint32_t ci = c.big_list[b];
        const uint32_t lo = c.mm[2 * b], hi = c.mm[2 * b + 1];
        uint32_t m = lo;
        if (lo != hi) {
            const long long *mom = c.mom + uint64_t(b) * 2 * FOURIER_JMAX;
            m = fourier_solve_wave(mom, mom + FOURIER_JMAX, int(c.J), lo, hi,
                                   fourier_exponent(lo, hi), c.trig, cf[wave()]);
        }
        if (lane() == 0) c.res[ci].cand = m;
    }
}

// Subset boundaries of a cell (§3.2: any partition; App. C.2: {r, X_r}).
// Equal: floor(r * n / S).  Pool: row splitmix64(seed ^ depth << 32 ^ rank)
// mod P of cumulative 32-bit weights, bounds[r] = max(bounds[r-1], n*W_r >> 32).
__device__ __forceinline__ void subset_bounds(const Ctx &c, uint32_t n, uint32_t level,
                                              uint32_t rank, uint32_t *B) {
    const uint32_t S = c.S;
    if (!c.pool) {
        for (uint32_t r = 0; r <= S; r++) B[r] = uint32_t((uint64_t(r) * n) / S);
        return;
    }
    const unsigned long long k =
        splitmix64(c.seed ^ ((unsigned long long)level << 32) ^ (unsigned long long)rank) %
        c.pool_entries;
    const uint32_t *W = c.pool + k * S;
    B[0] = 0;
    for (uint32_t r = 1; r < S; r++) {
        const uint32_t b = uint32_t((uint64_t(n) * W[r]) >> 32);
        B[r] = max(b, B[r - 1]);
    }
    B[S] = n;
}

// Size-weighted mean of the subset lower medians, in subset order (fp64),
// rounded to fp32 and mapped to a key.
__device__ __forceinline__ uint32_t subset_mean(const uint32_t *B, const uint32_t *med,
                                                uint32_t S, uint32_t n_c) {
    double acc = 0.0;
    uint32_t r = 0;
    for (; r + 4 <= S; r += 4) {  // four subsets' sizes and medians read at a time
        uint32_t ns[4], md[4];
#pragma unroll
        for (int t = 0; t < 4; t++) {
            ns[t] = B[r + t + 1] - B[r + t];
            md[t] = med[r + t];
        }
#pragma unroll
        for (int t = 0; t < 4; t++) {
            if (ns[t] == 0) continue;
            const double prod = double(ns[t]) * value_of_key(md[t]);
            acc = acc + prod;
        }
    }
    for (; r < S; r++) {
        const uint32_t ns = B[r + 1] - B[r];
        if (ns == 0) continue;
        const double prod = double(ns) * value_of_key(med[r]);
        acc = acc + prod;
    }
    const double mean = acc / double(n_c);
    return key_of_bits(__float_as_uint(float(mean)));
}

// SUBSET, large cells: subset bounds of every cell.
__global__ __launch_bounds__(NT) void k_big_bounds(Ctx c, uint32_t level) {
    const uint32_t cur = level & 1;
    const uint32_t nbig = c.info[level].num_big;
    for (uint32_t b = blockIdx.x * NT + threadIdx.x; b < nbig; b += gridDim.x * NT) {
        const uint32_t ci = c.big_list[b];
        const Cell cl = c.cells[cur][ci];
        subset_bounds(c, cl.end - cl.begin, level, ci - c.ts[cl.tree].first[cur],
                      c.bounds + uint64_t(b) * (c.S + 1));
    }
}

// SUBSET, large cells: lower medians of the subsets of at most SMALL_MAX
// points.  A workgroup takes four subsets: those of at most WAVE_SUB points go
// to one wave each (keys staged in the wave's part of LDS), larger ones to the
// whole workgroup afterwards.
constexpr uint32_t WAVE_SUB = 1024;
__global__ __launch_bounds__(NT) void k_subset_select(Ctx c, uint32_t level) {
    __shared__ uint32_t keys[SMALL_MAX + SMALL_MAX / 32];
    __shared__ uint32_t h[NW][NBINS];
    __shared__ uint32_t sh[NW + 1], s3[3];
    const uint32_t cur = level & 1;
    const uint32_t nbig = c.info[level].num_big;
    const int w = wave(), l = lane();
    const uint64_t jobs = uint64_t(nbig) * c.S;
    auto subset = [&](uint64_t job, const uint32_t *&col, uint32_t &ns) {
        const uint32_t b = uint32_t(job / c.S), s = uint32_t(job % c.S);
        const uint32_t ci = c.big_list[b];
        const Cell cl = c.cells[cur][ci];
        const KD_CONST TreeDesc &T = cref(&c.trees[cl.tree]);
        const uint32_t *B = c.bounds + uint64_t(b) * (c.S + 1);
        ns = B[s + 1] - B[s];
        col = level_col(T, level, c.res[ci].dim) + cl.begin + B[s];
    };
    for (uint64_t j0 = uint64_t(blockIdx.x) * NW; j0 < jobs; j0 += uint64_t(gridDim.x) * NW) {
        // one wave per small subset
        {
            const uint64_t job = j0 + w;
            if (job < jobs) {
                const uint32_t *col;
                uint32_t ns;
                subset(job, col, ns);
                if (ns <= WAVE_SUB) {
                    uint32_t m = NONE;
                    if (ns > 0) {
                        const uint32_t off = uint32_t(w) * WAVE_SUB;
                        for (uint32_t i = l; i < ns; i += WAVE) {
                            const uint32_t g = off + i;
                            keys[g + (g >> 5)] = key_of_bits(col[i]);
                        }
                        wave_sync();
                        m = wave_select(keys, off, ns, (ns - 1) / 2, h[w]);
                    }
                    if (l == 0) c.med[job] = m;
                }
            }
        }
        __syncthreads();
        // the workgroup for the others up to SMALL_MAX points
        for (int q = 0; q < NW; q++) {
            const uint64_t job = j0 + q;
            if (job >= jobs) break;
            const uint32_t *col;
            uint32_t ns;
            subset(job, col, ns);
            if (ns <= WAVE_SUB || ns > uint32_t(SMALL_MAX)) continue;
            for (uint32_t i = threadIdx.x; i < ns; i += NT) keys[px(i)] = key_of_bits(col[i]);
            __syncthreads();
            const uint32_t m =
                block_select([&](uint32_t i) { return keys[px(i)]; }, ns, (ns - 1) / 2, h[0], sh, s3)
                    .key;
            if (threadIdx.x == 0) c.med[job] = m;
            __syncthreads();
        }
    }
}

// SUBSET, large cells: subsets of more than SMALL_MAX points are selected by
// several workgroups each, one per SEG_CHUNK points up to SEG_FAN.  A list of
// them (and of their workgroups) is made first; then per 8-bit digit, each
// workgroup adds the digit histogram of its part into the subset's
// histogram, and one workgroup per subset picks the digit.
constexpr uint32_t SEG_FAN = 64;
constexpr uint32_t SEG_CHUNK = PER_THREAD * NT;  // one pass of a workgroup's loads
static_assert(SEG_FAN <= 64, "(subset, part) packed in 32 bits for up to 2^26 subsets");
static_assert(SEG_CHUNK >= uint32_t(SMALL_MAX), "at most two workgroups per SMALL_MAX + 1 points");

__device__ __forceinline__ uint32_t seg_fan(uint32_t ns) {
    return min(SEG_FAN, (ns + SEG_CHUNK - 1) / SEG_CHUNK);
}

__global__ __launch_bounds__(NT) void k_seg_list(Ctx c, uint32_t level) {
    const uint32_t cur = level & 1;
    const uint32_t nbig = c.info[level].num_big;
    const uint64_t jobs = uint64_t(nbig) * c.S;
    for (uint64_t job = blockIdx.x * uint64_t(NT) + threadIdx.x; job < jobs;
         job += uint64_t(gridDim.x) * NT) {
        const uint32_t b = uint32_t(job / c.S), s = uint32_t(job % c.S);
        const uint32_t *B = c.bounds + uint64_t(b) * (c.S + 1);
        const uint32_t ns = B[s + 1] - B[s];
        if (ns > uint32_t(SMALL_MAX)) {
            const uint32_t i = atomicAdd(c.seg_count, 1u);
            const uint32_t fan = seg_fan(ns), k0 = atomicAdd(c.seg_count + 1, fan);
            const uint32_t ci = c.big_list[b];
            const Cell cl = c.cells[cur][ci];
            const KD_CONST TreeDesc &T = cref(&c.trees[cl.tree]);
            c.seg_job[i] = uint32_t(job);
            c.seg_prefix[i] = 0;
            c.seg_rank[i] = (ns - 1) / 2;
            c.seg_ns[i] = ns;
            c.seg_col[i] = level_col(T, level, c.res[ci].dim) + cl.begin + B[s];
            for (uint32_t f = 0; f < fan; f++) c.seg_blk[k0 + f] = i * SEG_FAN + f;
        }
    }
}

__global__ __launch_bounds__(NT) void k_seg_hist(Ctx c, uint32_t pass) {
    __shared__ uint32_t h[NBINS];
    const uint32_t nblk = c.seg_count[1];
    const int shift = 32 - RBITS * (pass + 1);
    const uint32_t mask = pass == 0 ? 0u : (~0u << (32 - RBITS * pass));
    for (uint32_t blk = blockIdx.x; blk < nblk; blk += gridDim.x) {
        const uint32_t bf = c.seg_blk[blk], i = bf / SEG_FAN, f = bf % SEG_FAN;
        const uint32_t ns = c.seg_ns[i], fan = seg_fan(ns);
        const uint32_t prefix = c.seg_prefix[i];
        const uint32_t per = (ns + fan - 1) / fan;
        const uint32_t a = min(f * per, ns), e = min(a + per, ns);
        h[threadIdx.x] = 0;
        __syncthreads();
        const KD_GLOBAL uint32_t *g = gp(c.seg_col[i]);
        for (uint32_t i0 = a; i0 < e; i0 += PER_THREAD * NT) {
            uint32_t u[PER_THREAD];
#pragma unroll
            for (int j = 0; j < PER_THREAD; j++) {
                const uint32_t x = i0 + j * NT + threadIdx.x;
                u[j] = key_of_bits(g[min(x, e - 1)]);  // used only where x < e
            }
#pragma unroll
            for (int j = 0; j < PER_THREAD; j++) {
                const uint32_t x = i0 + j * NT + threadIdx.x;
                if (x < e && (u[j] & mask) == prefix) atomicAdd(&h[(u[j] >> shift) & (NBINS - 1)], 1u);
            }
        }
        __syncthreads();
        if (h[threadIdx.x]) atomicAdd(&c.seg_hist[uint64_t(i) * NBINS + threadIdx.x], h[threadIdx.x]);
        __syncthreads();
    }
}

__global__ __launch_bounds__(NT) void k_seg_pick(Ctx c, uint32_t pass) {
    __shared__ uint32_t sh[NW + 1], s3[2];
    const uint32_t nseg = *c.seg_count;
    const int shift = 32 - RBITS * (pass + 1);
    for (uint32_t i = blockIdx.x; i < nseg; i += gridDim.x) {
        uint32_t *gh = c.seg_hist + uint64_t(i) * NBINS;
        const uint32_t hv = gh[threadIdx.x], rank = c.seg_rank[i];
        gh[threadIdx.x] = 0;
        uint32_t tot;
        const uint32_t ex = block_excl_scan(hv, sh, &tot);
        if (ex <= rank && rank < ex + hv) {
            s3[0] = threadIdx.x;
            s3[1] = ex;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            const uint32_t prefix = c.seg_prefix[i] | (s3[0] << shift);
            c.seg_prefix[i] = prefix;
            c.seg_rank[i] = rank - s3[1];
            if (pass == RPASSES - 1) c.med[c.seg_job[i]] = prefix;
        }
        __syncthreads();
    }
}

// SUBSET, large cells: the weighted mean (one thread per cell).
__global__ __launch_bounds__(NT) void k_subset_mean(Ctx c, uint32_t level) {
    const uint32_t cur = level & 1;
    const uint32_t nbig = c.info[level].num_big;
    for (uint32_t b = blockIdx.x * NT + threadIdx.x; b < nbig; b += gridDim.x * NT) {
        const uint32_t ci = c.big_list[b];
        const Cell cl = c.cells[cur][ci];
        c.res[ci].cand = subset_mean(c.bounds + uint64_t(b) * (c.S + 1),
                                     c.med + uint64_t(b) * c.S, c.S, cl.end - cl.begin);
    }
}

// a6, large cells: per tile, keys below and at the candidate.
// summ (EXACT): the last digit pass left each tile's keys below the prefix,
// on it, and their smallest and largest last digit (lshift, lmask); a tile
// is reread only when the candidate's last digit lies strictly between two
// different digits of its keys on the prefix.
__global__ __launch_bounds__(NT) void k_big_count(Ctx c, uint32_t level, uint32_t summ,
                                                  uint32_t lshift, uint32_t lmask) {
    __shared__ uint32_t s_cell;
    __shared__ uint32_t sh[NW + 1];
    const uint32_t cur = level & 1;
    const uint32_t ncells = c.info[level].num_cells, ntiles = c.info[level].num_tiles;
    // a run of consecutive tiles per workgroup (mostly of one cell, whose
    // records then stay in the scalar cache)
    const uint32_t per = (ntiles + gridDim.x - 1) / gridDim.x;
    const uint32_t t0 = blockIdx.x * per, t1 = min(t0 + per, ntiles);
    for (uint32_t t = t0; t < t1; t++) {
        const TileView v = tile_view(c, cur, ncells, t, &s_cell);
        const CellRes r = c.res[v.ci];
        if (summ) {
            // the decision depends only on the tile's digits, the same in
            // every wave (the counts below are rewritten by thread 0 only)
            const uint32_t below = c.tile_lt[t], on = c.tile_le[t], mm = c.tile_mm[t];
            const uint32_t dsel = (r.cand >> lshift) & lmask, dmn = mm & 0xffffu, dmx = mm >> 16;
            uint32_t lt = below, le = below;
            bool known = true;
            if (on == 0 || dsel < dmn) {
                // every key on the prefix is above the candidate
            } else if (dsel > dmx) {
                lt = le = below + on;  // every key on the prefix is below
            } else if (dmn == dmx) {
                le = below + on;  // every key on the prefix is the candidate
            } else {
                known = false;
            }
            if (known) {
                if (threadIdx.x == 0) {
                    c.tile_lt[t] = lt;
                    c.tile_le[t] = le;
                }
                continue;
            }
        }
        const KD_CONST TreeDesc &T = cref(&c.trees[v.cl.tree]);
        const KD_GLOBAL uint32_t *col = gp(level_col(T, level, r.dim));
        uint32_t lt = 0, le = 0, u[PER_THREAD];
#pragma unroll
        for (int j = 0; j < PER_THREAD; j++) {
            const uint32_t i = v.tb + j * NT + threadIdx.x;
            u[j] = key_of_bits(col[min(i, v.te - 1)]);  // used only where i < v.te
        }
#pragma unroll
        for (int j = 0; j < PER_THREAD; j++) {
            const uint32_t i = v.tb + j * NT + threadIdx.x;
            if (i < v.te) {
                lt += u[j] < r.cand;
                le += u[j] <= r.cand;
            }
        }
        // one workgroup sum of both counts (each at most TILE < 2^16)
        static_assert(TILE < (1 << 16), "tile counts fit 16 bits");
        uint32_t both;
        block_excl_scan(lt | (le << 16), sh, &both);
        if (threadIdx.x == 0) {
            c.tile_lt[t] = both & 0xffffu;
            c.tile_le[t] = both >> 16;
        }
    }
}

// a6, large cells: tie rule, then the exclusive scan of the chosen tile counts.
__global__ __launch_bounds__(NT) void k_big_decide(Ctx c, uint32_t level) {
    __shared__ uint32_t sh[NW + 1];
    const uint32_t cur = level & 1;
    const uint32_t nbig = c.info[level].num_big;
    for (uint32_t b = blockIdx.x; b < nbig; b += gridDim.x) {
        const uint32_t ci = c.big_list[b];
        const Cell cl = c.cells[cur][ci];
        const uint32_t n_c = cl.end - cl.begin;
        const uint32_t nt = (n_c + TILE - 1) / TILE;
        CellRes r = c.res[ci];
        // EXACT: the last digit pick left the cell's exact counts around the
        // candidate; the other rules add up the tiles' counts
        uint32_t lt = r.lt, le = r.le;
        if (c.split_rule != KD_SPLIT_EXACT) {
            lt = 0;
            le = 0;
            for (uint32_t k0 = 0; k0 < nt; k0 += NT) {
                const uint32_t k = k0 + threadIdx.x;
                const uint32_t a = k < nt ? c.tile_lt[cl.tile0 + k] : 0u;
                const uint32_t e = k < nt ? c.tile_le[cl.tile0 + k] : 0u;
                uint32_t ta, te;
                block_excl_scan(a, sh, &ta);
                block_excl_scan(e, sh, &te);
                lt += ta;
                le += te;
            }
        }
        finish_cell(c, level, c.trees[cl.tree].max_depth, n_c, r, r.cand, lt, le);
        const bool use_le = (r.flags & RES_SPLIT) && r.split == r.cand;
        const uint32_t li = ci - c.ts[cl.tree].first[cur];
        uint32_t base = 0;
        for (uint32_t k0 = 0; k0 < nt; k0 += NT) {
            const uint32_t k = k0 + threadIdx.x;
            uint32_t v = 0;
            if (k < nt) v = use_le ? c.tile_le[cl.tile0 + k] : c.tile_lt[cl.tile0 + k];
            uint32_t tot;
            const uint32_t ex = block_excl_scan(v, sh, &tot);
            if (k < nt) {
                const uint32_t loff = base + ex;  // left points of the cell before this tile
                TileDesc D;
                D.tb = cl.begin + k * TILE;
                D.cnt = min(uint32_t(TILE), cl.end - D.tb);
                if (r.flags & RES_SPLIT) {
                    D.lpos = cl.begin + loff;
                    D.rpos = cl.begin + r.nl + (k * TILE - loff);
                } else {  // unsplittable: the tile stays where it is (one "left" run)
                    D.lpos = D.tb;
                    D.rpos = D.tb + D.cnt;
                }
                D.split = r.split;
                D.flags = r.flags;
                D.dim = r.dim;
                D.tree = cl.tree;
                D.li = li;
                D.pad[0] = uint32_t(vsum_side(r.flags, r.nl, n_c));  // 0xffffffff: none
                D.pad[1] = D.pad[2] = 0;
                c.tiles[cl.tile0 + k] = D;
            }
            base += tot;
        }
        if (threadIdx.x == 0) c.res[ci] = r;
        __syncthreads();
    }
}

// a7, large cells: stable partition-scatter of one tile.  Ranks come from the
// staged key column; each column (and the permutation) is then permuted in
// LDS and written as two contiguous runs, the left and right children's.
// Workgroups per CU: four, or three with the largest-variance sums (their
// accumulators then fit without squeezing the rest into 128 VGPRs).
template <bool MAXVAR>
__global__ __launch_bounds__(NT, MAXVAR ? 3 : 4) void k_big_scatter(Ctx c, uint32_t level) {
    __shared__ uint32_t stage0[PADDED];  // staged keys / ranks, then a column buffer
    __shared__ uint32_t stage1[TILE];
    __shared__ uint32_t sh[NW + 1];
    __shared__ unsigned long long vacc[MAXVAR ? 16 : 1][3];  // a group of 16 columns
    const uint32_t cur = level & 1, nxt = cur ^ 1;
    const uint32_t ntiles = c.info[level].num_tiles;
    for (uint32_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const TileDesc D = c.tiles[__builtin_amdgcn_readfirstlane(t)];
        const KD_CONST TreeDesc &T = cref(&c.trees[D.tree]);
        const uint32_t cnt = D.cnt, d = T.d, n = T.n;
        const bool lleaf = D.flags & RES_LEFT_LEAF, rleaf = D.flags & RES_RIGHT_LEAF;
        uint32_t dr[PER_THREAD];
        uint32_t nleft_tile = 0;
        if (D.flags & RES_SPLIT) {
            const KD_GLOBAL uint32_t *col = gp(level_col(T, level, D.dim) + D.tb);
            uint32_t u[PER_THREAD];
#pragma unroll
            for (int j = 0; j < PER_THREAD; j++) {
                const uint32_t i = j * NT + threadIdx.x;
                u[j] = key_of_bits(col[min(i, cnt - 1)]);  // used only where i < cnt
            }
#pragma unroll
            for (int j = 0; j < PER_THREAD; j++) {
                const uint32_t i = j * NT + threadIdx.x;
                if (i < cnt) stage0[px(i)] = u[j];
            }
            __syncthreads();
            const uint32_t i0 = threadIdx.x * PER_THREAD;
            uint32_t f = 0, nleft = 0;
#pragma unroll
            for (int j = 0; j < PER_THREAD; j++) {
                const uint32_t i = i0 + j;
                const bool l = i < cnt && stage0[px(i)] <= D.split;
                f |= uint32_t(l) << j;
                nleft += l;
            }
            const uint32_t lpre = block_excl_scan(nleft, sh, &nleft_tile);
            uint32_t lo = lpre, ro = nleft_tile + (i0 - lpre);
#pragma unroll
            for (int j = 0; j < PER_THREAD; j++) {
                const uint32_t i = i0 + j;
                if (i < cnt) stage0[px(i)] = ((f >> j) & 1u) ? lo++ : ro++;
            }
            __syncthreads();
#pragma unroll
            for (int j = 0; j < PER_THREAD; j++) {
                const uint32_t i = j * NT + threadIdx.x;
                dr[j] = i < cnt ? stage0[px(i)] : 0u;
            }
        } else {
            // all keys equal: the cell is a leaf, its points go to the outputs in place
#pragma unroll
            for (int j = 0; j < PER_THREAD; j++) dr[j] = j * NT + threadIdx.x;
            nleft_tile = cnt;
        }
        const int shift = MAXVAR ? maxvar_shift(c.ts[D.tree].maxabs) : 0;
        // the one child whose sums this tile adds up (see vsum_side)
        const int vside = MAXVAR ? int(D.pad[0]) : -1;
        const bool stats = MAXVAR && vside >= 0;
        if (stats)
            for (uint32_t i = threadIdx.x; i < 16 * 3; i += NT) (&vacc[0][0])[i] = 0;
        __syncthreads();
        // column k is staged while column k + 1 is on its way
        uint32_t vn[PER_THREAD];
        {
            const KD_GLOBAL uint32_t *src = gp(level_col(T, level, 0) + D.tb);
#pragma unroll
            for (int j = 0; j < PER_THREAD; j++) {
                const uint32_t i = j * NT + threadIdx.x;
                vn[j] = src[min(i, cnt - 1)];  // used only where i < cnt
            }
        }
        for (uint32_t k = 0; k <= d; k++) {
            const bool is_perm = k == d;
            uint32_t *sg = (k & 1) ? stage1 : stage0;
            uint32_t v[PER_THREAD];
#pragma unroll
            for (int j = 0; j < PER_THREAD; j++) v[j] = vn[j];
            if (k < d) {
                const KD_GLOBAL uint32_t *src =
                    gp(k + 1 == d ? T.perm[cur] + D.tb : level_col(T, level, k + 1) + D.tb);
#pragma unroll
                for (int j = 0; j < PER_THREAD; j++) {
                    const uint32_t i = j * NT + threadIdx.x;
                    vn[j] = src[min(i, cnt - 1)];
                }
            }
#pragma unroll
            for (int j = 0; j < PER_THREAD; j++) {
                const uint32_t i = j * NT + threadIdx.x;
                if (i < cnt) sg[dr[j]] = v[j];
            }
            __syncthreads();
            KD_GLOBAL uint32_t *lnext =
                gp(is_perm ? T.perm[nxt] : T.cols[nxt] + uint64_t(k) * n);
            KD_GLOBAL uint32_t *lout =
                gp(is_perm ? T.out_perm : (T.pts_out ? T.pts_out + uint64_t(k) * n : nullptr));
            const bool kstats = stats && !is_perm;
            VarSums V;
            // left run: staged [0, nleft_tile) -> D.lpos; right run -> D.rpos
            KD_GLOBAL uint32_t *ldst = lleaf ? lout : lnext;
            if (ldst) ldst += D.lpos;
            for (uint32_t i0 = 0; i0 < nleft_tile; i0 += 8 * NT) {
#pragma unroll
                for (int jj = 0; jj < 8; jj++) {
                    const uint32_t i = i0 + jj * NT + threadIdx.x;
                    if (i < nleft_tile) {
                        const uint32_t val = sg[i];
                        if (ldst) ldst[i] = val;
                        if (kstats && vside == 0) V.add(maxvar_q32(val, shift));
                    }
                }
                V.fold();
            }
            KD_GLOBAL uint32_t *rdst = rleaf ? lout : lnext;
            if (rdst) rdst += D.rpos;
            for (uint32_t i0 = nleft_tile; i0 < cnt; i0 += 8 * NT) {
#pragma unroll
                for (int jj = 0; jj < 8; jj++) {
                    const uint32_t i = i0 + jj * NT + threadIdx.x;
                    if (i < cnt) {
                        const uint32_t val = sg[i];
                        if (rdst) rdst[i - nleft_tile] = val;
                        if (kstats && vside == 1) V.add(maxvar_q32(val, shift));
                    }
                }
                V.fold();
            }
            if (kstats) {
                // wave sums into the workgroup's accumulators of this column
                unsigned long long x[3] = {V.s1, V.hi, V.lo};
#pragma unroll
                for (int q = 0; q < 3; q++) x[q] = wave_scan64(x[q]);
                if (lane() == WAVE - 1)
#pragma unroll
                    for (int q = 0; q < 3; q++) atomicAdd(&vacc[k & 15][q], x[q]);
                if ((k & 15) == 15 || k + 1 == d) {
                    __syncthreads();
                    const uint32_t k0 = k & ~15u;
                    for (uint32_t i = threadIdx.x; i < 16 * 3; i += NT) {
                        const uint32_t kk = k0 + i / 3, q = i % 3;
                        if (kk < d)
                            atomicAdd(T.stats[nxt] + (uint64_t(2 * D.li + vside) * d + kk) * 3 + q,
                                      (&vacc[0][0])[i]);
                        (&vacc[0][0])[i] = 0;
                    }
                }
            }
        }
        __syncthreads();
    }
}

// Largest-variance key, large cells whose children both go on: the child
// the scatter did not sum gets the cell's sums minus the summed child's
// (exact integers), one thread per (cell, word) so that every load of the
// level is in flight at once.
__global__ __launch_bounds__(NT) void k_big_derive(Ctx c, uint32_t level) {
    const uint32_t cur = level & 1, nxt = cur ^ 1;
    const uint32_t nbig = c.info[level].num_big;
    const uint32_t wmax = 3 * c.max_d;
    for (uint64_t i = uint64_t(blockIdx.x) * NT + threadIdx.x; i < uint64_t(nbig) * wmax;
         i += uint64_t(gridDim.x) * NT) {
        const uint32_t b = uint32_t(i / wmax), k = uint32_t(i - uint64_t(b) * wmax);
        const uint32_t ci = c.big_list[b];
        const Cell cl = c.cells[cur][ci];
        const KD_CONST TreeDesc &T = cref(&c.trees[cl.tree]);
        if (k >= 3 * T.d) continue;
        const CellRes r = c.res[ci];
        if (!(r.flags & RES_SPLIT) || (r.flags & (RES_LEFT_LEAF | RES_RIGHT_LEAF))) continue;
        const int side = vsum_side(r.flags, r.nl, cl.end - cl.begin);
        const uint32_t li = ci - c.ts[cl.tree].first[cur];
        const uint64_t w3 = 3 * T.d;
        T.stats[nxt][(2 * li + (side ^ 1)) * w3 + k] =
            T.stats[cur][uint64_t(cl.slot) * w3 + k] - T.stats[nxt][(2 * li + side) * w3 + k];
    }
}

// ------------------------------------------------------------ small cells
//
// Cells of at most SMALL_MAX points.  Each small cell carries voff, the
// number of points in the level's earlier small cells, so the level's small
// points are numbered 0, 1, ... in cell order.  Those numbers are cut into
// buckets of TILE; a workgroup takes the cells that start in its bucket and
// works through them in chunks of whole cells of one tree (at most TILE points
// and SC cells), doing the whole level step of a chunk on chip: keys staged
// in LDS, the split of every cell (one wave per cell up to WAVE_CELL_MAX
// points, otherwise the workgroup), ranks from one chunk-wide scan, then every
// column and the permutation permuted through LDS.  A chunk's cells hold the
// same positions before and after the step, so each column is read and written
// over the same position ranges, with coalesced accesses.

// Cells per chunk: 64 keeps the plain kernel's LDS within four workgroups per
// CU; the largest-variance kernel (three per CU by registers) takes 128.
// Chunk-local cell ids fit a byte either way.
template <bool MAXVAR>
constexpr int chunk_cells() { return MAXVAR ? 128 : 64; }

template <int SC>
struct ChunkLds {
    uint32_t ci[SC];         // cell index in the level list
    uint32_t start[SC + 1];  // chunk-local number of the cell's first point
    uint32_t off[SC];        // position minus chunk-local number
    uint32_t dim[SC];
    uint32_t li[SC];         // index in the tree's level list
    uint32_t split[SC], nl[SC], flags[SC], base[SC];
    uint32_t wide[4];            // cells above WAVE_CELL_MAX points (at most 3)
    uint32_t count, total, tree, next, nwide;
    uint32_t goes_on;            // some child of the chunk is split again
};

// Wave 0: collect the next chunk, starting at cell `pos`, from the cells that
// start before number v1.  Big cells are skipped; a chunk stops at the first
// cell of another tree, at SC cells, and before a cell that runs past v1
// (such a cell, the bucket's last, forms a chunk of its own).
template <int SC>
__device__ void form_chunk(const Ctx &c, uint32_t cur, uint32_t ncells, uint32_t pos,
                           uint32_t v1, ChunkLds<SC> &C) {
    const int l = lane();
    uint32_t count = 0, total = 0, tree = NONE, first = 0, nwide = 0;
    for (;;) {
        const uint32_t ci = pos + l;
        const bool valid = ci < ncells;
        Cell cl{};
        if (valid) cl = c.cells[cur][ci];
        const bool small = valid && cl.big == NONE && cl.voff != NONE;  // not resolved ahead
        const uint32_t nk = cl.end - cl.begin;
        const bool beyond = !valid || (small && cl.voff >= v1);
        const unsigned long long bmask = __ballot(beyond);
        const int fb = bmask ? __builtin_ctzll(bmask) : WAVE;
        const unsigned long long below_fb = fb == WAVE ? ~0ull : ((1ull << fb) - 1);
        const unsigned long long smask = __ballot(small) & below_fb;
        if (tree == NONE && smask) {
            tree = wave_bcast(cl.tree, __builtin_ctzll(smask));
            first = c.ts[tree].first[cur];
        }
        const uint32_t before =
            count + uint32_t(__popcll(smask & ((1ull << l) - 1)));  // small cells before lane l
        const bool cross = small && !beyond && uint64_t(cl.voff) + nk > v1;
        const bool stop =
            beyond || (small && (cl.tree != tree || before >= uint32_t(SC) || (cross && before > 0)));
        const unsigned long long stmask = __ballot(stop);
        const int s = stmask ? __builtin_ctzll(stmask) : WAVE;
        const bool take = small && l < s;
        const uint32_t sz = take ? nk : 0u;
        const uint32_t incl = wave_incl_scan(sz);
        if (take) {
            const uint32_t k = before, st = total + incl - sz;
            C.ci[k] = ci;
            C.start[k] = st;
            C.off[k] = cl.begin - st;
            C.dim[k] = c.res[ci].dim;
            C.li[k] = ci - first;
        }
        const unsigned long long wmask = __ballot(take && nk > WAVE_CELL_MAX);
        if (take && nk > WAVE_CELL_MAX) C.wide[nwide + __popcll(wmask & ((1ull << l) - 1))] = before;
        nwide += uint32_t(__popcll(wmask));
        count += uint32_t(__popcll(__ballot(take)));
        total += wave_bcast(incl, WAVE - 1);
        pos += uint32_t(s);
        if (s < WAVE) break;
    }
    if (l == 0) {
        C.count = count;
        C.total = total;
        C.tree = tree;
        C.next = pos;
        C.nwide = nwide;
        C.start[count] = total;
        C.goes_on = 0;
    }
}

// Split of one chunk cell from its candidate and counts; the result goes to
// the level's cell results and to the chunk table.
template <int SC>
__device__ __forceinline__ void store_cell(const Ctx &c, uint32_t level, ChunkLds<SC> &C, uint32_t k,
                                           uint32_t m, uint32_t lt, uint32_t le) {
    const uint32_t n_c = C.start[k + 1] - C.start[k];
    CellRes r{};
    r.dim = C.dim[k];
    r.rank = (n_c - 1) / 2;
    finish_cell(c, level, c.trees[C.tree].max_depth, n_c, r, m, lt, le);
    r.lt = lt;
    r.le = le;
    c.res[C.ci[k]] = r;
    if ((r.flags & RES_SPLIT) && (~r.flags & (RES_LEFT_LEAF | RES_RIGHT_LEAF))) C.goes_on = 1;
    C.split[k] = r.split;
    C.nl[k] = r.nl;
    C.flags[k] = r.flags;
}

// Wave sums of 2 * FCHUNK per-lane values at once: each exchange hands the
// partner lane half of the values still held and adds the half it keeps, so
// lane l ends with the total of value l >> 1 (lanes 2k and 2k + 1 both).  The
// first two exchanges add at most four lanes' sums, which the caller bounds
// below 2^31; the rest run in 64 bits.  Integer sums, exact in any order.
__device__ __forceinline__ long long wave_sum_transposed(const int (&acc)[2 * FCHUNK]) {
    static_assert(2 * FCHUNK == WAVE / 2, "one value per pair of lanes");
    const int l = lane();
    int v16[16];
#pragma unroll
    for (int i = 0; i < 16; i++) {
        const bool up = l & 32;
        const int keep = up ? acc[16 + i] : acc[i], give = up ? acc[i] : acc[16 + i];
        v16[i] = keep + __shfl_xor(give, 32, WAVE);
    }
    int v8[8];
#pragma unroll
    for (int i = 0; i < 8; i++) {
        const bool up = l & 16;
        const int keep = up ? v16[8 + i] : v16[i], give = up ? v16[i] : v16[8 + i];
        v8[i] = keep + __shfl_xor(give, 16, WAVE);
    }
    long long v4[4];
#pragma unroll
    for (int i = 0; i < 4; i++) {
        const bool up = l & 8;
        const long long keep = up ? v8[4 + i] : v8[i], give = up ? v8[i] : v8[4 + i];
        v4[i] = keep + __shfl_xor(give, 8, WAVE);
    }
    long long v2[2];
#pragma unroll
    for (int i = 0; i < 2; i++) {
        const bool up = l & 4;
        const long long keep = up ? v4[2 + i] : v4[i], give = up ? v4[i] : v4[2 + i];
        v2[i] = keep + __shfl_xor(give, 4, WAVE);
    }
    const bool up = l & 2;
    const long long v1 = (up ? v2[1] : v2[0]) + __shfl_xor(up ? v2[0] : v2[1], 2, WAVE);
    return v1 + __shfl_xor(v1, 1, WAVE);
}

// Candidate of a cell of at most WAVE_CELL_MAX points by one wave (EXACT,
// FOURIER); keys at keys[px(s0 + i)], i < nk.
template <int RULE>
__device__ void wave_candidate(const Ctx &c, const uint32_t *keys, uint32_t s0, uint32_t nk,
                               uint32_t *h, long long *mom, uint32_t &m, uint32_t &lt,
                               uint32_t &le) {
    const int l = lane();
    if (RULE == KD_SPLIT_EXACT) {
        m = wave_select(keys, s0, nk, (nk - 1) / 2, h);
    } else {
        uint32_t mn = NONE, mx = 0;
        for (uint32_t i = l; i < nk; i += WAVE) {
            const uint32_t u = keys[px(s0 + i)];
            mn = min(mn, u);
            mx = max(mx, u);
        }
        mn = wave_min(mn);
        mx = wave_max(mx);
        m = mn;
        if (mn != mx) {
            const int J = int(c.J);
            const int e = fourier_exponent(mn, mx);
            const double xmin = value_of_key(mn), scale = fourier_scale(e);
            for (int j0 = 0; j0 < J; j0 += FCHUNK) {
                // the sums of four lanes fit 32 bits: at most 4 * WAVE_CELL_MAX / WAVE
                // terms, each at most 2^24 * (1 + 2^-10) (|cos|, |sin| of the
                // fp32 recurrence stay within that of 1)
                static_assert(4 * (WAVE_CELL_MAX / WAVE) * ((1ll << 24) + (1ll << 14)) < (1ll << 31),
                              "int32 sums");
                int acc[2 * FCHUNK];
#pragma unroll
                for (int k = 0; k < 2 * FCHUNK; k++) acc[k] = 0;
                for (uint32_t i = l; i < nk; i += WAVE)
                    fourier_terms(keys[px(s0 + i)], xmin, scale, J, j0, c.trig, acc);
                const long long sum = wave_sum_transposed(acc);
                const int k = l >> 1, j = j0 + (k % FCHUNK);
                if (!(l & 1) && j < J) mom[(k < FCHUNK ? 0 : FOURIER_JMAX) + j] = sum;
            }
            wave_sync();
            m = fourier_solve_wave(mom, mom + FOURIER_JMAX, J, mn, mx, e, c.trig, mom);
            wave_sync();
        }
    }
    uint32_t a = 0, b = 0;
    for (uint32_t i = l; i < nk; i += WAVE) {
        const uint32_t u = keys[px(s0 + i)];
        a += u < m;
        b += u <= m;
    }
    lt = uint32_t(wave_sum64(a));
    le = uint32_t(wave_sum64(b));
}

// Candidate of one cell by the whole workgroup (EXACT, FOURIER).
template <int RULE>
__device__ void block_candidate(const Ctx &c, uint32_t level, const uint32_t *keys, uint32_t s0,
                                uint32_t nk, uint32_t li, uint32_t (*h)[NBINS], uint32_t *sh,
                                uint32_t *s3, unsigned long long *sh64, long long *mom,
                                uint32_t *dyn, uint32_t &m, uint32_t &lt, uint32_t &le) {
    if (RULE == KD_SPLIT_EXACT) {
        const SelectResult sel = block_select([&](uint32_t i) { return keys[px(s0 + i)]; }, nk,
                                              (nk - 1) / 2, h[0], sh, s3);
        m = sel.key;
        lt = sel.lt;
        le = sel.le;
        return;
    }
    {  // FOURIER
        uint32_t mn = NONE, mx = 0;
        for (uint32_t i = threadIdx.x; i < nk; i += NT) {
            const uint32_t u = keys[px(s0 + i)];
            mn = min(mn, u);
            mx = max(mx, u);
        }
        block_minmax(mn, mx, sh);
        m = mn;
        if (mn != mx) {
            const int J = int(c.J);
            const int e = fourier_exponent(mn, mx);
            const double xmin = value_of_key(mn), scale = fourier_scale(e);
            for (int j0 = 0; j0 < J; j0 += FCHUNK) {
                // the sums of four threads fit 32 bits: at most 4 * TILE / NT
                // terms of at most 2^24 * (1 + 2^-10) (see wave_candidate)
                static_assert(4 * (TILE / NT) * ((1ll << 24) + (1ll << 14)) < (1ll << 31),
                              "int32 sums");
                int a32[2 * FCHUNK];
#pragma unroll
                for (int k = 0; k < 2 * FCHUNK; k++) a32[k] = 0;
                for (uint32_t i = threadIdx.x; i < nk; i += NT)
                    fourier_terms(keys[px(s0 + i)], xmin, scale, J, j0, c.trig, a32);
                // wave totals (transposed), then the workgroup's
                const long long ws = wave_sum_transposed(a32);
                if (!(lane() & 1)) sh64[wave() * 2 * FCHUNK + (lane() >> 1)] = ws;
                __syncthreads();
                if (threadIdx.x < 2 * FCHUNK) {
                    const int k = threadIdx.x, j = j0 + (k % FCHUNK);
                    if (j < J) {
                        long long t = 0;
                        for (int w = 0; w < NW; w++) t += (long long)sh64[w * 2 * FCHUNK + k];
                        mom[(k < FCHUNK ? 0 : FOURIER_JMAX) + j] = t;
                    }
                }
                __syncthreads();
            }
            if (wave() == 0) {
                const uint32_t mm = fourier_solve_wave(mom, mom + FOURIER_JMAX, J, mn, mx, e,
                                                       c.trig, mom);
                if (lane() == 0) s3[0] = mm;
            }
            __syncthreads();
            m = s3[0];
            __syncthreads();
        }
    }
    unsigned long long cnt2[2] = {0, 0};
    for (uint32_t i = threadIdx.x; i < nk; i += NT) {
        const uint32_t u = keys[px(s0 + i)];
        cnt2[0] += u < m;
        cnt2[1] += u <= m;
    }
    block_sum64n<2>(cnt2, sh64);
    lt = uint32_t(cnt2[0]);
    le = uint32_t(cnt2[1]);
}

// SUBSET, small cells: the split candidates of chunk cells [k0, k0 + G) at
// once.  dyn holds, per cell, its subset bounds B[0..S] and medians med[0..S).
// Subsets of at most RANK_MAX points find their lower median by counting
// ranks (each point counts the smaller points of its subset, ties broken by
// position); larger subsets use a wave radix select.  The weighted mean runs
// one thread per cell, in subset order.
constexpr uint32_t RANK_MAX = 64;

// Last r in [0, S) with B[r] <= i, for nondecreasing B with B[0] <= i: a
// four-way search whose three probes per step are read together.
__device__ __forceinline__ uint32_t last_at_most(const uint32_t *B, uint32_t S, uint32_t i) {
    uint32_t lo = 0, hi = S;  // B[lo] <= i; the answer lies in [lo, hi)
    while (hi - lo > 1) {
        const uint32_t w = hi - lo;
        const uint32_t q1 = lo + w / 4, q2 = lo + w / 2, q3 = lo + (3 * w) / 4;
        const uint32_t b1 = B[q1], b2 = B[q2], b3 = B[q3];
        if (b3 <= i) {
            lo = q3;
        } else if (b2 <= i) {
            lo = q2;
            hi = q3;
        } else if (b1 <= i) {
            lo = q1;
            hi = q2;
        } else {
            hi = q1;  // q1 > lo here: B[lo] <= i
        }
    }
    return lo;
}

// Rank of key u (at slot e) among the m keys at slots s0 .. s0+m-1, ties
// broken by slot; four keys read at a time.
__device__ __forceinline__ uint32_t rank_in_subset(const uint32_t *keys, uint32_t s0, uint32_t m,
                                                   uint32_t u, uint32_t e) {
    uint32_t rank = 0, j = 0;
    for (; j + 4 <= m; j += 4) {
        uint32_t v[4];
#pragma unroll
        for (int t = 0; t < 4; t++) v[t] = keys[px(s0 + j + t)];
#pragma unroll
        for (int t = 0; t < 4; t++) rank += (v[t] < u) || (v[t] == u && s0 + j + t < e);
    }
    for (; j < m; j++) {
        const uint32_t v = keys[px(s0 + j)];
        rank += (v < u) || (v == u && s0 + j < e);
    }
    return rank;
}
constexpr uint32_t SUBSET_DYN_WORDS = 7680;  // dynamic LDS of the SUBSET small-cell kernels (30 KB)
template <int SC>
__device__ void subset_cells(const Ctx &c, uint32_t level, const uint32_t *keys,
                             const uint8_t *seg, ChunkLds<SC> &C, uint32_t k0, uint32_t G,
                             uint32_t *dyn, uint32_t (*h)[NBINS]) {
    const uint32_t S = c.S, stride = 2 * S + 1;
    const int w = wave(), l = lane();
    // subset bounds, one wave per cell
    for (uint32_t g = w; g < G; g += NW) {
        const uint32_t k = k0 + g, n = C.start[k + 1] - C.start[k];
        uint32_t *B = dyn + g * stride;
        if (!c.pool) {
            for (uint32_t r = l; r <= S; r += WAVE) B[r] = uint32_t((uint64_t(r) * n) / S);
        } else {
            const unsigned long long row =
                splitmix64(c.seed ^ ((unsigned long long)level << 32) ^
                           (unsigned long long)C.li[k]) % c.pool_entries;
            const uint32_t *W = c.pool + row * S;
            // B[r] = max over 1 <= j <= r of (n * W[j]) >> 32: a running maximum,
            // lanes taking consecutive runs of r
            const uint32_t per = (S + WAVE - 1) / WAVE, r0 = 1 + l * per;
            uint32_t run = 0;
            for (uint32_t r = r0; r < min(r0 + per, S); r++)
                run = max(run, uint32_t((uint64_t(n) * W[r]) >> 32));
            // exclusive running maximum of the lanes before this one
            uint32_t x = run;
#pragma unroll
            for (int o = 1; o < WAVE; o <<= 1) {
                const uint32_t y = __shfl_up(x, o, WAVE);
                if (l >= o) x = max(x, y);
            }
            uint32_t before = __shfl_up(x, 1, WAVE);
            if (l == 0) before = 0;
            for (uint32_t r = r0; r < min(r0 + per, S); r++) {
                before = max(before, uint32_t((uint64_t(n) * W[r]) >> 32));
                B[r] = before;
            }
            if (l == 0) {
                B[0] = 0;
                B[S] = n;
            }
        }
    }
    __syncthreads();
    // lower medians of small subsets by counting ranks
    const uint32_t e0 = C.start[k0], e1 = C.start[k0 + G];
    for (uint32_t e = e0 + threadIdx.x; e < e1; e += NT) {
        const uint32_t g = seg[e] - k0, i = e - C.start[k0 + g];
        const uint32_t *B = dyn + g * stride;
        // subset of position i: the last r with B[r] <= i
        const uint32_t lo = last_at_most(B, S, i);
        const uint32_t b = B[lo], m = B[lo + 1] - b;
        if (m > RANK_MAX) continue;
        const uint32_t s0 = C.start[k0 + g] + b, u = keys[px(e)];
        if (rank_in_subset(keys, s0, m, u, e) == (m - 1) / 2) dyn[g * stride + S + 1 + lo] = u;
    }
    // empty subsets, and lower medians of the large ones (a wave select
    // each): a wave takes a cell and checks 64 subsets at a time
    for (uint32_t g = w; g < G; g += NW) {
        const uint32_t *B = dyn + g * stride;
        uint32_t *med = dyn + g * stride + S + 1;
        for (uint32_t r0 = 0; r0 < S; r0 += WAVE) {
            const uint32_t r = r0 + l;
            bool large = false;
            if (r < S) {
                const uint32_t m = B[r + 1] - B[r];
                if (m == 0) med[r] = NONE;
                large = m > RANK_MAX;
            }
            for (unsigned long long mask = __ballot(large); mask; mask &= mask - 1) {
                const uint32_t rr = r0 + uint32_t(__builtin_ctzll(mask));
                const uint32_t b = B[rr], m = B[rr + 1] - b;
                const uint32_t v = wave_select(keys, C.start[k0 + g] + b, m, (m - 1) / 2, h[w]);
                if (l == 0) med[rr] = v;
            }
        }
    }
    __syncthreads();
    // weighted mean of the medians, in subset order (one thread per cell)
    for (uint32_t g = threadIdx.x; g < G; g += NT) {
        const uint32_t k = k0 + g;
        C.split[k] = subset_mean(dyn + g * stride, dyn + g * stride + S + 1, S,
                                 C.start[k + 1] - C.start[k]);
    }
    __syncthreads();
    // counts around the candidate and the tie rule, one wave per cell
    for (uint32_t g = w; g < G; g += NW) {
        const uint32_t k = k0 + g, s0 = C.start[k], nk = C.start[k + 1] - s0, m = C.split[k];
        uint32_t a = 0, b = 0;
        for (uint32_t i = l; i < nk; i += WAVE) {
            const uint32_t u = keys[px(s0 + i)];
            a += u < m;
            b += u <= m;
        }
        a = uint32_t(wave_sum64(a));
        b = uint32_t(wave_sum64(b));
        if (l == 0) store_cell(c, level, C, k, m, a, b);
    }
    __syncthreads();
}

template <int RULE, bool MAXVAR>
__global__ __launch_bounds__(NT, MAXVAR ? (RULE != KD_SPLIT_FOURIER ? 3 : 1) : (RULE == KD_SPLIT_EXACT ? 4 : 1)) void k_small(Ctx c, uint32_t level) {
    constexpr int SC = chunk_cells<MAXVAR>();
    // the column buffer is idle while cells are split: the select scratch
    // (digit histograms, FOURIER moments, reductions) shares its space
    struct SelectScratch {
        uint32_t h[NW][NBINS];
        unsigned long long sh64[NW * 2 * FCHUNK];
        long long mom[NW][RULE == KD_SPLIT_FOURIER ? 2 * FOURIER_JMAX : 1];
    };
    union StageOrSelect {
        uint32_t stage[TILE];
        SelectScratch sel;
    };
    static_assert(sizeof(SelectScratch) <= sizeof(uint32_t) * TILE, "select scratch fits");
    __shared__ uint32_t keys[PADDED];  // staged keys, then each number's destination
    __shared__ __attribute__((aligned(16))) StageOrSelect lds;
    __shared__ __attribute__((aligned(16))) uint8_t seg[TILE];  // chunk cell of each number
    __shared__ ChunkLds<SC> C;
    __shared__ uint32_t sh[2 * NW + 1], s3[4];
    uint32_t *const stage = lds.stage;
    uint32_t(*const h)[NBINS] = lds.sel.h;
    unsigned long long *const sh64 = lds.sel.sh64;
    auto &mom = lds.sel.mom;
    // MAXVAR: chunk prefix sums (S1, hi, lo) at every cell start (2k) and split
    // point (2k + 1), and the chunk total (2K); per-wave totals of the scan
    __shared__ unsigned long long pat[MAXVAR ? 2 * SC + 1 : 1][3];
    __shared__ unsigned long long wtot[MAXVAR ? NW : 1][3];
    extern __shared__ uint32_t dyn[];  // SUBSET: bounds[S + 1], medians[S]
    const uint32_t cur = level & 1, nxt = cur ^ 1;
    const int w = wave(), l = lane();
    const LevelInfo I = c.info[level];
    const uint32_t ncells = I.num_cells;
    const uint32_t nbuckets = (I.points - I.big_points - I.resolved + TILE - 1) / TILE;
    for (uint32_t b = blockIdx.x; b < nbuckets; b += gridDim.x) {
        uint32_t pos = c.bucket_first[b];
        const uint32_t v1 = (b + 1) * uint32_t(TILE);
        for (;;) {
            if (w == 0) form_chunk(c, cur, ncells, pos, v1, C);
            __syncthreads();
            const uint32_t K = C.count, tot = C.total;
            pos = C.next;
            const uint32_t tr = __builtin_amdgcn_readfirstlane(C.tree);
            __syncthreads();
            if (K == 0) break;
            const KD_CONST TreeDesc &T = cref(&c.trees[tr]);
            const uint32_t d = T.d, n = T.n;
            for (uint32_t k = w; k < K; k += NW)
                for (uint32_t e = C.start[k] + l; e < C.start[k + 1]; e += WAVE) seg[e] = uint8_t(k);
            __syncthreads();
            // keys of the chunk (EXACT: the first column is requested at the same
            // time and arrives while the cells are split)
            uint32_t vn[PER_THREAD];
            {
                uint32_t u[PER_THREAD], p[PER_THREAD];
#pragma unroll
                for (int j = 0; j < PER_THREAD; j++) {
                    const uint32_t e = j * NT + threadIdx.x;
                    u[j] = 0;
                    vn[j] = 0;
                    if (e < tot) {
                        const uint32_t k = seg[e];
                        p[j] = C.off[k] + e;
                        u[j] = gp(T.cols[cur] + uint64_t(C.dim[k]) * n)[p[j]];
                        if (RULE == KD_SPLIT_EXACT) vn[j] = gp(T.cols[cur])[p[j]];
                    }
                }
#pragma unroll
                for (int j = 0; j < PER_THREAD; j++) {
                    const uint32_t e = j * NT + threadIdx.x;
                    if (e < tot) keys[px(e)] = key_of_bits(u[j]);
                }
            }
            __syncthreads();
            // split of every cell: wide cells by the workgroup, the rest one per wave
            if (RULE == KD_SPLIT_SUBSET) {
                const uint32_t G = max(1u, SUBSET_DYN_WORDS / (2 * c.S + 1));
                for (uint32_t k0 = 0; k0 < K; k0 += G)
                    subset_cells(c, level, keys, seg, C, k0, min(G, K - k0), dyn, h);
            } else {
                for (uint32_t q = 0; q < C.nwide; q++) {
                    const uint32_t k = C.wide[q];
                    uint32_t m, lt, le;
                    block_candidate<RULE>(c, level, keys, C.start[k], C.start[k + 1] - C.start[k],
                                          C.li[k], h, sh, s3, sh64, mom[0], dyn, m, lt, le);
                    if (threadIdx.x == 0) store_cell(c, level, C, k, m, lt, le);
                }
                for (uint32_t k = w; k < K; k += NW) {
                    const uint32_t s0 = C.start[k], nk = C.start[k + 1] - s0;
                    if (nk > WAVE_CELL_MAX) continue;
                    uint32_t m, lt, le;
                    wave_candidate<RULE>(c, keys, s0, nk, h[w], mom[w], m, lt, le);
                    if (l == 0) store_cell(c, level, C, k, m, lt, le);
                }
            }
            __syncthreads();
            // ranks: thread t owns numbers 16t .. 16t+15; one chunk-wide scan of
            // the left flags, less the scan value at each cell's first number.
            // MAXVAR records: bit j of rmask marks number 16t + j as a cell
            // start or a split point, byte j of rid its record index.
            uint32_t rmask = 0, rid[4] = {0, 0, 0, 0};
            {
                const uint32_t e0 = threadIdx.x * PER_THREAD;
                const uint4 sq = *reinterpret_cast<const uint4 *>(seg + e0);
                const uint32_t sw[4] = {sq.x, sq.y, sq.z, sq.w};
                uint32_t sk[PER_THREAD];
#pragma unroll
                for (int j = 0; j < PER_THREAD; j++) sk[j] = (sw[j >> 2] >> (8 * (j & 3))) & 0xffu;
                uint32_t nleft = 0, fl = 0;
#pragma unroll
                for (int j = 0; j < PER_THREAD; j++) {
                    const uint32_t e = e0 + j;
                    if (e < tot && keys[px(e)] <= C.split[sk[j]]) {
                        nleft++;
                        fl |= 1u << j;
                    }
                }
                uint32_t all;
                const uint32_t lbase = block_excl_scan(nleft, sh, &all);
                uint32_t run = lbase;
#pragma unroll
                for (int j = 0; j < PER_THREAD; j++) {
                    const uint32_t e = e0 + j;
                    if (e < tot && e == C.start[sk[j]]) C.base[sk[j]] = run;
                    run += (fl >> j) & 1u;
                }
                __syncthreads();
                run = lbase;
#pragma unroll
                for (int j = 0; j < PER_THREAD; j++) {
                    const uint32_t e = e0 + j;
                    if (e < tot) {
                        const uint32_t k = sk[j], s = C.start[k], lr = run - C.base[k];
                        const uint32_t dd = (fl >> j) & 1u ? s + lr : s + C.nl[k] + (e - s) - lr;
                        keys[px(e)] = min(dd, uint32_t(TILE - 1));
                        if (MAXVAR) {
                            const bool at_split = (C.flags[k] & RES_SPLIT) && e == s + C.nl[k];
                            if (e == s || at_split) {
                                rmask |= 1u << j;
                                rid[j >> 2] |= (2 * k + (at_split ? 1u : 0u)) << (8 * (j & 3));
                            }
                        }
                    }
                    run += (fl >> j) & 1u;
                }
            }
            __syncthreads();
            // every column and the permutation: stage at the destination, write
            // in number order; numbers whose child stops go to the outputs
            uint32_t ps[PER_THREAD], leafm = 0;
#pragma unroll
            for (int j = 0; j < PER_THREAD; j++) {
                const uint32_t e = j * NT + threadIdx.x;
                ps[j] = 0;
                if (e < tot) {
                    const uint32_t k = seg[e];
                    ps[j] = C.off[k] + e;
                    const bool right = e - C.start[k] >= C.nl[k];
                    if (C.flags[k] & (right ? RES_RIGHT_LEAF : RES_LEFT_LEAF)) leafm |= 1u << j;
                }
            }
            // every load issued (no branch; slots past the chunk read place 0)
            if (RULE != KD_SPLIT_EXACT) {
                const KD_GLOBAL uint32_t *src = gp(T.cols[cur]);
#pragma unroll
                for (int j = 0; j < PER_THREAD; j++) vn[j] = src[ps[j]];
            }
            const int shift = MAXVAR ? maxvar_shift(c.ts[tr].maxabs) : 0;
            const bool chunk_stats = MAXVAR && C.goes_on;
            for (uint32_t col = 0; col <= d; col++) {
                uint32_t v[PER_THREAD];
#pragma unroll
                for (int j = 0; j < PER_THREAD; j++) v[j] = vn[j];
                if (col < d) {
                    const KD_GLOBAL uint32_t *src =
                        gp(col + 1 == d ? T.perm[cur] : T.cols[cur] + uint64_t(col + 1) * n);
#pragma unroll
                    for (int j = 0; j < PER_THREAD; j++) vn[j] = src[ps[j]];  // place 0 past the chunk
                }
                // staged at the destination, in groups of eight whose places
                // are read together (no branch: slots past the chunk go to
                // their own place, which no number of the chunk goes to); one
                // at a time where registers are short
                constexpr int SG = (RULE == KD_SPLIT_EXACT && !MAXVAR) ? 4 : 8;
                if constexpr (RULE == KD_SPLIT_EXACT && !MAXVAR) {
#pragma unroll
                    for (int j = 0; j < PER_THREAD; j++) {
                        const uint32_t e = j * NT + threadIdx.x;
                        if (e < tot) stage[keys[px(e)]] = v[j];
                    }
                } else {
#pragma unroll
                    for (int j0 = 0; j0 < PER_THREAD; j0 += SG) {
                        uint32_t dd[SG];
#pragma unroll
                        for (int j = 0; j < SG; j++) dd[j] = keys[px((j0 + j) * NT + threadIdx.x)];
#pragma unroll
                        for (int j = 0; j < SG; j++) {
                            const uint32_t e = (j0 + j) * NT + threadIdx.x;
                            stage[e < tot ? dd[j] : e] = v[j0 + j];
                        }
                    }
                }
                __syncthreads();
                KD_GLOBAL uint32_t *nb =
                    gp(col == d ? T.perm[nxt] : T.cols[nxt] + uint64_t(col) * n);
                KD_GLOBAL uint32_t *ob =
                    col == d ? gp(T.out_perm)
                             : (T.pts_out ? gp(T.pts_out + uint64_t(col) * n) : nullptr);
#pragma unroll
                for (int j0 = 0; j0 < PER_THREAD; j0 += SG) {
                    uint32_t sv[SG];
#pragma unroll
                    for (int j = 0; j < SG; j++) sv[j] = stage[(j0 + j) * NT + threadIdx.x];
#pragma unroll
                    for (int j = 0; j < SG; j++) {
                        const uint32_t e = (j0 + j) * NT + threadIdx.x;
                        if (e < tot) {
                            KD_GLOBAL uint32_t *p = (leafm >> (j0 + j)) & 1u ? ob : nb;
                            if (p) p[ps[j0 + j]] = sv[j];
                        }
                    }
                }
                if (chunk_stats && col < d) {
                    // child sums as differences of chunk prefix sums.  Wave w
                    // holds numbers [1024w, 1024w + 1024), thread t numbers
                    // 16t .. 16t+15.  Each thread sums its numbers, taking a
                    // record of its running sum at every cell start and split
                    // point; a DPP scan adds the sums of the wave's earlier
                    // threads to the records; after the barrier below, a record
                    // plus the totals of the earlier waves is the chunk prefix
                    // there.  Every record is an exact prefix (hi * 2^32 + lo),
                    // so differences of records are exact.
                    const uint32_t e0 = threadIdx.x * PER_THREAD;
                    VarSums a;
#pragma unroll
                    for (int qq = 0; qq < 4; qq++) {
                        const uint4 x4 = *reinterpret_cast<const uint4 *>(stage + e0 + 4 * qq);
                        const uint32_t xv[4] = {x4.x, x4.y, x4.z, x4.w};
#pragma unroll
                        for (int jj = 0; jj < 4; jj++) {
                            const int j = 4 * qq + jj;
                            if ((rmask >> j) & 1u) {
                                a.fold();
                                const uint32_t r = (rid[j >> 2] >> (8 * (j & 3))) & 0xffu;
                                pat[r][0] = a.s1;
                                pat[r][1] = a.hi;
                                pat[r][2] = a.lo;
                            }
                            a.add(e0 + j < tot ? maxvar_q32(xv[jj], shift) : 0);
                            if (j == 7) a.fold();
                        }
                    }
                    a.fold();
                    unsigned long long x[3] = {a.s1, a.hi, a.lo};
#pragma unroll
                    for (int i = 0; i < 3; i++) x[i] = wave_scan64(x[i]);
                    if (rmask) {
                        const unsigned long long ex[3] = {x[0] - a.s1, x[1] - a.hi, x[2] - a.lo};
                        for (uint32_t m = rmask; m; m &= m - 1) {
                            const int j = __builtin_ctz(m);
                            const uint32_t r = (rid[j >> 2] >> (8 * (j & 3))) & 0xffu;
#pragma unroll
                            for (int i = 0; i < 3; i++) pat[r][i] += ex[i];
                        }
                    }
                    if (l == WAVE - 1)
#pragma unroll
                        for (int i = 0; i < 3; i++) wtot[w][i] = x[i];
                }
                __syncthreads();
                if (chunk_stats && col < d) {
                    // chunk prefix at record r (position pos): the record plus
                    // the totals of the waves before pos's wave; the chunk end
                    // (r = 2K) is the sum of all wave totals
                    auto prefix = [&](uint32_t r, uint32_t pos, int i) {
                        unsigned long long v = r < 2 * K ? pat[r][i] : 0ull;
                        const uint32_t wr = r < 2 * K ? pos / (WAVE * PER_THREAD) : uint32_t(NW);
                        for (uint32_t ww = 0; ww < wr; ww++) v += wtot[ww][i];
                        return v;
                    };
                    for (uint32_t s2 = threadIdx.x; s2 < 2 * K; s2 += NT) {
                        const uint32_t k = s2 >> 1, side = s2 & 1u;
                        if ((C.flags[k] & RES_SPLIT) &&
                            !(C.flags[k] & (side ? RES_RIGHT_LEAF : RES_LEFT_LEAF))) {
                            unsigned long long *st =
                                T.stats[nxt] + (uint64_t(2 * C.li[k] + side) * d + col) * 3;
                            const uint32_t mid = C.start[k] + C.nl[k];
                            const uint32_t r0 = 2 * k + side, p0 = side ? mid : C.start[k];
                            const uint32_t r1 = r0 + 1, p1 = side ? C.start[k + 1] : mid;
                            // sum q^2 = (hi1 - hi0) * 2^32 + (lo1 - lo0); the
                            // parts may differ in sign, the value is exact
                            const __int128 q2 =
                                (__int128)(long long)(prefix(r1, p1, 1) - prefix(r0, p0, 1)) *
                                    ((__int128)1 << 32) +
                                (__int128)(long long)(prefix(r1, p1, 2) - prefix(r0, p0, 2));
                            st[0] = prefix(r1, p1, 0) - prefix(r0, p0, 0);
                            st[1] = (unsigned long long)(q2 >> 32);
                            st[2] = (unsigned long long)(q2 & 0xffffffff);
                        }
                    }
                }
            }
            __syncthreads();
        }
    }
}

// ------------------------------------------------------------ kernels: small-cell subtrees

// A chunk of small cells is finished in one pass: every remaining level of
// its cells is split in LDS, and only the order of the chunk's numbers moves
// between levels (the keys of each level are read through it).  The columns
// and the permutation are moved once, at the end, to the outputs (points in
// leaves) or to the working buffers of the level where splitting stops.
// Splits below the current level go to records that the per-level loop
// reads when it reaches them, so node ids stay breadth-first.

// Active sub-cells of a chunk at one sub-depth (slot ranges, key coordinate,
// record link), their splits once found, and the numbering of their
// children.  CH >= SC: room for every child of SC sub-cells.
template <int SC, int CH>
struct SubTable {
    uint32_t start[CH], end[CH], dim[CH], rec[CH];  // rec: record index + 1
    uint32_t split[SC], nl[SC], flags[SC], base[SC];
    uint32_t kid[SC][2];  // child number at the next sub-depth, NONE for a leaf
    uint32_t wide[4];     // sub-cells above WAVE_CELL_MAX points (at most 3)
    uint32_t count, nwide;
};
constexpr uint32_t SEG_LEAF = 0xffu;
template <bool MAXVAR>
constexpr int subtree_cells() { return MAXVAR ? 80 : 64; }

template <int SC, int CH>
__device__ __forceinline__ void sub_result(const Ctx &c, uint32_t depth, uint32_t max_depth,
                                           SubTable<SC, CH> &A, uint32_t q, uint32_t m,
                                           uint32_t lt, uint32_t le) {
    CellRes r{};
    finish_cell(c, depth, max_depth, A.end[q] - A.start[q], r, m, lt, le);
    A.split[q] = r.split;
    A.nl[q] = r.nl;
    A.flags[q] = r.flags;
}

// SUBSET with equal subsets, inside a subtree chunk: the candidates of all
// active sub-cells, in groups whose subset bounds B[0..S] and medians
// med[0..S) fit `dyn` (dyn_words words).  Equal subsets depend only on a
// sub-cell's size, so no level-wide rank is needed.  Subsets of at most
// RANK_MAX points find their lower median by counting ranks (ties broken by
// slot, the stable order), larger ones by a wave radix select; the weighted
// mean is one thread per sub-cell in subset order; then the counts around the
// candidate and the tie rule, one wave per sub-cell.
template <int SC, int CH>
__device__ void subtree_subset(const Ctx &c, uint32_t depth, uint32_t max_depth, const uint32_t *keys,
                               const uint8_t *seg, SubTable<SC, CH> &A, uint32_t *dyn,
                               uint32_t dyn_words, uint32_t (*h)[NBINS]) {
    const uint32_t S = c.S, stride = 2 * S + 1, nq = A.count;
    const uint32_t G = dyn_words / stride;  // at least 1: dyn_words >= 2S + 1
    const int w = wave(), l = lane();
    for (uint32_t q0 = 0; q0 < nq; q0 += G) {
        const uint32_t g1 = min(G, nq - q0);
        for (uint32_t g = w; g < g1; g += NW) {
            const uint32_t n = A.end[q0 + g] - A.start[q0 + g];
            uint32_t *B = dyn + g * stride;
            for (uint32_t r = l; r <= S; r += WAVE) B[r] = uint32_t((uint64_t(r) * n) / S);
        }
        __syncthreads();
        const uint32_t e0 = A.start[q0], e1 = A.end[q0 + g1 - 1];
        for (uint32_t e = e0 + threadIdx.x; e < e1; e += NT) {
            const uint32_t q = seg[e];
            if (q == SEG_LEAF || q < q0 || q >= q0 + g1) continue;
            const uint32_t g = q - q0, i = e - A.start[q];
            const uint32_t *B = dyn + g * stride;
            const uint32_t lo = last_at_most(B, S, i);
            const uint32_t b = B[lo], m = B[lo + 1] - b;
            if (m > RANK_MAX) continue;
            const uint32_t s0 = A.start[q] + b, u = keys[px(e)];
            if (rank_in_subset(keys, s0, m, u, e) == (m - 1) / 2) dyn[g * stride + S + 1 + lo] = u;
        }
        for (uint32_t g = w; g < g1; g += NW) {
            const uint32_t *B = dyn + g * stride;
            uint32_t *med = dyn + g * stride + S + 1;
            for (uint32_t r0 = 0; r0 < S; r0 += WAVE) {
                const uint32_t r = r0 + l;
                bool large = false;
                if (r < S) {
                    const uint32_t m = B[r + 1] - B[r];
                    if (m == 0) med[r] = NONE;
                    large = m > RANK_MAX;
                }
                for (unsigned long long mask = __ballot(large); mask; mask &= mask - 1) {
                    const uint32_t rr = r0 + uint32_t(__builtin_ctzll(mask));
                    const uint32_t b = B[rr], m = B[rr + 1] - b;
                    const uint32_t v = wave_select(keys, A.start[q0 + g] + b, m, (m - 1) / 2, h[w]);
                    if (l == 0) med[rr] = v;
                }
            }
        }
        __syncthreads();
        for (uint32_t g = threadIdx.x; g < g1; g += NT) {
            const uint32_t q = q0 + g;
            A.split[q] = subset_mean(dyn + g * stride, dyn + g * stride + S + 1, S,
                                     A.end[q] - A.start[q]);
        }
        __syncthreads();
        for (uint32_t g = w; g < g1; g += NW) {
            const uint32_t q = q0 + g, s0 = A.start[q], nk = A.end[q] - s0, m = A.split[q];
            uint32_t a = 0, b = 0;
            for (uint32_t i = l; i < nk; i += WAVE) {
                const uint32_t u = keys[px(s0 + i)];
                a += u < m;
                b += u <= m;
            }
            a = uint32_t(wave_sum64(a));
            b = uint32_t(wave_sum64(b));
            if (l == 0) sub_result(c, depth, max_depth, A, q, m, a, b);
        }
        __syncthreads();
    }
}

template <int RULE, bool MAXVAR>
// Workgroups per CU: three (LDS about 53 KB with the largest-variance key and
// 80 chunk cells; a few spilled registers), two for the FOURIER moments with
// that key and for SUBSET.
__global__ __launch_bounds__(NT, MAXVAR ? (RULE == KD_SPLIT_EXACT ? 3 : 2)
                                        : (RULE == KD_SPLIT_SUBSET ? 2 : 3)) void k_subtree(
    Ctx c, uint32_t level) {
    constexpr int SC = subtree_cells<MAXVAR>();
    constexpr int CH = MAXVAR ? 2 * SC : SC;
    struct SelectScratch {
        uint32_t h[NW][NBINS];
        unsigned long long sh64[NW * 2 * FCHUNK];
        long long mom[NW][RULE == KD_SPLIT_FOURIER ? 2 * FOURIER_JMAX : 1];
    };
    union ScratchOrInv {
        SelectScratch sel;
        uint16_t inv[TILE];  // final slot of each chunk number
    };
    __shared__ __attribute__((aligned(16))) uint32_t keys[PADDED];  // keys of a sub-depth; staged values
    __shared__ __attribute__((aligned(16))) ScratchOrInv lds;
    __shared__ __attribute__((aligned(16))) uint8_t seg[TILE];   // sub-cell of each slot, SEG_LEAF in a leaf
    __shared__ __attribute__((aligned(16))) uint8_t seg0[TILE];  // chunk cell of each slot
    __shared__ __attribute__((aligned(16))) uint16_t lp[TILE];   // chunk number held by each slot
    __shared__ ChunkLds<SC> C;
    __shared__ SubTable<SC, CH> Q[2];
    __shared__ uint32_t sh[2 * NW + 1], s3[4];
    static_assert(CH < int(SEG_LEAF), "child numbers fit a byte below SEG_LEAF");
    // SUBSET: subset bounds and medians (dynamic LDS of max(4096, 2S + 1) words)
    extern __shared__ uint32_t dyn_lds[];
    const uint32_t dyn_words = RULE == KD_SPLIT_SUBSET ? max(SUBSET_DYN_WORDS, 2 * c.S + 1) : 0u;
    uint32_t(*const h)[NBINS] = lds.sel.h;
    unsigned long long *const sh64 = lds.sel.sh64;
    auto &mom = lds.sel.mom;
    const uint32_t cur = level & 1;
    const int w = wave(), l = lane();
    const LevelInfo I = c.info[level];
    const uint32_t ncells = I.num_cells;
    const uint32_t nbuckets = (I.points - I.big_points - I.resolved + TILE - 1) / TILE;
    for (uint32_t b = blockIdx.x; b < nbuckets; b += gridDim.x) {
        uint32_t pos = c.bucket_first[b];
        const uint32_t v1 = (b + 1) * uint32_t(TILE);
        for (;;) {
            if (w == 0) form_chunk(c, cur, ncells, pos, v1, C);
            __syncthreads();
            const uint32_t K = C.count, tot = C.total;
            pos = C.next;
            const uint32_t tr = __builtin_amdgcn_readfirstlane(C.tree);
            __syncthreads();
            if (K == 0) break;
            const KD_CONST TreeDesc &T = cref(&c.trees[tr]);
            const uint32_t d = T.d, n = T.n;
            for (uint32_t k = w; k < K; k += NW)
                for (uint32_t e = C.start[k] + l; e < C.start[k + 1]; e += WAVE) {
                    seg[e] = uint8_t(k);
                    seg0[e] = uint8_t(k);
                    lp[e] = uint16_t(e);
                }
            for (uint32_t k = threadIdx.x; k < K; k += NT) {
                Q[0].start[k] = C.start[k];
                Q[0].end[k] = C.start[k + 1];
                Q[0].dim[k] = C.dim[k];
                Q[0].rec[k] = 0;
            }
            if (threadIdx.x == 0) {
                Q[0].count = K;
                Q[0].nwide = C.nwide;
                for (int q = 0; q < 4; q++) Q[0].wide[q] = C.wide[q];
            }
            __syncthreads();
            uint32_t qa = 0, depth = level;  // depth of the sub-cells in Q[qa]
            for (;;) {
                SubTable<SC, CH> &A = Q[qa];
                SubTable<SC, CH> &N = Q[qa ^ 1];
                const uint32_t nq = A.count;
                // keys of the active slots, read through the numbers they hold;
                // every load is issued (no branch), idle slots all reading
                // the chunk's first place
                {
                    const KD_GLOBAL uint32_t *cols = gp(T.cols[cur]);
                    const uint64_t idle = C.off[seg0[0]];
                    uint32_t u[PER_THREAD];
                    bool live[PER_THREAD];
#pragma unroll
                    for (int jj = 0; jj < PER_THREAD; jj++) {
                        const uint32_t e = jj * NT + threadIdx.x, ec = min(e, tot - 1);
                        const uint32_t q = seg[ec], o = lp[ec];
                        live[jj] = e < tot && q != SEG_LEAF;
                        const uint64_t at = uint64_t(A.dim[live[jj] ? q : 0u]) * n + C.off[seg0[o]] + o;
                        u[jj] = cols[live[jj] ? at : idle];
                    }
#pragma unroll
                    for (int jj = 0; jj < PER_THREAD; jj++) u[jj] = live[jj] ? u[jj] : 0u;
#pragma unroll
                    for (int jj = 0; jj < PER_THREAD; jj++) {
                        const uint32_t e = jj * NT + threadIdx.x;
                        if (e < tot) keys[px(e)] = key_of_bits(u[jj]);
                    }
                }
                __syncthreads();
                // split of every active sub-cell: wide ones by the workgroup,
                // the others one per wave (SUBSET: all of them in groups)
                if constexpr (RULE == KD_SPLIT_SUBSET) {
                    subtree_subset(c, depth, T.max_depth, keys, seg, A, dyn_lds, dyn_words, h);
                } else {
                    for (uint32_t qq = 0; qq < A.nwide; qq++) {
                        const uint32_t q = A.wide[qq];
                        uint32_t m, lt, le;
                        block_candidate<RULE>(c, depth, keys, A.start[q], A.end[q] - A.start[q],
                                              0u, h, sh, s3, sh64, mom[0], nullptr, m, lt, le);
                        if (threadIdx.x == 0) sub_result(c, depth, T.max_depth, A, q, m, lt, le);
                    }
                    for (uint32_t q = w; q < nq; q += NW) {
                        const uint32_t s0 = A.start[q], nk = A.end[q] - s0;
                        if (nk > WAVE_CELL_MAX) continue;
                        uint32_t m, lt, le;
                        wave_candidate<RULE>(c, keys, s0, nk, h[w], mom[w], m, lt, le);
                        if (l == 0) sub_result(c, depth, T.max_depth, A, q, m, lt, le);
                    }
                }
                __syncthreads();
                // children that are split again, numbered in slot order; their
                // records (wave 0)
                if (w == 0) {
                    uint32_t run = 0;
                    for (uint32_t q0 = 0; q0 < nq; q0 += WAVE) {
                        const uint32_t q = q0 + l;
                        bool go0 = false, go1 = false;
                        if (q < nq) {
                            const uint32_t f = A.flags[q];
                            go0 = (f & RES_SPLIT) && !(f & RES_LEFT_LEAF);
                            go1 = (f & RES_SPLIT) && !(f & RES_RIGHT_LEAF);
                        }
                        const uint32_t cnt = uint32_t(go0) + uint32_t(go1);
                        const uint32_t incl = wave_incl_scan(cnt);
                        const uint32_t id0 = run + incl - cnt;
                        if (q < nq) {
                            A.kid[q][0] = go0 ? id0 : NONE;
                            A.kid[q][1] = go1 ? id0 + uint32_t(go0) : NONE;
                        }
                        run += wave_bcast(incl, WAVE - 1);
                    }
                    if (l == 0) {
                        // more than SC children: they stop here and are split at
                        // their own level (MAXVAR: with their key coordinate in
                        // a record)
                        const bool go_on = run > 0 && run <= uint32_t(SC);
                        const bool need = run > 0 && (go_on || MAXVAR);
                        uint32_t base = 0;
                        bool ok = false;
                        if (need) {
                            base = atomicAdd(c.rec_count, run);
                            ok = uint64_t(base) + run <= c.rec_cap;
                            if (!ok) c.ts[tr].status = KD_ECAPACITY;
                        }
                        s3[0] = run;
                        s3[1] = base;
                        s3[2] = (go_on && ok ? 1u : 0u) | (ok ? 2u : 0u);
                    }
                }
                __syncthreads();
                const uint32_t nact = s3[0], rbase = s3[1];
                const bool go_on = s3[2] & 1u, recs = s3[2] & 2u;
                // results of the sub-cells with their child links; the table
                // of the children
                for (uint32_t q = threadIdx.x; q < nq; q += NT) {
                    uint32_t link[2] = {0u, 0u};
                    for (int sd = 0; sd < 2; sd++) {
                        const uint32_t k = A.kid[q][sd];
                        if (k == NONE || !recs) continue;
                        link[sd] = (go_on ? REC_RESOLVED : 0u) | (rbase + k + 1);
                        N.start[k] = sd ? A.start[q] + A.nl[q] : A.start[q];
                        N.end[k] = sd ? A.end[q] : A.start[q] + A.nl[q];
                        N.rec[k] = rbase + k + 1;
                        N.dim[k] = (depth + 1) % d;
                    }
                    if (depth == level) {
                        CellRes r{};
                        r.dim = A.dim[q];
                        r.split = A.split[q];
                        r.nl = A.nl[q];
                        r.flags = A.flags[q];
                        r.rank = (A.end[q] - A.start[q] - 1) / 2;
                        r.crec[0] = link[0];
                        r.crec[1] = link[1];
                        c.res[C.ci[q]] = r;
                    } else {
                        c.subrec[A.rec[q] - 1] =
                            SubRec{A.dim[q], A.split[q], A.nl[q], A.flags[q], {link[0], link[1]}};
                    }
                }
                // stable partition of every sub-cell: each slot's new place,
                // and what goes there (its number and child)
                {
                    const uint32_t e0 = threadIdx.x * PER_THREAD;
                    const uint4 sq = *reinterpret_cast<const uint4 *>(seg + e0);
                    const uint32_t sw[4] = {sq.x, sq.y, sq.z, sq.w};
                    const uint4 lq0 = *reinterpret_cast<const uint4 *>(lp + e0);
                    const uint4 lq1 = *reinterpret_cast<const uint4 *>(lp + e0 + 8);
                    const uint32_t lw[8] = {lq0.x, lq0.y, lq0.z, lq0.w, lq1.x, lq1.y, lq1.z, lq1.w};
                    uint32_t nleft = 0, fl = 0;
#pragma unroll
                    for (int j = 0; j < PER_THREAD; j++) {
                        const uint32_t e = e0 + j, q = (sw[j >> 2] >> (8 * (j & 3))) & 0xffu;
                        if (e < tot && q != SEG_LEAF && keys[px(e)] <= A.split[q]) {
                            nleft++;
                            fl |= 1u << j;
                        }
                    }
                    uint32_t all;
                    const uint32_t lbase = block_excl_scan(nleft, sh, &all);
                    uint32_t run = lbase;
#pragma unroll
                    for (int j = 0; j < PER_THREAD; j++) {
                        const uint32_t e = e0 + j, q = (sw[j >> 2] >> (8 * (j & 3))) & 0xffu;
                        if (e < tot && q != SEG_LEAF && e == A.start[q]) A.base[q] = run;
                        run += (fl >> j) & 1u;
                    }
                    __syncthreads();
                    uint32_t mv[PER_THREAD];
                    run = lbase;
#pragma unroll
                    for (int j = 0; j < PER_THREAD; j++) {
                        const uint32_t e = e0 + j, q = (sw[j >> 2] >> (8 * (j & 3))) & 0xffu;
                        const uint32_t num = (lw[j >> 1] >> (16 * (j & 1))) & 0xffffu;
                        uint32_t dd = e, ns = SEG_LEAF;
                        if (e < tot && q != SEG_LEAF) {
                            const bool left = (fl >> j) & 1u;
                            const uint32_t s = A.start[q], lr = run - A.base[q];
                            dd = left ? s + lr : s + A.nl[q] + (e - s) - lr;
                            const uint32_t k = A.kid[q][left ? 0 : 1];
                            ns = k == NONE ? SEG_LEAF : k;
                        }
                        mv[j] = dd | (num << 12) | (ns << 24);
                        run += (fl >> j) & 1u;
                    }
                    __syncthreads();
#pragma unroll
                    for (int j = 0; j < PER_THREAD; j++) {
                        if (e0 + j < tot) {
                            const uint32_t dd = mv[j] & 0xfffu;
                            lp[dd] = uint16_t((mv[j] >> 12) & 0xfffu);
                            seg[dd] = uint8_t(mv[j] >> 24);
                        }
                    }
                    __syncthreads();
                }
                if (MAXVAR && recs) {
                    // key coordinate of every child: the largest fixed-point
                    // variance over the columns, ties to the lowest.  Every
                    // child is a contiguous run of slots.  One wave takes a
                    // sub-cell q: its lanes stride over the slots of one
                    // child and the exact sums of each column are wave
                    // reductions (no workgroup barrier between columns).
                    // When both children go on, only the smaller is summed
                    // from its points; the other's sums are q's minus it,
                    // exact integers either way.  Every child's sums are
                    // kept by record for the next sub-depth.  The place of
                    // each slot's point is staged in the key buffer (free
                    // until the next sub-depth's keys).
                    const int shift = maxvar_shift(c.ts[tr].maxabs);
                    const uint64_t rstride = uint64_t(c.recstats_stride) * 3;
                    for (uint32_t e = threadIdx.x; e < tot; e += NT) {
                        const uint32_t o = lp[e];
                        keys[e] = C.off[seg0[o]] + o;
                    }
                    __syncthreads();
                    // (sub-cell, column) items over the waves, column by
                    // column: the waves share a column's lines in the caches,
                    // and even one sub-cell keeps every wave busy
                    for (uint32_t it = w; it < nq * d; it += NW) {
                        const uint32_t col = it / nq, q = it - col * nq;
                        const uint32_t k0 = A.kid[q][0], k1 = A.kid[q][1];
                        if (k0 == NONE && k1 == NONE) continue;
                        uint32_t ka = k0 != NONE ? k0 : k1, kb = NONE;
                        if (k0 != NONE && k1 != NONE) {
                            const bool first = N.end[k0] - N.start[k0] <= N.end[k1] - N.start[k1];
                            ka = first ? k0 : k1;
                            kb = first ? k1 : k0;
                        }
                        const uint32_t s0 = N.start[ka], s1 = N.end[ka];
                        const KD_GLOBAL uint32_t *src = gp(T.cols[cur] + uint64_t(col) * n);
                        // q's own sums of this column (needed when kb is
                        // derived), requested before the gathers
                        unsigned long long pq[3] = {0ull, 0ull, 0ull};
                        if (kb != NONE) {
                            const unsigned long long *ps;
                            if (depth == level) {
                                const uint32_t ci = C.ci[q], link = c.cell_rec[cur][ci];
                                ps = link ? c.recstats + uint64_t((link & REC_INDEX) - 1) * rstride
                                          : T.stats[cur] + uint64_t(c.cells[cur][ci].slot) * d * 3;
                            } else {
                                ps = c.recstats + uint64_t(A.rec[q] - 1) * rstride;
                            }
#pragma unroll
                            for (int i = 0; i < 3; i++) pq[i] = ps[col * 3 + i];
                        }
                        VarSums a;
                        // up to eight loads in flight per lane, at most eight
                        // values between folds (no wrap): each batch of B * WAVE
                        // slots reads its places first and then issues every
                        // load, the slots past the child's end reading its last
                        // place again and adding zero (no branch: a load under
                        // a condition is issued only after the others
                        // complete).  Batches of eight while more than four
                        // rows of the wave remain, then one of four, two or one
                        // (most children hold 129 to 512 points).
                        auto batch = [&](auto bc, uint32_t eb) {
                            constexpr int B = decltype(bc)::value;
                            uint32_t kx[B], xv[B];
#pragma unroll
                            for (int j = 0; j < B; j++) kx[j] = keys[min(eb + j * WAVE + l, s1 - 1)];
#pragma unroll
                            for (int j = 0; j < B; j++) xv[j] = src[kx[j]];
#pragma unroll
                            for (int j = 0; j < B; j++) {
                                const int q = maxvar_q32(xv[j], shift);
                                a.add(eb + j * WAVE + l < s1 ? q : 0);
                            }
                            a.fold();
                        };
                        uint32_t eb = s0;
                        for (; eb < s1 && s1 - eb > 4 * WAVE; eb += 8 * WAVE)
                            batch(std::integral_constant<int, 8>{}, eb);
                        if (eb < s1) {
                            const uint32_t rem = s1 - eb;
                            if (rem > 2 * WAVE) batch(std::integral_constant<int, 4>{}, eb);
                            else if (rem > WAVE) batch(std::integral_constant<int, 2>{}, eb);
                            else batch(std::integral_constant<int, 1>{}, eb);
                        }
                        const unsigned long long v[3] = {wave_sum64(a.s1), wave_sum64(a.hi),
                                                         wave_sum64(a.lo)};
                        if (l == 0) {
                            unsigned long long *sa = c.recstats + uint64_t(N.rec[ka] - 1) * rstride;
#pragma unroll
                            for (int i = 0; i < 3; i++) sa[col * 3 + i] = v[i];
                            if (kb != NONE) {
                                // q's own sums minus ka's
                                unsigned long long *sb =
                                    c.recstats + uint64_t(N.rec[kb] - 1) * rstride;
#pragma unroll
                                for (int i = 0; i < 3; i++) sb[col * 3 + i] = pq[i] - v[i];
                            }
                        }
                    }
                    __syncthreads();
                    // each child's coordinate from its sums
                    for (uint32_t k = threadIdx.x; k < nact; k += NT) {
                        const unsigned long long *sk = c.recstats + uint64_t(N.rec[k] - 1) * rstride;
                        const __int128 nc = N.end[k] - N.start[k];
                        __int128 best = -1;
                        uint32_t bd = 0;
                        for (uint32_t c0 = 0; c0 < d; c0 += 8) {
                            // eight columns' sums requested at once
                            unsigned long long x[8][3];
#pragma unroll
                            for (int j = 0; j < 8; j++)
#pragma unroll
                                for (int i = 0; i < 3; i++)
                                    x[j][i] = sk[min(c0 + j, d - 1) * 3 + i];
#pragma unroll
                            for (int j = 0; j < 8; j++) {
                                if (c0 + j >= d) break;
                                const __int128 S1 = (long long)x[j][0];
                                const __int128 S2 =
                                    (__int128)(long long)x[j][1] * ((__int128)1 << 32) +
                                    (__int128)(long long)x[j][2];
                                const __int128 V = nc * S2 - S1 * S1;
                                if (V > best) {
                                    best = V;
                                    bd = c0 + j;
                                }
                            }
                        }
                        N.dim[k] = bd;
                        // children that stop here take their coordinate along
                        if (!go_on) c.subrec[rbase + k] = SubRec{bd, 0u, 0u, 0u, {0u, 0u}};
                    }
                    __syncthreads();
                }
                if (!go_on) break;
                // the children become the next sub-depth
                if (w == 0) {
                    uint32_t nw = 0;
                    for (uint32_t k0 = 0; k0 < nact; k0 += WAVE) {
                        const uint32_t k = k0 + l;
                        const bool wide = k < nact && N.end[k] - N.start[k] > WAVE_CELL_MAX;
                        const unsigned long long bm = __ballot(wide);
                        if (wide) N.wide[nw + __popcll(bm & ((1ull << l) - 1))] = k;
                        nw += uint32_t(__popcll(bm));
                    }
                    if (l == 0) {
                        N.count = nact;
                        N.nwide = nw;
                    }
                }
                __syncthreads();
                qa ^= 1;
                depth++;
            }
            // the final move: every column and the permutation, from the
            // numbers' places to their slots' places; slots in a leaf go to the
            // outputs, the others to the working buffers of the level below
            // the last sub-depth
            for (uint32_t e = threadIdx.x; e < tot; e += NT) lds.inv[lp[e]] = uint16_t(e);
            __syncthreads();
            const uint32_t op = (depth + 1) & 1;
            uint32_t ps[PER_THREAD], leafm = 0;
#pragma unroll
            for (int jj = 0; jj < PER_THREAD; jj++) {
                const uint32_t e = jj * NT + threadIdx.x;
                ps[jj] = 0;
                if (e < tot) {
                    ps[jj] = C.off[seg0[e]] + e;  // place of number e, and of slot e
                    if (seg[e] == SEG_LEAF) leafm |= 1u << jj;
                }
            }
            uint32_t vn[PER_THREAD];
            {
                const KD_GLOBAL uint32_t *src = gp(T.cols[cur]);
#pragma unroll
                for (int jj = 0; jj < PER_THREAD; jj++)
                    vn[jj] = src[ps[jj]];  // place 0 where the slot is unused
            }
            for (uint32_t col = 0; col <= d; col++) {
                uint32_t v[PER_THREAD];
#pragma unroll
                for (int jj = 0; jj < PER_THREAD; jj++) v[jj] = vn[jj];
                if (col < d) {
                    const KD_GLOBAL uint32_t *src =
                        gp(col + 1 == d ? T.perm[cur] : T.cols[cur] + uint64_t(col + 1) * n);
#pragma unroll
                    for (int jj = 0; jj < PER_THREAD; jj++)
                        vn[jj] = src[ps[jj]];
                }
                // staged at the slot's number; slots past the chunk at their
                // own place, which no number uses (no branch)
#pragma unroll
                for (int j0 = 0; j0 < PER_THREAD; j0 += 8) {
                    uint32_t dd[8];
#pragma unroll
                    for (int jj = 0; jj < 8; jj++) dd[jj] = lds.inv[(j0 + jj) * NT + threadIdx.x];
#pragma unroll
                    for (int jj = 0; jj < 8; jj++) {
                        const uint32_t e = (j0 + jj) * NT + threadIdx.x;
                        keys[e < tot ? dd[jj] : e] = v[j0 + jj];
                    }
                }
                __syncthreads();
                KD_GLOBAL uint32_t *nb = gp(col == d ? T.perm[op] : T.cols[op] + uint64_t(col) * n);
                KD_GLOBAL uint32_t *ob =
                    col == d ? gp(T.out_perm)
                             : (T.pts_out ? gp(T.pts_out + uint64_t(col) * n) : nullptr);
                uint32_t sv[PER_THREAD];
#pragma unroll
                for (int jj = 0; jj < PER_THREAD; jj++) sv[jj] = keys[jj * NT + threadIdx.x];
#pragma unroll
                for (int jj = 0; jj < PER_THREAD; jj++) {
                    const uint32_t e = jj * NT + threadIdx.x;
                    if (e < tot) {
                        KD_GLOBAL uint32_t *p = (leafm >> jj) & 1u ? ob : nb;
                        if (p) p[ps[jj]] = sv[jj];
                    }
                }
                __syncthreads();
            }
        }
    }
}

// ------------------------------------------------------------ kernels: emit

__device__ __forceinline__ void emit_counts(const Ctx &c, uint32_t level, uint32_t ci,
                                            uint32_t ncells, uint32_t cnt[EMIT_COUNTERS]) {
    for (int k = 0; k < EMIT_COUNTERS; k++) cnt[k] = 0;
    if (ci >= ncells) return;
    const Cell cl = c.cells[level & 1][ci];
    const CellRes r = c.res[ci];
    if (!(r.flags & RES_SPLIT)) {
        cnt[7] = 1;
        return;
    }
    cnt[0] = 1;
    cnt[6] = cl.end - cl.begin;
    const uint32_t sz[2] = {r.nl, cl.end - cl.begin - r.nl};
    const uint32_t leaf[2] = {r.flags & RES_LEFT_LEAF, r.flags & RES_RIGHT_LEAF};
    for (int s = 0; s < 2; s++) {
        if (leaf[s]) continue;
        cnt[1]++;
        cnt[3] += sz[s];
        if (r.crec[s] & REC_RESOLVED) cnt[8] += sz[s];
        if (sz[s] > uint32_t(SMALL_MAX)) {
            cnt[2] += (sz[s] + TILE - 1) / TILE;
            cnt[4] += sz[s];
            cnt[5]++;
        }
    }
}

__global__ __launch_bounds__(NT) void k_emit_sum(Ctx c, uint32_t level) {
    __shared__ uint32_t sh[NW + 1];
    const uint32_t ncells = c.info[level].num_cells;
    uint32_t cnt[EMIT_COUNTERS];
    emit_counts(c, level, blockIdx.x * NT + threadIdx.x, ncells, cnt);
    for (int k = 0; k < EMIT_COUNTERS; k++) {
        uint32_t tot;
        block_excl_scan(cnt[k], sh, &tot);
        if (threadIdx.x == 0) c.scan_tmp[blockIdx.x * EMIT_STRIDE + k] = tot;
    }
}

__global__ __launch_bounds__(NT) void k_emit_scan(Ctx c, uint32_t level, uint32_t nblocks) {
    __shared__ uint32_t sh[NW + 1];
    const uint32_t ncells = c.info[level].num_cells;
    uint32_t base[EMIT_COUNTERS] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (uint32_t b0 = 0; b0 < nblocks; b0 += NT) {
        const uint32_t b = b0 + threadIdx.x;
        for (int k = 0; k < EMIT_COUNTERS; k++) {
            const uint32_t v = b < nblocks ? c.scan_tmp[b * EMIT_STRIDE + k] : 0u;
            uint32_t tot;
            const uint32_t ex = block_excl_scan(v, sh, &tot);
            if (b < nblocks) c.scan_tmp[b * EMIT_STRIDE + k] = base[k] + ex;
            base[k] += tot;
        }
    }
    if (threadIdx.x < EMIT_COUNTERS)
        c.pre[uint64_t(ncells) * EMIT_STRIDE + threadIdx.x] = base[threadIdx.x];
    if (threadIdx.x == 0) {
        LevelInfo in{};
        in.num_cells = base[1];
        in.num_tiles = base[2];
        in.points = base[3];
        in.big_points = base[4];
        in.num_big = base[5];
        in.resolved = base[8];
        c.info[level + 1] = in;
    }
}

__global__ __launch_bounds__(NT) void k_emit_prefix(Ctx c, uint32_t level) {
    __shared__ uint32_t sh[NW + 1];
    const uint32_t ncells = c.info[level].num_cells;
    const uint32_t ci = blockIdx.x * NT + threadIdx.x;
    uint32_t cnt[EMIT_COUNTERS];
    emit_counts(c, level, ci, ncells, cnt);
    for (int k = 0; k < EMIT_COUNTERS; k++) {
        uint32_t tot;
        const uint32_t p =
            block_excl_scan(cnt[k], sh, &tot) + c.scan_tmp[blockIdx.x * EMIT_STRIDE + k];
        if (ci < ncells) c.pre[uint64_t(ci) * EMIT_STRIDE + k] = p;
    }
}

// Per tree: node-id base of the new children, next level's cell range and
// the tree's counters.
// pre: the prefix rows (row ci at pre + ci * stride; row ncells the totals).
__device__ __forceinline__ void emit_tree(const Ctx &c, uint32_t level, uint32_t t,
                                          const uint32_t *pre, uint32_t stride) {
    const uint32_t cur = level & 1, nxt = cur ^ 1;
    {
        TreeState &S = c.ts[t];
        const uint32_t f = S.first[cur], n = S.count[cur];
        S.nodes_base = S.num_nodes;
        if (n > 0) {
            const uint32_t *pf = pre + uint64_t(f) * stride;
            const uint32_t *pe = pre + uint64_t(f + n) * stride;
            const uint32_t splits = pe[0] - pf[0];
            S.split_base = pf[0];
            if (uint64_t(S.num_nodes) + 2ull * splits > c.trees[t].cap) S.status = KD_ECAPACITY;
            S.num_nodes += 2 * splits;
            S.first[nxt] = pf[1];
            S.count[nxt] = pe[1] - pf[1];
            S.point_levels += pe[6] - pf[6];
            S.unsplittable += pe[7] - pf[7];
            if (splits > 0) S.depth = level + 1;
        } else {
            S.count[nxt] = 0;
        }
        S.depth_first[level + 2] = S.num_nodes;
    }
}
__global__ void k_emit_trees(Ctx c, uint32_t level) {
    for (uint32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < c.ntrees;
         t += gridDim.x * blockDim.x)
        emit_tree(c, level, t, c.pre, EMIT_STRIDE);
}

// pre: the cell's prefix row.
__device__ __forceinline__ void emit_cell(const Ctx &c, uint32_t level, uint32_t ci,
                                          const uint32_t *pre) {
    const uint32_t cur = level & 1, nxt = cur ^ 1;
    const CellRes r = c.res[ci];
    if (!(r.flags & RES_SPLIT)) return;
    const Cell cl = c.cells[cur][ci];
    const KD_CONST TreeDesc &T = cref(&c.trees[cl.tree]);
    const TreeState &S = c.ts[cl.tree];
    const uint32_t left = S.nodes_base + 2 * (pre[0] - S.split_base);
    const uint32_t li = ci - S.first[cur];
    const uint32_t mid = cl.begin + r.nl;
    if (cl.node < T.cap) {
        T.node_child[cl.node] = int32_t(left);
        T.node_dim[cl.node] = r.dim;
        T.node_split[cl.node] = r.split;
        T.node_split_f[cl.node] = __uint_as_float(bits_of_key(r.split));
    }
    if (uint64_t(left) + 1 < T.cap) {
        T.node_begin[left] = cl.begin;
        T.node_end[left] = mid;
        T.node_begin[left + 1] = mid;
        T.node_end[left + 1] = cl.end;
    }
    // small cells resolved ahead stay out of the small-point numbering
    uint32_t slot = pre[1], tile = pre[2], big = pre[5], voff = pre[3] - pre[4] - pre[8];
    const uint32_t b[2] = {cl.begin, mid}, e[2] = {mid, cl.end};
    const uint32_t leaf[2] = {r.flags & RES_LEFT_LEAF, r.flags & RES_RIGHT_LEAF};
    for (int s = 0; s < 2; s++) {
        if (leaf[s]) continue;
        const uint32_t sz = e[s] - b[s];
        const bool isbig = sz > uint32_t(SMALL_MAX);
        const bool resolved = r.crec[s] & REC_RESOLVED;
        c.cells[nxt][slot] = Cell{b[s], e[s], left + s, tile, isbig ? big : NONE, 2 * li + s,
                                  cl.tree, resolved ? NONE : voff};
        c.cell_rec[nxt][slot] = r.crec[s];
        if (isbig) {
            c.big_list[big] = slot;
            big++;
            tile += (sz + TILE - 1) / TILE;
        } else if (!resolved) {
            mark_buckets(c, voff, sz, slot);
            voff += sz;
        }
        slot++;
    }
}
__global__ __launch_bounds__(NT) void k_emit_write(Ctx c, uint32_t level) {
    const uint32_t ncells = c.info[level].num_cells;
    const uint32_t ci = blockIdx.x * NT + threadIdx.x;
    if (ci < ncells) emit_cell(c, level, ci, c.pre + uint64_t(ci) * EMIT_STRIDE);
}

// The whole emit step in one workgroup of EMIT_NT threads (each thread takes
// EMIT_PER consecutive cells).  Up to EMIT_ONE_MAX cells: the counts and
// their prefix rows in LDS, the totals, the per-tree update, then the node
// records and next cells.  More cells (a level run in tail shape): the same
// in chunks of EMIT_ONE_MAX cells with the prefix rows in the workspace.
constexpr int EMIT_NT = 1024;
constexpr int EMIT_NW = EMIT_NT / WAVE;
constexpr uint32_t EMIT_ONE_MAX = 2048;
constexpr uint32_t EMIT_PER = EMIT_ONE_MAX / EMIT_NT;

// Exclusive scan over the workgroup of one value per thread and counter;
// swave: per-wave scratch.  Returns the totals in tot[].
__device__ __forceinline__ void emit_wg_scan(const uint32_t (&local)[EMIT_COUNTERS],
                                             uint32_t (&excl)[EMIT_COUNTERS],
                                             uint32_t (&tot)[EMIT_COUNTERS],
                                             uint32_t (*swave)[EMIT_COUNTERS]) {
    const int w = threadIdx.x / WAVE;
    uint32_t incl[EMIT_COUNTERS];
#pragma unroll
    for (int k = 0; k < EMIT_COUNTERS; k++) {
        incl[k] = wave_incl_scan(local[k]);
        if (lane() == WAVE - 1) swave[w][k] = incl[k];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < EMIT_COUNTERS; k++) {
        uint32_t before = 0, all = 0;
        for (int v = 0; v < EMIT_NW; v++) {
            const uint32_t t = swave[v][k];
            before += v < w ? t : 0u;
            all += t;
        }
        excl[k] = before + incl[k] - local[k];
        tot[k] = all;
    }
    __syncthreads();
}

__device__ void emit_chunked(const Ctx &c, uint32_t level, uint32_t ncells,
                             uint32_t (*swave)[EMIT_COUNTERS]) {
    uint32_t base[EMIT_COUNTERS] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (uint32_t b0 = 0; b0 < ncells; b0 += EMIT_ONE_MAX) {
        const uint32_t c0 = b0 + threadIdx.x * EMIT_PER;
        uint32_t cnt[EMIT_PER][EMIT_COUNTERS], local[EMIT_COUNTERS], excl[EMIT_COUNTERS],
            tot[EMIT_COUNTERS];
#pragma unroll
        for (uint32_t j = 0; j < EMIT_PER; j++) emit_counts(c, level, c0 + j, ncells, cnt[j]);
#pragma unroll
        for (int k = 0; k < EMIT_COUNTERS; k++) {
            local[k] = 0;
#pragma unroll
            for (uint32_t j = 0; j < EMIT_PER; j++) local[k] += cnt[j][k];
        }
        emit_wg_scan(local, excl, tot, swave);
#pragma unroll
        for (int k = 0; k < EMIT_COUNTERS; k++) {
            uint32_t run = base[k] + excl[k];
#pragma unroll
            for (uint32_t j = 0; j < EMIT_PER; j++) {
                if (c0 + j < ncells) c.pre[uint64_t(c0 + j) * EMIT_STRIDE + k] = run;
                run += cnt[j][k];
            }
            base[k] += tot[k];
        }
    }
    if (threadIdx.x < uint32_t(EMIT_COUNTERS))
        c.pre[uint64_t(ncells) * EMIT_STRIDE + threadIdx.x] = base[threadIdx.x];
    if (threadIdx.x == 0) {
        LevelInfo in{};
        in.num_cells = base[1];
        in.num_tiles = base[2];
        in.points = base[3];
        in.big_points = base[4];
        in.num_big = base[5];
        in.resolved = base[8];
        c.info[level + 1] = in;
    }
    __threadfence_block();
    __syncthreads();
    for (uint32_t t = threadIdx.x; t < c.ntrees; t += EMIT_NT)
        emit_tree(c, level, t, c.pre, EMIT_STRIDE);
    __threadfence_block();
    __syncthreads();
    for (uint32_t ci = threadIdx.x; ci < ncells; ci += EMIT_NT)
        emit_cell(c, level, ci, c.pre + uint64_t(ci) * EMIT_STRIDE);
}

__global__ __launch_bounds__(EMIT_NT) void k_emit_one(Ctx c, uint32_t level) {
    __shared__ uint32_t spre[(EMIT_ONE_MAX + 1) * EMIT_COUNTERS];
    __shared__ uint32_t swave[EMIT_NW][EMIT_COUNTERS];
    const uint32_t ncells = c.info[level].num_cells;
    if (ncells > EMIT_ONE_MAX) {
        emit_chunked(c, level, ncells, swave);
        return;
    }
    const uint32_t c0 = threadIdx.x * EMIT_PER;
    const int w = threadIdx.x / WAVE;
    uint32_t cnt[EMIT_PER][EMIT_COUNTERS];
#pragma unroll
    for (uint32_t j = 0; j < EMIT_PER; j++) emit_counts(c, level, c0 + j, ncells, cnt[j]);
    uint32_t local[EMIT_COUNTERS], incl[EMIT_COUNTERS];
#pragma unroll
    for (int k = 0; k < EMIT_COUNTERS; k++) {
        local[k] = 0;
#pragma unroll
        for (uint32_t j = 0; j < EMIT_PER; j++) local[k] += cnt[j][k];
        incl[k] = wave_incl_scan(local[k]);
        if (lane() == WAVE - 1) swave[w][k] = incl[k];
    }
    __syncthreads();
    if (threadIdx.x < uint32_t(EMIT_COUNTERS)) {
        const int k = threadIdx.x;
        uint32_t run = 0;
        for (int v = 0; v < EMIT_NW; v++) {
            const uint32_t t = swave[v][k];
            swave[v][k] = run;
            run += t;
        }
        spre[ncells * EMIT_COUNTERS + k] = run;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < EMIT_COUNTERS; k++) {
        uint32_t run = swave[w][k] + incl[k] - local[k];
#pragma unroll
        for (uint32_t j = 0; j < EMIT_PER; j++) {
            if (c0 + j < ncells) spre[(c0 + j) * EMIT_COUNTERS + k] = run;
            run += cnt[j][k];
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const uint32_t *tot = spre + ncells * EMIT_COUNTERS;
        LevelInfo in{};
        in.num_cells = tot[1];
        in.num_tiles = tot[2];
        in.points = tot[3];
        in.big_points = tot[4];
        in.num_big = tot[5];
        in.resolved = tot[8];
        c.info[level + 1] = in;
    }
    for (uint32_t t = threadIdx.x; t < c.ntrees; t += EMIT_NT)
        emit_tree(c, level, t, spre, EMIT_COUNTERS);
    __threadfence_block();
    __syncthreads();
#pragma unroll
    for (uint32_t j = 0; j < EMIT_PER; j++)
        if (c0 + j < ncells) emit_cell(c, level, c0 + j, spre + (c0 + j) * EMIT_COUNTERS);
}

// ------------------------------------------------------------ kernels: leaves

// Leaves in position order.  Leaves tile a tree's positions and each holds
// at least one point, so a leaf's index is the number of leaf starts before
// its first position: one bit per position, popcount prefix sums.
constexpr uint32_t LEAF_WPB = NT * 16;  // bitmap words per scan block

__device__ __forceinline__ uint32_t leaf_rank(const Ctx &c, uint64_t pos) {
    const uint64_t w = pos >> 5;
    const uint32_t below = c.leafbits[w] & ((1u << (pos & 31)) - 1u);
    return c.leafblk[w / LEAF_WPB] + c.leafpre[w] + uint32_t(__popc(below));
}

__global__ void k_leaf_mark(Ctx c) {
    const uint32_t t = blockIdx.y;
    const TreeState &S = c.ts[t];
    if (S.status != KD_OK) return;
    const KD_CONST TreeDesc &T = cref(&c.trees[t]);
    for (uint32_t k = blockIdx.x * NT + threadIdx.x; k < S.num_nodes; k += gridDim.x * NT) {
        if (T.node_child[k] < 0) {
            const uint64_t pos = T.pbase + T.node_begin[k];
            atomicOr(&c.leafbits[pos >> 5], 1u << (pos & 31));
        }
    }
}

// Per scan block of LEAF_WPB words: each word's exclusive prefix of set bits
// within the block, and the block's total.
__global__ __launch_bounds__(NT) void k_leaf_scan1(Ctx c, uint64_t words) {
    __shared__ uint32_t sh[NW + 1];
    const uint64_t w0 = uint64_t(blockIdx.x) * LEAF_WPB + uint64_t(threadIdx.x) * 16;
    uint32_t cnt[16], local = 0;
#pragma unroll
    for (int j = 0; j < 16; j++) {
        cnt[j] = w0 + j < words ? uint32_t(__popc(c.leafbits[w0 + j])) : 0u;
        local += cnt[j];
    }
    uint32_t tot;
    uint32_t run = block_excl_scan(local, sh, &tot);
#pragma unroll
    for (int j = 0; j < 16; j++) {
        if (w0 + j < words) c.leafpre[w0 + j] = run;
        run += cnt[j];
    }
    if (threadIdx.x == 0) c.leafblk[blockIdx.x] = tot;
}

// Exclusive prefix of the block totals (one workgroup).
__global__ __launch_bounds__(NT) void k_leaf_scan2(Ctx c, uint32_t nblocks) {
    __shared__ uint32_t sh[NW + 1];
    uint32_t base = 0;
    for (uint32_t b0 = 0; b0 < nblocks; b0 += NT) {
        const uint32_t b = b0 + threadIdx.x;
        const uint32_t v = b < nblocks ? c.leafblk[b] : 0u;
        uint32_t tot;
        const uint32_t ex = block_excl_scan(v, sh, &tot);
        if (b < nblocks) c.leafblk[b] = base + ex;
        base += tot;
    }
}

__global__ __launch_bounds__(NT) void k_leaf_write(Ctx c) {
    __shared__ unsigned long long sh64[NW];
    const uint32_t t = blockIdx.y;
    const TreeState &S = c.ts[t];
    if (S.status != KD_OK) return;
    const KD_CONST TreeDesc &T = cref(&c.trees[t]);
    const uint32_t first = leaf_rank(c, T.pbase);
    unsigned long long over = 0;
    for (uint32_t k = blockIdx.x * NT + threadIdx.x; k < S.num_nodes; k += gridDim.x * NT) {
        if (T.node_child[k] < 0) {
            const uint32_t f = leaf_rank(c, T.pbase + T.node_begin[k]) - first;
            T.leaf_node[f] = k;
            T.leaf_offsets[f] = T.node_begin[k];
            T.node_leaf[k] = f;
            over += (T.node_end[k] - T.node_begin[k]) > c.leaf_size;
        }
    }
    block_sum64n<1>(&over, sh64);
    if (threadIdx.x == 0 && over) atomicAdd(&c.ts[t].oversize, uint32_t(over));
}

__global__ void k_header(Ctx c) {
    for (uint32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < c.ntrees;
         t += gridDim.x * blockDim.x) {
        const TreeState &S = c.ts[t];
        const KD_CONST TreeDesc &T = cref(&c.trees[t]);
        const uint32_t leaves =
            S.status == KD_OK ? leaf_rank(c, T.pbase + T.n) - leaf_rank(c, T.pbase) : 0u;
        if (S.status == KD_OK) T.leaf_offsets[leaves] = T.n;
        kd_header h{};
        h.num_nodes = S.num_nodes;
        h.num_leaves = leaves;
        h.depth = S.depth;
        h.status = S.status;
        h.point_levels = S.point_levels;
        h.unsplittable = S.unsplittable;
        h.oversize = S.oversize;
        *T.hdr = h;
    }
}

// a9: leaf of each query by descent.
__global__ void k_query(const int32_t *child, const uint32_t *dim, const uint32_t *split,
                        const uint32_t *node_leaf, const float *q, uint64_t nq, uint64_t ldq,
                        uint32_t *out) {
    for (uint64_t i = blockIdx.x * uint64_t(NT) + threadIdx.x; i < nq;
         i += uint64_t(gridDim.x) * NT) {
        uint32_t node = 0;
        bool nan = false;
        // a valid tree is at most MAX_LEVELS deep; the bound also ends the
        // walk on a corrupt node array
        for (int step = 0; step <= MAX_LEVELS; step++) {
            const int32_t ch = child[node];
            if (ch < 0) break;
            const uint32_t b = __float_as_uint(q[uint64_t(dim[node]) * ldq + i]);
            if ((b & 0x7fffffffu) > 0x7f800000u) {
                nan = true;
                break;
            }
            node = uint32_t(ch) + (key_of_bits(b) > split[node] ? 1u : 0u);
        }
        out[i] = nan ? NONE : node_leaf[node];
    }
}

// ------------------------------------------------------------ host side

bool params_ok(const kd_params *p) {
    if (!p || p->leaf_size == 0 || p->num_subsets == 0 || p->num_subsets > MAX_SUBSETS)
        return false;
    if (p->key_rule > KD_KEY_MAXVAR || p->split_rule > KD_SPLIT_SUBSET) return false;
    if (p->split_rule == KD_SPLIT_FOURIER && (p->fourier_J == 0 || p->fourier_J > FOURIER_JMAX))
        return false;
    if (p->subset_pool && p->pool_entries == 0) return false;
    if (p->max_depth > MAX_LEVELS) return false;
    if (p->flags & ~uint32_t(KD_FLAG_LEVEL_BY_LEVEL)) return false;
    return true;
}

bool shape_ok(uint64_t n, uint32_t d) { return n > 0 && n <= 0xffffff00ull && d > 0 && d <= 4096; }

uint64_t default_capacity(uint64_t n, uint32_t leaf) { return 4 * ((n + leaf - 1) / leaf) + 64; }

// Depth cap for max_depth = 0: ten levels beyond the depth h of a balanced
// tree of n points with leaves of at most `leaf` points (leaf * 2^h >= n),
// at most 64.  Cells at the cap stay leaves (counted in hdr->oversize when
// they hold more than `leaf` points).
uint32_t default_depth(uint64_t n, uint32_t leaf) {
    uint32_t h = 0;
    while (h < 40 && (uint64_t(leaf) << h) < n) h++;
    return std::min<uint32_t>(64, h + 10);
}

uint64_t align256(uint64_t x) { return (x + 255) & ~uint64_t(255); }

struct Bump {
    uint64_t o = 0;
    uint64_t take(uint64_t bytes) {
        const uint64_t r = o;
        o = align256(o + bytes);
        return r;
    }
};

struct TreeLayout {
    uint64_t cols[2], perm[2], stats[2];
    uint64_t max_cells;
};

struct Layout {
    uint64_t cell_rec[2], subrec, rec_count, rec_cap, recstats, recstats_stride;
    uint64_t trees, ts, cells[2], res, big_list, tile_lt, tile_le, tile_mm, tile_cell, tiles, hist, mm, mom,
        bounds, med, pre, scan, buckets, segs, info, leafbits, leafpre, leafblk, total;
    uint64_t max_cells, max_tiles, max_big, scan_blocks, all_points, leaf_words, leaf_blocks;
    std::vector<TreeLayout> per_tree;
};

Layout plan(uint32_t T, const uint64_t *n, const uint32_t *d, const uint64_t *cap,
            const kd_params *p) {
    Layout L{};
    for (uint32_t t = 0; t < T; t++) {
        L.max_cells += n[t] / (uint64_t(p->leaf_size) + 1) + 1;
        L.max_tiles += n[t] / TILE + n[t] / (SMALL_MAX + 1) + 2;
        L.max_big += n[t] / (SMALL_MAX + 1) + 1;
    }
    L.scan_blocks = (L.max_cells + NT - 1) / NT;
    Bump B;
    L.trees = B.take(sizeof(TreeDesc) * T);
    L.ts = B.take(sizeof(TreeState) * T);
    for (int b = 0; b < 2; b++) L.cells[b] = B.take(L.max_cells * sizeof(Cell));
    for (int b = 0; b < 2; b++) L.cell_rec[b] = B.take(L.max_cells * 4);
    // records of cells resolved ahead: each is a node of its tree
    uint64_t caps = 0;
    for (uint32_t t = 0; t < T; t++) caps += cap[t];
    // records of splits found ahead: the subtree path (every rule but SUBSET
    // with a subset pool or the largest-variance key)
    const bool per_level = (p->flags & KD_FLAG_LEVEL_BY_LEVEL) ||
                           (p->split_rule == KD_SPLIT_SUBSET &&
                            (p->subset_pool != nullptr || p->key_rule == KD_KEY_MAXVAR));
    L.rec_cap = per_level ? 0 : std::min<uint64_t>(caps, REC_INDEX - 1);
    L.subrec = B.take(L.rec_cap * sizeof(SubRec));
    // largest-variance key on the subtree path: every record's per-coordinate
    // sums (the widest tree's dimension as the stride)
    L.recstats_stride = 0;
    if (p->key_rule == KD_KEY_MAXVAR && L.rec_cap)
        for (uint32_t t = 0; t < T; t++)
            L.recstats_stride = std::max<uint64_t>(L.recstats_stride, d[t]);
    L.recstats = B.take(L.rec_cap * L.recstats_stride * 3 * 8);
    L.rec_count = B.take(4);
    L.res = B.take(L.max_cells * sizeof(CellRes));
    L.big_list = B.take(L.max_big * 4);
    L.tile_lt = B.take(L.max_tiles * 4);
    L.tile_le = B.take(L.max_tiles * 4);
    L.tile_mm = B.take(L.max_tiles * 4);
    L.tile_cell = B.take(L.max_tiles * 4);
    L.tiles = B.take(L.max_tiles * sizeof(TileDesc));
    L.hist = B.take(L.max_big * BIG_BINS_MAX * 4);
    const bool fourier = p->split_rule == KD_SPLIT_FOURIER;
    const bool subset = p->split_rule == KD_SPLIT_SUBSET;
    L.mm = B.take(fourier ? L.max_big * 8 : 0);
    L.mom = B.take(fourier ? L.max_big * 2 * FOURIER_JMAX * 8 : 0);
    L.bounds = B.take(subset ? L.max_big * (p->num_subsets + 1) * 4 : 0);
    L.med = B.take(subset ? L.max_big * p->num_subsets * 4 : 0);
    L.pre = B.take((L.max_cells + 1) * EMIT_STRIDE * 4);
    L.scan = B.take((L.scan_blocks + 1) * EMIT_STRIDE * 4);
    uint64_t all_points = 0;
    for (uint32_t t = 0; t < T; t++) all_points += n[t];
    L.all_points = all_points;
    L.buckets = B.take((all_points / TILE + 2) * 4);
    // at most one large subset per SMALL_MAX + 1 points, and at most two
    // histogram workgroups per SMALL_MAX + 1 points (a subset of ns >
    // SMALL_MAX points has ceil(ns / SEG_CHUNK) <= 2 ns / (SMALL_MAX + 1)):
    // per subset 3 + NBINS + 1 words, two for workgroups and two for the
    // address of its first key
    L.segs = B.take(subset ? (all_points / (SMALL_MAX + 1) + 2) * 4 * (3 + NBINS + 1 + 2 + 2) + 256
                           : 0);
    L.info = B.take(sizeof(LevelInfo) * (MAX_LEVELS + 1));
    // one bit per position of every tree, plus the position after the last
    L.leaf_words = all_points / 32 + 1;
    L.leaf_blocks = (L.leaf_words + LEAF_WPB - 1) / LEAF_WPB;
    L.leafbits = B.take(L.leaf_words * 4);
    L.leafpre = B.take(L.leaf_words * 4);
    L.leafblk = B.take(L.leaf_blocks * 4);
    L.per_tree.resize(T);
    for (uint32_t t = 0; t < T; t++) {
        TreeLayout &tl = L.per_tree[t];
        tl.max_cells = n[t] / (uint64_t(p->leaf_size) + 1) + 1;
        for (int b = 0; b < 2; b++) tl.cols[b] = B.take(uint64_t(d[t]) * n[t] * 4);
        for (int b = 0; b < 2; b++) tl.perm[b] = B.take(n[t] * 4);
        for (int b = 0; b < 2; b++)
            tl.stats[b] = B.take(p->key_rule == KD_KEY_MAXVAR
                                     ? 2 * tl.max_cells * uint64_t(d[t]) * 3 * 8
                                     : 0);
    }
    L.total = B.o;
    return L;
}

TrigTables make_trig() {
    TrigTables T{};
    double f[26];
    f[0] = 1.0;
    for (int k = 1; k < 26; k++) {
        double v = 1.0;
        for (int i = 2; i <= k; i++) v *= double(i);
        f[k] = v;
    }
    for (int m = 0; m < 9; m++) {
        const float sg = (m % 2) ? -1.0f : 1.0f;
        T.s32[m] = sg * float(1.0 / f[2 * m + 1]);
        T.c32[m] = sg * float(1.0 / f[2 * m]);
    }
    for (int m = 0; m < 13; m++) {
        const double sg = (m % 2) ? -1.0 : 1.0;
        T.s64[m] = sg * (1.0 / f[2 * m + 1]);
        T.c64[m] = sg * (1.0 / f[2 * m]);
    }
    for (int j = 0; j < FOURIER_JMAX; j++) T.w[j] = 1.0 / double(2 * j + 1);
    return T;
}

uint32_t grid_for(uint64_t work, uint32_t cap = 65535u) {
    if (work == 0) return 1;
    return uint32_t(work < cap ? work : cap);
}

// roctx ranges on the host timeline (a profiler shows what each enqueue
// belongs to: the build, each level, each kernel class).
struct Range {
    explicit Range(const char *m) { roctxRangePushA(m); }
    ~Range() { roctxRangePop(); }
    Range(const Range &) = delete;
    Range &operator=(const Range &) = delete;
};
const char *const PROF_NAMES[KD_PROF_KINDS] = {"ingest", "select", "pick",  "count",
                                               "big_scatter", "small", "emit", "other"};

// Per-kernel-class timing with HIP events on the build's stream (only when
// the caller asks for a profile).
struct Prof {
    struct Rec {
        int kind;
        hipEvent_t a, b;
        uint64_t points, bytes;
    };
    kd_profile *p;
    hipStream_t st;
    std::vector<Rec> recs;
    Prof(kd_profile *prof, hipStream_t s) : p(prof), st(s) {
        if (p) memset(p, 0, sizeof(*p));
    }
    template <class F>
    void run(int kind, uint64_t points, uint64_t bytes, F &&launch) {
        const Range phase(PROF_NAMES[kind]);
        if (!p) {
            launch();
            return;
        }
        Rec r{kind, nullptr, nullptr, points, bytes};
        (void)hipEventCreate(&r.a);
        (void)hipEventCreate(&r.b);
        (void)hipEventRecord(r.a, st);
        launch();
        (void)hipEventRecord(r.b, st);
        recs.push_back(r);
    }
    bool finish(uint32_t levels) {
        if (!p) return true;
        bool ok = hipStreamSynchronize(st) == hipSuccess;
        for (auto &r : recs) {
            float ms = 0.0f;
            if (hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) ok = false;
            kd_kernel_stat &k = p->k[r.kind];
            k.ms += ms;
            k.launches += 1;
            k.points += r.points;
            k.bytes += r.bytes;
            (void)hipEventDestroy(r.a);
            (void)hipEventDestroy(r.b);
        }
        p->levels = levels;
        return ok;
    }
};

#define KD_LAUNCH_CHECK()                                       \
    do {                                                        \
        if (hipGetLastError() != hipSuccess) return KD_EDEVICE; \
    } while (0)

struct HostTree {
    const float *pts;
    uint64_t n, ld;
    uint32_t d;
    const kd_tree *out;
};

// Upper bounds of a level's totals that hold whatever the data: from the
// level-0 totals `K` (known on the host) and the level number.  Cells hold
// more than leaf_size points and at most double per level; large cells (more
// than SMALL_MAX points) only descend from large cells; a cell of s points
// spans at most s / TILE + 1 tiles.
struct LevelBound {
    uint64_t cells, tiles, big, big_points, small_points;
};

uint64_t shl_sat(uint64_t x, uint32_t s) { return s >= 40 || x >= (uint64_t(1) << (63 - s)) ? ~uint64_t(0) >> 1 : x << s; }

LevelBound level_bound(const LevelInfo &K, uint32_t level, uint32_t leaf_size, const Layout &L) {
    LevelBound b;
    if (level == 0) {
        b = LevelBound{K.num_cells, K.num_tiles, K.num_big, K.big_points,
                       uint64_t(K.points) - K.big_points};
    } else {
        b.cells = std::min<uint64_t>(shl_sat(K.num_cells, level), K.points / (uint64_t(leaf_size) + 1));
        b.big = std::min<uint64_t>(shl_sat(K.num_big, level), K.big_points / (SMALL_MAX + 1));
        b.big_points = b.big ? K.big_points : 0;
        b.tiles = b.big ? b.big_points / TILE + b.big : 0;
        b.small_points = K.points;
    }
    b.cells = std::min(b.cells, L.max_cells);
    b.big = std::min(b.big, L.max_big);
    b.tiles = std::min(b.tiles, L.max_tiles);
    return b;
}

// Tree descriptors reach the workspace as kernel arguments, so a build keeps
// no host buffer past the call and a captured graph holds its own copy.
constexpr uint32_t DESC_CHUNK = 8;
struct DescChunk {
    TreeDesc d[DESC_CHUNK];
    uint32_t first, count;
};
__global__ void k_set_desc(TreeDesc *dst, DescChunk ch) {
    for (uint32_t i = threadIdx.x; i < ch.count; i += blockDim.x) dst[ch.first + i] = ch.d[i];
}

// Levels past the depth a balanced tree of the largest input would reach
// (plus TAIL_SLACK) run in "tail" shape: every kernel on a few workgroups
// (they loop over whatever work the level holds) and the emit step in one
// workgroup, so the empty levels at the end cost a few microseconds each.
constexpr uint32_t TAIL_SLACK = 2;
constexpr uint32_t TAIL_GRID = 64;

// The level loop over every tree of the build.
// Process-wide launch shapes (set by kd_set_tuning / kd_autotune).
std::mutex g_tuning_mu;
kd_tuning g_tuning{};

kd_tuning current_tuning() {
    std::lock_guard<std::mutex> lk(g_tuning_mu);
    return g_tuning;
}

kd_status run_build(uint32_t ntrees, const HostTree *ht, const kd_params *p, void *workspace,
                    uint64_t ws_bytes, hipStream_t st, kd_profile *prof, const kd_tuning &tune) {
    const Range whole(ntrees == 1 ? "kd_build" : "kd_build_batched");
    std::vector<uint64_t> n(ntrees), cap(ntrees);
    std::vector<uint32_t> d(ntrees);
    uint64_t total_points = 0, sum_d = 0;
    for (uint32_t t = 0; t < ntrees; t++) {
        n[t] = ht[t].n;
        d[t] = ht[t].d;
        cap[t] = ht[t].out->node_capacity;
        total_points += n[t];
        sum_d += uint64_t(d[t]) * n[t];
    }
    if (total_points > 0xffffff00ull) return KD_EINVAL;
    const Layout L = plan(ntrees, n.data(), d.data(), cap.data(), p);
    if (ws_bytes < L.total) return KD_ENOMEM;
    char *ws = static_cast<char *>(workspace);
    Prof P(prof, st);

    std::vector<TreeDesc> desc(ntrees);
    uint64_t pbase = 0;
    for (uint32_t t = 0; t < ntrees; t++) {
        const TreeLayout &tl = L.per_tree[t];
        const kd_tree *o = ht[t].out;
        TreeDesc &D = desc[t];
        D.pts = reinterpret_cast<const uint32_t *>(ht[t].pts);
        D.ld = ht[t].ld;
        for (int b = 0; b < 2; b++) {
            D.cols[b] = reinterpret_cast<uint32_t *>(ws + tl.cols[b]);
            D.perm[b] = reinterpret_cast<uint32_t *>(ws + tl.perm[b]);
            D.stats[b] = reinterpret_cast<unsigned long long *>(ws + tl.stats[b]);
        }
        D.out_perm = o->perm;
        D.pts_out = reinterpret_cast<uint32_t *>(o->points_out);
        D.node_begin = o->node_begin;
        D.node_end = o->node_end;
        D.node_child = o->node_child;
        D.node_dim = o->node_dim;
        D.node_split = o->node_split;
        D.node_split_f = o->node_split_f;
        D.node_leaf = o->node_leaf;
        D.leaf_node = o->leaf_node;
        D.leaf_offsets = o->leaf_offsets;
        D.hdr = o->hdr;
        D.cap = cap[t];
        D.n = uint32_t(n[t]);
        D.pbase = pbase;
        pbase += n[t];
        D.d = d[t];
        D.max_depth = p->max_depth ? p->max_depth : default_depth(n[t], p->leaf_size);
        // a root that is a large cell is split at level 0 by the large-cell
        // kernels only, which read the caller's points in place
        D.direct = n[t] > uint64_t(SMALL_MAX) && n[t] > p->leaf_size && D.max_depth > 0 ? 1u : 0u;
    }
    for (uint32_t t0 = 0; t0 < ntrees; t0 += DESC_CHUNK) {
        DescChunk ch{};
        ch.first = t0;
        ch.count = std::min<uint32_t>(DESC_CHUNK, ntrees - t0);
        for (uint32_t i = 0; i < ch.count; i++) ch.d[i] = desc[t0 + i];
        hipLaunchKernelGGL(k_set_desc, dim3(1), dim3(64), 0, st,
                           reinterpret_cast<TreeDesc *>(ws + L.trees), ch);
    }
    KD_LAUNCH_CHECK();

    Ctx c{};
    c.trees = reinterpret_cast<TreeDesc *>(ws + L.trees);
    c.ts = reinterpret_cast<TreeState *>(ws + L.ts);
    c.ntrees = ntrees;
    for (int b = 0; b < 2; b++) c.cells[b] = reinterpret_cast<Cell *>(ws + L.cells[b]);
    c.res = reinterpret_cast<CellRes *>(ws + L.res);
    c.big_list = reinterpret_cast<uint32_t *>(ws + L.big_list);
    c.tile_lt = reinterpret_cast<uint32_t *>(ws + L.tile_lt);
    c.tile_le = reinterpret_cast<uint32_t *>(ws + L.tile_le);
    c.tile_mm = reinterpret_cast<uint32_t *>(ws + L.tile_mm);
    c.tile_cell = reinterpret_cast<uint32_t *>(ws + L.tile_cell);
    c.tiles = reinterpret_cast<TileDesc *>(ws + L.tiles);
    c.hist = reinterpret_cast<uint32_t *>(ws + L.hist);
    c.mm = reinterpret_cast<uint32_t *>(ws + L.mm);
    c.mom = reinterpret_cast<long long *>(ws + L.mom);
    c.bounds = reinterpret_cast<uint32_t *>(ws + L.bounds);
    c.med = reinterpret_cast<uint32_t *>(ws + L.med);
    c.pre = reinterpret_cast<uint32_t *>(ws + L.pre);
    c.scan_tmp = reinterpret_cast<uint32_t *>(ws + L.scan);
    c.bucket_first = reinterpret_cast<uint32_t *>(ws + L.buckets);
    {
        const uint64_t max_seg = L.all_points / (SMALL_MAX + 1) + 2;
        uint32_t *sg = reinterpret_cast<uint32_t *>(ws + L.segs);
        c.seg_count = sg;
        c.seg_job = sg + 64;
        c.seg_prefix = c.seg_job + max_seg;
        c.seg_rank = c.seg_prefix + max_seg;
        c.seg_hist = c.seg_rank + max_seg;
        c.seg_ns = c.seg_hist + max_seg * NBINS;
        c.seg_blk = c.seg_ns + max_seg;
        // 64 + max_seg * (3 + NBINS + 1 + 2) words before it: 8-byte aligned
        static_assert((3 + NBINS + 1 + 2) % 2 == 0, "aligned addresses");
        c.seg_col = reinterpret_cast<const uint32_t **>(c.seg_blk + 2 * max_seg);
    }
    c.info = reinterpret_cast<LevelInfo *>(ws + L.info);
    c.leafbits = reinterpret_cast<uint32_t *>(ws + L.leafbits);
    c.leafpre = reinterpret_cast<uint32_t *>(ws + L.leafpre);
    c.leafblk = reinterpret_cast<uint32_t *>(ws + L.leafblk);
    for (int b = 0; b < 2; b++) c.cell_rec[b] = reinterpret_cast<uint32_t *>(ws + L.cell_rec[b]);
    c.subrec = reinterpret_cast<SubRec *>(ws + L.subrec);
    c.rec_count = reinterpret_cast<uint32_t *>(ws + L.rec_count);
    c.rec_cap = uint32_t(L.rec_cap);
    c.recstats = reinterpret_cast<unsigned long long *>(ws + L.recstats);
    c.recstats_stride = uint32_t(L.recstats_stride);
    c.max_d = 0;
    for (uint32_t t = 0; t < ntrees; t++) c.max_d = std::max(c.max_d, ht[t].d);
    c.pool = p->subset_pool;
    c.pool_entries = p->pool_entries;
    c.seed = p->seed;
    c.leaf_size = p->leaf_size;
    c.key_rule = p->key_rule;
    c.split_rule = p->split_rule;
    c.J = p->fourier_J;
    c.S = p->num_subsets;
    c.trig = make_trig();

    uint64_t maxcap = 0, maxn = 0;
    uint32_t maxd = 0;
    for (uint32_t t = 0; t < ntrees; t++) {
        maxcap = cap[t] > maxcap ? cap[t] : maxcap;
        maxn = n[t] > maxn ? n[t] : maxn;
        maxd = d[t] > maxd ? d[t] : maxd;
    }
    const dim3 per_tree_nodes(grid_for(maxcap / NT + 1, 1024), ntrees);
    const dim3 per_tree_points(grid_for(maxn / NT + 1, 1024), ntrees);
    P.run(KD_PROF_OTHER, 0, 0, [&] {
        hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(L.max_big * BIG_BINS_MAX / NT + 1, 4096)),
                           dim3(NT), 0, st, c.hist, L.max_big * BIG_BINS_MAX, 0u);
        hipLaunchKernelGGL(k_init, per_tree_nodes, dim3(NT), 0, st, c);
        hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(NT), 0, st, c.rec_count, 1ull, 0u);
        hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(L.leaf_words / NT + 1, 4096)), dim3(NT), 0,
                           st, c.leafbits, L.leaf_words, 0u);
        if (p->split_rule == KD_SPLIT_SUBSET) {
            const uint64_t words = (L.all_points / (SMALL_MAX + 1) + 2) * (3 + NBINS) + 64;
            hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(words / NT + 1, 4096)), dim3(NT), 0, st,
                               c.seg_count, words, 0u);
        }
    });
    // bytes: the points read (and copied unless read in place at level 0),
    // the identity permutation written
    uint64_t ingest_bytes = 4 * total_points;
    for (uint32_t t = 0; t < ntrees; t++) ingest_bytes += (desc[t].direct ? 4 : 8) * uint64_t(d[t]) * n[t];
    P.run(KD_PROF_INGEST, total_points, ingest_bytes, [&] {
        hipLaunchKernelGGL(k_ingest, dim3(grid_for(maxn / (NT * 16) + 1, 1024), maxd, ntrees),
                           dim3(NT), 0, st, c);
    });
    P.run(KD_PROF_OTHER, 0, 0, [&] {
        hipLaunchKernelGGL(k_roots, dim3(1), dim3(NT), 0, st, c);
        if (p->key_rule == KD_KEY_MAXVAR)
            hipLaunchKernelGGL(k_root_stats, dim3(grid_for(maxn / (NT * 8) + 1, 512), maxd, ntrees),
                               dim3(NT), 0, st, c);
        hipLaunchKernelGGL(k_copy_leafroots, per_tree_points, dim3(NT), 0, st, c);
    });
    KD_LAUNCH_CHECK();

    const uint64_t scatter_avg_bpp = (8 * sum_d + 8 * total_points) / total_points;
    const bool maxvar = p->key_rule == KD_KEY_MAXVAR;
    // launch shapes: workgroups of the digit passes, of the count and scatter
    // (grid-stride over tiles) and of the small-cell kernel (over buckets)
    const uint32_t hist_grid = tune.hist_blocks ? tune.hist_blocks : 2048u;
    const uint32_t tile_grid = tune.scatter_blocks ? tune.scatter_blocks : 65535u;
    const uint32_t small_grid = tune.small_blocks ? tune.small_blocks : (1u << 20);
    const int digit = tune.digit_bits ? int(tune.digit_bits) : BIG_DIGIT_DEFAULT;
    // dynamic LDS of the small-cell kernel (SUBSET: subset bounds and medians)
    const size_t small_dyn =
        p->split_rule == KD_SPLIT_SUBSET
            ? std::max<size_t>(SUBSET_DYN_WORDS, 2 * size_t(c.S) + 1) * 4
            : 0;
    static_assert(sizeof(uint32_t) * (2 * MAX_SUBSETS + 1) + 64 * 1024 <= 160 * 1024,
                  "small-cell kernel LDS");
    auto fail = [&]() {
        (void)hipStreamSynchronize(st);
        return KD_EDEVICE;
    };
    // level 0 on the host: one root cell per tree with more than leaf_size points
    LevelInfo K{};
    uint32_t likely = 0;  // levels a balanced tree of the largest input would have, + slack
    for (uint32_t t = 0; t < ntrees; t++) {
        if (n[t] <= p->leaf_size || desc[t].max_depth == 0) continue;
        K.num_cells++;
        K.points += uint32_t(n[t]);
        if (n[t] > uint64_t(SMALL_MAX)) {
            K.num_tiles += uint32_t((n[t] + TILE - 1) / TILE);
            K.big_points += uint32_t(n[t]);
            K.num_big++;
        }
        uint32_t h = 0;
        while (h < 64 && (uint64_t(p->leaf_size) << h) < n[t]) h++;  // ceil(log2(n / leaf))
        likely = std::max<uint32_t>(likely, h + 1 + TAIL_SLACK);
    }
    // Profiled builds (measurement only) read every level's totals back and
    // stop at the first empty level, so their launch shapes and byte counts
    // are exact; every other build enqueues all levels at once and returns.
    const bool paced = prof != nullptr;
    uint32_t level_cap = 0;  // the deepest cap of any tree with a root cell
    for (uint32_t t = 0; t < ntrees; t++)
        if (n[t] > p->leaf_size) level_cap = std::max(level_cap, desc[t].max_depth);
    level_cap = std::min<uint32_t>(level_cap, MAX_LEVELS);
    uint32_t levels_run = 0;
    for (uint32_t level = 0; level < level_cap; level++) {
        LevelBound B;
        bool tail = false;
        if (paced) {
            LevelInfo I{};
            if (hipMemcpyAsync(&I, c.info + level, sizeof(LevelInfo), hipMemcpyDeviceToHost, st) !=
                    hipSuccess ||
                hipStreamSynchronize(st) != hipSuccess)
                return fail();
            if (I.num_cells == 0) break;
            B = LevelBound{I.num_cells, I.num_tiles, I.num_big, I.big_points,
                           uint64_t(I.points) - I.big_points - I.resolved};
        } else {
            B = level_bound(K, level, p->leaf_size, L);
            tail = level >= likely;
        }
        levels_run++;
        char level_name[32];
        snprintf(level_name, sizeof(level_name), "level %u%s", level, tail ? " (tail)" : "");
        const Range level_range(level_name);
        // launch shape: the bound's workgroups, or a few in tail shape
        auto G = [&](uint64_t work, uint32_t cap) {
            const uint32_t g = grid_for(work, cap);
            return dim3(tail ? std::min<uint32_t>(g, TAIL_GRID) : g);
        };
        const uint64_t nc = B.cells, ntl = B.tiles, nbig = B.big;
        const uint64_t bigp = B.big_points, smallp = B.small_points;
        P.run(KD_PROF_OTHER, 0, 0, [&] {
            hipLaunchKernelGGL(k_level_init, G(std::max(nc, ntl) / NT + 1, 4096),
                               dim3(NT), 0, st, c, level, nbig > 0 ? 1u : 0u);
        });
        if (nbig > 0) {
            if (p->split_rule == KD_SPLIT_EXACT) {
                const uint32_t passes =
                    digit == 8 ? BigDigits<8>::PASSES : BigDigits<11>::PASSES;
                for (uint32_t pass = 0; pass < passes; pass++) {
                    P.run(KD_PROF_SELECT, bigp, 4 * bigp, [&] {
                        if (digit == 8)
                            hipLaunchKernelGGL(k_big_hist<8>, G(ntl, hist_grid), dim3(NT), 0,
                                               st, c, level, pass);
                        else
                            hipLaunchKernelGGL(k_big_hist<11>, G(ntl, hist_grid), dim3(NT), 0,
                                               st, c, level, pass);
                    });
                    P.run(KD_PROF_PICK, 0, 0, [&] {
                        const dim3 g = G((nbig + NW - 1) / NW, 65535);
                        if (digit == 8)
                            hipLaunchKernelGGL(k_big_pick<8>, g, dim3(NT), 0, st, c, level, pass);
                        else
                            hipLaunchKernelGGL(k_big_pick<11>, g, dim3(NT), 0, st, c, level, pass);
                    });
                }
            } else if (p->split_rule == KD_SPLIT_FOURIER) {
                P.run(KD_PROF_SELECT, bigp, 8 * bigp, [&] {
                    hipLaunchKernelGGL(k_big_minmax, G(ntl, hist_grid), dim3(NT), 0,
                                       st, c, level);
                    hipLaunchKernelGGL(k_big_moments, G(ntl, hist_grid), dim3(NT), 0,
                                       st, c, level);
                });
                P.run(KD_PROF_PICK, 0, 0, [&] {
                    hipLaunchKernelGGL(k_big_fsolve, G((nbig + NW - 1) / NW, 65535),
                                       dim3(NT), 0, st, c, level);
                });
            } else {
                // subsets above SMALL_MAX points (at most one per SMALL_MAX + 1
                // large-cell points): segmented passes over many workgroups,
                // which read the list's length on the device; the rest: one
                // workgroup or wave each, in LDS
                const uint64_t nseg = std::min<uint64_t>(bigp / (SMALL_MAX + 1), nbig * c.S);
                P.run(KD_PROF_SELECT, bigp, 4 * bigp, [&] {
                    hipLaunchKernelGGL(k_big_bounds, G(nbig / NT + 1, 4096), dim3(NT),
                                       0, st, c, level);
                    hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(NT), 0, st, c.seg_count, 2ull, 0u);
                    hipLaunchKernelGGL(k_seg_list, G(nbig * c.S / NT + 1, 4096),
                                       dim3(NT), 0, st, c, level);
                    const uint64_t nblk = std::min<uint64_t>(bigp / SEG_CHUNK + nseg, nseg * SEG_FAN);
                    for (uint32_t pass = 0; nseg > 0 && pass < uint32_t(RPASSES); pass++) {
                        hipLaunchKernelGGL(k_seg_hist, G(nblk, 65535),
                                           dim3(NT), 0, st, c, pass);
                        hipLaunchKernelGGL(k_seg_pick, G(nseg, 65535), dim3(NT), 0, st,
                                           c, pass);
                    }
                    hipLaunchKernelGGL(k_subset_select, G(nbig * c.S / NW + 1, 65535),
                                       dim3(NT), 0, st, c, level);
                });
                P.run(KD_PROF_PICK, 0, 0, [&] {
                    hipLaunchKernelGGL(k_subset_mean, G(nbig / NT + 1, 4096),
                                       dim3(NT), 0, st, c, level);
                });
            }
            // EXACT counts come from the last digit pass's tile summaries
            const uint64_t count_bytes = p->split_rule == KD_SPLIT_EXACT ? 0 : 4 * bigp;
            P.run(KD_PROF_COUNT, bigp, count_bytes, [&] {
                const bool summ = p->split_rule == KD_SPLIT_EXACT;
                const int lpass = (digit == 8 ? BigDigits<8>::PASSES : BigDigits<11>::PASSES) - 1;
                const uint32_t lshift = uint32_t(digit == 8 ? BigDigits<8>::shift(lpass)
                                                            : BigDigits<11>::shift(lpass));
                const uint32_t lbits = uint32_t(digit == 8 ? BigDigits<8>::bits(lpass)
                                                           : BigDigits<11>::bits(lpass));
                // EXACT: runs of eight tiles, most of them settled from the
                // summaries alone
                hipLaunchKernelGGL(k_big_count, summ ? G((ntl + 7) / 8, 65535) : G(ntl, tile_grid),
                                   dim3(NT), 0, st, c, level, summ ? 1u : 0u, lshift,
                                   (1u << lbits) - 1u);
                hipLaunchKernelGGL(k_big_decide, G(nbig, 65535), dim3(NT), 0, st, c,
                                   level);
            });
            P.run(KD_PROF_BIG_SCATTER, bigp, scatter_avg_bpp * bigp, [&] {
                if (maxvar) {
                    hipLaunchKernelGGL(k_big_scatter<true>, G(ntl, tile_grid), dim3(NT), 0,
                                       st, c, level);
                    const uint64_t words = uint64_t(nbig) * 3 * c.max_d;
                    hipLaunchKernelGGL(k_big_derive, G(uint32_t((words + NT - 1) / NT), 4096),
                                       dim3(NT), 0, st, c, level);
                } else
                    hipLaunchKernelGGL(k_big_scatter<false>, G(ntl, tile_grid), dim3(NT),
                                       0, st, c, level);
            });
        }
        if (smallp > 0) {
            P.run(KD_PROF_SMALL, smallp, scatter_avg_bpp * smallp, [&] {
                const dim3 g = G((smallp + TILE - 1) / TILE, small_grid);
#define KD_SUB(R, M) hipLaunchKernelGGL((k_subtree<R, M>), g, dim3(NT), small_dyn, st, c, level)
#define KD_SMALL(R, M) hipLaunchKernelGGL((k_small<R, M>), g, dim3(NT), small_dyn, st, c, level)
                // EXACT, FOURIER and SUBSET with equal subsets finish small
                // cells' subtrees in one pass; a subset pool's rows depend on a
                // cell's rank within its level, known only level by level
                if (p->flags & KD_FLAG_LEVEL_BY_LEVEL) {
                    switch (p->split_rule * 2 + (maxvar ? 1 : 0)) {
                        case 0: KD_SMALL(KD_SPLIT_EXACT, false); break;
                        case 1: KD_SMALL(KD_SPLIT_EXACT, true); break;
                        case 2: KD_SMALL(KD_SPLIT_FOURIER, false); break;
                        case 3: KD_SMALL(KD_SPLIT_FOURIER, true); break;
                        case 4: KD_SMALL(KD_SPLIT_SUBSET, false); break;
                        default: KD_SMALL(KD_SPLIT_SUBSET, true); break;
                    }
                    return;
                }
                switch (p->split_rule * 2 + (maxvar ? 1 : 0)) {
                    case 0: KD_SUB(KD_SPLIT_EXACT, false); break;
                    case 1: KD_SUB(KD_SPLIT_EXACT, true); break;
                    case 2: KD_SUB(KD_SPLIT_FOURIER, false); break;
                    case 3: KD_SUB(KD_SPLIT_FOURIER, true); break;
                    case 4:
                        // equal subsets depend only on a cell's size: the
                        // subtree path; pool rows need the level-wide rank
                        if (c.pool) KD_SMALL(KD_SPLIT_SUBSET, false);
                        else KD_SUB(KD_SPLIT_SUBSET, false);
                        break;
                    default: KD_SMALL(KD_SPLIT_SUBSET, true); break;
                }
#undef KD_SMALL
#undef KD_SUB
            });
        }
        const uint32_t nb = uint32_t((nc + NT - 1) / NT);
        P.run(KD_PROF_EMIT, 0, 0, [&] {
            if (nc <= EMIT_ONE_MAX || tail) {
                hipLaunchKernelGGL(k_emit_one, dim3(1), dim3(EMIT_NT), 0, st, c, level);
                return;
            }
            hipLaunchKernelGGL(k_emit_sum, dim3(nb), dim3(NT), 0, st, c, level);
            hipLaunchKernelGGL(k_emit_scan, dim3(1), dim3(NT), 0, st, c, level, nb);
            hipLaunchKernelGGL(k_emit_prefix, dim3(nb), dim3(NT), 0, st, c, level);
            hipLaunchKernelGGL(k_emit_trees, G(ntrees / NT + 1, 1024), dim3(NT), 0,
                               st, c, level);
            hipLaunchKernelGGL(k_emit_write, dim3(nb), dim3(NT), 0, st, c, level);
        });
        if (hipGetLastError() != hipSuccess) return fail();
    }
    P.run(KD_PROF_OTHER, 0, 0, [&] {
        hipLaunchKernelGGL(k_leaf_mark, per_tree_nodes, dim3(NT), 0, st, c);
        hipLaunchKernelGGL(k_leaf_scan1, dim3(uint32_t(L.leaf_blocks)), dim3(NT), 0, st, c,
                           L.leaf_words);
        hipLaunchKernelGGL(k_leaf_scan2, dim3(1), dim3(NT), 0, st, c, uint32_t(L.leaf_blocks));
        hipLaunchKernelGGL(k_leaf_write, per_tree_nodes, dim3(NT), 0, st, c);
        hipLaunchKernelGGL(k_header, dim3(grid_for(ntrees / NT + 1, 1024)), dim3(NT), 0, st, c);
    });
    KD_LAUNCH_CHECK();
    if (!P.finish(levels_run)) return KD_EDEVICE;
    return KD_OK;
}

bool tree_ok(const kd_tree *o) {
    return o && o->perm && o->node_begin && o->node_end && o->node_child && o->node_dim &&
           o->node_split && o->node_split_f && o->node_leaf && o->leaf_node && o->leaf_offsets &&
           o->hdr && o->node_capacity > 0 && o->node_capacity <= 0xfffffff0ull;
}

}  // namespace

// ------------------------------------------------------------ fixed scratch

// Workspace of kd_build_noalloc: one array per device, held until the
// process ends.  Host code never passes `scratch` itself to a kernel (on the
// host the name is a stand-in, not the device address): the address is
// taken once per device with hipGetSymbolAddress and kept in g_scratch.
static_assert(KD_NOALLOC_SCRATCH_BYTES % 256 == 0, "scratch size");
__device__ __align__(256) uint8_t scratch[KD_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int SCRATCH_DEVICES = 64;
std::mutex g_scratch_mu;
void *g_scratch[SCRATCH_DEVICES] = {};

// Device address of the current device's scratch (nullptr on failure).
void *device_scratch() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= SCRATCH_DEVICES) return nullptr;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch[dev]) {
        void *ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return nullptr;
        g_scratch[dev] = ptr;
    }
    return g_scratch[dev];
}
}  // namespace

// ------------------------------------------------------------ C ABI

extern "C" {

int kd_version(void) { return 2; }

const char *kd_status_string(kd_status s) {
    switch (s) {
        case KD_OK: return "ok";
        case KD_EINVAL: return "invalid argument";
        case KD_ENOMEM: return "workspace too small";
        case KD_ENAN: return "non-finite input value";
        case KD_ECAPACITY: return "node capacity exceeded";
        case KD_EDEVICE: return "device error";
        case KD_ECANCELLED: return "cancelled";
        default: return "unknown status";
    }
}

kd_status kd_tree_bounds(uint64_t n, uint32_t d, const kd_params *params,
                         uint64_t *node_capacity, uint64_t *workspace_bytes) {
    if (!params_ok(params) || !shape_ok(n, d)) return KD_EINVAL;
    const uint64_t cap = params->node_capacity ? params->node_capacity
                                               : default_capacity(n, params->leaf_size);
    if (cap > 0xfffffff0ull) return KD_EINVAL;
    const Layout L = plan(1, &n, &d, &cap, params);
    if (node_capacity) *node_capacity = cap;
    if (workspace_bytes) *workspace_bytes = L.total;
    return KD_OK;
}

kd_status kd_build_profiled(const float *pts, uint64_t n, uint32_t d, uint64_t ld,
                            const kd_params *p, kd_tree *out, void *workspace, uint64_t ws_bytes,
                            void *stream, kd_profile *prof) {
    if (!params_ok(p) || !shape_ok(n, d) || !pts || ld < n || !workspace || !tree_ok(out))
        return KD_EINVAL;
    out->n = n;
    out->d = d;
    const HostTree ht{pts, n, ld, d, out};
    return run_build(1, &ht, p, workspace, ws_bytes, reinterpret_cast<hipStream_t>(stream), prof,
                     current_tuning());
}

kd_status kd_build(const float *pts, uint64_t n, uint32_t d, uint64_t ld, const kd_params *p,
                   kd_tree *out, void *workspace, uint64_t ws_bytes, void *stream) {
    return kd_build_profiled(pts, n, d, ld, p, out, workspace, ws_bytes, stream, nullptr);
}

kd_status kd_build_noalloc(const float *pts, uint64_t n, uint32_t d, uint64_t ld,
                           const kd_params *p, kd_tree *out, void *stream) {
    if (!params_ok(p) || !shape_ok(n, d) || !pts || ld < n || !tree_ok(out)) return KD_EINVAL;
    const uint64_t cap = out->node_capacity;
    const Layout L = plan(1, &n, &d, &cap, p);
    if (L.total > KD_NOALLOC_SCRATCH_BYTES) return KD_ENOMEM;
    void *ws = device_scratch();
    if (!ws) return KD_EDEVICE;
    return kd_build(pts, n, d, ld, p, out, ws, KD_NOALLOC_SCRATCH_BYTES, stream);
}

kd_status kd_query_leaf(const kd_tree *tree, const float *q, uint64_t nq, uint32_t d,
                        uint64_t ldq, uint32_t *leaf_out, void *stream) {
    if (!tree || !q || !leaf_out || d == 0 || d != tree->d || ldq < nq || !tree->node_child ||
        !tree->node_dim || !tree->node_split || !tree->node_leaf)
        return KD_EINVAL;
    if (nq == 0) return KD_OK;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    hipLaunchKernelGGL(k_query, dim3(grid_for(nq / NT + 1, 65535)), dim3(NT), 0, st,
                       tree->node_child, tree->node_dim, tree->node_split, tree->node_leaf, q, nq,
                       ldq, leaf_out);
    KD_LAUNCH_CHECK();
    return KD_OK;
}

static bool query_tree_ok(const kd_tree *t) {
    return t && t->perm && t->node_begin && t->node_end && t->node_child && t->node_dim &&
           t->node_split && t->node_split_f && t->points_out;
}

kd_status kd_query_knn(const kd_tree *tree, uint64_t n, const float *q, uint64_t nq, uint32_t d,
                       uint64_t ldq, uint32_t k, uint32_t *idx_out, double *dist_out,
                       void *stream) {
    if (!query_tree_ok(tree) || n == 0 || n != tree->n || !q || !idx_out || !dist_out || d == 0 ||
        d != tree->d || ldq < nq || k == 0 || k > KNN_MAX)
        return KD_EINVAL;
    if (nq == 0) return KD_OK;
    hipLaunchKernelGGL(k_knn, dim3(grid_for((nq + NW - 1) / NW, 65535)), dim3(NT), 0,
                       reinterpret_cast<hipStream_t>(stream), tree->node_child, tree->node_dim,
                       tree->node_split, tree->node_split_f, tree->node_begin, tree->node_end,
                       tree->points_out, n, tree->perm, q, nq, d, ldq, k, idx_out, dist_out);
    KD_LAUNCH_CHECK();
    return KD_OK;
}

kd_status kd_query_box(const kd_tree *tree, uint64_t n, const float *lo, const float *hi,
                       uint64_t nb, uint32_t d, uint64_t ldb, uint32_t *count_out,
                       const uint64_t *offsets, uint32_t *ids_out, void *stream) {
    if (!query_tree_ok(tree) || n == 0 || n != tree->n || !lo || !hi || !count_out || d == 0 ||
        d != tree->d || ldb < nb || (ids_out && !offsets))
        return KD_EINVAL;
    if (nb == 0) return KD_OK;
    hipLaunchKernelGGL(k_box, dim3(grid_for(nb / NT + 1, 65535)), dim3(NT), 0,
                       reinterpret_cast<hipStream_t>(stream), tree->node_child, tree->node_dim,
                       tree->node_split, tree->node_begin, tree->node_end, tree->points_out, n,
                       tree->perm, lo, hi, nb, d, ldb, count_out, offsets, ids_out);
    KD_LAUNCH_CHECK();
    return KD_OK;
}

kd_status kd_global_moments(const float *pts, uint64_t n, uint32_t p, uint64_t ld, uint32_t J,
                            long long *moments, void *stream) {
    if (!pts || !moments || n == 0 || n > 0xffffff00ull || ld < n || p < 1 || p > 3 || J < 1 ||
        J > uint32_t(GLOBAL_JMAX))
        return KD_EINVAL;
    const uint32_t E = 2 * J + 1;
    const uint32_t rows = (p >= 3 ? E : 1u) * (p >= 2 ? E : 1u);
    const uint32_t groups = (rows + NT - 1) / NT;
    // point ranges: every workgroup's sums stay exact, and about 2048 workgroups
    uint64_t splits = std::min<uint64_t>((2048 + groups - 1) / groups, (n + GLOBAL_CHUNK - 1) / GLOBAL_CHUNK);
    splits = std::max<uint64_t>(splits, (n + GLOBAL_EXACT_POINTS - 1) / GLOBAL_EXACT_POINTS);
    const uint64_t per = (n + splits - 1) / splits;
    splits = (n + per - 1) / per;
    const TrigTables T = make_trig();
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    unsigned long long *C = reinterpret_cast<unsigned long long *>(moments);
    const dim3 g(groups, uint32_t(splits));
    if (p == 1) {
        hipLaunchKernelGGL(k_gmom<1>, g, dim3(NT), 0, st, pts, n, ld, J, per, T, C);
    } else if (p == 2) {
        hipLaunchKernelGGL(k_gmom<2>, g, dim3(NT), 0, st, pts, n, ld, J, per, T, C);
    } else {
        // one workgroup per compute unit, each holding every row of the statistics
        uint64_t s3 = std::min<uint64_t>(256, (n + GLOBAL_CHUNK - 1) / GLOBAL_CHUNK);
        s3 = std::max<uint64_t>(s3, (n + GLOBAL_EXACT_POINTS - 1) / GLOBAL_EXACT_POINTS);
        const uint64_t per3 = (n + s3 - 1) / s3;
        s3 = (n + per3 - 1) / per3;
        hipLaunchKernelGGL(k_gmom3_mfma, dim3(1, uint32_t(s3)), dim3(GMM_NT), 0, st, pts, n, ld, J,
                           per3, T, C);
    }
    KD_LAUNCH_CHECK();
    return KD_OK;
}

kd_status kd_global_solve(const long long *moments, uint32_t p, uint32_t J, uint32_t depth,
                          double *medians, void *stream) {
    if (!moments || !medians || p < 1 || p > 3 || J < 1 || J > uint32_t(GLOBAL_JMAX) || depth < 1 ||
        depth > uint32_t(GLOBAL_MAX_DEPTH))
        return KD_EINVAL;
    const TrigTables T = make_trig();
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    for (uint32_t level = 0; level < depth; level++) {
        const dim3 g(((1u << level) + NW - 1) / NW);
        if (p == 1) hipLaunchKernelGGL(k_gsolve<1>, g, dim3(NT), 0, st, moments, J, level, T, medians);
        else if (p == 2) hipLaunchKernelGGL(k_gsolve<2>, g, dim3(NT), 0, st, moments, J, level, T, medians);
        else hipLaunchKernelGGL(k_gsolve<3>, g, dim3(NT), 0, st, moments, J, level, T, medians);
        KD_LAUNCH_CHECK();
    }
    return KD_OK;
}

kd_status kd_global_counts(const float *pts, uint64_t n, uint32_t p, uint64_t ld,
                           const double *medians, uint32_t depth, unsigned long long *counts,
                           void *stream) {
    if (!pts || !medians || !counts || n == 0 || ld < n || p < 1 || p > 3 || depth < 1 ||
        depth > uint32_t(GLOBAL_MAX_DEPTH))
        return KD_EINVAL;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    hipLaunchKernelGGL(k_fill_u32, dim3(grid_for((2ull << depth) / NT + 1, 64)), dim3(NT), 0, st,
                       reinterpret_cast<uint32_t *>(counts), 2ull << depth, 0u);
    hipLaunchKernelGGL(k_gcount, dim3(grid_for(n / NT + 1, 2048)), dim3(NT), 0, st, pts, n, ld, p,
                       medians, depth, counts);
    KD_LAUNCH_CHECK();
    return KD_OK;
}

kd_status kd_batch_bounds(uint32_t count, const kd_batch_item *items, const kd_params *params,
                          uint64_t *workspace_bytes) {
    if (count == 0 || !items || !params || !workspace_bytes || !params_ok(params))
        return KD_EINVAL;
    std::vector<uint64_t> n(count), cap(count);
    std::vector<uint32_t> d(count);
    for (uint32_t t = 0; t < count; t++) {
        if (!shape_ok(items[t].n, items[t].d)) return KD_EINVAL;
        n[t] = items[t].n;
        d[t] = items[t].d;
        cap[t] = items[t].out.node_capacity ? items[t].out.node_capacity
                                            : default_capacity(n[t], params->leaf_size);
    }
    *workspace_bytes = plan(count, n.data(), d.data(), cap.data(), params).total;
    return KD_OK;
}

kd_status kd_build_batched(uint32_t count, const kd_batch_item *items, const kd_params *params,
                           void *workspace, uint64_t ws_bytes, void *stream) {
    if (count == 0 || !items || !params_ok(params) || !workspace) return KD_EINVAL;
    std::vector<HostTree> ht(count);
    for (uint32_t t = 0; t < count; t++) {
        const kd_batch_item &it = items[t];
        if (!shape_ok(it.n, it.d) || !it.pts || it.ld < it.n || !tree_ok(&it.out) ||
            (it.out.n != 0 && it.out.n != it.n) || (it.out.d != 0 && it.out.d != it.d))
            return KD_EINVAL;
        ht[t] = HostTree{it.pts, it.n, it.ld, it.d, &it.out};
    }
    return run_build(count, ht.data(), params, workspace, ws_bytes,
                     reinterpret_cast<hipStream_t>(stream), nullptr, current_tuning());
}

kd_status kd_set_tuning(const kd_tuning *t) {
    if (!t) return KD_EINVAL;
    std::lock_guard<std::mutex> lk(g_tuning_mu);
    if (t->digit_bits != 0 && t->digit_bits != 8 && t->digit_bits != 11) return KD_EINVAL;
    g_tuning = *t;
    return KD_OK;
}

kd_status kd_get_tuning(kd_tuning *t) {
    if (!t) return KD_EINVAL;
    std::lock_guard<std::mutex> lk(g_tuning_mu);
    *t = g_tuning;
    return KD_OK;
}

namespace {

// Host copy of the parts of a built tree that identify it.
struct TreeSnapshot {
    kd_header hdr{};
    std::vector<uint32_t> perm, child, split;
    bool operator==(const TreeSnapshot &o) const {
        return memcmp(&hdr, &o.hdr, sizeof(hdr)) == 0 && perm == o.perm && child == o.child &&
               split == o.split;
    }
};

kd_status snapshot(const kd_tree *out, uint64_t n, hipStream_t st, TreeSnapshot &s) {
    if (hipMemcpyAsync(&s.hdr, out->hdr, sizeof(kd_header), hipMemcpyDeviceToHost, st) !=
            hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        return KD_EDEVICE;
    const uint64_t nn = s.hdr.num_nodes;
    s.perm.resize(n);
    s.child.resize(nn);
    s.split.resize(nn);
    if (hipMemcpyAsync(s.perm.data(), out->perm, n * 4, hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipMemcpyAsync(s.child.data(), out->node_child, nn * 4, hipMemcpyDeviceToHost, st) !=
            hipSuccess ||
        hipMemcpyAsync(s.split.data(), out->node_split, nn * 4, hipMemcpyDeviceToHost, st) !=
            hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        return KD_EDEVICE;
    return KD_OK;
}

}  // namespace

kd_status kd_autotune(const float *pts, uint64_t n, uint32_t d, uint64_t ld,
                      const kd_params *p, kd_tree *out, void *workspace, uint64_t ws_bytes,
                      void *stream, kd_tuning *best) {
    if (!params_ok(p) || !shape_ok(n, d) || !pts || ld < n || !workspace || !tree_ok(out) || !best)
        return KD_EINVAL;
    const hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const HostTree ht{pts, n, ld, d, out};
    kd_tuning cur = current_tuning();
    kd_status s = run_build(1, &ht, p, workspace, ws_bytes, st, nullptr, cur);
    if (s != KD_OK) return s;
    TreeSnapshot ref;
    if ((s = snapshot(out, n, st, ref)) != KD_OK) return s;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return KD_EDEVICE;
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return KD_EDEVICE;
    }
    auto timed = [&](const kd_tuning &t, float &ms, bool &same) -> kd_status {
        kd_status r = run_build(1, &ht, p, workspace, ws_bytes, st, nullptr, t);  // warm
        if (r != KD_OK) return r;
        TreeSnapshot got;
        if ((r = snapshot(out, n, st, got)) != KD_OK) return r;
        same = got == ref;
        if (hipEventRecord(e0, st) != hipSuccess) return KD_EDEVICE;
        for (int i = 0; i < 3; i++)
            if ((r = run_build(1, &ht, p, workspace, ws_bytes, st, nullptr, t)) != KD_OK) return r;
        if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
            return KD_EDEVICE;
        return KD_OK;
    };
    float best_ms = 0.0f;
    bool same = true;
    s = timed(cur, best_ms, same);
    // one field at a time: each candidate replaces that field of the best so far
    static const uint32_t kHist[] = {0, 65535, 4096, 1024, 512};
    static const uint32_t kTile[] = {0, 4096, 2048, 1024};
    static const uint32_t kSmall[] = {0, 8192, 4096, 2048};
    static const uint32_t kDigit[] = {0, 8};  // 0: 11-bit digits
    for (int field = 0; field < 4 && s == KD_OK; field++) {
        const uint32_t *vals = field == 0 ? kHist : field == 1 ? kTile : field == 2 ? kSmall : kDigit;
        const int nv = field == 0 ? 5 : field == 3 ? 2 : 4;
        for (int i = 0; i < nv && s == KD_OK; i++) {
            kd_tuning t = cur;
            uint32_t &f = field == 0   ? t.hist_blocks
                          : field == 1 ? t.scatter_blocks
                          : field == 2 ? t.small_blocks
                                       : t.digit_bits;
            if (f == vals[i]) continue;
            f = vals[i];
            float ms = 0.0f;
            bool ok = true;
            s = timed(t, ms, ok);
            if (s == KD_OK && !ok) s = KD_EDEVICE;
            if (s == KD_OK && ms < best_ms) {
                best_ms = ms;
                cur = t;
            }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (s == KD_OK && !same) s = KD_EDEVICE;
    if (s != KD_OK) return s;
    kd_set_tuning(&cur);
    *best = cur;
    return KD_OK;
}

}  // extern "C"

// kdtree.hip -- MI355X (gfx950) level-by-level k-d tree build behind the C ABI
// declared in include/kdtree.h.
//
// One level (§2: every cell of a level is split along its key at an
// approximate median, producing the next level's cells):
//   large cells (> SMALL_MAX points), tile-parallel over TILE-point tiles:
//     radix-select histograms per tile, added into per-cell histograms
//     (the "map" and "reduce by +" of App. C.2; tiles are the subsets),
//     one pick per cell and digit, then a per-tile count, a per-cell scan of
//     the tile counts and a stable scatter of every column and the perm;
//   small cells, one workgroup per cell: keys staged in LDS, radix select in
//     LDS, stable ranks from a workgroup scan, then the same scatter;
//   emit: node records and the next level's cells (device-wide scan).
// Children that stop being split are written straight to their final place
// in the output permutation (and the optional permuted points), so no
// separate gather is needed at the end.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <vector>

#include "kdtree.h"
#include "kd_device.hpp"

using namespace kd;

static_assert(NBINS == NT, "one histogram bin per thread");
static_assert(PER_THREAD * NT == TILE && SMALL_MAX <= TILE, "tile shape");

namespace {

constexpr uint32_t NONE = 0xffffffffu;
constexpr int EMIT_COUNTERS = 5;  // splits, active children, tiles, points, large-cell points
constexpr int EMIT_STRIDE = 8;

struct Ctx {
    // working buffers (ping-pong by level parity)
    uint32_t *cols[2];
    uint32_t *perm[2];
    Cell *cells[2];
    CellRes *res;
    uint32_t *tile_left;
    uint32_t *tile_off;
    uint32_t *hist;
    uint32_t *scan_tmp;
    LevelInfo *info;
    uint32_t *leaf_cnt;
    uint32_t *leaf_first;
    // outputs
    uint32_t *out_perm;
    uint32_t *pts_out;  // float bits, may be null
    uint32_t *node_begin, *node_end;
    int32_t *node_child;
    uint32_t *node_dim, *node_split;
    float *node_split_f;
    uint32_t *node_leaf, *leaf_node, *leaf_offsets;
    kd_header *hdr;
    // sizes and parameters
    uint64_t cap;
    uint32_t n, d, leaf_size, max_depth;
    uint32_t key_rule, split_rule, J, S;
};

// ------------------------------------------------------------ sizing

struct Layout {
    uint64_t off_cols[2], off_perm[2], off_cells[2], off_res, off_tile_left, off_tile_off,
        off_hist, off_scan, off_info, off_leaf_cnt, off_leaf_first, total;
    uint64_t max_cells, max_tiles, hist_words, scan_blocks;
};

uint64_t align256(uint64_t x) { return (x + 255) & ~uint64_t(255); }

Layout layout_for(uint64_t n, uint32_t d, uint32_t leaf_size, uint64_t cap) {
    Layout L{};
    L.max_cells = n / (uint64_t(leaf_size) + 1) + 1;
    L.max_tiles = n / TILE + n / (SMALL_MAX + 1) + 2;
    L.hist_words = L.max_tiles * NBINS;
    L.scan_blocks = (L.max_cells + NT - 1) / NT;
    uint64_t o = 0;
    auto take = [&](uint64_t bytes) {
        uint64_t r = o;
        o = align256(o + bytes);
        return r;
    };
    for (int b = 0; b < 2; b++) L.off_cols[b] = take(uint64_t(d) * n * 4);
    for (int b = 0; b < 2; b++) L.off_perm[b] = take(n * 4);
    for (int b = 0; b < 2; b++) L.off_cells[b] = take(L.max_cells * sizeof(Cell));
    L.off_res = take(L.max_cells * sizeof(CellRes));
    L.off_tile_left = take(L.max_tiles * 4);
    L.off_tile_off = take(L.max_tiles * 4);
    L.off_hist = take(L.hist_words * 4);
    L.off_scan = take((L.scan_blocks + 1) * EMIT_STRIDE * 4);
    L.off_info = take(sizeof(LevelInfo));
    L.off_leaf_cnt = take(cap * 4);
    L.off_leaf_first = take(cap * 4);
    L.total = o;
    return L;
}

// ------------------------------------------------------------ kernels

__global__ void k_fill_u32(uint32_t *p, uint64_t count, uint32_t v) {
    for (uint64_t i = blockIdx.x * uint64_t(NT) + threadIdx.x; i < count;
         i += uint64_t(gridDim.x) * NT)
        p[i] = v;
}

__global__ void k_init(Ctx c, uint32_t root_active) {
    for (uint64_t i = blockIdx.x * uint64_t(NT) + threadIdx.x; i < c.cap;
         i += uint64_t(gridDim.x) * NT) {
        c.node_begin[i] = 0;
        c.node_end[i] = 0;
        c.node_child[i] = -1;
        c.node_dim[i] = 0;
        c.node_split[i] = 0;
        c.node_split_f[i] = 0.0f;
        c.node_leaf[i] = NONE;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        LevelInfo z{};
        z.num_nodes = 1;
        z.num_cells = root_active ? 1u : 0u;
        z.num_tiles = (root_active && c.n > uint32_t(SMALL_MAX)) ? (c.n + TILE - 1) / TILE : 0u;
        z.points = root_active ? c.n : 0u;
        z.big_points = z.num_tiles ? c.n : 0u;
        *c.info = z;
        c.node_begin[0] = 0;
        c.node_end[0] = c.n;
        Cell root{0u, c.n, 0u, 0u};
        c.cells[0][0] = root;
    }
}

// a1: copy the caller's points into working buffer 0 (float bits), identity
// permutation, reject NaN / Inf.
__global__ void k_ingest(Ctx c, const float *pts, uint64_t ld) {
    const uint32_t col = blockIdx.y;
    const uint32_t *src = reinterpret_cast<const uint32_t *>(pts) + uint64_t(col) * ld;
    uint32_t *dst = c.cols[0] + uint64_t(col) * c.n;
    bool bad = false;
    for (uint32_t i = blockIdx.x * NT + threadIdx.x; i < c.n; i += gridDim.x * NT) {
        uint32_t b = src[i];
        bad |= (b & 0x7f800000u) == 0x7f800000u;
        dst[i] = b;
        if (col == 0) c.perm[0][i] = i;
    }
    if (__any(bad) && lane() == 0) atomicExch(&c.info->status, int32_t(KD_ENAN));
}

// Root that is already a leaf: everything goes straight to the outputs.
__global__ void k_copy_all(Ctx c) {
    for (uint32_t i = blockIdx.x * NT + threadIdx.x; i < c.n; i += gridDim.x * NT) {
        c.out_perm[i] = c.perm[0][i];
        if (c.pts_out)
            for (uint32_t k = 0; k < c.d; k++)
                c.pts_out[uint64_t(k) * c.n + i] = c.cols[0][uint64_t(k) * c.n + i];
    }
}

// Per-level cell state: key coordinate and radix-select start.
__global__ void k_level_init(Ctx c, uint32_t level, uint32_t ncells) {
    const uint32_t cur = level & 1;
    for (uint32_t i = blockIdx.x * NT + threadIdx.x; i < ncells; i += gridDim.x * NT) {
        Cell cl = c.cells[cur][i];
        CellRes r{};
        r.dim = level % c.d;
        r.rank = (cl.end - cl.begin - 1) / 2;
        r.split = 0;
        c.res[i] = r;
    }
}

__device__ __forceinline__ uint32_t find_tile_cell(const Cell *cells, uint32_t ncells, uint32_t t) {
    uint32_t lo = 0, hi = ncells;
    while (hi - lo > 1) {
        uint32_t mid = (lo + hi) >> 1;
        if (cells[mid].tile0 <= t) lo = mid;
        else hi = mid;
    }
    return lo;
}

// After the candidate m and its counts are known: tie rule and leaf flags.
__device__ __forceinline__ void finish_cell(const Ctx &c, uint32_t level, uint32_t n_c, CellRes &r,
                                            uint32_t m) {
    uint32_t split, nl;
    if (tie_rule(n_c, r.lt, r.le, m, &split, &nl)) {
        r.split = split;
        r.nl = nl;
        bool deep = level + 1 >= c.max_depth;
        r.flags = RES_SPLIT | ((nl <= c.leaf_size || deep) ? RES_LEFT_LEAF : 0u) |
                  ((n_c - nl <= c.leaf_size || deep) ? RES_RIGHT_LEAF : 0u);
    } else {
        // all keys equal: the cell stays a leaf and its points go to the outputs
        r.split = m;
        r.nl = n_c;
        r.flags = RES_LEFT_LEAF | RES_RIGHT_LEAF;
    }
}

// a4 (EXACT, large cells): one radix-select digit histogram per tile, added
// into the cell's histogram.
__global__ __launch_bounds__(NT) void k_big_hist(Ctx c, uint32_t level, uint32_t pass,
                                                 uint32_t ncells, uint32_t ntiles) {
    __shared__ uint32_t h[NBINS];
    __shared__ uint32_t s_cell;
    const uint32_t cur = level & 1;
    const int shift = 32 - RBITS * (pass + 1);
    const uint32_t mask = pass == 0 ? 0u : (~0u << (32 - RBITS * pass));
    for (uint32_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        if (threadIdx.x == 0) s_cell = find_tile_cell(c.cells[cur], ncells, t);
        for (int b = threadIdx.x; b < NBINS; b += NT) h[b] = 0;
        __syncthreads();
        const uint32_t ci = s_cell;
        const Cell cl = c.cells[cur][ci];
        const CellRes r = c.res[ci];
        const uint32_t tb = cl.begin + (t - cl.tile0) * TILE;
        const uint32_t te = min(tb + TILE, cl.end);
        const uint32_t *col = c.cols[cur] + uint64_t(r.dim) * c.n;
        for (uint32_t i = tb + threadIdx.x; i < te; i += NT) {
            uint32_t u = key_of_bits(col[i]);
            if ((u & mask) == r.prefix) atomicAdd(&h[(u >> shift) & (NBINS - 1)], 1u);
        }
        __syncthreads();
        uint32_t *gh = c.hist + uint64_t(cl.tile0) * NBINS;
        for (int b = threadIdx.x; b < NBINS; b += NT)
            if (h[b]) atomicAdd(&gh[b], h[b]);
        __syncthreads();
    }
}

// a5 (EXACT, large cells): pick the digit holding the target rank.
__global__ __launch_bounds__(NT) void k_big_pick(Ctx c, uint32_t level, uint32_t pass,
                                                 uint32_t ncells) {
    __shared__ uint32_t sh[NW + 1];
    __shared__ uint32_t s_bin, s_below, s_cnt;
    const uint32_t cur = level & 1;
    const int shift = 32 - RBITS * (pass + 1);
    for (uint32_t ci = blockIdx.x; ci < ncells; ci += gridDim.x) {
        const Cell cl = c.cells[cur][ci];
        const uint32_t n_c = cl.end - cl.begin;
        if (n_c <= uint32_t(SMALL_MAX)) continue;
        CellRes r = c.res[ci];
        uint32_t *gh = c.hist + uint64_t(cl.tile0) * NBINS;
        uint32_t hv = gh[threadIdx.x];
        gh[threadIdx.x] = 0;
        uint32_t tot;
        uint32_t ex = block_excl_scan(hv, sh, &tot);
        if (ex <= r.rank && r.rank < ex + hv) {
            s_bin = threadIdx.x;
            s_below = ex;
            s_cnt = hv;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            r.prefix |= s_bin << shift;
            r.rank -= s_below;
            r.lt += s_below;
            if (pass == RPASSES - 1) {
                r.le = r.lt + s_cnt;
                finish_cell(c, level, n_c, r, r.prefix);
            }
            c.res[ci] = r;
        }
        __syncthreads();
    }
}

// a6/a7 (large cells): left count of every tile.
__global__ __launch_bounds__(NT) void k_big_count(Ctx c, uint32_t level, uint32_t ncells,
                                                  uint32_t ntiles) {
    __shared__ uint32_t s_cell;
    __shared__ uint32_t sh[NW + 1];
    const uint32_t cur = level & 1;
    for (uint32_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        if (threadIdx.x == 0) s_cell = find_tile_cell(c.cells[cur], ncells, t);
        __syncthreads();
        const uint32_t ci = s_cell;
        const Cell cl = c.cells[cur][ci];
        const CellRes r = c.res[ci];
        const uint32_t tb = cl.begin + (t - cl.tile0) * TILE;
        const uint32_t te = min(tb + TILE, cl.end);
        uint32_t cnt = 0;
        if (r.flags & RES_SPLIT) {
            const uint32_t *col = c.cols[cur] + uint64_t(r.dim) * c.n;
            for (uint32_t i = tb + threadIdx.x; i < te; i += NT)
                cnt += key_of_bits(col[i]) <= r.split;
        }
        uint32_t tot;
        block_excl_scan(cnt, sh, &tot);
        if (threadIdx.x == 0) c.tile_left[t] = tot;
    }
}

// Exclusive scan of the tile left counts inside each large cell.
__global__ __launch_bounds__(NT) void k_big_tilescan(Ctx c, uint32_t level, uint32_t ncells) {
    __shared__ uint32_t sh[NW + 1];
    const uint32_t cur = level & 1;
    for (uint32_t ci = blockIdx.x; ci < ncells; ci += gridDim.x) {
        const Cell cl = c.cells[cur][ci];
        const uint32_t n_c = cl.end - cl.begin;
        if (n_c <= uint32_t(SMALL_MAX)) continue;
        const uint32_t nt = (n_c + TILE - 1) / TILE;
        uint32_t base = 0;
        for (uint32_t k0 = 0; k0 < nt; k0 += NT) {
            uint32_t k = k0 + threadIdx.x;
            uint32_t v = k < nt ? c.tile_left[cl.tile0 + k] : 0u;
            uint32_t tot;
            uint32_t ex = block_excl_scan(v, sh, &tot);
            if (k < nt) c.tile_off[cl.tile0 + k] = base + ex;
            base += tot;
        }
    }
}

// Move every column and the permutation of positions [tb, tb+cnt) of cell
// cl to cell-relative destinations dest[] (LDS).  Children that stop here
// go to the outputs, the others to the next working buffer.
__device__ __forceinline__ void move_columns(const Ctx &c, uint32_t cur, const Cell &cl,
                                             const CellRes &r, uint32_t tb, uint32_t cnt,
                                             const uint32_t *dest) {
    const uint32_t nxt = cur ^ 1;
    const uint32_t n_c = cl.end - cl.begin;
    const bool lleaf = r.flags & RES_LEFT_LEAF, rleaf = r.flags & RES_RIGHT_LEAF;
    for (uint32_t k = 0; k <= c.d; k++) {
        const bool is_perm = k == c.d;
        const uint32_t *src = is_perm ? c.perm[cur] : c.cols[cur] + uint64_t(k) * c.n;
        uint32_t *dnext = is_perm ? c.perm[nxt] : c.cols[nxt] + uint64_t(k) * c.n;
        uint32_t *dout = is_perm ? c.out_perm : (c.pts_out ? c.pts_out + uint64_t(k) * c.n : nullptr);
        uint32_t v[PER_THREAD];
#pragma unroll
        for (int j = 0; j < PER_THREAD; j++) {
            uint32_t i = j * NT + threadIdx.x;
            if (i < cnt) v[j] = src[tb + i];
        }
#pragma unroll
        for (int j = 0; j < PER_THREAD; j++) {
            uint32_t i = j * NT + threadIdx.x;
            if (i < cnt) {
                uint32_t dr = dest[i];
                bool leaf = dr < r.nl ? lleaf : rleaf;
                uint32_t *dst = leaf ? dout : dnext;
                if (dst && dr < n_c) dst[cl.begin + dr] = v[j];
            }
        }
    }
}

// a7 (large cells): stable partition-scatter of one tile.
__global__ __launch_bounds__(NT) void k_big_scatter(Ctx c, uint32_t level, uint32_t ncells,
                                                    uint32_t ntiles) {
    __shared__ uint32_t dest[TILE];
    __shared__ uint32_t sh[NW + 1];
    __shared__ uint32_t s_cell;
    const uint32_t cur = level & 1;
    for (uint32_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        if (threadIdx.x == 0) s_cell = find_tile_cell(c.cells[cur], ncells, t);
        __syncthreads();
        const uint32_t ci = s_cell;
        const Cell cl = c.cells[cur][ci];
        const CellRes r = c.res[ci];
        const uint32_t tb = cl.begin + (t - cl.tile0) * TILE;
        const uint32_t te = min(tb + TILE, cl.end);
        const uint32_t cnt = te - tb;
        if (r.flags & RES_SPLIT) {
            const uint32_t *col = c.cols[cur] + uint64_t(r.dim) * c.n;
            // stage keys (coalesced), then each thread ranks PER_THREAD consecutive ones
            for (uint32_t i = threadIdx.x; i < cnt; i += NT) dest[i] = key_of_bits(col[tb + i]);
            __syncthreads();
            const uint32_t i0 = threadIdx.x * PER_THREAD;
            uint32_t f = 0, nleft = 0;
#pragma unroll
            for (int j = 0; j < PER_THREAD; j++) {
                uint32_t i = i0 + j;
                bool l = i < cnt && dest[i] <= r.split;
                f |= uint32_t(l) << j;
                nleft += l;
            }
            uint32_t tot;
            uint32_t lpre = block_excl_scan(nleft, sh, &tot);
            const uint32_t lbase = c.tile_off[t];
            const uint32_t rbase = r.nl + (tb - cl.begin) - lbase;
            uint32_t lo = lbase + lpre, ro = rbase + (i0 - lpre);
#pragma unroll
            for (int j = 0; j < PER_THREAD; j++) {
                uint32_t i = i0 + j;
                if (i < cnt) {
                    if ((f >> j) & 1u) dest[i] = lo++;
                    else dest[i] = ro++;
                }
            }
        } else {
            for (uint32_t i = threadIdx.x; i < cnt; i += NT) dest[i] = tb - cl.begin + i;
        }
        __syncthreads();
        move_columns(c, cur, cl, r, tb, cnt, dest);
        __syncthreads();
    }
}

// Small cells: the whole cell in one workgroup (select, rank, scatter).
__global__ __launch_bounds__(NT) void k_small(Ctx c, uint32_t level, uint32_t ncells) {
    __shared__ uint32_t keys[SMALL_MAX];
    __shared__ uint32_t h[NBINS];
    __shared__ uint32_t sh[NW + 1];
    __shared__ uint32_t s_bin, s_below, s_cnt;
    const uint32_t cur = level & 1;
    for (uint32_t ci = blockIdx.x; ci < ncells; ci += gridDim.x) {
        const Cell cl = c.cells[cur][ci];
        const uint32_t n_c = cl.end - cl.begin;
        if (n_c > uint32_t(SMALL_MAX)) continue;
        CellRes r = c.res[ci];
        const uint32_t *col = c.cols[cur] + uint64_t(r.dim) * c.n;
        for (uint32_t i = threadIdx.x; i < n_c; i += NT) keys[i] = key_of_bits(col[cl.begin + i]);
        // radix select of rank floor((n_c - 1) / 2) in LDS
        uint32_t prefix = 0, rank = r.rank, lt = 0, cnt_eq = 0;
        for (int pass = 0; pass < RPASSES; pass++) {
            const int shift = 32 - RBITS * (pass + 1);
            const uint32_t mask = pass == 0 ? 0u : (~0u << (32 - RBITS * pass));
            for (int b = threadIdx.x; b < NBINS; b += NT) h[b] = 0;
            __syncthreads();
            for (uint32_t i = threadIdx.x; i < n_c; i += NT) {
                uint32_t u = keys[i];
                if ((u & mask) == prefix) atomicAdd(&h[(u >> shift) & (NBINS - 1)], 1u);
            }
            __syncthreads();
            uint32_t hv = h[threadIdx.x], tot;
            uint32_t ex = block_excl_scan(hv, sh, &tot);
            if (ex <= rank && rank < ex + hv) {
                s_bin = threadIdx.x;
                s_below = ex;
                s_cnt = hv;
            }
            __syncthreads();
            prefix |= s_bin << shift;
            rank -= s_below;
            lt += s_below;
            cnt_eq = s_cnt;
            __syncthreads();
        }
        r.lt = lt;
        r.le = lt + cnt_eq;
        finish_cell(c, level, n_c, r, prefix);
        // ranks: thread t owns E consecutive positions
        const uint32_t E = (n_c + NT - 1) / NT;
        const uint32_t i0 = min(threadIdx.x * E, n_c), i1 = min(i0 + E, n_c);
        if (r.flags & RES_SPLIT) {
            uint32_t nleft = 0;
            for (uint32_t i = i0; i < i1; i++) nleft += keys[i] <= r.split;
            uint32_t tot;
            uint32_t lpre = block_excl_scan(nleft, sh, &tot);
            uint32_t lo = lpre, ro = r.nl + (i0 - lpre);
            for (uint32_t i = i0; i < i1; i++) keys[i] = keys[i] <= r.split ? lo++ : ro++;
        } else {
            __syncthreads();
            for (uint32_t i = i0; i < i1; i++) keys[i] = i;
        }
        __syncthreads();
        move_columns(c, cur, cl, r, cl.begin, n_c, keys);
        if (threadIdx.x == 0) c.res[ci] = r;
        __syncthreads();
    }
}

// a8 emit, phase 1: per-workgroup totals of (splits, active children, tiles,
// active points, large-cell points).
__device__ __forceinline__ void emit_counts(const Ctx &c, uint32_t level, uint32_t ci,
                                            uint32_t ncells, uint32_t cnt[EMIT_COUNTERS]) {
    for (int k = 0; k < EMIT_COUNTERS; k++) cnt[k] = 0;
    if (ci >= ncells) return;
    const Cell cl = c.cells[level & 1][ci];
    const CellRes r = c.res[ci];
    if (!(r.flags & RES_SPLIT)) return;
    cnt[0] = 1;
    const uint32_t sz[2] = {r.nl, cl.end - cl.begin - r.nl};
    const uint32_t leaf[2] = {r.flags & RES_LEFT_LEAF, r.flags & RES_RIGHT_LEAF};
    for (int s = 0; s < 2; s++) {
        if (leaf[s]) continue;
        cnt[1]++;
        cnt[3] += sz[s];
        if (sz[s] > uint32_t(SMALL_MAX)) {
            cnt[2] += (sz[s] + TILE - 1) / TILE;
            cnt[4] += sz[s];
        }
    }
}

__global__ __launch_bounds__(NT) void k_emit_sum(Ctx c, uint32_t level, uint32_t ncells) {
    __shared__ uint32_t sh[NW + 1];
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
    uint32_t base[EMIT_COUNTERS] = {0, 0, 0, 0, 0};
    for (uint32_t b0 = 0; b0 < nblocks; b0 += NT) {
        uint32_t b = b0 + threadIdx.x;
        for (int k = 0; k < EMIT_COUNTERS; k++) {
            uint32_t v = b < nblocks ? c.scan_tmp[b * EMIT_STRIDE + k] : 0u;
            uint32_t tot;
            uint32_t ex = block_excl_scan(v, sh, &tot);
            if (b < nblocks) c.scan_tmp[b * EMIT_STRIDE + k] = base[k] + ex;
            base[k] += tot;
        }
    }
    if (threadIdx.x == 0) {
        LevelInfo *in = c.info;
        in->nodes_base = in->num_nodes;
        in->splits = base[0];
        uint64_t after = uint64_t(in->num_nodes) + 2ull * base[0];
        if (after > c.cap) {
            in->status = KD_ECAPACITY;
            in->num_cells = 0;
            in->num_tiles = 0;
            in->points = 0;
            in->big_points = 0;
        } else {
            in->num_nodes = uint32_t(after);
            in->num_cells = base[1];
            in->num_tiles = base[2];
            in->points = base[3];
            in->big_points = base[4];
        }
    }
}

__global__ __launch_bounds__(NT) void k_emit_write(Ctx c, uint32_t level, uint32_t ncells) {
    __shared__ uint32_t sh[NW + 1];
    __shared__ unsigned long long sh64[NW];
    const uint32_t ci = blockIdx.x * NT + threadIdx.x;
    uint32_t cnt[EMIT_COUNTERS], pre[3];
    emit_counts(c, level, ci, ncells, cnt);
    for (int k = 0; k < 3; k++) {
        uint32_t tot;
        pre[k] = block_excl_scan(cnt[k], sh, &tot) + c.scan_tmp[blockIdx.x * EMIT_STRIDE + k];
    }
    const LevelInfo in = *c.info;
    unsigned long long pl = 0;
    uint32_t unsplit = 0;
    if (ci < ncells && in.status != KD_ECAPACITY) {
        const Cell cl = c.cells[level & 1][ci];
        const CellRes r = c.res[ci];
        if (r.flags & RES_SPLIT) {
            const uint32_t left = in.nodes_base + 2 * pre[0];
            pl = cl.end - cl.begin;
            c.node_child[cl.node] = int32_t(left);
            c.node_dim[cl.node] = r.dim;
            c.node_split[cl.node] = r.split;
            c.node_split_f[cl.node] = __uint_as_float(bits_of_key(r.split));
            const uint32_t mid = cl.begin + r.nl;
            c.node_begin[left] = cl.begin;
            c.node_end[left] = mid;
            c.node_begin[left + 1] = mid;
            c.node_end[left + 1] = cl.end;
            uint32_t slot = pre[1], tile = pre[2];
            Cell *nx = c.cells[(level + 1) & 1];
            const uint32_t b[2] = {cl.begin, mid}, e[2] = {mid, cl.end};
            const uint32_t leaf[2] = {r.flags & RES_LEFT_LEAF, r.flags & RES_RIGHT_LEAF};
            for (int s = 0; s < 2; s++) {
                if (leaf[s]) continue;
                nx[slot++] = Cell{b[s], e[s], left + s, tile};
                uint32_t sz = e[s] - b[s];
                if (sz > uint32_t(SMALL_MAX)) tile += (sz + TILE - 1) / TILE;
            }
        } else {
            unsplit = 1;
        }
    }
    unsigned long long s_pl = block_sum64(pl, sh64);
    unsigned long long s_un = block_sum64(unsplit, sh64);
    if (threadIdx.x == 0) {
        if (s_pl) atomicAdd(&c.info->point_levels, s_pl);
        if (s_un) atomicAdd(&c.info->unsplittable, uint32_t(s_un));
    }
}

// Leaves in position order: subtree leaf counts bottom-up, first leaf index
// top-down, both one tree level per launch over its node-id range.
__global__ void k_leaf_count(Ctx c, uint32_t a, uint32_t b) {
    for (uint32_t k = a + blockIdx.x * NT + threadIdx.x; k < b; k += gridDim.x * NT) {
        int32_t ch = c.node_child[k];
        c.leaf_cnt[k] = ch < 0 ? 1u : c.leaf_cnt[ch] + c.leaf_cnt[ch + 1];
    }
}

__global__ void k_leaf_first(Ctx c, uint32_t a, uint32_t b) {
    for (uint32_t k = a + blockIdx.x * NT + threadIdx.x; k < b; k += gridDim.x * NT) {
        if (k == 0) c.leaf_first[0] = 0;
        int32_t ch = c.node_child[k];
        if (ch >= 0) {
            uint32_t f = k == 0 ? 0u : c.leaf_first[k];
            c.leaf_first[ch] = f;
            c.leaf_first[ch + 1] = f + c.leaf_cnt[ch];
        }
    }
}

__global__ __launch_bounds__(NT) void k_leaf_write(Ctx c, uint32_t num_nodes) {
    __shared__ unsigned long long sh64[NW];
    uint32_t over = 0;
    for (uint32_t k = blockIdx.x * NT + threadIdx.x; k < num_nodes; k += gridDim.x * NT) {
        if (c.node_child[k] < 0) {
            uint32_t f = k == 0 ? 0u : c.leaf_first[k];
            c.leaf_node[f] = k;
            c.leaf_offsets[f] = c.node_begin[k];
            c.node_leaf[k] = f;
            over += (c.node_end[k] - c.node_begin[k]) > c.leaf_size;
        }
    }
    unsigned long long s = block_sum64(over, sh64);
    if (threadIdx.x == 0 && s) atomicAdd(&c.info->oversize, uint32_t(s));
}

__global__ void k_header(Ctx c, uint32_t depth) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const LevelInfo in = *c.info;
    const uint32_t leaves = in.status == KD_OK ? c.leaf_cnt[0] : 0u;
    if (in.status == KD_OK) c.leaf_offsets[leaves] = c.n;
    kd_header h{};
    h.num_nodes = in.num_nodes;
    h.num_leaves = leaves;
    h.depth = depth;
    h.status = in.status;
    h.point_levels = in.point_levels;
    h.unsplittable = in.unsplittable;
    h.oversize = in.oversize;
    *c.hdr = h;
}

// a9: leaf of each query by descent.
__global__ void k_query(const int32_t *child, const uint32_t *dim, const uint32_t *split,
                        const uint32_t *node_leaf, const float *q, uint64_t nq, uint64_t ldq,
                        uint32_t *out) {
    for (uint64_t i = blockIdx.x * uint64_t(NT) + threadIdx.x; i < nq;
         i += uint64_t(gridDim.x) * NT) {
        uint32_t node = 0, res = 0;
        bool nan = false;
        // a valid tree is at most 128 levels deep; the bound also ends the
        // walk on a corrupt node array
        for (int step = 0; step < 256; step++) {
            int32_t ch = child[node];
            if (ch < 0) break;
            uint32_t b = __float_as_uint(q[uint64_t(dim[node]) * ldq + i]);
            if ((b & 0x7fffffffu) > 0x7f800000u) {
                nan = true;
                break;
            }
            node = uint32_t(ch) + (key_of_bits(b) > split[node] ? 1u : 0u);
        }
        res = nan ? NONE : node_leaf[node];
        out[i] = res;
    }
}

// ------------------------------------------------------------ host helpers

bool params_ok(uint64_t n, uint32_t d, const kd_params *p) {
    if (!p || n == 0 || n > 0xffffffffull - TILE || d == 0 || d > 4096) return false;
    if (p->leaf_size == 0 || p->num_subsets == 0 || p->num_subsets > 65536) return false;
    if (p->key_rule > KD_KEY_MAXVAR || p->split_rule > KD_SPLIT_SUBSET) return false;
    if (p->split_rule == KD_SPLIT_FOURIER && (p->fourier_J == 0 || p->fourier_J > 64)) return false;
    if (p->subset_pool && p->pool_entries == 0) return false;
    return true;
}

uint64_t default_capacity(uint64_t n, uint32_t leaf) { return 4 * ((n + leaf - 1) / leaf) + 64; }

uint32_t grid_for(uint64_t work, uint32_t cap = 65535u) {
    if (work == 0) return 1;
    return uint32_t(work < cap ? work : cap);
}

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

#define KD_LAUNCH_CHECK()                                   \
    do {                                                    \
        if (hipGetLastError() != hipSuccess) return KD_EDEVICE; \
    } while (0)

}  // namespace

// ------------------------------------------------------------ C ABI

extern "C" {

int kd_version(void) { return 1; }

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
    if (!params_ok(n, d, params)) return KD_EINVAL;
    uint64_t cap = params->node_capacity ? params->node_capacity
                                         : default_capacity(n, params->leaf_size);
    if (cap > 0xfffffff0ull) return KD_EINVAL;
    Layout L = layout_for(n, d, params->leaf_size, cap);
    if (node_capacity) *node_capacity = cap;
    if (workspace_bytes) *workspace_bytes = L.total;
    return KD_OK;
}

kd_status kd_build_profiled(const float *pts, uint64_t n, uint32_t d, uint64_t ld,
                            const kd_params *p, kd_tree *out, void *workspace, uint64_t ws_bytes,
                            void *stream, kd_profile *prof) {
    if (!params_ok(n, d, p) || !pts || !out || ld < n || !workspace) return KD_EINVAL;
    if (!out->perm || !out->node_begin || !out->node_end || !out->node_child || !out->node_dim ||
        !out->node_split || !out->node_split_f || !out->node_leaf || !out->leaf_node ||
        !out->leaf_offsets || !out->hdr || out->node_capacity == 0)
        return KD_EINVAL;
    if (p->key_rule != KD_KEY_CYCLIC || p->split_rule != KD_SPLIT_EXACT) return KD_EINVAL;
    const uint64_t cap = out->node_capacity;
    if (cap > 0xfffffff0ull) return KD_EINVAL;
    Layout L = layout_for(n, d, p->leaf_size, cap);
    if (ws_bytes < L.total) return KD_ENOMEM;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    char *ws = static_cast<char *>(workspace);
    Prof P(prof, st);

    Ctx c{};
    for (int b = 0; b < 2; b++) {
        c.cols[b] = reinterpret_cast<uint32_t *>(ws + L.off_cols[b]);
        c.perm[b] = reinterpret_cast<uint32_t *>(ws + L.off_perm[b]);
        c.cells[b] = reinterpret_cast<Cell *>(ws + L.off_cells[b]);
    }
    c.res = reinterpret_cast<CellRes *>(ws + L.off_res);
    c.tile_left = reinterpret_cast<uint32_t *>(ws + L.off_tile_left);
    c.tile_off = reinterpret_cast<uint32_t *>(ws + L.off_tile_off);
    c.hist = reinterpret_cast<uint32_t *>(ws + L.off_hist);
    c.scan_tmp = reinterpret_cast<uint32_t *>(ws + L.off_scan);
    c.info = reinterpret_cast<LevelInfo *>(ws + L.off_info);
    c.leaf_cnt = reinterpret_cast<uint32_t *>(ws + L.off_leaf_cnt);
    c.leaf_first = reinterpret_cast<uint32_t *>(ws + L.off_leaf_first);
    c.out_perm = out->perm;
    c.pts_out = reinterpret_cast<uint32_t *>(out->points_out);
    c.node_begin = out->node_begin;
    c.node_end = out->node_end;
    c.node_child = out->node_child;
    c.node_dim = out->node_dim;
    c.node_split = out->node_split;
    c.node_split_f = out->node_split_f;
    c.node_leaf = out->node_leaf;
    c.leaf_node = out->leaf_node;
    c.leaf_offsets = out->leaf_offsets;
    c.hdr = out->hdr;
    c.cap = cap;
    c.n = uint32_t(n);
    c.d = d;
    c.leaf_size = p->leaf_size;
    c.max_depth = p->max_depth ? p->max_depth : 64;
    c.key_rule = p->key_rule;
    c.split_rule = p->split_rule;
    c.J = p->fourier_J;
    c.S = p->num_subsets;

    const uint64_t scatter_bpp = 8ull * d + 8;  // algorithmic bytes per point of a scatter
    const uint32_t root_active = (n > p->leaf_size && c.max_depth > 0) ? 1u : 0u;
    P.run(KD_PROF_OTHER, 0, 0, [&] {
        hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(L.hist_words / NT + 1, 4096)), dim3(NT), 0,
                           st, c.hist, L.hist_words, 0u);
        hipLaunchKernelGGL(k_init, dim3(grid_for(cap / NT + 1, 4096)), dim3(NT), 0, st, c,
                           root_active);
    });
    P.run(KD_PROF_INGEST, n, n * (8ull * d + 4), [&] {
        hipLaunchKernelGGL(k_ingest, dim3(grid_for(n / (NT * 4) + 1, 1024), d), dim3(NT), 0, st,
                           c, pts, ld);
    });
    KD_LAUNCH_CHECK();

    // level loop; node ids of depth l are [level_first[l], level_first[l + 1])
    uint32_t level_first[130];
    uint32_t nlevels = 1;  // depths holding nodes
    level_first[0] = 0;
    level_first[1] = 1;
    LevelInfo hi{};
    if (!root_active) {
        P.run(KD_PROF_OTHER, n, 0, [&] {
            hipLaunchKernelGGL(k_copy_all, dim3(grid_for(n / NT + 1, 4096)), dim3(NT), 0, st, c);
        });
        KD_LAUNCH_CHECK();
    }
    uint32_t levels_run = 0;
    for (uint32_t level = 0;; level++) {
        if (hipMemcpyAsync(&hi, c.info, sizeof(hi), hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess)
            return KD_EDEVICE;
        if (level > 0 && hi.splits > 0) {
            level_first[nlevels + 1] = hi.num_nodes;
            nlevels++;
        }
        if (hi.status != KD_OK || hi.num_cells == 0 || level >= 128) break;
        levels_run++;
        const uint32_t nc = hi.num_cells, ntl = hi.num_tiles;
        const uint64_t bigp = hi.big_points, smallp = hi.points - hi.big_points;
        P.run(KD_PROF_OTHER, 0, 0, [&] {
            hipLaunchKernelGGL(k_level_init, dim3(grid_for(nc / NT + 1, 4096)), dim3(NT), 0, st,
                               c, level, nc);
        });
        if (ntl > 0) {
            for (uint32_t pass = 0; pass < uint32_t(RPASSES); pass++) {
                P.run(KD_PROF_SELECT, bigp, 4 * bigp, [&] {
                    hipLaunchKernelGGL(k_big_hist, dim3(grid_for(ntl, 65535)), dim3(NT), 0, st, c,
                                       level, pass, nc, ntl);
                });
                P.run(KD_PROF_PICK, 0, 0, [&] {
                    hipLaunchKernelGGL(k_big_pick, dim3(grid_for(nc, 65535)), dim3(NT), 0, st, c,
                                       level, pass, nc);
                });
            }
            P.run(KD_PROF_COUNT, bigp, 4 * bigp, [&] {
                hipLaunchKernelGGL(k_big_count, dim3(grid_for(ntl, 65535)), dim3(NT), 0, st, c,
                                   level, nc, ntl);
                hipLaunchKernelGGL(k_big_tilescan, dim3(grid_for(nc, 65535)), dim3(NT), 0, st, c,
                                   level, nc);
            });
            P.run(KD_PROF_BIG_SCATTER, bigp, scatter_bpp * bigp, [&] {
                hipLaunchKernelGGL(k_big_scatter, dim3(grid_for(ntl, 65535)), dim3(NT), 0, st, c,
                                   level, nc, ntl);
            });
        }
        if (smallp > 0) {
            P.run(KD_PROF_SMALL, smallp, scatter_bpp * smallp, [&] {
                hipLaunchKernelGGL(k_small, dim3(grid_for(nc, 1u << 20)), dim3(NT), 0, st, c, level,
                                   nc);
            });
        }
        const uint32_t nb = (nc + NT - 1) / NT;
        P.run(KD_PROF_EMIT, 0, 0, [&] {
            hipLaunchKernelGGL(k_emit_sum, dim3(nb), dim3(NT), 0, st, c, level, nc);
            hipLaunchKernelGGL(k_emit_scan, dim3(1), dim3(NT), 0, st, c, level, nb);
            hipLaunchKernelGGL(k_emit_write, dim3(nb), dim3(NT), 0, st, c, level, nc);
        });
        KD_LAUNCH_CHECK();
    }
    const uint32_t depth = nlevels - 1;
    P.run(KD_PROF_OTHER, 0, 0, [&] {
        if (hi.status == KD_OK) {
            for (int l = int(nlevels) - 1; l >= 0; l--) {
                uint32_t a = level_first[l], b = level_first[l + 1];
                hipLaunchKernelGGL(k_leaf_count, dim3(grid_for((b - a) / NT + 1, 4096)), dim3(NT),
                                   0, st, c, a, b);
            }
            for (uint32_t l = 0; l < nlevels; l++) {
                uint32_t a = level_first[l], b = level_first[l + 1];
                hipLaunchKernelGGL(k_leaf_first, dim3(grid_for((b - a) / NT + 1, 4096)), dim3(NT),
                                   0, st, c, a, b);
            }
            hipLaunchKernelGGL(k_leaf_write, dim3(grid_for(hi.num_nodes / NT + 1, 4096)), dim3(NT),
                               0, st, c, hi.num_nodes);
        }
        hipLaunchKernelGGL(k_header, dim3(1), dim3(64), 0, st, c, depth);
    });
    KD_LAUNCH_CHECK();
    if (!P.finish(levels_run)) return KD_EDEVICE;
    return KD_OK;
}

kd_status kd_build(const float *pts, uint64_t n, uint32_t d, uint64_t ld, const kd_params *p,
                   kd_tree *out, void *workspace, uint64_t ws_bytes, void *stream) {
    return kd_build_profiled(pts, n, d, ld, p, out, workspace, ws_bytes, stream, nullptr);
}

kd_status kd_query_leaf(const kd_tree *tree, const float *q, uint64_t nq, uint32_t d,
                        uint64_t ldq, uint32_t *leaf_out, void *stream) {
    if (!tree || !q || !leaf_out || d == 0 || ldq < nq || !tree->node_child || !tree->node_dim ||
        !tree->node_split || !tree->node_leaf)
        return KD_EINVAL;
    if (nq == 0) return KD_OK;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    hipLaunchKernelGGL(k_query, dim3(grid_for(nq / NT + 1, 65535)), dim3(NT), 0, st,
                       tree->node_child, tree->node_dim, tree->node_split, tree->node_leaf, q, nq,
                       ldq, leaf_out);
    KD_LAUNCH_CHECK();
    return KD_OK;
}

kd_status kd_batch_bounds(uint32_t count, const kd_batch_item *items, const kd_params *params,
                          uint64_t *workspace_bytes) {
    if (count == 0 || !items || !params || !workspace_bytes) return KD_EINVAL;
    uint64_t mx = 0;
    for (uint32_t t = 0; t < count; t++) {
        uint64_t cap, ws;
        kd_status s = kd_tree_bounds(items[t].n, items[t].d, params, &cap, &ws);
        if (s != KD_OK) return s;
        if (ws > mx) mx = ws;
    }
    *workspace_bytes = mx;
    return KD_OK;
}

kd_status kd_build_batched(uint32_t count, const kd_batch_item *items, const kd_params *params,
                           void *workspace, uint64_t ws_bytes, void *stream) {
    if (count == 0 || !items || !params) return KD_EINVAL;
    for (uint32_t t = 0; t < count; t++) {
        kd_tree o = items[t].out;
        kd_status s = kd_build(items[t].pts, items[t].n, items[t].d, items[t].ld, params, &o,
                               workspace, ws_bytes, stream);
        if (s != KD_OK) return s;
    }
    return KD_OK;
}

}  // extern "C"

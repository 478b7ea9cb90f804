// kd_query.hpp -- queries that use a built tree (§1 and §2: the cells of the
// tree answer nearest-neighbour and range questions): exact k nearest
// neighbours (one wave per query) and axis-aligned box search (one thread
// per box), by a depth-first walk with an explicit stack.
//
// Cells: a node with split key s sends points with key <= s left and the rest
// right, so its left child's region along the node's coordinate is
// {x : key(x) <= s} and the right child's is {x : key(x) > s}.  With s_f the
// float of key s, every left point has x <= s_f and every right point x > s_f.
#pragma once
#include "kd_device.hpp"

namespace kd {

constexpr uint32_t KNN_MAX = 64;             // largest k of a neighbour query
constexpr int QUERY_STACK = MAX_LEVELS + 2;  // a walk holds at most one entry per depth

// (distance, point index) order of the neighbour lists.
__device__ __forceinline__ bool knn_less(double da, uint32_t ia, double db, uint32_t ib) {
    return da < db || (da == db && ia < ib);
}

// One wave per query: the k nearest points of the tree, ascending by
// (squared distance, original index).  Lane j holds the j-th entry of the
// list; the 64 lanes take a leaf's points 64 at a time (coalesced reads) and
// the candidates that beat the current k-th entry are inserted one by one.
// The walk's stack is the wave's part of LDS (every lane writes the same
// entry, so each lane reads back its own store).  pts: the tree's points in
// position order [d][n]; perm: original index of each position.  Fewer than
// k points: the list ends with (NONE, +inf).  A query with a NaN coordinate
// gets (NONE, NaN) throughout.
//
// Bound of a far child: with d <= 64, lane c holds the query's distance to
// the current cell's box along coordinate c, and a far child's bound is the
// squared distance to its box (the cell's bound with coordinate c's term
// replaced by the gap to the split plane); a stack entry restores the
// coordinate's distance once that subtree is done.  With larger d the bound
// is the largest squared gap on the path.  A child is skipped only when its
// bound exceeds the k-th distance by a relative margin far above the
// rounding of these sums, so ties and rounding never drop a point.
constexpr int KNN_BOX_DIMS = WAVE;
__device__ __forceinline__ bool knn_visit(double lb, double worst) {
    return lb <= worst + worst * 0x1p-30;
}

__global__ __launch_bounds__(NT) void k_knn(const int32_t *child, const uint32_t *dim,
                                            const uint32_t *split, const float *split_f,
                                            const uint32_t *nbeg, const uint32_t *nend,
                                            const float *pts, uint64_t n, const uint32_t *perm,
                                            const float *q, uint64_t nq, uint32_t d, uint64_t ldq,
                                            uint32_t k, uint32_t *idx_out, double *dist_out) {
    // stack entry: a node to visit (with its bound, and the coordinate whose
    // box distance changes there), or (NONE) a coordinate distance to restore
    __shared__ uint32_t snode_all[NW][QUERY_STACK], sdim_all[NW][QUERY_STACK];
    __shared__ double slb_all[NW][QUERY_STACK], soff_all[NW][QUERY_STACK];
    uint32_t *snode = snode_all[wave()], *sdim = sdim_all[wave()];
    double *slb = slb_all[wave()], *soff = soff_all[wave()];
    const int l = lane();
    const bool box = d <= uint32_t(KNN_BOX_DIMS);
    for (uint64_t i = blockIdx.x * uint64_t(NW) + wave(); i < nq; i += uint64_t(gridDim.x) * NW) {
        bool nan = false;
        for (uint32_t c = l; c < d; c += WAVE) {
            const float v = q[uint64_t(c) * ldq + i];
            nan |= v != v;
        }
        if (__any(nan)) {
            for (uint32_t j = l; j < k; j += WAVE) {
                idx_out[i * k + j] = NONE;
                dist_out[i * k + j] = __builtin_nan("");
            }
            continue;
        }
        double bd = __builtin_inf();  // this lane's list entry
        uint32_t bi = NONE;
        double worst = __builtin_inf();  // the k-th entry (lane k - 1)
        uint32_t worst_i = NONE;
        double off = 0.0;  // lane c: distance to the current cell's box along c
        snode[0] = 0;
        slb[0] = 0.0;
        sdim[0] = 0;
        soff[0] = 0.0;
        int sp = 1;
        while (sp > 0) {
            sp--;
            uint32_t node = snode[sp];
            const uint32_t ec = sdim[sp];
            const double eoff = soff[sp];
            if (node == NONE) {  // leaving a far subtree
                if (uint32_t(l) == ec) off = eoff;
                continue;
            }
            double lb = slb[sp];
            if (!knn_visit(lb, worst)) continue;
            if (box && node != 0) {
                // entering a far child: its box distance along ec; restore later
                const double old = __shfl(off, int(ec), WAVE);
                snode[sp] = NONE;
                sdim[sp] = ec;
                soff[sp] = old;
                sp++;
                if (uint32_t(l) == ec) off = eoff;
            }
            for (int step = 0; step <= MAX_LEVELS; step++) {
                const int32_t ch = child[node];
                if (ch < 0) break;
                const uint32_t c = dim[node];
                const float qv = q[uint64_t(c) * ldq + i];
                const bool left = key_of_bits(__float_as_uint(qv)) <= split[node];
                double gap = double(split_f[node]) - double(qv);
                gap = gap < 0.0 ? -gap : gap;
                gap = gap != gap ? 0.0 : gap;  // no bound from infinite coordinates
                double flb;
                if (box) {
                    const double oc = __shfl(off, int(c), WAVE);
                    flb = lb - oc * oc + gap * gap;
                    flb = flb > lb ? flb : lb;
                } else {
                    flb = gap * gap;
                    flb = flb > lb ? flb : lb;
                }
                if (knn_visit(flb, worst) && sp < QUERY_STACK) {
                    snode[sp] = uint32_t(ch) + (left ? 1u : 0u);
                    slb[sp] = flb;
                    sdim[sp] = c;
                    soff[sp] = gap;
                    sp++;
                }
                node = uint32_t(ch) + (left ? 0u : 1u);
            }
            const uint32_t pb = nbeg[node], pe = nend[node];
            for (uint32_t p0 = pb; p0 < pe; p0 += WAVE) {
                const uint32_t p = p0 + l;
                double dv = __builtin_inf();
                uint32_t id = NONE;
                if (p < pe) {
                    // squared distance in fp64, summed in coordinate order (no
                    // fused operations: the build compiles with contraction
                    // off); a NaN sum (infinite coordinates) counts as +inf
                    dv = 0.0;
                    for (uint32_t c = 0; c < d; c++) {
                        const double t = double(pts[uint64_t(c) * n + p]) - double(q[uint64_t(c) * ldq + i]);
                        dv = dv + t * t;
                    }
                    dv = dv != dv ? __builtin_inf() : dv;
                    id = perm[p];
                }
                bool cand = p < pe && knn_less(dv, id, worst, worst_i);
                for (unsigned long long m = __ballot(cand); m; m = __ballot(cand)) {
                    const int src = __builtin_ctzll(m);
                    const double cd = __shfl(dv, src, WAVE);
                    const uint32_t cidx = __shfl(id, src, WAVE);
                    if (l == src) cand = false;
                    if (!knn_less(cd, cidx, worst, worst_i)) continue;  // the list moved on
                    // lanes at or after the candidate's place shift up by one
                    const bool after = !knn_less(bd, bi, cd, cidx);
                    const double ud = __shfl_up(bd, 1, WAVE);
                    const uint32_t ui = __shfl_up(bi, 1, WAVE);
                    const bool prev_after = __shfl_up(after ? 1 : 0, 1, WAVE) != 0 && l > 0;
                    if (after) {
                        bd = prev_after ? ud : cd;
                        bi = prev_after ? ui : cidx;
                    }
                    worst = __shfl(bd, int(k) - 1, WAVE);
                    worst_i = __shfl(bi, int(k) - 1, WAVE);
                }
            }
        }
        if (uint32_t(l) < k) {
            idx_out[i * k + l] = bi;
            dist_out[i * k + l] = bd;
        }
    }
}

// One thread per box [lo, hi] (inclusive in every coordinate): the number of
// points inside, and with `ids` their original indices in tree position
// order, written from offsets[i].  A box with a NaN bound holds nothing.
__global__ void k_box(const int32_t *child, const uint32_t *dim, const uint32_t *split,
                      const uint32_t *nbeg, const uint32_t *nend, const float *pts, uint64_t n,
                      const uint32_t *perm, const float *lo, const float *hi, uint64_t nb,
                      uint32_t d, uint64_t ldb, uint32_t *count, const uint64_t *offsets,
                      uint32_t *ids) {
    for (uint64_t i = blockIdx.x * uint64_t(NT) + threadIdx.x; i < nb;
         i += uint64_t(gridDim.x) * NT) {
        bool nan = false;
        for (uint32_t c = 0; c < d; c++) {
            const float a = lo[uint64_t(c) * ldb + i], b = hi[uint64_t(c) * ldb + i];
            nan |= a != a || b != b;
        }
        uint32_t found = 0;
        uint32_t *out = ids ? ids + offsets[i] : nullptr;
        uint32_t snode[QUERY_STACK];
        int sp = 0;
        if (!nan) snode[sp++] = 0;
        while (sp > 0) {
            uint32_t node = snode[--sp];
            bool reach = true;
            for (int step = 0; step <= MAX_LEVELS; step++) {
                const int32_t ch = child[node];
                if (ch < 0) break;
                const uint32_t c = dim[node];
                const bool go_l = key_of_bits(__float_as_uint(lo[uint64_t(c) * ldb + i])) <= split[node];
                const bool go_r = key_of_bits(__float_as_uint(hi[uint64_t(c) * ldb + i])) > split[node];
                if (go_l && go_r && sp < QUERY_STACK) snode[sp++] = uint32_t(ch) + 1u;
                if (!go_l && !go_r) {
                    reach = false;
                    break;
                }
                node = uint32_t(ch) + (go_l ? 0u : 1u);
            }
            if (!reach) continue;
            for (uint32_t p = nbeg[node]; p < nend[node]; p++) {
                bool in = true;
                for (uint32_t c = 0; c < d && in; c++) {
                    const uint32_t x = key_of_bits(__float_as_uint(pts[uint64_t(c) * n + p]));
                    in = key_of_bits(__float_as_uint(lo[uint64_t(c) * ldb + i])) <= x &&
                         x <= key_of_bits(__float_as_uint(hi[uint64_t(c) * ldb + i]));
                }
                if (in) {
                    if (out) out[found] = perm[p];
                    found++;
                }
            }
        }
        count[i] = found;
    }
}

}  // namespace kd

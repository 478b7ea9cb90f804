// kd_query.hpp -- queries that use a built tree (§1 and §2: the cells of the
// tree answer nearest-neighbour and range questions): exact k nearest
// neighbours and axis-aligned box search, one query per thread, by a
// depth-first walk with an explicit stack.
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

// Squared Euclidean distance in fp64, summed in coordinate order (no fused
// operations: the build compiles with contraction off).  A NaN sum (from
// infinite coordinates) counts as +inf.
__device__ __forceinline__ double knn_dist(const float *pts, uint64_t n, uint64_t p,
                                           const float *q, uint64_t ldq, uint64_t i, uint32_t d) {
    double s = 0.0;
    for (uint32_t c = 0; c < d; c++) {
        const double t = double(pts[uint64_t(c) * n + p]) - double(q[uint64_t(c) * ldq + i]);
        s = s + t * t;
    }
    return s != s ? __builtin_inf() : s;
}

// (distance, point index) order of the neighbour lists.
__device__ __forceinline__ bool knn_less(double da, uint32_t ia, double db, uint32_t ib) {
    return da < db || (da == db && ia < ib);
}

// One thread per query: the k nearest points of the tree, ascending by
// (squared distance, original index).  pts: the tree's points in position
// order [d][n]; perm: original index of each position.  Fewer than k points:
// the rest of the list is (NONE, +inf).  A query with a NaN coordinate gets
// (NONE, NaN) throughout.
__global__ void k_knn(const int32_t *child, const uint32_t *dim, const uint32_t *split,
                      const float *split_f, const uint32_t *nbeg, const uint32_t *nend,
                      const float *pts, uint64_t n, const uint32_t *perm, const float *q,
                      uint64_t nq, uint32_t d, uint64_t ldq, uint32_t k, uint32_t *idx_out,
                      double *dist_out) {
    for (uint64_t i = blockIdx.x * uint64_t(NT) + threadIdx.x; i < nq;
         i += uint64_t(gridDim.x) * NT) {
        uint32_t *io = idx_out + i * k;
        double *dout = dist_out + i * k;
        bool nan = false;
        for (uint32_t c = 0; c < d; c++) {
            const float v = q[uint64_t(c) * ldq + i];
            nan |= v != v;
        }
        if (nan) {
            for (uint32_t j = 0; j < k; j++) {
                io[j] = NONE;
                dout[j] = __builtin_nan("");
            }
            continue;
        }
        double bd[KNN_MAX];
        uint32_t bi[KNN_MAX];
        uint32_t m = 0;  // entries in the list
        uint32_t snode[QUERY_STACK];
        double slb[QUERY_STACK];
        int sp = 0;
        snode[sp] = 0;
        slb[sp] = 0.0;
        sp++;
        while (sp > 0) {
            sp--;
            uint32_t node = snode[sp];
            const double lb = slb[sp];
            if (m == k && lb > bd[k - 1]) continue;
            // down to a leaf, keeping each far child with its lower bound
            for (int step = 0; step <= MAX_LEVELS; step++) {
                const int32_t ch = child[node];
                if (ch < 0) break;
                const uint32_t c = dim[node];
                const float qv = q[uint64_t(c) * ldq + i];
                const bool left = key_of_bits(__float_as_uint(qv)) <= split[node];
                const double gap = double(split_f[node]) - double(qv);
                double flb = gap * gap;
                flb = flb != flb ? 0.0 : flb;  // no bound from infinite coordinates
                flb = flb > lb ? flb : lb;
                const uint32_t far = uint32_t(ch) + (left ? 1u : 0u);
                if ((m < k || flb <= bd[k - 1]) && sp < QUERY_STACK) {
                    snode[sp] = far;
                    slb[sp] = flb;
                    sp++;
                }
                node = uint32_t(ch) + (left ? 0u : 1u);
            }
            for (uint32_t p = nbeg[node]; p < nend[node]; p++) {
                const double dv = knn_dist(pts, n, p, q, ldq, i, d);
                const uint32_t id = perm[p];
                if (m == k && !knn_less(dv, id, bd[k - 1], bi[k - 1])) continue;
                uint32_t j = m < k ? m++ : k - 1;  // insertion from the end
                while (j > 0 && knn_less(dv, id, bd[j - 1], bi[j - 1])) {
                    bd[j] = bd[j - 1];
                    bi[j] = bi[j - 1];
                    j--;
                }
                bd[j] = dv;
                bi[j] = id;
            }
        }
        for (uint32_t j = 0; j < k; j++) {
            io[j] = j < m ? bi[j] : NONE;
            dout[j] = j < m ? bd[j] : __builtin_inf();
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

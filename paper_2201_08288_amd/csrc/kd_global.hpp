// kd_global.hpp -- the paper's global single-pass construction (§3.2 with
// Eq. (1) and (2); App. C, basic form): one pass over points in (0,1)^p sums
// C_j = sum_i prod_l c_{j_l}(x_il) for every j in {0..2J}^p; each median of a
// depth-D tree is then the solution of Eq. (2) for its cell box, computed
// from the C_j alone.
//
// Map step: per point and coordinate the basis c_0 = 1, c_{2j-1} =
// cos((2j-1)u), c_{2j} = sin((2j-1)u) in fp32 (own series and the harmonic
// recurrence), each quantised as rint(c * Q_p) with Q_1 = 2^24, Q_2 = 2^15,
// Q_3 = 2^10.  Every product of p quantised values is an integer of at most
// 2^30; a workgroup adds at most 2^23 points' products in fp64 (exact: every
// partial sum is an integer below 2^53), converts once to int64 and adds
// atomically, so the statistics are exact and independent of how the points
// are split (the paper's map-reduce).
// Solve step: for a cell (a, b) split on coordinate t, the statistics are
// contracted with the Lemma 3.1 weights g_j(a_l, b_l) of the other
// coordinates (fp64, fixed order), and Eq. (2) becomes F(m) = 0 with
//   F(m) = sum_j D_j (g_j(a_t, m) - g_j(m, b_t)),
// solved by bisection in fp64 from (a_t, b_t).
#pragma once
#include "kd_fourier.hpp"

namespace kd {

constexpr int GLOBAL_JMAX = 15;
constexpr int GLOBAL_EP = 32;           // basis entries per coordinate, padded (2J+1 <= 31)
constexpr int GLOBAL_CHUNK = 64;        // points staged in LDS per step
constexpr int GLOBAL_MAX_DEPTH = 12;
constexpr uint64_t GLOBAL_EXACT_POINTS = 1ull << 23;  // per workgroup: fp64 sums stay exact

__host__ __device__ constexpr float global_quantum(int p) {
    return p == 1 ? 16777216.0f : (p == 2 ? 32768.0f : 1024.0f);
}

// Quantised basis of one coordinate value (integers, stored as OUT);
// q[2J+1 .. GLOBAL_EP) = 0.
template <class OUT>
__device__ __forceinline__ void global_basis(float u, int J, float Q, const TrigTables &T, OUT *q) {
    float s1, c1;
    sincos32(u, T, s1, c1);
    const float ss = s1 * s1;
    const float C2 = 1.0f - 2.0f * ss;
    const float sc = s1 * c1;
    const float S2 = 2.0f * sc;
    float cj = c1, sj = s1;
    q[0] = OUT(Q);
    for (int j = 0; j < J; j++) {
        q[2 * j + 1] = OUT(rintf(cj * Q));
        q[2 * j + 2] = OUT(rintf(sj * Q));
        const float a = cj * C2, b = sj * S2;
        const float g = sj * C2, h = cj * S2;
        cj = a - b;
        sj = g + h;
    }
    for (int k = 2 * J + 1; k < GLOBAL_EP; k++) q[k] = OUT(0);
}

// Map step for p = 1 and 2 (p = 3 runs on the matrix cores, below).  Thread
// item (a, b): the row of entries (a, b, 0 .. 2J) of the statistics for p = 3
// (first coordinate slowest); for p = 2 the row (b, .), for p = 1 the only row.  The staged basis is fp64 in LDS: the row's values
// are the same for every lane (broadcast reads), a and b differ.  Grid: (row
// groups, point ranges of `per` points each, per <= GLOBAL_EXACT_POINTS).
// C: int64 as uint64, added to.
template <int P>
__global__ __launch_bounds__(NT) void k_gmom(const float *pts, uint64_t n, uint64_t ld, uint32_t J,
                                             uint64_t per, TrigTables T, unsigned long long *C) {
    __shared__ __attribute__((aligned(16))) double q[P][GLOBAL_CHUNK][GLOBAL_EP];
    const uint32_t E = 2 * J + 1;
    const float Q = global_quantum(P);
    const uint32_t rows = (P >= 3 ? E : 1u) * (P >= 2 ? E : 1u);
    const uint32_t item = blockIdx.x * NT + threadIdx.x;
    const bool active = item < rows;
    const uint32_t b = P >= 2 ? item % E : 0u, a = P >= 3 ? item / E : 0u;
    double acc[GLOBAL_EP];
#pragma unroll
    for (int k = 0; k < GLOBAL_EP; k++) acc[k] = 0.0;
    const uint64_t p0 = uint64_t(blockIdx.y) * per;
    const uint64_t p1 = p0 + per < n ? p0 + per : n;
    for (uint64_t c0 = p0; c0 < p1; c0 += GLOBAL_CHUNK) {
        const uint32_t m = uint32_t(p1 - c0 < GLOBAL_CHUNK ? p1 - c0 : GLOBAL_CHUNK);
        __syncthreads();  // the previous chunk is consumed
        for (uint32_t w = threadIdx.x; w < uint32_t(P * GLOBAL_CHUNK); w += NT) {
            const uint32_t c = w / GLOBAL_CHUNK, i = w % GLOBAL_CHUNK;
            if (i < m) global_basis(pts[uint64_t(c) * ld + c0 + i], int(J), Q, T, q[c][i]);
        }
        __syncthreads();
        if (active) {
            for (uint32_t i = 0; i < m; i++) {
                const double qa = P >= 3 ? q[0][i][a] : 1.0;
                const double qb = P >= 2 ? q[P >= 2 ? P - 2 : 0][i][b] : 1.0;
                const double qab = qa * qb;
                const double2 *row = reinterpret_cast<const double2 *>(q[P - 1][i]);
#pragma unroll
                for (int k = 0; k < GLOBAL_EP / 2; k++) {
                    const double2 x = row[k];
                    acc[2 * k] = __fma_rn(qab, x.x, acc[2 * k]);
                    acc[2 * k + 1] = __fma_rn(qab, x.y, acc[2 * k + 1]);
                }
            }
        }
    }
    if (!active) return;
    const uint64_t base = P == 3 ? (uint64_t(a) * E + b) * E : (P == 2 ? uint64_t(b) * E : 0u);
#pragma unroll
    for (int k = 0; k < GLOBAL_EP; k++)
        if (uint32_t(k) < E && acc[k] != 0.0)
            atomicAdd(&C[base + uint32_t(k)], (unsigned long long)(long long)acc[k]);
}

// Map step for p = 3 on the matrix cores.  The statistics are the product
// C[(a, b), c] = sum_i A[(a, b), i] B[i, c] of A = q_a(x_i) q_b(y_i) (E^2 rows,
// E = 2J + 1) and B = q_c(z_i) (E columns, padded to 32).  One workgroup of
// 16 waves holds every row: wave w owns rows 64w .. 64w + 63 (four 16-row
// tiles) and both 16-column tiles; each fp64 16x16x4 MFMA adds four points.
// Operand layout of that instruction: lane l holds A[l % 16][l / 16] and
// B[l / 16][l % 16], and its accumulator register r holds row l / 16 + 4r,
// column l % 16.  Every operand, product and partial sum is an integer below
// 2^53 (at most GLOBAL_EXACT_POINTS points per workgroup), so the sums are
// exact whatever order the matrix core adds them in.  Grid: (1, point ranges
// of `per` points each).  C: int64 as uint64, added to.
constexpr int GMM_NT = 1024;
constexpr int GMM_STRIDE = GLOBAL_EP + 2;  // LDS row stride in doubles: a step's four points fall in different banks
typedef double gmm_acc __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(GMM_NT) void k_gmom3_mfma(const float *pts, uint64_t n, uint64_t ld,
                                                      uint32_t J, uint64_t per, TrigTables T,
                                                      unsigned long long *C) {
    __shared__ __attribute__((aligned(16))) double q[3][GLOBAL_CHUNK][GMM_STRIDE];
    const uint32_t E = 2 * J + 1, rows = E * E;
    const float Q = global_quantum(3);
    const uint32_t w = threadIdx.x / WAVE, l = threadIdx.x % WAVE;
    const uint32_t lr = l % 16, lk = l / 16;
    uint32_t ra[4], rb[4];
    bool rv[4];
#pragma unroll
    for (int t = 0; t < 4; t++) {
        const uint32_t R = 64 * w + 16 * t + lr;
        rv[t] = R < rows;
        ra[t] = rv[t] ? R / E : 0u;
        rb[t] = rv[t] ? R % E : 0u;
    }
    gmm_acc acc[4][2];
#pragma unroll
    for (int t = 0; t < 4; t++)
#pragma unroll
        for (int u = 0; u < 2; u++) acc[t][u] = gmm_acc{0.0, 0.0, 0.0, 0.0};
    const uint64_t p0 = uint64_t(blockIdx.y) * per;
    const uint64_t p1 = p0 + per < n ? p0 + per : n;
    for (uint64_t c0 = p0; c0 < p1; c0 += GLOBAL_CHUNK) {
        const uint32_t m = uint32_t(p1 - c0 < GLOBAL_CHUNK ? p1 - c0 : GLOBAL_CHUNK);
        __syncthreads();  // the previous chunk is consumed
        for (uint32_t wk = threadIdx.x; wk < uint32_t(3 * GLOBAL_CHUNK); wk += GMM_NT) {
            const uint32_t c = wk / GLOBAL_CHUNK, i = wk % GLOBAL_CHUNK;
            double *row = q[c][i];
            if (i < m) {
                global_basis(pts[uint64_t(c) * ld + c0 + i], int(J), Q, T, row);
            } else {  // past the range: a zero row adds nothing
                for (int e = 0; e < GLOBAL_EP; e++) row[e] = 0.0;
            }
        }
        __syncthreads();
        for (uint32_t s = 0; s < uint32_t(GLOBAL_CHUNK / 4); s++) {
            const uint32_t i = 4 * s + lk;
            const double b0 = q[2][i][lr], b1 = q[2][i][16 + lr];
#pragma unroll
            for (int t = 0; t < 4; t++) {
                const double a = rv[t] ? q[0][i][ra[t]] * q[1][i][rb[t]] : 0.0;
                acc[t][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b0, acc[t][0], 0, 0, 0);
                acc[t][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b1, acc[t][1], 0, 0, 0);
            }
        }
    }
#pragma unroll
    for (int t = 0; t < 4; t++)
#pragma unroll
        for (int u = 0; u < 2; u++)
#pragma unroll
            for (int r = 0; r < 4; r++) {
                const uint32_t R = 64 * w + 16 * t + lk + 4 * r, col = 16 * u + lr;
                const double v = acc[t][u][r];
                if (R < rows && col < E && v != 0.0)
                    atomicAdd(&C[uint64_t(R) * E + col], (unsigned long long)(long long)v);
            }
}

// sin((2j-1)x), cos((2j-1)x), j = 1..J (fp64, own series, recurrence).
__device__ __forceinline__ void global_harmonics(double x, int J, const TrigTables &T, double *s,
                                                 double *c) {
    double s1, c1;
    sincos64(x, T, s1, c1);
    const double ss = s1 * s1;
    const double C2 = 1.0 - 2.0 * ss;
    const double sc = s1 * c1;
    const double S2 = 2.0 * sc;
    double cj = c1, sj = s1;
    for (int j = 0; j < J; j++) {
        s[j] = sj;
        c[j] = cj;
        const double a = cj * C2, b = sj * S2;
        const double g = sj * C2, h = cj * S2;
        cj = a - b;
        sj = g + h;
    }
}

// g_0 .. g_{2J} of Lemma 3.1 for the interval (a, b) of (0, 1).
__device__ __forceinline__ void global_g(double a, double b, int J, const TrigTables &T, double *g) {
    double sa[GLOBAL_JMAX], ca[GLOBAL_JMAX], sb[GLOBAL_JMAX], cb[GLOBAL_JMAX];
    const bool ia = a > 0.0, ib = b < 1.0;
    global_harmonics(a, J, T, sa, ca);
    global_harmonics(b, J, T, sb, cb);
    g[0] = 1.0 - 0.5 * double(int(ia) + int(ib));
    for (int j = 1; j <= J; j++) {
        const double k = 2.0 / (3.14159265358979323846 * double(2 * j - 1));
        const double s_b = ib ? sb[j - 1] : 0.0, s_a = ia ? sa[j - 1] : 0.0;
        const double c_a = ia ? ca[j - 1] : 0.0, c_b = ib ? cb[j - 1] : 0.0;
        g[2 * j - 1] = k * (s_b - s_a);
        g[2 * j] = k * (c_a - c_b);
    }
}

// One point's harmonics sin((2j-1)x), cos((2j-1)x), advanced one j at a
// time by the same recurrence as global_harmonics (identical values).
struct GlobalHarm {
    double s, c, C2, S2;
    __device__ __forceinline__ GlobalHarm(double x, const TrigTables &T) {
        double s1, c1;
        sincos64(x, T, s1, c1);
        const double ss = s1 * s1;
        C2 = 1.0 - 2.0 * ss;
        const double sc = s1 * c1;
        S2 = 2.0 * sc;
        s = s1;
        c = c1;
    }
    __device__ __forceinline__ void next() {
        const double a = c * C2, b = s * S2;
        const double g = s * C2, h = c * S2;
        c = a - b;
        s = g + h;
    }
};

// F(m) = sum_j D_j (g_j(at, m) - g_j(m, bt)), the terms of g taken as in
// global_g and summed in order j = 0 .. 2J, one harmonic at a time (no
// arrays, so nothing is spilled).
__device__ __forceinline__ double global_F(const double *D, int J, const TrigTables &T, double at,
                                           double bt, double m) {
    GlobalHarm ha(at, T), hm(m, T), hb(bt, T);
    const bool la = at > 0.0, lb = m < 1.0;  // left interval (at, m)
    const bool ra = m > 0.0, rb = bt < 1.0;  // right interval (m, bt)
    const double gl0 = 1.0 - 0.5 * double(int(la) + int(lb));
    const double gr0 = 1.0 - 0.5 * double(int(ra) + int(rb));
    double F = 0.0;
    F = F + D[0] * (gl0 - gr0);
    for (int j = 1; j <= J; j++) {
        const double k = 2.0 / (3.14159265358979323846 * double(2 * j - 1));
        const double gl1 = k * ((lb ? hm.s : 0.0) - (la ? ha.s : 0.0));
        const double gl2 = k * ((la ? ha.c : 0.0) - (lb ? hm.c : 0.0));
        const double gr1 = k * ((rb ? hb.s : 0.0) - (ra ? hm.s : 0.0));
        const double gr2 = k * ((ra ? hm.c : 0.0) - (rb ? hb.c : 0.0));
        F = F + D[2 * j - 1] * (gl1 - gr1);
        F = F + D[2 * j] * (gl2 - gr2);
        ha.next();
        hm.next();
        hb.next();
    }
    return F;
}

// Solve step for the cells of one level (one wave per cell).  The cell's
// box comes from its ancestors' medians; node i's children are 2i+1 (low
// side) and 2i+2; levels cycle through the coordinates.
template <int P>
__global__ __launch_bounds__(NT) void k_gsolve(const long long *C, uint32_t J, uint32_t level,
                                               TrigTables T, double *med) {
    __shared__ double sW[NW][P][GLOBAL_EP];
    __shared__ double sD[NW][GLOBAL_EP];
    const int w = wave(), l = lane();
    const uint64_t cell = uint64_t(blockIdx.x) * NW + w;
    if (cell >= (1ull << level)) return;  // whole wave
    const uint64_t node = (1ull << level) - 1 + cell;
    const uint32_t t = level % P;
    const uint32_t E = 2 * J + 1;
    double lo[P], hi[P];
    for (int c = 0; c < P; c++) {
        lo[c] = 0.0;
        hi[c] = 1.0;
    }
    const uint64_t k1 = node + 1;  // 1-based heap index
    for (uint32_t d = 0; d < level; d++) {
        const uint64_t anc = (k1 >> (level - d)) - 1;
        const bool right = (k1 >> (level - d - 1)) & 1ull;
        const double m = med[anc];
        if (right) lo[d % P] = m;
        else hi[d % P] = m;
    }
    if (l == 0)
        for (int c = 0; c < P; c++)
            if (uint32_t(c) != t) global_g(lo[c], hi[c], int(J), T, sW[w][c]);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    uint32_t oth[2] = {0, 0}, no = 0;
    for (uint32_t c = 0; c < uint32_t(P); c++)
        if (c != t) oth[no++] = c;
    if (uint32_t(l) < E) {
        const uint32_t jt = uint32_t(l);
        double D;
        if (P == 1) {
            D = double(C[jt]);
        } else if (P == 2) {
            double acc = 0.0;
            for (uint32_t ju = 0; ju < E; ju++) {
                uint32_t idx[2];
                idx[t] = jt;
                idx[oth[0]] = ju;
                acc = acc + double(C[idx[0] * E + idx[1]]) * sW[w][oth[0]][ju];
            }
            D = acc;
        } else {
            double acc = 0.0;
            for (uint32_t ju = 0; ju < E; ju++) {
                double inner = 0.0;
                for (uint32_t jv = 0; jv < E; jv++) {
                    uint32_t idx[3];
                    idx[t] = jt;
                    idx[oth[0]] = ju;
                    idx[oth[1]] = jv;
                    inner = inner + double(C[(idx[0] * E + idx[1]) * E + idx[2]]) * sW[w][oth[1]][jv];
                }
                acc = acc + inner * sW[w][oth[0]][ju];
            }
            D = acc;
        }
        sD[w][jt] = D;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // Bisection of F on (at, bt): while F(a) < 0, halve at mid = a + (b - a)/2
    // (a = mid where F(mid) < 0, else b = mid) until no double lies strictly
    // between a and b or 200 halvings; the median is b.  The wave takes six
    // halvings per round: lane j (1 .. 63) is node j of the six-level tree of
    // halvings below (a, b) and finds its interval by the same halvings along
    // its path, so every midpoint is the one the sequence would compute; the
    // signs of F there then decide the path of the round.
    const double at = lo[t], bt = hi[t];
    double a = at, b = bt, m;
    if (global_F(sD[w], int(J), T, at, bt, a) >= 0.0) {
        m = a;
    } else {
        int it = 0;
        bool done = false;
        while (!done) {
            double la = a, lb = b;
            const int depth = l > 0 ? 31 - __builtin_clz(uint32_t(l)) : 0;
            for (int r = depth - 1; r >= 0; r--) {
                const double mid = la + (lb - la) * 0.5;
                if ((l >> r) & 1) la = mid;
                else lb = mid;
            }
            const double mj = la + (lb - la) * 0.5;
            const bool valid = l > 0 && mj > la && mj < lb;
            const bool neg = valid && global_F(sD[w], int(J), T, at, bt, mj) < 0.0;
            const unsigned long long vm = __ballot(valid), nm = __ballot(neg);
            int nd = 1;
            for (int r = 0; r < 6; r++) {
                if (it == 200 || !((vm >> nd) & 1ull)) {
                    done = true;
                    break;
                }
                const double mid = __shfl(mj, nd, WAVE);
                if ((nm >> nd) & 1ull) {
                    a = mid;
                    nd = 2 * nd + 1;
                } else {
                    b = mid;
                    nd = 2 * nd;
                }
                it++;
            }
        }
        m = b;
    }
    if (l == 0) med[node] = m;
}

// Points per leaf cell (descent: u_t <= m to the low side).  counts must
// start at zero.
__global__ __launch_bounds__(NT) void k_gcount(const float *pts, uint64_t n, uint64_t ld, uint32_t P,
                                               const double *med, uint32_t depth,
                                               unsigned long long *counts) {
    __shared__ uint32_t h[1 << GLOBAL_MAX_DEPTH];
    const uint32_t leaves = 1u << depth;
    const uint64_t nodes = uint64_t(leaves) - 1;
    for (uint32_t k = threadIdx.x; k < leaves; k += NT) h[k] = 0;
    __syncthreads();
    for (uint64_t i = blockIdx.x * uint64_t(NT) + threadIdx.x; i < n; i += uint64_t(gridDim.x) * NT) {
        uint64_t k = 0;
        for (uint32_t d = 0; d < depth; d++) {
            const uint32_t t = d % P;
            k = double(pts[uint64_t(t) * ld + i]) <= med[k] ? 2 * k + 1 : 2 * k + 2;
        }
        atomicAdd(&h[k - nodes], 1u);
    }
    __syncthreads();
    for (uint32_t k = threadIdx.x; k < leaves; k += NT)
        if (h[k]) atomicAdd(&counts[k], (unsigned long long)h[k]);
}

}  // namespace kd

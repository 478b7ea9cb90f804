/*
 * kd_oracle.c -- plain, slow CPU reference for the level-by-level k-d tree
 * build of Chakravorty, Cleveland & Wolfe, "Scalable k-d trees for
 * distributed data".
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or constant generator with the GPU library: every formula
 * below is written out here on its own.
 *
 * Build: gcc -O2 -march=x86-64-v2 -std=gnu11 -fopenmp -ffp-contract=off -fno-fast-math -shared
 * -fPIC (contraction off: every a*b+c below is two rounded IEEE operations).
 *
 * Threads (OpenMP) only share out independent work: the cells of a level,
 * the trees of a batch, and inside a large cell its coordinates, subsets or
 * points.  Every floating-point value is computed by the same operations in
 * the same order whatever the thread count, and the only sums formed across
 * threads are integer sums, which are exact; so the results do not depend
 * on the number of threads.
 *
 * What is computed (one cell at a time, level by level, as in §2 and §4):
 *   - the cell's key coordinate: cyclic (§1, §2) or largest variance (§1);
 *   - a split candidate m from one of three rules:
 *       EXACT   the lower median of the cell's keys (§1, §2: the canonical
 *               tree splits at the median);
 *       FOURIER the paper's approximate median: a sign change of the
 *               equal-count equation Eq. (2) of §3.2, built from the additive
 *               trigonometric statistics of Lemma 3.1 / Eq. (1), restricted
 *               to the cell's key (p = 1);
 *       SUBSET  NOT FROM THE PAPER: the size-weighted mean, in subset order,
 *               of the lower medians of the cell's subsets;
 *   - a tie rule turning m into a valid, closest-to-balanced split (the
 *     paper discards boundary points, §4, and assumes no ties, §3.2);
 *   - a stable partition of the cell into its two children (§2).
 *
 * Parity pins for every function live in tests/ (marker "not gpu").
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#include <omp.h>

#define KDO_OK 0
#define KDO_EINVAL 1
#define KDO_ENOMEM 2
#define KDO_ENONFINITE 3
#define KDO_ECAPACITY 4

#define KDO_KEY_CYCLIC 0
#define KDO_KEY_MAXVAR 1
#define KDO_SPLIT_EXACT 0
#define KDO_SPLIT_FOURIER 1
#define KDO_SPLIT_SUBSET 2

typedef struct kdo_params {
    uint32_t leaf_size;     /* cells with more than leaf_size points are split  */
    uint32_t max_depth;     /* cells at this depth are not split (0 -> default) */
    uint32_t num_subsets;   /* S: subsets per cell (>= 1)                        */
    uint32_t key_rule;      /* KDO_KEY_*                                         */
    uint32_t split_rule;    /* KDO_SPLIT_*                                       */
    uint32_t fourier_J;     /* number of odd harmonics (1..64)                   */
    const uint32_t *pool;   /* pool_entries x S cumulative weights, or NULL      */
    uint32_t pool_entries;
    uint32_t pad_;
    uint64_t seed;
    uint64_t node_capacity; /* size of the node arrays                           */
} kdo_params;

/* ------------------------------------------------------------------ */
/* Order-preserving map from fp32 bit patterns to uint32.              */
/* -0 is folded onto +0; comparisons of keys equal comparisons of the  */
/* real values for every non-NaN input.                                */
/* ------------------------------------------------------------------ */
uint32_t kdo_key_of_bits(uint32_t b)
{
    if (b == 0x80000000u) b = 0u;
    if (b & 0x80000000u) return ~b;
    return b | 0x80000000u;
}

uint32_t kdo_bits_of_key(uint32_t u)
{
    if (u & 0x80000000u) return u & 0x7fffffffu;
    return ~u;
}

static float float_of_bits(uint32_t b) { float f; memcpy(&f, &b, 4); return f; }
static uint32_t bits_of_float(float f) { uint32_t b; memcpy(&b, &f, 4); return b; }
static double value_of_key(uint32_t u) { return (double)float_of_bits(kdo_bits_of_key(u)); }

/* splitmix64 (Steele, Lea & Flood 2014): one counter-based 64-bit mix. */
uint64_t kdo_splitmix64(uint64_t x)
{
    uint64_t z = x + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

/* Ascending sort of uint32 values: insertion sort below 64 values, else a
 * least-significant-digit radix sort, four stable counting-sort passes over
 * the bytes (lowest byte first).                                           */
static void sort_u32(uint32_t *a, uint64_t n)
{
    if (n < 64) {
        for (uint64_t i = 1; i < n; i++) {
            uint32_t v = a[i];
            uint64_t j = i;
            while (j > 0 && a[j - 1] > v) { a[j] = a[j - 1]; j--; }
            a[j] = v;
        }
        return;
    }
    uint32_t *b = (uint32_t *)malloc((n ? n : 1) * sizeof(uint32_t));
    for (int shift = 0; shift < 32; shift += 8) {
        uint64_t count[257];
        memset(count, 0, sizeof(count));
        for (uint64_t i = 0; i < n; i++) count[((a[i] >> shift) & 0xffu) + 1]++;
        for (int v = 0; v < 256; v++) count[v + 1] += count[v];
        for (uint64_t i = 0; i < n; i++) b[count[(a[i] >> shift) & 0xffu]++] = a[i];
        uint32_t *t = a; a = b; b = t;
    }
    /* four passes: the sorted values are back in the caller's array */
    free(b);
}

/* ------------------------------------------------------------------ */
/* Exact lower median: sort, then take 0-based rank floor((n-1)/2).     */
/* The canonical tree splits at the median (§1, Fig. 1, §2); for an    */
/* even count the lower one is taken so the left child gets ceil(n/2). */
/* ------------------------------------------------------------------ */
uint32_t kdo_lower_median(const uint32_t *keys, uint64_t n)
{
    uint32_t *tmp = (uint32_t *)malloc(n * sizeof(uint32_t));
    memcpy(tmp, keys, n * sizeof(uint32_t));
    sort_u32(tmp, n);
    uint32_t m = tmp[(n - 1) / 2];
    free(tmp);
    return m;
}

/* ------------------------------------------------------------------ */
/* Tie rule.  Two candidate children exist for a candidate m:           */
/*   "u <= m" (left size le) and "u < m" (left size lt).                */
/* Take "u <= m" when it leaves both sides non-empty and is no further  */
/* from n/2 than the other (le + lt <= n); otherwise take "u < m" when  */
/* it is non-empty; otherwise the cell cannot be split (all keys equal). */
/* The split is stored so that descent is always "u <= split -> left". */
/* Returns 1 and sets *split when the cell splits, 0 otherwise.        */
/* ------------------------------------------------------------------ */
int kdo_tie_rule(uint64_t n, uint64_t lt, uint64_t le, uint32_t m, uint32_t *split)
{
    if (le < n && le + lt <= n) { *split = m; return 1; }
    if (lt > 0) { *split = m - 1u; return 1; }
    return 0;
}

/* ------------------------------------------------------------------ */
/* Subsets of a cell (§3.2: any partition; App. C.2: key-value pairs    */
/* {r, X_r}).  Subsets are contiguous position ranges of the cell in    */
/* its current (stable) order.  bounds[0..S]: bounds[0]=0, bounds[S]=n. */
/* Equal subsets: bounds[r] = floor(r*n/S).  Pool subsets: a row k of   */
/* S cumulative 32-bit weights (entry 0 unused), chosen by a splitmix64 */
/* hash of (seed, depth, rank of the cell in its level);                */
/* bounds[r] = max(bounds[r-1], (n*W[k][r]) >> 32) for 0 < r < S.       */
/* ------------------------------------------------------------------ */
void kdo_subset_bounds(uint64_t n, uint32_t S, const uint32_t *pool, uint32_t P,
                       uint64_t seed, uint32_t depth, uint64_t rank, uint64_t *bounds)
{
    uint32_t r;
    if (pool == NULL || P == 0) {
        for (r = 0; r <= S; r++) bounds[r] = ((uint64_t)r * n) / S;
        return;
    }
    uint64_t k = kdo_splitmix64(seed ^ ((uint64_t)depth << 32) ^ rank) % P;
    const uint32_t *W = pool + k * (uint64_t)S;
    bounds[0] = 0;
    for (r = 1; r < S; r++) {
        uint64_t b = (n * (uint64_t)W[r]) >> 32;
        bounds[r] = b > bounds[r - 1] ? b : bounds[r - 1];
    }
    bounds[S] = n;
}

/* ------------------------------------------------------------------ */
/* Largest-variance key (§1: key = coordinate of largest variance).    */
/* Values are put on one fixed-point grid for the whole data set:      */
/* E = frexp exponent of max|x| (so max|x| < 2^E), q = rint(x*2^(30-E)) */
/* (|q| < 2^30).  For each coordinate c of a cell with n points,        */
/* V_c = n*sum(q^2) - (sum q)^2 = n^2 * variance, exact in 128 bits.   */
/* The key is the smallest c with the largest V_c.                      */
/* ------------------------------------------------------------------ */
/* Work of at least this many points is shared among threads. */
#define KDO_PAR_MIN 65536

int kdo_maxvar_shift(const float *pts, uint64_t n, uint32_t d, uint64_t ld)
{
    double mx = 0.0;
    for (uint32_t c = 0; c < d; c++) {
#pragma omp parallel for reduction(max : mx) if (n >= KDO_PAR_MIN)
        for (uint64_t i = 0; i < n; i++) {
            double a = fabs((double)pts[c * ld + i]);
            if (a > mx) mx = a;
        }
    }
    if (mx == 0.0) return 0;
    int E;
    frexp(mx, &E);
    return 30 - E;
}

/* q = rint(x * 2^shift); the product by a power of two is exact in double
 * (|x * 2^shift| < 2^30, far from the double range's ends). */
static int32_t fixed_q(float x, double two_to_shift)
{
    double t = (double)x * two_to_shift;
    return (int32_t)nearbyint(t);
}

uint32_t kdo_maxvar_key(const float *pts, uint32_t d, uint64_t ld,
                        const uint32_t *idx, uint64_t n, int shift)
{
    __int128 *V = (__int128 *)malloc(d * sizeof(__int128));
    const double two_to_shift = ldexp(1.0, shift);
#pragma omp parallel for schedule(dynamic, 1) if (n >= KDO_PAR_MIN)
    for (uint32_t c = 0; c < d; c++) {
        int64_t s1 = 0;
        uint64_t s2hi = 0, s2lo = 0;
        for (uint64_t i = 0; i < n; i++) {
            int64_t q = fixed_q(pts[c * ld + (idx ? idx[i] : i)], two_to_shift);
            uint64_t q2 = (uint64_t)(q * q);
            s1 += q;
            s2hi += q2 >> 32;
            s2lo += q2 & 0xffffffffull;
        }
        __int128 S2 = ((__int128)s2hi << 32) + (__int128)s2lo;
        V[c] = (__int128)n * S2 - (__int128)s1 * (__int128)s1;
    }
    uint32_t best = 0;
    __int128 bestv = -1;
    for (uint32_t c = 0; c < d; c++)
        if (V[c] > bestv) { bestv = V[c]; best = c; }
    free(V);
    return best;
}

/* ------------------------------------------------------------------ */
/* Own sine and cosine on [0, 2] (Taylor series about 0, Horner in     */
/* z = x^2).  fp32 variant: terms up to x^17/17! and x^16/16!;          */
/* fp64 variant: terms up to x^25/25! and x^24/24!.  The coefficient   */
/* of x^k is 1/f_k with f_1 = 1, f_k = f_(k-1) * k, both in double      */
/* (f_k is exact for k <= 22), then rounded to the working precision.  */
/* Each multiply and add is rounded separately.                          */
/* ------------------------------------------------------------------ */
static double inv_factorial_of(int k)
{
    double f = 1.0;
    for (int i = 2; i <= k; i++) f *= (double)i;
    return 1.0 / f;
}

/* 1/k! for k = 0..25, formed once when the library is loaded */
static double inv_fact_table[26];
__attribute__((constructor)) static void make_inv_fact_table(void)
{
    for (int k = 0; k < 26; k++) inv_fact_table[k] = inv_factorial_of(k);
}

static double inv_factorial(int k) { return inv_fact_table[k]; }

void kdo_sincos_f32(float x, float *s, float *c)
{
    float z = x * x;
    float ps = (float)inv_factorial(17);
    for (int k = 15; k >= 1; k -= 2) {
        float a = (float)inv_factorial(k);
        if ((k / 2) % 2 == 1) a = -a;
        ps = ps * z;
        ps = ps + a;
    }
    *s = x * ps;
    float pc = (float)inv_factorial(16);
    for (int k = 14; k >= 0; k -= 2) {
        float a = (float)inv_factorial(k);
        if ((k / 2) % 2 == 1) a = -a;
        pc = pc * z;
        pc = pc + a;
    }
    *c = pc;
}

void kdo_sincos_f64(double x, double *s, double *c)
{
    double z = x * x;
    double ps = inv_factorial(25);
    for (int k = 23; k >= 1; k -= 2) {
        double a = inv_factorial(k);
        if ((k / 2) % 2 == 1) a = -a;
        ps = ps * z;
        ps = ps + a;
    }
    *s = x * ps;
    double pc = inv_factorial(24);
    for (int k = 22; k >= 0; k -= 2) {
        double a = inv_factorial(k);
        if ((k / 2) % 2 == 1) a = -a;
        pc = pc * z;
        pc = pc + a;
    }
    *c = pc;
}

/* ------------------------------------------------------------------ */
/* FOURIER rule: per-cell affine map of the key.                       */
/* §2 takes every observation to lie in (0, 1), and Lemma 3.1 states    */
/* c_j and g_j there; how data are brought there is not said.  Each     */
/* cell maps its key by x -> (x - min) * 2^-e with 2^(e-1) <= max - min  */
/* < 2^e: a power of two, so the map is exact in double; the smallest    */
/* key lands on 0 and the largest in [1/2, 1).  The cell is the whole    */
/* unit interval (a = 0, b = 1), so the boundary terms of Lemma 3.1      */
/* vanish, and every difference of two mapped values lies in (-1, 1),    */
/* inside (-pi, pi) where the expansion of 1(x < c) holds (App. A).      */
/* Returns e.                                                            */
/* ------------------------------------------------------------------ */
int kdo_fourier_exponent(uint32_t lo_key, uint32_t hi_key)
{
    double delta = value_of_key(hi_key) - value_of_key(lo_key);
    int e;
    frexp(delta, &e);
    return e;
}

/* The map step of App. C.2 for one subset: for j = 1..J the sums       */
/*   Cc[j-1] += Q(cos((2j-1)u)),  Cs[j-1] += Q(sin((2j-1)u))           */
/* over the subset's points (the statistics C_{2j-1}, C_{2j} of §3.2,  */
/* p = 1), with u the scaled key in fp32, the harmonics from the own   */
/* fp32 sine/cosine of u and the angle-addition recurrence with the    */
/* double angle, and Q(t) = rint(t * 2^24) as an integer so that sums  */
/* are exact and independent of order and partition (§3.2).            */
void kdo_fourier_map(const uint32_t *keys, uint64_t n, uint32_t lo_key, int e,
                     uint32_t J, int64_t *Cc, int64_t *Cs)
{
    double xmin = value_of_key(lo_key);
    double scale = ldexp(1.0, -e);
    for (uint64_t i = 0; i < n; i++) {
        double diff = value_of_key(keys[i]) - xmin;
        float u = (float)(diff * scale);
        float s1, c1;
        kdo_sincos_f32(u, &s1, &c1);
        float ss = s1 * s1;
        float C2 = 1.0f - 2.0f * ss;
        float sc = s1 * c1;
        float S2 = 2.0f * sc;
        float cj = c1, sj = s1;
        for (uint32_t j = 0; j < J; j++) {
            Cc[j] += (int64_t)rintf(cj * 16777216.0f);
            Cs[j] += (int64_t)rintf(sj * 16777216.0f);
            float a = cj * C2, b = sj * S2;
            float g = sj * C2, h = cj * S2;
            cj = a - b;
            sj = g + h;
        }
    }
}

/* Equal-count function of Eq. (2) for p = 1 on a scaled cell: the      */
/* left child is bounded above by v only, the right child below by v    */
/* only, so with the coefficients g_j of Lemma 3.1                      */
/*   1_J(X,-,v) - 1_J(X,v,-) = (4/pi) * sum_j [sin((2j-1)v) C_{2j-1}    */
/*                               - cos((2j-1)v) C_{2j}] / (2j-1)        */
/* (the g_0 terms cancel).  F below is the bracket sum without the      */
/* positive factor 4/pi, in fp64, j ascending.                           */
double kdo_fourier_F(const int64_t *Cc, const int64_t *Cs, uint32_t J, double v)
{
    double s1, c1;
    kdo_sincos_f64(v, &s1, &c1);
    double ss = s1 * s1;
    double C2 = 1.0 - 2.0 * ss;
    double sc = s1 * c1;
    double S2 = 2.0 * sc;
    double cj = c1, sj = s1, F = 0.0;
    const double q = 1.0 / 16777216.0;
    for (uint32_t j = 0; j < J; j++) {
        double a = (double)Cc[j] * q;
        double b = (double)Cs[j] * q;
        double t1 = a * sj, t2 = b * cj;
        double t = t1 - t2;
        double w = 1.0 / (double)(2 * j + 1);
        double wt = w * t;
        F = F + wt;
        double p1 = cj * C2, p2 = sj * S2;
        double p3 = sj * C2, p4 = cj * S2;
        cj = p1 - p2;
        sj = p3 + p4;
    }
    return F;
}

/* Solve Eq. (2) on the key grid: bisection over the order-preserving   */
/* keys between the cell's smallest and largest key for a sign change  */
/* of F (F(v(lo)) <= 0 <= F(v(hi)) because the odd-harmonic partial     */
/* sums are positive on (0, pi)).  Returns the key m with F(v(m)) >= 0 */
/* reached by the bisection, or lo when F(0) >= 0.                      */
uint32_t kdo_fourier_solve(const int64_t *Cc, const int64_t *Cs, uint32_t J,
                           uint32_t lo_key, uint32_t hi_key, int e)
{
    double xmin = value_of_key(lo_key);
    double scale = ldexp(1.0, -e);
    uint32_t lo = lo_key, hi = hi_key;
    if (kdo_fourier_F(Cc, Cs, J, 0.0) >= 0.0) return lo;
    while (hi - lo > 1u) {
        uint32_t mid = lo + (hi - lo) / 2u;
        double v = (value_of_key(mid) - xmin) * scale;
        if (kdo_fourier_F(Cc, Cs, J, v) < 0.0) lo = mid;
        else hi = mid;
    }
    return hi;
}

/* ------------------------------------------------------------------ */
/* One cell: key choice, candidate, tie rule.                           */
/* cell_idx[0..nc): indices into pts of the cell's points, in the      */
/* cell's current (stable) order; NULL: the cell's points are           */
/* pts[c * ld + i] for i < nc, already in that order.                   */
/* Returns 1 if the cell splits (dim/split set).                        */
/* ------------------------------------------------------------------ */
int kdo_cell_split(const float *pts, uint32_t d, uint64_t ld, const kdo_params *p,
                   int maxvar_shift, const uint32_t *cell_idx, uint64_t nc,
                   uint32_t depth, uint64_t rank, uint32_t *dim_out, uint32_t *split_out,
                   uint32_t *cand_out)
{
    uint32_t t;
    if (p->key_rule == KDO_KEY_MAXVAR)
        t = kdo_maxvar_key(pts, d, ld, cell_idx, nc, maxvar_shift);
    else
        t = depth % d;
    *dim_out = t;

    uint32_t *keys = (uint32_t *)malloc(nc * sizeof(uint32_t));
#pragma omp parallel for if (nc >= KDO_PAR_MIN)
    for (uint64_t i = 0; i < nc; i++)
        keys[i] = kdo_key_of_bits(bits_of_float(pts[t * ld + (cell_idx ? cell_idx[i] : i)]));

    uint32_t m;
    if (p->split_rule == KDO_SPLIT_EXACT) {
        m = kdo_lower_median(keys, nc);
    } else {
        uint32_t S = p->num_subsets;
        uint64_t *B = (uint64_t *)malloc((S + 1) * sizeof(uint64_t));
        kdo_subset_bounds(nc, S, p->pool, p->pool_entries, p->seed, depth, rank, B);
        uint32_t lo = keys[0], hi = keys[0];
        for (uint64_t i = 1; i < nc; i++) {
            if (keys[i] < lo) lo = keys[i];
            if (keys[i] > hi) hi = keys[i];
        }
        if (p->split_rule == KDO_SPLIT_FOURIER) {
            if (lo == hi) {
                m = lo;
            } else {
                uint32_t J = p->fourier_J;
                int e = kdo_fourier_exponent(lo, hi);
                /* map per subset (each subset's own sums), then reduce by
                 * addition (App. C.2); integer sums, so exact in any order */
                int64_t Cc[64], Cs[64];
                memset(Cc, 0, sizeof(Cc));
                memset(Cs, 0, sizeof(Cs));
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : Cc, Cs) if (nc >= KDO_PAR_MIN)
                for (uint32_t r = 0; r < S; r++) {
                    int64_t pc[64], ps[64];
                    memset(pc, 0, J * sizeof(int64_t));
                    memset(ps, 0, J * sizeof(int64_t));
                    kdo_fourier_map(keys + B[r], B[r + 1] - B[r], lo, e, J, pc, ps);
                    for (uint32_t j = 0; j < J; j++) { Cc[j] += pc[j]; Cs[j] += ps[j]; }
                }
                m = kdo_fourier_solve(Cc, Cs, J, lo, hi, e);
            }
        } else {
            /* SUBSET (not from the paper): weighted mean of subset lower medians */
            uint32_t *med = (uint32_t *)malloc(S * sizeof(uint32_t));
#pragma omp parallel for schedule(dynamic, 1) if (nc >= KDO_PAR_MIN)
            for (uint32_t r = 0; r < S; r++) {
                uint64_t ns = B[r + 1] - B[r];
                med[r] = ns ? kdo_lower_median(keys + B[r], ns) : 0u;
            }
            double acc = 0.0;
            for (uint32_t r = 0; r < S; r++) {
                uint64_t ns = B[r + 1] - B[r];
                if (ns == 0) continue;
                double prod = (double)ns * value_of_key(med[r]);
                acc = acc + prod;
            }
            free(med);
            double mean = acc / (double)nc;
            /* the rounded mean stays within [smallest, largest] subset median:
             * the double sum errs by at most S * 2^-53 relative, far below
             * half an fp32 ulp, so no clamp to the cell's range is needed */
            m = kdo_key_of_bits(bits_of_float((float)mean));
        }
        free(B);
    }
    *cand_out = m;

    uint64_t lt = 0, le = 0;
#pragma omp parallel for reduction(+ : lt, le) if (nc >= KDO_PAR_MIN)
    for (uint64_t i = 0; i < nc; i++) {
        lt += keys[i] < m;
        le += keys[i] <= m;
    }
    free(keys);
    return kdo_tie_rule(nc, lt, le, m, split_out);
}

/* ------------------------------------------------------------------ */
/* Whole build.                                                          */
/* Node ids are breadth first: the root is node 0; the children of the  */
/* cells split at depth l get the next ids, two per split cell, in the  */
/* order of the cells' first positions.  Leaves are listed in position  */
/* order.  perm lists original indices in leaf order; within a leaf the */
/* original order is kept (every partition is stable).                  */
/* hdr: [0] num_nodes [1] num_leaves [2] depth [3] status               */
/*      [4] point_levels [5] unsplittable [6] oversize leaves           */
/* ------------------------------------------------------------------ */
typedef struct { uint64_t begin, end; uint32_t node, depth; } kdo_cell;
typedef struct { int ok; uint32_t dim, split, cand; uint64_t nl; } kdo_split;

static int cmp_leaf(const void *a, const void *b)
{
    uint64_t x = ((const uint64_t *)a)[0], y = ((const uint64_t *)b)[0];
    return (x > y) - (x < y);
}

int kdo_build(const float *pts, uint64_t n, uint32_t d, uint64_t ld, const kdo_params *p,
              uint32_t *perm, uint32_t *node_begin, uint32_t *node_end, int32_t *node_child,
              uint32_t *node_dim, uint32_t *node_split, uint32_t *node_leaf,
              uint32_t *leaf_node, uint32_t *leaf_offsets, uint64_t *hdr)
{
    memset(hdr, 0, 7 * sizeof(uint64_t));
    if (n == 0 || n > 0xffffffffull || d == 0 || ld < n || p->leaf_size == 0 ||
        p->num_subsets == 0 || p->num_subsets > 4096 || p->key_rule > 1 || p->split_rule > 2 ||
        (p->split_rule == KDO_SPLIT_FOURIER && (p->fourier_J == 0 || p->fourier_J > 64)) ||
        p->node_capacity == 0)
        return KDO_EINVAL;
    uint64_t nonfinite = 0;
    for (uint32_t c = 0; c < d; c++) {
#pragma omp parallel for reduction(+ : nonfinite) if (n >= KDO_PAR_MIN)
        for (uint64_t i = 0; i < n; i++) nonfinite += !isfinite(pts[c * ld + i]);
    }
    if (nonfinite) { hdr[3] = KDO_ENONFINITE; return KDO_ENONFINITE; }

    /* the default cap: ten levels beyond the depth h of a balanced tree with
     * leaves of at most leaf_size points (leaf_size * 2^h >= n), at most 64 */
    uint32_t h = 0;
    while (h < 40 && ((uint64_t)p->leaf_size << h) < n) h++;
    uint32_t max_depth = p->max_depth ? p->max_depth : (h + 10 < 64 ? h + 10 : 64);
    uint64_t cap = p->node_capacity;
    int shift = p->key_rule == KDO_KEY_MAXVAR ? kdo_maxvar_shift(pts, n, d, ld) : 0;

    /* work: original index of the point at each position; wp: the points
     * themselves in the same position order ([d][n]), moved with work by
     * every partition, so a cell's points are always contiguous */
    uint32_t *work = (uint32_t *)malloc(n * sizeof(uint32_t));
    uint32_t *tmp = (uint32_t *)malloc(n * sizeof(uint32_t));
    float *wp = (float *)malloc((size_t)d * n * sizeof(float));
    float *wtmp = (float *)malloc((size_t)d * n * sizeof(float));
    uint8_t *side_of = (uint8_t *)malloc(n);
    for (uint32_t c = 0; c < d; c++) memcpy(wp + (size_t)c * n, pts + c * ld, n * sizeof(float));
    kdo_cell *cur = (kdo_cell *)malloc(sizeof(kdo_cell));
    uint64_t ncur = 0, num_nodes = 1, point_levels = 0, unsplittable = 0;
    uint32_t max_node_depth = 0;
    for (uint64_t i = 0; i < n; i++) work[i] = (uint32_t)i;

    for (uint64_t k = 0; k < cap; k++) {
        node_child[k] = -1; node_dim[k] = 0; node_split[k] = 0;
        node_begin[k] = 0; node_end[k] = 0; node_leaf[k] = 0xffffffffu;
    }
    node_begin[0] = 0; node_end[0] = (uint32_t)n;
    if (n > p->leaf_size && max_depth > 0) {
        cur[0].begin = 0; cur[0].end = n; cur[0].node = 0; cur[0].depth = 0;
        ncur = 1;
    }
    int status = KDO_OK;
    while (ncur > 0 && status == KDO_OK) {
        /* every cell of the level: its split and the stable partition of its
         * own index range (§2: the two children).  Cells own disjoint ranges,
         * so they are handled by as many threads as there are cells; a level
         * of few cells shares the work inside each cell instead. */
        kdo_split *res = (kdo_split *)malloc(ncur * sizeof(kdo_split));
        int nthr = omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 1) if (ncur >= (uint64_t)nthr && ncur > 1)
        for (uint64_t r = 0; r < ncur; r++) {
            kdo_cell c = cur[r];
            uint64_t nc = c.end - c.begin;
            kdo_split *q = &res[r];
            q->ok = kdo_cell_split(wp + c.begin, d, n, p, shift, NULL, nc, c.depth, r,
                                   &q->dim, &q->split, &q->cand);
            q->nl = 0;
            if (!q->ok) continue;
            /* stable partition of the cell's positions: the points with key
             * <= split first, each side in its previous order; the original
             * indices and every coordinate move together */
            const float *key = wp + (size_t)q->dim * n;
            uint64_t nl = 0;
            for (uint64_t i = c.begin; i < c.end; i++) {
                side_of[i] = kdo_key_of_bits(bits_of_float(key[i])) > q->split;
                nl += !side_of[i];
            }
            uint64_t l = c.begin, w = c.begin + nl;
            for (uint64_t i = c.begin; i < c.end; i++) tmp[side_of[i] ? w++ : l++] = work[i];
            memcpy(work + c.begin, tmp + c.begin, nc * sizeof(uint32_t));
#pragma omp parallel for if (nc >= KDO_PAR_MIN)
            for (uint32_t col = 0; col < d; col++) {
                float *src = wp + (size_t)col * n, *dst = wtmp + (size_t)col * n;
                uint64_t l2 = c.begin, w2 = c.begin + nl;
                for (uint64_t i = c.begin; i < c.end; i++) dst[side_of[i] ? w2++ : l2++] = src[i];
                memcpy(src + c.begin, dst + c.begin, nc * sizeof(float));
            }
            q->nl = nl;
        }
        /* node records in cell order (ids breadth first) */
        kdo_cell *next = (kdo_cell *)malloc(2 * ncur * sizeof(kdo_cell));
        uint64_t nnext = 0;
        for (uint64_t r = 0; r < ncur; r++) {
            kdo_cell c = cur[r];
            uint64_t nc = c.end - c.begin, nl = res[r].nl;
            if (!res[r].ok) { unsplittable++; continue; }
            if (num_nodes + 2 > cap) { status = KDO_ECAPACITY; break; }
            point_levels += nc;
            uint32_t left = (uint32_t)num_nodes;
            num_nodes += 2;
            node_child[c.node] = (int32_t)left;
            node_dim[c.node] = res[r].dim;
            node_split[c.node] = res[r].split;
            node_begin[left] = (uint32_t)c.begin;
            node_end[left] = (uint32_t)(c.begin + nl);
            node_begin[left + 1] = (uint32_t)(c.begin + nl);
            node_end[left + 1] = (uint32_t)c.end;
            if (c.depth + 1 > max_node_depth) max_node_depth = c.depth + 1;
            for (int side = 0; side < 2; side++) {
                uint64_t b = side ? c.begin + nl : c.begin, e = side ? c.end : c.begin + nl;
                if (e - b > p->leaf_size && c.depth + 1 < max_depth) {
                    next[nnext].begin = b; next[nnext].end = e;
                    next[nnext].node = left + side; next[nnext].depth = c.depth + 1;
                    nnext++;
                }
            }
        }
        free(res);
        free(cur);
        cur = next;
        ncur = nnext;
    }
    free(cur);

    /* leaves in position order */
    uint64_t nleaves = 0, oversize = 0;
    uint64_t *lv = (uint64_t *)malloc(2 * num_nodes * sizeof(uint64_t));
    for (uint64_t k = 0; k < num_nodes; k++)
        if (node_child[k] < 0) { lv[2 * nleaves] = node_begin[k]; lv[2 * nleaves + 1] = k; nleaves++; }
    qsort(lv, nleaves, 2 * sizeof(uint64_t), cmp_leaf);
    for (uint64_t k = 0; k < nleaves; k++) {
        uint32_t node = (uint32_t)lv[2 * k + 1];
        leaf_node[k] = node;
        leaf_offsets[k] = node_begin[node];
        node_leaf[node] = (uint32_t)k;
        if (node_end[node] - node_begin[node] > p->leaf_size) oversize++;
    }
    leaf_offsets[nleaves] = (uint32_t)n;
    free(lv);
    memcpy(perm, work, n * sizeof(uint32_t));
    free(work); free(tmp); free(wp); free(wtmp); free(side_of);

    hdr[0] = num_nodes; hdr[1] = nleaves; hdr[2] = max_node_depth; hdr[3] = (uint64_t)status;
    hdr[4] = point_levels; hdr[5] = unsplittable; hdr[6] = oversize;
    return status;
}

/* Threads used by the calls that follow (omp_set_num_threads); the     */
/* results do not depend on it.  Returns the previous setting.           */
int kdo_set_threads(int nthreads)
{
    int prev = omp_get_max_threads();
    if (nthreads > 0) omp_set_num_threads(nthreads);
    return prev;
}

/* Many independent trees (the batched workload): tree k is built exactly */
/* as kdo_build builds it alone; trees are shared out among threads, and  */
/* each tree's own levels then run on its thread.  pts[k], n[k], d[k] and */
/* the output arrays out[k][0..9] (perm, node_begin, node_end,            */
/* node_child, node_dim, node_split, node_leaf, leaf_node, leaf_offsets,  */
/* hdr, in kdo_build's order) describe tree k; params[k] its parameters.  */
/* status[k] receives kdo_build's return value.                           */
void kdo_build_batched(uint32_t count, const float *const *pts, const uint64_t *n,
                       const uint32_t *d, const kdo_params *params, void *const *out,
                       int *status)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (uint32_t k = 0; k < count; k++) {
        void *const *o = out + (size_t)k * 10;
        status[k] = kdo_build(pts[k], n[k], d[k], n[k], &params[k], (uint32_t *)o[0],
                              (uint32_t *)o[1], (uint32_t *)o[2], (int32_t *)o[3],
                              (uint32_t *)o[4], (uint32_t *)o[5], (uint32_t *)o[6],
                              (uint32_t *)o[7], (uint32_t *)o[8], (uint64_t *)o[9]);
    }
}

/* Leaf lookup by descent: u <= split -> left child (the same rule the */
/* partition used), for one query point given as d floats.             */
uint32_t kdo_query_leaf(const int32_t *node_child, const uint32_t *node_dim,
                        const uint32_t *node_split, const uint32_t *node_leaf,
                        const float *q, uint64_t stride)
{
    uint32_t node = 0;
    while (node_child[node] >= 0) {
        float x = q[node_dim[node] * stride];
        if (isnan(x)) return 0xffffffffu;
        uint32_t u = kdo_key_of_bits(bits_of_float(x));
        node = (uint32_t)node_child[node] + (u > node_split[node] ? 1u : 0u);
    }
    return node_leaf[node];
}

/* ------------------------------------------------------------------ */
/* Checks of a large tree built elsewhere, for sizes where rebuilding it */
/* here is too slow.  Counts violations of the partition property:     */
/* for every internal node, every point of the left child has key <=   */
/* split and every point of the right child has key > split on the     */
/* node's coordinate.  perm == NULL reads pts in position order (pts    */
/* then holds the points already permuted, [d][ld]).                     */
/* ------------------------------------------------------------------ */
uint64_t kdo_check_partition(const float *pts, uint32_t d, uint64_t ld, const uint32_t *perm,
                             uint64_t num_nodes, const uint32_t *node_begin,
                             const uint32_t *node_end, const int32_t *node_child,
                             const uint32_t *node_dim, const uint32_t *node_split)
{
    uint64_t bad = 0;
    for (uint64_t k = 0; k < num_nodes; k++) {
        if (node_child[k] < 0) continue;
        uint32_t t = node_dim[k];
        if (t >= d) { bad++; continue; }
        uint32_t lc = (uint32_t)node_child[k];
        uint32_t mid = node_end[lc];
        for (uint64_t i = node_begin[k]; i < node_end[k]; i++) {
            uint64_t j = perm ? perm[i] : i;
            uint32_t u = kdo_key_of_bits(bits_of_float(pts[t * ld + j]));
            int left = i < mid;
            if (left != (u <= node_split[k])) bad++;
        }
    }
    return bad;
}

/* ------------------------------------------------------------------ */
/* The paper's global single-pass construction (§3.2 with Eq. (1) and  */
/* (2); App. C, basic form K = 1): one pass over the data gives the    */
/* statistics C_j(X) = sum_i prod_l c_{j_l}(x_il) for j in {0..2J}^p;  */
/* every median of a depth-D tree then comes from solving Eq. (2) for  */
/* its cell box (a, b), without revisiting the data.                   */
/*                                                                     */
/* Readings: the points are given in (0,1)^p (the paper's standing     */
/* assumption; how data get there is left to the caller); c_0 = 1,     */
/* c_{2j-1} = cos((2j-1)u), c_{2j} = sin((2j-1)u) in fp32 (own series  */
/* and the harmonic recurrence, as the per-level rule), each quantised */
/* as rint(c * Q_p), Q_1 = 2^24, Q_2 = 2^15, Q_3 = 2^10, so that every */
/* product is an integer of at most 2^30 and the sums over up to 2^32  */
/* points are exact in int64; the sums are not standardised (dividing  */
/* by |X| does not move a root).                                       */
/* Levels cycle through the coordinates; node i's children are 2i+1    */
/* (low side) and 2i+2.                                                */
/* ------------------------------------------------------------------ */

float kdo_global_quantum(uint32_t p) { return p == 1 ? 16777216.0f : (p == 2 ? 32768.0f : 1024.0f); }

/* q[0..2J] of one coordinate value u, quantum Q */
void kdo_global_basis(float u, uint32_t J, float Q, float *q)
{
    float s1, c1;
    kdo_sincos_f32(u, &s1, &c1);
    float ss = s1 * s1;
    float C2 = 1.0f - 2.0f * ss;
    float sc = s1 * c1;
    float S2 = 2.0f * sc;
    float cj = c1, sj = s1;
    q[0] = Q;
    for (uint32_t j = 0; j < J; j++) {
        q[2 * j + 1] = rintf(cj * Q);
        q[2 * j + 2] = rintf(sj * Q);
        float a = cj * C2, b = sj * S2;
        float g = sj * C2, h = cj * S2;
        cj = a - b;
        sj = g + h;
    }
}

/* C[(2J+1)^p] += the statistics of n points (pts: [p][ld], in (0,1)). */
void kdo_global_moments(const float *pts, uint64_t n, uint32_t p, uint64_t ld, uint32_t J,
                        int64_t *C)
{
    uint32_t E = 2 * J + 1;
    float q[3][64];
    float Q = kdo_global_quantum(p);
    for (uint64_t i = 0; i < n; i++) {
        for (uint32_t c = 0; c < p; c++) kdo_global_basis(pts[c * ld + i], J, Q, q[c]);
        if (p == 1) {
            for (uint32_t a = 0; a < E; a++) C[a] += (int64_t)q[0][a];
        } else if (p == 2) {
            for (uint32_t a = 0; a < E; a++)
                for (uint32_t b = 0; b < E; b++) C[a * E + b] += (int64_t)q[0][a] * (int64_t)q[1][b];
        } else {
            for (uint32_t a = 0; a < E; a++)
                for (uint32_t b = 0; b < E; b++) {
                    int64_t ab = (int64_t)q[0][a] * (int64_t)q[1][b];
                    for (uint32_t d = 0; d < E; d++) C[(a * E + b) * E + d] += ab * (int64_t)q[2][d];
                }
        }
    }
}

/* sin((2j-1)x), cos((2j-1)x) for j = 1..J (fp64, own series, recurrence) */
static void global_harmonics(double x, uint32_t J, double *s, double *c)
{
    double s1, c1;
    kdo_sincos_f64(x, &s1, &c1);
    double ss = s1 * s1;
    double C2 = 1.0 - 2.0 * ss;
    double sc = s1 * c1;
    double S2 = 2.0 * sc;
    double cj = c1, sj = s1;
    for (uint32_t j = 0; j < J; j++) {
        s[j] = sj;
        c[j] = cj;
        double a = cj * C2, b = sj * S2;
        double g = sj * C2, h = cj * S2;
        cj = a - b;
        sj = g + h;
    }
}

/* g_0..g_{2J} of Lemma 3.1 for the interval (a, b) of (0, 1) */
void kdo_global_g(double a, double b, uint32_t J, double *g)
{
    double sa[64], ca[64], sb[64], cb[64];
    int ia = a > 0.0, ib = b < 1.0;
    global_harmonics(a, J, sa, ca);
    global_harmonics(b, J, sb, cb);
    g[0] = 1.0 - 0.5 * (double)(ia + ib);
    for (uint32_t j = 1; j <= J; j++) {
        double k = 2.0 / (M_PI * (double)(2 * j - 1));
        double s_b = ib ? sb[j - 1] : 0.0, s_a = ia ? sa[j - 1] : 0.0;
        double c_a = ia ? ca[j - 1] : 0.0, c_b = ib ? cb[j - 1] : 0.0;
        g[2 * j - 1] = k * (s_b - s_a);
        g[2 * j] = k * (c_a - c_b);
    }
}

/* Eq. (2) for one cell: F(m) = 1_J(X, a, b_t <- m) - 1_J(X, a_t <- m, b),
 * given D_j = the statistics contracted with the g weights of the other
 * coordinates. */
static double global_F(const double *D, uint32_t J, double at, double bt, double m)
{
    double gl[129], gr[129];
    kdo_global_g(at, m, J, gl);
    kdo_global_g(m, bt, J, gr);
    double F = 0.0;
    for (uint32_t j = 0; j <= 2 * J; j++) F = F + D[j] * (gl[j] - gr[j]);
    return F;
}

/* The 2^depth - 1 medians (mapped domain) in heap order. */
void kdo_global_solve(const int64_t *C, uint32_t p, uint32_t J, uint32_t depth, double *med)
{
    uint32_t E = 2 * J + 1;
    uint64_t nodes = ((uint64_t)1 << depth) - 1;
    double *lo = calloc((2 * nodes + 1) * p, sizeof(double));
    double *hi = calloc((2 * nodes + 1) * p, sizeof(double));
    for (uint32_t c = 0; c < p; c++) hi[c] = 1.0;
    double W[3][129], D[129];
    for (uint64_t i = 0; i < nodes; i++) {
        uint32_t dep = 0;
        while ((((uint64_t)2 << dep) - 1) <= i) dep++;
        uint32_t t = dep % p;
        const double *a = lo + i * p, *b = hi + i * p;
        for (uint32_t c = 0; c < p; c++)
            if (c != t) kdo_global_g(a[c], b[c], J, W[c]);
        uint32_t oth[2] = {0, 0}, no = 0;
        for (uint32_t c = 0; c < p; c++)
            if (c != t) oth[no++] = c;
        for (uint32_t jt = 0; jt < E; jt++) {
            if (p == 1) {
                D[jt] = (double)C[jt];
            } else if (p == 2) {
                double acc = 0.0;
                for (uint32_t ju = 0; ju < E; ju++) {
                    uint32_t idx[2];
                    idx[t] = jt;
                    idx[oth[0]] = ju;
                    acc = acc + (double)C[idx[0] * E + idx[1]] * W[oth[0]][ju];
                }
                D[jt] = acc;
            } else {
                double acc = 0.0;
                for (uint32_t ju = 0; ju < E; ju++) {
                    double inner = 0.0;
                    for (uint32_t jv = 0; jv < E; jv++) {
                        uint32_t idx[3];
                        idx[t] = jt;
                        idx[oth[0]] = ju;
                        idx[oth[1]] = jv;
                        inner = inner + (double)C[(idx[0] * E + idx[1]) * E + idx[2]] * W[oth[1]][jv];
                    }
                    acc = acc + inner * W[oth[0]][ju];
                }
                D[jt] = acc;
            }
        }
        double l = a[t], h = b[t], m;
        if (global_F(D, J, a[t], b[t], l) >= 0.0) {
            m = l;
        } else {
            for (int it = 0; it < 200; it++) {
                double mid = l + (h - l) * 0.5;
                if (!(mid > l && mid < h)) break;
                if (global_F(D, J, a[t], b[t], mid) < 0.0) l = mid;
                else h = mid;
            }
            m = h;
        }
        med[i] = m;
        uint64_t L = 2 * i + 1, R = 2 * i + 2;
        for (uint32_t c = 0; c < p; c++) {
            lo[L * p + c] = a[c];
            hi[L * p + c] = b[c];
            lo[R * p + c] = a[c];
            hi[R * p + c] = b[c];
        }
        hi[L * p + t] = m;
        lo[R * p + t] = m;
    }
    free(lo);
    free(hi);
}

/* Points per leaf cell: descend with u_t <= m to the low side. */
void kdo_global_counts(const float *pts, uint64_t n, uint32_t p, uint64_t ld, const double *med,
                       uint32_t depth, uint64_t *counts)
{
    uint64_t nodes = ((uint64_t)1 << depth) - 1;
    for (uint64_t i = 0; i < n; i++) {
        uint64_t k = 0;
        for (uint32_t d = 0; d < depth; d++) {
            uint32_t t = d % p;
            k = (double)pts[t * ld + i] <= med[k] ? 2 * k + 1 : 2 * k + 2;
        }
        counts[k - nodes]++;
    }
}

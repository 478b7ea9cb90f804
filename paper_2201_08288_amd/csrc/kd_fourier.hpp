// kd_fourier.hpp -- the paper's approximate median on one cell's key (§3.1
// Lemma 3.1, §3.2 Eq. (1)-(2), p = 1), device side.
//
// Map step (App. C.2): §2 takes every observation to lie in (0, 1), and
// Lemma 3.1 states c_j and g_j there.  Each cell maps its key into that unit
// interval by u = (x - min) * 2^-e, 2^(e-1) <= max - min < 2^e, a power of
// two so the map is exact in fp64: the smallest key lands on 0 and the
// largest in [1/2, 1).  The cell itself is the whole interval (a = 0, b = 1),
// so the boundary terms 1(a > 0), 1(b < 1) of Lemma 3.1 vanish.
// In fp32: sin u, cos u by Taylor series (Horner in u^2), then the odd
// harmonics cos((2j-1)u), sin((2j-1)u) by the angle-addition recurrence with
// the double angle; each term is quantized as rint(t * 2^24) and summed in
// int64, so the statistics C_{2j-1}, C_{2j} of the cell are exact and do not
// depend on how the cell is split into subsets (§3.2).
// Solve step: the equal-count equation becomes F(v) = 0 with
//   F(v) = sum_j [C_{2j-1} sin((2j-1)v) - C_{2j} cos((2j-1)v)] / (2j-1),
// evaluated in fp64; the split is the key reached by bisection over the
// order-preserving keys between the cell's smallest and largest key.
// Every multiply and add is a separately rounded IEEE operation (the file is
// compiled with contraction off).
#pragma once
#include "kd_device.hpp"

namespace kd {

constexpr int FOURIER_JMAX = 64;
constexpr int FCHUNK = 16;  // harmonics accumulated per register chunk

// Series coefficients and weights, filled on the host: term m of the sine
// series is s[m] * x^(2m+1), of the cosine series c[m] * x^(2m); the values
// are (-1)^m / (2m+1)! and (-1)^m / (2m)! with the factorial formed by
// repeated multiplication in double and the quotient rounded to the working
// precision.  w[j] = 1 / (2j+1).
struct TrigTables {
    float s32[9], c32[9];
    double s64[13], c64[13];
    double w[FOURIER_JMAX];
};

__device__ __forceinline__ void sincos32(float x, const TrigTables &T, float &s, float &c) {
    const float z = x * x;
    float ps = T.s32[8];
#pragma unroll
    for (int m = 7; m >= 0; m--) {
        ps = ps * z;
        ps = ps + T.s32[m];
    }
    s = x * ps;
    float pc = T.c32[8];
#pragma unroll
    for (int m = 7; m >= 0; m--) {
        pc = pc * z;
        pc = pc + T.c32[m];
    }
    c = pc;
}

__device__ __forceinline__ void sincos64(double x, const TrigTables &T, double &s, double &c) {
    const double z = x * x;
    double ps = T.s64[12];
#pragma unroll
    for (int m = 11; m >= 0; m--) {
        ps = ps * z;
        ps = ps + T.s64[m];
    }
    s = x * ps;
    double pc = T.c64[12];
#pragma unroll
    for (int m = 11; m >= 0; m--) {
        pc = pc * z;
        pc = pc + T.c64[m];
    }
    c = pc;
}

__device__ __forceinline__ double value_of_key(uint32_t u) {
    return double(__uint_as_float(bits_of_key(u)));
}

// Exponent e of the cell map: 2^(e-1) <= max - min < 2^e (max > min).
__device__ __forceinline__ int fourier_exponent(uint32_t lo, uint32_t hi) {
    const double delta = value_of_key(hi) - value_of_key(lo);
    const unsigned long long b = __double_as_longlong(delta);
    return int((b >> 52) & 0x7ff) - 1022;
}

// Scale 2^-e as an exact double (e is within [-148, 129] for fp32 keys).
__device__ __forceinline__ double fourier_scale(int e) {
    return __longlong_as_double((long long)(uint64_t(1023 - e) << 52));
}

// Accumulate the quantized harmonics j0 .. j0+FCHUNK-1 of one key into
// acc[0..FCHUNK) (cosines) and acc[FCHUNK..2*FCHUNK) (sines).
template <class ACC>
__device__ __forceinline__ void fourier_terms(uint32_t key, double xmin, double scale, int J,
                                              int j0, const TrigTables &T, ACC *acc) {
    const double diff = value_of_key(key) - xmin;
    const float u = float(diff * scale);
    float s1, c1;
    sincos32(u, T, s1, c1);
    const float ss = s1 * s1;
    const float C2 = 1.0f - 2.0f * ss;
    const float sc = s1 * c1;
    const float S2 = 2.0f * sc;
    float cj = c1, sj = s1;
    for (int j = 0; j < j0; j++) {  // advance the recurrence to harmonic j0
        const float a = cj * C2, b = sj * S2;
        const float g = sj * C2, h = cj * S2;
        cj = a - b;
        sj = g + h;
    }
#pragma unroll
    for (int k = 0; k < FCHUNK; k++) {
        if (j0 + k < J) {
            acc[k] += ACC((int)rintf(cj * 16777216.0f));
            acc[FCHUNK + k] += ACC((int)rintf(sj * 16777216.0f));
        }
        const float a = cj * C2, b = sj * S2;
        const float g = sj * C2, h = cj * S2;
        cj = a - b;
        sj = g + h;
    }
}

// F(v) from the summed statistics: cf[2j] and cf[2j+1] hold the bits of
// a_j = Cc[j] * 2^-24 and b_j = Cs[j] * 2^-24 (harmonic 2j+1, j < J) in LDS,
// read by every lane at once; each lane evaluates F at its own v.  The harmonics are taken
// four at a time so that their weights are fetched together; the sum runs
// over j in order either way.
__device__ __forceinline__ void fourier_F_term(const long long *cf, const TrigTables &T, int j,
                                               double C2, double S2, double &cj, double &sj,
                                               double &F) {
    const double a = __longlong_as_double(cf[2 * j]), b = __longlong_as_double(cf[2 * j + 1]);
    const double t1 = a * sj, t2 = b * cj;
    const double t = t1 - t2;
    const double wt = T.w[j] * t;
    F = F + wt;
    const double p1 = cj * C2, p2 = sj * S2;
    const double p3 = sj * C2, p4 = cj * S2;
    cj = p1 - p2;
    sj = p3 + p4;
}

__device__ __forceinline__ double fourier_F(const long long *cf, int J, double v,
                                            const TrigTables &T) {
    double s1, c1;
    sincos64(v, T, s1, c1);
    const double ss = s1 * s1;
    const double C2 = 1.0 - 2.0 * ss;
    const double sc = s1 * c1;
    const double S2 = 2.0 * sc;
    double cj = c1, sj = s1, F = 0.0;
    int j = 0;
    for (; j + 4 <= J; j += 4) {
#pragma unroll
        for (int k = 0; k < 4; k++) fourier_F_term(cf, T, j + k, C2, S2, cj, sj, F);
    }
    for (; j < J; j++) fourier_F_term(cf, T, j, C2, S2, cj, sj, F);
    return F;
}

// Bisection for the sign change of F between keys lo < hi, run by one wave64:
// each round evaluates F at the 63 midpoints of the next six bisection steps
// in parallel (lane i-1 holds heap node i) and then follows the path the
// sequential bisection would take, so the result is the sequential one.
// Returns the key m (lo when F(v(lo)) >= 0).  Every lane gets the result.
// cf: this wave's LDS for 2J values (16-byte aligned); it may be the LDS
// that holds Cc and Cs (the same type, so the reads stay before the writes).
__device__ uint32_t fourier_solve_wave(const long long *Cc, const long long *Cs, int J,
                                       uint32_t lo, uint32_t hi, int e, const TrigTables &T,
                                       long long *cf) {
    const double xmin = value_of_key(lo);
    const double scale = fourier_scale(e);
    const int l = lane();
    // the statistics as doubles
    const double q = 1.0 / 16777216.0;
    double a = 0.0, b = 0.0;
    if (l < J) {
        a = double(Cc[l]) * q;
        b = double(Cs[l]) * q;
    }
    __builtin_amdgcn_wave_barrier();
    if (l < J) {
        cf[2 * l] = __double_as_longlong(a);
        cf[2 * l + 1] = __double_as_longlong(b);
    }
    __builtin_amdgcn_wave_barrier();
    // F at v = 0 (the smallest key)
    const double f0 = fourier_F(cf, J, 0.0, T);
    if (f0 >= 0.0) return lo;
    while (hi - lo > 1u) {
        // heap node of this lane and its interval
        const uint32_t node = uint32_t(l) + 1u;  // 1..64; node 64 unused
        uint32_t a = lo, b = hi;
        const int depth = 31 - __clz(node);       // 0..6
        bool live = node < 64u;
        for (int t = depth - 1; t >= 0 && live; t--) {
            if (b - a <= 1u) {
                live = false;
                break;
            }
            const uint32_t mid = a + (b - a) / 2u;
            if ((node >> t) & 1u) a = mid;  // right branch: F(mid) < 0
            else b = mid;                   // left branch: F(mid) >= 0
        }
        live = live && (b - a > 1u);
        const uint32_t mid = a + (b - a) / 2u;
        // evaluated by every lane; lanes without a live node use v = 0
        const double v = live ? (value_of_key(mid) - xmin) * scale : 0.0;
        const double f = fourier_F(cf, J, v, T);
        const unsigned long long neg = __ballot(live && f < 0.0);
        // follow the sequential path for up to six steps
        uint32_t nd = 1;
        for (int t = 0; t < 6 && hi - lo > 1u; t++) {
            const uint32_t m2 = lo + (hi - lo) / 2u;
            if ((neg >> (nd - 1)) & 1ull) {
                lo = m2;
                nd = 2 * nd + 1;
            } else {
                hi = m2;
                nd = 2 * nd;
            }
        }
    }
    return hi;
}

}  // namespace kd

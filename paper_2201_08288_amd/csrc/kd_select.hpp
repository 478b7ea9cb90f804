// kd_select.hpp -- k-th smallest key by radix select (8-bit digits, most
// significant first) for one workgroup or one wave64, over keys staged in LDS
// or read from global memory.
#pragma once
#include "kd_device.hpp"

namespace kd {

// Memory ordering point for LDS traffic between the lanes of one wave.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

struct SelectResult {
    uint32_t key;  // the k-th smallest key
    uint32_t lt;   // keys smaller than it
    uint32_t le;   // keys smaller or equal
};

// The digits of a select start at the highest bit where the smallest and
// largest key differ: the bits above it are common to every key and need no
// pass, and the first pass then spreads the keys over at least two bins.
// Digit p covers bits [pos - width, pos) with pos = top + 1 - RBITS * p.
__device__ __forceinline__ uint32_t above_mask(int pos) { return pos >= 32 ? 0u : ~0u << pos; }

// Workgroup radix select.  KEYS(i) yields key i of n (n >= 1); h: NBINS words
// of LDS; sh: NW+1 words; s3: 3 words.  Every thread gets the result.
template <class KEYS>
__device__ SelectResult block_select(KEYS keys, uint32_t n, uint32_t k, uint32_t *h,
                                     uint32_t *sh, uint32_t *s3) {
    uint32_t mn = ~0u, mx = 0;
    for (uint32_t i = threadIdx.x; i < n; i += NT) {
        const uint32_t u = keys(i);
        mn = min(mn, u);
        mx = max(mx, u);
    }
    mn = wave_min(mn);
    mx = wave_max(mx);
    if (threadIdx.x == 0) {
        s3[0] = ~0u;
        s3[1] = 0;
    }
    __syncthreads();
    if (lane() == 0) {
        atomicMin(&s3[0], mn);
        atomicMax(&s3[1], mx);
    }
    __syncthreads();
    mn = s3[0];
    mx = s3[1];
    __syncthreads();
    if (mn == mx) return SelectResult{mn, 0u, n};
    const int top = 31 - __builtin_clz(mn ^ mx);
    uint32_t prefix = mn & above_mask(top + 1), lt = 0, cnt = 0;
    for (int pos = top + 1; pos > 0; pos -= RBITS) {
        const int width = pos < RBITS ? pos : RBITS, shift = pos - width;
        const uint32_t mask = above_mask(pos), dmask = (1u << width) - 1u;
        for (int b = threadIdx.x; b < NBINS; b += NT) h[b] = 0;
        __syncthreads();
        for (uint32_t i = threadIdx.x; i < n; i += NT) {
            uint32_t u = keys(i);
            if ((u & mask) == prefix) atomicAdd(&h[(u >> shift) & dmask], 1u);
        }
        __syncthreads();
        uint32_t hv = h[threadIdx.x], tot;
        uint32_t ex = block_excl_scan(hv, sh, &tot);
        if (ex <= k && k < ex + hv) {
            s3[0] = threadIdx.x;
            s3[1] = ex;
            s3[2] = hv;
        }
        __syncthreads();
        prefix |= s3[0] << shift;
        k -= s3[1];
        lt += s3[1];
        cnt = s3[2];
        __syncthreads();
    }
    return SelectResult{prefix, lt, lt + cnt};
}

// Workgroup radix select of the k-th smallest key of a column in global
// memory, col[0 .. n) holding fp32 bits: sixteen loads per thread in flight per
// step.  h: NBINS words of LDS; sh: NW+1 words; s3: 3 words.
__device__ uint32_t block_select_global(const uint32_t *col, uint32_t n, uint32_t k, uint32_t *h,
                                        uint32_t *sh, uint32_t *s3) {
    constexpr int U = 16;
    const KD_GLOBAL uint32_t *g = gp(col);
    uint32_t prefix = 0;
    for (int pass = 0; pass < RPASSES; pass++) {
        const int shift = 32 - RBITS * (pass + 1);
        const uint32_t mask = pass == 0 ? 0u : (~0u << (32 - RBITS * pass));
        for (int b = threadIdx.x; b < NBINS; b += NT) h[b] = 0;
        __syncthreads();
        for (uint32_t i0 = 0; i0 < n; i0 += U * NT) {
            uint32_t u[U];
#pragma unroll
            for (int j = 0; j < U; j++) {
                const uint32_t i = i0 + j * NT + threadIdx.x;
                u[j] = i < n ? key_of_bits(g[i]) : 0u;
            }
#pragma unroll
            for (int j = 0; j < U; j++) {
                const uint32_t i = i0 + j * NT + threadIdx.x;
                if (i < n && (u[j] & mask) == prefix) atomicAdd(&h[(u[j] >> shift) & (NBINS - 1)], 1u);
            }
        }
        __syncthreads();
        uint32_t hv = h[threadIdx.x], tot;
        uint32_t ex = block_excl_scan(hv, sh, &tot);
        if (ex <= k && k < ex + hv) {
            s3[0] = threadIdx.x;
            s3[1] = ex;
        }
        __syncthreads();
        prefix |= s3[0] << shift;
        k -= s3[1];
        __syncthreads();
    }
    return prefix;
}

// Wave radix select over keys[off .. off+n) of an LDS array stored with one
// pad word per 32 (element i at i + i / 32); h: this wave's NBINS words; n >= 1.
__device__ uint32_t wave_select(const uint32_t *keys, uint32_t off, uint32_t n, uint32_t k,
                                uint32_t *h) {
    const int l = lane();
    uint32_t mn = ~0u, mx = 0;
    for (uint32_t i = l; i < n; i += WAVE) {
        const uint32_t g = off + i;
        const uint32_t u = keys[g + (g >> 5)];
        mn = min(mn, u);
        mx = max(mx, u);
    }
    mn = wave_min(mn);
    mx = wave_max(mx);
    if (mn == mx) return mn;
    const int top = 31 - __builtin_clz(mn ^ mx);
    uint32_t prefix = mn & above_mask(top + 1);
    for (int pos = top + 1; pos > 0; pos -= RBITS) {
        const int width = pos < RBITS ? pos : RBITS, shift = pos - width;
        const uint32_t mask = above_mask(pos), dmask = (1u << width) - 1u;
        for (int b = l; b < NBINS; b += WAVE) h[b] = 0;
        wave_sync();
        for (uint32_t i = l; i < n; i += WAVE) {
            const uint32_t g = off + i;
            uint32_t u = keys[g + (g >> 5)];
            if ((u & mask) == prefix) atomicAdd(&h[(u >> shift) & dmask], 1u);
        }
        wave_sync();
        // lane l owns bins 4l .. 4l+3
        uint32_t c[4], local = 0;
#pragma unroll
        for (int j = 0; j < 4; j++) {
            c[j] = h[4 * l + j];
            local += c[j];
        }
        uint32_t ex = wave_incl_scan(local) - local;
        const bool mine = ex <= k && k < ex + local;
        const unsigned long long m = __ballot(mine);
        const int src = __builtin_ctzll(m);  // exactly one lane holds rank k
        uint32_t bin = 0, below = ex;
        bool found = false;
#pragma unroll
        for (int j = 0; j < 4; j++) {
            if (!found && k < below + c[j]) {
                bin = 4 * l + j;
                found = true;
            } else if (!found) {
                below += c[j];
            }
        }
        bin = wave_bcast(bin, src);
        below = wave_bcast(below, src);
        prefix |= bin << shift;
        k -= below;
        wave_sync();
    }
    return prefix;
}

}  // namespace kd

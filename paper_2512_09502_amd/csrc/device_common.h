// Device helpers: the Philox4x32-10 stream, value mappings, node-set lookups
// and wave64/workgroup scans.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "bm_math.h"
#include "internal.h"

namespace snnc {

enum : uint32_t { PURPOSE_IDX = 0, PURPOSE_SYN = 1, PURPOSE_BERN = 2 };

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two
// 32x32->64 products of counter words 0 and 2 with the round multipliers,
// the high halves xor-ed with the other counter words and the key; the key
// advances by the Weyl increments between rounds.
__device__ __forceinline__ uint4 philox10(uint4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        const uint64_t a = (uint64_t)0xD2511F53u * c.x;
        const uint64_t b = (uint64_t)0xCD9E8D57u * c.z;
        c = make_uint4((uint32_t)(b >> 32) ^ c.y ^ k0, (uint32_t)b, (uint32_t)(a >> 32) ^ c.w ^ k1, (uint32_t)a);
    }
    return c;
}

// Block `purpose` of element e in the stream of (seed, call).
__device__ __forceinline__ uint4 draw(uint32_t seed, uint32_t call, uint64_t e, uint32_t purpose) {
    return philox10(make_uint4((uint32_t)e, (uint32_t)(e >> 32), purpose, 0u), seed, call);
}

// floor(((hi << 32) | lo) * n / 2^64) for n < 2^32.
__device__ __forceinline__ uint32_t uniform_index(uint32_t lo, uint32_t hi, uint32_t n) {
    const uint64_t p_lo = (uint64_t)lo * n;
    const uint64_t p_hi = (uint64_t)hi * n + (p_lo >> 32);
    return (uint32_t)(p_hi >> 32);
}

// fp32 weight N(mean, sd): Box-Muller, cosine branch, in double precision,
// u1 = (w0 + 1) / 2^32, u2 = w1 / 2^32, one rounding to fp32.  ln u1 and
// cos(2pi_d u2) come from the argument-exact helpers of bm_math.h (within two
// double ulp of the library functions).  Contraction is off so that the
// final product and sum round as written.
__device__ __forceinline__ float normal_weight(uint32_t w0, uint32_t w1, double mean, double sd) {
#pragma clang fp contract(off)
    const double radius = sqrt(-2.0 * log_u32_frac((uint64_t)w0 + 1));
    const double z = radius * cos_2pi_u32(w1);
    const double scaled = sd * z;
    return (float)(mean + scaled);
}

// Delay step from the threshold table: k_lo + #{k : w >= t_k}.  The guide
// bounds the search to the thresholds inside w's 2^24-wide slice (usually
// none or one).
__device__ __forceinline__ uint16_t delay_step(const uint32_t* tab, const uint32_t* guide, uint32_t klo,
                                               uint32_t w) {
    uint32_t a = guide[w >> 24], b = guide[(w >> 24) + 1];
    while (a < b) {
        const uint32_t m = (a + b) >> 1;
        if (tab[m] <= w) a = m + 1; else b = m;
    }
    return (uint16_t)(klo + a);
}

__device__ __forceinline__ void syn_values(const SynD& s, uint32_t seed, uint32_t call, uint64_t e,
                                           float& w, uint16_t& d) {
    if (s.w_normal | s.d_normal) {
        const uint4 b = draw(seed, call, e, PURPOSE_SYN);
        w = s.w_normal ? normal_weight(b.x, b.y, s.w_mean, s.w_sd) : s.w_const;
        d = s.d_normal ? delay_step(s.dtab, s.dguide, s.d_klo, b.z) : (uint16_t)s.d_const;
    } else {
        w = s.w_const;
        d = (uint16_t)s.d_const;
    }
}

// Ordinal -> (host, local id) in a node set (segments sorted by ordinal).
__device__ __forceinline__ void set_lookup(const SegD* seg, uint32_t nseg, uint64_t ord, uint32_t& host,
                                           uint32_t& local) {
    uint32_t a = 0, b = nseg;   // last segment with ord_begin <= ord
    while (b - a > 1) {
        const uint32_t m = (a + b) >> 1;
        if (seg[m].ord_begin <= ord) a = m; else b = m;
    }
    const SegD s = seg[a];
    host = s.host;
    local = s.first + (uint32_t)(ord - s.ord_begin);
}

// Unsigned division by a run-time constant d for x < 2^32 (Granlund and
// Montgomery, "Division by invariant integers using multiplication", 1994):
// with l = ceil(log2 d) and m = floor(2^(32+l) / d) + 1, x / d = (x m) >> (32+l).
struct FastDiv {
    uint64_t m;
    uint32_t shift;
    uint32_t d;
};

inline FastDiv make_fastdiv(uint32_t d) {
    uint32_t l = 0;
    while ((1ull << l) < d) ++l;
    FastDiv f;
    f.d = d;
    f.shift = 32 + l;
    const unsigned __int128 one = 1;
    f.m = (uint64_t)(((one << (32 + l)) / d) + 1);
    return f;
}

__device__ __forceinline__ uint32_t fastdiv(uint32_t x, const FastDiv& f) {
    // x * m < 2^31 * 2^33 for the x < 2^31 used here
    return (uint32_t)(((uint64_t)x * f.m) >> f.shift);
}

// Add 1 to bin `bin` of an LDS histogram for every valid lane; when the
// whole wave hits one bin (common for the high digits of sorted-ish data) a
// single atomic adds the wave's count.  Call with the whole wave converged.
__device__ __forceinline__ void wave_hist_add(uint32_t* h, uint32_t bin, bool valid) {
    const uint64_t act = __ballot(valid);
    if (!act) return;
    const int leader = __ffsll((unsigned long long)act) - 1;
    const uint32_t b0 = __shfl(bin, leader, 64);
    const uint64_t same = __ballot(valid && bin == b0);
    if (same == act) {
        if ((int)(threadIdx.x & 63) == leader) atomicAdd(&h[b0], (uint32_t)__popcll(act));
    } else if (valid) {
        atomicAdd(&h[bin], 1u);
    }
}

// ------------------------------------------------------------------ scans
// Inclusive prefix sum across a wave64 (Hillis-Steele with shuffles).
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t t = __shfl_up(v, o, 64);
        if (lane >= o) v += t;
    }
    return v;
}

__device__ __forceinline__ uint64_t wave_incl_scan64(uint64_t v) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint64_t t = __shfl_up(v, o, 64);
        if (lane >= o) v += t;
    }
    return v;
}

// Exclusive scan across a workgroup of NT threads; returns the exclusive
// prefix of this thread and the total in *total.  `scratch` holds NT/64
// entries.  Contains barriers: every thread must call it.
template <int NT, class T>
__device__ __forceinline__ T block_excl_scan(T v, T* scratch, T* total) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    T incl;
    if constexpr (sizeof(T) == 8) incl = wave_incl_scan64(v);
    else incl = wave_incl_scan(v);
    if (lane == 63) scratch[wave] = incl;
    __syncthreads();
    T wave_off = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < NT / 64; ++w) {
        const T s = scratch[w];
        if (w < wave) wave_off += s;
        tot += s;
    }
    __syncthreads();
    *total = tot;
    return wave_off + incl - v;
}

}  // namespace snnc

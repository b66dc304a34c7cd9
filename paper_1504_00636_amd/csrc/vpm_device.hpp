// Device-side helpers for the Voronoi particle-merging kernels (gfx950, wave64).
//
//  * exact wide unsigned integers (128/256 bit) for the split decisions,
//  * power-of-two lane groups inside one wavefront (a group of g lanes, g | 64, works on one
//    subset: sums, counts and stable compaction without workgroup barriers),
//  * workgroup reductions and scans through LDS.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define VPM_DEV __device__ __forceinline__

namespace vpm {

constexpr int WAVE = 64;

// ------------------------------------------------------------------------------------------
// Exact unsigned arithmetic
// ------------------------------------------------------------------------------------------

struct U128 { uint64_t lo, hi; };
struct U256 { uint64_t w0, w1, w2, w3; };

VPM_DEV U128 u128_make(uint64_t lo, uint64_t hi) { U128 r; r.lo = lo; r.hi = hi; return r; }

VPM_DEV U128 mul64(uint64_t a, uint64_t b) { return u128_make(a * b, __umul64hi(a, b)); }

VPM_DEV U128 add128(U128 a, U128 b) {
    U128 r;
    r.lo = a.lo + b.lo;
    r.hi = a.hi + b.hi + (r.lo < a.lo ? 1u : 0u);
    return r;
}

VPM_DEV U128 sub128(U128 a, U128 b) {          // a >= b
    U128 r;
    r.lo = a.lo - b.lo;
    r.hi = a.hi - b.hi - (a.lo < b.lo ? 1u : 0u);
    return r;
}

VPM_DEV U128 shl128(U128 a, int s) {            // 0 < s < 64
    return u128_make(a.lo << s, (a.hi << s) | (a.lo >> (64 - s)));
}

VPM_DEV bool is_zero128(U128 a) { return (a.lo | a.hi) == 0; }

VPM_DEV int cmp128(U128 a, U128 b) {
    if (a.hi != b.hi) return a.hi < b.hi ? -1 : 1;
    if (a.lo != b.lo) return a.lo < b.lo ? -1 : 1;
    return 0;
}

// full 128 x 128 -> 256 product
VPM_DEV U256 mul128(U128 a, U128 b) {
    U128 p00 = mul64(a.lo, b.lo);
    U128 p01 = mul64(a.lo, b.hi);
    U128 p10 = mul64(a.hi, b.lo);
    U128 p11 = mul64(a.hi, b.hi);
    U256 r;
    r.w0 = p00.lo;
    // column 1: p00.hi + p01.lo + p10.lo
    uint64_t c1 = p00.hi;
    uint64_t carry2 = 0;
    uint64_t t = c1 + p01.lo; carry2 += (t < c1); c1 = t;
    t = c1 + p10.lo; carry2 += (t < c1); c1 = t;
    r.w1 = c1;
    // column 2: p01.hi + p10.hi + p11.lo + carry2
    uint64_t c2 = p11.lo, carry3 = 0;
    t = c2 + p01.hi; carry3 += (t < c2); c2 = t;
    t = c2 + p10.hi; carry3 += (t < c2); c2 = t;
    t = c2 + carry2; carry3 += (t < c2); c2 = t;
    r.w2 = c2;
    r.w3 = p11.hi + carry3;
    return r;
}

VPM_DEV int cmp256(U256 a, U256 b) {
    if (a.w3 != b.w3) return a.w3 < b.w3 ? -1 : 1;
    if (a.w2 != b.w2) return a.w2 < b.w2 ? -1 : 1;
    if (a.w1 != b.w1) return a.w1 < b.w1 ? -1 : 1;
    if (a.w0 != b.w0) return a.w0 < b.w0 ? -1 : 1;
    return 0;
}

// ------------------------------------------------------------------------------------------
// Lane groups: g lanes (g a power of two <= 64) starting at a lane multiple of g.
// ------------------------------------------------------------------------------------------

VPM_DEV int lane_id() { return __lane_id(); }

VPM_DEV uint64_t lanes_below() {                 // bit mask of the lanes below this one
    const int l = lane_id();
    return l == 0 ? 0ull : (~0ull >> (64 - l));
}

// Bits of `ballot` that belong to this lane's group, shifted down to bit 0.
VPM_DEV uint64_t group_bits(uint64_t ballot, int gbase, int g) {
    const uint64_t m = g == 64 ? ~0ull : ((1ull << g) - 1ull);
    return (ballot >> gbase) & m;
}

template <typename V>
VPM_DEV V group_sum(V v, int g) {
    for (int m = 1; m < g; m <<= 1) v += __shfl_xor(v, m);
    return v;
}

VPM_DEV U128 group_sum128(U128 v, int g) {
    for (int m = 1; m < g; m <<= 1) {
        U128 o = u128_make(__shfl_xor(v.lo, m), __shfl_xor(v.hi, m));
        v = add128(v, o);
    }
    return v;
}

// ------------------------------------------------------------------------------------------
// Workgroup helpers (all threads must call; `red` is LDS scratch of >= blockDim/64 slots).
// ------------------------------------------------------------------------------------------

template <typename V, typename Op>
VPM_DEV V wave_reduce(V v, Op op) {
    for (int m = 1; m < WAVE; m <<= 1) v = op(v, __shfl_xor(v, m));
    return v;
}

template <int T, typename V, typename Op>
VPM_DEV V block_reduce(V v, Op op, V* red) {
    v = wave_reduce(v, op);
    const int w = threadIdx.x / WAVE;
    __syncthreads();
    if (lane_id() == 0) red[w] = v;
    __syncthreads();
    V r = red[0];
#pragma unroll
    for (int i = 1; i < T / WAVE; ++i) r = op(r, red[i]);
    return r;
}

// Exclusive scan of one value per thread across the workgroup; returns the prefix and sets
// *total.  `red` needs T/64 + 1 slots.
template <int T, typename V>
VPM_DEV V block_exclusive_scan(V v, V* red, V* total) {
    const int l = lane_id();
    V inc = v;
    for (int d = 1; d < WAVE; d <<= 1) {
        V o = __shfl_up(inc, d);
        if (l >= d) inc += o;
    }
    const int w = threadIdx.x / WAVE;
    __syncthreads();
    if (l == WAVE - 1) red[w] = inc;
    __syncthreads();
    V base = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < T / WAVE; ++i) {
        if (i < w) base += red[i];
        tot += red[i];
    }
    *total = tot;
    return base + inc - v;
}

}  // namespace vpm

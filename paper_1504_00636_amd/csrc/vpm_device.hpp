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

struct U320 { uint64_t w[5]; };

// a 256-bit value times a 64-bit one
VPM_DEV U320 mul256x64(U256 a, uint64_t b) {
    const uint64_t in[4] = {a.w0, a.w1, a.w2, a.w3};
    U320 r;
    uint64_t carry = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const uint64_t lo = in[i] * b, hi = __umul64hi(in[i], b);
        const uint64_t s = lo + carry;
        r.w[i] = s;
        carry = hi + (s < lo ? 1u : 0u);
    }
    r.w[4] = carry;
    return r;
}

VPM_DEV int cmp320(const U320& a, const U320& b) {
#pragma unroll
    for (int i = 4; i >= 0; --i)
        if (a.w[i] != b.w[i]) return a.w[i] < b.w[i] ? -1 : 1;
    return 0;
}

// ------------------------------------------------------------------------------------------
// Lane groups: g lanes (g a power of two <= 64) starting at a lane multiple of g.
// ------------------------------------------------------------------------------------------

VPM_DEV int lane_id() { return __lane_id(); }

// Wave ballot of a boolean.  (HIP's __ballot takes an int, and the int -> bool test it adds is
// compiled as a move of the condition into a vector register and a compare back: two VALU
// instructions per ballot that the boolean form does not need.)
VPM_DEV uint64_t ballot(bool p) { return __builtin_amdgcn_ballot_w64(p); }

VPM_DEV uint64_t lanes_below_of(int l) {         // bit mask of the lanes below lane l
    return l == 0 ? 0ull : (~0ull >> (64 - l));
}
VPM_DEV uint64_t lanes_below() { return lanes_below_of(lane_id()); }

// The lane index as a value the compiler cannot precompute: values derived from it are then formed
// where they are used instead of being hoisted out of the kernel's outer loops, where they would
// occupy registers for the whole kernel.
VPM_DEV int opaque_lane() {
    int l = lane_id();
    asm volatile("" : "+v"(l));
    return l;
}
VPM_DEV int opaque_tid() {
    int t = (int)threadIdx.x;
    asm volatile("" : "+v"(t));
    return t;
}

// Partner value for step m of a butterfly sum inside aligned groups of lanes.  Steps 1 and 2 are
// DPP quad permutes; steps 4 and 8 are the DPP half-row and row mirrors, which pair each lane with
// one of the other half of its 8- or 16-lane block (equivalent to xor for a sum, because after the
// earlier steps every lane of a half holds the same partial); step 16 is a swizzle with xor 16;
// step 32 a cross-half permute.  Every partner lies in the caller's group, so it is active.
// (mov_dpp rather than update_dpp: every lane's source is valid, so no "old" value has to be
// materialised in the destination first, one VALU move less per exchange.)
template <int M>
VPM_DEV int xchg32(int v) {
    if constexpr (M == 1) return __builtin_amdgcn_mov_dpp(v, 0xB1, 0xF, 0xF, false);
    else if constexpr (M == 2) return __builtin_amdgcn_mov_dpp(v, 0x4E, 0xF, 0xF, false);
    else if constexpr (M == 4) return __builtin_amdgcn_mov_dpp(v, 0x141, 0xF, 0xF, false);
    else if constexpr (M == 8) return __builtin_amdgcn_mov_dpp(v, 0x140, 0xF, 0xF, false);
    else if constexpr (M == 16) return __builtin_amdgcn_ds_swizzle(v, 0x401F);
    else return __shfl_xor(v, 32);
}

// Partner value at lane l ^ M exactly (M = 1 ... 16): a swizzle in xor mode (the LDS unit's
// crossbar, no VALU move; the kernels are bound by VALU issue).
template <int M>
VPM_DEV int xor32(int v) {
    static_assert(M >= 1 && M <= 16, "ds_swizzle exchanges within 32 lanes");
    return __builtin_amdgcn_ds_swizzle(v, (M << 10) | 0x1F);       // and 0x1F, or 0, xor M
}
template <int M>
VPM_DEV double xor_dbl(double v) {
    const int64_t u = __double_as_longlong(v);
    auto x = [](int w) {
        if constexpr (M >= 32 || M <= 2) return xchg32<M>(w);         // xor 1, 2: DPP quad permutes, exact
        else return xor32<M>(w);
    };
    const int lo = x((int)(uint32_t)u), hi = x((int)((uint64_t)u >> 32));
    return __longlong_as_double((int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo));
}

template <int M>
VPM_DEV int xchg(int v) { return xchg32<M>(v); }
template <int M>
VPM_DEV uint32_t xchg(uint32_t v) { return (uint32_t)xchg32<M>((int)v); }
template <int M>
VPM_DEV int64_t xchg(int64_t v) {
    const int lo = xchg32<M>((int)(uint32_t)(uint64_t)v), hi = xchg32<M>((int)((uint64_t)v >> 32));
    return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}
template <int M>
VPM_DEV uint64_t xchg(uint64_t v) { return (uint64_t)xchg<M>((int64_t)v); }
template <int M>
VPM_DEV double xchg(double v) { return __longlong_as_double(xchg<M>((int64_t)__double_as_longlong(v))); }
template <int M>
VPM_DEV float xchg(float v) { return __int_as_float(xchg32<M>(__float_as_int(v))); }

// Maximum over an aligned group of g lanes (every lane of the group receives it).
VPM_DEV float group_max(float v, int g) {
    if (g > 1) v = fmaxf(v, xchg<1>(v));
    if (g > 2) v = fmaxf(v, xchg<2>(v));
    if (g > 4) v = fmaxf(v, xchg<4>(v));
    if (g > 8) v = fmaxf(v, xchg<8>(v));
    if (g > 16) v = fmaxf(v, xchg<16>(v));
    if (g > 32) v = fmaxf(v, xchg<32>(v));
    return v;
}

// Sum over an aligned group of g lanes (g a power of two, the same for all lanes of a group);
// every lane of the group receives the total.
template <typename V>
VPM_DEV V group_sum(V v, int g) {
    if (g > 1) v += xchg<1>(v);
    if (g > 2) v += xchg<2>(v);
    if (g > 4) v += xchg<4>(v);
    if (g > 8) v += xchg<8>(v);
    if (g > 16) v += xchg<16>(v);
    if (g > 32) v += xchg<32>(v);
    return v;
}


// ------------------------------------------------------------------------------------------
// Workgroup helpers (all threads must call; `red` is LDS scratch of >= blockDim/64 slots).
// ------------------------------------------------------------------------------------------

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

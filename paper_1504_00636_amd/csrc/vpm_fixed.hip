// Fixed-point Voronoi particle merging on gfx950 (the batched FP32 hot path).
//
// One wavefront owns one simulation cell at a time (persistent grid; each wave pops cells from a
// size-binned queue and works in its own LDS slice, or in a global slab for very large cells).
// The cell's particles are turned into integer codes once (Sec. "Algorithm", Step 1 collects the
// cell; the codes fix its frame):
//     weight    omega = rint(w * 2^(15 - e_w))          e_w: frexp exponent of the cell's max w
//     position  c     = min(rint((x - lo) * s), 65535) - 32768,  s = fl32(65536 / L), lo = cell min
//     momentum  c     = rint(p * 2^(22 - e_a))          e_a: frexp exponent of the cell's max |p_a|
// and every subset ("Voronoi cell") is described by integer moments
//     S0 = sum omega,  S1_l = sum omega c_l,  S2_l = sum omega c_l^2.
// The coefficient of variation (Eqs. cv_x, cv_p) is compared as an exact rational:
//     Delta_l^2 = V_l / D_l,  V_l = S0 S2_l - S1_l^2,  D = 2^32 S0^2 (positions), S1_l^2 (momenta)
// Step 3 (stop when all six CVs <= tolerance), Step 4 (largest CV, ties to the lowest axis) and
// Step 5 (cut q <= Q, i.e. c S0 <= S1) are decided exactly, so the partition does not depend on
// summation order or launch shape.  S0 and S1 are exact in FP64 (they stay below 2^53); S2 is
// accumulated with FP64 FMAs, and every comparison is first made in FP64 with a proven error
// bound.  Only a comparison that falls inside its bound is redone with exact 128/256-bit integer
// moments recomputed from the codes, which gives the same answer the exact rule would.
//
// Splitting is level-synchronous inside the wave.  Every unfinished subset of a level is handled
// by a group of g lanes (g a power of two chosen from the subset size): the group counts the lower
// side, compacts the subset stably with ballots into the other index buffer (Step 6), sums the
// moments of both children, and its first two lanes decide the children.
//
// Replacement (Step 7): each finished subset of at least min_subset particles is merged from the
// FP32 data with order-independent int64 fixed-point sums and an FP64 solve for the centroid or
// the energy-conserving pair.
#include "vpm_device.hpp"
#include "vpm_internal.h"

namespace vpm {
namespace {


// info byte per slot once its final subset is known
constexpr uint8_t INF_PARITY = 0x01;   // index buffer that holds the final order
constexpr uint8_t INF_HEAD = 0x02;     // first slot of its final subset
constexpr uint8_t INF_MERGED = 0x04;   // the subset is merged (else copied)
constexpr int INF_JSHIFT = 3;          // bits 3-4: pair-direction axis
constexpr uint8_t INF_SET = 0x80;

template <typename IdxT>
struct Node { IdxT start, len; int32_t thr_axis; };
// thr_axis = (threshold << 8) | (cell << 4) | (reversed << 3) | axis; `cell`: index of the subset's
// cell within a batch of small cells (0 otherwise); `reversed`: the subset's slots hold its
// members in decreasing input order

struct Frame {
    float lo[3], hi[3], pmax[3], wmax;
    int ew, ep[3], pzero[3];
    int ext_e[3];        // frexp exponent of the cell's extent per position axis
    int eb;              // frexp exponent of a bound on |eps_i - eps_j| over the cell
    int amask;           // bit l: the codes of axis l are not all equal in the cell
    double mass;         // the particle mass of the cell (Step 7 energies)
};

// ------------------------------------------------------------------------------------------
// Moments
// ------------------------------------------------------------------------------------------

// FP64 moments: s0 and s1 hold exact integers (|S1| <= 2^53); s2 is rounded.
struct FSums { double s0, s1[6], s2[6]; };

VPM_DEV void fsums_zero(FSums& S) {
    S.s0 = 0.0;
#pragma unroll
    for (int l = 0; l < 6; ++l) { S.s1[l] = 0.0; S.s2[l] = 0.0; }
}

// Axes whose codes are all equal in the cell carry code 0, so their sums stay exactly 0.
VPM_DEV void fsums_add(FSums& S, int om, int c0, int c1, int c2, int c3, int c4, int c5) {
    const double o = (double)om;
    const int c[6] = {c0, c1, c2, c3, c4, c5};
    S.s0 += o;
#pragma unroll
    for (int l = 0; l < 6; ++l) {
        const double cl = (double)c[l];
        const double t = o * cl;                  // exact: |t| <= 2^37
        S.s1[l] += t;                             // exact while the partial sum stays below 2^53
        S.s2[l] = fma(t, cl, S.s2[l]);
    }
}

template <int M>
VPM_DEV void fsums_step(FSums& S) {
    S.s0 += xchg<M>(S.s0);
#pragma unroll
    for (int l = 0; l < 6; ++l) { S.s1[l] += xchg<M>(S.s1[l]); S.s2[l] += xchg<M>(S.s2[l]); }
}

// Reduction of the two children's moments over an aligned group of g >= 2 lanes, ending with V1's
// totals in the even lanes and V2's in the odd lanes, in L.  The first step trades the other
// child's partials between the lanes of a pair; the later steps pair lanes of equal parity (exact
// xor partners), so they reduce one set of moments instead of two.
VPM_DEV void fsums_pair_reduce(FSums& L, const FSums& R, int lid, int g) {
    const bool odd = lid & 1;
    auto first = [&](double& l, double r) {
        const double send = odd ? l : r;
        l = (odd ? r : l) + xchg<1>(send);
    };
    first(L.s0, R.s0);
#pragma unroll
    for (int l = 0; l < 6; ++l) { first(L.s1[l], R.s1[l]); first(L.s2[l], R.s2[l]); }
    auto step = [&](auto m) {
        constexpr int M = decltype(m)::value;
        L.s0 += xor_dbl<M>(L.s0);
#pragma unroll
        for (int l = 0; l < 6; ++l) { L.s1[l] += xor_dbl<M>(L.s1[l]); L.s2[l] += xor_dbl<M>(L.s2[l]); }
    };
    if (g > 2) step(std::integral_constant<int, 2>());
    if (g > 4) step(std::integral_constant<int, 4>());
    if (g > 8) step(std::integral_constant<int, 8>());
    if (g > 16) step(std::integral_constant<int, 16>());
    if (g > 32) step(std::integral_constant<int, 32>());
}

VPM_DEV void fsums_group_reduce(FSums& S, int g) {
    if (g > 1) fsums_step<1>(S);
    if (g > 2) fsums_step<2>(S);
    if (g > 4) fsums_step<4>(S);
    if (g > 8) fsums_step<8>(S);
    if (g > 16) fsums_step<16>(S);
    if (g > 32) fsums_step<32>(S);
}

// Exact integer moments (used only when an FP64 comparison is too close to call).
struct ISums { uint32_t s0; int64_t s1[6]; int64_t s2p[3]; U128 s2m[3]; };

VPM_DEV void isums_add(ISums& S, uint32_t om, const int c[6]) {
    S.s0 += om;
    const int64_t o = (int64_t)om;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const int64_t t = o * c[a];                       // |t| <= 2^30
        S.s1[a] += t;
        S.s2p[a] += t * c[a];
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const int64_t t = o * c[3 + a];                   // |t| <= 2^37
        S.s1[3 + a] += t;
        const uint64_t q = (uint64_t)(t * c[3 + a]);      // <= 2^59
        const uint64_t lo = S.s2m[a].lo + q;
        S.s2m[a].hi += (lo < q) ? 1u : 0u;
        S.s2m[a].lo = lo;
    }
}

// ------------------------------------------------------------------------------------------
// Decisions (Steps 3-5)
// ------------------------------------------------------------------------------------------

enum { D_SPLIT = 0, D_MERGED = 1, D_COPY = 2 };

struct Decision { int kind, axis, thr, jdir; };

VPM_DEV uint64_t uabs64(int64_t v) { return v < 0 ? (uint64_t)(-v) : (uint64_t)v; }

// Pair-direction axis: the momentum component with the smallest |mean| (exact: |S1| 2^e_a).
VPM_DEV int pair_axis(const double s1[6], const Frame& F) {
    int best = 0;
    double bv = 0.0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const double v = F.pzero[a] ? 0.0 : ldexp(fabs(s1[3 + a]), F.ep[a]);
        if (a == 0 || v < bv) { bv = v; best = a; }
    }
    return best;
}

// Step 5 threshold: c * S0 <= S1  <=>  c <= floor(S1 / S0), exact for |S1| <= 2^53, S0 <= 2^31.
VPM_DEV int cut_threshold(double s1, double s0) {
    const int64_t S1 = (int64_t)s1, S0 = (int64_t)s0;
    int64_t t = (int64_t)floor(s1 / s0);
    if (t * S0 > S1) t -= 1;
    else if ((t + 1) * S0 <= S1) t += 1;
    return (int)t;
}

// Is Delta_a^2 = Va/Da strictly larger than Delta_b^2 = Vb/Db?  D == 0 with V > 0 is +infinity.
VPM_DEV bool frac_gt(U128 Va, U128 Da, U128 Vb, U128 Db) {
    const bool az = is_zero128(Va), bz = is_zero128(Vb);
    if (az) return false;
    if (bz) return true;
    const bool ainf = is_zero128(Da), binf = is_zero128(Db);
    if (ainf) return !binf;
    if (binf) return false;
    return cmp256(mul128(Va, Db), mul128(Vb, Da)) > 0;
}

// Is Delta_a^2 / Ta^2 > Delta_b^2 / Tb^2 (the normalised axis rule)?  With T^2 = T2 / 2^48 this
// compares Va Db T2b with Vb Da T2a (< 2^320).  Zero D or zero T2 under V > 0 is +infinity.
VPM_DEV bool frac_gt_norm(U128 Va, U128 Da, uint64_t T2a, U128 Vb, U128 Db, uint64_t T2b) {
    if (is_zero128(Va)) return false;
    if (is_zero128(Vb)) return true;
    const bool ainf = is_zero128(Da) || T2a == 0, binf = is_zero128(Db) || T2b == 0;
    if (ainf) return !binf;
    if (binf) return false;
    return cmp320(mul256x64(mul128(Va, Db), T2b), mul256x64(mul128(Vb, Da), T2a)) > 0;
}

// The decision rule's constants.  Each workgroup copies them from the kernel arguments into LDS
// once and the decisions read them there: kernel-argument values live across a whole kernel hold
// scalar registers, and their spills to vector lanes slow the particle loops.
struct DecideConsts {
    float t2x_lo, t2x_hi, t2p_lo, t2p_hi;   // Step 3: FP32 brackets of T_x^2, T_p^2
    float wx_lo, wx_hi, wp_lo, wp_hi;       // Step 4: FP32 brackets of the axis weights (raw rule 1,
                                            // normalised 1 / T^2, +infinity for T = 0)
    uint64_t thx2, thp2;                    // That_x^2, That_p^2 (Step 3, exact)
    uint64_t tx2, tp2;                      // Step 4 exact weights: 1, or That^2 (normalised rule)
    int32_t norm;                           // the normalised rule (else the weights are 1)
    int32_t force_exact;                    // skip the FP64 evaluation: every decision exactly
};

VPM_DEV DecideConsts decide_consts(const FixedParams& P) {
    DecideConsts K;
    K.t2x_lo = P.t2x_lo; K.t2x_hi = P.t2x_hi; K.t2p_lo = P.t2p_lo; K.t2p_hi = P.t2p_hi;
    const bool norm = P.axis_rule != 0;
    K.wx_lo = !norm ? 1.0f : P.that_x == 0 ? INFINITY : P.it2x_lo;
    K.wx_hi = !norm ? 1.0f : P.that_x == 0 ? INFINITY : P.it2x_hi;
    K.wp_lo = !norm ? 1.0f : P.that_p == 0 ? INFINITY : P.it2p_lo;
    K.wp_hi = !norm ? 1.0f : P.that_p == 0 ? INFINITY : P.it2p_hi;
    K.thx2 = P.that_x * P.that_x;
    K.thp2 = P.that_p * P.that_p;
    K.tx2 = P.tx2;
    K.tp2 = P.tp2;
    K.norm = norm ? 1 : 0;
    K.force_exact = P.force_exact ? 1 : 0;
    return K;
}

// The exact rule on exact integer moments.
VPM_DEV Decision decide_exact(const ISums& S, const DecideConsts& K, const Frame& F) {
    Decision d;
    d.axis = 0; d.thr = 0;
    double s1d[6];
#pragma unroll
    for (int l = 0; l < 6; ++l) s1d[l] = (double)S.s1[l];
    d.jdir = pair_axis(s1d, F);
    if (S.s0 == 0) { d.kind = D_MERGED; return d; }
    const uint64_t s0 = S.s0;
    const U128 s0sq = mul64(s0, s0);                 // <= 2^62
    U128 V[6], D[6];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const uint64_t s1 = uabs64(S.s1[a]);
        V[a] = sub128(mul64(s0, (uint64_t)S.s2p[a]), mul64(s1, s1));
        D[a] = shl128(s0sq, 32);
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const uint64_t s1 = uabs64(S.s1[3 + a]);
        U128 s0s2 = mul64(s0, S.s2m[a].lo);
        s0s2.hi += s0 * S.s2m[a].hi;
        D[3 + a] = mul64(s1, s1);
        V[3 + a] = sub128(s0s2, D[3 + a]);
    }
    bool done = true;
    {
        const U128 rhs = mul64(K.thx2, s0sq.lo);     // That^2 S0^2
#pragma unroll
        for (int a = 0; a < 3; ++a)
            if (!is_zero128(V[a]) && cmp128(shl128(V[a], 16), rhs) > 0) done = false;
        const U128 tp2 = u128_make(K.thp2, 0);
#pragma unroll
        for (int a = 3; a < 6; ++a) {
            if (is_zero128(V[a])) continue;
            if (is_zero128(D[a])) { done = false; continue; }
            U256 lhs;                                              // V * 2^48
            lhs.w0 = V[a].lo << 48;
            lhs.w1 = (V[a].hi << 48) | (V[a].lo >> 16);
            lhs.w2 = V[a].hi >> 16;
            lhs.w3 = 0;
            if (cmp256(lhs, mul128(tp2, D[a])) > 0) done = false;
        }
    }
    if (done) { d.kind = D_MERGED; return d; }
    // Step 4 in two stages: the position axes share D, so their largest CV is their largest V; the
    // momentum axes compare as fractions among themselves; then one comparison across the groups
    // (raw, or each CV over its tolerance), which the momentum axis wins only when strictly larger
    // (ties go to the lower axis, a position).  Under the normalised rule a zero tolerance makes every
    // CV > 0 of its group infinite: the group's first such axis is its largest.
    const bool xinf = K.tx2 == 0, pinf = K.tp2 == 0;
    // (The running maxima are carried by value: indexing V and D with a variable would put them in
    // private memory.)
    int kx = 0;
    U128 xV = V[0];
#pragma unroll
    for (int l = 1; l < 3; ++l)
        if (xinf ? is_zero128(xV) && !is_zero128(V[l]) : cmp128(V[l], xV) > 0) { kx = l; xV = V[l]; }
    int kp = 3;
    U128 pV = V[3], pD = D[3];
#pragma unroll
    for (int l = 4; l < 6; ++l)
        if (pinf ? is_zero128(pV) && !is_zero128(V[l]) : frac_gt(V[l], D[l], pV, pD)) { kp = l; pV = V[l]; pD = D[l]; }
    const bool mom = frac_gt_norm(pV, pD, K.tp2, xV, D[0], K.tx2);      // raw rule: tx2 = tp2 = 1
    const int k = mom ? kp : kx;
    double s1k = s1d[0];
#pragma unroll
    for (int l = 1; l < 6; ++l) if (l == k) s1k = s1d[l];
    d.kind = D_SPLIT;
    d.axis = k;
    d.thr = cut_threshold(s1k, (double)S.s0);
    return d;
}

// ------------------------------------------------------------------------------------------
// Subsets above 2^16 particles (a whole simulation box merged as one cell: the method's first
// subset may be the box itself).  With up to 2^24 particles |S1| reaches 2^61, past the 2^53 that
// FP64 holds exactly, so these subsets are decided by the exact rule only, on integer moments
// summed exactly: S0 <= 2^39, |S1| <= 2^61, S2 <= 2^83 (128 bits).  The products of Steps 3-4 stay
// below 2^256 (2^320 under the normalised axis rule).
// ------------------------------------------------------------------------------------------

constexpr int NMAX_NARROW = 65536;     // largest subset decided through the FP64 filter

struct WSums { uint64_t s0; int64_t s1[6]; U128 s2[6]; };

VPM_DEV void wsums_zero(WSums& S) {
    S.s0 = 0;
#pragma unroll
    for (int l = 0; l < 6; ++l) { S.s1[l] = 0; S.s2[l] = u128_make(0, 0); }
}

VPM_DEV void wsums_add(WSums& S, int om, const int c[6]) {
    S.s0 += (uint64_t)om;
#pragma unroll
    for (int l = 0; l < 6; ++l) {
        const int64_t t = (int64_t)om * c[l];                  // |t| <= 2^37
        S.s1[l] += t;
        S.s2[l] = add128(S.s2[l], u128_make((uint64_t)(t * c[l]), 0));   // omega c^2 < 2^60
    }
}

VPM_DEV void wsums_acc(WSums& S, const WSums& T) {
    S.s0 += T.s0;
#pragma unroll
    for (int l = 0; l < 6; ++l) { S.s1[l] += T.s1[l]; S.s2[l] = add128(S.s2[l], T.s2[l]); }
}

// Sum over the wavefront (every lane receives the total).
VPM_DEV void wsums_wave_reduce(WSums& S) {
#pragma unroll
    for (int m = 1; m < WAVE; m <<= 1) {
        WSums T;
        T.s0 = __shfl_xor(S.s0, m);
#pragma unroll
        for (int l = 0; l < 6; ++l) {
            T.s1[l] = __shfl_xor(S.s1[l], m);
            T.s2[l] = u128_make(__shfl_xor(S.s2[l].lo, m), __shfl_xor(S.s2[l].hi, m));
        }
        wsums_acc(S, T);
    }
}

// Pair-direction axis from exact S1: argmin over the momentum axes of |S1_a| 2^e_a, ties to the
// lowest axis (compared exactly: first by magnitude, bit length plus exponent, then the aligned
// values).
VPM_DEV int pair_axis_exact(const int64_t s1[6], const Frame& F) {
    int best = 0;
    uint64_t bm = 0;
    int be = 0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const uint64_t m = F.pzero[a] ? 0 : uabs64(s1[3 + a]);
        const int e = F.ep[a];
        bool less = false;
        if (a > 0) {
            if (m == 0 || bm == 0) {
                less = m == 0 && bm != 0;
            } else {
                const int lm = 64 - __clzll((long long)m) + e, lb = 64 - __clzll((long long)bm) + be;
                if (lm != lb) less = lm < lb;
                else less = e >= be ? (m << (e - be)) < bm : m < (bm << (be - e));
            }
        }
        if (a == 0 || less) { best = a; bm = m; be = e; }
    }
    return best;
}

// The exact rule on exact wide moments (the same comparisons as decide_exact, in wider integers).
VPM_DEV Decision decide_exact_wide(const WSums& S, const DecideConsts& K, const Frame& F) {
    Decision d;
    d.axis = 0; d.thr = 0;
    d.jdir = pair_axis_exact(S.s1, F);
    if (S.s0 == 0) { d.kind = D_MERGED; return d; }
    const uint64_t s0 = S.s0;
    const U128 s0sq = mul64(s0, s0);                 // <= 2^78
    auto times_s0 = [&](U128 v) {                    // s0 v < 2^128
        U128 r = mul64(s0, v.lo);
        r.hi += s0 * v.hi;
        return r;
    };
    U128 V[6], D[6];
#pragma unroll
    for (int l = 0; l < 6; ++l) {
        const uint64_t s1 = uabs64(S.s1[l]);
        const U128 sq = mul64(s1, s1);
        V[l] = sub128(times_s0(S.s2[l]), sq);
        D[l] = l < 3 ? shl128(s0sq, 32) : sq;
    }
    bool done = true;
    {
        const U256 rhs = mul128(u128_make(K.thx2, 0), s0sq);      // That^2 S0^2
#pragma unroll
        for (int a = 0; a < 3; ++a)
            if (!is_zero128(V[a]) && cmp256(mul128(V[a], u128_make(1ull << 16, 0)), rhs) > 0) done = false;
        const U128 tp2 = u128_make(K.thp2, 0);
#pragma unroll
        for (int a = 3; a < 6; ++a) {
            if (is_zero128(V[a])) continue;
            if (is_zero128(D[a])) { done = false; continue; }
            if (cmp256(mul128(V[a], u128_make(1ull << 48, 0)), mul128(tp2, D[a])) > 0) done = false;
        }
    }
    if (done) { d.kind = D_MERGED; return d; }
    const bool xinf = K.tx2 == 0, pinf = K.tp2 == 0;
    int kx = 0;
    U128 xV = V[0];
#pragma unroll
    for (int l = 1; l < 3; ++l)
        if (xinf ? is_zero128(xV) && !is_zero128(V[l]) : cmp128(V[l], xV) > 0) { kx = l; xV = V[l]; }
    int kp = 3;
    U128 pV = V[3], pD = D[3];
#pragma unroll
    for (int l = 4; l < 6; ++l)
        if (pinf ? is_zero128(pV) && !is_zero128(V[l]) : frac_gt(V[l], D[l], pV, pD)) { kp = l; pV = V[l]; pD = D[l]; }
    const int k = frac_gt_norm(pV, pD, K.tp2, xV, D[0], K.tx2) ? kp : kx;
    int64_t s1k = S.s1[0];
#pragma unroll
    for (int l = 1; l < 6; ++l) if (l == k) s1k = S.s1[l];
    // Step 5: floor(S1 / S0) in integers (|S1 / S0| <= 2^22)
    const int64_t den = (int64_t)s0;
    int64_t t = s1k / den;
    if (t * den > s1k) t -= 1;
    d.kind = D_SPLIT;
    d.axis = k;
    d.thr = (int)t;
    return d;
}

// The same rule evaluated in floating point with error bounds.  Sets ok = false when a comparison
// cannot be certified (the caller then applies the exact rule).
//   V = S0 S2 - S1^2 in FP64 (S0, S1 exact): S2 is rounded over at most len + 6 operations, the FMA
//   and the rounding of S1^2 add at most 2 ulp of S0 S2 (S1^2 <= S0 S2), so
//       |V_fp64 - V| <= S0 S2 (len + 9) 2^-53 < EV = S2 fl(S0 (len + 16) 2^-51).
//   When S2 comes with its own error bound e2 (moments formed as a parent's minus a sibling's),
//       |V_fp64 - V| <= S0 (e2 + |S2| 2^-52) (1 + 2^-52) < EV = S0 (e2 + |S2| 2^-51) (1 + 2^-40).
//   Both Step 3 and Step 4 compare Delta_l^2 = V_l / D_l: Step 3 against tau^2 = (T^ / 2^24)^2 (given as
//   an FP32 bracket), Step 4 against the other axes.  Delta_l^2 is bracketed in FP32 from [V - EV,
//   V + EV] (conversions, a 1-ulp reciprocal and the products stay below 2^-21 relative; the
//   bracket is widened by 2^-19).  A subtraction of two floats has the sign of the exact difference,
//   so the maxima below decide the comparisons exactly.
// `amask` has bit l set for the axes whose codes vary in the cell; the others have V = 0.
VPM_DEV Decision decide_fast(const FSums& S, int len, const DecideConsts& K, const Frame& F, int amask, bool& ok,
                             const double* e2 = nullptr) {
    Decision d;
    d.axis = 0; d.thr = 0; d.jdir = 0;
    ok = true;
    const double s0 = S.s0;
    if (s0 == 0.0) { d.kind = D_MERGED; d.jdir = pair_axis(S.s1, F); return d; }
    const double s0slack = s0 * ((double)(len + 16) * 0x1p-51);
    const float rdx = __builtin_amdgcn_rcpf((float)(s0 * s0 * 0x1p32));
    const float rdx_lo = rdx * (1.0f - 0x1p-19f), rdx_hi = rdx * (1.0f + 0x1p-19f);
    float lo[6], hi[6];
    float over = -INFINITY;     // max_l (lower bound of Delta_l^2 - upper bound of tau^2) > 0: some axis fails
    float under = -INFINITY;    // max_l (upper bound of Delta_l^2 - lower bound of tau^2) <= 0: all pass
#pragma unroll
    for (int l = 0; l < 6; ++l) {
        lo[l] = 0.0f; hi[l] = 0.0f;
        if (!((amask >> l) & 1)) continue;            // wave-uniform
        const double s1 = S.s1[l], s2 = S.s2[l];
        const double bh = s1 * s1;
        const double V = fma(s0, s2, -bh);
        const double EV = e2 ? s0 * (e2[l] + fabs(s2) * 0x1p-51) * (1.0 + 0x1p-40) : s2 * s0slack;
        const double vlo = V - EV, vhi = V + EV;
        float rlo, rhi;
        if (l < 3) {
            rlo = rdx_lo; rhi = rdx_hi;
        } else {                                       // D = S1^2; D = 0 gives +infinity
            const float r = __builtin_amdgcn_rcpf((float)bh);
            rlo = r * (1.0f - 0x1p-19f); rhi = r * (1.0f + 0x1p-19f);
        }
        const float lf = vlo > 0.0 ? (float)vlo * rlo : 0.0f;     // V > 0 certain
        const float hf = vhi < 1.0 ? 0.0f : (float)vhi * rhi;     // V is an integer: vhi < 1 gives V = 0
        lo[l] = lf; hi[l] = hf;
        over = fmaxf(over, lf - (l < 3 ? K.t2x_hi : K.t2p_hi));
        under = fmaxf(under, hf - (l < 3 ? K.t2x_lo : K.t2p_lo));
    }
    if (!(over > 0.0f)) {
        if (under > 0.0f) { ok = false; return d; }   // an axis too close to its tolerance
        d.kind = D_MERGED;
        d.jdir = pair_axis(S.s1, F);
        return d;
    }
    // Step 4 on the weighted CVs: under the normalised rule, outward FP32 brackets of 1 / T^2 (each
    // product rounds by at most 2^-24, inside the brackets' 2^-22 margin); an infinite weight (zero
    // tolerance) makes any CV > 0 infinite.  The raw rule's weights are 1.
    if (__builtin_amdgcn_readfirstlane(K.norm)) {
#pragma unroll
        for (int l = 0; l < 6; ++l) {
            const bool pos = l < 3;
            lo[l] = lo[l] > 0.0f ? lo[l] * (pos ? K.wx_lo : K.wp_lo) : 0.0f;
            hi[l] = hi[l] > 0.0f ? hi[l] * (pos ? K.wx_hi : K.wp_hi) : 0.0f;
        }
    }
    int k = 0;
    float best = lo[0];
#pragma unroll
    for (int l = 1; l < 6; ++l) if (lo[l] > best) { best = lo[l]; k = l; }
    float rival = -INFINITY;
#pragma unroll
    for (int l = 0; l < 6; ++l) rival = fmaxf(rival, l == k ? -INFINITY : hi[l]);
    if (!(best > rival)) { ok = false; return d; }
    double s1k = S.s1[0];
#pragma unroll
    for (int l = 1; l < 6; ++l) if (l == k) s1k = S.s1[l];
    // Step 5 threshold floor(S1/S0): approximate quotient, then exact correction (all products
    // below 2^53, so exact in FP64)
    double t = floor(s1k * __builtin_amdgcn_rcp(s0));
    while (t * s0 > s1k) t -= 1.0;
    while ((t + 1.0) * s0 <= s1k) t += 1.0;
    d.kind = D_SPLIT;
    d.axis = k;
    d.thr = (int)t;
    return d;
}

VPM_DEV int pack_decision(const Decision& d) {
    return (d.kind & 3) | ((d.axis & 7) << 2) | ((d.jdir & 3) << 5) | (d.thr << 7);
}
VPM_DEV Decision unpack_decision(int v) {
    Decision d;
    d.kind = v & 3; d.axis = (v >> 2) & 7; d.jdir = (v >> 5) & 3; d.thr = v >> 7;
    return d;
}

// log2 of the lane-group size for a subset of len particles: about 2^ppl_shift particles per lane,
// at most one wavefront.
VPM_DEV int group_class_for(int len, int ppl_shift) {
    const int want = (len + (1 << ppl_shift) - 1) >> ppl_shift;
    return want <= 1 ? 0 : min(32 - __clz(want - 1), 6);        // ceil(log2(want)), at most 6
}

VPM_DEV void wave_fence() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

VPM_DEV int frexp_exp(float v) {
    int e = 0;
    if (v > 0.0f) frexpf(v, &e);
    return e;
}

VPM_DEV int ceil_log2(int v) {
    int b = 0;
    while ((1 << b) < v) ++b;
    return b;
}

// q(a*b, G): the exact FP32 x FP32 product, rounded to nearest on the grid 2^-G.
VPM_DEV int64_t fixq(float a, float b, int G) {
    return __double2ll_rn(ldexp((double)a * (double)b, G));
}

// ------------------------------------------------------------------------------------------
// Per-cell memory (an LDS slice or a global slab) and kernel arguments.
// ------------------------------------------------------------------------------------------

struct CellShared {          // per-cell bookkeeping, in LDS
    int nnext;
    int nmerged;
    int cls_cnt[8];
    int cls_cur[8];
    uint32_t flags;
    int qi;                  // queue position of the current cell
    int rootv;               // packed decision of the root
    int kind;                // large-cell kernel: the claimed work (0 none, 1 a cell, 2 a task)
    int last;                // large-cell kernel: this workgroup finished the cell's last piece
    DecideConsts dc;         // written once per workgroup at the start of a kernel
};

// Subsets of a large cell handed to other workgroups (the large-cell kernel): those that a split
// leaves unfinished with at least TASK_MIN particles.  A level collects them here and publishes
// them as tasks once the level's writes are complete.  Smaller pieces are finished faster where
// they are than through a hand-off (measured over 2,048 to 32,768: 8,192 is best on whole boxes of
// 2 to 4 million particles and on populations with cells of up to 32,768).
constexpr int TASK_MIN = 8192;
constexpr int SPAWN_MAX = 64;          // per level: spawned subsets are disjoint, each >= TASK_MIN
template <typename IdxT>
struct SpawnList { int n; Node<IdxT> node[SPAWN_MAX]; };

// A subset handed from one wavefront to another in the inherited top levels of a cell shared by
// several wavefronts: its node, its moments and their S2 error bound.
struct Handoff {
    double P[13];            // S0, S1[6], S2[6]
    double E2[6];
    int32_t start, len, thr_axis, act;
};

// Cross-wave scratch of a cell processed by WPB > 1 wavefronts.
template <int WPB>
struct BlockScratch {
    float fmax[WPB][11];     // per-wave frame maxima
    int bad[WPB];
    double sums[WPB][13];    // per-wave root moments
    int64_t scan[WPB];       // per-wave totals of the output scan
    Handoff ho[WPB];         // inherited levels: the subset each wavefront takes over
    int vote[2][WPB];        // inherited levels: per-wave votes, alternating between levels
};

template <int WPB>
__host__ __device__ constexpr size_t header_bytes() {
    return ((sizeof(CellShared) + 15) & ~(size_t)15) + (WPB > 1 ? ((sizeof(BlockScratch<WPB>) + 15) & ~(size_t)15) : 0);
}

// Codes of particle i: rec[i] = {c_px, c_py, c_pz, omega | c_x << 16} (16 bytes, one 128-bit load)
// and pyz[i] = c_y | c_z << 16 (position codes are int16, momentum codes int32).
template <typename IdxT>
struct CellMem {
    CellShared* sh;
    int4* rec;
    int32_t* pyz;
    IdxT *idx0, *idx1;
    uint8_t* info;
    IdxT* emit;                    // output slot per position
    IdxT* sched;                   // schedule table of a level's subsets (the emit array in LDS bins)
    Node<IdxT> *nodes0, *nodes1;   // current / next level (leaf tables at the end)
};

__host__ __device__ constexpr size_t rnd16(size_t b) { return (b + 15) & ~(size_t)15; }

// Bytes of the per-cell arrays (without the LDS header).
template <typename IdxT>
__host__ __device__ constexpr size_t slice_bytes(int nmax) {
    return 2 * rnd16(((size_t)nmax / 2 + 2) * sizeof(Node<IdxT>)) + rnd16((size_t)nmax * 16) +
           rnd16((size_t)nmax * 4) + 2 * rnd16((size_t)nmax * sizeof(IdxT)) +
           rnd16(((size_t)nmax + 1) * sizeof(IdxT)) + rnd16((size_t)nmax);
}

template <typename IdxT>
VPM_DEV CellMem<IdxT> carve(uint8_t* base, int nmax) {
    CellMem<IdxT> M;
    size_t o = 0;
    auto take = [&](size_t bytes) { uint8_t* p = base + o; o += rnd16(bytes); return p; };
    M.sh = nullptr;
    M.nodes0 = (Node<IdxT>*)take(((size_t)nmax / 2 + 2) * sizeof(Node<IdxT>));
    M.nodes1 = (Node<IdxT>*)take(((size_t)nmax / 2 + 2) * sizeof(Node<IdxT>));
    M.rec = (int4*)take((size_t)nmax * 16);
    M.pyz = (int32_t*)take((size_t)nmax * 4);
    M.idx0 = (IdxT*)take((size_t)nmax * sizeof(IdxT));
    M.idx1 = (IdxT*)take((size_t)nmax * sizeof(IdxT));
    M.emit = (IdxT*)take(((size_t)nmax + 1) * sizeof(IdxT));
    M.info = (uint8_t*)take((size_t)nmax);
    M.sched = M.emit;
    return M;
}

// The particle input is FP32 (InT = float) or FP64 (InT = double, rounded to FP32 as it is loaded:
// the fixed-point path works on the FP32 values either way, so both give identical results).
template <typename InT>
struct FixedArgsT {
    using In = InT;
    SoaIn<InT> in;
    const int64_t* cell_off;
    const int32_t* queue;
    int32_t* counters;             // [qlen_index] = queue length, [work_index] = work counter
    int qlen_index, work_index;
    FixedParams P;
    int mode;                      // 0 run, 1 partition
    Soa32Out tmp;
    int64_t* out_count;
    uint8_t* cell_mode;
    uint32_t* flags;
    int32_t *perm, *subset_id, *n_subsets;
    const int32_t* bigq[BIGQ_CLASSES];   // the large-cell queue by size class (large-cell bin only)
};

template <typename IdxT>
VPM_DEV IdxT* idx_buf(const CellMem<IdxT>& M, int par) { return par ? M.idx1 : M.idx0; }


template <typename IdxT>
VPM_DEV void codes_of(const CellMem<IdxT>& M, int i, int c[6], int& om) {
    const int4 r = M.rec[i];
    const int v = M.pyz[i];
    om = r.w & 0xffff;
    c[0] = r.w >> 16; c[1] = (v << 16) >> 16; c[2] = v >> 16;
    c[3] = r.x; c[4] = r.y; c[5] = r.z;
}

// Decide one subset [start, start+len) of buffer `buf` from its FP64 moments; falls back to
// exact integer moments recomputed from the codes when the FP64 evaluation is inconclusive.
template <typename IdxT>
VPM_DEV Decision decide(const CellMem<IdxT>& M, const FSums& S, const IdxT* buf, int start, int len,
                        const FixedParams& P, const Frame& F, const double* e2 = nullptr) {
    Decision d;
    if (len < P.min_subset) { d.kind = D_COPY; d.axis = 0; d.thr = 0; d.jdir = 0; return d; }
    bool ok;
    const DecideConsts& K = M.sh->dc;
    d = decide_fast(S, len, K, F, F.amask, ok, e2);
    if (__builtin_expect(ok && !K.force_exact, 1)) return d;   // the exact path below is rare: laid out apart
    ISums E;
    E.s0 = 0;
#pragma unroll
    for (int l = 0; l < 6; ++l) E.s1[l] = 0;
#pragma unroll
    for (int a = 0; a < 3; ++a) { E.s2p[a] = 0; E.s2m[a] = u128_make(0, 0); }
    for (int j = 0; j < len; ++j) {
        int c[6], om;
        codes_of(M, buf[start + j], c, om);
        isums_add(E, (uint32_t)om, c);
    }
    return decide_exact(E, K, F);
}

// Make the cell's shared memory writes visible to all wavefronts working on the cell.
template <int WPB>
VPM_DEV void cell_sync() {
    if constexpr (WPB == 1) wave_fence();
    else __syncthreads();
}

// Sort the m items of a list into power-of-two lane-group classes (largest first).  Afterwards
// the lane groups of class c occupy virtual lanes [lb[c], lb[c] + (cnt[c] << c)) and
// sched[fb[c] + k] holds the k-th item of class c.  All threads of the cell call.
struct Sched { int lb[7], fb[7], cnt[7], total; };

template <int WPB, typename IdxT, typename LenFn>
VPM_DEV Sched schedule(const CellMem<IdxT>& M, IdxT* sched, int m, int ppl_shift, LenFn len_of) {
    const int tid = threadIdx.x;
    if (tid < 8) { M.sh->cls_cnt[tid] = 0; M.sh->cls_cur[tid] = 0; }
    cell_sync<WPB>();
    for (int it = tid; it < m; it += WAVE * WPB) atomicAdd(&M.sh->cls_cnt[group_class_for(len_of(it), ppl_shift)], 1);
    cell_sync<WPB>();
    Sched s;
    int l = 0, f = 0, top = 0;
#pragma unroll
    for (int c = 6; c >= 0; --c) {
        s.cnt[c] = M.sh->cls_cnt[c];
        s.lb[c] = l; s.fb[c] = f;
        l += s.cnt[c] << c; f += s.cnt[c];
        if (top == 0 && s.cnt[c] != 0) top = c;
    }
    s.total = l;
    // When the groups fill at most half of the cell's lanes, every group is widened by 2^bump (up
    // to a wavefront) while they still fit: fewer trips per lane, the same result.
    int bump = 0;
    while (bump < 6 - top && (l << (bump + 1)) <= WAVE * WPB) ++bump;
    if (bump > 0) {
        l = 0; f = 0;
#pragma unroll
        for (int c = 6; c >= 0; --c) {
            s.cnt[c] = c >= bump ? M.sh->cls_cnt[c - bump] : 0;
            s.lb[c] = l; s.fb[c] = f;
            l += s.cnt[c] << c; f += s.cnt[c];
        }
        s.total = l;
    }
    for (int it = tid; it < m; it += WAVE * WPB) {
        const int c = group_class_for(len_of(it), ppl_shift) + bump;
        const int r = atomicAdd(&M.sh->cls_cur[c], 1);
        int fbc = s.fb[0];
#pragma unroll
        for (int q = 1; q < 7; ++q) if (q == c) fbc = s.fb[q];
        sched[fbc + r] = (IdxT)it;
    }
    cell_sync<WPB>();
    return s;
}

// Virtual lane v -> (item slot, class).  Returns false if v is past the last group.
// The classes' lane ranges follow each other from class 6 (at 0) down to class 0, so v lies in the
// lowest class whose range starts at or before v (an empty class starts where the next one does).
VPM_DEV bool sched_lookup(const Sched& s, int v, int& slot, int& cls) {
    if (v >= s.total) return false;
    int c0 = 6, lbv = 0, fbv = 0;
#pragma unroll
    for (int c = 5; c >= 0; --c) {
        const bool in = v >= s.lb[c];
        c0 = in ? c : c0;
        lbv = in ? s.lb[c] : lbv;
        fbv = in ? s.fb[c] : fbv;
    }
    cls = c0;
    slot = fbv + ((v - lbv) >> c0);
    return true;
}

// Step 6 for one unfinished subset with a lane group: its members split into V1 (front of the slot
// range) and V2 (back); returns |V1|.  solo: every group of the round is a single lane.
template <typename IdxT>
VPM_DEV int compact_node(const CellMem<IdxT>& M, Node<IdxT> nd, int cur, int lid, int g, int gbase, bool solo) {
    const int start = nd.start, len = nd.len;
    const int k = nd.thr_axis & 7;
    const int thr = nd.thr_axis >> 8;
    const IdxT* src = idx_buf(M, cur);
    IdxT* dst = idx_buf(M, cur ^ 1);

    // Step 6 as one stable pass: the lower side V1 = {c <= thr} fills the range from the front in
    // slot order, V2 from the back in reverse slot order (so V2's member order flips).  Past the end
    // of the subset a lane reads the last slot again and stores nothing; ranks come from the wave
    // ballots restricted to the lane's group.
    const uint64_t gmask = (g == 64 ? ~0ull : ((1ull << g) - 1ull)) << gbase;
    // the axis-k code of particle i is one aligned 32-bit load: a word of rec[i] (x: its upper half,
    // momenta: whole words) or pyz[i] (y: lower half, z: upper half), then half-selected and
    // sign-extended for the int16 position codes
    const bool kpyz = k == 1 || k == 2;
    const uint8_t* cbase = kpyz ? (const uint8_t*)M.pyz : (const uint8_t*)M.rec + (k == 0 ? 12 : 4 * (k - 3));
    const uint32_t cstride = kpyz ? 4u : 16u;
    // one signed bit-field extract: bits [16, 32) for x and z, [0, 16) for y, [0, 24) for a momentum
    // code (|code| <= 2^22)
    const uint32_t boff = (k == 0 || k == 2) ? 16u : 0u, bwid = k < 3 ? 16u : 24u;
    auto code_of = [&](IdxT i) {
        const int w = *(const int32_t*)(cbase + (uint32_t)i * cstride);
        return __builtin_amdgcn_sbfe(w, boff, bwid);
    };
    // Batches of CB rounds: the indices of a batch are loaded together, then their codes, before
    // any is used (two LDS round trips per batch instead of a dependent pair per round; positions
    // past the subset's end repeat its last slot and store nothing).
    constexpr int CB = 4;
    const IdxT* sp = src + start;
    const int last = len - 1;
    int lb = 0, rb = 0;
    if (solo) {
        // every group of the round is a single lane (a wave-uniform fact): no ranks to exchange
        for (int j0 = 0; j0 < len; j0 += CB) {
            IdxT ix[CB];
            int cv[CB];
#pragma unroll
            for (int u = 0; u < CB; ++u) ix[u] = sp[min(j0 + u, last)];
#pragma unroll
            for (int u = 0; u < CB; ++u) cv[u] = code_of(ix[u]);
#pragma unroll
            for (int u = 0; u < CB; ++u) {                      // predicated: no branch per round
                const bool act = j0 + u < len;
                const bool right = cv[u] > thr;
                if (act) dst[start + (right ? last - rb : lb)] = ix[u];
                rb += (act && right) ? 1 : 0;
                lb += (act && !right) ? 1 : 0;
            }
        }
    } else
    for (int j0 = 0; j0 < len; j0 += CB * g) {
        IdxT ix[CB];
        int cv[CB];
#pragma unroll
        for (int u = 0; u < CB; ++u) ix[u] = sp[min(j0 + u * g + lid, last)];
#pragma unroll
        for (int u = 0; u < CB; ++u) cv[u] = code_of(ix[u]);
#pragma unroll
        for (int u = 0; u < CB; ++u) {
            const int jb = j0 + u * g;                          // the round's first position (group-uniform)
            // the active lanes of a group are a prefix of it: an active lane has lid active lanes
            // below it in the group, and the group has max(0, min(g, len - jb)) active lanes
            // (rounds past the end are predicated off rather than left by a branch)
            const bool act = jb + lid < len;
            const bool right = cv[u] > thr;
            const uint64_t bra = ballot(right) & ballot(act) & gmask;            // this group's lanes only
            const int rr = (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(bra >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)bra, 0u));
            if (act) dst[start + (right ? len - 1 - (rb + rr) : lb + (lid - rr))] = ix[u];
            const int nr = __popcll(bra);
            lb += max(0, min(g, len - jb)) - nr;
            rb += nr;
        }
    }
    wave_fence();
    return lb;

}

// The global-memory bin's Step 6 with the children's moments: as compact_node, but each member's
// whole record is loaded and added to the moments of the child it goes to while it is placed, so
// the members are read from global memory once instead of twice.  Eight rounds of indices, then
// records, are loaded before any is used.  Returns |V1|.
template <typename IdxT>
VPM_DEV int compact_sum_node(const CellMem<IdxT>& M, Node<IdxT> nd, int cur, int lid, int g, int gbase, bool solo,
                             FSums& L, FSums& R) {
    const int start = nd.start, len = nd.len;
    const int k = nd.thr_axis & 7;
    const int thr = nd.thr_axis >> 8;
    const IdxT* sp = idx_buf(M, cur) + start;
    IdxT* dst = idx_buf(M, cur ^ 1);
    const uint64_t gmask = (g == 64 ? ~0ull : ((1ull << g) - 1ull)) << gbase;
    const int last = len - 1;
    constexpr int B = 8;
    const int step = solo ? 1 : g;
    const int l0 = solo ? 0 : lid;
    int lb = 0, rb = 0;
    for (int j0 = 0; j0 < len; j0 += B * step) {
        IdxT ix[B];
        int4 r[B];
        int32_t v[B];
#pragma unroll
        for (int u = 0; u < B; ++u) ix[u] = sp[min(j0 + u * step + l0, last)];
#pragma unroll
        for (int u = 0; u < B; ++u) { r[u] = M.rec[ix[u]]; v[u] = M.pyz[ix[u]]; }
#pragma unroll
        for (int u = 0; u < B; ++u) {
            const int jb = j0 + u * step;                      // the round's first position (group-uniform)
            if (jb >= len) break;
            const int c0 = r[u].w >> 16, c1 = (v[u] << 16) >> 16, c2 = v[u] >> 16;
            const int cv = k == 0 ? c0 : k == 1 ? c1 : k == 2 ? c2 : k == 3 ? r[u].x : k == 4 ? r[u].y : r[u].z;
            const bool right = cv > thr;
            bool act = true;
            if (solo) {
                dst[start + (right ? last - rb : lb)] = ix[u];
                rb += right ? 1 : 0;
                lb += right ? 0 : 1;
            } else {
                act = jb + lid < len;
                const uint64_t bra = ballot(right) & ballot(act) & gmask;
                const int rr = (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(bra >> 32),
                                                              __builtin_amdgcn_mbcnt_lo((uint32_t)bra, 0u));
                if (act) dst[start + (right ? len - 1 - (rb + rr) : lb + (lid - rr))] = ix[u];
                const int nr = __popcll(bra);
                lb += min(g, len - jb) - nr;
                rb += nr;
            }
            const int om = act ? (r[u].w & 0xffff) : 0;            // weight 0 adds nothing
            fsums_add(L, right ? 0 : om, c0, c1, c2, r[u].x, r[u].y, r[u].z);
            fsums_add(R, right ? om : 0, c0, c1, c2, r[u].x, r[u].y, r[u].z);
        }
    }
    wave_fence();
    return lb;
}

// A final subset [cs, cs + cl) of the new slot order: its flags for the output, and its members put
// back into increasing input order where that order is observable (copied particles, or the
// partition output).  Lanes lid < g of its group take part.
template <typename IdxT, typename Args>
VPM_DEV void record_final(const CellMem<IdxT>& M, const Args& A, const Decision& d, int cs, int cl, int crev,
                          int cur, int lid, int g) {
    IdxT* dst = idx_buf(M, cur ^ 1);
    if (crev && (d.kind == D_COPY || A.mode == 1)) {
        for (int j = lid; j < cl / 2; j += g) {
            const IdxT a = dst[cs + j], b = dst[cs + cl - 1 - j];
            dst[cs + j] = b;
            dst[cs + cl - 1 - j] = a;
        }
    }
    const uint8_t base = INF_SET | (uint8_t)((cur ^ 1) & 1) | (d.kind == D_MERGED ? INF_MERGED : 0) |
                         (uint8_t)(d.jdir << INF_JSHIFT);
    for (int j = lid; j < cl; j += g) M.info[cs + j] = base | (j == 0 ? INF_HEAD : 0);
}

// Moments of the members src[0 .. cnt) over a lane group (lanes lid < g take part).
template <typename IdxT>
VPM_DEV void sum_members(const CellMem<IdxT>& M, FSums& S, const IdxT* src, int cnt, int lid, int g) {
#pragma unroll 2
    for (int j = lid; j < cnt; j += g) {
        int c[6], om;
        codes_of(M, src[j], c, om);
        fsums_add(S, om, c[0], c[1], c[2], c[3], c[4], c[5]);
    }
}

// Process one unfinished subset with a lane group: compaction, child moments, child decisions.
template <typename IdxT, typename Args>
VPM_DEV void split_node(const CellMem<IdxT>& M, const Args& A, const Frame& F0, const Frame* frames, Node<IdxT> nd,
                        int cur, int lid, int g, int gbase, Node<IdxT>* next, bool solo,
                        SpawnList<IdxT>* spawn = nullptr) {
    const int start = nd.start, len = nd.len;
    const int rev = (nd.thr_axis >> 3) & 1;
    const int cell = (nd.thr_axis >> 4) & 15;
    const Frame& F = frames ? frames[cell] : F0;            // the frame of the subset's cell
    IdxT* dst = idx_buf(M, cur ^ 1);
    FSums L, R;
    fsums_zero(L); fsums_zero(R);
    int nl;
    if constexpr (sizeof(IdxT) == 4) nl = compact_sum_node(M, nd, cur, lid, g, gbase, solo, L, R);
    else nl = compact_node(M, nd, cur, lid, g, gbase, solo);

    const int n1 = nl, n2 = len - nl;
    int dv0, dv1;
    if (n1 == 0 || n2 == 0) {
        // Impossible under the exact rule (the chosen axis has V > 0); end the subset.
        Decision d; d.kind = D_MERGED; d.axis = 0; d.thr = 0; d.jdir = 0;
        if (lid == 0) atomicOr(&M.sh->flags, FLAG_INTERNAL);
        dv0 = pack_decision(d);
        dv1 = -1;
    } else {
        if constexpr (sizeof(IdxT) != 4) {
            // a child below min_subset is copied whatever its moments: skip its sums
            const int e1 = n1 >= A.P.min_subset ? n1 : 0, e2 = n2 >= A.P.min_subset ? n2 : 0;
            sum_members(M, L, dst + start, e1, lid, g);
            sum_members(M, R, dst + start + n1, e2, lid, g);
        }
        // lane 0 of the group decides V1 and lane 1 decides V2; a single lane decides both in turn
        if (g > 1) fsums_pair_reduce(L, R, lid, g);
        int mine0 = 0, mine1 = 0;
        const int ms = A.P.min_subset;
        // a one-lane group decides the first child that needs a decision; a second pass runs only
        // where both do
        const bool pick_r = g == 1 && n1 < ms;                 // V1 is copied: decide V2 first
        if (g == 1 || lid < 2) {
            const bool second = (g > 1 && lid == 1) || pick_r;
            FSums C;
            C.s0 = pick_r ? R.s0 : L.s0;
#pragma unroll
            for (int l = 0; l < 6; ++l) { C.s1[l] = pick_r ? R.s1[l] : L.s1[l]; C.s2[l] = pick_r ? R.s2[l] : L.s2[l]; }
            mine0 = pack_decision(decide(M, C, dst, second ? start + n1 : start, second ? n2 : n1, A.P, F));
        }
        if (g == 1) {
            Decision cp; cp.kind = D_COPY; cp.axis = 0; cp.thr = 0; cp.jdir = 0;
            if (pick_r) { mine1 = mine0; mine0 = pack_decision(cp); }
            else if (n2 < ms) mine1 = pack_decision(cp);
            else mine1 = pack_decision(decide(M, R, dst, start + n1, n2, A.P, F));
        }
        if (g == 1) {
            dv0 = mine0;
            dv1 = mine1;
        } else {
            dv0 = __shfl(mine0, gbase);
            dv1 = __shfl(mine0, gbase + 1);
        }
    }

    // record the children
    for (int ch = 0; ch < 2; ++ch) {
        const int dvv = ch == 0 ? dv0 : dv1;
        if (dvv == -1) continue;
        const Decision d = unpack_decision(dvv);
        const int cs = (dv1 == -1) ? start : (ch == 0 ? start : start + n1);
        const int cl = (dv1 == -1) ? len : (ch == 0 ? n1 : n2);
        const int crev = (dv1 == -1) ? (n1 == 0 ? rev ^ 1 : rev) : (ch == 0 ? rev : rev ^ 1);
        if (d.kind == D_SPLIT) {
            if (lid == 0) {
                Node<IdxT> c;
                c.start = (IdxT)cs; c.len = (IdxT)cl;
                c.thr_axis = (d.thr << 8) | (cell << 4) | (crev << 3) | d.axis;
                if (spawn && cl >= TASK_MIN) spawn->node[atomicAdd(&spawn->n, 1)] = c;   // to another workgroup
                else next[atomicAdd(&M.sh->nnext, 1)] = c;
            }
        } else {
            record_final(M, A, d, cs, cl, crev, cur, lid, g);
        }
    }
}

// Top levels without a scheduler.  Each unfinished subset owns an aligned group of g = 64 >> depth
// lanes that already hold its moments (and a bound e2 on the rounding error of its S2 sums): V1
// goes to the lower half of the group and V2 to the upper half, which then hold its moments.  Only
// the smaller child is summed; the other child's moments are the parent's minus these (S0 and S1
// exactly, S2 with its error bound carried along).
template <typename IdxT, typename Args>
VPM_DEV void split_inherit(const CellMem<IdxT>& M, const Args& A, const Frame& F, Node<IdxT>& nd, bool& act,
                           FSums& P, double (&E2)[6], int cur, int lid, int g, int gbase) {
    const int start = nd.start, len = nd.len;
    const int rev = (nd.thr_axis >> 3) & 1;
    IdxT* dst = idx_buf(M, cur ^ 1);
    const int n1 = compact_node(M, nd, cur, lid, g, gbase, false);
    const int n2 = len - n1;
    act = false;
    if (n1 == 0 || n2 == 0) {
        // impossible under the exact rule (the chosen axis has V > 0); end the subset
        if (lid == 0) atomicOr(&M.sh->flags, FLAG_INTERNAL);
        Decision d; d.kind = D_MERGED; d.axis = 0; d.thr = 0; d.jdir = 0;
        record_final(M, A, d, start, len, n1 == 0 ? rev ^ 1 : rev, cur, lid, g);
        return;
    }
    const bool s_first = n1 <= n2;                       // V1 is the smaller child
    const int ss = s_first ? start : start + n1, sl = s_first ? n1 : n2, ol = len - sl;
    FSums S;
    fsums_zero(S);
    if (ol >= A.P.min_subset) {                           // else both children are copied
#pragma unroll 2
        for (int j = lid; j < sl; j += g) {
            int c[6], om;
            codes_of(M, dst[ss + j], c, om);
            fsums_add(S, om, c[0], c[1], c[2], c[3], c[4], c[5]);
        }
        fsums_group_reduce(S, g);
    }
    double eS[6];
#pragma unroll
    for (int l = 0; l < 6; ++l) eS[l] = S.s2[l] * ((double)(sl + 16) * 0x1p-51);
    // the other child's moments and their S2 error bound
    auto other = [&](FSums& O, double (&eO)[6]) {
        O.s0 = P.s0 - S.s0;
#pragma unroll
        for (int l = 0; l < 6; ++l) {
            O.s1[l] = P.s1[l] - S.s1[l];
            O.s2[l] = P.s2[l] - S.s2[l];
            eO[l] = (E2[l] + eS[l] + fabs(O.s2[l]) * 0x1p-52) * (1.0 + 0x1p-40);
        }
    };
    const int h = g >> 1;
    const bool upper = lid >= h;                          // this lane's child: V2 if upper, else V1
    const bool mine_s = upper != s_first;
    // this lane's child's moments replace the parent's (P, E2), also for the next level
    {
        FSums O;
        double eO[6];
        other(O, eO);
        P.s0 = mine_s ? S.s0 : O.s0;
#pragma unroll
        for (int l = 0; l < 6; ++l) {
            P.s1[l] = mine_s ? S.s1[l] : O.s1[l];
            P.s2[l] = mine_s ? S.s2[l] : O.s2[l];
            E2[l] = mine_s ? eS[l] : eO[l];
        }
    }
    const int cs = upper ? start + n1 : start, cl = upper ? n2 : n1;
    int mine = 0;
    if ((lid & (h - 1)) == 0) mine = pack_decision(decide(M, P, dst, cs, cl, A.P, F, E2));
    const Decision d = unpack_decision(__shfl(mine, gbase + (upper ? h : 0)));
    const int crev = upper ? rev ^ 1 : rev;
    if (d.kind == D_SPLIT) {
        nd.start = (IdxT)cs; nd.len = (IdxT)cl;
        nd.thr_axis = (d.thr << 8) | (crev << 3) | d.axis;
        act = true;
    } else {
        record_final(M, A, d, cs, cl, crev, cur, lid & (h - 1), h);
    }
}

// The last inherited level: one lane per subset, which decides both children in turn and hands the
// unfinished ones to the scheduled levels (list `next`).
template <typename IdxT, typename Args>
VPM_DEV void split_inherit_solo(const CellMem<IdxT>& M, const Args& A, const Frame& F, Node<IdxT> nd,
                                const FSums& P, const double (&E2)[6], int cur, Node<IdxT>* next) {
    const int start = nd.start, len = nd.len;
    const int rev = (nd.thr_axis >> 3) & 1;
    IdxT* dst = idx_buf(M, cur ^ 1);
    const int n1 = compact_node(M, nd, cur, 0, 1, opaque_lane(), true);
    const int n2 = len - n1;
    if (n1 == 0 || n2 == 0) {
        atomicOr(&M.sh->flags, FLAG_INTERNAL);
        Decision d; d.kind = D_MERGED; d.axis = 0; d.thr = 0; d.jdir = 0;
        record_final(M, A, d, start, len, n1 == 0 ? rev ^ 1 : rev, cur, 0, 1);
        return;
    }
    const bool s_first = n1 <= n2;
    const int ss = s_first ? start : start + n1, sl = s_first ? n1 : n2, ol = len - sl;
    FSums S;
    fsums_zero(S);
    if (ol >= A.P.min_subset) {
#pragma unroll 2
        for (int j = 0; j < sl; ++j) {
            int c[6], om;
            codes_of(M, dst[ss + j], c, om);
            fsums_add(S, om, c[0], c[1], c[2], c[3], c[4], c[5]);
        }
    }
    FSums O;
    double eO[6];
    O.s0 = P.s0 - S.s0;
#pragma unroll
    for (int l = 0; l < 6; ++l) {
        O.s1[l] = P.s1[l] - S.s1[l];
        O.s2[l] = P.s2[l] - S.s2[l];
        eO[l] = (E2[l] + S.s2[l] * ((double)(sl + 16) * 0x1p-51) + fabs(O.s2[l]) * 0x1p-52) * (1.0 + 0x1p-40);
    }
    const int os = s_first ? start + n1 : start;
    const Decision dS = decide(M, S, dst, ss, sl, A.P, F);
    const Decision dO = decide(M, O, dst, os, ol, A.P, F, eO);
    for (int ch = 0; ch < 2; ++ch) {
        const Decision d = (ch == 0) == s_first ? dS : dO;
        const int cs = ch == 0 ? start : start + n1, cl = ch == 0 ? n1 : n2;
        const int crev = ch == 0 ? rev : rev ^ 1;
        if (d.kind == D_SPLIT) {
            Node<IdxT> c;
            c.start = (IdxT)cs; c.len = (IdxT)cl;
            c.thr_axis = (d.thr << 8) | (crev << 3) | d.axis;
            next[atomicAdd(&M.sh->nnext, 1)] = c;
        } else {
            record_final(M, A, d, cs, cl, crev, cur, 0, 1);
        }
    }
}

// The inherited levels of a one-wavefront cell from its root (a split, moments R over n particles)
// down to two lanes per subset, or until some subset would need more than INHERIT_PPL particles per
// lane; the unfinished subsets then go to the scheduled levels.  Leaves in cur / m the level and
// the number of subsets in its list.
constexpr int INHERIT_PPL = 32;

template <typename IdxT, typename Args>
VPM_DEV void inherit_levels(const CellMem<IdxT>& M, const Args& A, const Frame& F, const FSums& R, int n,
                            const Decision& rd, int lane, int& cur, int& m) {
    Node<IdxT> nd;
    nd.start = 0; nd.len = (IdxT)n; nd.thr_axis = (rd.thr << 8) | rd.axis;
    bool act = true;
    FSums P = R;
    double E2[6];
#pragma unroll
    for (int l = 0; l < 6; ++l) E2[l] = R.s2[l] * ((double)(n + 16) * 0x1p-51);
    int g = WAVE;
    for (; g >= 2; g >>= 1) {
        if (ballot(act && (int)nd.len > INHERIT_PPL * g) != 0) break;
        if (act) split_inherit(M, A, F, nd, act, P, E2, cur, lane & (g - 1), g, lane & ~(g - 1));
        wave_fence();
        cur ^= 1;
    }
    if (g == 1 && ballot(act && (int)nd.len > INHERIT_PPL) == 0) {
        if (lane == 0) M.sh->nnext = 0;
        wave_fence();
        if (act) split_inherit_solo(M, A, F, nd, P, E2, cur, cur ? M.nodes0 : M.nodes1);
        wave_fence();
        cur ^= 1;
        m = M.sh->nnext;
        return;
    }
    // the unfinished subsets, one per group of g lanes, to the scheduled levels
    Node<IdxT>* list = cur ? M.nodes1 : M.nodes0;
    const bool lead = act && (lane & (g - 1)) == 0;
    const uint64_t b = ballot(lead);
    if (lead) list[__popcll(b & lanes_below_of(lane))] = nd;
    m = __popcll(b);
    wave_fence();
}

// A top level of a cell shared by several wavefronts: the wavefront that owns subset nd splits it with
// all its lanes (compaction, the smaller child's moments, the other's as the parent's minus these, the
// two children's decisions), keeps V1 and hands V2 to another wavefront through `out` (written by
// lane 0; out->act stays 0 when V2 is final).  Finished children are recorded by the whole wavefront.
template <typename IdxT, typename Args>
VPM_DEV void split_handoff(const CellMem<IdxT>& M, const Args& A, const Frame& F, Node<IdxT>& nd, bool& act,
                           FSums& P, double (&E2)[6], int cur, Handoff* out) {
    const int lane = opaque_lane();
    const int start = nd.start, len = nd.len;
    const int rev = (nd.thr_axis >> 3) & 1;
    IdxT* dst = idx_buf(M, cur ^ 1);
    const int n1 = compact_node(M, nd, cur, lane, WAVE, 0, false);
    const int n2 = len - n1;
    act = false;
    if (n1 == 0 || n2 == 0) {
        // impossible under the exact rule (the chosen axis has V > 0); end the subset
        if (lane == 0) atomicOr(&M.sh->flags, FLAG_INTERNAL);
        Decision d; d.kind = D_MERGED; d.axis = 0; d.thr = 0; d.jdir = 0;
        record_final(M, A, d, start, len, n1 == 0 ? rev ^ 1 : rev, cur, lane, WAVE);
        return;
    }
    const bool s_first = n1 <= n2;
    const int ss = s_first ? start : start + n1, sl = s_first ? n1 : n2, ol = len - sl;
    FSums S;
    fsums_zero(S);
    if (ol >= A.P.min_subset) {                           // else both children are copied
#pragma unroll 2
        for (int j = lane; j < sl; j += WAVE) {
            int c[6], om;
            codes_of(M, dst[ss + j], c, om);
            fsums_add(S, om, c[0], c[1], c[2], c[3], c[4], c[5]);
        }
        fsums_group_reduce(S, WAVE);
    }
    double eS[6];
#pragma unroll
    for (int l = 0; l < 6; ++l) eS[l] = S.s2[l] * ((double)(sl + 16) * 0x1p-51);
    FSums O;
    double eO[6];
    O.s0 = P.s0 - S.s0;
#pragma unroll
    for (int l = 0; l < 6; ++l) {
        O.s1[l] = P.s1[l] - S.s1[l];
        O.s2[l] = P.s2[l] - S.s2[l];
        eO[l] = (E2[l] + eS[l] + fabs(O.s2[l]) * 0x1p-52) * (1.0 + 0x1p-40);
    }
    // lane 0 decides V1 and lane 1 decides V2
    const bool second = lane == 1;
    const bool mine_s = second != s_first;
    FSums C;
    double eC[6];
    C.s0 = mine_s ? S.s0 : O.s0;
#pragma unroll
    for (int l = 0; l < 6; ++l) {
        C.s1[l] = mine_s ? S.s1[l] : O.s1[l];
        C.s2[l] = mine_s ? S.s2[l] : O.s2[l];
        eC[l] = mine_s ? eS[l] : eO[l];
    }
    int mine = 0;
    if (lane < 2) mine = pack_decision(decide(M, C, dst, second ? start + n1 : start, second ? n2 : n1, A.P, F, eC));
    const Decision d1 = unpack_decision(__shfl(mine, 0)), d2 = unpack_decision(__shfl(mine, 1));
    if (d2.kind == D_SPLIT) {
        if (second) {                                      // lane 1 holds V2's moments in C
            out->start = start + n1;
            out->len = n2;
            out->thr_axis = (d2.thr << 8) | ((rev ^ 1) << 3) | d2.axis;
            out->act = 1;
            out->P[0] = C.s0;
#pragma unroll
            for (int l = 0; l < 6; ++l) { out->P[1 + l] = C.s1[l]; out->P[7 + l] = C.s2[l]; out->E2[l] = eC[l]; }
        }
    } else {
        record_final(M, A, d2, start + n1, n2, rev ^ 1, cur, lane, WAVE);
    }
    if (d1.kind == D_SPLIT) {
        nd.start = (IdxT)start; nd.len = (IdxT)n1;
        nd.thr_axis = (d1.thr << 8) | (rev << 3) | d1.axis;
        act = true;
        const bool v1s = s_first;                          // V1's moments: S if V1 is the smaller child
        P.s0 = v1s ? S.s0 : O.s0;
#pragma unroll
        for (int l = 0; l < 6; ++l) {
            P.s1[l] = v1s ? S.s1[l] : O.s1[l];
            P.s2[l] = v1s ? S.s2[l] : O.s2[l];
            E2[l] = v1s ? eS[l] : eO[l];
        }
    } else {
        record_final(M, A, d1, start, n1, rev, cur, lane, WAVE);
    }
}

// Block-wide vote: whether pred holds in any thread of the workgroup (every thread calls; one
// barrier; the vote slots alternate between calls so that a slot is rewritten only after the
// barrier of the next call).
template <int WPB>
VPM_DEV bool block_any(BlockScratch<WPB>* bs, bool pred, int& parity) {
    const int wv = threadIdx.x / WAVE;
    if (lane_id() == 0) bs->vote[parity][wv] = ballot(pred) != 0;
    __syncthreads();
    bool any = false;
#pragma unroll
    for (int w = 0; w < WPB; ++w) any |= bs->vote[parity][w] != 0;
    parity ^= 1;
    return any;
}

// The inherited levels of a cell shared by WPB > 1 wavefronts.  The root (a split; its moments and
// node in bs->ho[0], written by the thread that decided it) belongs to wavefront 0.  For the first
// log2(WPB) levels every wavefront that owns a subset splits it with all its lanes, keeps V1 and
// hands V2 to wavefront wv + step; from then on each wavefront continues alone with the
// one-wavefront inherited levels (lane groups halving down to one lane).  All wavefronts take the
// same number of levels (block-wide votes), so that all open subsets sit in the same index buffer
// when they go to the scheduled levels.  Leaves in cur / m the level and the length of its list.
template <int WPB, typename IdxT, typename Args>
VPM_DEV void inherit_block(const CellMem<IdxT>& M, const Args& A, const Frame& F, BlockScratch<WPB>* bs, int& cur,
                           int& m) {
    const int wv = threadIdx.x / WAVE;
    const int lane = opaque_lane();
    Node<IdxT> nd;
    bool act;
    FSums P;
    double E2[6];
    auto take = [&](int w) {
        const Handoff& h = bs->ho[w];
        act = h.act != 0;
        nd.start = (IdxT)h.start; nd.len = (IdxT)h.len; nd.thr_axis = h.thr_axis;
        P.s0 = h.P[0];
#pragma unroll
        for (int l = 0; l < 6; ++l) { P.s1[l] = h.P[1 + l]; P.s2[l] = h.P[7 + l]; E2[l] = h.E2[l]; }
    };
    take(wv);                                           // wavefront 0: the root; the others: nothing yet
    for (int step = 1; step < WPB; step <<= 1) {
        if (wv < step && act) split_handoff(M, A, F, nd, act, P, E2, cur, &bs->ho[wv + step]);
        cur ^= 1;
        __syncthreads();
        if (wv >= step && wv < 2 * step) take(wv);
    }
    int parity = 0;
    int g = WAVE;
    for (; g >= 2; g >>= 1) {
        if (block_any<WPB>(bs, act && (int)nd.len > INHERIT_PPL * g, parity)) break;
        if (act) split_inherit(M, A, F, nd, act, P, E2, cur, lane & (g - 1), g, lane & ~(g - 1));
        wave_fence();
        cur ^= 1;
    }
    const bool solo = g == 1 && !block_any<WPB>(bs, act && (int)nd.len > INHERIT_PPL, parity);
    if (threadIdx.x == 0) M.sh->nnext = 0;
    __syncthreads();
    if (solo) {
        if (act) split_inherit_solo(M, A, F, nd, P, E2, cur, cur ? M.nodes0 : M.nodes1);
        cur ^= 1;
    } else {
        // the open subsets, one per group of g lanes, to the scheduled levels
        Node<IdxT>* list = cur ? M.nodes1 : M.nodes0;
        const bool lead = act && (lane & (g - 1)) == 0;
        const uint64_t b = ballot(lead);
        int base = 0;
        if (lane == 0 && b != 0) base = atomicAdd(&M.sh->nnext, __popcll(b));
        base = __shfl(base, 0);
        if (lead) list[base + __popcll(b & lanes_below_of(lane))] = nd;
    }
    __syncthreads();
    m = M.sh->nnext;
    __syncthreads();                                    // nnext is read before the levels reset it
}

// Copy particles unchanged from the input to the staging arrays.// Copy particles unchanged from the input to the staging arrays.  For positions p = first,
// first + stride, ... below end, slot(p, src, dst) gives the input index and the staging slot, or
// dst < 0 for nothing (src must then still be a valid input index).  The loads of CB positions are
// all issued before their stores: the two arrays never overlap, but the compiler cannot know that
// and would otherwise wait for every load before the next store.  The slots are looked up without
// branches (positions past the end look up the last one and store nothing), so that no branch
// separates the loads of a batch.
constexpr int COPY_BATCH = 4;          // particles per lane whose loads are in flight together

template <int CB, typename InT, typename SlotFn>
VPM_DEV void copy_particles(const SoaIn<InT>& in, const Soa32Out& out, int first, int end, int stride, SlotFn slot) {
    for (int p0 = first; p0 < end; p0 += CB * stride) {
        int64_t si[CB], so[CB];
#pragma unroll
        for (int u = 0; u < CB; ++u) {
            const int p = p0 + u * stride;
            slot(min(p, end - 1), si[u], so[u]);
            if (p >= end) so[u] = -1;
        }
        float v[CB][7];
#pragma unroll
        for (int u = 0; u < CB; ++u) {
            const int64_t i = si[u];
            v[u][0] = (float)in.x[i]; v[u][1] = (float)in.y[i]; v[u][2] = (float)in.z[i];
            v[u][3] = (float)in.px[i]; v[u][4] = (float)in.py[i]; v[u][5] = (float)in.pz[i]; v[u][6] = (float)in.w[i];
        }
#pragma unroll
        for (int u = 0; u < CB; ++u) {
            if (so[u] < 0) continue;
            const int64_t o = so[u];
            out.x[o] = v[u][0]; out.y[o] = v[u][1]; out.z[o] = v[u][2];
            out.px[o] = v[u][3]; out.py[o] = v[u][4]; out.pz[o] = v[u][5]; out.w[o] = v[u][6];
        }
    }
}

// Merge one finished subset with a lane group (Step 7) and write its 1 or 2 particles.
//
// Two passes over the subset, all sums exact int64 on fixed grids (so the result does not depend
// on the summation order):
//   pass 1: W = sum w and sum w p on cell-wide grids  ->  a pivot momentum pt ~ P (FP32);
//   pass 2: sum w (x - lo), sum w (p - pt), sum w (eps_i - eps(pt)) on grids scaled to this
//           subset's own W, so subsets of light particles keep full precision.
// eps_i - eps(pt) is formed as (|d|^2 + 2 pt.d) / (eps_i + eps(pt)), d = p - pt, which does not
// cancel; the FP64 solve then forms r = mean(eps)^2 - m^2 - |P|^2 from these differences.
// gidx(j) gives the global index of the j-th member; the result goes to output slot `o` (and o+1).
template <typename Args, typename IdxFn>
VPM_DEV void merge_subset(const Args& A, const Frame& F, IdxFn gidx, int len, int jdir, int64_t o,
                          int lid, int g) {
    const int gb = 62 - ceil_log2(len);          // |term| < 2^gb keeps the sum below 2^62

    // pass 1
    const int gw = gb - F.ew;
    const int g1x = gb - F.ew - F.ep[0], g1y = gb - F.ew - F.ep[1], g1z = gb - F.ew - F.ep[2];
    int64_t sw = 0, s1x = 0, s1y = 0, s1z = 0;
    for (int j = lid; j < len; j += g) {
        const int64_t i = gidx(j);
        const float w = (float)A.in.w[i];
        sw += fixq(w, 1.0f, gw);
        s1x += fixq(w, (float)A.in.px[i], g1x);
        s1y += fixq(w, (float)A.in.py[i], g1y);
        s1z += fixq(w, (float)A.in.pz[i], g1z);
    }
    sw = group_sum(sw, g);
    s1x = group_sum(s1x, g); s1y = group_sum(s1y, g); s1z = group_sum(s1z, g);
    const double W = ldexp((double)sw, -gw);
    const float q0 = (float)(ldexp((double)s1x, -g1x) / W);
    const float q1 = (float)(ldexp((double)s1y, -g1y) / W);
    const float q2 = (float)(ldexp((double)s1z, -g1z) / W);

    // pass 2
    int eW = 0;
    frexp(W, &eW);                                // W < 2^eW
    const int gx0 = 61 - eW - F.ext_e[0], gx1 = 61 - eW - F.ext_e[1], gx2 = 61 - eW - F.ext_e[2];
    const int gd0 = 61 - eW - F.ep[0] - 1, gd1 = 61 - eW - F.ep[1] - 1, gd2 = 61 - eW - F.ep[2] - 1;
    const int ge = 61 - eW - F.eb;
    const float m = (float)F.mass;
    const float m2 = m * m;
    const float e0f = sqrtf(m2 + (q0 * q0 + q1 * q1 + q2 * q2));
    int64_t sx0 = 0, sx1 = 0, sx2 = 0, sd0 = 0, sd1 = 0, sd2 = 0, se = 0;
    for (int j = lid; j < len; j += g) {
        const int64_t i = gidx(j);
        const float w = (float)A.in.w[i];
        const float x = (float)A.in.x[i] - F.lo[0], y = (float)A.in.y[i] - F.lo[1], z = (float)A.in.z[i] - F.lo[2];
        const float px = (float)A.in.px[i], py = (float)A.in.py[i], pz = (float)A.in.pz[i];
        const float d0 = px - q0, d1 = py - q1, d2 = pz - q2;
        sx0 += fixq(w, x, gx0); sx1 += fixq(w, y, gx1); sx2 += fixq(w, z, gx2);
        sd0 += fixq(w, d0, gd0); sd1 += fixq(w, d1, gd1); sd2 += fixq(w, d2, gd2);
        if (A.P.merge_mode == VPM_MERGE_PAIR) {
            const float eps = sqrtf(m2 + (px * px + py * py + pz * pz));
            const float den = eps + e0f;
            const float num = (d0 * d0 + d1 * d1 + d2 * d2) + 2.0f * (q0 * d0 + q1 * d1 + q2 * d2);
            se += fixq(w, den > 0.0f ? num / den : 0.0f, ge);
        }
    }
    sx0 = group_sum(sx0, g); sx1 = group_sum(sx1, g); sx2 = group_sum(sx2, g);
    sd0 = group_sum(sd0, g); sd1 = group_sum(sd1, g); sd2 = group_sum(sd2, g);
    se = group_sum(se, g);
    if (lid != 0) return;

    const double X[3] = {F.lo[0] + ldexp((double)sx0, -gx0) / W,
                         F.lo[1] + ldexp((double)sx1, -gx1) / W,
                         F.lo[2] + ldexp((double)sx2, -gx2) / W};
    const double pt[3] = {q0, q1, q2};
    const double Pm[3] = {pt[0] + ldexp((double)sd0, -gd0) / W,
                          pt[1] + ldexp((double)sd1, -gd1) / W,
                          pt[2] + ldexp((double)sd2, -gd2) / W};
    if (A.P.merge_mode == VPM_MERGE_CENTROID) {
        A.tmp.w[o] = (float)W;
        A.tmp.x[o] = (float)X[0]; A.tmp.y[o] = (float)X[1]; A.tmp.z[o] = (float)X[2];
        A.tmp.px[o] = (float)Pm[0]; A.tmp.py[o] = (float)Pm[1]; A.tmp.pz[o] = (float)Pm[2];
        return;
    }
    const double md = F.mass;
    const double et = sqrt(md * md + (pt[0] * pt[0] + pt[1] * pt[1] + pt[2] * pt[2]));
    const double P2 = Pm[0] * Pm[0] + Pm[1] * Pm[1] + Pm[2] * Pm[2];
    const double e0 = sqrt(md * md + P2);
    const double a1 = ldexp((double)se, -ge) / W;               // mean energy - eps(pt)
    const double dn = et + e0;
    const double a2 = dn > 0.0 ? ((pt[0] - Pm[0]) * (pt[0] + Pm[0]) + (pt[1] - Pm[1]) * (pt[1] + Pm[1]) +
                                  (pt[2] - Pm[2]) * (pt[2] + Pm[2])) / dn
                               : 0.0;                             // eps(pt) - eps(P)
    const double Aex = a1 + a2;                                   // mean energy - eps(P)
    double r = Aex * (Aex + 2.0 * e0);
    if (!(r > 0.0)) r = 0.0;
    const double pj = jdir == 0 ? Pm[0] : (jdir == 1 ? Pm[1] : Pm[2]);
    double u[3] = {jdir == 0 ? 1.0 : 0.0, jdir == 1 ? 1.0 : 0.0, jdir == 2 ? 1.0 : 0.0};
    if (P2 > 0.0) {
        const double f = pj / P2;
        u[0] -= f * Pm[0]; u[1] -= f * Pm[1]; u[2] -= f * Pm[2];
    }
    const double un = sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
    const double s = sqrt(r) / un;
    for (int h = 0; h < 2; ++h) {
        const double sg = h == 0 ? s : -s;
        A.tmp.w[o + h] = (float)(0.5 * W);
        A.tmp.x[o + h] = (float)X[0]; A.tmp.y[o + h] = (float)X[1]; A.tmp.z[o + h] = (float)X[2];
        A.tmp.px[o + h] = (float)(Pm[0] + sg * u[0]);
        A.tmp.py[o + h] = (float)(Pm[1] + sg * u[1]);
        A.tmp.pz[o + h] = (float)(Pm[2] + sg * u[2]);
    }
}

VPM_DEV float wave_max(float v) { return group_max(v, WAVE); }

// Inclusive scan over the wavefront; `ln` is this lane's index (passed in so that the exchange
// addresses are formed here rather than precomputed for the whole kernel).
template <typename V>
VPM_DEV V wave_incl_scan(V v, int ln) {
#pragma unroll
    for (int d = 1; d < WAVE; d <<= 1) {
        const V o = __shfl(v, ln - d);
        if (ln >= d) v += o;
    }
    return v;
}

// Step 1 accumulators: validity and the cell's extreme values.
struct FrameAcc {
    float v[11];     // max w; max -x_a (so min x_a); max x_a; max |p_a|
    bool bad;
};

VPM_DEV void facc_init(FrameAcc& a) {
    a.v[0] = 0.0f;
    for (int k = 0; k < 3; ++k) { a.v[1 + k] = -INFINITY; a.v[4 + k] = -INFINITY; a.v[7 + k] = 0.0f; }
    a.bad = false;
}

VPM_DEV void facc_add(FrameAcc& a, const float q[7]) {
    const float w = q[6];
    bool ok = w > 0.0f && isfinite(w);
    for (int l = 0; l < 6; ++l) ok = ok && isfinite(q[l]);
    a.bad |= !ok;
    a.v[0] = fmaxf(a.v[0], w);
    for (int k = 0; k < 3; ++k) {
        a.v[1 + k] = fmaxf(a.v[1 + k], -q[k]);
        a.v[4 + k] = fmaxf(a.v[4 + k], q[k]);
        a.v[7 + k] = fmaxf(a.v[7 + k], fabsf(q[3 + k]));
    }
}

// Reads particles off + p for p = first, first + stride, ... below n, LOAD_BATCH positions per lane at
// a time with every load of a batch unconditional (a position past the end reads particle n - 1
// again), so that a batch's loads are in flight together; fn(p, q, in_range) sees each of them.
constexpr int LOAD_BATCH = 8;

template <typename InT, typename Fn>
VPM_DEV void load_particles(const SoaIn<InT>& in, int64_t off, int first, int n, int stride, Fn fn) {
    constexpr int LB = sizeof(InT) == 4 ? LOAD_BATCH : LOAD_BATCH / 2;    // FP64: as many bytes in flight
    const InT* const b[7] = {in.x + off, in.y + off, in.z + off, in.px + off, in.py + off, in.pz + off, in.w + off};
    for (int p0 = first; p0 < n; p0 += LB * stride) {
        float q[LB][7];
#pragma unroll
        for (int u = 0; u < LB; ++u) {
            const uint32_t i = (uint32_t)min(p0 + u * stride, n - 1);
#pragma unroll
            for (int f = 0; f < 7; ++f) q[u][f] = (float)b[f][i];            // FP64: rounded to nearest
        }
#pragma unroll
        for (int u = 0; u < LB; ++u) fn(p0 + u * stride, q[u], p0 + u * stride < n);
    }
}

// Frame accumulation over positions first, first + stride, ... of a cell (duplicates change nothing).
template <typename InT>
VPM_DEV void facc_cell(FrameAcc& a, const SoaIn<InT>& in, int64_t off, int first, int n, int stride) {
    load_particles(in, off, first, n, stride, [&](int, const float* q, bool) { facc_add(a, q); });
}

// The frame from the cell maxima v (identical in every lane).
VPM_DEV void frame_from(const float v[11], double mass, Frame& F) {
    F.mass = mass;
    F.wmax = v[0];
    F.ew = frexp_exp(F.wmax);
    F.amask = 0;
    for (int k = 0; k < 3; ++k) {
        F.lo[k] = -v[1 + k];
        F.hi[k] = v[4 + k];
        F.pmax[k] = v[7 + k];
        F.pzero[k] = F.pmax[k] == 0.0f;
        F.ep[k] = frexp_exp(F.pmax[k]);
        F.ext_e[k] = frexp_exp(F.hi[k] - F.lo[k]);
        if (F.hi[k] > F.lo[k]) F.amask |= 1 << k;          // else every position code is equal
        if (!F.pzero[k]) F.amask |= 1 << (3 + k);          // else every momentum code is 0
    }
    // |eps_i - eps_j| <= m + |p|_1 for any two particles of the cell; 4x margin
    F.eb = frexp_exp(4.0f * ((float)mass + F.pmax[0] + F.pmax[1] + F.pmax[2]));
}

// The frame of a cell from the accumulators of a whole wavefront.  Returns false if some weight is
// not positive or some value is not finite.
VPM_DEV bool frame_of_wave(FrameAcc& acc, double mass, Frame& F) {
    if (ballot(acc.bad) != 0) return false;
#pragma unroll
    for (int r = 0; r < 11; ++r) acc.v[r] = wave_max(acc.v[r]);
    frame_from(acc.v, mass, F);
    F.amask = __builtin_amdgcn_readfirstlane(F.amask);     // wave-uniform: scalar branches
    return true;
}

// Step 1 for one cell (whole wave): validate the values and build the cell frame.
template <typename InT>
VPM_DEV bool cell_frame(const SoaIn<InT>& in, int64_t off, int n, double mass, Frame& F) {
    FrameAcc acc;
    facc_init(acc);
    facc_cell(acc, in, off, lane_id(), n, WAVE);
    return frame_of_wave(acc, mass, F);
}

// The same for a cell shared by WPB wavefronts (all threads call; the result is the same in all).
template <int WPB, typename InT>
VPM_DEV bool cell_frame_block(const SoaIn<InT>& in, int64_t off, int n, double mass, Frame& F, BlockScratch<WPB>* bs) {
    if constexpr (WPB == 1) {
        return cell_frame(in, off, n, mass, F);
    } else {
        const int wv = threadIdx.x / WAVE;
        FrameAcc acc;
        facc_init(acc);
        facc_cell(acc, in, off, threadIdx.x, n, WAVE * WPB);
        const bool bad = ballot(acc.bad) != 0;
#pragma unroll
        for (int r = 0; r < 11; ++r) acc.v[r] = wave_max(acc.v[r]);
        if (lane_id() == 0) {
            bs->bad[wv] = bad;
            for (int r = 0; r < 11; ++r) bs->fmax[wv][r] = acc.v[r];
        }
        __syncthreads();
        bool any_bad = false;
        float v[11];
        for (int r = 0; r < 11; ++r) v[r] = bs->fmax[0][r];
        for (int w = 0; w < WPB; ++w) {
            any_bad |= bs->bad[w] != 0;
            for (int r = 0; r < 11; ++r) v[r] = fmaxf(v[r], bs->fmax[w][r]);
        }
        __syncthreads();                                   // the scratch is reused below
        if (any_bad) return false;
        frame_from(v, mass, F);
        F.amask = __builtin_amdgcn_readfirstlane(F.amask);
        return true;
    }
}

// The whole cell in registers: thread t holds positions t, t + NT, ..., t + (RP - 1) NT (clamped to
// the last one past the end).  All the loads are issued before any is used, so that the cell costs
// one memory round trip; the frame and the codes are then formed from the registers.
template <int RP, int NT, typename InT>
VPM_DEV void load_cell_regs(const SoaIn<InT>& in, int64_t off, int n, int t, float (&q)[RP][7]) {
    const InT* const b[7] = {in.x + off, in.y + off, in.z + off, in.px + off, in.py + off, in.pz + off, in.w + off};
#pragma unroll
    for (int u = 0; u < RP; ++u) {
        const uint32_t i = (uint32_t)min(t + u * NT, n - 1);
#pragma unroll
        for (int f = 0; f < 7; ++f) q[u][f] = (float)b[f][i];            // FP64: rounded to nearest
    }
}

// Step 1 from a cell held in registers (load_cell_regs); all threads of the cell call.
template <int WPB, int RP>
VPM_DEV bool cell_frame_regs(const float (&q)[RP][7], int n, int t, double mass, Frame& F, BlockScratch<WPB>* bs) {
    constexpr int NT = WAVE * WPB;
    FrameAcc acc;
    facc_init(acc);
#pragma unroll
    for (int u = 0; u < RP; ++u)
        if (t + u * NT < n) facc_add(acc, q[u]);
    if constexpr (WPB == 1) {
        return frame_of_wave(acc, mass, F);
    } else {
        const int wv = threadIdx.x / WAVE;
        const bool bad = ballot(acc.bad) != 0;
#pragma unroll
        for (int r = 0; r < 11; ++r) acc.v[r] = wave_max(acc.v[r]);
        if (lane_id() == 0) {
            bs->bad[wv] = bad;
            for (int r = 0; r < 11; ++r) bs->fmax[wv][r] = acc.v[r];
        }
        __syncthreads();
        bool any_bad = false;
        float v[11];
        for (int r = 0; r < 11; ++r) v[r] = bs->fmax[0][r];
        for (int w = 0; w < WPB; ++w) {
            any_bad |= bs->bad[w] != 0;
            for (int r = 0; r < 11; ++r) v[r] = fmaxf(v[r], bs->fmax[w][r]);
        }
        __syncthreads();                                   // the scratch is reused below
        if (any_bad) return false;
        frame_from(v, mass, F);
        F.amask = __builtin_amdgcn_readfirstlane(F.amask);
        return true;
    }
}

// ------------------------------------------------------------------------------------------
// Replacement from a given partition (vpm_merge): one wavefront per cell, one lane per subset.
// ------------------------------------------------------------------------------------------

template <typename InT>
struct MergeArgs {
    FixedArgsT<InT> A;                   // in, params, tmp, out_count, cell_mode, flags
    const int32_t *perm, *subset_id, *n_subsets;
    int32_t* starts;               // scratch: first slot of every subset, indexed by input position
    int32_t* marks;                // scratch: a slot holding each member, indexed by input position
};

template <typename InT>
__global__ __launch_bounds__(WAVE) void k_fixed_merge(MergeArgs<InT> G) {
    const auto& A = G.A;
    const int lane = lane_id();
    const int npair = A.P.merge_mode == VPM_MERGE_PAIR ? 2 : 1;
    const int qlen = A.counters[A.qlen_index];
    if (qlen == 0) return;                         // an empty bin claims nothing
    for (;;) {
        int qi = 0;
        if (lane == 0) qi = atomicAdd(&A.counters[A.work_index], 1);
        qi = __shfl(qi, 0);
        if (qi >= qlen) break;
        const int c = A.queue[qi];
        const int64_t off = A.cell_off[c];
        const int n = (int)(A.cell_off[c + 1] - off);
        const int nsub = G.n_subsets[c];
        // the partition must be one of this cell's: members inside the cell, subset ordinals
        // 0, 1, ..., nsub-1 in runs; otherwise (or for an untouched cell) copy the cell unchanged
        bool ok = nsub >= 1 && nsub <= n;
        for (int p = lane; p < n && ok; p += WAVE) {
            const int32_t m = G.perm[off + p];
            const int32_t sd = G.subset_id[off + p];
            const int32_t prev = p == 0 ? -1 : G.subset_id[off + p - 1];
            ok = m >= off && m < off + n && sd >= 0 && sd < nsub && (sd == prev || sd == prev + 1) &&
                 (p != n - 1 || sd == nsub - 1);
        }
        bool part_ok = ballot(!ok) == 0;
        if (part_ok) {
            // every member exactly once: each slot writes its position at its member's mark, then
            // checks that the mark holds it (of two slots naming one member only one can pass, and
            // n slots naming n distinct members of the cell's n form a permutation)
            for (int p = lane; p < n; p += WAVE) G.marks[G.perm[off + p]] = (int32_t)(off + p);
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
            bool once = true;
            for (int p = lane; p < n; p += WAVE) once = once && G.marks[G.perm[off + p]] == (int32_t)(off + p);
            part_ok = ballot(!once) == 0;
        }
        Frame F;
        const bool vals_ok = part_ok && cell_frame(A.in, off, n, cell_mass(A.P.mass, A.P.species, A.P.species_mass, c), F);
        if (!vals_ok) {
            if (lane == 0) {
                if (part_ok || nsub >= 1) atomicOr(A.flags, part_ok ? FLAG_BAD_VALUE : FLAG_BAD_PARTITION);
                A.out_count[c] = n;
                A.cell_mode[c] = CELL_UNTOUCHED;
            }
            continue;
        }
        int32_t* st = G.starts + off;
        for (int p = lane; p < n; p += WAVE)
            if (p == 0 || G.subset_id[off + p] != G.subset_id[off + p - 1]) st[G.subset_id[off + p]] = p;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
        int64_t base = 0;
        for (int s0 = 0; s0 < nsub; s0 += WAVE) {
            const int sidx = s0 + lane;
            int b = 0, len = 0, e = 0;
            if (sidx < nsub) {
                b = st[sidx];
                len = (sidx + 1 < nsub ? st[sidx + 1] : n) - b;
                e = len >= A.P.min_subset ? npair : len;
            }
            int inc = e;
            for (int d = 1; d < WAVE; d <<= 1) {
                const int o = __shfl_up(inc, d);
                if (lane >= d) inc += o;
            }
            const int64_t slot = base + inc - e;
            base += __shfl(inc, WAVE - 1);
            if (sidx >= nsub) continue;
            const int32_t* mem = G.perm + off + b;
            if (len < A.P.min_subset) {
                copy_particles<4>(A.in, A.tmp, 0, len, 1, [&](int j, int64_t& si, int64_t& so) {
                    si = mem[j];
                    so = off + slot + j;
                });
                continue;
            }
            // pair direction from the momentum codes, exactly as the partition kernel does
            double s1[6] = {0, 0, 0, 0, 0, 0};
            for (int j = 0; j < len; ++j) {
                const int64_t i = mem[j];
                const double om = rintf(ldexpf((float)A.in.w[i], 15 - F.ew));
                const float pv[3] = {(float)A.in.px[i], (float)A.in.py[i], (float)A.in.pz[i]};
#pragma unroll
                for (int a = 0; a < 3; ++a)
                    s1[3 + a] += om * (F.pzero[a] ? 0.0 : (double)rintf(ldexpf(pv[a], 22 - F.ep[a])));
            }
            merge_subset(A, F, [&](int j) { return (int64_t)mem[j]; }, len, pair_axis(s1, F), off + slot, 0, 1);
        }
        if (lane == 0) {
            A.out_count[c] = base;
            A.cell_mode[c] = CELL_PROCESSED;
        }
    }
}

// The fixed-point codes of one particle (values q = x, y, z, px, py, pz, w) into slot i, and its
// contribution to the moments R; `oob` is set if a position lies more than one cell length above
// the cell's lowest one.
template <typename IdxT>
VPM_DEV void encode_particle(const CellMem<IdxT>& M, const FixedParams& P, const Frame& F, int i, const float* q,
                             FSums& R, bool& oob) {
    const int om = (int)rintf(ldexpf(q[6], 15 - F.ew));
    int cc[6];
    for (int a = 0; a < 3; ++a) {
        const float d = q[a] - F.lo[a];
        float r = rintf(d * P.s[a]);
        oob |= r > 65536.0f;
        r = fminf(r, 65535.0f);
        cc[a] = ((F.amask >> a) & 1) ? (int)r - 32768 : 0;   // constant axis: code 0
        cc[3 + a] = F.pzero[a] ? 0 : (int)rintf(ldexpf(q[3 + a], 22 - F.ep[a]));
    }
    M.rec[i] = make_int4(cc[3], cc[4], cc[5], (om & 0xffff) | (cc[0] << 16));
    M.pyz[i] = (cc[1] & 0xffff) | (cc[2] << 16);
    M.idx0[i] = (IdxT)i;
    fsums_add(R, om, cc[0], cc[1], cc[2], cc[3], cc[4], cc[5]);
}

// The output of a cell whose final subsets are recorded in info (all its splitting done): one scan
// over the cell's slots gives leaf ordinals and output slots; copied particles go to the staging
// arrays, merged subsets are replaced (Step 7).  In partition mode the permutation and subset
// ordinals are written instead.  leaf_start (n + 1 entries), mlist and msched (n each) are scratch.
// defer: only the slots, leaf starts and the merged list are formed (and the counts recorded); the
// copies and merges are left to the caller (a cell above NMAX_NARROW hands them to other workgroups).
template <int WPB, typename IdxT, typename Args, int RP = 0>
VPM_DEV void cell_output(const CellMem<IdxT>& M, const Args& A, const Frame& F, int c, int64_t off, int n,
                         BlockScratch<WPB>* bs, IdxT* leaf_start, IdxT* mlist, IdxT* msched, bool defer = false) {
    constexpr int NT = WAVE * WPB;
    const int lane = opaque_lane();
    const int tid = WPB == 1 ? lane : opaque_tid();
    const int wv = threadIdx.x / WAVE;
    CellShared& sh = *M.sh;
    // one scan over the cell's slots gives leaf ordinals and output slots
    const int npair = A.P.merge_mode == VPM_MERGE_PAIR ? 2 : 1;
    // a slot's contribution: (1 if it heads a subset) << 32 | (its outputs)
    auto slot_val = [&](uint8_t inf) -> int64_t {
        const int e = (inf & INF_MERGED) ? ((inf & INF_HEAD) ? npair : 0) : 1;
        return ((int64_t)((inf & INF_HEAD) ? 1 : 0) << 32) | (int64_t)e;
    };
    // what a slot records once its prefix `pre` (over the slots before it) is known
    auto record_slot = [&](int p, uint8_t inf, int64_t pre) {
        const int ord = (int)(pre >> 32) + ((inf & INF_HEAD) ? 1 : 0) - 1;
        if (A.mode == 0) {
            M.emit[p] = (IdxT)(pre & 0xffffffff);
        } else {
            A.perm[off + p] = (int32_t)(off + idx_buf(M, inf & INF_PARITY)[p]);
            A.subset_id[off + p] = ord;
        }
        if (inf & INF_HEAD) {
            leaf_start[ord] = (IdxT)p;
            if ((inf & INF_MERGED) && A.mode == 0) mlist[atomicAdd(&sh.nmerged, 1)] = (IdxT)ord;
        }
    };
    int nleaves, out_total;
    bool seg_scan = false;
    if constexpr (WPB > 1 && RP == 0) seg_scan = n > NMAX_NARROW;   // global-memory cells only
    if (seg_scan) {
        // A cell above NMAX_NARROW: each wavefront scans one contiguous segment in rounds of 64
        // consecutive slots (coalesced, RB rounds' loads in flight together), after a first pass
        // that totals the segments.
        constexpr int RB = 8;
        const int seg = (n + WPB - 1) / WPB;
        const int s0 = min(n, wv * seg), s1 = min(n, s0 + seg);
        int64_t acc = 0;
        for (int j0 = s0; j0 < s1; j0 += RB * WAVE) {
            uint8_t b[RB];
#pragma unroll
            for (int u = 0; u < RB; ++u) b[u] = M.info[min(j0 + u * WAVE + lane, s1 - 1)];
#pragma unroll
            for (int u = 0; u < RB; ++u) acc += j0 + u * WAVE + lane < s1 ? slot_val(b[u]) : 0;
        }
        const int64_t wtot = __shfl(wave_incl_scan(acc, lane), WAVE - 1);
        if (lane == 0) bs->scan[wv] = wtot;
        __syncthreads();
        int64_t run = 0, tot = 0;
        for (int w = 0; w < WPB; ++w) {
            if (w < wv) run += bs->scan[w];
            tot += bs->scan[w];
        }
        nleaves = (int)(tot >> 32);
        out_total = (int)(tot & 0xffffffff);
        if (tid == 0) sh.nmerged = 0;
        __syncthreads();
        for (int j0 = s0; j0 < s1; j0 += RB * WAVE) {
            uint8_t b[RB];
#pragma unroll
            for (int u = 0; u < RB; ++u) b[u] = M.info[min(j0 + u * WAVE + lane, s1 - 1)];
#pragma unroll
            for (int u = 0; u < RB; ++u) {
                const int p = j0 + u * WAVE + lane;
                const int64_t v = p < s1 ? slot_val(b[u]) : 0;
                const int64_t inc = wave_incl_scan(v, lane);
                if (p < s1) record_slot(p, b[u], run + inc - v);
                run += __shfl(inc, WAVE - 1);
            }
        }
    } else {
        const int per = (n + NT - 1) / NT;
        const int b0 = min(n, tid * per), b1 = min(n, b0 + per);
        int64_t loc = 0;
        for (int p = b0; p < b1; ++p) loc += slot_val(M.info[p]);
        const int64_t inc = wave_incl_scan(loc, lane);
        int64_t tot, wbase = 0;
        if constexpr (WPB > 1) {
            if (lane == WAVE - 1) bs->scan[wv] = inc;
            __syncthreads();
            tot = 0;
            for (int w = 0; w < WPB; ++w) {
                if (w < wv) wbase += bs->scan[w];
                tot += bs->scan[w];
            }
        } else {
            tot = __shfl(inc, WAVE - 1);
        }
        int64_t pre = wbase + inc - loc;
        nleaves = (int)(tot >> 32);
        out_total = (int)(tot & 0xffffffff);
        if (tid == 0) sh.nmerged = 0;
        cell_sync<WPB>();
        for (int p = b0; p < b1; ++p) {
            const uint8_t inf = M.info[p];
            record_slot(p, inf, pre);
            pre += slot_val(inf);
        }
    }
    if (tid == 0) leaf_start[nleaves] = (IdxT)n;
    cell_sync<WPB>();
    const uint32_t fl = sh.flags;
    if (A.mode == 1) {
        if (tid == 0) {
            A.n_subsets[c] = nleaves;
            if (fl) atomicOr(A.flags, fl);
        }
        return;
    }
    if (defer) {
        if (tid == 0) {
            A.out_count[c] = out_total;
            A.cell_mode[c] = CELL_PROCESSED;
            if (fl) atomicOr(A.flags, fl);
        }
        return;
    }
    // copied particles (subsets below min_subset): the cell's arrays from wave-uniform base
    // pointers with 32-bit lane offsets (no 64-bit address arithmetic per access)
    const typename Args::In* const ib[7] = {A.in.x + off, A.in.y + off, A.in.z + off, A.in.px + off,
                                            A.in.py + off, A.in.pz + off, A.in.w + off};
    float* const ob[7] = {A.tmp.x + off, A.tmp.y + off, A.tmp.z + off, A.tmp.px + off,
                          A.tmp.py + off, A.tmp.pz + off, A.tmp.w + off};
    if constexpr (RP > 0) {
        // An LDS cell (at most RP positions per thread): every input particle is read once, in
        // input order (coalesced, the whole cell's loads in flight together), and stored to its
        // output slot.  inv maps an input position to that slot (0xffff: merged); the codes' pyz
        // array is free by now.
        static_assert(sizeof(IdxT) == 2, "slots of an LDS cell are 16-bit");
        uint16_t* inv = (uint16_t*)M.pyz;
        for (int p = tid; p < n; p += NT) {
            const uint8_t inf = M.info[p];
            inv[idx_buf(M, inf & INF_PARITY)[p]] = (inf & INF_MERGED) ? (uint16_t)0xffff : (uint16_t)M.emit[p];
        }
        cell_sync<WPB>();
        float v[RP][7];
#pragma unroll
        for (int u = 0; u < RP; ++u) {
            const uint32_t i = (uint32_t)min(tid + u * NT, n - 1);
#pragma unroll
            for (int f = 0; f < 7; ++f) v[u][f] = (float)ib[f][i];
        }
#pragma unroll
        for (int u = 0; u < RP; ++u) {
            const int i = tid + u * NT;
            const uint32_t so = i < n ? inv[i] : 0xffffu;
            if (so == 0xffffu) continue;
#pragma unroll
            for (int f = 0; f < 7; ++f) ob[f][so] = v[u][f];
        }
    } else {
        for (int p0 = tid; p0 < n; p0 += COPY_BATCH * NT) {
            uint32_t si[COPY_BATCH], so[COPY_BATCH];
            bool keep[COPY_BATCH];
#pragma unroll
            for (int u = 0; u < COPY_BATCH; ++u) {
                const int p = min(p0 + u * NT, n - 1);
                const uint8_t inf = M.info[p];
                si[u] = idx_buf(M, inf & INF_PARITY)[p];
                so[u] = M.emit[p];
                keep[u] = p0 + u * NT < n && !(inf & INF_MERGED);
            }
            float v[COPY_BATCH][7];
#pragma unroll
            for (int u = 0; u < COPY_BATCH; ++u)
#pragma unroll
                for (int f = 0; f < 7; ++f) v[u][f] = (float)ib[f][si[u]];
#pragma unroll
            for (int u = 0; u < COPY_BATCH; ++u) {
                if (!keep[u]) continue;
#pragma unroll
                for (int f = 0; f < 7; ++f) ob[f][so[u]] = v[u][f];
            }
        }
    }
    // merged subsets (Step 7)
    const int nm = sh.nmerged;
    if (nm > 0) {
        IdxT* sched = msched;
        const Sched s = schedule<WPB, IdxT>(M, sched, nm, A.P.ppl_shift, [&](int it) {
            const int ord = mlist[it];
            return (int)(leaf_start[ord + 1] - leaf_start[ord]);
        });
        for (int r0 = wv * WAVE; r0 < s.total; r0 += NT) {
            int slot, cls;
            if (sched_lookup(s, r0 + lane, slot, cls)) {
                const int ord = mlist[sched[slot]];
                const int st = leaf_start[ord];
                const int ln = leaf_start[ord + 1] - st;
                const int g = 1 << cls;
                const uint8_t inf = M.info[st];
                const IdxT* src = idx_buf(M, inf & INF_PARITY);
                merge_subset(A, F, [&](int j) { return off + (int64_t)src[st + j]; }, ln,
                             (inf >> INF_JSHIFT) & 3, off + M.emit[st], lane & (g - 1), g);
            }
        }
    }
    if (tid == 0) {
        A.out_count[c] = out_total;
        A.cell_mode[c] = CELL_PROCESSED;
        if (fl) atomicOr(A.flags, fl);
    }
}

// ------------------------------------------------------------------------------------------
// The cell kernel: one cell per workgroup of WPB wavefronts (one wavefront for the small bin).
// The subsets of a level are spread over the lane groups of all wavefronts; workgroup barriers
// separate the phases.
// ------------------------------------------------------------------------------------------

template <int NMAX, typename IdxT, bool IN_LDS, int WPB, typename InT>
__global__ __launch_bounds__(WAVE * WPB, 2) void k_fixed_cells(FixedArgsT<InT> A) {
    extern __shared__ __align__(16) uint8_t smem[];
    const int tid = threadIdx.x;
    const int lane = lane_id();
    const int wv = tid / WAVE;
    constexpr int NT = WAVE * WPB;
    constexpr size_t HDR = header_bytes<WPB>();
    constexpr int RP = (NMAX + NT - 1) / NT;       // positions per thread of a whole cell
    static_assert(IN_LDS, "cells above the LDS bins go to k_fixed_big");
    CellMem<IdxT> M = carve<IdxT>(smem + HDR, NMAX);
    M.sh = (CellShared*)smem;
    BlockScratch<WPB>* bs = (BlockScratch<WPB>*)(smem + ((sizeof(CellShared) + 15) & ~(size_t)15));
    CellShared& sh = *M.sh;

    // One cell per claim on the shared work counter: batching claims measured no faster for the
    // cell sizes here, and single claims keep the tail of the launch short.
    const int qlen = A.counters[A.qlen_index];
    if (qlen == 0) return;                         // an empty bin claims nothing
    if (tid == 0) sh.dc = decide_consts(A.P);      // visible after the loop's first barrier
    if constexpr (WPB == 1) wave_fence();
    for (;;) {
        int qi = 0;
        if constexpr (WPB == 1) {
            if (lane == 0) qi = atomicAdd(&A.counters[A.work_index], 1);
            qi = __builtin_amdgcn_readfirstlane(__shfl(qi, 0));   // wave-uniform: scalar loads
        } else {
            __syncthreads();                               // the previous cell is finished
            if (tid == 0) {
                sh.qi = atomicAdd(&A.counters[A.work_index], 1);
                sh.flags = 0;
                sh.nnext = 0;
            }
            __syncthreads();
            qi = __builtin_amdgcn_readfirstlane(sh.qi);
        }
        if (qi >= qlen) break;
        const int c = A.queue[qi];
        const int64_t off = A.cell_off[c];
        const int n = (int)(A.cell_off[c + 1] - off);
        // the lane and thread indices as values formed anew for each cell (see opaque_lane)
        const int lane = opaque_lane();
        const int tid = WPB == 1 ? lane : opaque_tid();

        // ---- Step 1: collect the cell (into registers: RP positions per thread), validate, frame ----
        Frame F;
        float q[RP][7];
        load_cell_regs<RP, NT>(A.in, off, n, tid, q);
        const bool valid = cell_frame_regs<WPB, RP>(q, n, tid, cell_mass(A.P.mass, A.P.species, A.P.species_mass, c), F, bs);
        if (!valid) {
            if (tid == 0) {
                atomicOr(A.flags, FLAG_BAD_VALUE);
                if (A.mode == 0) { A.out_count[c] = n; A.cell_mode[c] = CELL_UNTOUCHED; }
                else A.n_subsets[c] = 0;
            }
            if (A.mode == 1)
                for (int i = tid; i < n; i += NT) { A.perm[off + i] = (int32_t)(off + i); A.subset_id[off + i] = -1; }
            continue;
        }
        if constexpr (WPB == 1) {
            if (lane == 0) { sh.flags = 0; sh.nnext = 0; }
        }

        // ---- codes and the root's moments ----
        FSums R;
        fsums_zero(R);
        bool oob = false;
#pragma unroll
        for (int u = 0; u < RP; ++u)
            if (tid + u * NT < n) encode_particle(M, A.P, F, tid + u * NT, q[u], R, oob);
        const bool any_oob = ballot(oob) != 0;
        fsums_group_reduce(R, WAVE);
        if constexpr (WPB > 1) {
            if (lane == 0) {
                bs->sums[wv][0] = R.s0;
                for (int l = 0; l < 6; ++l) { bs->sums[wv][1 + l] = R.s1[l]; bs->sums[wv][7 + l] = R.s2[l]; }
                if (any_oob) atomicOr(&sh.flags, FLAG_OUT_OF_CELL);
            }
            __syncthreads();
            if (tid == 0) {
                fsums_zero(R);
                for (int w = 0; w < WPB; ++w) {
                    R.s0 += bs->sums[w][0];
                    for (int l = 0; l < 6; ++l) { R.s1[l] += bs->sums[w][1 + l]; R.s2[l] += bs->sums[w][7 + l]; }
                }
                const Decision d = decide(M, R, M.idx0, 0, n, A.P, F);
                sh.rootv = pack_decision(d);
                // the root as the first wavefront's subset for the inherited levels
                Handoff& h = bs->ho[0];
                h.start = 0; h.len = n; h.thr_axis = (d.thr << 8) | d.axis; h.act = 1;
                h.P[0] = R.s0;
                for (int l = 0; l < 6; ++l) {
                    h.P[1 + l] = R.s1[l];
                    h.P[7 + l] = R.s2[l];
                    h.E2[l] = R.s2[l] * ((double)(n + 16) * 0x1p-51);
                }
                for (int w = 1; w < WPB; ++w) bs->ho[w].act = 0;
            }
            __syncthreads();
        } else {
            if (any_oob && lane == 0) sh.flags |= FLAG_OUT_OF_CELL;
            wave_fence();
            if (lane == 0) sh.rootv = pack_decision(decide(M, R, M.idx0, 0, n, A.P, F));
            wave_fence();
        }
        const Decision rd = unpack_decision(sh.rootv);
        int m = 0;
        int cur = 0;
        if (rd.kind == D_SPLIT) {
            if constexpr (WPB == 1) inherit_levels<IdxT>(M, A, F, R, n, rd, lane, cur, m);
            else inherit_block<WPB, IdxT>(M, A, F, bs, cur, m);
        } else {
            const uint8_t base = INF_SET | (rd.kind == D_MERGED ? INF_MERGED : 0) | (uint8_t)(rd.jdir << INF_JSHIFT);
            for (int i = tid; i < n; i += NT) M.info[i] = base | (i == 0 ? INF_HEAD : 0);
        }
        cell_sync<WPB>();

        // ---- Steps 2-6, level by level ----
        while (m > 0) {
            Node<IdxT>* curl = cur ? M.nodes1 : M.nodes0;
            Node<IdxT>* nextl = cur ? M.nodes0 : M.nodes1;
            if (tid == 0) sh.nnext = 0;
            const Sched s = schedule<WPB, IdxT>(M, M.sched, m, A.P.ppl_shift, [&](int it) { return (int)curl[it].len; });
            const bool solo = __builtin_amdgcn_readfirstlane(s.total == s.cnt[0] ? 1 : 0) != 0;   // only 1-lane groups
            for (int r0 = wv * WAVE; r0 < s.total; r0 += NT) {
                int slot, cls;
                const int ln = opaque_lane();
                if (sched_lookup(s, r0 + ln, slot, cls)) {
                    const Node<IdxT> nd = curl[M.sched[slot]];
                    const int g = 1 << cls;
                    split_node<IdxT>(M, A, F, nullptr, nd, cur, ln & (g - 1), g, ln & ~(g - 1), nextl, solo);
                }
            }
            cell_sync<WPB>();
            m = sh.nnext;
            cur ^= 1;
            if constexpr (WPB > 1) __syncthreads();        // nnext is read before it is reset
        }

        // ---- output ----
        cell_output<WPB, IdxT, FixedArgsT<InT>, RP>(M, A, F, c, off, n, bs, (IdxT*)M.nodes0, (IdxT*)M.nodes1,
                                                    (IdxT*)M.rec);
        if constexpr (WPB == 1) wave_fence();
    }
}

// ------------------------------------------------------------------------------------------
// Cells above the LDS bins, several workgroups per cell.  A large cell's codes, index buffers, info
// bytes and output slots live in cell-wide global arrays indexed by input position.  The workgroup
// that claims the cell builds its frame and codes and splits it level by level as the other bins
// do.  Once no cell is left to claim, so that workgroups fall idle, every unfinished subset of at
// least TASK_MIN particles that a split leaves goes to a device task queue (a ring), from which any
// workgroup takes it and splits it in turn, spawning further tasks.  (Before that every workgroup
// has a cell of its own, and keeping a cell on one workgroup avoids the device-wide cache
// maintenance that handing data between workgroups costs.)  Each piece of a cell (its root, or a
// task) ends by decrementing the cell's count of open pieces; the workgroup that closes the last
// one runs the cell's output.  The grid drains when no cell is left to claim and no piece is queued
// or running (a device count, `pending`).
//   Queued tasks are pairwise disjoint subsets of >= TASK_MIN particles (a task's descendants are
// spawned only after it is claimed), so at most n_particles / TASK_MIN are queued at a time and the
// ring never overwrites an unclaimed task.  Node lists and the schedule table are per workgroup,
// in a global slab sized for a whole cell's frontier.
// ------------------------------------------------------------------------------------------

constexpr int BIG_NODES = NMAX_BIG / 2 + 2;
constexpr int C_TASK_HEAD = 28, C_TASK_RESERVE = 29, C_PENDING = 30;   // counters, reset per call

// A task: a subset to split (TASK_NODE), or part of the output of a cell above NMAX_NARROW once its
// partition is complete: the copies of slots nd.start .. nd.start + nd.len - 1 (TASK_COPY), or the
// merged subsets nd.start, nd.start + nd.len, nd.start + 2 nd.len, ... of its list (TASK_MERGE).
// TASK_WCOUNT and TASK_WPLACE are the two passes of one chunk of a subset above NMAX_NARROW split by
// several workgroups (nd.start: the job, nd.len: the chunk).
// TASK_CFRAME and TASK_CENCODE are the root passes of a cell above NMAX_NARROW (its frame, then its
// codes and exact root moments), one chunk each (nd.start: the job, nd.len: the chunk).
enum { TASK_NODE = 0, TASK_COPY = 1, TASK_MERGE = 2, TASK_WCOUNT = 3, TASK_WPLACE = 4, TASK_CFRAME = 5,
       TASK_CENCODE = 6 };
VPM_DEV bool task_is_piece(int kind) { return kind != TASK_COPY && kind != TASK_MERGE; }
struct BigTask { int32_t qi, cur; Node<uint32_t> nd; int32_t kind; };
// A subset above NMAX_NARROW split by several workgroups: its slots fall into `nchunks` chunks of at
// least NMAX_NARROW (records chunk0 ..); `left` counts the chunks still to finish the current pass.
struct WideJob { Node<uint32_t> nd; int32_t cur, qi, nchunks, chunk0, left, n1, d0, d1; };
// One chunk: the lower side's count per wavefront segment, the chunk's first V1 position, and (after
// the counting pass) the exact moments of the subset's and V1's members in the chunk.
struct WideChunk { int32_t cnt[8]; int32_t lb, pad; uint64_t P[19], L[19]; };
constexpr int C_JOBS = 16, C_CHUNKS = 17;     // allocation counters of jobs and chunks, reset per call
struct BigCell { Frame F; int64_t off; int32_t n, c, open, nmerged, bad, pad; };   // bad: passed through

template <typename InT>
struct BigArgs {
    FixedArgsT<InT> A;
    int4* rec;                     // cell-wide arrays of the large cells, indexed by input position
    int32_t* pyz;
    uint32_t *idx0, *idx1, *emit;
    uint8_t* info;
    BigCell* cells;                // per claimed cell (claim index): frame, offset, size, open pieces
    BigTask* tasks;                // ring of ring_size slots
    int32_t* ready;                // per slot: 1 once the task is written, 0 once it is taken
    int32_t ring_size;
    Node<uint32_t>* lists;         // per workgroup: two node lists of BIG_NODES
    uint32_t* sched;               // per workgroup: a schedule table of BIG_NODES
    WideJob* jobs;                 // subsets above NMAX_NARROW split by several workgroups (capacities:
    WideChunk* chunks;             // 0 splits every such subset with one workgroup)
    int32_t jobs_cap, chunks_cap;
    int32_t wait_idle;             // idle workgroups wait for tasks (else they leave the chip to
                                   // kernels running beside this one)
};

struct BigShared {                 // LDS after the header
    SpawnList<uint32_t> spawn;
    int spawn_ok;                  // the level may hand subsets to other workgroups
};

__host__ __device__ constexpr size_t big_lds_bytes() { return header_bytes<8>() + rnd16(sizeof(BigShared)); }

// Polling loads are relaxed: an acquire at device scope invalidates the caches of the whole XCD
// (other workgroups' working sets included), so it is made once, by one thread, after a claim.
VPM_DEV int ld_relaxed(const int32_t* p) { return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); }

// Queue subset nd of cell qi (its members in index buffer cur) as a task.  The caller has made the
// writes it depends on visible at device scope.
template <typename InT>
VPM_DEV void spawn_task(const BigArgs<InT>& B, int qi, int cur, Node<uint32_t> nd, int kind = TASK_NODE) {
    int32_t* const ctr = B.A.counters;
    if (task_is_piece(kind)) atomicAdd(&B.cells[qi].open, 1);    // output tasks are not pieces of the partition
    atomicAdd(&ctr[C_PENDING], 1);
    const int idx = atomicAdd(&ctr[C_TASK_RESERVE], 1);
    const int slot = idx % B.ring_size;
    BigTask t;
    t.qi = qi; t.cur = cur; t.nd = nd; t.kind = kind;
    B.tasks[slot] = t;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __hip_atomic_store(&B.ready[slot], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Exact wide moments of the whole workgroup: each wavefront's total goes to the workgroup's
// slab (`part`, WPB records of 19 words), then thread 0 adds them up.  All threads call; the result
// is valid in thread 0.
template <int WPB>
VPM_DEV void wsums_block_reduce(WSums& S, uint64_t* part) {
    wsums_wave_reduce(S);
    constexpr int W = 19;
    if (lane_id() == 0) {
        uint64_t* q = part + (size_t)(threadIdx.x / WAVE) * W;
        q[0] = S.s0;
        for (int l = 0; l < 6; ++l) {
            q[1 + l] = (uint64_t)S.s1[l];
            q[7 + 2 * l] = S.s2[l].lo;
            q[8 + 2 * l] = S.s2[l].hi;
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        wsums_zero(S);
        for (int w = 0; w < WPB; ++w) {
            const uint64_t* q = part + (size_t)w * W;
            WSums T;
            T.s0 = q[0];
            for (int l = 0; l < 6; ++l) {
                T.s1[l] = (int64_t)q[1 + l];
                T.s2[l] = u128_make(q[7 + 2 * l], q[8 + 2 * l]);
            }
            wsums_acc(S, T);
        }
    }
    __syncthreads();
}

// Thread 0: the decisions of the two children of a subset of len particles above NMAX_NARROW whose
// lower side V1 holds n1, from the subset's exact moments P and V1's L (V2's are P - L), into dv[0]
// and dv[1] (dv[1] = -1: the cut left a side empty, which the exact rule never does; the subset ends).
template <typename Args>
VPM_DEV void decide_children(const Args& A, const CellMem<uint32_t>& M, const Frame& F, const WSums& P,
                             const WSums& L, int len, int n1, int* dv) {
    const int n2 = len - n1;
    if (n1 == 0 || n2 == 0) {
        atomicOr(&M.sh->flags, FLAG_INTERNAL);
        Decision d; d.kind = D_MERGED; d.axis = 0; d.thr = 0; d.jdir = 0;
        dv[0] = pack_decision(d);
        dv[1] = -1;
        return;
    }
    const DecideConsts& K = M.sh->dc;
    Decision cp; cp.kind = D_COPY; cp.axis = 0; cp.thr = 0; cp.jdir = 0;
    WSums R;
    R.s0 = P.s0 - L.s0;
#pragma unroll
    for (int l = 0; l < 6; ++l) { R.s1[l] = P.s1[l] - L.s1[l]; R.s2[l] = sub128(P.s2[l], L.s2[l]); }
    dv[0] = pack_decision(n1 < A.P.min_subset ? cp : decide_exact_wide(L, K, F));
    dv[1] = pack_decision(n2 < A.P.min_subset ? cp : decide_exact_wide(R, K, F));
}

// The children of a subset above NMAX_NARROW once it is cut (its members placed in the other index
// buffer) and decided (d0, d1): finished children are recorded, unfinished ones of TASK_MIN or more
// become tasks, smaller ones go to `kept` (the node list of the other buffer).  All threads call;
// returns the number kept.
template <typename InT>
VPM_DEV int wide_children(const BigArgs<InT>& B, const CellMem<uint32_t>& M, BlockScratch<8>* bs,
                          Node<uint32_t> nd, int cur, int qi, int n1, int d0, int d1, Node<uint32_t>* kept) {
    constexpr int NT = WAVE * 8;
    const int tid = threadIdx.x;
    const int start = nd.start, len = nd.len, n2 = len - n1;
    const int rev = (nd.thr_axis >> 3) & 1;
    int* const dv = bs->vote[0];
    __syncthreads();                                    // dv may still be read
    if (tid == 0) { dv[2] = 0; dv[3] = 0; }             // children kept, children handed out
    __syncthreads();
    Node<uint32_t>* const hand = (Node<uint32_t>*)(dv + 4);   // bs->vote[0][4] on: two nodes
    for (int ch = 0; ch < 2; ++ch) {
        const int dvv = ch == 0 ? d0 : d1;
        if (dvv == -1) continue;
        const Decision d = unpack_decision(dvv);
        const int cs = d1 == -1 ? start : (ch == 0 ? start : start + n1);
        const int cl = d1 == -1 ? len : (ch == 0 ? n1 : n2);
        const int crev = d1 == -1 ? (n1 == 0 ? rev ^ 1 : rev) : (ch == 0 ? rev : rev ^ 1);
        if (d.kind == D_SPLIT) {
            if (tid == 0) {
                Node<uint32_t> c;
                c.start = (uint32_t)cs; c.len = (uint32_t)cl;
                c.thr_axis = (d.thr << 8) | (crev << 3) | d.axis;
                if (cl >= TASK_MIN) hand[dv[3]++] = c;
                else kept[dv[2]++] = c;
            }
        } else {
            record_final(M, B.A, d, cs, cl, crev, cur, tid, NT);
        }
    }
    // the cut and the info bytes, device-wide, before another workgroup may take a child
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __syncthreads();
    const int nk = dv[2], nh = dv[3];
    if (tid == 0)
        for (int h = 0; h < nh; ++h) spawn_task(B, qi, cur ^ 1, hand[h]);
    __syncthreads();                                    // dv is read before it is reused
    return nk;
}

// Steps 5-6 for one subset of more than NMAX_NARROW particles, by the whole workgroup: the stable
// cut into the other index buffer (V1 = {c <= thr} from the front in slot order, V2 from the back
// in reverse slot order, as compact_node lays them out), the exact moments of both children while
// they are placed, and their exact decisions (Steps 3-4).  Unfinished children of at least TASK_MIN
// particles become tasks; smaller ones go to `kept` (the node list of the other buffer).  Returns
// the number kept.
// The root decision of a cell above NMAX_NARROW (into sh.rootv): its moments summed exactly over
// the whole workgroup, then the exact rule.
VPM_DEV void wide_root(const CellMem<uint32_t>& M, const Frame& F, int n, int min_subset) {
    WSums W0;
    wsums_zero(W0);
    constexpr int WB = 4;                           // rounds whose codes are loaded together
    for (int i0 = 0; i0 < n; i0 += WB * (int)blockDim.x) {
        int cc[WB][6], om[WB];
#pragma unroll
        for (int u = 0; u < WB; ++u) codes_of(M, min(i0 + u * (int)blockDim.x + (int)threadIdx.x, n - 1), cc[u], om[u]);
#pragma unroll
        for (int u = 0; u < WB; ++u)
            if (i0 + u * (int)blockDim.x + (int)threadIdx.x < n) wsums_add(W0, om[u], cc[u]);
    }
    wsums_block_reduce<8>(W0, (uint64_t*)M.sched);
    if (threadIdx.x == 0) {
        Decision cp; cp.kind = D_COPY; cp.axis = 0; cp.thr = 0; cp.jdir = 0;
        M.sh->rootv = pack_decision(n < min_subset ? cp : decide_exact_wide(W0, M.sh->dc, F));
    }
}

template <typename InT>
VPM_DEV int wide_split(const BigArgs<InT>& B, const CellMem<uint32_t>& M, const Frame& F, BlockScratch<8>* bs,
                       Node<uint32_t> nd, int cur, int qi, Node<uint32_t>* kept) {
    constexpr int WPB = 8, NT = WAVE * WPB;
    const auto& A = B.A;
    const int tid = threadIdx.x, lane = lane_id(), wv = tid / WAVE;
    const int start = nd.start, len = nd.len;
    const int k = nd.thr_axis & 7, thr = nd.thr_axis >> 8, rev = (nd.thr_axis >> 3) & 1;
    const uint32_t* src = idx_buf(M, cur) + start;
    uint32_t* dst = idx_buf(M, cur ^ 1);
    // each wavefront takes one contiguous segment of the subset's slots
    const int seg = (len + WPB - 1) / WPB;
    const int s0 = min(len, wv * seg), s1 = min(len, s0 + seg);
    // Both passes take WB rounds of 64 slots at a time: their indices, then their codes, are loaded
    // before any is used, so that a wavefront keeps several gathers in flight.
    constexpr int WB = 4;
    // pass 1: the lower side's count per wavefront and the subset's moments
    WSums P;
    wsums_zero(P);
    int cnt = 0;
    for (int j0 = s0; j0 < s1; j0 += WB * WAVE) {
        uint32_t ix[WB];
#pragma unroll
        for (int u = 0; u < WB; ++u) ix[u] = src[min(j0 + u * WAVE + lane, s1 - 1)];
        int c[WB][6], om[WB];
#pragma unroll
        for (int u = 0; u < WB; ++u) codes_of(M, (int)ix[u], c[u], om[u]);
#pragma unroll
        for (int u = 0; u < WB; ++u) {
            if (j0 + u * WAVE + lane >= s1) continue;
            int ck = c[u][0];
#pragma unroll
            for (int l = 1; l < 6; ++l) if (l == k) ck = c[u][l];
            cnt += ck <= thr ? 1 : 0;
            wsums_add(P, om[u], c[u]);
        }
    }
    cnt = group_sum(cnt, WAVE);
    if (lane == 0) bs->scan[wv] = cnt;
    __syncthreads();
    int lb = 0, n1 = 0;
    for (int w = 0; w < WPB; ++w) {
        if (w < wv) lb += (int)bs->scan[w];
        n1 += (int)bs->scan[w];
    }
    int rb = s0 - lb;                                   // V2 members before this segment
    wsums_block_reduce<WPB>(P, (uint64_t*)M.sched);
    // pass 2: the cut, with V1's moments (V2's are the subset's minus V1's, exactly)
    WSums L;
    wsums_zero(L);
    const uint64_t below = lanes_below();
    for (int j0 = s0; j0 < s1; j0 += WB * WAVE) {
        uint32_t ix[WB];
#pragma unroll
        for (int u = 0; u < WB; ++u) ix[u] = src[min(j0 + u * WAVE + lane, s1 - 1)];
        int c[WB][6], om[WB];
#pragma unroll
        for (int u = 0; u < WB; ++u) codes_of(M, (int)ix[u], c[u], om[u]);
#pragma unroll
        for (int u = 0; u < WB; ++u) {
            const bool act = j0 + u * WAVE + lane < s1;
            int ck = c[u][0];
#pragma unroll
            for (int l = 1; l < 6; ++l) if (l == k) ck = c[u][l];
            const bool right = ck > thr;
            const uint64_t br = ballot(act && right), bl = ballot(act && !right);
            if (act) {
                if (right) dst[start + len - 1 - (rb + __popcll(br & below))] = ix[u];
                else {
                    dst[start + lb + __popcll(bl & below)] = ix[u];
                    wsums_add(L, om[u], c[u]);
                }
            }
            lb += __popcll(bl);
            rb += __popcll(br);
        }
    }
    wsums_block_reduce<WPB>(L, (uint64_t*)M.sched);
    int* const dv = bs->vote[0];
    if (tid == 0) decide_children(A, M, F, P, L, len, n1, dv);
    __syncthreads();
    return wide_children(B, M, bs, nd, cur, qi, n1, dv[0], dv[1], kept);
}

VPM_DEV void wsums_store(uint64_t* q, const WSums& S) {
    q[0] = S.s0;
    for (int l = 0; l < 6; ++l) {
        q[1 + l] = (uint64_t)S.s1[l];
        q[7 + 2 * l] = S.s2[l].lo;
        q[8 + 2 * l] = S.s2[l].hi;
    }
}

VPM_DEV WSums wsums_load(const uint64_t* q) {
    WSums S;
    S.s0 = q[0];
    for (int l = 0; l < 6; ++l) {
        S.s1[l] = (int64_t)q[1 + l];
        S.s2[l] = u128_make(q[7 + 2 * l], q[8 + 2 * l]);
    }
    return S;
}

// ------------------------------------------------------------------------------------------
// A subset above NMAX_NARROW split by several workgroups.  Its slots fall into K = len / NMAX_NARROW
// chunks; each chunk is a task in two passes.  Counting: the chunk's lower side per wavefront segment
// and the exact moments of its members and of its V1 members.  The workgroup that finishes the last
// count adds the chunks up in chunk order (integer sums: the result does not depend on which
// workgroup does what), decides both children by the exact rule and gives every chunk its first V1
// position.  Placing: each chunk puts its members at their positions in the other index buffer, V1
// from the front in slot order and V2 from the back in reverse order, as one workgroup would.  The
// workgroup that finishes the last placement records the children.
// ------------------------------------------------------------------------------------------

// Hand subset nd of cell qi (members in index buffer cur) to the chunk tasks of a new job.  All
// threads call, after the subset's members are visible device-wide; false when the job and chunk
// records are used up (the caller then splits the subset itself).
template <typename InT>
VPM_DEV bool start_wide_job(const BigArgs<InT>& B, BlockScratch<8>* bs, Node<uint32_t> nd, int cur, int qi,
                            int first_kind = TASK_WCOUNT) {
    int* const flag = &bs->vote[1][7];
    if (threadIdx.x == 0) {
        int ok = 0;
        const int K = (int)(nd.len / (uint32_t)NMAX_NARROW);          // >= 1
        if (B.jobs_cap > 0) {
            const int j = atomicAdd(&B.A.counters[C_JOBS], 1);
            const int c0 = atomicAdd(&B.A.counters[C_CHUNKS], K);
            if (j < B.jobs_cap && c0 <= B.chunks_cap - K) {
                WideJob& J = B.jobs[j];
                J.nd = nd; J.cur = cur; J.qi = qi; J.nchunks = K; J.chunk0 = c0; J.left = K;
                Node<uint32_t> r;
                r.start = (uint32_t)j; r.thr_axis = 0;
                for (int k = 0; k < K; ++k) { r.len = (uint32_t)k; spawn_task(B, qi, cur, r, first_kind); }
                ok = 1;
            }
        }
        *flag = ok;
    }
    __syncthreads();
    const bool ok = *flag != 0;
    __syncthreads();
    return ok;
}

// The slots of chunk k of a job, relative to its subset: [a, b), and wavefront wv's segment of it.
VPM_DEV void chunk_range(int len, int K, int k, int wv, int& s0, int& s1) {
    const int span = (len + K - 1) / K;
    const int a = min(len, k * span), b = min(len, a + span);
    const int seg = (b - a + 7) / 8;
    s0 = min(b, a + wv * seg);
    s1 = min(b, s0 + seg);
}

// The counting pass of chunk k of job j (all threads).
template <typename InT>
VPM_DEV void wide_count_task(const BigArgs<InT>& B, const CellMem<uint32_t>& M, const Frame& F,
                             BlockScratch<8>* bs, int j, int k) {
    constexpr int WPB = 8;
    const int tid = threadIdx.x, lane = lane_id(), wv = tid / WAVE;
    WideJob& J = B.jobs[j];
    const Node<uint32_t> nd = J.nd;
    const int cur = J.cur, K = J.nchunks, len = nd.len;
    const int ax = nd.thr_axis & 7, thr = nd.thr_axis >> 8;
    WideChunk& ck = B.chunks[J.chunk0 + k];
    const uint32_t* src = idx_buf(M, cur) + nd.start;
    int s0, s1;
    chunk_range(len, K, k, wv, s0, s1);
    constexpr int WB = 4;
    // two passes over the chunk (the subset's members, then V1's), so that one set of wide sums is
    // live at a time
    int cnt = 0;
    for (int pass = 0; pass < 2; ++pass) {
        WSums S;
        wsums_zero(S);
        for (int j0 = s0; j0 < s1; j0 += WB * WAVE) {
            uint32_t ix[WB];
#pragma unroll
            for (int u = 0; u < WB; ++u) ix[u] = src[min(j0 + u * WAVE + lane, s1 - 1)];
            int c[WB][6], om[WB];
#pragma unroll
            for (int u = 0; u < WB; ++u) codes_of(M, (int)ix[u], c[u], om[u]);
#pragma unroll
            for (int u = 0; u < WB; ++u) {
                if (j0 + u * WAVE + lane >= s1) continue;
                int cv = c[u][0];
#pragma unroll
                for (int l = 1; l < 6; ++l) if (l == ax) cv = c[u][l];
                if (pass == 0 || cv <= thr) wsums_add(S, om[u], c[u]);
                if (pass == 1 && cv <= thr) ++cnt;
            }
        }
        wsums_block_reduce<WPB>(S, (uint64_t*)M.sched);
        if (tid == 0) wsums_store(pass == 0 ? ck.P : ck.L, S);
    }
    cnt = group_sum(cnt, WAVE);
    if (lane == 0) ck.cnt[wv] = cnt;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __syncthreads();
    if (tid == 0 && atomicSub(&J.left, 1) == 1) {
        // the last count: the chunks in order, the children's decisions, each chunk's first V1 slot
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        WSums Pt, Lt;
        wsums_zero(Pt); wsums_zero(Lt);
        int n1 = 0;
        for (int q = 0; q < K; ++q) {
            WideChunk& cq = B.chunks[J.chunk0 + q];
            cq.lb = n1;
            for (int w = 0; w < 8; ++w) n1 += cq.cnt[w];
            wsums_acc(Pt, wsums_load(cq.P));
            wsums_acc(Lt, wsums_load(cq.L));
        }
        int dv[2];
        decide_children(B.A, M, F, Pt, Lt, len, n1, dv);
        J.n1 = n1; J.d0 = dv[0]; J.d1 = dv[1];
        J.left = K;
        Node<uint32_t> r;
        r.start = (uint32_t)j; r.thr_axis = 0;
        for (int q = 0; q < K; ++q) { r.len = (uint32_t)q; spawn_task(B, J.qi, cur, r, TASK_WPLACE); }
    }
}

// The placing pass of chunk k of job j (all threads).  The workgroup that places the last chunk
// records the children; it returns the number of children it keeps in `kept` (else 0).
template <typename InT>
VPM_DEV int wide_place_task(const BigArgs<InT>& B, const CellMem<uint32_t>& M, BlockScratch<8>* bs, int j, int k,
                            Node<uint32_t>* kept) {
    const int tid = threadIdx.x, lane = lane_id(), wv = tid / WAVE;
    WideJob& J = B.jobs[j];
    const Node<uint32_t> nd = J.nd;
    const int cur = J.cur, K = J.nchunks, len = nd.len, start = nd.start;
    const int ax = nd.thr_axis & 7, thr = nd.thr_axis >> 8;
    const WideChunk& ck = B.chunks[J.chunk0 + k];
    const uint32_t* src = idx_buf(M, cur) + start;
    uint32_t* dst = idx_buf(M, cur ^ 1);
    int s0, s1;
    chunk_range(len, K, k, wv, s0, s1);
    int lb = ck.lb;
    for (int w = 0; w < wv; ++w) lb += ck.cnt[w];
    int rb = s0 - lb;                                   // V2 members before this segment
    const uint64_t below = lanes_below();
    constexpr int WB = 4;
    for (int j0 = s0; j0 < s1; j0 += WB * WAVE) {
        uint32_t ix[WB];
#pragma unroll
        for (int u = 0; u < WB; ++u) ix[u] = src[min(j0 + u * WAVE + lane, s1 - 1)];
        int cv[WB];
#pragma unroll
        for (int u = 0; u < WB; ++u) {
            int c[6], om;
            codes_of(M, (int)ix[u], c, om);
            cv[u] = c[0];
#pragma unroll
            for (int l = 1; l < 6; ++l) if (l == ax) cv[u] = c[l];
        }
#pragma unroll
        for (int u = 0; u < WB; ++u) {
            const bool act = j0 + u * WAVE + lane < s1;
            const bool right = cv[u] > thr;
            const uint64_t br = ballot(act && right), bl = ballot(act && !right);
            if (act) {
                if (right) dst[start + len - 1 - (rb + __popcll(br & below))] = ix[u];
                else dst[start + lb + __popcll(bl & below)] = ix[u];
            }
            lb += __popcll(bl);
            rb += __popcll(br);
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __syncthreads();
    int* const flag = &bs->vote[1][7];
    if (tid == 0) {
        const int last = atomicSub(&J.left, 1) == 1 ? 1 : 0;
        if (last) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");   // every chunk's placements
        *flag = last;
    }
    __syncthreads();
    if (!*flag) return 0;
    return wide_children(B, M, bs, nd, cur, J.qi, J.n1, J.d0, J.d1, kept);
}

// The frame pass of chunk k of cell job j (all threads): the chunk's extreme values.  The workgroup
// that finishes the last chunk forms the cell's frame (or, with a bad value, passes the cell through)
// and starts the codes pass.
template <typename InT>
VPM_DEV void cell_frame_task(const BigArgs<InT>& B, BlockScratch<8>* bs, int j, int k) {
    constexpr int NT = WAVE * 8;
    const auto& A = B.A;
    const int tid = threadIdx.x, lane = lane_id(), wv = tid / WAVE;
    WideJob& J = B.jobs[j];
    const int K = J.nchunks, n = J.nd.len, qi = J.qi;
    BigCell& bc = B.cells[qi];
    const int64_t off = bc.off;
    const int c = bc.c;
    const int span = (n + K - 1) / K;
    const int a = min(n, k * span), b = min(n, a + span);
    FrameAcc acc;
    facc_init(acc);
    facc_cell(acc, A.in, off + a, tid, b - a, NT);
    const bool bad = ballot(acc.bad) != 0;
#pragma unroll
    for (int r = 0; r < 11; ++r) acc.v[r] = wave_max(acc.v[r]);
    if (lane == 0) {
        bs->bad[wv] = bad;
        for (int r = 0; r < 11; ++r) bs->fmax[wv][r] = acc.v[r];
    }
    __syncthreads();
    WideChunk& ck = B.chunks[J.chunk0 + k];
    if (tid == 0) {
        float v[11];
        int anybad = 0;
        for (int r = 0; r < 11; ++r) v[r] = bs->fmax[0][r];
        for (int w = 0; w < 8; ++w) {
            anybad |= bs->bad[w];
            for (int r = 0; r < 11; ++r) v[r] = fmaxf(v[r], bs->fmax[w][r]);
        }
        for (int r = 0; r < 11; ++r) ck.P[r] = (uint64_t)__float_as_uint(v[r]);
        ck.P[11] = (uint64_t)anybad;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __syncthreads();
    int* const flag = &bs->vote[1][7];
    if (tid == 0) {
        int out = 0;
        if (atomicSub(&J.left, 1) == 1) {
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            float v[11];
            int anybad = 0;
            for (int r = 0; r < 11; ++r) v[r] = -INFINITY;
            for (int q = 0; q < K; ++q) {
                const WideChunk& cq = B.chunks[J.chunk0 + q];
                for (int r = 0; r < 11; ++r) v[r] = fmaxf(v[r], __uint_as_float((uint32_t)cq.P[r]));
                anybad |= (int)cq.P[11];
            }
            if (anybad) {
                bc.bad = 1;
                atomicOr(A.flags, FLAG_BAD_VALUE);
                if (A.mode == 0) { A.out_count[c] = n; A.cell_mode[c] = CELL_UNTOUCHED; }
                else A.n_subsets[c] = 0;
                out = 2;
            } else {
                Frame F;
                frame_from(v, cell_mass(A.P.mass, A.P.species, A.P.species_mass, c), F);
                bc.F = F;
                J.left = K;
                Node<uint32_t> r;
                r.start = (uint32_t)j; r.thr_axis = 0;
                for (int q = 0; q < K; ++q) { r.len = (uint32_t)q; spawn_task(B, qi, 0, r, TASK_CENCODE); }
                out = 1;
            }
        }
        *flag = out;
    }
    __syncthreads();
    if (*flag == 2 && A.mode == 1)                      // a passed-through cell: the identity partition
        for (int i = tid; i < n; i += NT) { A.perm[off + i] = (int32_t)(off + i); A.subset_id[off + i] = -1; }
}

// The codes pass of chunk k of cell job j (all threads): the chunk's codes and its exact moments.
// The workgroup that finishes the last chunk decides the root (the exact rule) and splits it (a job of
// its own, or by itself when no records are left: then it returns the children it keeps in `kept`,
// members in index buffer 1) or records the whole cell as one finished subset.
template <typename InT>
VPM_DEV int cell_encode_task(const BigArgs<InT>& B, const CellMem<uint32_t>& M, const Frame& F, BlockScratch<8>* bs,
                             int j, int k, Node<uint32_t>* kept) {
    constexpr int NT = WAVE * 8;
    const auto& A = B.A;
    const int tid = threadIdx.x, lane = lane_id();
    WideJob& J = B.jobs[j];
    const int K = J.nchunks, n = J.nd.len, qi = J.qi;
    const int span = (n + K - 1) / K;
    const int a = min(n, k * span), b = min(n, a + span);
    FSums R;                                            // (the FP64 moments are not used here)
    fsums_zero(R);
    bool oob = false;
    load_particles(A.in, B.cells[qi].off, a + tid, b, NT, [&](int i, const float* q, bool ok) {
        if (ok) encode_particle(M, A.P, F, i, q, R, oob);
    });
    if (ballot(oob) != 0 && lane == 0) atomicOr(&M.sh->flags, FLAG_OUT_OF_CELL);
    WSums W;
    wsums_zero(W);
    for (int i = a + tid; i < b; i += NT) {             // the codes this thread has just written
        int cc[6], om;
        codes_of(M, i, cc, om);
        wsums_add(W, om, cc);
    }
    wsums_block_reduce<8>(W, (uint64_t*)M.sched);
    WideChunk& ck = B.chunks[J.chunk0 + k];
    if (tid == 0) wsums_store(ck.P, W);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __syncthreads();
    int* const flag = &bs->vote[1][7];
    int* const dec = &bs->vote[1][6];
    if (tid == 0) {
        int last = 0;
        if (atomicSub(&J.left, 1) == 1) {
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            WSums T;
            wsums_zero(T);
            for (int q = 0; q < K; ++q) wsums_acc(T, wsums_load(B.chunks[J.chunk0 + q].P));
            *dec = pack_decision(decide_exact_wide(T, M.sh->dc, F));
            last = 1;
        }
        *flag = last;
    }
    __syncthreads();
    if (!*flag) return 0;
    const Decision rd = unpack_decision(*dec);
    __syncthreads();
    if (rd.kind != D_SPLIT) {
        const uint8_t base = INF_SET | (rd.kind == D_MERGED ? INF_MERGED : 0) | (uint8_t)(rd.jdir << INF_JSHIFT);
        for (int i = tid; i < n; i += NT) M.info[i] = base | (i == 0 ? INF_HEAD : 0);
        return 0;
    }
    Node<uint32_t> root;
    root.start = 0; root.len = (uint32_t)n; root.thr_axis = (rd.thr << 8) | rd.axis;
    if (start_wide_job(B, bs, root, 0, qi)) return 0;
    return wide_split(B, M, F, bs, root, 0, qi, kept);
}

// One output task of a cell above NMAX_NARROW (its slots, leaf starts and merged list are complete):
// TASK_COPY copies the unmerged particles of slots a .. a + cnt - 1 to their output slots; TASK_MERGE
// merges the subsets a, a + cnt, a + 2 cnt, ... of the merged list (Step 7), one wavefront each.
template <typename InT>
VPM_DEV void output_task(const BigArgs<InT>& B, const CellMem<uint32_t>& M, const Frame& F, int64_t off, int n,
                         int kind, int a, int cnt, int nm) {
    constexpr int NT = WAVE * 8;
    const auto& A = B.A;
    const int tid = threadIdx.x, lane = lane_id(), wv = tid / WAVE;
    if (kind == TASK_COPY) {
        const InT* const ib[7] = {A.in.x + off, A.in.y + off, A.in.z + off, A.in.px + off,
                                  A.in.py + off, A.in.pz + off, A.in.w + off};
        float* const ob[7] = {A.tmp.x + off, A.tmp.y + off, A.tmp.z + off, A.tmp.px + off,
                              A.tmp.py + off, A.tmp.pz + off, A.tmp.w + off};
        const int end = a + cnt;
        for (int p0 = a + tid; p0 < end; p0 += COPY_BATCH * NT) {
            uint32_t si[COPY_BATCH], so[COPY_BATCH];
            bool keep[COPY_BATCH];
#pragma unroll
            for (int u = 0; u < COPY_BATCH; ++u) {
                const int p = min(p0 + u * NT, end - 1);
                const uint8_t inf = M.info[p];
                si[u] = idx_buf(M, inf & INF_PARITY)[p];
                so[u] = M.emit[p];
                keep[u] = p0 + u * NT < end && !(inf & INF_MERGED);
            }
            float v[COPY_BATCH][7];
#pragma unroll
            for (int u = 0; u < COPY_BATCH; ++u)
                if (keep[u])
#pragma unroll
                    for (int f = 0; f < 7; ++f) v[u][f] = (float)ib[f][si[u]];
#pragma unroll
            for (int u = 0; u < COPY_BATCH; ++u)
                if (keep[u])
#pragma unroll
                    for (int f = 0; f < 7; ++f) ob[f][so[u]] = v[u][f];
        }
    } else {
        const uint32_t* leaf_start = (const uint32_t*)M.rec;
        const uint32_t* mlist = leaf_start + (n + 1);
        for (int k = a + wv * cnt; k < nm; k += 8 * cnt) {
            const int ord = (int)mlist[k];
            const int st = (int)leaf_start[ord];
            const int ln = (int)leaf_start[ord + 1] - st;
            const uint8_t inf = M.info[st];
            const uint32_t* src = idx_buf(M, inf & INF_PARITY);
            merge_subset(A, F, [&](int j) { return off + (int64_t)src[st + j]; }, ln, (inf >> INF_JSHIFT) & 3,
                         off + M.emit[st], lane, WAVE);
        }
    }
}

template <typename InT>
__global__ __launch_bounds__(WAVE * 8, 2) void k_fixed_big(BigArgs<InT> B) {
    constexpr int WPB = 8, NT = WAVE * WPB;
    using IdxT = uint32_t;
    extern __shared__ __align__(16) uint8_t smem[];
    const auto& A = B.A;
    CellShared& sh = *(CellShared*)smem;
    BlockScratch<WPB>* bs = (BlockScratch<WPB>*)(smem + rnd16(sizeof(CellShared)));
    BigShared& bl = *(BigShared*)(smem + header_bytes<WPB>());
    const int wv = threadIdx.x / WAVE;
    int32_t* const ctr = A.counters;
    const int qlen = ctr[A.qlen_index];
    if (qlen == 0) return;                         // an empty bin claims nothing
    if (threadIdx.x == 0) sh.dc = decide_consts(A.P);   // visible after the loop's first barrier
    int nbig[BIGQ_CLASSES];
#pragma unroll
    for (int k = 0; k < BIGQ_CLASSES; ++k) nbig[k] = ctr[BIGQ_LEN0 + k];
    bool cells_left = true;                        // (thread 0)
    for (;;) {
        // ---- a piece of work: a queued task first (cells already started), else a new cell ----
        if (threadIdx.x == 0) {
            int kind = 0, q = 0;
            for (;;) {
                const int h = ld_relaxed(&ctr[C_TASK_HEAD]);
                if (h < ld_relaxed(&ctr[C_TASK_RESERVE]) && ld_relaxed(&B.ready[h % B.ring_size]) == 1) {
                    if (atomicCAS(&ctr[C_TASK_HEAD], h, h + 1) == h) { kind = 2; q = h % B.ring_size; break; }
                    continue;
                }
                if (cells_left) {
                    atomicAdd(&ctr[C_PENDING], 1);           // before the claim: no one sees the grid idle
                    const int qi = atomicAdd(&ctr[A.work_index], 1);
                    if (qi < qlen) { kind = 1; q = qi; break; }
                    atomicSub(&ctr[C_PENDING], 1);
                    cells_left = false;
                    continue;
                }
                // Nothing to take now.  Every queued task is taken at the latest by the workgroup
                // that spawned it, once its piece is done, so leaving is always safe; waiting for
                // tasks adds workgroups to the cells still open.
                if (!B.wait_idle || ld_relaxed(&ctr[C_PENDING]) == 0) break;
                __builtin_amdgcn_s_sleep(8);
            }
            if (kind != 0) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");   // the cell's data written elsewhere
            sh.kind = kind;
            sh.qi = q;
            sh.flags = 0;
            sh.nnext = 0;
        }
        __syncthreads();
        const int kind = __builtin_amdgcn_readfirstlane(sh.kind);
        if (kind == 0) break;
        const int lane = opaque_lane();
        const int tid = opaque_tid();
        int qi, c, n, m = 0, cur = 0;
        bool wide = false;                     // the piece starts with a subset above NMAX_NARROW
        Node<IdxT> wnode;
        int tkind = TASK_NODE, nmerged = 0;
        bool cell_job = false;                 // a new cell whose root passes went to chunk tasks
        int64_t off;
        Frame F;
        CellMem<IdxT> M;
        M.sh = &sh;
        M.nodes0 = B.lists + (int64_t)blockIdx.x * (2 * BIG_NODES);
        M.nodes1 = M.nodes0 + BIG_NODES;
        M.sched = B.sched + (int64_t)blockIdx.x * BIG_NODES;
        if (kind == 1) {
            // ---- a new cell: frame, codes, root moments and decision ----
            qi = __builtin_amdgcn_readfirstlane(sh.qi);
            int v = qi;
            const int32_t* qp = A.bigq[0];
            bool found = false;
#pragma unroll
            for (int k = BIGQ_CLASSES - 1; k > 0; --k) {          // largest size class first
                if (!found) {
                    if (v < nbig[k]) { qp = A.bigq[k]; found = true; } else v -= nbig[k];
                }
            }
            c = qp[v];
            off = A.cell_off[c];
            n = (int)(A.cell_off[c + 1] - off);
            if (n > NMAX_NARROW) {
                // a cell above NMAX_NARROW: its frame and codes are chunk tasks of a job (when job
                // records are left); this piece ends here
                if (tid == 0) {
                    BigCell& bc = B.cells[qi];
                    bc.off = off; bc.n = n; bc.c = c; bc.open = 1; bc.bad = 0;
                }
                Node<IdxT> whole;
                whole.start = 0; whole.len = (IdxT)n; whole.thr_axis = 0;
                cell_job = start_wide_job(B, bs, whole, 0, qi, TASK_CFRAME);
            }
        }
        if (kind == 1 && !cell_job) {
            const bool valid = cell_frame_block<WPB>(A.in, off, n, cell_mass(A.P.mass, A.P.species, A.P.species_mass, c),
                                                     F, bs);
            if (!valid) {
                if (tid == 0) {
                    atomicOr(A.flags, FLAG_BAD_VALUE);
                    if (A.mode == 0) { A.out_count[c] = n; A.cell_mode[c] = CELL_UNTOUCHED; }
                    else A.n_subsets[c] = 0;
                }
                if (A.mode == 1)
                    for (int i = tid; i < n; i += NT) { A.perm[off + i] = (int32_t)(off + i); A.subset_id[off + i] = -1; }
                __syncthreads();
                if (tid == 0) { __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent"); atomicSub(&ctr[C_PENDING], 1); }
                continue;
            }
            if (tid == 0) {
                BigCell& bc = B.cells[qi];
                bc.F = F; bc.off = off; bc.n = n; bc.c = c; bc.open = 1; bc.bad = 0;
            }
        } else if (kind == 2) {
            // ---- a task: a subset of a cell started elsewhere ----
            const BigTask t = B.tasks[sh.qi];
            qi = __builtin_amdgcn_readfirstlane(t.qi);
            const BigCell& bc = B.cells[qi];
            F = bc.F;
            off = bc.off;
            n = bc.n;
            c = bc.c;
            cur = t.cur;
            tkind = t.kind;
            wide = tkind == TASK_NODE && t.nd.len > (uint32_t)NMAX_NARROW;
            wnode = t.nd;
            m = wide || tkind != TASK_NODE ? 0 : 1;
            nmerged = bc.nmerged;
            __syncthreads();                           // every thread has read the slot
            if (tid == 0) {
                if (tkind == TASK_NODE && !wide) (cur ? M.nodes1 : M.nodes0)[0] = t.nd;
                __hip_atomic_store(&B.ready[sh.qi], 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
        M.rec = B.rec + off;
        M.pyz = B.pyz + off;
        M.idx0 = B.idx0 + off;
        M.idx1 = B.idx1 + off;
        M.emit = B.emit + off;
        M.info = B.info + off;
        if (!task_is_piece(tkind)) {
            // part of the output of a cell above NMAX_NARROW (not a piece of its partition)
            output_task(B, M, F, off, n, tkind, (int)wnode.start, (int)wnode.len, nmerged);
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            __syncthreads();
            if (tid == 0) atomicSub(&ctr[C_PENDING], 1);
            continue;
        }
        if (tkind == TASK_CFRAME) {
            cell_frame_task(B, bs, (int)wnode.start, (int)wnode.len);
        } else if (tkind == TASK_CENCODE) {
            m = cell_encode_task(B, M, F, bs, (int)wnode.start, (int)wnode.len, M.nodes1);
            if (m > 0) cur = 1;
        } else if (tkind == TASK_WCOUNT) {
            wide_count_task(B, M, F, bs, (int)wnode.start, (int)wnode.len);
        } else if (tkind == TASK_WPLACE) {
            m = wide_place_task(B, M, bs, (int)wnode.start, (int)wnode.len, cur ? M.nodes0 : M.nodes1);
            cur ^= 1;
        }
        if (kind == 1 && !cell_job) {
            FSums R;
            fsums_zero(R);
            bool oob = false;
            load_particles(A.in, off, tid, n, NT, [&](int i, const float* q, bool ok) {
                if (ok) encode_particle(M, A.P, F, i, q, R, oob);
            });
            const bool any_oob = ballot(oob) != 0;
            fsums_group_reduce(R, WAVE);
            if (lane == 0) {
                bs->sums[wv][0] = R.s0;
                for (int l = 0; l < 6; ++l) { bs->sums[wv][1 + l] = R.s1[l]; bs->sums[wv][7 + l] = R.s2[l]; }
                if (any_oob) atomicOr(&sh.flags, FLAG_OUT_OF_CELL);
            }
            __syncthreads();
            if (n > NMAX_NARROW) {
                // a cell above NMAX_NARROW: the root's moments summed exactly, the exact rule
                wide_root(M, F, n, A.P.min_subset);
            } else if (tid == 0) {
                fsums_zero(R);
                for (int w = 0; w < WPB; ++w) {
                    R.s0 += bs->sums[w][0];
                    for (int l = 0; l < 6; ++l) { R.s1[l] += bs->sums[w][1 + l]; R.s2[l] += bs->sums[w][7 + l]; }
                }
                sh.rootv = pack_decision(decide(M, R, M.idx0, 0, n, A.P, F));
            }
            __syncthreads();
            const Decision rd = unpack_decision(sh.rootv);
            if (rd.kind == D_SPLIT && n > NMAX_NARROW) {
                wide = true;
                wnode.start = 0; wnode.len = (IdxT)n; wnode.thr_axis = (rd.thr << 8) | rd.axis;
            } else if (rd.kind == D_SPLIT) {
                if (tid == 0) {
                    Node<IdxT> nd;
                    nd.start = 0; nd.len = (IdxT)n; nd.thr_axis = (rd.thr << 8) | rd.axis;
                    M.nodes0[0] = nd;
                }
                m = 1;
            } else {
                const uint8_t base = INF_SET | (rd.kind == D_MERGED ? INF_MERGED : 0) | (uint8_t)(rd.jdir << INF_JSHIFT);
                for (int i = tid; i < n; i += NT) M.info[i] = base | (i == 0 ? INF_HEAD : 0);
            }
        }
        __syncthreads();
        if (wide) {
            // a subset above NMAX_NARROW: split by several workgroups (a job of chunk tasks), or by
            // this whole workgroup when the job records are used up; unfinished children of at least
            // TASK_MIN particles become tasks, the smaller ones continue here
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");   // its members and codes, device-wide
            __syncthreads();
            if (!start_wide_job(B, bs, wnode, cur, qi)) {
                m = wide_split(B, M, F, bs, wnode, cur, qi, cur ? M.nodes0 : M.nodes1);
                cur ^= 1;
            }
        }

        // ---- Steps 2-6, level by level; large unfinished subsets become tasks ----
        while (m > 0) {
            Node<IdxT>* curl = cur ? M.nodes1 : M.nodes0;
            Node<IdxT>* nextl = cur ? M.nodes0 : M.nodes1;
            if (tid == 0) {
                sh.nnext = 0;
                bl.spawn.n = 0;
                bl.spawn_ok = ld_relaxed(&ctr[A.work_index]) >= qlen ? 1 : 0;     // no cell left to claim
            }
            const Sched s = schedule<WPB, IdxT>(M, M.sched, m, A.P.ppl_shift, [&](int it) { return (int)curl[it].len; });
            const bool solo = __builtin_amdgcn_readfirstlane(s.total == s.cnt[0] ? 1 : 0) != 0;
            for (int r0 = wv * WAVE; r0 < s.total; r0 += NT) {
                int slot, cls;
                const int ln = opaque_lane();
                if (sched_lookup(s, r0 + ln, slot, cls)) {
                    const Node<IdxT> nd = curl[M.sched[slot]];
                    const int g = 1 << cls;
                    split_node<IdxT>(M, A, F, nullptr, nd, cur, ln & (g - 1), g, ln & ~(g - 1), nextl, solo,
                                     bl.spawn_ok ? &bl.spawn : nullptr);
                }
            }
            __syncthreads();
            const int ns = bl.spawn.n;
            if (ns > 0) {
                // release every wave's writes of this level device-wide (a write-back, no invalidation),
                // then publish the spawned subsets
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
                __syncthreads();
                if (tid == 0)
                    for (int k = 0; k < ns; ++k) spawn_task(B, qi, cur ^ 1, bl.spawn.node[k]);
            }
            m = sh.nnext;
            cur ^= 1;
            __syncthreads();                           // nnext and the spawn list are read before reset
        }

        // ---- the piece is done; the workgroup that closes the cell's last piece writes its output ----
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");   // every wave's writes, device-wide
        __syncthreads();
        if (tid == 0) {
            if (sh.flags) atomicOr(A.flags, sh.flags);
            int last = atomicSub(&B.cells[qi].open, 1) == 1 ? 1 : 0;
            if (last) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");   // every other piece's writes
            if (last && B.cells[qi].bad) last = 0;     // passed through: its output is the input
            sh.last = last;
        }
        __syncthreads();
        if (sh.last) {
            IdxT* scratch = (IdxT*)M.rec;              // the codes are no longer needed
            // a cell above NMAX_NARROW: its copies and merges go to other workgroups as tasks
            const bool defer = n > NMAX_NARROW && A.mode == 0;
            cell_output<WPB, IdxT>(M, A, F, c, off, n, bs, scratch, scratch + (n + 1), scratch + (2 * n + 1),
                                   defer);
            if (defer) {
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");   // slots, leaf starts, merged list
                __syncthreads();
                if (tid == 0) {
                    const int nm = sh.nmerged;
                    B.cells[qi].nmerged = nm;
                    // at most n / NMAX_NARROW tasks of each kind (the ring holds n / TASK_MIN)
                    const int kc = (n + NMAX_NARROW - 1) / NMAX_NARROW, span = (n + kc - 1) / kc;
                    Node<IdxT> r;
                    r.thr_axis = 0;
                    for (int k = 0; k < kc; ++k) {
                        r.start = (IdxT)(k * span);
                        r.len = (IdxT)min(span, n - k * span);
                        spawn_task(B, qi, 0, r, TASK_COPY);
                    }
                    const int km = min(nm, kc);
                    for (int k = 0; k < km; ++k) {
                        r.start = (IdxT)k;
                        r.len = (IdxT)km;
                        spawn_task(B, qi, 0, r, TASK_MERGE);
                    }
                }
            }
        }
        __syncthreads();
        if (tid == 0) {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            atomicSub(&ctr[C_PENDING], 1);
        }
    }
}

// ------------------------------------------------------------------------------------------
// Small cells: one wavefront processes a batch of up to SMALL_CELLS cells (at most NMAX_S particles
// together).  Each cell of the batch is a root subset handled by a lane group: its frame, codes,
// moments and decision (Step 1).  The levels below proceed as for a single cell, the subsets of all
// cells of the batch sharing the lane groups; a subset carries its cell's index.
// ------------------------------------------------------------------------------------------

constexpr int SMALL_CELLS = 16;
constexpr uint8_t INF_SKIP = 0x40;     // slot of a batch cell that is passed through (invalid values)

struct SmallShared {
    int nc;                             // cells in the batch
    int cell[SMALL_CELLS];
    int base[SMALL_CELLS + 1];          // first slot of each cell; base[nc] = slots in use
    int64_t off[SMALL_CELLS];           // the cell's first particle
    int64_t pbase[SMALL_CELLS + 1];     // output-scan value (leaves << 32 | outputs) at each first slot
    uint32_t cflags[SMALL_CELLS];
    Frame frame[SMALL_CELLS];
};

__host__ __device__ constexpr size_t small_header_bytes() {
    return rnd16(sizeof(CellShared)) + rnd16(sizeof(SmallShared));
}

// Index of the batch cell that owns slot p.
VPM_DEV int small_cell_of(const SmallShared& ss, int p) {
    int lo = 0, hi = ss.nc - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (ss.base[mid] <= p) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Step 1 for batch cell j with a lane group: validity, frame, codes, root moments and decision.
template <typename Args>
VPM_DEV void small_root(const CellMem<uint16_t>& M, const Args& A, SmallShared& ss, int j, int g, int lid,
                        int gbase) {
    const int b = ss.base[j], n = ss.base[j + 1] - b;
    const int64_t off = ss.off[j];
    const uint64_t gm = (g == 64 ? ~0ull : ((1ull << g) - 1ull)) << gbase;
    FrameAcc acc;
    facc_init(acc);
    facc_cell(acc, A.in, off, lid, n, g);
    if ((ballot(acc.bad) & gm) != 0) {
        if (lid == 0) ss.cflags[j] = FLAG_BAD_VALUE;
        for (int p = lid; p < n; p += g) M.info[b + p] = INF_SKIP;
        return;
    }
#pragma unroll
    for (int r = 0; r < 11; ++r) acc.v[r] = group_max(acc.v[r], g);
    Frame F;
    frame_from(acc.v, cell_mass(A.P.mass, A.P.species, A.P.species_mass, ss.cell[j]), F);
    if (lid == 0) ss.frame[j] = F;
    FSums R;
    fsums_zero(R);
    bool oob = false;
    load_particles(A.in, off, lid, n, g, [&](int p, const float* q, bool ok) {
        if (ok) encode_particle(M, A.P, F, b + p, q, R, oob);
    });
    fsums_group_reduce(R, g);
    if ((ballot(oob) & gm) != 0 && lid == 0) atomicOr(&ss.cflags[j], FLAG_OUT_OF_CELL);
    wave_fence();
    int dv = 0;
    if (lid == 0) {
        const Decision d = decide(M, R, M.idx0, b, n, A.P, F);
        dv = pack_decision(d);
        if (d.kind == D_SPLIT) {
            const int slot = atomicAdd(&M.sh->nnext, 1);
            Node<uint16_t> nd;
            nd.start = (uint16_t)b; nd.len = (uint16_t)n; nd.thr_axis = (d.thr << 8) | (j << 4) | d.axis;
            M.nodes0[slot] = nd;
        }
    }
    const Decision d = unpack_decision(__shfl(dv, gbase));
    if (d.kind != D_SPLIT) {
        const uint8_t base = INF_SET | (d.kind == D_MERGED ? INF_MERGED : 0) | (uint8_t)(d.jdir << INF_JSHIFT);
        for (int p = lid; p < n; p += g) M.info[b + p] = base | (p == 0 ? INF_HEAD : 0);
    }
}

template <typename InT>
__global__ __launch_bounds__(WAVE, 2) void k_fixed_small(FixedArgsT<InT> A) {
    extern __shared__ __align__(16) uint8_t smem[];
    using IdxT = uint16_t;
    const int lane = lane_id();
    CellShared& sh = *(CellShared*)smem;
    SmallShared& ss = *(SmallShared*)(smem + rnd16(sizeof(CellShared)));
    CellMem<IdxT> M = carve<IdxT>(smem + small_header_bytes(), NMAX_S);
    M.sh = &sh;
    const int qlen = A.counters[A.qlen_index];
    if (qlen == 0) return;                         // an empty bin claims nothing
    if (lane == 0) sh.dc = decide_consts(A.P);
    wave_fence();
    const int npair = A.P.merge_mode == VPM_MERGE_PAIR ? 2 : 1;
    int qnext = 0, qend = 0;
    for (;;) {
        if (qnext >= qend) {
            if (lane == 0) qnext = atomicAdd(&A.counters[A.work_index], SMALL_CELLS);
            qnext = __shfl(qnext, 0);
            qend = min(qnext + SMALL_CELLS, qlen);
        }
        if (qnext >= qlen) break;

        // ---- a batch: the claimed entries in queue order, as many as fit NMAX_S slots ----
        const int avail = qend - qnext;
        int my_c = 0, my_n = 0;
        int64_t my_off = 0;
        if (lane < avail) {
            my_c = A.queue[qnext + lane];
            my_off = A.cell_off[my_c];
            my_n = (int)(A.cell_off[my_c + 1] - my_off);
        }
        int take = 0, tot = 0;
        for (int t = 0; t < avail; ++t) {             // every cell of this bin has at most NMAX_S / 2
            const int nt = __shfl(my_n, t);
            if (tot + nt > NMAX_S) break;
            tot += nt;
            ++take;
        }
        int inc = lane < take ? my_n : 0;
        for (int d = 1; d < WAVE; d <<= 1) {
            const int o = __shfl_up(inc, d);
            if (lane >= d) inc += o;
        }
        if (lane < take) {
            ss.cell[lane] = my_c;
            ss.off[lane] = my_off;
            ss.base[lane] = inc - my_n;
            ss.cflags[lane] = 0;
        }
        if (lane == 0) { ss.base[take] = tot; ss.nc = take; sh.nnext = 0; sh.flags = 0; }
        qnext += take;
        wave_fence();

        // ---- Step 1 for every cell of the batch ----
        {
            const Sched s0 = schedule<1, IdxT>(M, M.emit, take, A.P.ppl_shift,
                                               [&](int it) { return ss.base[it + 1] - ss.base[it]; });
            for (int r0 = 0; r0 < s0.total; r0 += WAVE) {
                int slot, cls;
                if (sched_lookup(s0, r0 + lane, slot, cls)) {
                    const int g = 1 << cls;
                    small_root(M, A, ss, M.emit[slot], g, lane & (g - 1), lane & ~(g - 1));
                }
            }
            wave_fence();
        }
        int m = sh.nnext;

        // ---- Steps 2-6, level by level, all cells of the batch together ----
        int cur = 0;
        while (m > 0) {
            Node<IdxT>* curl = cur ? M.nodes1 : M.nodes0;
            Node<IdxT>* nextl = cur ? M.nodes0 : M.nodes1;
            if (lane == 0) sh.nnext = 0;
            const Sched s = schedule<1, IdxT>(M, M.emit, m, A.P.ppl_shift, [&](int it) { return (int)curl[it].len; });
            const bool solo = __builtin_amdgcn_readfirstlane(s.total == s.cnt[0] ? 1 : 0) != 0;   // only 1-lane groups
            for (int r0 = 0; r0 < s.total; r0 += WAVE) {
                int slot, cls;
                if (sched_lookup(s, r0 + lane, slot, cls)) {
                    const Node<IdxT> nd = curl[M.emit[slot]];
                    const int g = 1 << cls;
                    split_node<IdxT>(M, A, ss.frame[0], ss.frame, nd, cur, lane & (g - 1), g, lane & ~(g - 1), nextl, solo);
                }
            }
            wave_fence();
            m = sh.nnext;
            cur ^= 1;
        }

        // ---- output: one scan over the batch's slots; each cell's values relative to its first slot ----
        const int per = (tot + WAVE - 1) / WAVE;
        const int b0 = min(tot, lane * per), b1 = min(tot, b0 + per);
        auto slot_value = [&](uint8_t inf) -> int64_t {
            if (inf & INF_SKIP) return 0;
            const int e = (inf & INF_MERGED) ? ((inf & INF_HEAD) ? npair : 0) : 1;
            return ((int64_t)((inf & INF_HEAD) ? 1 : 0) << 32) | (int64_t)e;
        };
        int64_t loc = 0;
        for (int p = b0; p < b1; ++p) loc += slot_value(M.info[p]);
        int64_t sinc = loc;
        for (int d = 1; d < WAVE; d <<= 1) {
            const int64_t o = __shfl_up(sinc, d);
            if (lane >= d) sinc += o;
        }
        const int64_t total = __shfl(sinc, WAVE - 1);
        const int64_t pre = sinc - loc;
        {
            int64_t run = pre;
            for (int p = b0; p < b1; ++p) {
                const int jj = small_cell_of(ss, p);
                if (ss.base[jj] == p) ss.pbase[jj] = run;
                run += slot_value(M.info[p]);
            }
            if (lane == 0) ss.pbase[ss.nc] = total;
        }
        IdxT* leaf_start = (IdxT*)M.nodes0;                // first slot of each final subset (batch-wide)
        IdxT* mlist = (IdxT*)M.nodes1;                     // batch-wide ordinals of the merged subsets
        if (lane == 0) sh.nmerged = 0;
        wave_fence();
        {
            int64_t run = pre;
            for (int p = b0; p < b1; ++p) {
                const uint8_t inf = M.info[p];
                const int64_t v = slot_value(inf);
                if (!(inf & INF_SKIP)) {
                    const int jj = small_cell_of(ss, p);
                    const int64_t rel = run - ss.pbase[jj];
                    const int head = (inf & INF_HEAD) ? 1 : 0;
                    const int ordg = (int)(run >> 32) + head - 1;
                    if (A.mode == 0) {
                        M.emit[p] = (IdxT)(rel & 0xffffffff);
                    } else {
                        const int64_t o = ss.off[jj] - ss.base[jj];
                        A.perm[o + p] = (int32_t)(o + idx_buf(M, inf & INF_PARITY)[p]);
                        A.subset_id[o + p] = (int)(rel >> 32) + head - 1;
                    }
                    if (head) {
                        leaf_start[ordg] = (IdxT)p;
                        if ((inf & INF_MERGED) && A.mode == 0) mlist[atomicAdd(&sh.nmerged, 1)] = (IdxT)ordg;
                    }
                }
                run += v;
            }
        }
        if (lane == 0) leaf_start[(int)(total >> 32)] = (IdxT)tot;
        wave_fence();
        if (lane < ss.nc) {
            const int c = ss.cell[lane];
            const int n = ss.base[lane + 1] - ss.base[lane];
            const uint32_t cf = ss.cflags[lane];
            if (cf & FLAG_BAD_VALUE) {
                if (A.mode == 0) { A.out_count[c] = n; A.cell_mode[c] = CELL_UNTOUCHED; }
                else {
                    A.n_subsets[c] = 0;
                    for (int i = 0; i < n; ++i) {
                        A.perm[ss.off[lane] + i] = (int32_t)(ss.off[lane] + i);
                        A.subset_id[ss.off[lane] + i] = -1;
                    }
                }
            } else {
                const int64_t d = ss.pbase[lane + 1] - ss.pbase[lane];
                if (A.mode == 0) { A.out_count[c] = d & 0xffffffff; A.cell_mode[c] = CELL_PROCESSED; }
                else A.n_subsets[c] = (int)(d >> 32);
            }
            const uint32_t fl = cf | (lane == 0 ? sh.flags : 0u);
            if (fl) atomicOr(A.flags, fl);
        }
        if (A.mode == 1) { wave_fence(); continue; }

        // copied particles (subsets below min_subset)
        copy_particles<COPY_BATCH>(A.in, A.tmp, lane, tot, WAVE, [&](int p, int64_t& si, int64_t& so) {
            const uint8_t inf = M.info[p];
            const int jj = small_cell_of(ss, p);
            const bool keep = !(inf & (INF_MERGED | INF_SKIP));       // skipped cells have no index lists
            si = ss.off[jj] - ss.base[jj] + (keep ? (int)idx_buf(M, inf & INF_PARITY)[p] : p);
            so = keep ? ss.off[jj] + M.emit[p] : -1;
        });
        // merged subsets (Step 7)
        const int nm = sh.nmerged;
        if (nm > 0) {
            IdxT* sched = (IdxT*)M.rec;                    // the codes are free now
            auto leaf_len = [&](int ord) {
                const int st = leaf_start[ord];
                return min((int)leaf_start[ord + 1], ss.base[small_cell_of(ss, st) + 1]) - st;
            };
            const Sched s = schedule<1, IdxT>(M, sched, nm, A.P.ppl_shift, [&](int it) { return leaf_len(mlist[it]); });
            for (int r0 = 0; r0 < s.total; r0 += WAVE) {
                int slot, cls;
                if (sched_lookup(s, r0 + lane, slot, cls)) {
                    const int ord = mlist[sched[slot]];
                    const int st = leaf_start[ord];
                    const int ln = leaf_len(ord);
                    const int jj = small_cell_of(ss, st);
                    const int64_t o0 = ss.off[jj] - ss.base[jj];
                    const int g = 1 << cls;
                    const uint8_t inf = M.info[st];
                    const IdxT* src = idx_buf(M, inf & INF_PARITY);
                    merge_subset(A, ss.frame[jj], [&](int x) { return o0 + (int64_t)src[st + x]; }, ln,
                                 (inf >> INF_JSHIFT) & 3, ss.off[jj] + M.emit[st], lane & (g - 1), g);
                }
            }
        }
        wave_fence();
    }
}

// ------------------------------------------------------------------------------------------
// The blind method, the paper's comparison (Sec. "Simulation", before the blocks test): pairs of
// particles picked at random are merged until at most ceil(alpha N) remain in a cell of N > N_min
// particles.  Draws: Philox4x64-10 (Salmon et al., SC 2011), key (seed, 0), counter (t, c, 0, 0)
// for the t-th merge of cell c; with M = N - t left, i = r0 mod M and j = r1 mod (M - 1), shifted
// past i.  The particle in slot j joins slot i's group and the last slot fills slot j.  Output k
// is the group of slot k: a single particle is copied, a larger group replaced by its centroid
// (the fixed-point Step 7 sums, one particle: weight and momentum kept).
// ------------------------------------------------------------------------------------------

template <typename InT>
struct BlindArgs {
    FixedArgsT<InT> A;                   // in, cell_off, P (mass; CENTROID), tmp, out_count, cell_mode, flags
    double alpha;
    uint64_t seed;
    int32_t n_min_cell;
    int64_t n_cells, n_particles;
    int32_t *slot, *parent, *aux;  // scratch indexed by input position
    int32_t* group;                // optional: cell-local output ordinal of each input particle
};

VPM_DEV void philox4x64_10(uint64_t& c0, uint64_t& c1, uint64_t& c2, uint64_t& c3, uint64_t k0, uint64_t k1) {
    constexpr uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
    constexpr uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t hi0 = __umul64hi(M0, c0), lo0 = M0 * c0;
        const uint64_t hi1 = __umul64hi(M1, c2), lo1 = M1 * c2;
        const uint64_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
        c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
        k0 += W0; k1 += W1;
    }
}

template <typename InT>
__global__ __launch_bounds__(WAVE) void k_fixed_blind(BlindArgs<InT> B) {
    const auto& A = B.A;
    const int lane = lane_id();
    for (int64_t c = blockIdx.x; c < B.n_cells; c += gridDim.x) {
        const int64_t lo = A.cell_off[c], hi = A.cell_off[c + 1];
        const bool range_ok = lo >= 0 && hi >= lo && hi <= B.n_particles && (c != 0 || lo == 0);
        const int64_t n64 = range_ok ? hi - lo : 0;
        const int n = (int)min<int64_t>(n64, (int64_t)NMAX_BIG + 1);
        const int64_t T = (int64_t)ceil(B.alpha * (double)n64);
        uint32_t fl = range_ok ? 0u : FLAG_BAD_OFFSETS;
        if (n64 > NMAX_BIG) fl |= FLAG_TOO_LARGE;
        bool touched = range_ok && n64 > 0 && n64 > B.n_min_cell && T < n64 && n64 <= NMAX_BIG;
        Frame F;
        if (touched && !cell_frame(A.in, lo, n, cell_mass(A.P.mass, nullptr, nullptr, c), F)) {
            fl |= FLAG_BAD_VALUE;
            touched = false;
        }
        if (fl && lane == 0) atomicOr(A.flags, fl);
        if (!touched) {
            if (lane == 0) { A.out_count[c] = n64; A.cell_mode[c] = CELL_UNTOUCHED; }
            if (B.group && range_ok)
                for (int64_t i = lane; i < n64; i += WAVE) B.group[lo + i] = (int32_t)i;
            continue;
        }
        int32_t* const S = B.slot + lo;
        int32_t* const Pa = B.parent + lo;
        int32_t* const X = B.aux + lo;
        for (int i = lane; i < n; i += WAVE) { S[i] = i; Pa[i] = i; }
        wave_fence();
        // the merges: 64 draws at a time in parallel, applied to the slots in order by lane 0
        const int nm = n - (int)T;
        for (int t0 = 0; t0 < nm; t0 += WAVE) {
            const int t = t0 + lane;
            int di = 0, dj = 0;
            if (t < nm) {
                uint64_t c0 = (uint64_t)t, c1 = (uint64_t)c, c2 = 0, c3 = 0;
                philox4x64_10(c0, c1, c2, c3, B.seed, 0);
                const uint32_t M = (uint32_t)(n - t);
                di = (int)(c0 % M);
                dj = (int)(c1 % (M - 1));
                dj += dj >= di ? 1 : 0;
            }
            const int cnt = min(WAVE, nm - t0);
            for (int u = 0; u < cnt; ++u) {
                const int i = __shfl(di, u), j = __shfl(dj, u);
                if (lane == 0) {
                    const int M = n - (t0 + u);
                    Pa[S[j]] = S[i];
                    S[j] = S[M - 1];
                }
            }
        }
        wave_fence();
        // output ordinal of each surviving group, then the group of every particle (into S)
        for (int k = lane; k < (int)T; k += WAVE) X[S[k]] = k;
        wave_fence();
        for (int i = lane; i < n; i += WAVE) {
            int r = i;
            while (Pa[r] != r) r = Pa[r];
            const int g = X[r];
            if (B.group) B.group[lo + i] = g;
            S[i] = g;                                  // S[k < T] was read above, before the fence
        }
        wave_fence();
        // members of each group (counting sort into X; Pa holds the running starts)
        for (int k = lane; k <= (int)T; k += WAVE) Pa[k] = 0;
        wave_fence();
        for (int i = lane; i < n; i += WAVE) atomicAdd(&Pa[S[i]], 1);
        wave_fence();
        int carry = 0;
        for (int k0 = 0; k0 < (int)T; k0 += WAVE) {
            const int k = k0 + lane;
            const int v = k < (int)T ? Pa[k] : 0;
            const int inc = wave_incl_scan(v, lane);
            if (k < (int)T) Pa[k] = carry + inc - v;
            carry += __shfl(inc, WAVE - 1);
        }
        wave_fence();
        for (int i = lane; i < n; i += WAVE) X[atomicAdd(&Pa[S[i]], 1)] = i;
        wave_fence();
        // Pa[k] is now the end of group k; one lane per output
        for (int k = lane; k < (int)T; k += WAVE) {
            const int b = k == 0 ? 0 : Pa[k - 1], len = Pa[k] - b;
            const int64_t o = lo + k;
            if (len == 1) {
                const int64_t i = lo + X[b];
                A.tmp.x[o] = (float)A.in.x[i]; A.tmp.y[o] = (float)A.in.y[i]; A.tmp.z[o] = (float)A.in.z[i];
                A.tmp.px[o] = (float)A.in.px[i]; A.tmp.py[o] = (float)A.in.py[i]; A.tmp.pz[o] = (float)A.in.pz[i];
                A.tmp.w[o] = (float)A.in.w[i];
            } else {
                merge_subset(A, F, [&](int j) { return lo + (int64_t)X[b + j]; }, len, 0, o, 0, 1);
            }
        }
        if (lane == 0) { A.out_count[c] = T; A.cell_mode[c] = CELL_PROCESSED; }
        wave_fence();
    }
}

constexpr int WPB_A = 1, WPB_D = 2, WPB_B = 4, WPB_C = 8, WPB_BIG = 8;

// Each LDS bin's limit is the largest cell for which 8 / 4 / 2 / 1 cells still fit a CU's 160 KB of
// LDS (the occupancy step the bin is sized for: two waves per SIMD at the cell kernels' VGPR count).
constexpr size_t LDS_PER_CU = 160 * 1024;
static_assert(header_bytes<WPB_A>() + slice_bytes<uint16_t>(NMAX_A) <= LDS_PER_CU / 8, "bin A: 8 cells per CU");
static_assert(header_bytes<WPB_D>() + slice_bytes<uint16_t>(NMAX_D) <= LDS_PER_CU / 4, "bin D: 4 cells per CU");
static_assert(header_bytes<WPB_B>() + slice_bytes<uint16_t>(NMAX_B) <= LDS_PER_CU / 2, "bin B: 2 cells per CU");
static_assert(header_bytes<WPB_C>() + slice_bytes<uint16_t>(NMAX_C) <= LDS_PER_CU, "bin C: 1 cell per CU");

}  // namespace

int fixed_lds_bytes(int which) {
    switch (which) {
        case 4: return (int)(small_header_bytes() + slice_bytes<uint16_t>(NMAX_S));
        case 0: return (int)(header_bytes<WPB_A>() + slice_bytes<uint16_t>(NMAX_A));
        case 1: return (int)(header_bytes<WPB_B>() + slice_bytes<uint16_t>(NMAX_B));
        case 2: return (int)(header_bytes<WPB_C>() + slice_bytes<uint16_t>(NMAX_C));
        case 5: return (int)(header_bytes<WPB_D>() + slice_bytes<uint16_t>(NMAX_D));
        default: return (int)big_lds_bytes();
    }
}

int64_t fixed_big_cell_bytes() { return (int64_t)sizeof(BigCell); }
int64_t fixed_big_task_bytes() { return (int64_t)sizeof(BigTask); }
int64_t fixed_wide_job_bytes() { return (int64_t)sizeof(WideJob); }
int64_t fixed_wide_chunk_bytes() { return (int64_t)sizeof(WideChunk); }
int fixed_task_min() { return TASK_MIN; }
int64_t fixed_big_lists_bytes() { return (int64_t)(2 * BIG_NODES) * (int64_t)sizeof(Node<uint32_t>); }
int64_t fixed_big_sched_bytes() { return (int64_t)BIG_NODES * 4; }

const void* fixed_kernel_ptr(int which) {
    switch (which) {
        case 4: return (const void*)k_fixed_small<float>;
        case 0: return (const void*)k_fixed_cells<NMAX_A, uint16_t, true, WPB_A, float>;
        case 1: return (const void*)k_fixed_cells<NMAX_B, uint16_t, true, WPB_B, float>;
        case 2: return (const void*)k_fixed_cells<NMAX_C, uint16_t, true, WPB_C, float>;
        case 5: return (const void*)k_fixed_cells<NMAX_D, uint16_t, true, WPB_D, float>;
        default: return (const void*)k_fixed_big<float>;
    }
}

int fixed_block_threads(int which) {
    return WAVE * (which == 0 || which == 4 ? 1 : which == 1 ? WPB_B : which == 2 ? WPB_C : which == 5 ? WPB_D : WPB_BIG);
}

namespace {

template <typename InT>
hipError_t fixed_merge_t(const Workspace& ws, const LaunchCfg& lc, const SoaIn<InT>& in, const int64_t* cell_off,
                         const FixedParams& fp, const int32_t* perm, const int32_t* subset_id,
                         const int32_t* n_subsets) {
    MergeArgs<InT> G;
    auto& A = G.A;
    A.in = in;
    A.cell_off = cell_off;
    A.counters = ws.counters;
    A.P = fp;
    A.mode = 0;
    A.tmp = Soa32Out{(float*)ws.tmp[0], (float*)ws.tmp[1], (float*)ws.tmp[2], (float*)ws.tmp[3],
                     (float*)ws.tmp[4], (float*)ws.tmp[5], (float*)ws.tmp[6]};
    A.out_count = ws.out_count;
    A.cell_mode = ws.cell_mode;
    A.flags = ws.flags;
    A.perm = nullptr; A.subset_id = nullptr; A.n_subsets = nullptr;
    for (int k = 0; k < BIGQ_CLASSES; ++k) A.bigq[k] = ws.bigq[k];
    G.perm = perm; G.subset_id = subset_id; G.n_subsets = n_subsets;
    G.starts = ws.perm2;
    G.marks = ws.perm2 + (ws.cap_particles + 1);   // the second of the two buffers
    const int qs[6] = {Q_BIG, Q_C, Q_B, Q_S, Q_D, Q_A};
    for (int q : qs) {
        A.queue = ws.queue[q];
        A.qlen_index = q;
        A.work_index = 8 + q;
        if (lc.pre) lc.pre(lc.prof, "fixed_merge", lc.stream);
        hipLaunchKernelGGL(k_fixed_merge<InT>, dim3(lc.grid_fp64), dim3(WAVE), 0, lc.stream, G);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        if (lc.post) lc.post(lc.prof, "fixed_merge", lc.stream);
    }
    return hipSuccess;
}

template <typename InT>
hipError_t fixed_cells_t(const Workspace& ws, const LaunchCfg& lc, const SoaIn<InT>& in, const int64_t* cell_off,
                         const FixedParams& fp, int mode, int32_t* perm, int32_t* subset_id, int32_t* n_subsets) {
    FixedArgsT<InT> A;
    A.in = in;
    A.cell_off = cell_off;
    A.counters = ws.counters;
    A.P = fp;
    A.mode = mode;
    A.tmp = Soa32Out{(float*)ws.tmp[0], (float*)ws.tmp[1], (float*)ws.tmp[2], (float*)ws.tmp[3],
                     (float*)ws.tmp[4], (float*)ws.tmp[5], (float*)ws.tmp[6]};
    A.out_count = ws.out_count;
    A.cell_mode = ws.cell_mode;
    A.flags = ws.flags;
    A.perm = perm; A.subset_id = subset_id; A.n_subsets = n_subsets;
    for (int k = 0; k < BIGQ_CLASSES; ++k) A.bigq[k] = ws.bigq[k];
    BigArgs<InT> G;
    G.rec = (int4*)ws.big_rec;
    G.pyz = ws.big_pyz;
    G.idx0 = ws.big_idx0;
    G.idx1 = ws.big_idx1;
    G.emit = ws.big_emit;
    G.info = ws.big_info;
    G.cells = (BigCell*)ws.big_cells;
    G.tasks = (BigTask*)ws.big_tasks;
    G.ready = ws.big_ready;
    G.ring_size = (int32_t)ws.ring_size;
    G.lists = (Node<uint32_t>*)ws.big_lists;
    G.sched = ws.big_sched;
    G.jobs = (WideJob*)ws.big_jobs;
    G.chunks = (WideChunk*)ws.big_chunks;
    G.jobs_cap = ws.big_jobs ? ws.jobs_cap : 0;
    G.chunks_cap = ws.big_chunks ? ws.chunks_cap : 0;

    // The bins touch disjoint cells, queues and counters, so they may run concurrently.  Mode 1: the
    // large-cell, eight- and four-wavefront bins go first on the side streams (their cells are the
    // longest) and the others fill the rest of the chip on the caller's stream: the two-wavefront
    // bin, the small-cell batches, then the one-wavefront bin (the order that measured fastest on
    // a population spread over every bin).  Mode 2: only the
    // two-wavefront bin goes to a side stream, where its cells (few, in a population centred on the
    // one-wavefront bin's sizes) overlap the one-wavefront bin instead of running alone before it.
    // The caller's stream then waits for the side streams.
    const int nside = lc.conc_mode == 2 ? 1 : 3;
    bool forked = lc.fork != nullptr;
    for (int i = 0; i < nside; ++i) forked = forked && lc.side[i] && lc.join[i];
    const bool big_side = forked && nside == 3, d_side = forked && nside == 1;
    // idle workgroups of the large-cell kernel wait for tasks unless that kernel shares the chip
    G.wait_idle = big_side ? 0 : 1;
    hipError_t e = hipSuccess;
    // The side streams that have waited on the fork are joined back to the caller's stream on
    // every return, also after a failure, so that a stream capture in progress stays well formed.
    int waited = 0;
    auto join_back = [&](hipError_t err) {
        for (int i = 0; i < waited; ++i) {
            const hipError_t r = hipEventRecord(lc.join[i], lc.side[i]);
            const hipError_t w = r == hipSuccess ? hipStreamWaitEvent(lc.stream, lc.join[i], 0) : r;
            if (err == hipSuccess) err = w;
        }
        return err;
    };
    if (forked) {
        e = hipEventRecord(lc.fork, lc.stream);
        for (int i = 0; i < nside && e == hipSuccess; ++i) {
            e = hipStreamWaitEvent(lc.side[i], lc.fork, 0);
            if (e == hipSuccess) waited = i + 1;
        }
        if (e != hipSuccess) return join_back(e);
    }
    struct Bin { int q; const char* name; hipStream_t s; };
    const Bin bins[6] = {{Q_BIG, "fixed_cells_big", big_side ? lc.side[0] : lc.stream},
                         {Q_C, "fixed_cells_4592", big_side ? lc.side[1] : lc.stream},
                         {Q_B, "fixed_cells_2288", big_side ? lc.side[2] : lc.stream},
                         {Q_D, "fixed_cells_1144", d_side ? lc.side[0] : lc.stream},
                         {Q_S, "fixed_cells_small", lc.stream},
                         {Q_A, "fixed_cells_576", lc.stream}};
    for (const Bin& b : bins) {
        A.queue = ws.queue[b.q];
        A.qlen_index = b.q;
        A.work_index = 8 + b.q;
        if (lc.pre) lc.pre(lc.prof, b.name, b.s);
        if (b.q == Q_A)
            hipLaunchKernelGGL((k_fixed_cells<NMAX_A, uint16_t, true, WPB_A, InT>), dim3(lc.grid_a), dim3(WAVE * WPB_A),
                               fixed_lds_bytes(0), b.s, A);
        else if (b.q == Q_B)
            hipLaunchKernelGGL((k_fixed_cells<NMAX_B, uint16_t, true, WPB_B, InT>), dim3(lc.grid_b), dim3(WAVE * WPB_B),
                               fixed_lds_bytes(1), b.s, A);
        else if (b.q == Q_D)
            hipLaunchKernelGGL((k_fixed_cells<NMAX_D, uint16_t, true, WPB_D, InT>), dim3(lc.grid_d), dim3(WAVE * WPB_D),
                               fixed_lds_bytes(5), b.s, A);
        else if (b.q == Q_S)
            hipLaunchKernelGGL(k_fixed_small<InT>, dim3(lc.grid_s), dim3(WAVE), fixed_lds_bytes(4), b.s, A);
        else if (b.q == Q_C)
            hipLaunchKernelGGL((k_fixed_cells<NMAX_C, uint16_t, true, WPB_C, InT>), dim3(lc.grid_c), dim3(WAVE * WPB_C),
                               fixed_lds_bytes(2), b.s, A);
        else {
            G.A = A;
            hipLaunchKernelGGL(k_fixed_big<InT>, dim3(lc.grid_big), dim3(WAVE * WPB_BIG), fixed_lds_bytes(3), b.s, G);
        }
        e = hipGetLastError();
        if (e != hipSuccess) return join_back(e);
        if (lc.post) lc.post(lc.prof, b.name, b.s);
    }
    return join_back(e);
}

template <typename InT>
hipError_t fixed_blind_t(const Workspace& ws, const LaunchCfg& lc, const SoaIn<InT>& in, const int64_t* cell_off,
                         int64_t n_cells, int64_t n_particles, const FixedParams& fp, double alpha, uint64_t seed,
                         int32_t n_min_cell, int32_t* group) {
    BlindArgs<InT> B;
    auto& A = B.A;
    A.in = in;
    A.cell_off = cell_off;
    A.counters = ws.counters;
    A.P = fp;
    A.P.merge_mode = VPM_MERGE_CENTROID;
    A.mode = 0;
    A.tmp = Soa32Out{(float*)ws.tmp[0], (float*)ws.tmp[1], (float*)ws.tmp[2], (float*)ws.tmp[3],
                     (float*)ws.tmp[4], (float*)ws.tmp[5], (float*)ws.tmp[6]};
    A.out_count = ws.out_count;
    A.cell_mode = ws.cell_mode;
    A.flags = ws.flags;
    A.perm = nullptr; A.subset_id = nullptr; A.n_subsets = nullptr;
    for (int k = 0; k < BIGQ_CLASSES; ++k) A.bigq[k] = nullptr;
    B.alpha = alpha;
    B.seed = seed;
    B.n_min_cell = n_min_cell;
    B.n_cells = n_cells;
    B.n_particles = n_particles;
    B.slot = ws.perm2;
    B.parent = ws.perm2 + (ws.cap_particles + 1);
    B.aux = (int32_t*)ws.stack;
    B.group = group;
    if (n_cells == 0) return hipSuccess;
    const int64_t cap = (int64_t)lc.grid_fp64 * 2;
    const int64_t grid = n_cells < cap ? n_cells : cap;
    if (lc.pre) lc.pre(lc.prof, "fixed_blind", lc.stream);
    hipLaunchKernelGGL(k_fixed_blind<InT>, dim3((unsigned)grid), dim3(WAVE), 0, lc.stream, B);
    const hipError_t e = hipGetLastError();
    if (lc.post) lc.post(lc.prof, "fixed_blind", lc.stream);
    return e;
}

}  // namespace

hipError_t launch_fixed_cells(const Workspace& ws, const LaunchCfg& lc, const Soa32& in, const int64_t* cell_off,
                              const FixedParams& fp, int mode, int32_t* perm, int32_t* subset_id, int32_t* n_subsets) {
    return fixed_cells_t(ws, lc, in, cell_off, fp, mode, perm, subset_id, n_subsets);
}
hipError_t launch_fixed_cells(const Workspace& ws, const LaunchCfg& lc, const Soa64& in, const int64_t* cell_off,
                              const FixedParams& fp, int mode, int32_t* perm, int32_t* subset_id, int32_t* n_subsets) {
    return fixed_cells_t(ws, lc, in, cell_off, fp, mode, perm, subset_id, n_subsets);
}
hipError_t launch_fixed_merge(const Workspace& ws, const LaunchCfg& lc, const Soa32& in, const int64_t* cell_off,
                              const FixedParams& fp, const int32_t* perm, const int32_t* subset_id,
                              const int32_t* n_subsets) {
    return fixed_merge_t(ws, lc, in, cell_off, fp, perm, subset_id, n_subsets);
}
hipError_t launch_fixed_merge(const Workspace& ws, const LaunchCfg& lc, const Soa64& in, const int64_t* cell_off,
                              const FixedParams& fp, const int32_t* perm, const int32_t* subset_id,
                              const int32_t* n_subsets) {
    return fixed_merge_t(ws, lc, in, cell_off, fp, perm, subset_id, n_subsets);
}
hipError_t launch_fixed_blind(const Workspace& ws, const LaunchCfg& lc, const Soa32& in, const int64_t* cell_off,
                              int64_t n_cells, int64_t n_particles, const FixedParams& fp, double alpha, uint64_t seed,
                              int32_t n_min_cell, int32_t* group) {
    return fixed_blind_t(ws, lc, in, cell_off, n_cells, n_particles, fp, alpha, seed, n_min_cell, group);
}
hipError_t launch_fixed_blind(const Workspace& ws, const LaunchCfg& lc, const Soa64& in, const int64_t* cell_off,
                              int64_t n_cells, int64_t n_particles, const FixedParams& fp, double alpha, uint64_t seed,
                              int32_t n_min_cell, int32_t* group) {
    return fixed_blind_t(ws, lc, in, cell_off, n_cells, n_particles, fp, alpha, seed, n_min_cell, group);
}

}  // namespace vpm

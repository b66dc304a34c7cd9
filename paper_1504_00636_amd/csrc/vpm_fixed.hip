// Fixed-point Voronoi particle merging on gfx950 (the batched FP32 hot path).
//
// One workgroup owns one simulation cell at a time (persistent grid popping a size-binned
// queue).  The cell's particles are turned into integer codes once (Sec. "Algorithm",
// Step 1 collects the cell; the codes fix its frame):
//     weight    omega = rint(w * 2^(15 - e_w))          e_w: frexp exponent of the cell's max w
//     position  c     = min(rint((x - lo) * s), 65535) - 32768,  s = fl32(65536 / L), lo = cell min
//     momentum  c     = rint(p * 2^(22 - e_a))          e_a: frexp exponent of the cell's max |p_a|
// and every subset ("Voronoi cell") is described by exact integer moments
//     S0 = sum omega,  S1_l = sum omega c_l,  S2_l = sum omega c_l^2.
// The coefficient of variation (Eqs. cv_x, cv_p) is compared exactly:
//     Delta_l^2 = V_l / D_l,  V_l = S0 S2_l - S1_l^2,  D = 2^32 S0^2 (positions), S1_l^2 (momenta)
// Step 3 (stop when all six CVs <= tolerance), Step 4 (largest CV, ties to the lowest axis) and
// Step 5 (cut q <= Q, i.e. c S0 <= S1) are all integer operations, so the partition does not
// depend on summation order or launch shape.
//
// Splitting is level-synchronous.  Every unfinished subset of a level is handled by a group of
// g lanes inside one wavefront (g a power of two chosen from the subset size): the group counts
// the lower side, compacts the subset stably with ballots into the other index buffer (Step 6),
// sums the moments of both children and its first two lanes decide the children.
//
// Replacement (Step 7): each finished subset of at least min_subset particles is merged from
// the FP32 data with order-independent int64 fixed-point sums (weight, weighted position,
// weighted momentum offset from the subset's first particle, weighted energy offset) and an
// FP64 solve for the centroid or the energy-conserving pair.
#include "vpm_device.hpp"
#include "vpm_internal.h"

namespace vpm {
namespace {

constexpr int BLOCK = 256;          // threads per workgroup
constexpr int PPL = 8;              // target particles per lane when sizing a group

// info byte per slot once its final subset is known
constexpr uint8_t INF_PARITY = 0x01;   // index buffer that holds the final order
constexpr uint8_t INF_HEAD = 0x02;     // first slot of its final subset
constexpr uint8_t INF_MERGED = 0x04;   // the subset is merged (else copied)
constexpr int INF_JSHIFT = 3;          // bits 3-4: pair-direction axis
constexpr uint8_t INF_SET = 0x80;

template <typename IdxT>
struct Node { IdxT start, len; int32_t thr_axis; };   // thr_axis = (threshold << 3) | axis

struct Frame {
    float lo[3], hi[3], pmax[3], wmax;
    int ew, ep[3], pzero[3];
    int ext_e[3];        // frexp exponent of the cell's extent per position axis
    int eb;              // frexp exponent of a bound on |eps_i - eps_pivot| over the cell
    int bad;
};

struct Sums {
    uint32_t s0;
    int64_t s1[6];
    int64_t s2p[3];      // positions: <= 2^61
    U128 s2m[3];         // momenta:   <= 2^75
};

VPM_DEV void sums_zero(Sums& S) {
    S.s0 = 0;
#pragma unroll
    for (int l = 0; l < 6; ++l) S.s1[l] = 0;
#pragma unroll
    for (int a = 0; a < 3; ++a) { S.s2p[a] = 0; S.s2m[a] = u128_make(0, 0); }
}

VPM_DEV void sums_add(Sums& S, uint32_t om, int c0, int c1, int c2, int c3, int c4, int c5) {
    S.s0 += om;
    const int64_t o = (int64_t)om;
    const int cp[3] = {c0, c1, c2};
    const int cm[3] = {c3, c4, c5};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const int64_t t = (int64_t)((int32_t)om * cp[a]);     // |t| <= 2^30
        S.s1[a] += t;
        S.s2p[a] += t * cp[a];
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const int64_t t = o * cm[a];                         // |t| <= 2^37
        S.s1[3 + a] += t;
        const uint64_t q = (uint64_t)(t * cm[a]);            // <= 2^59
        const uint64_t lo = S.s2m[a].lo + q;
        S.s2m[a].hi += (lo < q) ? 1u : 0u;
        S.s2m[a].lo = lo;
    }
}

VPM_DEV void sums_merge(Sums& A, const Sums& B) {
    A.s0 += B.s0;
#pragma unroll
    for (int l = 0; l < 6; ++l) A.s1[l] += B.s1[l];
#pragma unroll
    for (int a = 0; a < 3; ++a) { A.s2p[a] += B.s2p[a]; A.s2m[a] = add128(A.s2m[a], B.s2m[a]); }
}

VPM_DEV Sums sums_shfl_xor(const Sums& S, int m) {
    Sums R;
    R.s0 = __shfl_xor(S.s0, m);
#pragma unroll
    for (int l = 0; l < 6; ++l) R.s1[l] = __shfl_xor(S.s1[l], m);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        R.s2p[a] = __shfl_xor(S.s2p[a], m);
        R.s2m[a] = u128_make(__shfl_xor(S.s2m[a].lo, m), __shfl_xor(S.s2m[a].hi, m));
    }
    return R;
}

VPM_DEV void sums_group_reduce(Sums& S, int g) {
    for (int m = 1; m < g; m <<= 1) sums_merge(S, sums_shfl_xor(S, m));
}

// ------------------------------------------------------------------------------------------
// Decisions (Steps 3-5), exact.
// ------------------------------------------------------------------------------------------

enum { D_SPLIT = 0, D_MERGED = 1, D_COPY = 2 };

struct Decision { int kind, axis, thr, jdir; };

VPM_DEV uint64_t uabs64(int64_t v) { return v < 0 ? (uint64_t)(-v) : (uint64_t)v; }

// Pair-direction axis: the momentum component with the smallest |mean|, from the exact sums.
VPM_DEV int pair_axis(const Sums& S, const Frame& F) {
    int best = 0;
    double bv = 0.0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const double v = F.pzero[a] ? 0.0 : ldexp((double)uabs64(S.s1[3 + a]), F.ep[a]);
        if (a == 0 || v < bv) { bv = v; best = a; }
    }
    return best;
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

VPM_DEV Decision decide(const Sums& S, int len, const FixedParams& P, const Frame& F) {
    Decision d;
    d.axis = 0; d.thr = 0; d.jdir = 0;
    if (len < P.min_subset) { d.kind = D_COPY; return d; }
    d.jdir = pair_axis(S, F);
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
    // Step 3: all six CVs within tolerance?
    bool done = true;
    {
        const U128 rhs = mul64(P.that_x * P.that_x, s0sq.lo);     // That^2 S0^2
#pragma unroll
        for (int a = 0; a < 3; ++a)
            if (!is_zero128(V[a]) && cmp128(shl128(V[a], 16), rhs) > 0) done = false;
        const U128 tp2 = u128_make(P.that_p * P.that_p, 0);
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
    // Step 4: axis of the largest CV (ties to the lowest axis)
    int k = 0;
    U128 bV = V[0], bD = D[0];
    int64_t s1 = S.s1[0];
#pragma unroll
    for (int l = 1; l < 6; ++l)
        if (frac_gt(V[l], D[l], bV, bD)) { k = l; bV = V[l]; bD = D[l]; s1 = S.s1[l]; }
    // Step 5: c * S0 <= S1  <=>  c <= floor(S1 / S0)
    int64_t t = (int64_t)floor((double)s1 / (double)s0);
    if (t * (int64_t)s0 > s1) t -= 1;
    else if ((t + 1) * (int64_t)s0 <= s1) t += 1;
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

VPM_DEV int group_size_for(int len) {
    int want = (len + PPL - 1) / PPL;
    int g = 1;
    while (g < want && g < WAVE) g <<= 1;
    return g;
}

VPM_DEV void wave_fence() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// ------------------------------------------------------------------------------------------
// Per-cell memory (LDS or a global slab) and kernel arguments.
// ------------------------------------------------------------------------------------------

template <typename IdxT>
struct CellMem {
    uint16_t* om;
    int16_t *cp0, *cp1, *cp2;
    int32_t *cm0, *cm1, *cm2;
    IdxT *idx0, *idx1;
    uint8_t* info;
    IdxT* emit;                    // output slot per position; lane map while splitting
    Node<IdxT> *nodes0, *nodes1;   // current / next level (also leaf tables at the end)
};

template <typename IdxT>
__host__ __device__ constexpr size_t cell_mem_bytes(int nmax) {
    return (size_t)nmax * (2 + 6 + 12 + 2 * sizeof(IdxT) + 1 + sizeof(IdxT)) +
           sizeof(IdxT) + 2 * ((size_t)nmax / 2 + 2) * sizeof(Node<IdxT>) + 64;
}

template <typename IdxT>
VPM_DEV CellMem<IdxT> carve(uint8_t* base, int nmax) {
    CellMem<IdxT> M;
    size_t o = 0;
    auto take = [&](size_t bytes) { uint8_t* p = base + o; o += (bytes + 15) & ~(size_t)15; return p; };
    M.nodes0 = (Node<IdxT>*)take(((size_t)nmax / 2 + 2) * sizeof(Node<IdxT>));
    M.nodes1 = (Node<IdxT>*)take(((size_t)nmax / 2 + 2) * sizeof(Node<IdxT>));
    M.cm0 = (int32_t*)take((size_t)nmax * 4);
    M.cm1 = (int32_t*)take((size_t)nmax * 4);
    M.cm2 = (int32_t*)take((size_t)nmax * 4);
    M.idx0 = (IdxT*)take((size_t)nmax * sizeof(IdxT));
    M.idx1 = (IdxT*)take((size_t)nmax * sizeof(IdxT));
    M.emit = (IdxT*)take(((size_t)nmax + 1) * sizeof(IdxT));
    M.om = (uint16_t*)take((size_t)nmax * 2);
    M.cp0 = (int16_t*)take((size_t)nmax * 2);
    M.cp1 = (int16_t*)take((size_t)nmax * 2);
    M.cp2 = (int16_t*)take((size_t)nmax * 2);
    M.info = (uint8_t*)take((size_t)nmax);
    return M;
}

template <typename IdxT>
__host__ __device__ constexpr size_t carve_bytes(int nmax) {
    auto r = [](size_t b) { return (b + 15) & ~(size_t)15; };
    return 2 * r(((size_t)nmax / 2 + 2) * sizeof(Node<IdxT>)) + 3 * r((size_t)nmax * 4) +
           2 * r((size_t)nmax * sizeof(IdxT)) + r(((size_t)nmax + 1) * sizeof(IdxT)) +
           4 * r((size_t)nmax * 2) + r((size_t)nmax);
}

struct FixedArgs {
    Soa32 in;
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
    uint8_t* big;                  // global slabs for the big-cell path
    int64_t big_stride;            // bytes per slab
    int nslabs;
};

// Shared per-workgroup bookkeeping (always in LDS).
struct Shared {
    Frame F;
    int cell;
    int nnodes[2];
    int cls_cnt[8], cls_base[8], cls_cur[8];
    int total_lanes;
    int nleaves, nmerged, out_total;
    int root_dec;
    uint32_t flags;
    int64_t red64[16 * 2];
    float redf[16 * 11];
    Sums redS[BLOCK / WAVE];
};

// q(a*b, G): the exact FP32 x FP32 product, rounded to nearest on the grid 2^-G.
VPM_DEV int64_t fixq(float a, float b, int G) {
    return __double2ll_rn(ldexp((double)a * (double)b, G));
}

template <typename IdxT>
VPM_DEV IdxT* idx_buf(const CellMem<IdxT>& M, int par) { return par ? M.idx1 : M.idx0; }

template <typename IdxT>
VPM_DEV int code_of(const CellMem<IdxT>& M, int k, int i) {
    switch (k) {
        case 0: return M.cp0[i];
        case 1: return M.cp1[i];
        case 2: return M.cp2[i];
        case 3: return M.cm0[i];
        case 4: return M.cm1[i];
        default: return M.cm2[i];
    }
}

template <typename IdxT>
VPM_DEV void add_particle(Sums& S, const CellMem<IdxT>& M, int i) {
    sums_add(S, M.om[i], M.cp0[i], M.cp1[i], M.cp2[i], M.cm0[i], M.cm1[i], M.cm2[i]);
}

// Schedule `m` items (lengths from len_of(item)) onto power-of-two lane groups, largest first.
// Writes the lane map (virtual lane -> item) and sets S.total_lanes.  All threads call.
template <typename IdxT, typename LenFn>
VPM_DEV void schedule(Shared& S, IdxT* lanemap, int m, LenFn len_of) {
    const int tid = threadIdx.x;
    if (tid < 8) { S.cls_cnt[tid] = 0; S.cls_cur[tid] = 0; }
    __syncthreads();
    for (int it = tid; it < m; it += BLOCK) {
        const int g = group_size_for(len_of(it));
        atomicAdd(&S.cls_cnt[__ffs(g) - 1], 1);
    }
    __syncthreads();
    if (tid == 0) {
        int b = 0;
        for (int c = 6; c >= 0; --c) { S.cls_base[c] = b; b += S.cls_cnt[c] << c; }
        S.total_lanes = b;
    }
    __syncthreads();
    for (int it = tid; it < m; it += BLOCK) {
        const int g = group_size_for(len_of(it));
        const int c = __ffs(g) - 1;
        const int r = atomicAdd(&S.cls_cur[c], 1);
        const int off = S.cls_base[c] + (r << c);
        for (int v = 0; v < g; ++v) lanemap[off + v] = (IdxT)it;
    }
    __syncthreads();
}

// Process one unfinished subset with a lane group: compaction, child sums, child decisions.
template <typename IdxT>
VPM_DEV void split_node(Shared& S, const CellMem<IdxT>& M, const FixedArgs& A, Node<IdxT> nd,
                        int cur, int lid, int g, int gbase, Node<IdxT>* next, int nxt) {
    const int start = nd.start, len = nd.len;
    const int k = nd.thr_axis & 7;
    const int thr = nd.thr_axis >> 3;
    const IdxT* src = idx_buf(M, cur);
    IdxT* dst = idx_buf(M, cur ^ 1);

    // pass 1: size of the lower side V1 = {c <= thr}
    int nl = 0;
    for (int j = lid; j < len; j += g) nl += code_of(M, k, src[start + j]) <= thr ? 1 : 0;
    nl = group_sum(nl, g);

    // pass 2: stable compaction into the other buffer (Step 6)
    const uint64_t below = lanes_below() >> gbase;
    int lb = 0, rb = 0;
    for (int j0 = 0; j0 < len; j0 += g) {
        const int j = j0 + lid;
        const bool act = j < len;
        IdxT i = 0;
        bool right = false;
        if (act) { i = src[start + j]; right = code_of(M, k, i) > thr; }
        const uint64_t bl = group_bits(__ballot(act && !right), gbase, g);
        const uint64_t br = group_bits(__ballot(act && right), gbase, g);
        if (act) {
            const int d = right ? nl + rb + __popcll(br & below) : lb + __popcll(bl & below);
            dst[start + d] = i;
        }
        lb += __popcll(bl);
        rb += __popcll(br);
    }
    wave_fence();

    const int n1 = nl, n2 = len - nl;
    int dv0, dv1;
    if (n1 == 0 || n2 == 0) {
        // Cannot happen with exact arithmetic (the chosen axis has V > 0); end the subset.
        Decision d; d.kind = D_MERGED; d.axis = 0; d.thr = 0; d.jdir = 0;
        if (lid == 0) atomicOr(&S.flags, FLAG_INTERNAL);
        dv0 = pack_decision(d);
        dv1 = -1;
    } else {
        Sums L, R;
        sums_zero(L); sums_zero(R);
        for (int j = lid; j < n1; j += g) add_particle(L, M, dst[start + j]);
        for (int j = lid; j < n2; j += g) add_particle(R, M, dst[start + n1 + j]);
        sums_group_reduce(L, g);
        sums_group_reduce(R, g);
        int mine = 0;
        if (g == 1) {
            dv0 = pack_decision(decide(L, n1, A.P, S.F));
            dv1 = pack_decision(decide(R, n2, A.P, S.F));
        } else {
            if (lid < 2) mine = pack_decision(decide(lid == 0 ? L : R, lid == 0 ? n1 : n2, A.P, S.F));
            dv0 = __shfl(mine, gbase);
            dv1 = __shfl(mine, gbase + 1);
        }
    }

    // record the children
    for (int ch = 0; ch < 2; ++ch) {
        const int dvv = ch == 0 ? dv0 : dv1;
        if (dvv == -1) continue;
        const Decision d = unpack_decision(dvv);
        const int cs = (dv1 == -1) ? start : (ch == 0 ? start : start + n1);
        const int cl = (dv1 == -1) ? len : (ch == 0 ? n1 : n2);
        if (d.kind == D_SPLIT) {
            if (lid == 0) {
                const int slot = atomicAdd(&S.nnodes[nxt], 1);
                Node<IdxT> c;
                c.start = (IdxT)cs; c.len = (IdxT)cl; c.thr_axis = (d.thr << 3) | d.axis;
                next[slot] = c;
            }
        } else {
            const uint8_t base = INF_SET | (uint8_t)((cur ^ 1) & 1) |
                                 (d.kind == D_MERGED ? INF_MERGED : 0) |
                                 (uint8_t)(d.jdir << INF_JSHIFT);
            for (int j = lid; j < cl; j += g) M.info[cs + j] = base | (j == 0 ? INF_HEAD : 0);
        }
    }
}

VPM_DEV int ceil_log2(int v) {
    int b = 0;
    while ((1 << b) < v) ++b;
    return b;
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
template <typename IdxT>
VPM_DEV void merge_leaf(const Shared& S, const CellMem<IdxT>& M, const FixedArgs& A, int64_t off,
                        int start, int len, int lid, int g) {
    const Frame& F = S.F;
    const uint8_t inf = M.info[start];
    const IdxT* src = idx_buf(M, inf & INF_PARITY);
    const int jdir = (inf >> INF_JSHIFT) & 3;
    const int gb = 62 - ceil_log2(len);          // |term| < 2^gb keeps the sum below 2^62

    // pass 1
    const int gw = gb - F.ew;
    const int g1x = gb - F.ew - F.ep[0], g1y = gb - F.ew - F.ep[1], g1z = gb - F.ew - F.ep[2];
    int64_t sw = 0, s1x = 0, s1y = 0, s1z = 0;
    for (int j = lid; j < len; j += g) {
        const int64_t i = off + src[start + j];
        const float w = A.in.w[i];
        sw += fixq(w, 1.0f, gw);
        s1x += fixq(w, A.in.px[i], g1x);
        s1y += fixq(w, A.in.py[i], g1y);
        s1z += fixq(w, A.in.pz[i], g1z);
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
    const float m = (float)A.P.mass;
    const float m2 = m * m;
    const float e0f = sqrtf(m2 + (q0 * q0 + q1 * q1 + q2 * q2));
    int64_t sx0 = 0, sx1 = 0, sx2 = 0, sd0 = 0, sd1 = 0, sd2 = 0, se = 0;
    for (int j = lid; j < len; j += g) {
        const int64_t i = off + src[start + j];
        const float w = A.in.w[i];
        const float x = A.in.x[i] - F.lo[0], y = A.in.y[i] - F.lo[1], z = A.in.z[i] - F.lo[2];
        const float px = A.in.px[i], py = A.in.py[i], pz = A.in.pz[i];
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
    const int64_t o = off + M.emit[start];
    if (A.P.merge_mode == VPM_MERGE_CENTROID) {
        A.tmp.w[o] = (float)W;
        A.tmp.x[o] = (float)X[0]; A.tmp.y[o] = (float)X[1]; A.tmp.z[o] = (float)X[2];
        A.tmp.px[o] = (float)Pm[0]; A.tmp.py[o] = (float)Pm[1]; A.tmp.pz[o] = (float)Pm[2];
        return;
    }
    const double md = A.P.mass;
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

VPM_DEV int frexp_exp(float v) {
    int e = 0;
    if (v > 0.0f) frexpf(v, &e);
    return e;
}

// ------------------------------------------------------------------------------------------
// The cell kernel.
// ------------------------------------------------------------------------------------------

template <int NMAX, typename IdxT, bool IN_LDS>
__global__ __launch_bounds__(BLOCK) void k_fixed_cells(FixedArgs A) {
    extern __shared__ __align__(16) uint8_t smem[];
    __shared__ Shared S;
    const int tid = threadIdx.x;

    CellMem<IdxT> M;
    if (IN_LDS) M = carve<IdxT>(smem, NMAX);
    else M = carve<IdxT>(A.big + (int64_t)blockIdx.x * A.big_stride, NMAX);

    for (;;) {
        __syncthreads();
        if (tid == 0) {
            const int qi = atomicAdd(&A.counters[A.work_index], 1);
            S.cell = qi < A.counters[A.qlen_index] ? A.queue[qi] : -1;
            S.flags = 0;
        }
        __syncthreads();
        const int c = S.cell;
        if (c < 0) break;
        const int64_t off = A.cell_off[c];
        const int n = (int)(A.cell_off[c + 1] - off);

        // ---- Step 1: collect the cell, validate, frame ----
        {
            float v[11];
            v[0] = 0.0f;
            for (int a = 0; a < 3; ++a) { v[1 + a] = INFINITY; v[4 + a] = -INFINITY; v[7 + a] = 0.0f; }
            float bad = 0.0f;
            for (int i = tid; i < n; i += BLOCK) {
                const float w = A.in.w[off + i];
                const float q[6] = {A.in.x[off + i], A.in.y[off + i], A.in.z[off + i],
                                    A.in.px[off + i], A.in.py[off + i], A.in.pz[off + i]};
                bool ok = w > 0.0f && isfinite(w);
                for (int l = 0; l < 6; ++l) ok = ok && isfinite(q[l]);
                if (!ok) bad = 1.0f;
                v[0] = fmaxf(v[0], w);
                for (int a = 0; a < 3; ++a) {
                    v[1 + a] = fminf(v[1 + a], q[a]);
                    v[4 + a] = fmaxf(v[4 + a], q[a]);
                    v[7 + a] = fmaxf(v[7 + a], fabsf(q[3 + a]));
                }
            }
            v[10] = bad;
            // workgroup max/min of the 11 values (min as max of negatives)
            for (int a = 1; a < 4; ++a) v[a] = -v[a];
            for (int r = 0; r < 11; ++r)
                for (int m = 1; m < WAVE; m <<= 1) v[r] = fmaxf(v[r], __shfl_xor(v[r], m));
            if (lane_id() == 0)
                for (int r = 0; r < 11; ++r) S.redf[(tid / WAVE) * 11 + r] = v[r];
            __syncthreads();
            if (tid == 0) {
                for (int w = 1; w < BLOCK / WAVE; ++w)
                    for (int r = 0; r < 11; ++r) v[r] = fmaxf(v[r], S.redf[w * 11 + r]);
                Frame& F = S.F;
                F.wmax = v[0];
                for (int a = 0; a < 3; ++a) { F.lo[a] = -v[1 + a]; F.hi[a] = v[4 + a]; F.pmax[a] = v[7 + a]; }
                F.bad = v[10] != 0.0f;
                F.ew = frexp_exp(F.wmax);
                for (int a = 0; a < 3; ++a) {
                    F.pzero[a] = F.pmax[a] == 0.0f;
                    F.ep[a] = frexp_exp(F.pmax[a]);
                    F.ext_e[a] = frexp_exp(F.hi[a] - F.lo[a]);
                }
                // |eps_i - eps_j| <= m + |p|_1 for any two particles of the cell; 4x margin
                F.eb = frexp_exp(4.0f * ((float)A.P.mass + F.pmax[0] + F.pmax[1] + F.pmax[2]));
                S.nnodes[0] = 0; S.nnodes[1] = 0;
            }
            __syncthreads();
        }
        if (S.F.bad) {
            if (tid == 0) {
                atomicOr(A.flags, FLAG_BAD_VALUE);
                if (A.mode == 0) { A.out_count[c] = n; A.cell_mode[c] = CELL_UNTOUCHED; }
                else A.n_subsets[c] = 0;
            }
            if (A.mode == 1)
                for (int i = tid; i < n; i += BLOCK) { A.perm[off + i] = (int32_t)(off + i); A.subset_id[off + i] = -1; }
            continue;
        }

        // ---- codes and the root's moments ----
        {
            const Frame& F = S.F;
            Sums R;
            sums_zero(R);
            bool oob = false;
            for (int i = tid; i < n; i += BLOCK) {
                const float w = A.in.w[off + i];
                const uint32_t om = (uint32_t)rintf(ldexpf(w, 15 - F.ew));
                int cp[3], cm[3];
                const float x[3] = {A.in.x[off + i], A.in.y[off + i], A.in.z[off + i]};
                const float p[3] = {A.in.px[off + i], A.in.py[off + i], A.in.pz[off + i]};
                for (int a = 0; a < 3; ++a) {
                    const float d = x[a] - F.lo[a];
                    float r = rintf(d * A.P.s[a]);
                    if (r > 65536.0f) oob = true;
                    r = fminf(r, 65535.0f);
                    cp[a] = (int)r - 32768;
                    cm[a] = F.pzero[a] ? 0 : (int)rintf(ldexpf(p[a], 22 - F.ep[a]));
                }
                M.om[i] = (uint16_t)om;
                M.cp0[i] = (int16_t)cp[0]; M.cp1[i] = (int16_t)cp[1]; M.cp2[i] = (int16_t)cp[2];
                M.cm0[i] = cm[0]; M.cm1[i] = cm[1]; M.cm2[i] = cm[2];
                M.idx0[i] = (IdxT)i;
                sums_add(R, om, cp[0], cp[1], cp[2], cm[0], cm[1], cm[2]);
            }
            if (oob) atomicOr(&S.flags, FLAG_OUT_OF_CELL);
            sums_group_reduce(R, WAVE);
            if (lane_id() == 0) S.redS[tid / WAVE] = R;
            __syncthreads();
            if (tid == 0) {
                for (int w = 1; w < BLOCK / WAVE; ++w) sums_merge(R, S.redS[w]);
                const Decision d = decide(R, n, A.P, S.F);
                S.root_dec = pack_decision(d);
                if (d.kind == D_SPLIT) {
                    Node<IdxT> nd;
                    nd.start = 0; nd.len = (IdxT)n; nd.thr_axis = (d.thr << 3) | d.axis;
                    M.nodes0[0] = nd;
                    S.nnodes[0] = 1;
                }
            }
            __syncthreads();
            const Decision d = unpack_decision(S.root_dec);
            if (d.kind != D_SPLIT) {
                const uint8_t base = INF_SET | (d.kind == D_MERGED ? INF_MERGED : 0) |
                                     (uint8_t)(d.jdir << INF_JSHIFT);
                for (int i = tid; i < n; i += BLOCK) M.info[i] = base | (i == 0 ? INF_HEAD : 0);
            }
            __syncthreads();
        }

        // ---- Steps 2-6, level by level ----
        int cur = 0;
        while (S.nnodes[cur] > 0) {
            const int m = S.nnodes[cur];
            Node<IdxT>* curl = cur ? M.nodes1 : M.nodes0;
            Node<IdxT>* nextl = cur ? M.nodes0 : M.nodes1;
            if (tid == 0) S.nnodes[cur ^ 1] = 0;
            schedule<IdxT>(S, M.emit, m, [&](int it) { return (int)curl[it].len; });
            const int total = S.total_lanes;
            for (int r0 = 0; r0 < total; r0 += BLOCK) {
                const int v = r0 + tid;
                if (v < total) {
                    const int it = M.emit[v];
                    const Node<IdxT> nd = curl[it];
                    const int g = group_size_for((int)nd.len);
                    const int lid = v & (g - 1);
                    const int gbase = lane_id() & ~(g - 1);
                    split_node<IdxT>(S, M, A, nd, cur, lid, g, gbase, nextl, cur ^ 1);
                }
            }
            __syncthreads();
            cur ^= 1;
        }

        // ---- output ----
        // per slot: leaf ordinal and output slot, by one scan over the cell's slots
        const int per = (n + BLOCK - 1) / BLOCK;
        const int b0 = min(n, tid * per), b1 = min(n, b0 + per);
        const int npair = A.P.merge_mode == VPM_MERGE_PAIR ? 2 : 1;
        int64_t loc = 0;
        for (int p = b0; p < b1; ++p) {
            const uint8_t inf = M.info[p];
            const int e = (inf & INF_MERGED) ? ((inf & INF_HEAD) ? npair : 0) : 1;
            loc += ((int64_t)((inf & INF_HEAD) ? 1 : 0) << 32) | (int64_t)e;
        }
        int64_t tot;
        int64_t pre = block_exclusive_scan<BLOCK>(loc, S.red64, &tot);
        const int nleaves = (int)(tot >> 32);
        const int out_total = (int)(tot & 0xffffffff);
        // the node lists and the momentum codes are free now
        IdxT* leaf_start = (IdxT*)M.nodes0;                // first slot of each final subset
        IdxT* mlist = (IdxT*)M.nodes1;                     // ordinals of the merged subsets
        IdxT* lanemap = (IdxT*)M.cm0;
        if (tid == 0) { S.nmerged = 0; }
        __syncthreads();
        for (int p = b0; p < b1; ++p) {
            const uint8_t inf = M.info[p];
            const int e = (inf & INF_MERGED) ? ((inf & INF_HEAD) ? npair : 0) : 1;
            const int ord = (int)(pre >> 32) + ((inf & INF_HEAD) ? 1 : 0) - 1;
            if (A.mode == 0) {
                M.emit[p] = (IdxT)(pre & 0xffffffff);
            } else {
                A.perm[off + p] = (int32_t)(off + idx_buf(M, inf & INF_PARITY)[p]);
                A.subset_id[off + p] = ord;
            }
            if (inf & INF_HEAD) {
                leaf_start[ord] = (IdxT)p;
                if ((inf & INF_MERGED) && A.mode == 0) {
                    const int s = atomicAdd(&S.nmerged, 1);
                    mlist[s] = (IdxT)ord;
                }
            }
            pre += ((int64_t)((inf & INF_HEAD) ? 1 : 0) << 32) | (int64_t)e;
        }
        if (tid == 0) leaf_start[nleaves] = (IdxT)n;
        __syncthreads();
        if (A.mode == 1) {
            if (tid == 0) {
                A.n_subsets[c] = nleaves;
                if (S.flags) atomicOr(A.flags, S.flags);
            }
            continue;
        }
        // copied particles (subsets below min_subset)
        for (int p = tid; p < n; p += BLOCK) {
            const uint8_t inf = M.info[p];
            if (inf & INF_MERGED) continue;
            const int64_t i = off + idx_buf(M, inf & INF_PARITY)[p];
            const int64_t o = off + M.emit[p];
            A.tmp.x[o] = A.in.x[i]; A.tmp.y[o] = A.in.y[i]; A.tmp.z[o] = A.in.z[i];
            A.tmp.px[o] = A.in.px[i]; A.tmp.py[o] = A.in.py[i]; A.tmp.pz[o] = A.in.pz[i];
            A.tmp.w[o] = A.in.w[i];
        }
        // merged subsets (Step 7)
        const int nm = S.nmerged;
        if (nm > 0) {
            schedule<IdxT>(S, lanemap, nm, [&](int it) {
                const int ord = mlist[it];
                return (int)(leaf_start[ord + 1] - leaf_start[ord]);
            });
            const int total = S.total_lanes;
            for (int r0 = 0; r0 < total; r0 += BLOCK) {
                const int v = r0 + tid;
                if (v < total) {
                    const int ord = mlist[lanemap[v]];
                    const int st = leaf_start[ord];
                    const int ln = leaf_start[ord + 1] - st;
                    const int g = group_size_for(ln);
                    merge_leaf<IdxT>(S, M, A, off, st, ln, v & (g - 1), g);
                }
            }
        }
        if (tid == 0) {
            A.out_count[c] = out_total;
            A.cell_mode[c] = CELL_PROCESSED;
            if (S.flags) atomicOr(A.flags, S.flags);
        }
    }
}

}  // namespace

int fixed_lds_bytes(int nmax) {
    return (int)(nmax <= NMAX_A ? carve_bytes<uint16_t>(NMAX_A) : carve_bytes<uint16_t>(NMAX_B));
}

int64_t fixed_big_slab_bytes() { return (int64_t)carve_bytes<uint32_t>(NMAX_BIG); }

const void* fixed_kernel_ptr(int which) {
    if (which == 0) return (const void*)k_fixed_cells<NMAX_A, uint16_t, true>;
    if (which == 1) return (const void*)k_fixed_cells<NMAX_B, uint16_t, true>;
    return (const void*)k_fixed_cells<NMAX_BIG, uint32_t, false>;
}

hipError_t launch_fixed_cells(const Workspace& ws, const LaunchCfg& lc, const Soa32& in,
                              const int64_t* cell_off, const FixedParams& fp, int mode,
                              int32_t* perm, int32_t* subset_id, int32_t* n_subsets) {
    FixedArgs A;
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
    A.big = ws.big;
    A.big_stride = fixed_big_slab_bytes();
    A.nslabs = lc.grid_big;

    struct Bin { int q; const void* fn; int grid; size_t lds; const char* name; };
    const Bin bins[3] = {
        {Q_BIG, fixed_kernel_ptr(2), lc.grid_big, 0, "fixed_cells_big"},
        {Q_B, fixed_kernel_ptr(1), lc.grid_b, carve_bytes<uint16_t>(NMAX_B), "fixed_cells_4096"},
        {Q_A, fixed_kernel_ptr(0), lc.grid_a, carve_bytes<uint16_t>(NMAX_A), "fixed_cells_1024"},
    };
    for (const Bin& b : bins) {
        A.queue = ws.queue[b.q];
        A.qlen_index = b.q;
        A.work_index = 8 + b.q;
        if (lc.pre) lc.pre(lc.prof, b.name, lc.stream);
        if (b.q == Q_A)
            hipLaunchKernelGGL((k_fixed_cells<NMAX_A, uint16_t, true>), dim3(b.grid), dim3(BLOCK), b.lds, lc.stream, A);
        else if (b.q == Q_B)
            hipLaunchKernelGGL((k_fixed_cells<NMAX_B, uint16_t, true>), dim3(b.grid), dim3(BLOCK), b.lds, lc.stream, A);
        else
            hipLaunchKernelGGL((k_fixed_cells<NMAX_BIG, uint32_t, false>), dim3(b.grid), dim3(BLOCK), 0, lc.stream, A);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        if (lc.post) lc.post(lc.prof, b.name, lc.stream);
    }
    return hipSuccess;
}

}  // namespace vpm

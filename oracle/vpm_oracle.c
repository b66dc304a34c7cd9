/*
 * vpm_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, obviously-correct CPU implementation of the Voronoi
 * particle-merging algorithm of Luu, Tueckmantel and Pukhov ("Voronoi
 * Particle Merging Algorithm for PIC Codes", Sec. "Algorithm", Steps 1-7).
 * It exists to check the GPU library.  Only the test-suite, the smoke check
 * and the benchmark's CPU-baseline leg may load it; the product path never
 * does.  It shares no code, header or table with the GPU library.
 *
 * What it computes, per simulation cell (Sec. "Algorithm"):
 *   - a cell with N <= N_min particles is left untouched (the "Input" rule);
 *   - otherwise the cell's particles form the first Voronoi subset V0 (Step 1);
 *   - for a subset: weighted centroid and per-axis standard deviation (Steps 1-2),
 *     coefficients of variation Delta_X = sigma/L, Delta_P = sigma/|P| (Eqs. cv_x, cv_p),
 *     stop when all six are <= tolerance (Step 3), else cut through the centroid
 *     perpendicular to the axis of largest CV (Steps 4-5), q <= Q to V1, q > Q to V2,
 *     and repeat on V1 then V2 (Step 6);
 *   - every finished subset is replaced by its centroid (Step 7) or, in the
 *     energy-conserving variant the paper suggests in its remarks on the
 *     algorithm, by two particles of half the weight.
 *
 * Two decision modes:
 *   PAPER  the real-valued statistics exactly as the paper writes them, in
 *          IEEE double, summed sequentially in the subset's stable order.
 *   FIXED  the same recursion, but every decision is an exact integer function
 *          of per-cell fixed-point codes (weights 2^-15 of the cell maximum,
 *          positions 2^-16 of the cell length, momenta 2^-22 of the cell's
 *          largest |p| per axis), so that the partition does not depend on
 *          summation order.  Inputs are first rounded to FP32.
 *
 * Readings of the paper taken here (where it is silent or ambiguous):
 *   L in Delta_X is the simulation-cell side length, fixed for the cell;
 *   Delta_P divides by |P| (0/0 := 0; sigma > 0 with P = 0 gives +infinity);
 *   argmax over the six raw CVs, ties to the lowest axis (x,y,z,px,py,pz) -- or, as an option,
 *   over each CV divided by its tolerance (a CV > 0 over a zero tolerance counts as infinite);
 *   subsets with fewer than min_subset particles are final and passed through;
 *   a cut that leaves one side empty (possible only through rounding) ends the
 *   subset as finished;  energy of a particle is sqrt(m^2 + |p|^2).
 *
 * The merge is computed in long double with compensated sums.  The pair
 * direction is perpendicular to the mean momentum, built from the unit axis
 * e_j with the smallest |mean momentum| component.
 *
 * Parity status: the FIXED and PAPER partitions and both merges are pinned by
 * the tests in tests/test_oracle_pins.py (conservation identities, CV bound,
 * duplicate classes at zero tolerance, single-subset limit against a library
 * weighted average, 1-D bisection, separated beams, invariances, hand-worked
 * golden cells).  The paper's printed simulation results are not reproducible
 * here (they need a PIC code); that comparison is unpinned.
 */
#include <float.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef __int128 i128;
typedef unsigned __int128 u128;

/* ---------------------------------------------------------------- interface */

enum { ORC_PAIR = 0, ORC_CENTROID = 1 };
enum { ORC_FIXED = 0, ORC_PAPER = 1 };

enum {
    ORC_FLAG_BAD_VALUE = 1u << 0,   /* w <= 0, NaN or Inf in the cell: cell untouched */
    ORC_FLAG_OUT_OF_CELL = 1u << 1, /* a position code had to be clamped (FIXED)       */
    ORC_FLAG_TOO_LARGE = 1u << 2,   /* more particles than the mode's largest cell: untouched */
};

/* Largest cell processed.  The method's first subset V0 may be the whole simulation box (the
 * paper's remark after the algorithm on merging globally), so FIXED mode takes cells of up to
 * 2^24 particles: its integer moments stay exact there (S0 <= 2^39, |S1| <= 2^61, S2 <= 2^83; V
 * below 2^123 in 128 bits, the products of Steps 3-4 below 2^256 and 2^320).  PAPER mode, checked against the plain FP64
 * GPU form, keeps that form's limit of 2^16. */
#define ORC_NMAX_FIXED (1 << 24)
#define ORC_NMAX_PAPER 65536

typedef struct {
    double tol_x, tol_p;       /* T_X, T_P */
    int32_t n_min_cell;        /* N_min: a cell is processed only if N > N_min */
    int32_t min_subset;        /* subsets smaller than this are passed through */
    double cell_len[3];        /* L_x, L_y, L_z */
    double mass;               /* particle mass in m_e units (0 for photons) */
    int32_t merge_mode;        /* ORC_PAIR or ORC_CENTROID */
    int32_t decide;            /* ORC_FIXED or ORC_PAPER */
    int32_t axis_rule;         /* 0: Step 4 on the raw CVs; 1: on each CV over its tolerance */
} orc_params;

typedef struct {
    int32_t n_nodes;           /* subsets visited (internal + final) */
    int32_t n_leaves;          /* final subsets */
    int32_t n_merged;          /* final subsets that were merged */
    int32_t max_depth;         /* deepest final subset (root = 0) */
    int64_t particle_levels;   /* sum over particles of the depth of their final subset */
    double min_margin;         /* PAPER: smallest relative decision margin seen; FIXED: +inf */
    uint32_t flags;
    int32_t n_out;
} orc_cell_stats;

/* ------------------------------------------------------- small big integers */

typedef struct { uint64_t v[4]; } u256; /* little-endian limbs */

static u256 u256_mul(u128 a, u128 b) {
    uint64_t al[2] = {(uint64_t)a, (uint64_t)(a >> 64)};
    uint64_t bl[2] = {(uint64_t)b, (uint64_t)(b >> 64)};
    u256 r; memset(&r, 0, sizeof r);
    for (int i = 0; i < 2; ++i) {
        u128 carry = 0;
        for (int j = 0; j < 2; ++j) {
            u128 t = (u128)al[i] * bl[j] + r.v[i + j] + carry;
            r.v[i + j] = (uint64_t)t;
            carry = t >> 64;
        }
        int k = i + 2;
        while (carry) {
            u128 t = (u128)r.v[k] + carry;
            r.v[k] = (uint64_t)t;
            carry = t >> 64;
            ++k;
        }
    }
    return r;
}

static int u256_cmp(u256 a, u256 b) {
    for (int i = 3; i >= 0; --i) {
        if (a.v[i] < b.v[i]) return -1;
        if (a.v[i] > b.v[i]) return 1;
    }
    return 0;
}

/* a 256-bit value times a 64-bit one (five limbs, enough for the normalised comparison) */
typedef struct { uint64_t v[5]; } u320;

static u320 u320_mul(u256 a, uint64_t b) {
    u320 r;
    u128 carry = 0;
    for (int i = 0; i < 4; ++i) {
        u128 t = (u128)a.v[i] * b + carry;
        r.v[i] = (uint64_t)t;
        carry = t >> 64;
    }
    r.v[4] = (uint64_t)carry;
    return r;
}

static int u320_cmp(u320 a, u320 b) {
    for (int i = 4; i >= 0; --i) {
        if (a.v[i] < b.v[i]) return -1;
        if (a.v[i] > b.v[i]) return 1;
    }
    return 0;
}

/* -------------------------------------------------------- per-cell scratch */

typedef struct {
    int n;
    const orc_params *p;
    double *q[6];              /* x, y, z, px, py, pz as used by decisions and merge */
    double *w;
    /* FIXED-mode integer codes */
    int64_t *om;               /* weight codes, 0 .. 2^15 */
    int64_t *c[6];             /* position codes -2^15..2^15-1, momentum codes -2^22..2^22 */
    int mexp[3];               /* frexp exponent of the cell's largest |p| per axis */
    int mzero[3];              /* that largest |p| is zero */
    /* outputs for this cell */
    int *perm;                 /* cell-local particle index, final-subset order */
    int *sid;                  /* final subset ordinal per perm slot */
    int n_perm;
    double *out[7];            /* merged particles, cell-local */
    int n_out;
    orc_cell_stats st;
} cell_ctx;

/* ------------------------------------------------------------------ merge */

/* Neumaier-compensated long double accumulator */
typedef struct { long double s, c; } kacc;
static void kadd(kacc *a, long double x) {
    long double t = a->s + x;
    if (fabsl(a->s) >= fabsl(x)) a->c += (a->s - t) + x;
    else a->c += (x - t) + a->s;
    a->s = t;
}
static long double kval(const kacc *a) { return a->s + a->c; }

/* Replace subset `mem[0..cnt)` by its centroid (Step 7) or by an energy-
 * conserving pair.  `jdir` is the axis whose unit vector seeds the pair
 * direction (smallest |mean momentum| component).                        */
static void merge_subset(cell_ctx *cc, const int *mem, int cnt, int jdir) {
    const double m = cc->p->mass;
    kacc W = {0, 0}, WX[3] = {{0, 0}}, WP[3] = {{0, 0}};
    for (int t = 0; t < cnt; ++t) {
        int i = mem[t];
        long double wi = cc->w[i];
        kadd(&W, wi);
        for (int a = 0; a < 3; ++a) {
            kadd(&WX[a], wi * (long double)cc->q[a][i]);
            kadd(&WP[a], wi * (long double)cc->q[3 + a][i]);
        }
    }
    long double Wt = kval(&W), X[3], P[3];
    for (int a = 0; a < 3; ++a) { X[a] = kval(&WX[a]) / Wt; P[a] = kval(&WP[a]) / Wt; }

    long double P2 = P[0] * P[0] + P[1] * P[1] + P[2] * P[2];
    long double e0 = sqrtl((long double)m * m + P2);
    /* A = mean energy minus e0, from deviations: eps_i - e0 = (p_i-P).(p_i+P)/(eps_i+e0) */
    kacc A = {0, 0};
    for (int t = 0; t < cnt; ++t) {
        int i = mem[t];
        long double pp = 0, num = 0;
        for (int a = 0; a < 3; ++a) {
            long double pa = cc->q[3 + a][i];
            pp += pa * pa;
            num += (pa - P[a]) * (pa + P[a]);
        }
        long double ei = sqrtl((long double)m * m + pp);
        long double den = ei + e0;
        if (den > 0) kadd(&A, (long double)cc->w[i] * num / den);
    }
    long double Am = kval(&A) / Wt;
    long double r = Am * (Am + 2 * e0);          /* mean-energy^2 - m^2 - |P|^2 */
    if (r < 0) r = 0;

    int o = cc->n_out;
    if (cc->p->merge_mode == ORC_CENTROID) {
        cc->out[6][o] = (double)Wt;
        for (int a = 0; a < 3; ++a) { cc->out[a][o] = (double)X[a]; cc->out[3 + a][o] = (double)P[a]; }
        cc->n_out = o + 1;
        return;
    }
    /* u = e_j - (e_j . Phat) Phat, delta = sqrt(r) u/|u| */
    long double u[3] = {0, 0, 0};
    u[jdir] = 1;
    if (P2 > 0) for (int a = 0; a < 3; ++a) u[a] -= P[jdir] * P[a] / P2;
    long double un = sqrtl(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
    long double s = sqrtl(r) / un;
    for (int k = 0; k < 2; ++k) {
        long double sg = k == 0 ? 1 : -1;
        cc->out[6][o + k] = (double)(Wt / 2);
        for (int a = 0; a < 3; ++a) {
            cc->out[a][o + k] = (double)X[a];
            cc->out[3 + a][o + k] = (double)(P[a] + sg * s * u[a]);
        }
    }
    cc->n_out = o + 2;
}

static void passthrough_subset(cell_ctx *cc, const int *mem, int cnt) {
    for (int t = 0; t < cnt; ++t) {
        int i = mem[t], o = cc->n_out++;
        for (int a = 0; a < 6; ++a) cc->out[a][o] = cc->q[a][i];
        cc->out[6][o] = cc->w[i];
    }
}

static void record_leaf(cell_ctx *cc, const int *mem, int cnt, int depth, int merged, int jdir) {
    int id = cc->st.n_leaves++;
    for (int t = 0; t < cnt; ++t) { cc->perm[cc->n_perm] = mem[t]; cc->sid[cc->n_perm] = id; cc->n_perm++; }
    if (depth > cc->st.max_depth) cc->st.max_depth = depth;
    cc->st.particle_levels += (int64_t)cnt * depth;
    if (merged) { cc->st.n_merged++; merge_subset(cc, mem, cnt, jdir); }
    else passthrough_subset(cc, mem, cnt);
}

/* ------------------------------------------------------ FIXED-mode frame */

/* Per-cell integer codes.  Returns 0, or flags. */
static uint32_t fixed_codes(cell_ctx *cc) {
    const int n = cc->n;
    uint32_t flags = 0;
    float wmax = 0.0f;
    for (int i = 0; i < n; ++i) if ((float)cc->w[i] > wmax) wmax = (float)cc->w[i];
    int ew;
    frexpf(wmax, &ew);                                  /* wmax in [2^(ew-1), 2^ew) */
    for (int i = 0; i < n; ++i) cc->om[i] = (int64_t)rintf(ldexpf((float)cc->w[i], 15 - ew));

    for (int a = 0; a < 3; ++a) {                       /* positions */
        float lo = (float)cc->q[a][0];
        for (int i = 1; i < n; ++i) if ((float)cc->q[a][i] < lo) lo = (float)cc->q[a][i];
        float s = (float)(65536.0 / cc->p->cell_len[a]);
        for (int i = 0; i < n; ++i) {
            float d = (float)cc->q[a][i] - lo;          /* FP32, round to nearest even */
            float t = d * s;                            /* FP32, no contraction */
            float r = rintf(t);
            if (r > 65536.0f) flags |= ORC_FLAG_OUT_OF_CELL;
            if (r > 65535.0f) r = 65535.0f;
            cc->c[a][i] = (int64_t)r - 32768;
        }
    }
    for (int a = 0; a < 3; ++a) {                       /* momenta */
        float mx = 0.0f;
        for (int i = 0; i < n; ++i) { float v = fabsf((float)cc->q[3 + a][i]); if (v > mx) mx = v; }
        cc->mzero[a] = (mx == 0.0f);
        int e = 0;
        if (mx > 0.0f) frexpf(mx, &e);
        cc->mexp[a] = e;
        for (int i = 0; i < n; ++i)
            cc->c[3 + a][i] = mx > 0.0f ? (int64_t)rintf(ldexpf((float)cc->q[3 + a][i], 22 - e)) : 0;
    }
    return flags;
}

typedef struct { int64_t s0; int64_t s1[6]; i128 s2[6]; } isums;

static isums fixed_sums(const cell_ctx *cc, const int *mem, int cnt) {
    isums S; memset(&S, 0, sizeof S);
    for (int t = 0; t < cnt; ++t) {
        int i = mem[t];
        int64_t om = cc->om[i];
        S.s0 += om;
        for (int l = 0; l < 6; ++l) {
            int64_t c = cc->c[l][i];
            S.s1[l] += om * c;
            S.s2[l] += (i128)om * c * c;
        }
    }
    return S;
}

/* Delta_l^2 as the fraction num/den (den == 0 with num > 0 means +infinity). */
typedef struct { u128 num, den; } frac;

static frac fixed_delta2(const isums *S, int l) {
    frac f;
    i128 V = (i128)S->s0 * S->s2[l] - (i128)S->s1[l] * S->s1[l];   /* >= 0 */
    f.num = (u128)V;
    if (l < 3) f.den = ((u128)S->s0 * (u128)S->s0) << 32;           /* (2^16 S0)^2 */
    else f.den = (u128)((i128)S->s1[l] * S->s1[l]);
    if (f.num == 0) f.den = 1;                                       /* 0/0 := 0 */
    return f;
}

static int frac_gt(frac a, frac b) {          /* a > b ? */
    int ainf = a.den == 0, binf = b.den == 0;
    if (ainf) return !binf;
    if (binf) return 0;
    return u256_cmp(u256_mul(a.num, b.den), u256_mul(b.num, a.den)) > 0;
}

/* Step 4 with each CV over its tolerance: is Delta_a^2 / Ta^2 > Delta_b^2 / Tb^2 ?  With Delta^2 =
 * V / D and T^2 = T2 / 2^48 this compares V_a D_b T2_b with V_b D_a T2_a (< 2^320).  A zero D or a
 * zero T2 under V > 0 is infinite; V = 0 is 0. */
static int frac_gt_norm(frac a, uint64_t t2a, frac b, uint64_t t2b) {
    int az = a.num == 0, bz = b.num == 0;
    if (az) return 0;
    if (bz) return 1;
    int ainf = a.den == 0 || t2a == 0, binf = b.den == 0 || t2b == 0;
    if (ainf) return !binf;
    if (binf) return 0;
    return u320_cmp(u320_mul(u256_mul(a.num, b.den), t2b), u320_mul(u256_mul(b.num, a.den), t2a)) > 0;
}

/* Step 3 in integers: Delta^2 <= (T^2).  T = That / 2^24.
 *   position: V/(2^32 S0^2) <= That^2/2^48   <=>  V*2^16 <= That^2 S0^2
 *   momentum: V/S1^2        <= That^2/2^48   <=>  V*2^48 <= That^2 S1^2 */
static int fixed_within(const isums *S, int l, u128 That) {
    frac f = fixed_delta2(S, l);
    if (f.num == 0) return 1;
    if (f.den == 0) return 0;
    u256 lhs = u256_mul(f.num, (u128)1 << (l < 3 ? 16 : 48));
    u256 rhs = u256_mul(That * That, l < 3 ? (u128)S->s0 * (u128)S->s0 : f.den);
    return u256_cmp(lhs, rhs) <= 0;
}

/* pair-direction axis from the exact momentum code sums: argmin |S1_a| 2^e_a */
static int fixed_jdir(const cell_ctx *cc, const isums *S) {
    int best = 0;
    long double bv = 0;
    for (int a = 0; a < 3; ++a) {
        long double v = cc->mzero[a] ? 0.0L : ldexpl(fabsl((long double)S->s1[3 + a]), cc->mexp[a]);
        if (a == 0 || v < bv) { bv = v; best = a; }
    }
    return best;
}

/* ------------------------------------------------------ PAPER-mode stats */

static void margin_update(cell_ctx *cc, double m) { if (m < cc->st.min_margin) cc->st.min_margin = m; }

/* ------------------------------------------------------------- recursion */

typedef struct { int *mem; int cnt; int depth; } node_t;

static void run_cell(cell_ctx *cc) {
    const orc_params *p = cc->p;
    const int n = cc->n;
    u128 Tx = 0, Tp = 0;
    if (p->decide == ORC_FIXED) {
        cc->st.flags |= fixed_codes(cc);
        Tx = (u128)(uint64_t)llrint(p->tol_x * 16777216.0);
        Tp = (u128)(uint64_t)llrint(p->tol_p * 16777216.0);
    }
    node_t *stack = (node_t *)malloc(sizeof(node_t) * (size_t)(n + 2));
    int sp = 0;
    int *root = (int *)malloc(sizeof(int) * (size_t)n);
    for (int i = 0; i < n; ++i) root[i] = i;
    stack[sp++] = (node_t){root, n, 0};

    while (sp > 0) {
        node_t nd = stack[--sp];
        cc->st.n_nodes++;
        int *mem = nd.mem, cnt = nd.cnt;
        if (cnt < p->min_subset) { record_leaf(cc, mem, cnt, nd.depth, 0, 0); free(mem); continue; }

        int split = 0, k = 0, jdir = 0;
        int *v1 = NULL, *v2 = NULL, n1 = 0, n2 = 0;
        if (p->decide == ORC_FIXED) {
            isums S = fixed_sums(cc, mem, cnt);
            jdir = fixed_jdir(cc, &S);
            if (S.s0 > 0) {
                int done = 1;
                for (int l = 0; l < 6; ++l) done &= fixed_within(&S, l, l < 3 ? Tx : Tp);
                if (!done) {
                    frac best = fixed_delta2(&S, 0);
                    const uint64_t tx2 = (uint64_t)(Tx * Tx), tp2 = (uint64_t)(Tp * Tp);
                    for (int l = 1; l < 6; ++l) {
                        frac f = fixed_delta2(&S, l);
                        int gt = p->axis_rule ? frac_gt_norm(f, l < 3 ? tx2 : tp2, best, k < 3 ? tx2 : tp2)
                                              : frac_gt(f, best);
                        if (gt) { best = f; k = l; }
                    }
                    split = 1;
                    v1 = (int *)malloc(sizeof(int) * (size_t)cnt);
                    v2 = (int *)malloc(sizeof(int) * (size_t)cnt);
                    for (int t = 0; t < cnt; ++t) {
                        int i = mem[t];
                        /* q <= Q  <=>  c * S0 <= S1 */
                        if ((i128)cc->c[k][i] * S.s0 <= (i128)S.s1[k]) v1[n1++] = i; else v2[n2++] = i;
                    }
                }
            }
        } else {
            /* Step 1/5: W and centroid; Step 2: sigma about the centroid */
            double W = 0, mean[6] = {0}, var[6] = {0}, amax[6] = {0};
            for (int t = 0; t < cnt; ++t) W += cc->w[mem[t]];
            for (int l = 0; l < 6; ++l) {
                double s = 0;
                for (int t = 0; t < cnt; ++t) {
                    int i = mem[t];
                    s += cc->w[i] * cc->q[l][i];
                    if (fabs(cc->q[l][i]) > amax[l]) amax[l] = fabs(cc->q[l][i]);
                }
                mean[l] = s / W;
            }
            for (int l = 0; l < 6; ++l) {
                double s = 0;
                for (int t = 0; t < cnt; ++t) {
                    int i = mem[t];
                    double d = cc->q[l][i] - mean[l];
                    s += cc->w[i] * d * d;
                }
                var[l] = s / W;
            }
            /* pair direction: smallest |sum w p_a| in double */
            {
                double bv = 0;
                for (int a = 0; a < 3; ++a) {
                    double v = fabs(mean[3 + a] * W);
                    if (a == 0 || v < bv) { bv = v; jdir = a; }
                    for (int b = 0; b < a; ++b) {
                        double u = fabs(mean[3 + b] * W), mx = fmax(u, v);
                        if (mx > 0) margin_update(cc, fabs(u - v) / mx);
                    }
                }
            }
            /* Eqs. cv_x, cv_p */
            double D[6];
            for (int l = 0; l < 6; ++l) {
                double sig = sqrt(var[l]);
                if (l < 3) D[l] = sig / p->cell_len[l];
                else {
                    double P = fabs(mean[l]);
                    if (P == 0) D[l] = sig == 0 ? 0 : INFINITY;
                    else D[l] = sig / P;
                    /* a mean lost in rounding noise makes the CV order-dependent */
                    if (P <= 1e-12 * amax[l] && sig > 0) margin_update(cc, 0.0);
                }
            }
            int done = 1;
            for (int l = 0; l < 6; ++l) {
                double T = l < 3 ? p->tol_x : p->tol_p;
                if (!(D[l] <= T)) done = 0;
                if (isfinite(D[l])) margin_update(cc, T > 0 ? fabs(D[l] - T) / T : fabs(D[l]));
            }
            if (!done) {
                /* Step 4 on the raw CVs, or on each CV over its tolerance (then a CV > 0 over a
                 * zero tolerance is infinite) */
                double R[6];
                for (int l = 0; l < 6; ++l) {
                    double T = l < 3 ? p->tol_x : p->tol_p;
                    R[l] = !p->axis_rule ? D[l] : (T > 0 ? D[l] / T : (D[l] > 0 ? INFINITY : 0.0));
                }
                k = 0;
                for (int l = 1; l < 6; ++l) if (R[l] > R[k]) k = l;
                double second = -1;
                for (int l = 0; l < 6; ++l) if (l != k && R[l] > second) second = R[l];
                if (isinf(R[k])) margin_update(cc, isinf(second) ? 0.0 : 1.0);
                else if (R[k] > 0) margin_update(cc, (R[k] - second) / R[k]);
                split = 1;
                v1 = (int *)malloc(sizeof(int) * (size_t)cnt);
                v2 = (int *)malloc(sizeof(int) * (size_t)cnt);
                double Q = mean[k], scale = amax[k];
                for (int t = 0; t < cnt; ++t) {
                    int i = mem[t];
                    double q = cc->q[k][i];
                    if (q <= Q) v1[n1++] = i; else v2[n2++] = i;
                    if (scale > 0) margin_update(cc, fabs(q - Q) / scale);
                }
                if (n1 == 0 || n2 == 0) {           /* empty side: rounding only */
                    margin_update(cc, 0.0);
                    free(v1); free(v2); v1 = v2 = NULL;
                    split = 0;
                }
            }
        }
        if (!split) { record_leaf(cc, mem, cnt, nd.depth, 1, jdir); free(mem); continue; }
        free(mem);
        (void)n;
        stack[sp++] = (node_t){v2, n2, nd.depth + 1};   /* V1 is processed first */
        stack[sp++] = (node_t){v1, n1, nd.depth + 1};
    }
    free(stack);
}

/* ------------------------------------------------------------------ entry */

/* Returns 0 on success, negative on an invalid argument.
 * Inputs: 7 double arrays (FIXED mode rounds them to FP32 first), cell_off[n_cells+1].
 * Outputs (all caller-allocated, n = cell_off[n_cells] entries unless noted):
 *   perm[n]      global input index per slot, final subsets contiguous in DFS order
 *   subset_id[n] final-subset ordinal per slot (-1 for untouched cells)
 *   n_subsets[n_cells]
 *   out[7][n]    merged particles, cell-sorted, compacted
 *   out_off[n_cells+1]
 *   stats[n_cells], may be NULL                                           */
int orc_run(const orc_params *p, int64_t n_cells, const int64_t *cell_off,
            const double *x, const double *y, const double *z,
            const double *px, const double *py, const double *pz, const double *w,
            int32_t *perm, int32_t *subset_id, int32_t *n_subsets,
            double *ox, double *oy, double *oz, double *opx, double *opy, double *opz, double *ow,
            int64_t *out_off, orc_cell_stats *stats, int n_threads) {
    if (!p || n_cells < 0 || !cell_off) return -1;
    if (!(p->tol_x >= 0) || !(p->tol_p >= 0) || p->min_subset < 1) return -1;
    if (p->merge_mode == ORC_PAIR && p->min_subset < 2) return -1;
    for (int a = 0; a < 3; ++a) if (!(p->cell_len[a] > 0)) return -1;
    if (p->decide == ORC_FIXED && (p->tol_x >= 128 || p->tol_p >= 128)) return -1;
    if (!(p->mass >= 0)) return -1;
    for (int64_t c = 0; c < n_cells; ++c) if (cell_off[c + 1] < cell_off[c]) return -2;

    const int64_t N = cell_off[n_cells];
    const double *in[7] = {x, y, z, px, py, pz, w};
    double *outp[7] = {ox, oy, oz, opx, opy, opz, ow};
    int32_t *cnt_out = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n_cells + 1));
    double *tmp[7];
    for (int f = 0; f < 7; ++f) tmp[f] = (double *)malloc(sizeof(double) * (size_t)(N > 0 ? N : 1));

#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#pragma omp parallel for schedule(dynamic, 16)
#endif
    for (int64_t c = 0; c < n_cells; ++c) {
        const int64_t off = cell_off[c];
        const int n = (int)(cell_off[c + 1] - off);
        orc_cell_stats st; memset(&st, 0, sizeof st);
        st.min_margin = INFINITY;

        uint32_t bad = 0;
        for (int i = 0; i < n; ++i) {
            for (int f = 0; f < 7; ++f) {
                double v = in[f][off + i];
                if (p->decide == ORC_FIXED) v = (float)v;
                if (!isfinite(v)) bad |= ORC_FLAG_BAD_VALUE;
            }
            double wv = p->decide == ORC_FIXED ? (double)(float)w[off + i] : w[off + i];
            if (!(wv > 0)) bad |= ORC_FLAG_BAD_VALUE;
        }
        if (cell_off[c + 1] - off > (p->decide == ORC_FIXED ? ORC_NMAX_FIXED : ORC_NMAX_PAPER))
            bad |= ORC_FLAG_TOO_LARGE;

        if (n <= p->n_min_cell || bad || n == 0) {
            /* untouched: identity order, inputs copied (rounded to FP32 in FIXED mode) */
            for (int i = 0; i < n; ++i) {
                perm[off + i] = (int32_t)(off + i);
                subset_id[off + i] = -1;
                for (int f = 0; f < 7; ++f) {
                    double v = in[f][off + i];
                    tmp[f][off + i] = p->decide == ORC_FIXED ? (double)(float)v : v;
                }
            }
            n_subsets[c] = 0;
            cnt_out[c] = n;
            st.flags = bad;
            st.n_out = n;
            if (stats) stats[c] = st;
            continue;
        }

        cell_ctx cc; memset(&cc, 0, sizeof cc);
        cc.n = n; cc.p = p; cc.st = st;
        double *buf = (double *)malloc(sizeof(double) * (size_t)n * 14);
        for (int a = 0; a < 6; ++a) {
            cc.q[a] = buf + (size_t)a * n;
            for (int i = 0; i < n; ++i) {
                double v = in[a][off + i];
                cc.q[a][i] = p->decide == ORC_FIXED ? (double)(float)v : v;
            }
        }
        cc.w = buf + (size_t)6 * n;
        for (int i = 0; i < n; ++i) cc.w[i] = p->decide == ORC_FIXED ? (double)(float)w[off + i] : w[off + i];
        for (int f = 0; f < 7; ++f) cc.out[f] = buf + (size_t)(7 + f) * n;
        int64_t *ibuf = (int64_t *)malloc(sizeof(int64_t) * (size_t)n * 7);
        cc.om = ibuf;
        for (int l = 0; l < 6; ++l) cc.c[l] = ibuf + (size_t)(1 + l) * n;
        cc.perm = (int *)malloc(sizeof(int) * (size_t)n);
        cc.sid = (int *)malloc(sizeof(int) * (size_t)n);

        run_cell(&cc);

        for (int t = 0; t < n; ++t) { perm[off + t] = (int32_t)(off + cc.perm[t]); subset_id[off + t] = cc.sid[t]; }
        for (int o = 0; o < cc.n_out; ++o) for (int f = 0; f < 7; ++f) tmp[f][off + o] = cc.out[f][o];
        n_subsets[c] = cc.st.n_leaves;
        cnt_out[c] = cc.n_out;
        cc.st.n_out = cc.n_out;
        if (stats) stats[c] = cc.st;
        free(cc.perm); free(cc.sid); free(ibuf); free(buf);
    }

    out_off[0] = 0;
    for (int64_t c = 0; c < n_cells; ++c) out_off[c + 1] = out_off[c] + cnt_out[c];
#ifdef _OPENMP
#pragma omp parallel for schedule(static)
#endif
    for (int64_t c = 0; c < n_cells; ++c)
        for (int64_t o = 0; o < cnt_out[c]; ++o)
            for (int f = 0; f < 7; ++f) outp[f][out_off[c] + o] = tmp[f][cell_off[c] + o];
    for (int f = 0; f < 7; ++f) free(tmp[f]);
    free(cnt_out);
    return 0;
}

/* ------------------------------------------------------- the blind method */

/* The paper's comparison method (Sec. "Simulation", its description before the blocks test; Tables 1
 * and 2 give the merging fraction alpha): in a cell of N particles, pairs of particles picked at
 * random are merged until at most ceil(alpha N) remain.  A cell is merged only if ceil(alpha N) < N
 * (and N > N_min).  Each merge replaces the two by one particle carrying their summed weight and
 * their weighted centroid in position and momentum (weight and momentum kept, energy not).
 *
 * Random numbers: Philox4x64-10 (Salmon, Moraes, Dror and Shaw, "Parallel random numbers: as easy
 * as 1, 2, 3", SC 2011) with key (seed, 0) and counter (t, c, 0, 0) for the t-th merge of cell c.
 * With M = N - t particles left, outputs r0, r1 pick i = r0 mod M and j = r1 mod (M - 1), j
 * shifted past i.  The survivors are kept in an array of slots; the particle in slot j joins the
 * group of slot i and the last slot moves into slot j.  The output of a cell is its surviving slots
 * in slot order: a group of one particle is copied, a larger group is replaced by its centroid,
 * computed from its members (the same particle pairwise merges would give, in exact arithmetic).
 * group[k] (cell-local) is the output ordinal of input particle k. */

static void philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]) {
    const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
    const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
    uint64_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3], k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        u128 p0 = (u128)M0 * c0, p1 = (u128)M1 * c2;
        uint64_t hi0 = (uint64_t)(p0 >> 64), lo0 = (uint64_t)p0;
        uint64_t hi1 = (uint64_t)(p1 >> 64), lo1 = (uint64_t)p1;
        c0 = hi1 ^ c1 ^ k0; c1 = lo1; c2 = hi0 ^ c3 ^ k1; c3 = lo0;
        k0 += W0; k1 += W1;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* exported for the generator's known-answer test */
void orc_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]) {
    philox4x64_10(ctr, key, out);
}

static int blind_root(const int *parent, int i) {
    while (parent[i] != i) i = parent[i];
    return i;
}

/* Inputs as orc_run (rounded to FP32 first when f32 != 0).  Outputs: group[n] (may be NULL),
 * out[7] compacted cell by cell, out_off[n_cells+1]. */
int orc_blind(double alpha, uint64_t seed, int32_t n_min_cell, double mass, int f32, int64_t n_cells,
              const int64_t *cell_off, const double *x, const double *y, const double *z,
              const double *px, const double *py, const double *pz, const double *w, int32_t *group,
              double *ox, double *oy, double *oz, double *opx, double *opy, double *opz, double *ow,
              int64_t *out_off, int n_threads) {
    if (n_cells < 0 || !cell_off || !(alpha >= 0) || !(alpha <= 1e9) || n_min_cell < 0 || !(mass >= 0)) return -1;
    for (int64_t c = 0; c < n_cells; ++c) if (cell_off[c + 1] < cell_off[c]) return -2;
    const int64_t N = cell_off[n_cells];
    const double *in[7] = {x, y, z, px, py, pz, w};
    double *outp[7] = {ox, oy, oz, opx, opy, opz, ow};
    int32_t *cnt_out = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n_cells + 1));
    double *tmp[7];
    for (int f = 0; f < 7; ++f) tmp[f] = (double *)malloc(sizeof(double) * (size_t)(N > 0 ? N : 1));
    orc_params prm;
    memset(&prm, 0, sizeof prm);
    prm.mass = mass;
    prm.merge_mode = ORC_CENTROID;

#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#pragma omp parallel for schedule(dynamic, 16)
#endif
    for (int64_t c = 0; c < n_cells; ++c) {
        const int64_t off = cell_off[c];
        const int n = (int)(cell_off[c + 1] - off);
        const int64_t T = (int64_t)ceil(alpha * (double)n);
        int bad = 0;
        for (int i = 0; i < n; ++i) {
            for (int f = 0; f < 7; ++f) {
                double v = f32 ? (double)(float)in[f][off + i] : in[f][off + i];
                if (!isfinite(v) || (f == 6 && !(v > 0))) bad = 1;
            }
        }
        const int untouched = n == 0 || n <= n_min_cell || T >= n || n > 65536 || bad;
        double *buf = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1) * 14);
        cell_ctx cc;
        memset(&cc, 0, sizeof cc);
        cc.n = n; cc.p = &prm;
        for (int a = 0; a < 6; ++a) cc.q[a] = buf + (size_t)a * n;
        cc.w = buf + (size_t)6 * n;
        for (int f = 0; f < 7; ++f) cc.out[f] = buf + (size_t)(7 + f) * n;
        for (int i = 0; i < n; ++i) {
            for (int a = 0; a < 6; ++a) cc.q[a][i] = f32 ? (double)(float)in[a][off + i] : in[a][off + i];
            cc.w[i] = f32 ? (double)(float)w[off + i] : w[off + i];
        }
        if (untouched) {
            for (int i = 0; i < n; ++i) {
                for (int a = 0; a < 6; ++a) tmp[a][off + i] = cc.q[a][i];
                tmp[6][off + i] = cc.w[i];
                if (group) group[off + i] = i;
            }
            cnt_out[c] = n;
            free(buf);
            continue;
        }
        int *slot = (int *)malloc(sizeof(int) * (size_t)n * 5 + sizeof(int) * (size_t)(T + 1));
        int *parent = slot + n, *mem = slot + 2 * n, *gid = slot + 3 * n, *ordk = slot + 4 * n;
        int *start = slot + 5 * n;
        for (int i = 0; i < n; ++i) { slot[i] = i; parent[i] = i; }
        const uint64_t key[2] = {seed, 0};
        for (int64_t t = 0; t < n - T; ++t) {
            const uint64_t M = (uint64_t)(n - t);
            const uint64_t ctr[4] = {(uint64_t)t, (uint64_t)c, 0, 0};
            uint64_t r[4];
            philox4x64_10(ctr, key, r);
            uint64_t i = r[0] % M, j = r[1] % (M - 1);
            if (j >= i) j += 1;
            parent[slot[j]] = slot[i];            /* slot j's group joins slot i's */
            slot[j] = slot[M - 1];                /* the last slot fills the gap   */
        }
        /* output k = 0 .. T-1: the group rooted at slot[k], members in input order */
        for (int64_t k = 0; k < T; ++k) ordk[slot[k]] = (int)k;
        for (int64_t k = 0; k <= T; ++k) start[k] = 0;
        for (int i = 0; i < n; ++i) {
            gid[i] = ordk[blind_root(parent, i)];
            start[gid[i] + 1]++;
            if (group) group[off + i] = gid[i];
        }
        for (int64_t k = 0; k < T; ++k) start[k + 1] += start[k];
        for (int i = 0; i < n; ++i) mem[start[gid[i]]++] = i;      /* start[k] becomes start[k + 1] */
        cc.n_out = 0;
        for (int64_t k = 0; k < T; ++k) {
            const int b = k == 0 ? 0 : start[k - 1], cntm = start[k] - b;
            if (cntm == 1) passthrough_subset(&cc, mem + b, 1);
            else merge_subset(&cc, mem + b, cntm, 0);
        }
        for (int o = 0; o < cc.n_out; ++o) for (int f = 0; f < 7; ++f) tmp[f][off + o] = cc.out[f][o];
        cnt_out[c] = cc.n_out;
        free(slot);
        free(buf);
    }
    out_off[0] = 0;
    for (int64_t c = 0; c < n_cells; ++c) out_off[c + 1] = out_off[c] + cnt_out[c];
    for (int64_t c = 0; c < n_cells; ++c)
        for (int64_t o = 0; o < cnt_out[c]; ++o)
            for (int f = 0; f < 7; ++f) outp[f][out_off[c] + o] = tmp[f][cell_off[c] + o];
    for (int f = 0; f < 7; ++f) free(tmp[f]);
    free(cnt_out);
    return 0;
}

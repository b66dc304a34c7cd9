// Plain FP64 Voronoi particle merging: one wavefront per cell, the paper's statistics in IEEE
// double (Sec. "Algorithm", Steps 1-7), subsets visited depth first.
//
// For a subset: W = sum w, centroid X = sum w x / W, P = sum w p / W (Steps 1, 5), standard
// deviation about the centroid (Step 2), CVs sigma/L and sigma/|P| (Eqs. cv_x, cv_p), stop when
// all six are <= tolerance (Step 3), else cut through the centroid on the axis of largest CV
// (Steps 4-5) into V1 = {q <= Q} and V2 = {q > Q} in stable order (Step 6).  Finished subsets
// are replaced by their centroid or by the energy-conserving pair (Step 7).
//
// This is the baseline "one cell per workgroup" form: the particle data stay in global memory
// and are read through a permutation that is ping-ponged between two buffers; the node stack
// lives in global scratch.  Sums are wavefront tree reductions, so results can differ from a
// sequential sum in the last bits; decisions can then differ only at near-ties.
#include "vpm_device.hpp"
#include "vpm_internal.h"

namespace vpm {
namespace {

struct Fp64Args {
    Soa64 in;
    const int64_t* cell_off;
    const int32_t* queue;
    int32_t* counters;
    int qlen_index, work_index;
    Fp64Params P;
    int mode;                  // 0 run, 1 partition
    Soa64Out tmp;
    int64_t* out_count;
    uint8_t* cell_mode;
    int32_t* perm2;            // two buffers, each cap entries
    int64_t cap;
    int64_t* stack;
    int32_t *perm, *subset_id, *n_subsets;
    uint32_t* flags;
};

VPM_DEV double wsum(double v) {
    for (int m = 1; m < WAVE; m <<= 1) v += __shfl_xor(v, m);
    return v;
}

VPM_DEV void fence_wave() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

VPM_DEV int64_t pack_node(int start, int len, int par) {
    return (int64_t)start | ((int64_t)len << 20) | ((int64_t)par << 40);
}

VPM_DEV double qval(const Soa64& in, int l, int64_t i) {
    switch (l) {
        case 0: return in.x[i];
        case 1: return in.y[i];
        case 2: return in.z[i];
        case 3: return in.px[i];
        case 4: return in.py[i];
        default: return in.pz[i];
    }
}

// Replace a finished subset (Step 7) in FP64: the whole wave sums; lane 0 writes slot o (and o+1).
// W and mean[6] are the subset's weight and centroid; gidx(j) is the global index of member j.
template <typename IdxFn>
VPM_DEV void fp64_merge_out(const Fp64Args& A, int64_t o, double W, const double mean[6], IdxFn gidx, int len,
                            double m) {
    const int lane = threadIdx.x;
    const double P[3] = {mean[3], mean[4], mean[5]};
    const double P2 = P[0] * P[0] + P[1] * P[1] + P[2] * P[2];
    const double e0 = sqrt(m * m + P2);
    double a = 0;
    for (int j = lane; j < len; j += WAVE) {
        const int64_t i = gidx(j);
        const double p0 = A.in.px[i], p1 = A.in.py[i], p2 = A.in.pz[i];
        const double ei = sqrt(m * m + (p0 * p0 + p1 * p1 + p2 * p2));
        const double num = (p0 - P[0]) * (p0 + P[0]) + (p1 - P[1]) * (p1 + P[1]) + (p2 - P[2]) * (p2 + P[2]);
        const double den = ei + e0;
        if (den > 0.0) a += A.in.w[i] * num / den;
    }
    const double Am = wsum(a) / W;
    double r = Am * (Am + 2.0 * e0);
    if (!(r > 0.0)) r = 0.0;
    if (lane != 0) return;
    if (A.P.merge_mode == VPM_MERGE_CENTROID) {
        A.tmp.w[o] = W;
        A.tmp.x[o] = mean[0]; A.tmp.y[o] = mean[1]; A.tmp.z[o] = mean[2];
        A.tmp.px[o] = P[0]; A.tmp.py[o] = P[1]; A.tmp.pz[o] = P[2];
        return;
    }
    int jd = 0;
    double bv = 0;
    for (int q = 0; q < 3; ++q) {
        const double v = fabs(mean[3 + q] * W);
        if (q == 0 || v < bv) { bv = v; jd = q; }
    }
    double u[3] = {jd == 0 ? 1.0 : 0.0, jd == 1 ? 1.0 : 0.0, jd == 2 ? 1.0 : 0.0};
    const double pj = jd == 0 ? P[0] : (jd == 1 ? P[1] : P[2]);
    if (P2 > 0) for (int q = 0; q < 3; ++q) u[q] -= pj * P[q] / P2;
    const double un = sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
    const double s = sqrt(r) / un;
    for (int h = 0; h < 2; ++h) {
        const double sg = h == 0 ? s : -s;
        A.tmp.w[o + h] = W / 2;
        A.tmp.x[o + h] = mean[0]; A.tmp.y[o + h] = mean[1]; A.tmp.z[o + h] = mean[2];
        A.tmp.px[o + h] = P[0] + sg * u[0];
        A.tmp.py[o + h] = P[1] + sg * u[1];
        A.tmp.pz[o + h] = P[2] + sg * u[2];
    }
}

__global__ __launch_bounds__(64) void k_fp64_cells(Fp64Args A) {
    const int lane = threadIdx.x;
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
        const double mass = cell_mass(A.P.mass, A.P.species, A.P.species_mass, c);

        // validate the cell (w > 0, all values finite)
        bool ok = true;
        for (int i = lane; i < n; i += WAVE) {
            const double w = A.in.w[off + i];
            ok = ok && w > 0.0 && isfinite(w);
            for (int l = 0; l < 6; ++l) ok = ok && isfinite(qval(A.in, l, off + i));
        }
        if (ballot(!ok) != 0) {
            if (lane == 0) {
                atomicOr(A.flags, FLAG_BAD_VALUE);
                if (A.mode == 0) { A.out_count[c] = n; A.cell_mode[c] = CELL_UNTOUCHED; }
                else A.n_subsets[c] = 0;
            }
            if (A.mode == 1)
                for (int i = lane; i < n; i += WAVE) { A.perm[off + i] = (int32_t)(off + i); A.subset_id[off + i] = -1; }
            continue;
        }

        int32_t* buf0 = A.perm2 + off;
        int32_t* buf1 = A.perm2 + A.cap + off;
        int64_t* stk = A.stack + off;
        for (int i = lane; i < n; i += WAVE) buf0[i] = i;
        if (lane == 0) stk[0] = pack_node(0, n, 0);
        fence_wave();
        int sp = 1, out_pos = 0, nleaf = 0;
        const int npair = A.P.merge_mode == VPM_MERGE_PAIR ? 2 : 1;

        while (sp > 0) {
            --sp;
            const int64_t e = stk[sp];
            const int start = (int)(e & 0xfffff), len = (int)((e >> 20) & 0xfffff), par = (int)(e >> 40);
            const int32_t* src = par ? buf1 : buf0;
            int32_t* dst = par ? buf0 : buf1;
            bool merged = false, leaf = true;
            double W = 0, S[6], mean[6];
            if (len >= A.P.min_subset) {
                merged = true;
                double s[7] = {0, 0, 0, 0, 0, 0, 0};
                for (int j = lane; j < len; j += WAVE) {
                    const int64_t i = off + src[start + j];
                    const double w = A.in.w[i];
                    s[6] += w;
                    for (int l = 0; l < 6; ++l) s[l] += w * qval(A.in, l, i);
                }
                W = wsum(s[6]);
                for (int l = 0; l < 6; ++l) { S[l] = wsum(s[l]); mean[l] = S[l] / W; }
                double v[6] = {0, 0, 0, 0, 0, 0};
                for (int j = lane; j < len; j += WAVE) {
                    const int64_t i = off + src[start + j];
                    const double w = A.in.w[i];
                    for (int l = 0; l < 6; ++l) { const double d = qval(A.in, l, i) - mean[l]; v[l] += w * d * d; }
                }
                double D[6];
                bool done = true;
                for (int l = 0; l < 6; ++l) {
                    const double sig = sqrt(wsum(v[l]) / W);
                    if (l < 3) D[l] = sig / A.P.L[l];
                    else {
                        const double Pl = fabs(mean[l]);
                        D[l] = Pl == 0.0 ? (sig == 0.0 ? 0.0 : INFINITY) : sig / Pl;
                    }
                    const double T = l < 3 ? A.P.tol_x : A.P.tol_p;
                    if (!(D[l] <= T)) done = false;
                }
                if (!done) {
                    // Step 4: the largest CV, or with the normalised rule the largest CV over its
                    // tolerance (> 0 over a zero tolerance: infinite); ties to the lowest axis
                    if (A.P.axis_rule) {
                        for (int l = 0; l < 6; ++l) {
                            const double T = l < 3 ? A.P.tol_x : A.P.tol_p;
                            D[l] = T > 0.0 ? D[l] / T : (D[l] > 0.0 ? INFINITY : 0.0);
                        }
                    }
                    int k = 0;
                    for (int l = 1; l < 6; ++l) if (D[l] > D[k]) k = l;
                    const double Q = mean[k];
                    int n1 = 0;
                    for (int j = lane; j < len; j += WAVE) n1 += qval(A.in, k, off + src[start + j]) <= Q ? 1 : 0;
                    for (int m = 1; m < WAVE; m <<= 1) n1 += __shfl_xor(n1, m);
                    if (n1 > 0 && n1 < len) {
                        int lb = 0, rb = 0;
                        for (int j0 = 0; j0 < len; j0 += WAVE) {
                            const int j = j0 + lane;
                            const bool act = j < len;
                            int32_t li = 0;
                            bool right = false;
                            if (act) { li = src[start + j]; right = !(qval(A.in, k, off + li) <= Q); }
                            const uint64_t bl = ballot(act && !right), br = ballot(act && right);
                            if (act) {
                                const int d = right ? n1 + rb + __popcll(br & lanes_below()) : lb + __popcll(bl & lanes_below());
                                dst[start + d] = li;
                            }
                            lb += __popcll(bl);
                            rb += __popcll(br);
                        }
                        if (lane == 0) {
                            stk[sp] = pack_node(start + n1, len - n1, par ^ 1);
                            stk[sp + 1] = pack_node(start, n1, par ^ 1);
                        }
                        fence_wave();
                        sp += 2;
                        leaf = false;
                    }
                }
            }
            if (!leaf) continue;

            // final subset (DFS order): record / replace
            if (A.mode == 1) {
                for (int j = lane; j < len; j += WAVE) {
                    A.perm[off + start + j] = (int32_t)(off + src[start + j]);
                    A.subset_id[off + start + j] = nleaf;
                }
            } else if (!merged) {
                for (int j = lane; j < len; j += WAVE) {
                    const int64_t i = off + src[start + j];
                    const int64_t o = off + out_pos + j;
                    A.tmp.x[o] = A.in.x[i]; A.tmp.y[o] = A.in.y[i]; A.tmp.z[o] = A.in.z[i];
                    A.tmp.px[o] = A.in.px[i]; A.tmp.py[o] = A.in.py[i]; A.tmp.pz[o] = A.in.pz[i];
                    A.tmp.w[o] = A.in.w[i];
                }
                out_pos += len;
            } else {
                fp64_merge_out(A, off + out_pos, W, mean, [&](int j) { return off + (int64_t)src[start + j]; }, len,
                               mass);
                out_pos += npair;
            }
            ++nleaf;
        }
        if (lane == 0) {
            if (A.mode == 0) { A.out_count[c] = out_pos; A.cell_mode[c] = CELL_PROCESSED; }
            else A.n_subsets[c] = nleaf;
        }
    }
}


// Replacement from a given partition (vpm_merge, FP64): one wavefront per cell, subsets in order.
struct Fp64MergeArgs {
    Fp64Args A;
    const int32_t *perm, *subset_id, *n_subsets;
};

__global__ __launch_bounds__(64) void k_fp64_merge(Fp64MergeArgs G) {
    const Fp64Args& A = G.A;
    const int lane = threadIdx.x;
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
        const double mass = cell_mass(A.P.mass, A.P.species, A.P.species_mass, c);
        const int nsub = G.n_subsets[c];
        bool ok = nsub >= 1 && nsub <= n;
        for (int p = lane; p < n && ok; p += WAVE) {
            const int32_t mm = G.perm[off + p];
            const int32_t sd = G.subset_id[off + p];
            const int32_t prev = p == 0 ? -1 : G.subset_id[off + p - 1];
            const double wv = ok && mm >= off && mm < off + n ? A.in.w[mm] : 0.0;
            ok = mm >= off && mm < off + n && sd >= 0 && sd < nsub && (sd == prev || sd == prev + 1) &&
                 (p != n - 1 || sd == nsub - 1) && wv > 0.0 && isfinite(wv);
            for (int l = 0; ok && l < 6; ++l) ok = isfinite(qval(A.in, l, mm));
        }
        bool part_ok = ballot(!ok) == 0;
        if (part_ok) {
            // every member exactly once: each slot writes its position at its member's mark (the
            // first permutation buffer serves as the marks), then checks that the mark holds it
            for (int p = lane; p < n; p += WAVE) A.perm2[G.perm[off + p]] = (int32_t)(off + p);
            fence_wave();
            bool once = true;
            for (int p = lane; p < n; p += WAVE) once = once && A.perm2[G.perm[off + p]] == (int32_t)(off + p);
            part_ok = ballot(!once) == 0;
        }
        if (!part_ok) {
            if (lane == 0) {
                if (nsub >= 1) atomicOr(A.flags, FLAG_BAD_PARTITION);
                A.out_count[c] = n;
                A.cell_mode[c] = CELL_UNTOUCHED;
            }
            continue;
        }
        int out_pos = 0, b = 0;
        while (b < n) {
            // the subset starting at slot b ends where the ordinal changes
            const int sd = G.subset_id[off + b];
            int e = b + 1;
            while (e < n) {
                const int j = e + lane;
                const bool same = j < n && G.subset_id[off + j] == sd;
                const uint64_t notsame = ballot(!same);
                if (notsame != 0) { e += __ffsll((unsigned long long)notsame) - 1; break; }
                e += WAVE;
            }
            if (e > n) e = n;
            const int len = e - b;
            const int32_t* mem = G.perm + off + b;
            if (len < A.P.min_subset) {
                for (int j = lane; j < len; j += WAVE) {
                    const int64_t i = mem[j];
                    const int64_t o = off + out_pos + j;
                    A.tmp.x[o] = A.in.x[i]; A.tmp.y[o] = A.in.y[i]; A.tmp.z[o] = A.in.z[i];
                    A.tmp.px[o] = A.in.px[i]; A.tmp.py[o] = A.in.py[i]; A.tmp.pz[o] = A.in.pz[i];
                    A.tmp.w[o] = A.in.w[i];
                }
                out_pos += len;
            } else {
                double s[7] = {0, 0, 0, 0, 0, 0, 0};
                for (int j = lane; j < len; j += WAVE) {
                    const int64_t i = mem[j];
                    const double w = A.in.w[i];
                    s[6] += w;
                    for (int l = 0; l < 6; ++l) s[l] += w * qval(A.in, l, i);
                }
                const double W = wsum(s[6]);
                double mean[6];
                for (int l = 0; l < 6; ++l) mean[l] = wsum(s[l]) / W;
                fp64_merge_out(A, off + out_pos, W, mean, [&](int j) { return (int64_t)mem[j]; }, len, mass);
                out_pos += npair;
            }
            b = e;
        }
        if (lane == 0) { A.out_count[c] = out_pos; A.cell_mode[c] = CELL_PROCESSED; }
    }
}

}  // namespace

hipError_t launch_fp64_cells(const Workspace& ws, const LaunchCfg& lc, const Soa64& in, const int64_t* cell_off,
                             int64_t n_cells, const Fp64Params& fp, int mode, int32_t* perm, int32_t* subset_id,
                             int32_t* n_subsets) {
    (void)n_cells;
    Fp64Args A;
    A.in = in;
    A.cell_off = cell_off;
    A.counters = ws.counters;
    A.P = fp;
    A.mode = mode;
    A.tmp = Soa64Out{(double*)ws.tmp[0], (double*)ws.tmp[1], (double*)ws.tmp[2], (double*)ws.tmp[3],
                     (double*)ws.tmp[4], (double*)ws.tmp[5], (double*)ws.tmp[6]};
    A.out_count = ws.out_count;
    A.cell_mode = ws.cell_mode;
    A.perm2 = ws.perm2;
    A.cap = ws.cap_particles;
    A.stack = ws.stack;
    A.perm = perm; A.subset_id = subset_id; A.n_subsets = n_subsets;
    A.flags = ws.flags;
    const int qs[6] = {Q_BIG, Q_C, Q_B, Q_S, Q_D, Q_A};
    for (int q : qs) {
        A.queue = ws.queue[q];
        A.qlen_index = q;
        A.work_index = 8 + q;
        if (lc.pre) lc.pre(lc.prof, "fp64_cells", lc.stream);
        hipLaunchKernelGGL(k_fp64_cells, dim3(lc.grid_fp64), dim3(64), 0, lc.stream, A);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        if (lc.post) lc.post(lc.prof, "fp64_cells", lc.stream);
    }
    return hipSuccess;
}

hipError_t launch_fp64_merge(const Workspace& ws, const LaunchCfg& lc, const Soa64& in, const int64_t* cell_off,
                             int64_t n_cells, const Fp64Params& fp, const int32_t* perm, const int32_t* subset_id,
                             const int32_t* n_subsets) {
    (void)n_cells;
    Fp64MergeArgs G;
    Fp64Args& A = G.A;
    A.in = in;
    A.cell_off = cell_off;
    A.counters = ws.counters;
    A.P = fp;
    A.mode = 0;
    A.tmp = Soa64Out{(double*)ws.tmp[0], (double*)ws.tmp[1], (double*)ws.tmp[2], (double*)ws.tmp[3],
                     (double*)ws.tmp[4], (double*)ws.tmp[5], (double*)ws.tmp[6]};
    A.out_count = ws.out_count;
    A.cell_mode = ws.cell_mode;
    A.perm2 = ws.perm2;
    A.cap = ws.cap_particles;
    A.stack = ws.stack;
    A.perm = nullptr; A.subset_id = nullptr; A.n_subsets = nullptr;
    A.flags = ws.flags;
    G.perm = perm; G.subset_id = subset_id; G.n_subsets = n_subsets;
    const int qs[6] = {Q_BIG, Q_C, Q_B, Q_S, Q_D, Q_A};
    for (int q : qs) {
        A.queue = ws.queue[q];
        A.qlen_index = q;
        A.work_index = 8 + q;
        if (lc.pre) lc.pre(lc.prof, "fp64_merge", lc.stream);
        hipLaunchKernelGGL(k_fp64_merge, dim3(lc.grid_fp64), dim3(64), 0, lc.stream, G);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        if (lc.post) lc.post(lc.prof, "fp64_merge", lc.stream);
    }
    return hipSuccess;
}

}  // namespace vpm

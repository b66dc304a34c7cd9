// Common kernels: per-call reset, cell binning, output-offset scan, compaction copy, identity
// partition for cells that are not processed.
#include "vpm_device.hpp"
#include "vpm_internal.h"

namespace vpm {
namespace {

constexpr int SCAN_BLOCK = 1024;
constexpr int SCAN_PER_THREAD = 4;
constexpr int SCAN_TILE = SCAN_BLOCK * SCAN_PER_THREAD;

__global__ void k_reset(int32_t* counters) {
    // queue lengths [0, 8), work counters [8, 16), size-class list lengths [BIGQ_LEN0, +4), the
    // large-cell kernel's task ring and pending counts [28, 32)
    if (threadIdx.x < 32) counters[threadIdx.x] = 0;
}

// Classify every cell by size and append it to its queue (workgroup-aggregated atomics).
__global__ __launch_bounds__(256) void k_bin(const int64_t* cell_off, int64_t n_cells, int64_t n_particles,
                                             int32_t n_min_cell, int32_t* counters, int32_t* q_untouched,
                                             int32_t* q_a, int32_t* q_b, int32_t* q_c, int32_t* q_big, int32_t* q_s,
                                             int32_t* q_d,
                                             int64_t* out_count,
                                             uint8_t* cell_mode, uint32_t* flags, BinLimits lim,
                                             const uint8_t* species, int n_species, int32_t* bq0,
                                             int32_t* bq1, int32_t* bq2, int32_t* bq3) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int cls = -1, big = -1;
    if (c < n_cells) {
        const int64_t lo = cell_off[c], hi = cell_off[c + 1];
        int64_t n = hi - lo;
        uint32_t f = 0;
        const bool range_ok = lo >= 0 && hi >= lo && hi <= n_particles;
        if (!range_ok) { f |= FLAG_BAD_OFFSETS; n = 0; }     // never read outside the arrays
        if (c == 0 && lo != 0) f |= FLAG_BAD_OFFSETS;
        if (n > lim.big) f |= FLAG_TOO_LARGE;
        const bool species_ok = !species || species[c] < n_species;
        if (!species_ok) f |= FLAG_BAD_SPECIES;
        if (f) atomicOr(flags, f);
        if (n == 0 || n <= n_min_cell || n > lim.big || !range_ok || !species_ok) {
            cls = Q_UNTOUCHED;
            out_count[c] = n;
            cell_mode[c] = CELL_UNTOUCHED;
        } else if (n <= lim.s) {
            cls = Q_S;
        } else if (n <= lim.a) {
            cls = Q_A;
        } else if (n <= lim.d) {
            cls = Q_D;
        } else if (n <= lim.b) {
            cls = Q_B;
        } else if (n <= lim.c) {
            cls = Q_C;
        } else {
            cls = Q_BIG;
            big = n <= 8192 ? 0 : n <= 16384 ? 1 : n <= 32768 ? 2 : 3;
        }
    }
    // Appends: each wave reserves its run within the workgroup's count of each list (LDS atomics),
    // then one global atomic per list and workgroup reserves the workgroup's run in the list (one
    // global atomic per wave and list queued up on the few shared counters otherwise).
    constexpr int NL = Q_COUNT + BIGQ_CLASSES;   // the queues, then the large-cell size classes
    __shared__ int s_cnt[NL], s_base[NL];
    if (threadIdx.x < NL) s_cnt[threadIdx.x] = 0;
    __syncthreads();
    int pos_q = 0, pos_b = 0;
#pragma unroll
    for (int L = 0; L < NL; ++L) {
        const bool mine = L < Q_COUNT ? cls == L : big == L - Q_COUNT;
        const uint64_t m = ballot(mine);
        if (m == 0) continue;
        const int leader = __ffsll((unsigned long long)m) - 1;
        int wbase = 0;
        if (lane_id() == leader) wbase = atomicAdd(&s_cnt[L], __popcll(m));
        wbase = __shfl(wbase, leader);
        if (mine) {
            const int r = wbase + __popcll(m & lanes_below());
            if (L < Q_COUNT) pos_q = r; else pos_b = r;
        }
    }
    __syncthreads();
    if (threadIdx.x < NL) {
        const int k = s_cnt[threadIdx.x];
        const int ci = threadIdx.x < Q_COUNT ? threadIdx.x : BIGQ_LEN0 + (threadIdx.x - Q_COUNT);
        s_base[threadIdx.x] = k ? atomicAdd(&counters[ci], k) : 0;
    }
    __syncthreads();
    int32_t* const qs[Q_COUNT] = {q_untouched, q_a, q_b, q_c, q_big, q_s, q_d};
    int32_t* const bqs[BIGQ_CLASSES] = {bq0, bq1, bq2, bq3};
#pragma unroll
    for (int q = 0; q < Q_COUNT; ++q)
        if (cls == q) qs[q][s_base[q] + pos_q] = (int32_t)c;
#pragma unroll
    for (int k = 0; k < BIGQ_CLASSES; ++k)
        if (big == k) bqs[k][s_base[Q_COUNT + k] + pos_b] = (int32_t)c;
}

// Scan phase 1: per-tile totals of out_count.
__global__ __launch_bounds__(SCAN_BLOCK) void k_scan_tiles(const int64_t* cnt, int64_t n, int64_t* tiles) {
    __shared__ int64_t red[SCAN_BLOCK / WAVE + 1];
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_PER_THREAD;
    int64_t s = 0;
#pragma unroll
    for (int k = 0; k < SCAN_PER_THREAD; ++k) if (base + k < n) s += cnt[base + k];
    int64_t tot;
    block_exclusive_scan<SCAN_BLOCK>(s, red, &tot);
    if (threadIdx.x == 0) tiles[blockIdx.x] = tot;
}

// Scan phase 2: exclusive scan of the tile totals (single workgroup, loops over chunks).  The total
// is clamped to n_particles: offsets that decrease somewhere (flagged by k_bin) can make cells
// overlap, and their counts then add up to more than the output arrays hold.
__global__ __launch_bounds__(SCAN_BLOCK) void k_scan_tile_totals(int64_t* tiles, int64_t ntiles, int64_t* out_total,
                                                                 int64_t n_particles) {
    __shared__ int64_t red[SCAN_BLOCK / WAVE + 1];
    int64_t carry = 0;
    for (int64_t b = 0; b < ntiles; b += SCAN_BLOCK) {
        const int64_t i = b + threadIdx.x;
        const int64_t v = i < ntiles ? tiles[i] : 0;
        int64_t tot;
        const int64_t pre = block_exclusive_scan<SCAN_BLOCK>(v, red, &tot);
        if (i < ntiles) tiles[i] = carry + pre;
        carry += tot;
        __syncthreads();
    }
    if (threadIdx.x == 0) *out_total = min(carry, n_particles);
}

// Scan phase 3: write the exclusive prefix (out_off, clamped to n_particles like the total; clamping
// keeps it non-decreasing) and out_off[n].
__global__ __launch_bounds__(SCAN_BLOCK) void k_scan_apply(const int64_t* cnt, int64_t n, const int64_t* tiles,
                                                           int64_t* out_off, const int64_t* out_total,
                                                           int64_t n_particles) {
    __shared__ int64_t red[SCAN_BLOCK / WAVE + 1];
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_PER_THREAD;
    int64_t v[SCAN_PER_THREAD];
    int64_t s = 0;
#pragma unroll
    for (int k = 0; k < SCAN_PER_THREAD; ++k) { v[k] = base + k < n ? cnt[base + k] : 0; s += v[k]; }
    int64_t tot;
    int64_t pre = block_exclusive_scan<SCAN_BLOCK>(s, red, &tot) + tiles[blockIdx.x];
#pragma unroll
    for (int k = 0; k < SCAN_PER_THREAD; ++k) {
        if (base + k < n) out_off[base + k] = min(pre, n_particles);
        pre += v[k];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) out_off[n] = *out_total;
}

// Compaction: every output slot o finds its cell by binary search in out_off, then copies from the
// cell's temporary output (processed cells) or from the input (untouched cells).
template <typename TI, typename TO>
struct Tables { const TO* tmp[7]; const TI* in[7]; TO* out[7]; };

constexpr int SC_PER = 8, SC_CACHE = 256;

template <typename TI, typename TO>
__global__ __launch_bounds__(256) void k_scatter(const int64_t* cell_off, int64_t n_cells, const int64_t* out_off,
                                                 const uint8_t* cell_mode, Tables<TI, TO> tb) {
    const int64_t total = out_off[n_cells];
    const int64_t per_block = (int64_t)blockDim.x * SC_PER;
    const int64_t o0 = (int64_t)blockIdx.x * per_block;
    if (o0 >= total) return;
    __shared__ int64_t s_lo, s_hi;
    if (threadIdx.x == 0) {
        // cells holding the block's first and last output slots
        auto find = [&](int64_t o) {
            int64_t lo = 0, hi = n_cells - 1;
            while (lo < hi) {
                const int64_t mid = (lo + hi + 1) >> 1;
                if (out_off[mid] <= o) lo = mid; else hi = mid - 1;
            }
            return lo;
        };
        s_lo = find(o0);
        s_hi = find(min(total, o0 + per_block) - 1);
    }
    __syncthreads();
    const int64_t clo = s_lo, chi = s_hi;
    // the block's cells: output offsets, input offsets and modes cached in LDS when they fit
    __shared__ int64_t s_oo[SC_CACHE + 1], s_co[SC_CACHE + 1];
    __shared__ uint8_t s_md[SC_CACHE];
    const int64_t ncell = chi - clo + 1;
    const bool cached = ncell <= SC_CACHE;
    if (cached) {
        for (int64_t k = threadIdx.x; k <= ncell; k += blockDim.x) {
            s_oo[k] = out_off[clo + k];
            s_co[k] = cell_off[clo + k];
            if (k < ncell) s_md[k] = cell_mode[clo + k];
        }
    }
    __syncthreads();
    // all of a thread's slots are located first, then all their loads issued, then the stores (the
    // compiler cannot tell that the source and output arrays never overlap, and would otherwise wait
    // on each load before the next store)
    int64_t src[SC_PER];
    bool untouched[SC_PER];
#pragma unroll
    for (int k = 0; k < SC_PER; ++k) {
        const int64_t o = min(o0 + (int64_t)k * blockDim.x + threadIdx.x, total - 1);
        if (cached) {
            int lo = 0, hi = (int)ncell - 1;
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (s_oo[mid] <= o) lo = mid; else hi = mid - 1;
            }
            src[k] = s_co[lo] + (o - s_oo[lo]);
            untouched[k] = s_md[lo] == CELL_UNTOUCHED;
        } else {
            int64_t lo = clo, hi = chi;
            while (lo < hi) {
                const int64_t mid = (lo + hi + 1) >> 1;
                if (out_off[mid] <= o) lo = mid; else hi = mid - 1;
            }
            src[k] = cell_off[lo] + (o - out_off[lo]);
            untouched[k] = cell_mode[lo] == CELL_UNTOUCHED;
        }
    }
    TO v[SC_PER][7];
#pragma unroll
    for (int k = 0; k < SC_PER; ++k)
#pragma unroll
        for (int f = 0; f < 7; ++f) {
            if constexpr (sizeof(TI) == sizeof(TO))
                v[k][f] = __builtin_nontemporal_load((untouched[k] ? (const TO*)tb.in[f] : tb.tmp[f]) + src[k]);
            else                                               // FP64 input of the FP32 path: rounded
                v[k][f] = untouched[k] ? (TO)__builtin_nontemporal_load(tb.in[f] + src[k])
                                       : __builtin_nontemporal_load(tb.tmp[f] + src[k]);
        }
#pragma unroll
    for (int k = 0; k < SC_PER; ++k) {
        const int64_t o = o0 + (int64_t)k * blockDim.x + threadIdx.x;
        if (o >= total) break;
#pragma unroll
        for (int f = 0; f < 7; ++f) __builtin_nontemporal_store(v[k][f], tb.out[f] + o);
    }
}

__global__ __launch_bounds__(256) void k_identity(const int64_t* cell_off, int64_t n_particles, const int32_t* queue,
                                                  const int32_t* counters, int qidx, int32_t* perm, int32_t* subset_id,
                                                  int32_t* n_subsets) {
    const int nq = counters[qidx];
    for (int q = blockIdx.x; q < nq; q += gridDim.x) {
        const int c = queue[q];
        int64_t lo = cell_off[c], hi = cell_off[c + 1];
        if (lo < 0 || hi < lo || hi > n_particles) hi = lo;           // invalid range: write nothing
        for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) { perm[i] = (int32_t)i; subset_id[i] = -1; }
        if (threadIdx.x == 0) n_subsets[c] = 0;
    }
}

}  // namespace

hipError_t launch_bin(const Workspace& ws, const LaunchCfg& lc, const int64_t* cell_off, int64_t n_cells,
                      int64_t n_particles, int32_t n_min_cell, BinLimits lim, const uint8_t* species,
                      int n_species) {
    if (lc.pre) lc.pre(lc.prof, "reset", lc.stream);
    hipLaunchKernelGGL(k_reset, dim3(1), dim3(64), 0, lc.stream, ws.counters);
    if (lc.post) lc.post(lc.prof, "reset", lc.stream);
    if (n_cells == 0) return hipGetLastError();
    if (lc.pre) lc.pre(lc.prof, "bin", lc.stream);
    const int64_t blocks = (n_cells + 255) / 256;
    hipLaunchKernelGGL(k_bin, dim3((unsigned)blocks), dim3(256), 0, lc.stream, cell_off, n_cells, n_particles,
                       n_min_cell, ws.counters, ws.queue[Q_UNTOUCHED], ws.queue[Q_A], ws.queue[Q_B],
                       ws.queue[Q_C], ws.queue[Q_BIG], ws.queue[Q_S], ws.queue[Q_D], ws.out_count, ws.cell_mode,
                       ws.flags, lim,
                       species, n_species, ws.bigq[0], ws.bigq[1], ws.bigq[2], ws.bigq[3]);
    if (lc.post) lc.post(lc.prof, "bin", lc.stream);
    return hipGetLastError();
}

hipError_t launch_scan_offsets(const Workspace& ws, const LaunchCfg& lc, int64_t n_cells, int64_t n_particles,
                               int64_t* out_off, int64_t* out_total) {
    const int64_t ntiles = (n_cells + SCAN_TILE - 1) / SCAN_TILE;
    if (lc.pre) lc.pre(lc.prof, "scan", lc.stream);
    if (ntiles > 0)
        hipLaunchKernelGGL(k_scan_tiles, dim3((unsigned)ntiles), dim3(SCAN_BLOCK), 0, lc.stream, ws.out_count,
                           n_cells, ws.scan_blocks);
    hipLaunchKernelGGL(k_scan_tile_totals, dim3(1), dim3(SCAN_BLOCK), 0, lc.stream, ws.scan_blocks, ntiles,
                       out_total, n_particles);
    hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)(ntiles > 0 ? ntiles : 1)), dim3(SCAN_BLOCK), 0, lc.stream,
                       ws.out_count, n_cells, ws.scan_blocks, out_off, out_total, n_particles);
    if (lc.post) lc.post(lc.prof, "scan", lc.stream);
    return hipGetLastError();
}

template <typename TI, typename TO>
void scatter_launch(const Workspace& ws, const LaunchCfg& lc, const int64_t* cell_off, int64_t n_cells,
                    const int64_t* out_off, const void* const in[7], void* const out[7], int64_t blocks) {
    Tables<TI, TO> tb;
    for (int f = 0; f < 7; ++f) { tb.tmp[f] = (const TO*)ws.tmp[f]; tb.in[f] = (const TI*)in[f]; tb.out[f] = (TO*)out[f]; }
    hipLaunchKernelGGL((k_scatter<TI, TO>), dim3((unsigned)blocks), dim3(256), 0, lc.stream, cell_off, n_cells,
                       out_off, ws.cell_mode, tb);
}

hipError_t launch_scatter(const Workspace& ws, const LaunchCfg& lc, const int64_t* cell_off, int64_t n_cells,
                          int64_t n_particles, const int64_t* out_off, const void* const in[7], void* const out[7],
                          int in_size, int out_size) {
    if (n_cells == 0 || n_particles == 0) return hipSuccess;
    const int64_t blocks = (n_particles + 256 * SC_PER - 1) / (256 * SC_PER);   // out_total <= n_particles
    if (lc.pre) lc.pre(lc.prof, "scatter", lc.stream);
    if (in_size == 4) scatter_launch<float, float>(ws, lc, cell_off, n_cells, out_off, in, out, blocks);
    else if (out_size == 4) scatter_launch<double, float>(ws, lc, cell_off, n_cells, out_off, in, out, blocks);
    else scatter_launch<double, double>(ws, lc, cell_off, n_cells, out_off, in, out, blocks);
    if (lc.post) lc.post(lc.prof, "scatter", lc.stream);
    return hipGetLastError();
}

hipError_t launch_identity(const Workspace& ws, const LaunchCfg& lc, const int64_t* cell_off, int64_t n_particles,
                           int32_t* perm, int32_t* subset_id, int32_t* n_subsets) {
    if (lc.pre) lc.pre(lc.prof, "identity", lc.stream);
    hipLaunchKernelGGL(k_identity, dim3(1024), dim3(256), 0, lc.stream, cell_off, n_particles, ws.queue[Q_UNTOUCHED],
                       ws.counters, (int)Q_UNTOUCHED, perm, subset_id, n_subsets);
    if (lc.post) lc.post(lc.prof, "identity", lc.stream);
    return hipGetLastError();
}

}  // namespace vpm

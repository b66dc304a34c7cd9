// Internal declarations shared by the host library and the kernel translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/vpm.h"

namespace vpm {

// Per-cell handling decided by the binning kernel.
enum CellMode : uint8_t { CELL_PROCESSED = 0, CELL_UNTOUCHED = 1 };

// Size bins of the fixed-point path.
constexpr int NMAX_A = 576;     // 1 wavefront per cell, working set in LDS (8 cells per CU)
constexpr int NMAX_D = 1144;    // 2 wavefronts per cell, working set in LDS (4 cells per CU)
constexpr int NMAX_B = 2288;    // 4 wavefronts per cell, working set in LDS (2 cells per CU)
constexpr int NMAX_C = 4592;    // 8 wavefronts per cell, working set in LDS (1 cell per CU)
constexpr int NMAX_BIG = 65536; // 8 wavefronts per piece, several workgroups per cell, working set global
constexpr int NMAX_WIDE = 1 << 24;  // largest cell of the fixed-point vpm_run / vpm_partition (a whole box;
                                    // subsets above NMAX_BIG are split by one workgroup each, exactly)
constexpr int NMAX_S = 512;     // batches of small cells: 1 wavefront, up to 512 particles in LDS
constexpr int SMALL_MAX = 256;  // largest cell the small-cell bin may take
enum Queue { Q_UNTOUCHED = 0, Q_A = 1, Q_B = 2, Q_C = 3, Q_BIG = 4, Q_S = 5, Q_D = 6, Q_COUNT = 7 };
// The cells of Q_BIG are also listed by size class (k: up to 8192 << k particles), so that the
// global-memory bin can claim its largest cells first; the lists' lengths are counters
// [BIGQ_LEN0, BIGQ_LEN0 + 4).
constexpr int BIGQ_CLASSES = 4, BIGQ_LEN0 = 24;

// Status bits (mirrors VPM_FLAG_* plus one internal bit).
constexpr uint32_t FLAG_BAD_VALUE = VPM_FLAG_BAD_VALUE;
constexpr uint32_t FLAG_OUT_OF_CELL = VPM_FLAG_OUT_OF_CELL;
constexpr uint32_t FLAG_TOO_LARGE = VPM_FLAG_CELL_TOO_LARGE;
constexpr uint32_t FLAG_BAD_OFFSETS = VPM_FLAG_BAD_OFFSETS;
constexpr uint32_t FLAG_BAD_PARTITION = VPM_FLAG_BAD_PARTITION;
constexpr uint32_t FLAG_BAD_SPECIES = VPM_FLAG_BAD_SPECIES;
constexpr uint32_t FLAG_INTERNAL = 0x80000000u;  // a cut left one side empty (never expected)

// Device workspace, allocated by vpm_reserve.
struct Workspace {
    int64_t cap_particles = 0, cap_cells = 0;
    void* tmp[7] = {};              // temporary per-cell outputs at the cell's input offset (8 B/elt)
    int64_t* out_count = nullptr;   // [cap_cells]
    uint8_t* cell_mode = nullptr;   // [cap_cells]
    int32_t* queue[Q_COUNT] = {};   // [cap_cells] each
    int32_t* bigq[BIGQ_CLASSES] = {};   // [cap_cells] each: Q_BIG's cells by size class
    int32_t* counters = nullptr;    // [64]: queue lengths, work counters
    uint32_t* flags = nullptr;      // sticky status
    int64_t* scan_blocks = nullptr; // block totals for the offset scan
    // cells above the LDS bins: cell-wide codes, index buffers, output slots and info bytes
    // (indexed by input position), per-cell records and the task ring of the large-cell kernel
    void* big_rec = nullptr;        // [cap_particles] 16 B
    int32_t* big_pyz = nullptr;     // [cap_particles]
    uint32_t *big_idx0 = nullptr, *big_idx1 = nullptr;
    uint32_t* big_emit = nullptr;   // [cap_particles + 1]
    uint8_t* big_info = nullptr;
    void* big_cells = nullptr;      // [cap_cells] records
    void* big_tasks = nullptr;      // [ring_size] tasks
    int32_t* big_ready = nullptr;   // [ring_size], zero between calls
    int64_t ring_size = 0;
    void* big_lists = nullptr;      // per workgroup of the large-cell kernel: node lists
    uint32_t* big_sched = nullptr;  // and a schedule table
    int big_wgs = 0;                // workgroups the slabs serve (the kernel's grid)
    void* big_jobs = nullptr;       // subsets above 65,536 split by several workgroups: job records
    void* big_chunks = nullptr;     // and their chunk records (none: one workgroup splits such a subset)
    int32_t jobs_cap = 0, chunks_cap = 0;
    // scratch for the FP64 path: two permutation buffers and a node stack per particle slot
    int32_t* perm2 = nullptr;       // [2 * cap_particles]
    int64_t* stack = nullptr;       // [cap_particles]
};

// Fixed-point decision parameters derived on the host from vpm_params.
struct FixedParams {
    uint64_t that_x, that_p;        // round(T * 2^24)
    float t2x_lo, t2x_hi;           // FP32 bracket of (that_x / 2^24)^2
    float t2p_lo, t2p_hi;           // FP32 bracket of (that_p / 2^24)^2
    float s[3];                     // fl32(65536 / L_a)
    int32_t axis_rule;              // vpm_axis_rule
    uint64_t tx2, tp2;              // normalised rule: that_x^2, that_p^2 (< 2^62); raw rule: 1, 1
    float it2x_lo, it2x_hi;         // FP32 bracket of 1 / (that_x / 2^24)^2 (0 if that_x = 0)
    float it2p_lo, it2p_hi;
    int32_t min_subset;
    int32_t merge_mode;
    int32_t ppl_shift;              // log2 of the target particles per lane of a lane group
    int32_t force_exact;            // every decision by the exact integer rule (cross-checking)
    double mass;
    const uint8_t* species;         // per-cell species index (null: every cell has `mass`)
    double species_mass[VPM_MAX_SPECIES];
};

// Step 4's tolerance scale for the normalised axis rule, derived from that_x and that_p.
inline void fixed_axis_rule(FixedParams& f, int rule) {
    f.axis_rule = rule;
    f.tx2 = rule ? f.that_x * f.that_x : 1;      // the raw rule compares the CVs with unit weights
    f.tp2 = rule ? f.that_p * f.that_p : 1;
    auto inv = [](uint64_t t, float& lo, float& hi) {      // 2^48 / t^2, bracketed 2^-22 each side
        if (t == 0) { lo = hi = 0.0f; return; }
        const float f = (float)(0x1p48 / ((double)t * (double)t));
        lo = f * (1.0f - 0x1p-22f);
        hi = f * (1.0f + 0x1p-22f);
    };
    inv(f.that_x, f.it2x_lo, f.it2x_hi);
    inv(f.that_p, f.it2p_lo, f.it2p_hi);
}

// The particle mass of cell c (c wave-uniform).  The table is read with constant indices only.
__host__ __device__ inline double cell_mass(double mass, const uint8_t* species, const double* table, int64_t c) {
    if (!species) return mass;
    const int s = species[c];
    double m = table[0];
#pragma unroll
    for (int k = 1; k < VPM_MAX_SPECIES; ++k) if (s == k) m = table[k];
    return m;
}

// Routing thresholds of the size bins: cells of up to `s` particles go to the small-cell batches,
// up to `a` to bin A, up to `b` to B, up to `c` to C, larger ones to the global-memory bin.
struct BinLimits { int32_t a, b, c, s, big, d; };   // big: the largest cell processed; a <= d <= b

struct LaunchCfg {
    hipStream_t stream;
    int grid_a, grid_b, grid_c, grid_big, grid_s, grid_fp64, grid_d;   // persistent grid sizes
    // Optional fork/join for the size bins: bins run concurrently on side streams (default
    // priority) that wait on `fork` (recorded on `stream`) and are joined back through `join`.
    // conc_mode 1: the large-cell, eight- and four-wavefront bins on side[0..2]; 2: only the
    // two-wavefront bin, on side[0] (the others one after another on `stream`).
    hipStream_t side[3];
    hipEvent_t fork, join[3];
    int conc_mode;
    // profiling hooks (may be null)
    void (*pre)(void* prof, const char* name, hipStream_t s);
    void (*post)(void* prof, const char* name, hipStream_t s);
    void* prof;
};

template <typename T>
struct SoaIn { const T *x, *y, *z, *px, *py, *pz, *w; };
using Soa32 = SoaIn<float>;
using Soa64 = SoaIn<double>;
struct Soa32Out { float *x, *y, *z, *px, *py, *pz, *w; };
struct Soa64Out { double *x, *y, *z, *px, *py, *pz, *w; };

// ---- launchers (vpm_common.hip) ----
// species (may be null): cells whose species index is not below n_species are passed through.
hipError_t launch_bin(const Workspace& ws, const LaunchCfg& lc, const int64_t* cell_off,
                      int64_t n_cells, int64_t n_particles, int32_t n_min_cell, BinLimits lim,
                      const uint8_t* species = nullptr, int n_species = 0);
// out_off and out_total are clamped to n_particles (reached only with offsets flagged as bad).
hipError_t launch_scan_offsets(const Workspace& ws, const LaunchCfg& lc, int64_t n_cells, int64_t n_particles,
                               int64_t* out_off, int64_t* out_total);
// in_size, out_size: element bytes of the input and output arrays (4 or 8; FP64 input with FP32
// output for the fixed-point path, rounded to nearest as untouched cells are copied).
hipError_t launch_scatter(const Workspace& ws, const LaunchCfg& lc, const int64_t* cell_off,
                          int64_t n_cells, int64_t n_particles, const int64_t* out_off,
                          const void* const in[7], void* const out[7], int in_size, int out_size);
hipError_t launch_identity(const Workspace& ws, const LaunchCfg& lc, const int64_t* cell_off,
                           int64_t n_particles, int32_t* perm, int32_t* subset_id,
                           int32_t* n_subsets);

// ---- fixed-point path (vpm_fixed.hip) ----
// mode 0: run (partition + merge into ws.tmp, FP32), mode 1: partition only.  FP64 particles are
// rounded to FP32 as they are loaded (the fixed-point path works on FP32 values).
hipError_t launch_fixed_cells(const Workspace& ws, const LaunchCfg& lc, const Soa32& in, const int64_t* cell_off,
                              const FixedParams& fp, int mode, int32_t* perm, int32_t* subset_id, int32_t* n_subsets);
hipError_t launch_fixed_cells(const Workspace& ws, const LaunchCfg& lc, const Soa64& in, const int64_t* cell_off,
                              const FixedParams& fp, int mode, int32_t* perm, int32_t* subset_id, int32_t* n_subsets);
hipError_t launch_fixed_merge(const Workspace& ws, const LaunchCfg& lc, const Soa32& in, const int64_t* cell_off,
                              const FixedParams& fp, const int32_t* perm, const int32_t* subset_id,
                              const int32_t* n_subsets);
hipError_t launch_fixed_merge(const Workspace& ws, const LaunchCfg& lc, const Soa64& in, const int64_t* cell_off,
                              const FixedParams& fp, const int32_t* perm, const int32_t* subset_id,
                              const int32_t* n_subsets);
// The blind method (random pair merges down to ceil(alpha N) per cell) into ws.tmp, out_count and
// cell_mode for every cell (validation included; no binning needed).
hipError_t launch_fixed_blind(const Workspace& ws, const LaunchCfg& lc, const Soa32& in, const int64_t* cell_off,
                              int64_t n_cells, int64_t n_particles, const FixedParams& fp, double alpha,
                              uint64_t seed, int32_t n_min_cell, int32_t* group);
hipError_t launch_fixed_blind(const Workspace& ws, const LaunchCfg& lc, const Soa64& in, const int64_t* cell_off,
                              int64_t n_cells, int64_t n_particles, const FixedParams& fp, double alpha,
                              uint64_t seed, int32_t n_min_cell, int32_t* group);
// bins: 0 = A, 1 = B, 2 = C (LDS), 3 = big (global slabs), 4 = small-cell batches
int fixed_lds_bytes(int which);            // dynamic LDS per workgroup
const void* fixed_kernel_ptr(int which);   // for occupancy queries
int fixed_block_threads(int which);
int64_t fixed_big_cell_bytes();            // per-cell record of the large-cell kernel
int64_t fixed_big_task_bytes();            // one task of its ring
int64_t fixed_wide_job_bytes();            // a subset above 65,536 split by several workgroups
int64_t fixed_wide_chunk_bytes();          // one chunk of it
int fixed_task_min();                      // smallest subset handed to another workgroup
int64_t fixed_big_lists_bytes();           // per workgroup of the large-cell kernel
int64_t fixed_big_sched_bytes();

// ---- plain FP64 path (vpm_fp64.hip) ----
struct Fp64Params {
    double tol_x, tol_p, L[3], mass;
    int32_t min_subset, merge_mode, n_min_cell, axis_rule;
    const uint8_t* species;         // as in FixedParams
    double species_mass[VPM_MAX_SPECIES];
};
hipError_t launch_fp64_cells(const Workspace& ws, const LaunchCfg& lc, const Soa64& in,
                             const int64_t* cell_off, int64_t n_cells, const Fp64Params& fp,
                             int mode, int32_t* perm, int32_t* subset_id, int32_t* n_subsets);
hipError_t launch_fp64_merge(const Workspace& ws, const LaunchCfg& lc, const Soa64& in,
                             const int64_t* cell_off, int64_t n_cells, const Fp64Params& fp,
                             const int32_t* perm, const int32_t* subset_id,
                             const int32_t* n_subsets);

}  // namespace vpm

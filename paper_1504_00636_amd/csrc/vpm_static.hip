// vpm_run_noalloc: the fused merge (vpm_run, fixed-point decisions) for callers that cannot allocate
// device memory.  Its working memory is one file-scope device array, `scratch`, of a fixed size; each
// GPU the library runs on holds its own copy until the process ends.  The array's device address is
// taken with hipGetSymbolAddress once per device (with that device current) and only that address is
// passed to kernels: in host code the array's name is a host-side stand-in, not device memory.
//
// The call enqueues exactly the kernels vpm_run enqueues (binning, the size-binned cell kernels, the
// offset scan and the output compaction) over a workspace carved from the array, so its results are
// bit-identical to vpm_run's with the default tuning.  Calls on one GPU share the array: calls whose
// work overlaps in time on that GPU race, and must be ordered by the caller (one stream, or events).
#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>

#include "vpm_internal.h"

namespace vpm {
namespace {

// The limits of one call, and the bytes of the array.
constexpr int64_t NA_MAX_PARTICLES = VPM_NOALLOC_MAX_PARTICLES;
constexpr int64_t NA_MAX_CELLS = VPM_NOALLOC_MAX_CELLS;
constexpr int NA_BIG_WGS = 4;              // workgroups of the large-cell kernel (their node-list slabs)
constexpr size_t NA_SCRATCH_BYTES = (size_t)48 << 20;

static __device__ __align__(256) uint8_t scratch[NA_SCRATCH_BYTES];

constexpr int NA_MAX_DEVICES = 64;
std::mutex g_mutex;
uint8_t* g_ptr[NA_MAX_DEVICES] = {};        // device address of `scratch` per device (null: not yet)
int g_grid[NA_MAX_DEVICES][6] = {};        // persistent grid sizes of the LDS bins per device

__global__ void k_na_clear(uint32_t* flags) {
    if (threadIdx.x == 0) *flags = 0;
}

__global__ void k_na_flags_out(const uint32_t* flags, uint32_t* out) {
    if (threadIdx.x == 0) *out = *flags;
}

size_t rnd256(size_t b) { return (b + 255) & ~(size_t)255; }

// The workspace of one call carved from the array at `base`; returns the bytes it spans.
size_t carve(uint8_t* base, Workspace& ws) {
    size_t o = 0;
    auto take = [&](size_t bytes) { uint8_t* p = base + o; o += rnd256(bytes); return p; };
    ws.cap_particles = NA_MAX_PARTICLES;
    ws.cap_cells = NA_MAX_CELLS;
    for (int f = 0; f < 7; ++f) ws.tmp[f] = take((size_t)NA_MAX_PARTICLES * sizeof(float));
    ws.out_count = (int64_t*)take((size_t)NA_MAX_CELLS * 8);
    ws.cell_mode = (uint8_t*)take((size_t)NA_MAX_CELLS);
    for (int q = 0; q < Q_COUNT; ++q) ws.queue[q] = (int32_t*)take((size_t)NA_MAX_CELLS * 4);
    for (int k = 0; k < BIGQ_CLASSES; ++k) ws.bigq[k] = (int32_t*)take((size_t)NA_MAX_CELLS * 4);
    ws.counters = (int32_t*)take(4096);
    ws.flags = (uint32_t*)take(256);
    ws.scan_blocks = (int64_t*)take((size_t)(NA_MAX_CELLS / 4096 + 2) * 8);
    ws.big_rec = take((size_t)NA_MAX_PARTICLES * 16);
    ws.big_pyz = (int32_t*)take((size_t)NA_MAX_PARTICLES * 4);
    ws.big_idx0 = (uint32_t*)take((size_t)NA_MAX_PARTICLES * 4);
    ws.big_idx1 = (uint32_t*)take((size_t)NA_MAX_PARTICLES * 4);
    ws.big_emit = (uint32_t*)take((size_t)(NA_MAX_PARTICLES + 1) * 4);
    ws.big_info = take((size_t)NA_MAX_PARTICLES);
    ws.big_cells = take((size_t)NA_MAX_CELLS * (size_t)fixed_big_cell_bytes());
    ws.ring_size = NA_MAX_PARTICLES / fixed_task_min() + 1024;
    ws.big_tasks = take((size_t)ws.ring_size * (size_t)fixed_big_task_bytes());
    ws.big_ready = (int32_t*)take((size_t)ws.ring_size * 4);     // zero at load, zero after every call
    ws.big_wgs = NA_BIG_WGS;
    ws.big_lists = take((size_t)NA_BIG_WGS * (size_t)fixed_big_lists_bytes());
    ws.big_sched = (uint32_t*)take((size_t)NA_BIG_WGS * (size_t)fixed_big_sched_bytes());
    ws.perm2 = nullptr;                    // used only by the FP64 form and vpm_merge
    ws.stack = nullptr;
    return o;
}

// Set-up on the current device, once: the array's device address and the bins' grid sizes.
vpm_status device_setup(int dev, uint8_t** ptr, int grid[6]) {
    std::lock_guard<std::mutex> lock(g_mutex);
    if (!g_ptr[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return VPM_ERR_HIP;
        Workspace probe;
        if (carve((uint8_t*)p, probe) > NA_SCRATCH_BYTES) return VPM_ERR_HIP;   // layout/array mismatch
        int cus = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
            cus = 256;
        for (int b = 0; b < 6; ++b) {
            int nb = 0;
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fixed_kernel_ptr(b), fixed_block_threads(b),
                                                         fixed_lds_bytes(b));
            g_grid[dev][b] = b == 3 ? NA_BIG_WGS : cus * (nb > 0 ? nb : 1);
        }
        g_ptr[dev] = (uint8_t*)p;
    }
    *ptr = g_ptr[dev];
    for (int b = 0; b < 6; ++b) grid[b] = g_grid[dev][b];
    return VPM_OK;
}

}  // namespace
}  // namespace vpm

using namespace vpm;

extern "C" vpm_status vpm_run_noalloc(const vpm_soa* in, const int64_t* cell_off, int64_t n_cells,
                                      int64_t n_particles, const vpm_params* p, vpm_soa* out, int64_t* out_off,
                                      int64_t* out_total, uint32_t* flags_out, hipStream_t stream) {
    if (!in || !out || !cell_off || !out_off || !out_total || n_cells < 0 || n_particles < 0) return VPM_ERR_INVALID_ARG;
    const void* ip[7] = {in->x, in->y, in->z, in->px, in->py, in->pz, in->w};
    void* op[7] = {out->x, out->y, out->z, out->px, out->py, out->pz, out->w};
    for (int f = 0; f < 7; ++f) if (!ip[f] || !op[f]) return VPM_ERR_INVALID_ARG;
    vpm_status st = vpm_check_params(p);
    if (st != VPM_OK) return st;
    if (p->decide != VPM_DECIDE_FIXED || p->dtype != VPM_F32) return VPM_ERR_UNSUPPORTED;
    if (n_particles > NA_MAX_PARTICLES || n_cells > NA_MAX_CELLS) return VPM_ERR_CAPACITY;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= NA_MAX_DEVICES) return VPM_ERR_NO_DEVICE;
    uint8_t* base = nullptr;
    int grid[6];
    st = device_setup(dev, &base, grid);
    if (st != VPM_OK) return st;

    Workspace ws;
    carve(base, ws);
    LaunchCfg lc;
    lc.stream = stream;
    lc.grid_a = grid[0]; lc.grid_b = grid[1]; lc.grid_c = grid[2]; lc.grid_big = grid[3]; lc.grid_s = grid[4];
    lc.grid_d = grid[5];
    lc.grid_fp64 = 0;
    for (int i = 0; i < 3; ++i) { lc.side[i] = nullptr; lc.join[i] = nullptr; }
    lc.fork = nullptr;                     // the bins run one after another on the caller's stream
    lc.conc_mode = 0;
    lc.pre = nullptr; lc.post = nullptr; lc.prof = nullptr;

    // the default tuning of a context: 16 particles per lane, bins 576 / 1144 / 2288 / 4592, batches <= 128
    FixedParams fp;
    fp.that_x = (uint64_t)llrint(p->tol_x * 16777216.0);
    fp.that_p = (uint64_t)llrint(p->tol_p * 16777216.0);
    auto bracket = [](uint64_t t, float& lo, float& hi) {
        const float f = (float)((double)t * (double)t * 0x1p-48);
        lo = f * (1.0f - 0x1p-22f);
        hi = f * (1.0f + 0x1p-22f);
    };
    bracket(fp.that_x, fp.t2x_lo, fp.t2x_hi);
    bracket(fp.that_p, fp.t2p_lo, fp.t2p_hi);
    fixed_axis_rule(fp, p->axis_rule);
    for (int a = 0; a < 3; ++a) fp.s[a] = (float)(65536.0 / p->cell_len[a]);
    fp.min_subset = p->min_subset;
    fp.merge_mode = p->merge_mode;
    fp.ppl_shift = 4;
    fp.force_exact = 0;
    fp.mass = p->mass;
    fp.species = nullptr;
    for (int k = 0; k < VPM_MAX_SPECIES; ++k) fp.species_mass[k] = p->mass;
    const BinLimits lim{NMAX_A, NMAX_B, NMAX_C, 128, NMAX_WIDE, NMAX_D};

    // the flags start at zero for every call (a kernel, not a memset: the call may be captured)
    hipLaunchKernelGGL(k_na_clear, dim3(1), dim3(64), 0, stream, ws.flags);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = launch_bin(ws, lc, cell_off, n_cells, n_particles, p->n_min_cell, lim);
    if (e == hipSuccess) {
        const Soa32 s{(const float*)in->x, (const float*)in->y, (const float*)in->z, (const float*)in->px,
                      (const float*)in->py, (const float*)in->pz, (const float*)in->w};
        e = launch_fixed_cells(ws, lc, s, cell_off, fp, 0, nullptr, nullptr, nullptr);
    }
    if (e == hipSuccess) e = launch_scan_offsets(ws, lc, n_cells, n_particles, out_off, out_total);
    if (e == hipSuccess) e = launch_scatter(ws, lc, cell_off, n_cells, n_particles, out_off, ip, op, 4, 4);
    if (e == hipSuccess && flags_out) {
        hipLaunchKernelGGL(k_na_flags_out, dim3(1), dim3(64), 0, stream, ws.flags, flags_out);
        e = hipGetLastError();
    }
    return e == hipSuccess ? VPM_OK : VPM_ERR_HIP;
}

// Host side of the C ABI (include/vpm.h): argument validation, the context and its workspace,
// and stream-ordered enqueue of the kernels.  Nothing here synchronises except vpm_reserve,
// vpm_destroy, vpm_device_status and vpm_profile_read.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "vpm_internal.h"

using namespace vpm;

struct vpm_ctx {
    int device = 0;
    int cu_count = 0;
    Workspace ws;
    int grid_a = 0, grid_b = 0, grid_c = 0, grid_big = 0, grid_s = 0, grid_fp64 = 0, grid_d = 0;
    vpm_tuning tune = {16, NMAX_A, NMAX_B, NMAX_C, 0, 128, 0, NMAX_D};
    hipStream_t side[3] = {nullptr, nullptr, nullptr};
    hipEvent_t fork = nullptr, join[3] = {nullptr, nullptr, nullptr};
    std::string last_error;
    // profiling
    bool profiling = false;
    struct Rec { int kernel; hipEvent_t a, b; };
    std::vector<std::string> knames;
    std::vector<int64_t> klaunch;
    std::vector<double> kms;
    std::vector<Rec> pending;
    std::vector<hipEvent_t> pool;
    int open_kernel = -1;
    hipEvent_t open_event = nullptr;
};

namespace {

vpm_status hip_fail(vpm_ctx* ctx, hipError_t e, const char* what) {
    if (ctx) {
        ctx->last_error = std::string(what) + ": " + hipGetErrorString(e);
    }
    return VPM_ERR_HIP;
}

hipEvent_t take_event(vpm_ctx* c) {
    if (!c->pool.empty()) {
        hipEvent_t e = c->pool.back();
        c->pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

void prof_pre(void* p, const char* name, hipStream_t s) {
    vpm_ctx* c = (vpm_ctx*)p;
    int k = -1;
    for (size_t i = 0; i < c->knames.size(); ++i)
        if (c->knames[i] == name) k = (int)i;
    if (k < 0) {
        c->knames.push_back(name);
        c->klaunch.push_back(0);
        c->kms.push_back(0.0);
        k = (int)c->knames.size() - 1;
    }
    hipEvent_t e = take_event(c);
    if (e) hipEventRecord(e, s);
    c->open_kernel = k;
    c->open_event = e;
}

void prof_post(void* p, const char* name, hipStream_t s) {
    (void)name;
    vpm_ctx* c = (vpm_ctx*)p;
    hipEvent_t e = take_event(c);
    if (e && c->open_event) {
        hipEventRecord(e, s);
        c->pending.push_back({c->open_kernel, c->open_event, e});
    }
    c->open_event = nullptr;
}

LaunchCfg make_cfg(vpm_ctx* c, hipStream_t s) {
    LaunchCfg lc;
    lc.stream = s;
    lc.grid_a = c->grid_a;
    lc.grid_b = c->grid_b;
    lc.grid_c = c->grid_c;
    lc.grid_s = c->grid_s;
    lc.grid_d = c->grid_d;
    lc.grid_big = std::min(c->grid_big, c->ws.big_wgs > 0 ? c->ws.big_wgs : c->grid_big);
    lc.grid_fp64 = c->grid_fp64;
    const bool fork = c->tune.concurrent_bins != 0;
    for (int i = 0; i < 3; ++i) { lc.side[i] = fork ? c->side[i] : nullptr; lc.join[i] = fork ? c->join[i] : nullptr; }
    lc.fork = fork ? c->fork : nullptr;
    lc.conc_mode = c->tune.concurrent_bins;
    lc.pre = c->profiling ? prof_pre : nullptr;
    lc.post = c->profiling ? prof_post : nullptr;
    lc.prof = c;
    return lc;
}

bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

void free_ws(Workspace& ws) {
    for (int f = 0; f < 7; ++f) if (ws.tmp[f]) hipFree(ws.tmp[f]);
    if (ws.out_count) hipFree(ws.out_count);
    if (ws.cell_mode) hipFree(ws.cell_mode);
    for (int q = 0; q < Q_COUNT; ++q) if (ws.queue[q]) hipFree(ws.queue[q]);
    for (int k = 0; k < BIGQ_CLASSES; ++k) if (ws.bigq[k]) hipFree(ws.bigq[k]);
    if (ws.counters) hipFree(ws.counters);
    if (ws.flags) hipFree(ws.flags);
    if (ws.scan_blocks) hipFree(ws.scan_blocks);
    void* bigs[] = {ws.big_rec, ws.big_pyz, ws.big_idx0, ws.big_idx1, ws.big_emit, ws.big_info, ws.big_cells,
                    ws.big_tasks, ws.big_ready, ws.big_lists, ws.big_sched, ws.big_jobs, ws.big_chunks};
    for (void* b : bigs) if (b) hipFree(b);
    if (ws.perm2) hipFree(ws.perm2);
    if (ws.stack) hipFree(ws.stack);
    ws = Workspace();
}

vpm_status check_soa(const vpm_soa* s) {
    if (!s || !s->x || !s->y || !s->z || !s->px || !s->py || !s->pz || !s->w) return VPM_ERR_INVALID_ARG;
    return VPM_OK;
}

vpm_status common_checks(vpm_ctx* ctx, const vpm_soa* in, const int64_t* cell_off, int64_t n_cells,
                         int64_t n_particles, const vpm_params* p) {
    if (!ctx || !cell_off || n_cells < 0 || n_particles < 0) return VPM_ERR_INVALID_ARG;
    vpm_status st = vpm_check_params(p);
    if (st != VPM_OK) return st;
    if (check_soa(in) != VPM_OK) return VPM_ERR_INVALID_ARG;
    if (p->decide == VPM_DECIDE_FP64 && p->dtype != VPM_F64) return VPM_ERR_UNSUPPORTED;
    if (n_particles > ctx->ws.cap_particles || n_cells > ctx->ws.cap_cells) return VPM_ERR_CAPACITY;
    if (n_particles >= (int64_t)1 << 31) return VPM_ERR_CAPACITY;   // int32 permutation indices
    return VPM_OK;
}

int ilog2(int v) {
    int s = 0;
    while ((1 << (s + 1)) <= v) ++s;
    return s;
}

// big: the largest cell processed (the fixed-point partition takes whole boxes; the FP64 form and
// vpm_merge keep to NMAX_BIG)
BinLimits bin_limits(const vpm_ctx* c, int32_t big) {
    return BinLimits{c->tune.bin_a_max, c->tune.bin_b_max, c->tune.bin_c_max, c->tune.bin_s_max, big,
                     c->tune.bin_d_max};
}

FixedParams fixed_params(const vpm_params* p, const vpm_tuning& t) {
    FixedParams f;
    f.that_x = (uint64_t)llrint(p->tol_x * 16777216.0);
    f.that_p = (uint64_t)llrint(p->tol_p * 16777216.0);
    // (T^ / 2^24)^2 to double precision, then an FP32 bracket 2^-22 wide on each side
    auto bracket = [](uint64_t t, float& lo, float& hi) {
        const float f = (float)((double)t * (double)t * 0x1p-48);
        lo = f * (1.0f - 0x1p-22f);
        hi = f * (1.0f + 0x1p-22f);
    };
    bracket(f.that_x, f.t2x_lo, f.t2x_hi);
    bracket(f.that_p, f.t2p_lo, f.t2p_hi);
    fixed_axis_rule(f, p->axis_rule);
    for (int a = 0; a < 3; ++a) f.s[a] = (float)(65536.0 / p->cell_len[a]);
    f.min_subset = p->min_subset;
    f.merge_mode = p->merge_mode;
    f.ppl_shift = ilog2(t.ppl);
    f.force_exact = t.exact_decisions;
    f.mass = p->mass;
    f.species = nullptr;
    for (int k = 0; k < VPM_MAX_SPECIES; ++k) f.species_mass[k] = p->mass;
    return f;
}

Fp64Params fp64_params(const vpm_params* p) {
    Fp64Params f;
    f.tol_x = p->tol_x;
    f.tol_p = p->tol_p;
    for (int a = 0; a < 3; ++a) f.L[a] = p->cell_len[a];
    f.mass = p->mass;
    f.min_subset = p->min_subset;
    f.merge_mode = p->merge_mode;
    f.n_min_cell = p->n_min_cell;
    f.axis_rule = p->axis_rule;
    f.species = nullptr;
    for (int k = 0; k < VPM_MAX_SPECIES; ++k) f.species_mass[k] = p->mass;
    return f;
}

// Element bytes of the input arrays and of the output arrays (the fixed-point path emits FP32).
int elem_in(const vpm_params* p) { return p->dtype == VPM_F32 ? 4 : 8; }
int elem_out(const vpm_params* p) { return p->decide == VPM_DECIDE_FIXED || p->dtype == VPM_F32 ? 4 : 8; }

Soa32 soa32(const vpm_soa* s) {
    return Soa32{(const float*)s->x, (const float*)s->y, (const float*)s->z, (const float*)s->px,
                 (const float*)s->py, (const float*)s->pz, (const float*)s->w};
}
Soa64 soa64(const vpm_soa* s) {
    return Soa64{(const double*)s->x, (const double*)s->y, (const double*)s->z, (const double*)s->px,
                 (const double*)s->py, (const double*)s->pz, (const double*)s->w};
}

// vpm_run and vpm_run_species: species (device, may be null) with its mass table (host).
vpm_status run_impl(vpm_ctx* ctx, const vpm_soa* in, const int64_t* cell_off, int64_t n_cells,
                    int64_t n_particles, const vpm_params* p, const uint8_t* species, const double* species_mass,
                    int32_t n_species, vpm_soa* out, int64_t* out_off, int64_t* out_total, hipStream_t stream) {
    vpm_status st = common_checks(ctx, in, cell_off, n_cells, n_particles, p);
    if (st != VPM_OK) return st;
    if (check_soa(out) != VPM_OK || !out_off || !out_total) return VPM_ERR_INVALID_ARG;
    hipSetDevice(ctx->device);
    LaunchCfg lc = make_cfg(ctx, stream);
    hipError_t e = launch_bin(ctx->ws, lc, cell_off, n_cells, n_particles, p->n_min_cell,
                              bin_limits(ctx, p->decide == VPM_DECIDE_FIXED ? NMAX_WIDE : NMAX_BIG), species,
                              n_species);
    if (e != hipSuccess) return hip_fail(ctx, e, "bin");
    if (p->decide == VPM_DECIDE_FIXED) {
        FixedParams fp = fixed_params(p, ctx->tune);
        if (species) {
            fp.species = species;
            for (int k = 0; k < VPM_MAX_SPECIES; ++k) fp.species_mass[k] = species_mass[k < n_species ? k : 0];
        }
        e = p->dtype == VPM_F32 ? launch_fixed_cells(ctx->ws, lc, soa32(in), cell_off, fp, 0, nullptr, nullptr, nullptr)
                                : launch_fixed_cells(ctx->ws, lc, soa64(in), cell_off, fp, 0, nullptr, nullptr, nullptr);
    } else {
        Fp64Params fp = fp64_params(p);
        if (species) {
            fp.species = species;
            for (int k = 0; k < VPM_MAX_SPECIES; ++k) fp.species_mass[k] = species_mass[k < n_species ? k : 0];
        }
        e = launch_fp64_cells(ctx->ws, lc, soa64(in), cell_off, n_cells, fp, 0, nullptr, nullptr, nullptr);
    }
    if (e != hipSuccess) return hip_fail(ctx, e, "cells");
    e = launch_scan_offsets(ctx->ws, lc, n_cells, n_particles, out_off, out_total);
    if (e != hipSuccess) return hip_fail(ctx, e, "scan");
    const void* ins[7] = {in->x, in->y, in->z, in->px, in->py, in->pz, in->w};
    void* outs[7] = {out->x, out->y, out->z, out->px, out->py, out->pz, out->w};
    e = launch_scatter(ctx->ws, lc, cell_off, n_cells, n_particles, out_off, ins, outs, elem_in(p), elem_out(p));
    if (e != hipSuccess) return hip_fail(ctx, e, "scatter");
    return VPM_OK;
}


}  // namespace

extern "C" {

const char* vpm_version(void) { return "vpm 0.1 gfx950"; }

const char* vpm_status_string(vpm_status st) {
    switch (st) {
        case VPM_OK: return "ok";
        case VPM_ERR_INVALID_ARG: return "invalid argument";
        case VPM_ERR_UNSUPPORTED: return "unsupported dtype/decision combination";
        case VPM_ERR_CAPACITY: return "workspace capacity exceeded (call vpm_reserve)";
        case VPM_ERR_HIP: return "HIP runtime error";
        case VPM_ERR_NO_DEVICE: return "no GPU device";
    }
    return "unknown status";
}

const char* vpm_last_error(vpm_ctx* ctx) { return ctx ? ctx->last_error.c_str() : ""; }

vpm_status vpm_check_params(const vpm_params* p) {
    if (!p) return VPM_ERR_INVALID_ARG;
    if (!(std::isfinite(p->tol_x) && p->tol_x >= 0.0) || !(std::isfinite(p->tol_p) && p->tol_p >= 0.0))
        return VPM_ERR_INVALID_ARG;
    if (p->decide != VPM_DECIDE_FIXED && p->decide != VPM_DECIDE_FP64) return VPM_ERR_INVALID_ARG;
    if (p->decide == VPM_DECIDE_FIXED && (p->tol_x >= 128.0 || p->tol_p >= 128.0)) return VPM_ERR_INVALID_ARG;
    if (p->n_min_cell < 0) return VPM_ERR_INVALID_ARG;
    if (p->min_subset < 1 || p->min_subset > NMAX_BIG) return VPM_ERR_INVALID_ARG;
    if (p->merge_mode != VPM_MERGE_PAIR && p->merge_mode != VPM_MERGE_CENTROID) return VPM_ERR_INVALID_ARG;
    if (p->merge_mode == VPM_MERGE_PAIR && p->min_subset < 2) return VPM_ERR_INVALID_ARG;
    for (int a = 0; a < 3; ++a) if (!finite_pos(p->cell_len[a])) return VPM_ERR_INVALID_ARG;
    if (!(std::isfinite(p->mass) && p->mass >= 0.0)) return VPM_ERR_INVALID_ARG;
    if (p->dtype != VPM_F32 && p->dtype != VPM_F64) return VPM_ERR_INVALID_ARG;
    if (p->axis_rule != VPM_AXIS_RAW && p->axis_rule != VPM_AXIS_NORMALISED) return VPM_ERR_INVALID_ARG;
    return VPM_OK;
}

vpm_status vpm_create(vpm_ctx** out, int device) {
    if (!out) return VPM_ERR_INVALID_ARG;
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || n <= 0) return VPM_ERR_NO_DEVICE;
    if (device < 0 || device >= n) return VPM_ERR_INVALID_ARG;
    vpm_ctx* c = new vpm_ctx();
    c->device = device;
    hipError_t e = hipSetDevice(device);
    if (e != hipSuccess) { delete c; return VPM_ERR_HIP; }
    hipDeviceGetAttribute(&c->cu_count, hipDeviceAttributeMultiprocessorCount, device);
    if (c->cu_count <= 0) c->cu_count = 256;
    // persistent grids: as many workgroups as fit on the chip at once
    int* grids[6] = {&c->grid_a, &c->grid_b, &c->grid_c, &c->grid_big, &c->grid_s, &c->grid_d};
    for (int b = 0; b < 6; ++b) {
        int nb = 0;
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fixed_kernel_ptr(b), fixed_block_threads(b), fixed_lds_bytes(b));
        *grids[b] = c->cu_count * (nb > 0 ? nb : 1);
    }
    c->grid_fp64 = c->cu_count * 16;
    // side streams and events for running the size bins concurrently
    bool side_ok = true;
    for (int i = 0; i < 3 && side_ok; ++i)
        side_ok = hipStreamCreateWithFlags(&c->side[i], hipStreamNonBlocking) == hipSuccess &&
                  hipEventCreateWithFlags(&c->join[i], hipEventDisableTiming) == hipSuccess;
    if (side_ok) side_ok = hipEventCreateWithFlags(&c->fork, hipEventDisableTiming) == hipSuccess;
    if (!side_ok) {
        for (int i = 0; i < 3; ++i) {
            if (c->side[i]) hipStreamDestroy(c->side[i]);
            if (c->join[i]) hipEventDestroy(c->join[i]);
            c->side[i] = nullptr; c->join[i] = nullptr;
        }
        if (c->fork) hipEventDestroy(c->fork);
        c->fork = nullptr;
    }
    *out = c;
    return VPM_OK;
}

vpm_status vpm_destroy(vpm_ctx* ctx) {
    if (!ctx) return VPM_ERR_INVALID_ARG;
    hipSetDevice(ctx->device);
    hipDeviceSynchronize();
    free_ws(ctx->ws);
    for (auto& r : ctx->pending) { hipEventDestroy(r.a); hipEventDestroy(r.b); }
    for (auto e : ctx->pool) hipEventDestroy(e);
    for (int i = 0; i < 3; ++i) {
        if (ctx->side[i]) hipStreamDestroy(ctx->side[i]);
        if (ctx->join[i]) hipEventDestroy(ctx->join[i]);
    }
    if (ctx->fork) hipEventDestroy(ctx->fork);
    delete ctx;
    return VPM_OK;
}

vpm_status vpm_reserve(vpm_ctx* ctx, int64_t max_particles, int64_t max_cells) {
    if (!ctx || max_particles < 0 || max_cells < 0) return VPM_ERR_INVALID_ARG;
    if (max_particles <= ctx->ws.cap_particles && max_cells <= ctx->ws.cap_cells && ctx->ws.counters)
        return VPM_OK;
    hipSetDevice(ctx->device);
    hipDeviceSynchronize();
    const int64_t np = std::max<int64_t>(max_particles, ctx->ws.cap_particles) + 1;
    const int64_t nc = std::max<int64_t>(max_cells, ctx->ws.cap_cells) + 1;
    free_ws(ctx->ws);
    Workspace& ws = ctx->ws;
    hipError_t e = hipSuccess;
    auto alloc = [&](void** p, size_t bytes) {
        if (e != hipSuccess) return;
        e = hipMalloc(p, bytes ? bytes : 16);
    };
    for (int f = 0; f < 7; ++f) alloc(&ws.tmp[f], (size_t)np * 8);
    alloc((void**)&ws.out_count, (size_t)nc * 8);
    alloc((void**)&ws.cell_mode, (size_t)nc);
    for (int q = 0; q < Q_COUNT; ++q) alloc((void**)&ws.queue[q], (size_t)nc * 4);
    for (int k = 0; k < BIGQ_CLASSES; ++k) alloc((void**)&ws.bigq[k], (size_t)nc * 4);
    alloc((void**)&ws.counters, 4096);
    alloc((void**)&ws.flags, 256);
    alloc((void**)&ws.scan_blocks, (size_t)(nc / 4096 + 2) * 8);
    // the large-cell kernel: cell-wide arrays by input position, per-cell records, and a task ring
    // with room for every task that can be queued at once (queued tasks are disjoint subsets of at
    // least fixed_task_min() particles)
    alloc(&ws.big_rec, (size_t)np * 16);
    alloc((void**)&ws.big_pyz, (size_t)np * 4);
    alloc((void**)&ws.big_idx0, (size_t)np * 4);
    alloc((void**)&ws.big_idx1, (size_t)np * 4);
    alloc((void**)&ws.big_emit, (size_t)(np + 1) * 4);
    alloc((void**)&ws.big_info, (size_t)np);
    alloc(&ws.big_cells, (size_t)nc * (size_t)fixed_big_cell_bytes());
    ws.ring_size = np / fixed_task_min() + 1024;
    alloc(&ws.big_tasks, (size_t)ws.ring_size * (size_t)fixed_big_task_bytes());
    alloc((void**)&ws.big_ready, (size_t)ws.ring_size * 4);
    if (e == hipSuccess) e = hipMemset(ws.big_ready, 0, (size_t)ws.ring_size * 4);
    ws.big_wgs = ctx->grid_big;
    alloc(&ws.big_lists, (size_t)ws.big_wgs * (size_t)fixed_big_lists_bytes());
    alloc((void**)&ws.big_sched, (size_t)ws.big_wgs * (size_t)fixed_big_sched_bytes());
    // subsets above 65,536 particles split by several workgroups: over one call, every level of such
    // subsets holds at most np / 65,536 of them (disjoint), and there are at most 8 levels (cells of up
    // to 2^24); a call that runs out falls back to one workgroup per subset
    ws.jobs_cap = (int32_t)(2 * (np / 65536) + 256);
    ws.chunks_cap = (int32_t)(9 * (np / 65536) + 256);
    alloc(&ws.big_jobs, (size_t)ws.jobs_cap * (size_t)fixed_wide_job_bytes());
    alloc(&ws.big_chunks, (size_t)ws.chunks_cap * (size_t)fixed_wide_chunk_bytes());
    alloc((void**)&ws.perm2, (size_t)np * 2 * 4);
    alloc((void**)&ws.stack, (size_t)np * 8);
    if (e == hipSuccess) e = hipMemset(ws.counters, 0, 4096);
    if (e == hipSuccess) e = hipMemset(ws.flags, 0, 256);
    if (e != hipSuccess) {
        free_ws(ws);
        return hip_fail(ctx, e, "vpm_reserve");
    }
    ws.cap_particles = np - 1;
    ws.cap_cells = nc - 1;
    return VPM_OK;
}

vpm_status vpm_run(vpm_ctx* ctx, const vpm_soa* in, const int64_t* cell_off, int64_t n_cells,
                   int64_t n_particles, const vpm_params* p, vpm_soa* out, int64_t* out_off,
                   int64_t* out_total, hipStream_t stream) {
    return run_impl(ctx, in, cell_off, n_cells, n_particles, p, nullptr, nullptr, 0, out, out_off, out_total,
                    stream);
}

vpm_status vpm_run_species(vpm_ctx* ctx, const vpm_soa* in, const int64_t* cell_off, int64_t n_cells,
                           int64_t n_particles, const vpm_params* p, const uint8_t* cell_species,
                           const double* species_mass, int32_t n_species, vpm_soa* out, int64_t* out_off,
                           int64_t* out_total, hipStream_t stream) {
    if (!species_mass || n_species < 1 || n_species > VPM_MAX_SPECIES) return VPM_ERR_INVALID_ARG;
    if (!cell_species && n_cells > 0) return VPM_ERR_INVALID_ARG;
    for (int k = 0; k < n_species; ++k)
        if (!(std::isfinite(species_mass[k]) && species_mass[k] >= 0.0)) return VPM_ERR_INVALID_ARG;
    return run_impl(ctx, in, cell_off, n_cells, n_particles, p, cell_species, species_mass, n_species, out,
                    out_off, out_total, stream);
}

vpm_status vpm_partition(vpm_ctx* ctx, const vpm_soa* in, const int64_t* cell_off, int64_t n_cells,
                         int64_t n_particles, const vpm_params* p, int32_t* perm, int32_t* subset_id,
                         int32_t* n_subsets, hipStream_t stream) {
    vpm_status st = common_checks(ctx, in, cell_off, n_cells, n_particles, p);
    if (st != VPM_OK) return st;
    if (!perm || !subset_id || !n_subsets) return VPM_ERR_INVALID_ARG;
    hipSetDevice(ctx->device);
    LaunchCfg lc = make_cfg(ctx, stream);
    hipError_t e = launch_bin(ctx->ws, lc, cell_off, n_cells, n_particles, p->n_min_cell,
                              bin_limits(ctx, p->decide == VPM_DECIDE_FIXED ? NMAX_WIDE : NMAX_BIG));
    if (e != hipSuccess) return hip_fail(ctx, e, "bin");
    if (p->decide == VPM_DECIDE_FIXED)
        e = p->dtype == VPM_F32
                ? launch_fixed_cells(ctx->ws, lc, soa32(in), cell_off, fixed_params(p, ctx->tune), 1, perm, subset_id, n_subsets)
                : launch_fixed_cells(ctx->ws, lc, soa64(in), cell_off, fixed_params(p, ctx->tune), 1, perm, subset_id, n_subsets);
    else
        e = launch_fp64_cells(ctx->ws, lc, soa64(in), cell_off, n_cells, fp64_params(p), 1, perm, subset_id,
                              n_subsets);
    if (e != hipSuccess) return hip_fail(ctx, e, "cells");
    e = launch_identity(ctx->ws, lc, cell_off, n_particles, perm, subset_id, n_subsets);
    if (e != hipSuccess) return hip_fail(ctx, e, "identity");
    return VPM_OK;
}

vpm_status vpm_merge(vpm_ctx* ctx, const vpm_soa* in, const int64_t* cell_off, int64_t n_cells,
                     int64_t n_particles, const vpm_params* p, const int32_t* perm, const int32_t* subset_id,
                     const int32_t* n_subsets, vpm_soa* out, int64_t* out_off, int64_t* out_total,
                     hipStream_t stream) {
    vpm_status st = common_checks(ctx, in, cell_off, n_cells, n_particles, p);
    if (st != VPM_OK) return st;
    if (!perm || !subset_id || !n_subsets || check_soa(out) != VPM_OK || !out_off || !out_total)
        return VPM_ERR_INVALID_ARG;
    hipSetDevice(ctx->device);
    LaunchCfg lc = make_cfg(ctx, stream);
    hipError_t e = launch_bin(ctx->ws, lc, cell_off, n_cells, n_particles, p->n_min_cell, bin_limits(ctx, NMAX_BIG));
    if (e != hipSuccess) return hip_fail(ctx, e, "bin");
    if (p->decide == VPM_DECIDE_FIXED)
        e = p->dtype == VPM_F32
                ? launch_fixed_merge(ctx->ws, lc, soa32(in), cell_off, fixed_params(p, ctx->tune), perm, subset_id, n_subsets)
                : launch_fixed_merge(ctx->ws, lc, soa64(in), cell_off, fixed_params(p, ctx->tune), perm,
                               subset_id, n_subsets);
    else
        e = launch_fp64_merge(ctx->ws, lc, soa64(in), cell_off, n_cells, fp64_params(p), perm, subset_id,
                              n_subsets);
    if (e != hipSuccess) return hip_fail(ctx, e, "merge");
    e = launch_scan_offsets(ctx->ws, lc, n_cells, n_particles, out_off, out_total);
    if (e != hipSuccess) return hip_fail(ctx, e, "scan");
    const void* ins[7] = {in->x, in->y, in->z, in->px, in->py, in->pz, in->w};
    void* outs[7] = {out->x, out->y, out->z, out->px, out->py, out->pz, out->w};
    e = launch_scatter(ctx->ws, lc, cell_off, n_cells, n_particles, out_off, ins, outs, elem_in(p), elem_out(p));
    if (e != hipSuccess) return hip_fail(ctx, e, "scatter");
    return VPM_OK;
}

vpm_status vpm_blind(vpm_ctx* ctx, const vpm_soa* in, const int64_t* cell_off, int64_t n_cells,
                     int64_t n_particles, const vpm_params* p, double alpha, uint64_t seed, vpm_soa* out,
                     int64_t* out_off, int64_t* out_total, int32_t* group, hipStream_t stream) {
    vpm_status st = common_checks(ctx, in, cell_off, n_cells, n_particles, p);
    if (st != VPM_OK) return st;
    if (p->decide != VPM_DECIDE_FIXED) return VPM_ERR_UNSUPPORTED;
    if (!(std::isfinite(alpha) && alpha >= 0.0)) return VPM_ERR_INVALID_ARG;
    if (check_soa(out) != VPM_OK || !out_off || !out_total) return VPM_ERR_INVALID_ARG;
    hipSetDevice(ctx->device);
    LaunchCfg lc = make_cfg(ctx, stream);
    const FixedParams fp = fixed_params(p, ctx->tune);
    hipError_t e = p->dtype == VPM_F32
                       ? launch_fixed_blind(ctx->ws, lc, soa32(in), cell_off, n_cells, n_particles, fp, alpha, seed,
                                            p->n_min_cell, group)
                       : launch_fixed_blind(ctx->ws, lc, soa64(in), cell_off, n_cells, n_particles, fp, alpha, seed,
                                            p->n_min_cell, group);
    if (e != hipSuccess) return hip_fail(ctx, e, "blind");
    e = launch_scan_offsets(ctx->ws, lc, n_cells, n_particles, out_off, out_total);
    if (e != hipSuccess) return hip_fail(ctx, e, "scan");
    const void* ins[7] = {in->x, in->y, in->z, in->px, in->py, in->pz, in->w};
    void* outs[7] = {out->x, out->y, out->z, out->px, out->py, out->pz, out->w};
    e = launch_scatter(ctx->ws, lc, cell_off, n_cells, n_particles, out_off, ins, outs, elem_in(p), 4);
    if (e != hipSuccess) return hip_fail(ctx, e, "scatter");
    return VPM_OK;
}

vpm_status vpm_check_tuning(const vpm_tuning* t) {
    if (!t) return VPM_ERR_INVALID_ARG;
    if (t->ppl != 8 && t->ppl != 16 && t->ppl != 32) return VPM_ERR_INVALID_ARG;
    if (t->bin_a_max < 1 || t->bin_a_max > NMAX_A) return VPM_ERR_INVALID_ARG;
    if (t->bin_b_max < t->bin_a_max || t->bin_b_max > NMAX_B) return VPM_ERR_INVALID_ARG;
    if (t->bin_c_max < t->bin_b_max || t->bin_c_max > NMAX_C) return VPM_ERR_INVALID_ARG;
    if (t->concurrent_bins < 0 || t->concurrent_bins > 2) return VPM_ERR_INVALID_ARG;
    if (t->bin_s_max < 0 || t->bin_s_max > SMALL_MAX) return VPM_ERR_INVALID_ARG;
    if (t->exact_decisions != 0 && t->exact_decisions != 1) return VPM_ERR_INVALID_ARG;
    if (t->bin_d_max < t->bin_a_max || t->bin_d_max > NMAX_D || t->bin_d_max > t->bin_b_max) return VPM_ERR_INVALID_ARG;
    return VPM_OK;
}

vpm_status vpm_get_tuning(vpm_ctx* ctx, vpm_tuning* t) {
    if (!ctx || !t) return VPM_ERR_INVALID_ARG;
    *t = ctx->tune;
    return VPM_OK;
}

vpm_status vpm_set_tuning(vpm_ctx* ctx, const vpm_tuning* t) {
    if (!ctx) return VPM_ERR_INVALID_ARG;
    vpm_status st = vpm_check_tuning(t);
    if (st != VPM_OK) return st;
    ctx->tune = *t;
    return VPM_OK;
}

vpm_status vpm_autotune(vpm_ctx* ctx, const vpm_soa* in, const int64_t* cell_off, int64_t n_cells,
                        int64_t n_particles, const vpm_params* p, vpm_soa* out, int64_t* out_off,
                        int64_t* out_total, hipStream_t stream, vpm_tuning* best) {
    vpm_status st = common_checks(ctx, in, cell_off, n_cells, n_particles, p);
    if (st != VPM_OK) return st;
    if (p->decide != VPM_DECIDE_FIXED) return VPM_ERR_UNSUPPORTED;
    if (check_soa(out) != VPM_OK || !out_off || !out_total) return VPM_ERR_INVALID_ARG;
    hipSetDevice(ctx->device);
    const bool was_profiling = ctx->profiling;
    const vpm_tuning was_tuned = ctx->tune;        // restored if a trial fails
    ctx->profiling = false;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        if (e0) hipEventDestroy(e0);
        ctx->profiling = was_profiling;
        return hip_fail(ctx, hipGetLastError(), "vpm_autotune");
    }
    // time one configuration: one untimed run, then the best of `reps` samples, each the mean of
    // three back-to-back runs (the steady state a caller's loop of events sees; a lone event after
    // a synchronisation runs 1-2 % slower and less repeatably)
    auto time_cfg = [&](const vpm_tuning& t, float& ms, int reps) -> vpm_status {
        ctx->tune = t;
        constexpr int BATCH = 3;
        float bestms = 1e30f;
        for (int r = 0; r <= reps; ++r) {
            const int runs = r == 0 ? 1 : BATCH;
            hipEventRecord(e0, stream);
            for (int k = 0; k < runs; ++k) {
                vpm_status s = vpm_run(ctx, in, cell_off, n_cells, n_particles, p, out, out_off, out_total, stream);
                if (s != VPM_OK) return s;
            }
            hipEventRecord(e1, stream);
            hipError_t e = hipEventSynchronize(e1);
            if (e != hipSuccess) return hip_fail(ctx, e, "vpm_autotune");
            float m = 0.f;
            hipEventElapsedTime(&m, e0, e1);
            if (r > 0 && m / runs < bestms) bestms = m / runs;
        }
        ms = bestms;
        return VPM_OK;
    };
    const vpm_tuning dflt = {16, NMAX_A, NMAX_B, NMAX_C, 0, 128, was_tuned.exact_decisions, NMAX_D};
    vpm_tuning cur = dflt;
    float cur_ms = 0.f;
    st = time_cfg(cur, cur_ms, 3);
    // coordinate search: each parameter in turn over its candidates, keeping the others; a second
    // pass when the first changed something.  Concurrency goes first: it changes which bin limits
    // are best more than the limits change whether concurrency pays.
    const int ppls[3] = {8, 16, 32};
    const int as[5] = {320, 384, 448, 512, NMAX_A};
    const int bs[3] = {1024, 1536, NMAX_B};
    const int cs[3] = {2560, 3456, NMAX_C};
    const int conc[3] = {0, 1, 2};
    const int ss[5] = {0, 32, 64, 128, SMALL_MAX};
    const int ds[3] = {0, 864, NMAX_D};            // 0: no two-wavefront bin (bin_d_max = bin_a_max)
    bool changed = true;
    for (int pass = 0; pass < 2 && changed && st == VPM_OK; ++pass) {
        changed = false;
        const int order[7] = {4, 0, 1, 6, 2, 3, 5};
        for (int di = 0; di < 7 && st == VPM_OK; ++di) {
            const int dim = order[di];
            const int* cand = dim == 0 ? ppls : dim == 1 ? as : dim == 2 ? bs : dim == 3 ? cs : dim == 4 ? conc
                            : dim == 5 ? ss : ds;
            const int nc = dim == 1 || dim == 5 ? 5 : 3;
            for (int k = 0; k < nc && st == VPM_OK; ++k) {
                vpm_tuning t = cur;
                if (dim == 0) t.ppl = cand[k];
                else if (dim == 1) t.bin_a_max = cand[k];
                else if (dim == 2) t.bin_b_max = cand[k];
                else if (dim == 3) t.bin_c_max = cand[k];
                else if (dim == 4) t.concurrent_bins = cand[k];
                else if (dim == 5) t.bin_s_max = cand[k];
                else t.bin_d_max = cand[k] == 0 ? t.bin_a_max : cand[k];
                // keep the two-wavefront bin's limit inside the others' when they move
                if (dim != 6) t.bin_d_max = std::max(t.bin_a_max, std::min(t.bin_d_max, t.bin_b_max));
                if (vpm_check_tuning(&t) != VPM_OK) continue;
                if (t.ppl == cur.ppl && t.bin_a_max == cur.bin_a_max && t.bin_b_max == cur.bin_b_max &&
                    t.bin_c_max == cur.bin_c_max && t.concurrent_bins == cur.concurrent_bins &&
                    t.bin_s_max == cur.bin_s_max && t.bin_d_max == cur.bin_d_max)
                    continue;
                float ms = 0.f;
                st = time_cfg(t, ms, 3);
                if (st == VPM_OK && ms < cur_ms * 0.99f) { cur = t; cur_ms = ms; changed = true; }
            }
        }
    }
    // a search step accepts a candidate on the best of three samples, so a lucky timing can leave
    // it on a configuration no faster than the default: keep the choice only if it still wins by
    // 1 % on the best of six samples of each
    const bool moved = cur.ppl != dflt.ppl || cur.bin_a_max != dflt.bin_a_max || cur.bin_b_max != dflt.bin_b_max ||
                       cur.bin_c_max != dflt.bin_c_max || cur.concurrent_bins != dflt.concurrent_bins ||
                       cur.bin_s_max != dflt.bin_s_max || cur.bin_d_max != dflt.bin_d_max;
    if (st == VPM_OK && moved) {
        float ms_cur = 0.f, ms_dflt = 0.f;
        st = time_cfg(cur, ms_cur, 6);
        if (st == VPM_OK) st = time_cfg(dflt, ms_dflt, 6);
        if (st == VPM_OK && !(ms_cur < ms_dflt * 0.99f)) cur = dflt;
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    ctx->profiling = was_profiling;
    if (st != VPM_OK) {
        ctx->tune = was_tuned;
        return st;
    }
    ctx->tune = cur;
    if (best) *best = cur;
    // leave the chosen configuration's result in the outputs
    return vpm_run(ctx, in, cell_off, n_cells, n_particles, p, out, out_off, out_total, stream);
}

vpm_status vpm_device_status(vpm_ctx* ctx, uint32_t* flags_out, int clear) {
    if (!ctx || !flags_out) return VPM_ERR_INVALID_ARG;
    if (!ctx->ws.flags) { *flags_out = 0; return VPM_OK; }
    hipSetDevice(ctx->device);
    hipError_t e = hipDeviceSynchronize();
    if (e == hipSuccess) e = hipMemcpy(flags_out, ctx->ws.flags, 4, hipMemcpyDeviceToHost);
    if (e == hipSuccess && clear) e = hipMemset(ctx->ws.flags, 0, 4);
    if (e != hipSuccess) return hip_fail(ctx, e, "vpm_device_status");
    return VPM_OK;
}

vpm_status vpm_profile_enable(vpm_ctx* ctx, int enable) {
    if (!ctx) return VPM_ERR_INVALID_ARG;
    ctx->profiling = enable != 0;
    return VPM_OK;
}

vpm_status vpm_profile_read(vpm_ctx* ctx, int max_kernels, char names[][48], int64_t* launches,
                            double* total_ms, int* n_out, int reset) {
    if (!ctx || !n_out || max_kernels < 0) return VPM_ERR_INVALID_ARG;
    hipSetDevice(ctx->device);
    for (auto& r : ctx->pending) {
        hipError_t e = hipEventSynchronize(r.b);
        if (e != hipSuccess) return hip_fail(ctx, e, "vpm_profile_read");
        float ms = 0.f;
        hipEventElapsedTime(&ms, r.a, r.b);
        ctx->kms[r.kernel] += ms;
        ctx->klaunch[r.kernel] += 1;
        ctx->pool.push_back(r.a);
        ctx->pool.push_back(r.b);
    }
    ctx->pending.clear();
    const int n = (int)ctx->knames.size();
    *n_out = n;
    for (int i = 0; i < n && i < max_kernels; ++i) {
        if (names) { std::strncpy(names[i], ctx->knames[i].c_str(), 47); names[i][47] = 0; }
        if (launches) launches[i] = ctx->klaunch[i];
        if (total_ms) total_ms[i] = ctx->kms[i];
    }
    if (reset) {
        for (auto& v : ctx->klaunch) v = 0;
        for (auto& v : ctx->kms) v = 0.0;
    }
    return VPM_OK;
}

}  // extern "C"

/*
 * vpm.h -- C ABI of the Voronoi particle-merging library for AMD Instinct MI355X (gfx950).
 *
 * The operation (Luu, Tueckmantel, Pukhov, "Voronoi Particle Merging Algorithm for PIC
 * Codes", Sec. "Algorithm", Steps 1-7): for every simulation cell holding more than
 * N_min macroparticles, split the cell's particles recursively in 6-D phase space
 * (x, y, z, px, py, pz).  A subset is cut by the hyperplane through its weighted centroid
 * perpendicular to the axis whose coefficient of variation is largest (Steps 4-5; the CV is
 * sigma/L for positions and sigma/|P| for momenta, Eqs. cv_x and cv_p), until all six CVs of
 * every subset are within the tolerances T_X and T_P (Step 3).  Each finished subset is then
 * replaced by merged particles (Step 7): its centroid (weight and momentum conserved), or a
 * pair of half-weight particles at the centroid whose momenta P +- delta also conserve the
 * subset's total energy (the two-particle merge the paper proposes in its remarks).
 *
 * Conventions shared by every entry point
 *  - Particles are a structure of arrays (vpm_soa) of 7 DEVICE arrays x,y,z,px,py,pz,w of one
 *    element type (vpm_params.dtype), sorted by cell.  Momenta are in units of m_e c.
 *  - cell_off is a DEVICE array of n_cells+1 int64 offsets: cell c owns particles
 *    cell_off[c] .. cell_off[c+1]-1; cell_off[0] = 0 and cell_off[n_cells] <= n_particles.
 *    n_particles is the length of the particle (and output) arrays; particles from
 *    cell_off[n_cells] on are ignored.  Because the population size is read from the device, one
 *    captured sequence of calls (a HIP graph) can be replayed for merge events whose particle
 *    counts differ, as long as the buffers, n_cells and n_particles stay the same.
 *  - All device buffers are owned by the caller.  Entry points enqueue work on `stream` and
 *    return without synchronising; results are valid once the stream has completed.  They
 *    never allocate: the context's workspace is allocated by vpm_reserve only.  vpm_run,
 *    vpm_partition and vpm_merge may be captured into a HIP graph (with profiling disabled);
 *    internally they fork to the context's side streams and join back before returning.
 *  - A context may be used by one host thread and one stream at a time.
 *  - Host-checkable argument errors are returned immediately and nothing is enqueued.
 *    Data-dependent problems found on the device (bad values, offsets that decrease,
 *    cells above the largest size, below) set sticky flags read by vpm_device_status; the
 *    affected cells are passed through unchanged.
 *
 * Decision modes (vpm_params.decide)
 *  VPM_DECIDE_FIXED  every split decision is an exact integer function of per-cell fixed-point
 *                    codes (weights 2^-15 of the cell's largest weight, positions 2^-16 of
 *                    the cell length, momenta 2^-22 of the cell's largest |p| per axis, all
 *                    taken from the FP32 values), so partitions are bit-reproducible across
 *                    launch shapes and runs.  Tolerances are used as round(T * 2^24) / 2^24 and
 *                    must be < 128.  dtype VPM_F32 or VPM_F64: FP64 particles are rounded to FP32
 *                    (to nearest) as they are loaded, so both give identical results; the output
 *                    particles are FP32 either way.  Cells of up to 2^24 particles (a whole box).
 *  VPM_DECIDE_FP64   the paper's statistics evaluated literally in IEEE double, one workgroup
 *                    per cell.  Requires dtype VPM_F64.  Cells of up to 65,536 particles.
 */
#ifndef VPM_H
#define VPM_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    VPM_OK = 0,
    VPM_ERR_INVALID_ARG = -1,   /* null pointer, negative size, tolerance/length out of range */
    VPM_ERR_UNSUPPORTED = -2,   /* a dtype/decide combination the library does not implement */
    VPM_ERR_CAPACITY = -3,      /* more particles or cells than vpm_reserve provided for       */
    VPM_ERR_HIP = -4,           /* a HIP runtime call failed (message: vpm_last_error)         */
    VPM_ERR_NO_DEVICE = -5      /* no usable GPU                                               */
} vpm_status;

typedef enum { VPM_F32 = 0, VPM_F64 = 1 } vpm_dtype;
typedef enum { VPM_DECIDE_FIXED = 0, VPM_DECIDE_FP64 = 1 } vpm_decide;
typedef enum { VPM_MERGE_PAIR = 0, VPM_MERGE_CENTROID = 1 } vpm_merge_mode;
/* Step 4's axis: the largest raw CV (the paper's rule, default), or the largest CV over its own
 * tolerance, Delta_l / T_l (a CV > 0 over a zero tolerance counts as infinite; ties still go to the
 * lowest axis).  Step 3's test is the same under both. */
typedef enum { VPM_AXIS_RAW = 0, VPM_AXIS_NORMALISED = 1 } vpm_axis_rule;

/* Sticky device flags (vpm_device_status). */
#define VPM_FLAG_BAD_VALUE      0x1u  /* w <= 0, NaN or Inf in a cell: that cell passed through     */
#define VPM_FLAG_OUT_OF_CELL    0x2u  /* a particle lay more than one cell length from the cell's
                                         lowest coordinate; its position code was clamped (FIXED)  */
#define VPM_FLAG_CELL_TOO_LARGE 0x4u  /* a cell above the largest size: passed through (2^24 =
                                         16,777,216 particles for vpm_run, vpm_run_species and
                                         vpm_partition with fixed-point decisions; 65,536 for
                                         the FP64 form, vpm_merge and vpm_blind)                */
#define VPM_FLAG_BAD_OFFSETS    0x8u  /* cell_off decreasing, not starting at 0, or past n_particles;
                                         a cell whose own range is invalid is passed through, but
                                         cells whose ranges overlap make the whole output
                                         unspecified (out_off and out_total are clamped to
                                         n_particles and nothing is written past it)              */
#define VPM_FLAG_BAD_PARTITION  0x10u /* vpm_merge: a cell's perm/subset_id/n_subsets is not a
                                         partition of that cell; the cell was copied unchanged     */
#define VPM_FLAG_BAD_SPECIES    0x20u /* vpm_run_species: a cell's species index is not below
                                         n_species; the cell was copied unchanged                  */

/* Largest number of species in one vpm_run_species call. */
#define VPM_MAX_SPECIES 8

typedef struct {
    double  tol_x;        /* T_X >= 0: position tolerance (Step 3)                            */
    double  tol_p;        /* T_P >= 0: momentum tolerance (Step 3)                            */
    int32_t n_min_cell;   /* N_min >= 0: a cell is merged only if it holds more particles     */
    int32_t min_subset;   /* >= 1 (>= 2 for PAIR): finished subsets smaller than this are not
                             merged; their particles are copied unchanged                     */
    double  cell_len[3];  /* L_x, L_y, L_z > 0: the cell side lengths in Delta_X = sigma/L     */
    double  mass;         /* particle mass in m_e units (1 for e-/e+, 0 for photons): the
                             energy of a particle is sqrt(mass^2 + |p|^2)                     */
    int32_t merge_mode;   /* vpm_merge_mode */
    int32_t decide;       /* vpm_decide */
    int32_t dtype;        /* vpm_dtype of every particle array */
    int32_t axis_rule;    /* vpm_axis_rule */
} vpm_params;

typedef struct { void *x, *y, *z, *px, *py, *pz, *w; } vpm_soa;   /* device pointers */

typedef struct vpm_ctx vpm_ctx;

/* Create a context on HIP device `device`.  Returns VPM_ERR_NO_DEVICE if there is none. */
vpm_status vpm_create(vpm_ctx **ctx, int device);

/* Free the context and its workspace.  Waits for work the context enqueued. */
vpm_status vpm_destroy(vpm_ctx *ctx);

/* Allocate the context's device workspace for up to max_particles particles and max_cells
 * cells per call (about 110 bytes per particle plus 160 bytes per cell).  The only call that
 * allocates device memory.  May be called again to grow; it synchronises the device. */
vpm_status vpm_reserve(vpm_ctx *ctx, int64_t max_particles, int64_t max_cells);

/* Host-only validation of a parameter block (no device needed). */
vpm_status vpm_check_params(const vpm_params *p);

/* The fused hot path: partition every cell (Steps 1-6) and replace its finished subsets
 * (Step 7).  Output, per cell in cell order: the cell's final subsets in depth-first order
 * (the lower side V1 of each cut before the upper side V2); a merged subset emits 1 particle
 * (CENTROID) or 2 (PAIR, the +delta one first); a subset below min_subset emits its particles
 * unchanged in input order; a cell with N <= N_min, or one flagged on the device, is copied
 * unchanged.
 *   out        7 device arrays with capacity >= n_particles, FP32 with VPM_DECIDE_FIXED and FP64 with
 *              VPM_DECIDE_FP64
 *   out_off    device int64[n_cells+1]: exclusive prefix of the per-cell output counts
 *   out_total  device int64 scalar: out_off[n_cells]                                         */
vpm_status vpm_run(vpm_ctx *ctx, const vpm_soa *in, const int64_t *cell_off, int64_t n_cells,
                   int64_t n_particles, const vpm_params *p, vpm_soa *out, int64_t *out_off,
                   int64_t *out_total, hipStream_t stream);

/* Several particle species in one launch, e.g. the electrons, positrons and photons that the
 * paper's shower simulation merges (Sec. "Simulation", subsection "Magnetic Shower"): every cell holds particles
 * of one species, and only the energy sqrt(m^2 + |p|^2) of Step 7 depends on the mass.
 *   cell_species  device uint8[n_cells]: species index s of each cell
 *   species_mass  host double[n_species]: mass of each species in m_e units (finite, >= 0);
 *                 read during the call only
 *   n_species     1 ... VPM_MAX_SPECIES
 * p->mass is not used.  The result equals vpm_run's on the cells of each species with
 * p->mass = species_mass[s].  A cell with s >= n_species is copied unchanged and raises
 * VPM_FLAG_BAD_SPECIES.  Other arguments, output and errors as vpm_run (FIXED and FP64
 * decisions).                                                                                */
vpm_status vpm_run_species(vpm_ctx *ctx, const vpm_soa *in, const int64_t *cell_off, int64_t n_cells,
                           int64_t n_particles, const vpm_params *p, const uint8_t *cell_species,
                           const double *species_mass, int32_t n_species, vpm_soa *out,
                           int64_t *out_off, int64_t *out_total, hipStream_t stream);

/* Partition only (Steps 1-6).
 *   perm       device int32[n_particles]: for each slot of cell c's range, the global index of
 *              the input particle in that slot; final subsets are contiguous and in depth-first
 *              order, members in input order; identity for cells that are not processed
 *   subset_id  device int32[n_particles]: cell-local ordinal of the final subset of each slot,
 *              -1 for cells that are not processed
 *   n_subsets  device int32[n_cells]: number of final subsets per cell (0 if not processed)    */
vpm_status vpm_partition(vpm_ctx *ctx, const vpm_soa *in, const int64_t *cell_off,
                         int64_t n_cells, int64_t n_particles, const vpm_params *p,
                         int32_t *perm, int32_t *subset_id, int32_t *n_subsets,
                         hipStream_t stream);

/* Replacement only (Step 7), from a partition in vpm_partition's format: subsets of size
 * >= min_subset are merged, smaller ones copied.  Output as vpm_run.  In FIXED mode the
 * pair direction uses the cell's fixed-point codes, exactly as vpm_run does.                */
vpm_status vpm_merge(vpm_ctx *ctx, const vpm_soa *in, const int64_t *cell_off, int64_t n_cells,
                     int64_t n_particles, const vpm_params *p, const int32_t *perm,
                     const int32_t *subset_id, const int32_t *n_subsets, vpm_soa *out,
                     int64_t *out_off, int64_t *out_total, hipStream_t stream);

/* The blind method, the paper's comparison method (Sec. "Simulation", described before the
 * counter-propagating blocks; merging fraction alpha = 0.965 and 0.88 in Tables 1 and 2): in every
 * cell of N > N_min particles with ceil(alpha N) < N, pairs of particles picked at random are merged
 * until ceil(alpha N) remain.  A merge replaces two particles by one with their summed weight at
 * their weighted centroid in position and momentum (weight and momentum kept, energy not).
 *   Draws: Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC 2011), key (seed, 0), counter (t, c, 0, 0)
 *   for the t-th merge of cell c.  With M = N - t particles left, outputs r0, r1 pick slots
 *   i = r0 mod M and j = r1 mod (M - 1) (plus one if >= i): the group in slot j joins the group in
 *   slot i, and the last slot moves into slot j.  Output k of the cell is the group left in slot
 *   k: copied unchanged if it is one particle, else replaced by its centroid.
 *   alpha     >= 0 (finite); alpha >= 1 merges nothing
 *   group     device int32[n_particles] (may be NULL): the cell-local output ordinal of each input
 *             particle (its own index in untouched cells)
 * p: n_min_cell, mass and dtype (VPM_F32 only) are used; tolerances, min_subset, merge_mode and
 * decide are not (p must still pass vpm_check_params).  Output and errors as vpm_run; cells above
 * 65,536 particles are flagged VPM_FLAG_CELL_TOO_LARGE and copied.                               */
vpm_status vpm_blind(vpm_ctx *ctx, const vpm_soa *in, const int64_t *cell_off, int64_t n_cells,
                     int64_t n_particles, const vpm_params *p, double alpha, uint64_t seed, vpm_soa *out,
                     int64_t *out_off, int64_t *out_total, int32_t *group, hipStream_t stream);

/* Launch configuration of the fixed-point path (batching, not arithmetic: every configuration gives
 * bit-identical results).  A cell of n particles (n > N_min) is processed
 *   in a batch with other small cells by one wavefront (up to 16 cells, 512 particles, in LDS)
 *                                                  if n <= bin_s_max  (bin_s_max <= 256; 0: none)
 *   by one wavefront, working set in LDS          if n <= bin_a_max  (bin_a_max <= 576)
 *   two wavefronts, working set in LDS            if n <= bin_d_max  (bin_d_max <= 1144)
 *   four wavefronts, working set in LDS           if n <= bin_b_max  (bin_b_max <= 2288)
 *   eight wavefronts, working set in LDS          if n <= bin_c_max  (bin_c_max <= 4592)
 *   eight wavefronts, working set in global memory otherwise (n <= 2^24: a whole box may be one
 *     cell, the method's first subset (Sec. "Algorithm", the remark on merging globally); a
 *     subset above 65,536 particles is split by one workgroup on exact integer moments and its
 *     unfinished children are handed to other workgroups);
 * a subset of len particles is handled by a group of about len / ppl lanes (ppl = 8, 16 or 32;
 * at most 64 lanes).  Limits must satisfy 1 <= bin_a_max <= bin_d_max <= bin_b_max <= bin_c_max
 * (bin_d_max = bin_a_max: no two-wavefront bin).
 * concurrent_bins = 1 runs the large-cell, eight- and four-wavefront bins on the context's side
 * streams (forked from and joined back to the caller's stream) beside the others; 2 runs only the
 * two-wavefront bin on a side stream, beside the others one after another on the caller's stream
 * (for populations centred on the one-wavefront bin, whose few larger cells then overlap it); 0
 * runs every bin one after another on the caller's stream.
 * exact_decisions = 1 takes every Step 3-5 decision of the fixed-point path by the exact integer
 * rule (Sec. "Algorithm", Steps 3-5, on 128/256/320-bit moments recomputed from the codes) instead
 * of first trying the certified FP64 evaluation: slower, and by construction the same result; it
 * exists to cross-check that evaluation on whole populations.  0 (the default) is the fast form.
 * The autotuner keeps the value it finds in the context.                                         */
typedef struct {
    int32_t ppl;
    int32_t bin_a_max;
    int32_t bin_b_max;
    int32_t bin_c_max;
    int32_t concurrent_bins;
    int32_t bin_s_max;
    int32_t exact_decisions;
    int32_t bin_d_max;
} vpm_tuning;

/* Host-only validation of a tuning block (no device needed). */
vpm_status vpm_check_tuning(const vpm_tuning *t);

/* The context's current tuning (initially ppl 16, limits 576 / 1144 / 2288 / 4592, bins in sequence,
 * small-cell batches for cells of up to 128 particles). */
vpm_status vpm_get_tuning(vpm_ctx *ctx, vpm_tuning *t);
vpm_status vpm_set_tuning(vpm_ctx *ctx, const vpm_tuning *t);

/* Choose the tuning for a population: runs vpm_run with candidate configurations on the given
 * data (coordinate search over ppl, the bin limits, concurrent_bins and bin_s_max), times each on `stream` with HIP
 * events (best of three samples of three back-to-back runs), keeps the fastest in the context and
 * returns it in *best (host, may be NULL); the default tuning is kept unless the choice beats it
 * by 1 % on the best of six samples.  Leaves
 * vpm_run's result of the chosen configuration in out / out_off / out_total.  Synchronises
 * `stream`; cannot be captured in a graph.  Arguments as vpm_run (FIXED decisions only).      */
vpm_status vpm_autotune(vpm_ctx *ctx, const vpm_soa *in, const int64_t *cell_off, int64_t n_cells,
                        int64_t n_particles, const vpm_params *p, vpm_soa *out, int64_t *out_off,
                        int64_t *out_total, hipStream_t stream, vpm_tuning *best);

/* Read (and, if clear != 0, reset) the sticky device flags.  Synchronises the device. */
vpm_status vpm_device_status(vpm_ctx *ctx, uint32_t *flags_out, int clear);

/* Per-kernel timing of the context's launches, for benchmarking.  When enabled, every
 * internal kernel launch is bracketed by HIP events on the caller's stream.  vpm_profile_read
 * synchronises, and returns up to max_kernels entries: name, number of launches and total
 * milliseconds since the last reset.  Returns the number of kernels in *n_out.              */
vpm_status vpm_profile_enable(vpm_ctx *ctx, int enable);
vpm_status vpm_profile_read(vpm_ctx *ctx, int max_kernels, char names[][48], int64_t *launches,
                            double *total_ms, int *n_out, int reset);

/* Text for a status code; message of the last HIP failure in this context (or ""). */
const char *vpm_status_string(vpm_status st);
const char *vpm_last_error(vpm_ctx *ctx);

/* Limits of vpm_run_noalloc. */
#define VPM_NOALLOC_MAX_PARTICLES 524288
#define VPM_NOALLOC_MAX_CELLS     32768

/* vpm_run without a context, for callers that cannot allocate device memory (code being captured
 * into a HIP graph, serving loops and harnesses that forbid hipMalloc).  It allocates nothing: its
 * working memory is a fixed array of 48 MiB in the library's device code, one copy per GPU, held
 * until the process ends.  Runs on the current HIP device with vpm_create's default tuning and
 * gives results bit-identical to vpm_run's with that tuning.
 *   Only VPM_DECIDE_FIXED with dtype VPM_F32.  n_particles <= VPM_NOALLOC_MAX_PARTICLES and
 *   n_cells <= VPM_NOALLOC_MAX_CELLS, else VPM_ERR_CAPACITY before anything is enqueued.
 *   flags_out  device uint32 (may be NULL): this call's VPM_FLAG_* bits (cleared at its start).
 * Other arguments, output and errors as vpm_run.  Every call on one GPU uses that GPU's single
 * array: calls that overlap in time on one GPU (other streams, other host threads) race, so the
 * caller must order them.                                                                        */
vpm_status vpm_run_noalloc(const vpm_soa *in, const int64_t *cell_off, int64_t n_cells, int64_t n_particles,
                           const vpm_params *p, vpm_soa *out, int64_t *out_off, int64_t *out_total,
                           uint32_t *flags_out, hipStream_t stream);

/* Library build identification (target architecture and version). */
const char *vpm_version(void);

#ifdef __cplusplus
}
#endif

#endif /* VPM_H */

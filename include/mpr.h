/*
 * mpr.h -- C ABI of the gfx950 (MI355X) library for spatial prediction with the modified
 * planar rotator (MPR) model.
 *
 * The method (Lach, Borovsky, Zukovic, "Numerical Precision Effects on GPU Simulation of
 * Massive Spatial Data, Based on the Modified Planar Rotator Model"):
 *   Sec. 1-2   measured values on a 2-D grid are mapped onto spin angles phi in [0, 2 pi];
 *   Eq. (2)    H = -J sum_<ij> cos[q (phi_i - phi_j)], q in (0, 1/2], nearest neighbours;
 *   Sec. 2     the reduced temperature, the only parameter, is inferred from the incomplete
 *              data through the specific energy; a conditional Monte Carlo simulation with
 *              the hybrid algorithm (deterministic over-relaxation + Metropolis) then changes
 *              only the spins at prediction sites; the average over equilibrium
 *              configurations, mapped back, is the prediction;
 *   Sec. 2     the spins and the energy can be kept in double or single precision, and the
 *              functions evaluated in double precision or with hardware intrinsics
 *              (the X_S X_E X_F settings); Sec. 3 names 16-bit variables as the next step.
 *
 * Angles are stored in revolutions u = phi / 2 pi in [0, 1].  All steps run in this library's
 * HIP kernels on the stream given at creation.
 *
 * Conventions for every entry point:
 *   - Returns MPR_OK (0) or an mpr_status code; never aborts or throws across the ABI.
 *     mpr_last_error(ctx) holds a human-readable detail for the last failure.
 *   - A failed call leaves the context usable, except after MPR_EHIP (a HIP runtime error;
 *     destroy the context).
 *   - Pointers named *_dev are device pointers (hipMalloc / torch CUDA tensors) on the
 *     context's device; *_host are host pointers.  The caller owns every buffer it passes;
 *     inputs are read in stream order during the call and may be released after it returns.
 *   - Calls that return host values (mpr_infer_temperature with T_host, mpr_get_*)
 *     synchronise the stream; the others only enqueue work.
 *   - One context must not be used by two host threads at the same time.
 *
 * Batched layout: a context holds G grids (1 for mpr_create) and n_chains independent chains
 * per grid.  Grid g has H_g x W_g sites, row-major; packed arrays place the grids back to
 * back (offset_g = sum_{h<g} H_h W_h).  Per-chain arrays are [g][chain][H_g W_g].
 */
#ifndef MPR_H
#define MPR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MPR_ABI_VERSION 1

typedef struct mpr_ctx mpr_ctx;

typedef enum mpr_status {
    MPR_OK = 0,
    MPR_EINVAL = 1,      /* bad argument: q outside (0, 1/2], J <= 0, side < 2, mask value
                            not 0/1, non-finite sample value, negative sweep count, ... */
    MPR_ENOSAMPLE = 2,   /* fewer than two distinct sample values, or no bond joining two
                            sample sites (the sample energy is undefined) */
    MPR_EBIPARTITE = 3,  /* periodic boundary with an odd side (no checkerboard colouring) */
    MPR_ESTATE = 4,      /* call out of order: run before a temperature exists,
                            predictions before any averaging sweep, ... */
    MPR_ENOMEM = 5,      /* device or host allocation failed */
    MPR_EHIP = 6         /* HIP runtime error or a device-side time-out; context unusable */
} mpr_status;

/* storage of the spin angles (the paper's X_S, extended by two 16-bit formats: IEEE half, and
 * fixed point u = k / 32767 with a uniform resolution of 3.1e-5 of a turn) */
typedef enum mpr_precision { MPR_FP64 = 0, MPR_FP32 = 1, MPR_FP16 = 2, MPR_FIX16 = 3 } mpr_precision;
/* precision of the energy accumulation (X_E) and of the functions (X_F) */
typedef enum mpr_fprec { MPR_PREC_DEFAULT = -1, MPR_PREC_DOUBLE = 0, MPR_PREC_SINGLE = 1 } mpr_fprec;
typedef enum mpr_boundary { MPR_OPEN = 0, MPR_PERIODIC = 1 } mpr_boundary;

typedef struct mpr_config {
    double q;                 /* Eq. (2) modification parameter, (0, 1/2]              */
    double J;                 /* exchange coupling, > 0                                */
    int32_t precision;        /* mpr_precision: angle storage                          */
    int32_t energy_prec;      /* mpr_fprec (X_E); DEFAULT = double                     */
    int32_t func_prec;        /* mpr_fprec (X_F); DEFAULT = double for FP64 storage,
                                 single (hardware sin/cos/exp) otherwise; 16-bit
                                 storage needs single                               */
    int32_t boundary;         /* mpr_boundary; periodic needs even H and W % 4 == 0    */
    int32_t n_chains;         /* independent chains per grid, >= 1                     */
    int32_t grid_offset;      /* global index of this context's grid 0, >= 0: the Philox
                                 chain word of (grid g, chain c) is
                                 (grid_offset + g) * n_chains + c, so a grid gives the
                                 same bits alone or inside any batch (or shard)        */
    uint64_t seed;            /* Philox4x32-10 key                                     */
    double alpha0;            /* initial Metropolis window, fraction of a turn, (0, 1] */
    double acc_target;        /* acceptance rate the window control aims at, (0, 1)    */
    double T_min, T_max;      /* temperature clamp, 0 < T_min <= T_max                 */
    int32_t tile_rows;        /* rows per work item of the fused path, 0 = heuristic,
                                 -1 = autotune at load (with sweep_mode AUTO also the
                                 sweep path; see mpr_autotune)                       */
    int32_t graph_sweeps;     /* sweeps per captured HIP graph, 0 = automatic,
                                 -1 = launch kernels without graphs                   */
    int32_t sweep_mode;       /* mpr_sweep_mode: how a sweep visits the sites          */
    int32_t tile_shape;       /* tiled path's block shape: 0 = automatic (rule, or the
                                 autotuner with tile_rows = -1), 1 + mpr_tile_shape
                                 forces one (all but MPR_TILE_W4_BASE need
                                 single-precision functions, EINVAL otherwise)        */
    int32_t group_waves;      /* compacted path: list waves (64 prediction sites each) one
                                 wave sweeps per launch, 1 ... 32; 0 = automatic (as
                                 many as keep about 20 480 groups per colour, at most
                                 32); results do not depend on it                     */
    int32_t reserved[3];
} mpr_config;

/* Block shapes of the tiled path: waves per block and tile height (the base height is 16 rows,
 * 8 for 8-byte spins with single-precision functions; tall tiles have twice as many rows). */
typedef enum mpr_tile_shape {
    MPR_TILE_W4_BASE = 0, MPR_TILE_W8_TALL = 1, MPR_TILE_W4_TALL = 2, MPR_TILE_W8_BASE = 3
} mpr_tile_shape;

/* How a sweep visits the sites.
 * FUSED: one launch per sweep over every site in row blocks, both colours in one pass with halo
 *   recomputation; best when most sites are prediction sites and the grid is large.
 * SPARSE: two launches per sweep (one per colour) over lists of the prediction sites only, built
 *   at load, one wave per group of up to group_waves list waves of one (grid, chain); needs
 *   double-precision energy and grids with H < 65536 and ceil(ceil(W / 2) / 2) * 2 < 65536.
 * TILED: one launch per sweep, one block per tile of 128 columns staged in LDS with its halo
 *   (the block shape, mpr_tile_shape, unless forced or tuned: eight-wave blocks on tiles of 32
 *   rows, 16 with 8-byte spins, while the grids hold fewer than 2048 tiles of half that height;
 *   otherwise four-wave blocks on tiles of 16 rows, 8 with 8-byte spins; with double-precision
 *   functions always four-wave blocks on 16-row tiles); each colour's prediction sites are
 *   compacted into a list inside the block, and the colour-0 sites around the tile are
 *   recomputed; needs double-precision energy.
 * All three take identical decisions from identical states; SPARSE and TILED also sum the
 * energy identically (bitwise equal results), while FUSED groups the bonds differently, so its
 * temperature trajectories agree with theirs to rounding, not bitwise.
 * AUTO picks TILED when the energy is summed in double precision, sites x chains <= 1.5 * 2^20
 * (small grids, where a sweep is bound by latency: one launch instead of two) and either the
 * functions are evaluated in single precision or more than 60 % of the sites are prediction
 * sites; otherwise SPARSE when it is possible and either the functions are evaluated in double
 * precision with at most 60 % prediction sites, or at most 70 % and sites x chains <= 2^23, or
 * the angles are stored in 16 bits with at most 50 % prediction sites, or in FP32 with at most
 * 40 % prediction sites and sites x chains <= 2^23 (measured crossovers on MI355X); FUSED
 * otherwise.  The choice depends on the loaded data and
 * configuration only (or, with tile_rows = -1, on the autotuner's timing) and is fixed for the
 * context until the next load. */
typedef enum mpr_sweep_mode {
    MPR_SWEEP_AUTO = 0, MPR_SWEEP_FUSED = 1, MPR_SWEEP_SPARSE = 2, MPR_SWEEP_TILED = 3
} mpr_sweep_mode;

/* Defaults: q = 1/2, J = 1, FP64 storage, open boundary, 1 chain, seed 1, alpha0 = 1,
 * acc_target = 0.3, T_min = 1e-6, T_max = 10, automatic tiles and graphs. */
void mpr_config_default(mpr_config* cfg);

/* Create a context for one grid on the current HIP device; `hip_stream` is a hipStream_t
 * (NULL = the default stream).  Allocates nothing on the device until mpr_load. */
int mpr_create(const mpr_config* cfg, void* hip_stream, mpr_ctx** out);

/* Create a context for n_grids independent grids of sides H[g] x W[g] (host arrays, copied),
 * run together: every sweep of every grid and chain is one launch. */
int mpr_batch_create(const mpr_config* cfg, void* hip_stream, int32_t n_grids,
                     const int64_t* H, const int64_t* W, mpr_ctx** out);

void mpr_destroy(mpr_ctx* ctx);

/* Load one grid (single-grid context; H, W must be >= 2): z_dev[H*W] FP64 data, mask_dev[H*W]
 * with 1 = sample site (value known), 0 = prediction site (value ignored, may be NaN).
 * Maps samples onto u = (z - zmin)/(zmax - zmin) (Sec. 1-2), computes the sample energy
 * e_smp = -(J/|B_s|) sum over sample-sample bonds of cos[q(phi_i - phi_j)] (Eq. (2)), and
 * draws the initial angles of the prediction sites.  Synchronises once (validation). */
int mpr_load(mpr_ctx* ctx, int64_t H, int64_t W, const double* z_dev, const uint8_t* mask_dev);

/* Batched load: z_dev and mask_dev packed as described above. */
int mpr_batch_load(mpr_ctx* ctx, const double* z_dev, const uint8_t* mask_dev);

/* Temperature inference (Sec. 2): n_equil hybrid sweeps; after each one the temperature of
 * every chain is moved by the ratio (e_smp + J)/(e_sim + J) (clamped to [1/2, 2] and to
 * [T_min, T_max]) and the Metropolis window towards acc_target; the estimate is the mean of
 * the temperatures used in the second half of the sweeps.  T_host (may be NULL) receives the
 * estimates [n_grids * n_chains].  Starts from T_0 = 4 (e_smp + J). */
int mpr_infer_temperature(mpr_ctx* ctx, int32_t n_equil, double* T_host);

/* Use temperature T for every chain instead of inferring it. */
int mpr_set_temperature(mpr_ctx* ctx, double T);

/* n hybrid sweeps at each chain's current temperature (kept fixed) with the Metropolis window
 * control and the per-sweep trace of mpr_infer_temperature (Sec. 2: conditional simulation in
 * equilibrium at the inferred T).  T_host (may be NULL) receives the unchanged temperatures.
 * ESTATE before a temperature is set or inferred; EINVAL for n < 0. */
int mpr_equilibrate(mpr_ctx* ctx, int32_t n, double* T_host);

/* Second reading of the temperature inference of Sec. 2: match the sample energy to the
 * unconditional (data-free) model instead of the conditional simulation.
 *
 * mpr_energy_curve: mean bond energy e(T) = -(J/|B|) sum over all bonds of cos[q(phi_i-phi_j)]
 * (Eq. (2)) of the model with no data on a periodic side x side lattice, at each of the n_T
 * temperatures T_host[i] (host array, finite and > 0).  Chain i (Philox chain word
 * grid_offset * n_T + i, every site drawn uniformly at sweep 0) runs n_burn hybrid sweeps at
 * fixed T_host[i] with the window control of cfg, then n_meas sweeps with the window fixed (an
 * adapting window makes the kernel depend on the chain's past, which biases the average);
 * e_host[i] (host) = mean of e over the n_meas sweeps; trace_host (host, may be NULL) receives
 * [n_T][n_burn + n_meas][4] = (e, T, alpha, acceptance) of every sweep.  Uses cfg's q, J, precision, seed, alpha0, acc_target and
 * grid_offset; the boundary is periodic and the sweep path the row-window one whatever cfg
 * says.  side must be even, >= 4 and divisible by 4 (periodic lattices; EINVAL / EBIPARTITE
 * otherwise); n_burn >= 0, n_meas >= 1.  Allocates and frees its own device memory, runs on
 * `hip_stream` (a hipStream_t, NULL = default) and synchronises before returning.
 *
 * mpr_set_temperature_curve: every chain's T <- the curve's temperature at its grid's sample
 * energy e_smp: linear between the first pair of points (from the low-T end) whose energies
 * bracket e_smp, T_host[0] below the curve, T_host[n_T-1] above it.  T_host ascending, n_T >= 1,
 * finite values (EINVAL otherwise).  T_out (host, may be NULL) receives the temperatures
 * [n_grids * n_chains].  Needs loaded data (ESTATE). */
int mpr_energy_curve(const mpr_config* cfg, void* hip_stream, int32_t side, int32_t n_T,
                     const double* T_host, int32_t n_burn, int32_t n_meas, double* e_host,
                     double* trace_host);
int mpr_set_temperature_curve(mpr_ctx* ctx, int32_t n_T, const double* T_host,
                              const double* e_host, double* T_out);

/* For callers that cannot allocate device memory (code that runs where hipMalloc is not
 * allowed, tight serving loops): mpr_set_temperature_curve with the same arguments, results and
 * error codes, which allocates nothing.  The curve table and the temperatures read back stage
 * through a static device array of 8192 doubles (64 KiB) that each device holds until the
 * process ends: 2 n_T + (T_out ? n_grids * n_chains : 0) must not exceed 8192 (EINVAL
 * otherwise, context unchanged).  Every call writes all of the array it reads, so nothing of an
 * earlier call leaks into the next; the array is shared by every context on the device, so
 * calls that overlap on one device (two host threads, two streams) race and must be
 * serialised by the caller.  The context's device must be the current device (EINVAL
 * otherwise).  Synchronises the context's stream. */
int mpr_set_temperature_curve_noalloc(mpr_ctx* ctx, int32_t n_T, const double* T_host,
                                      const double* e_host, double* T_out);

/* n sweeps at the current temperatures and windows, without averaging (no control). */
int mpr_burn_in(mpr_ctx* ctx, int32_t n);

/* n_avg averaging sweeps (Sec. 2: configurations averaged in equilibrium); may be called
 * repeatedly, the averages accumulate.  Needs a temperature (ESTATE otherwise). */
int mpr_run(mpr_ctx* ctx, int32_t n_avg);

/* Predictions zhat_dev[packed sites] (FP64, caller-allocated): prediction sites get
 * zmin + (zmax - zmin) * (mean over sweeps and chains of u); sample sites get their data
 * value exactly.  ESTATE before the first averaging sweep. */
int mpr_get_predictions(mpr_ctx* ctx, double* zhat_dev);

typedef struct mpr_chain_stats {
    double T;              /* current temperature (the estimate after inference)   */
    double alpha;          /* current Metropolis window                             */
    double e_sample;       /* e_smp of the chain's grid (per bond)                  */
    double e_sim;          /* e_sim after the last inference sweep (per bond)       */
    double acc_rate;       /* acceptance rate of the last inference sweep           */
    int64_t n_pred, n_bonds, n_sample_bonds;
    double zmin, zmax;
} mpr_chain_stats;

/* out_host[n_grids * n_chains]; synchronises. */
int mpr_get_stats(mpr_ctx* ctx, mpr_chain_stats* out_host);

/* Stream time of the last call of each phase, in milliseconds, from events the library records
 * on its stream before the call's first and after its last enqueued work (so it includes any
 * time the stream waited in between): the last load (with the autotuner's timing if it ran),
 * the last inference or equilibration, the last averaging run, the last predictions; -1 for a
 * phase not run yet.  infer_sweeps / run_sweeps: the sweeps of those calls.  Synchronises. */
typedef struct mpr_timings {
    double load_ms, infer_ms, run_ms, predict_ms;
    int64_t infer_sweeps, run_sweeps;
} mpr_timings;
int mpr_get_timings(mpr_ctx* ctx, mpr_timings* out_host);

/* Per-sweep record of the last inference of chain `grid_chain` (= g * n_chains + chain):
 * out_host[max_entries][4] = (e_sim, T, alpha, acceptance) of each sweep; *n_out entries. */
int mpr_get_trace(mpr_ctx* ctx, int32_t grid_chain, int32_t max_entries, double* out_host,
                  int32_t* n_out);

/* Checkpoint.  u_dev[packed per-chain sites] angles in revolutions (FP64), acc_dev the same
 * shape (running sums of u over averaging sweeps), ctl_host[n_grids*n_chains][2] = (T, alpha),
 * meta_host[3] = (next sweep index, averaging sweeps done, phase).  NULL pointers are skipped.
 * The Philox streams are keyed by the sweep index, so save + restore + continue is bitwise
 * identical to an uninterrupted run. */
int mpr_get_state(mpr_ctx* ctx, double* u_dev, double* acc_dev, double* ctl_host,
                  int64_t* meta_host);
/* Restores the same items; u values at sample sites are ignored, values at prediction sites
 * must lie in [0, 1] (EINVAL otherwise, state unchanged). */
int mpr_set_state(mpr_ctx* ctx, const double* u_dev, const double* acc_dev,
                  const double* ctl_host, const int64_t* meta_host);

/* One sweep with Philox sweep index `sweep` at the current temperatures and windows, without
 * control or averaging, recording per site decisions_dev[packed per-chain sites]:
 * bit 0 = over-relaxation applied, bit 1 = Metropolis move accepted, bit 2 = proposal
 * outside [0, 1] (rejected).  Sample sites get 0.  Advances the state, not the sweep index. */
int mpr_debug_sweep(mpr_ctx* ctx, int32_t sweep, uint8_t* decisions_dev);

/* n back-to-back launches of the inference sweep kernel (the hot kernel of
 * mpr_infer_temperature, with its energy and acceptance reductions) at the current
 * temperatures and windows, without the control step: for timing the kernel alone with events
 * recorded on the context's stream.  Advances the state and the sweep index like burn-in. */
int mpr_bench_sweeps(mpr_ctx* ctx, int32_t n);

/* Autotuner: times n_sweeps inference-variant sweeps of each candidate from the current state,
 * which is restored after each, and keeps the fastest.  Candidates: the fused path's rows per
 * work item (the six best of 2 ... 256 by a cost model), when the configuration's sweep_mode is
 * MPR_SWEEP_AUTO the sweep path itself (fused, compacted where possible, tiled where possible;
 * the path changes only the rounding of the energy sums, see mpr_sweep_mode), on the tiled path
 * its block shape (the four mpr_tile_shape values with single-precision functions, unless
 * tile_shape forces one), and, when graph_sweeps is 0, the sweeps per captured graph (16, 32,
 * 64; timed as graph replays).  Results do not depend on the rows, the tile shape or the graph
 * length.  mpr_get_tuning reports the choice.  Winners are remembered per shape, precision,
 * sweep_mode, tile_shape, graph_sweeps and percentage of prediction sites in the process, and in
 * the text file named by the environment variable MPR_TUNE_CACHE if it is set (an entry this
 * context cannot use is ignored and tuned again).
 * mpr_config tile_rows = -1 runs it at every load (8 sweeps; a remembered winner costs no
 * timing).  *rows_out (may be NULL) receives the fused path's rows per work item. */
int mpr_autotune(mpr_ctx* ctx, int32_t n_sweeps, int32_t* rows_out);

/* The configuration the context sweeps with (chosen at the last load by the rule, the
 * configuration or the autotuner): *path_out the sweep path (MPR_SWEEP_FUSED, _SPARSE or
 * _TILED), *rows_out the fused path's rows per work item, *tile_shape_out the tiled path's
 * mpr_tile_shape (-1 on the other paths), *graph_sweeps_out the sweeps per captured graph (-1:
 * no graphs).  Any pointer may be NULL; ESTATE before a load. */
int mpr_get_tuning(mpr_ctx* ctx, int32_t* path_out, int32_t* rows_out, int32_t* tile_shape_out,
                   int32_t* graph_sweeps_out);

/* The sweep path chosen at the last load (MPR_SWEEP_FUSED, _SPARSE or _TILED); ESTATE before
 * a load. */
int mpr_get_sweep_mode(mpr_ctx* ctx, int32_t* mode_out);

/* Number of grids, chains and sites of a context (any pointer may be NULL). */
int mpr_get_shape(mpr_ctx* ctx, int32_t* n_grids, int32_t* n_chains, int64_t* n_sites);

const char* mpr_strerror(int status);
const char* mpr_last_error(mpr_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif

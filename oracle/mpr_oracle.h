/*
 * mpr_oracle.h -- FP64 CPU oracle of the modified planar rotator (MPR) prediction method.
 *
 * TEST INFRASTRUCTURE ONLY.  This is a plain, slow, double-precision implementation that
 * the tests, the smoke check and the benchmark's CPU-baseline leg use to check the GPU
 * library.  The GPU library never includes, links or calls it, and it shares no code with
 * the GPU library (not even this header's constants).
 *
 * Method (Lach, Borovsky, Zukovic, "Numerical Precision Effects on GPU Simulation of
 * Massive Spatial Data, Based on the Modified Planar Rotator Model"):
 *   - Sec. 2, Eq. (2): H = -J sum_<ij> cos[q (phi_i - phi_j)], q in (0, 1/2], phi in [0, 2pi],
 *     nearest-neighbour pairs on a square grid.
 *   - Sec. 1 / Sec. 2: the measured values are mapped onto spin angles; the single parameter,
 *     the reduced temperature, is inferred from the incomplete data; a conditional Monte
 *     Carlo simulation with the hybrid (over-relaxation + Metropolis) algorithm changes only
 *     the spins at prediction sites; averaging equilibrium configurations gives predictions.
 *   - Sec. 2: the specific energy e = <H>/L^2 drives the temperature inference.
 *   - Sec. 3, Eq. (4): AAE = (1/P) sum_{prediction sites} |Z - Zhat|.
 *
 * Points the paper leaves to its references are fixed as follows (one reading, shared with
 * the GPU library by specification, not by code):
 *   map      phi = 2 pi (z - zmin) / (zmax - zmin), zmin/zmax over the sample sites.
 *   energy   per bond:  e = -(J/|B|) sum_bonds cos[q(phi_i - phi_j)].
 *   RNG      Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11), key = (seed lo, seed hi),
 *            counter = (pair, sweep, chain, (tag << 1) | colour), pair = y*NP + (x>>1)>>1,
 *            NP = ceil(ceil(W/2)/2); member (x>>1)&1 takes words (0,1) or (2,3).
 *            tag 0 = sweep update, tag 1 = initial state.  U(w) = (w + 1/2) 2^-32.
 *   init     prediction site phi = 2 pi U(w_a) from the (tag 1, sweep 0) counter.
 *   OR       phi' = 2 psi / q - phi with psi = atan2(S, C), C = sum_j cos(q phi_j),
 *            S = sum_j sin(q phi_j); kept only if phi' in [0, 2pi] and (C, S) != 0.
 *   MH       phi_p = phi + 2 pi alpha (U(w_a) - 1/2); rejected if outside [0, 2pi]; else
 *            accepted iff U(w_b) < exp(-(E_i(phi_p) - E_i(phi)) / T).
 *   sweep    colour 0 = (x + y) even, then colour 1; per site OR then MH.
 *   control  after every inference sweep: r = (e_smp + J)/(e_sim + J) (2 if the
 *            denominator <= 1e-300), clamped to [1/2, 2]; T <- clamp(T r, T_min, T_max);
 *            alpha <- clamp(alpha A / A_target, 1e-3, 1), A = accepts / P.
 *            T_0 = clamp(4 (e_smp + J), T_min, T_max).  T_hat = mean of the temperatures
 *            used in sweeps floor(n/2) .. n-1.  Averaging sweeps use T_hat and a frozen alpha.
 *   average  mean of phi over averaging sweeps, then over chains; mapped back linearly.
 */
#ifndef MPR_ORACLE_H
#define MPR_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_OK = 0, ORC_EINVAL = 1, ORC_ENOSAMPLE = 2, ORC_EBIPARTITE = 3, ORC_ESTATE = 4,
       ORC_ENOMEM = 5 };
enum { ORC_OPEN = 0, ORC_PERIODIC = 1 };
/* decision bits written by orc_site_update / debug sweeps */
enum { ORC_DEC_OR = 1, ORC_DEC_ACCEPT = 2, ORC_DEC_OUTSIDE = 4 };

typedef struct orc_config {
    double q, J;
    int32_t boundary;      /* ORC_OPEN or ORC_PERIODIC */
    int32_t n_chains;      /* independent chains, >= 1 */
    uint64_t seed;
    double alpha0;         /* initial Metropolis window, fraction of 2 pi, in (0, 1] */
    double acc_target;     /* target acceptance rate, in (0, 1) */
    double T_min, T_max;
    int32_t grid_id;       /* chain counter word = grid_id * n_chains + chain */
    int32_t n_threads;     /* OpenMP threads for row loops; 0 = runtime default */
} orc_config;

/* ---- primitives on plain arrays (row-major H x W, phi in radians) ---- */
void   orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
double orc_uniform(uint32_t w);
void   orc_site_words(uint64_t seed, int64_t W, int64_t y, int64_t x, uint32_t sweep,
                      uint32_t chain, uint32_t tag, uint32_t* wa, uint32_t* wb);
int    orc_map(int64_t n, const double* z, const uint8_t* mask, double* zmin, double* zmax,
               double* phi);
double orc_bond_sum(int64_t H, int64_t W, const double* phi, const uint8_t* mask,
                    int32_t boundary, double q, int64_t* n_bonds, int32_t n_threads);
void   orc_local_field(int64_t H, int64_t W, const double* phi, int32_t boundary, double q,
                       int64_t y, int64_t x, double* C, double* S);
double orc_site_energy(int64_t H, int64_t W, const double* phi, int32_t boundary, double q,
                       double J, int64_t y, int64_t x, double phi_i);
double orc_overrelax(double phi_i, double C, double S, double q, int32_t* applied);
int32_t orc_site_update(int64_t H, int64_t W, double* phi, int32_t boundary, double q,
                        double J, double T, double alpha, int64_t y, int64_t x,
                        uint32_t wa, uint32_t wb);
int64_t orc_sweep(int64_t H, int64_t W, double* phi, const uint8_t* mask, int32_t boundary,
                  double q, double J, double T, double alpha, uint64_t seed, uint32_t sweep,
                  uint32_t chain, int32_t n_threads, uint8_t* decisions);
void   orc_init_chain(int64_t H, int64_t W, double* phi, const uint8_t* mask, uint64_t seed,
                      uint32_t chain);

/* ---- context verbs (host pointers) ---- */
typedef struct orc_ctx orc_ctx;

typedef struct orc_chain_stats {
    double T, alpha, e_sample, e_sim, acc_rate;
    int64_t n_pred, n_bonds, n_sample_bonds;
    double zmin, zmax;
} orc_chain_stats;

int  orc_create(const orc_config* cfg, orc_ctx** out);
void orc_destroy(orc_ctx* ctx);
int  orc_load(orc_ctx* ctx, int64_t H, int64_t W, const double* z, const uint8_t* mask);
int  orc_infer_temperature(orc_ctx* ctx, int32_t n_equil, double* T_out);
int  orc_set_temperature(orc_ctx* ctx, double T);
int  orc_run(orc_ctx* ctx, int32_t n_avg);
int  orc_get_predictions(orc_ctx* ctx, double* zhat);
int  orc_get_stats(orc_ctx* ctx, orc_chain_stats* out);
int  orc_get_trace(orc_ctx* ctx, int32_t chain, int32_t max_entries, double* out,
                   int32_t* n_out);
/* state: phi [n_chains][H*W] radians, acc [n_chains][H*W], ctl [n_chains][2] = (T, alpha),
 * meta [3] = (next_sweep, n_avg, phase).  NULL pointers are skipped. */
int  orc_get_state(orc_ctx* ctx, double* phi, double* acc, double* ctl, int64_t* meta);
int  orc_set_state(orc_ctx* ctx, const double* phi, const double* acc, const double* ctl,
                   const int64_t* meta);
int  orc_debug_sweep(orc_ctx* ctx, int32_t sweep, uint8_t* decisions);
/* n sweeps at the current (fixed) T and alpha, without averaging */
int  orc_burn_in(orc_ctx* ctx, int32_t n);
/* n sweeps at each chain's current (fixed) T with the window control and the trace of the
 * inference; T_hat = that T */
int  orc_equilibrate(orc_ctx* ctx, int32_t n, double* T_out);

/* ---- alternative temperature reading: invert the model's energy-temperature curve ----
 * Unconditional mean bond energy of Eq. (2) (no data) on a periodic side x side lattice at
 * each T[i]: chain i (counter word grid_id * n_T + i) starts from the (tag 1, sweep 0) uniform
 * state and runs n_burn sweeps at fixed T[i] with the window control, then n_meas sweeps with
 * the window fixed; e_out[i] = mean e over the n_meas sweeps; trace_out (may be NULL) gets
 * [n_T][n_burn + n_meas][4]. */
int  orc_energy_curve(const orc_config* cfg, int64_t side, int32_t n_T, const double* T,
                      int32_t n_burn, int32_t n_meas, double* e_out, double* trace_out);
/* T with e(T) = e_target, linear between the bracketing points of a curve sampled at
 * increasing T (first bracket from the low end), clamped to the end points */
double orc_curve_temperature(int32_t n_T, const double* T, const double* e, double e_target);
/* every chain's T <- the curve's temperature at the loaded data's sample energy */
int  orc_set_temperature_curve(orc_ctx* ctx, int32_t n_T, const double* T, const double* e,
                               double* T_out);
/* n sweeps of chain 0 at its current T and alpha; phi of the listed sites after each sweep
 * goes to out[n][n_sites] */
int  orc_run_record(orc_ctx* ctx, int32_t n, int32_t n_sites, const int64_t* sites, double* out);

#ifdef __cplusplus
}
#endif
#endif

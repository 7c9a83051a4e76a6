/*
 * mpr_oracle.c -- FP64 CPU oracle of the MPR prediction method.  TEST INFRASTRUCTURE ONLY:
 * called by the tests, the smoke check and the benchmark's CPU-baseline leg, never by the
 * GPU library.  Every step is written in the paper's notation (angles phi in radians) and
 * in the order the method states it; see mpr_oracle.h for the readings of the points the
 * paper leaves open.  Loops are plain; OpenMP only splits the rows of one colour (sites of
 * one colour are independent, so this does not change any decision) and the rows of the
 * energy sum (per-row partial sums are added in row order, so the result does not depend on
 * the thread count).
 */
#include "mpr_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

static const double TWO_PI = 6.283185307179586476925286766559;

/* ------------------------------------------------------------------ Philox4x32-10 */
/* Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy as 1, 2, 3", SC'11:
 * ten rounds of (hi, lo) = M * x on words 0 and 2, mixed with words 1, 3 and the key; the
 * key is bumped by the Weyl constants between rounds. */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        uint64_t p0 = (uint64_t)0xD2511F53u * x0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * x2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        x0 = hi1 ^ x1 ^ k0;
        x1 = lo1;
        x2 = hi0 ^ x3 ^ k1;
        x3 = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* uniform on the open interval (0, 1): (w + 1/2) / 2^32 */
double orc_uniform(uint32_t w) { return ((double)w + 0.5) * (1.0 / 4294967296.0); }

/* the two 32-bit words of site (y, x) for one (sweep, chain, tag) */
void orc_site_words(uint64_t seed, int64_t W, int64_t y, int64_t x, uint32_t sweep,
                    uint32_t chain, uint32_t tag, uint32_t* wa, uint32_t* wb)
{
    int64_t Wc = (W + 1) / 2;            /* sites of one colour per row, rounded up */
    int64_t NP = (Wc + 1) / 2;           /* Philox calls per row and colour */
    int64_t kx = x / 2;                  /* column inside the colour's row */
    uint32_t colour = (uint32_t)((x + y) & 1);
    uint32_t ctr[4] = { (uint32_t)(y * NP + kx / 2), sweep, chain, (tag << 1) | colour };
    uint32_t key[2] = { (uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32) };
    uint32_t out[4];
    orc_philox4x32_10(ctr, key, out);
    if ((kx & 1) == 0) { *wa = out[0]; *wb = out[1]; }
    else               { *wa = out[2]; *wb = out[3]; }
}

/* ------------------------------------------------------------------ mapping */
/* Sec. 1-2: measured values are mapped onto spin angles; linear onto [0, 2 pi] using the
 * sample minimum and maximum.  Prediction sites get phi = 0 here (set later by init). */
int orc_map(int64_t n, const double* z, const uint8_t* mask, double* zmin, double* zmax,
            double* phi)
{
    double lo = INFINITY, hi = -INFINITY;
    for (int64_t i = 0; i < n; ++i) {
        if (mask[i] > 1) return ORC_EINVAL;
        if (mask[i] == 1) {
            if (!isfinite(z[i])) return ORC_EINVAL;
            if (z[i] < lo) lo = z[i];
            if (z[i] > hi) hi = z[i];
        }
    }
    if (!(hi > lo)) return ORC_ENOSAMPLE;
    for (int64_t i = 0; i < n; ++i)
        phi[i] = mask[i] ? TWO_PI * ((z[i] - lo) / (hi - lo)) : 0.0;
    *zmin = lo;
    *zmax = hi;
    return ORC_OK;
}

/* ------------------------------------------------------------------ energy */
/* Eq. (2) without the -J factor: sum over nearest-neighbour bonds of cos[q(phi_i - phi_j)].
 * Each bond is visited once, from its left (right bond) or upper (down bond) end.  With a
 * mask, only bonds whose two ends are sample sites (mask == 1) are summed. */
double orc_bond_sum(int64_t H, int64_t W, const double* phi, const uint8_t* mask,
                    int32_t boundary, double q, int64_t* n_bonds, int32_t n_threads)
{
    double* row_sum = (double*)calloc((size_t)H, sizeof(double));
    int64_t* row_cnt = (int64_t*)calloc((size_t)H, sizeof(int64_t));
#ifdef _OPENMP
    int nt = n_threads > 0 ? n_threads : omp_get_max_threads();
#pragma omp parallel for schedule(static) num_threads(nt)
#endif
    for (int64_t y = 0; y < H; ++y) {
        double s = 0.0;
        int64_t c = 0;
        for (int64_t x = 0; x < W; ++x) {
            int64_t i = y * W + x;
            /* right neighbour */
            int64_t xr = x + 1;
            if (xr == W) xr = (boundary == ORC_PERIODIC) ? 0 : -1;
            if (xr >= 0) {
                int64_t j = y * W + xr;
                if (!mask || (mask[i] && mask[j])) { s += cos(q * (phi[i] - phi[j])); ++c; }
            }
            /* lower neighbour */
            int64_t yd = y + 1;
            if (yd == H) yd = (boundary == ORC_PERIODIC) ? 0 : -1;
            if (yd >= 0) {
                int64_t j = yd * W + x;
                if (!mask || (mask[i] && mask[j])) { s += cos(q * (phi[i] - phi[j])); ++c; }
            }
        }
        row_sum[y] = s;
        row_cnt[y] = c;
    }
    double total = 0.0;
    int64_t cnt = 0;
    for (int64_t y = 0; y < H; ++y) { total += row_sum[y]; cnt += row_cnt[y]; }
    free(row_sum);
    free(row_cnt);
    if (n_bonds) *n_bonds = cnt;
    return total;
}

/* in-grid neighbours of (y, x): up to 4 for an open grid, 4 for a periodic one */
static int neighbours(int64_t H, int64_t W, int32_t boundary, int64_t y, int64_t x,
                      int64_t nb[4])
{
    int n = 0;
    int per = boundary == ORC_PERIODIC;
    if (x > 0) nb[n++] = y * W + x - 1;       else if (per) nb[n++] = y * W + W - 1;
    if (x < W - 1) nb[n++] = y * W + x + 1;   else if (per) nb[n++] = y * W;
    if (y > 0) nb[n++] = (y - 1) * W + x;     else if (per) nb[n++] = (H - 1) * W + x;
    if (y < H - 1) nb[n++] = (y + 1) * W + x; else if (per) nb[n++] = x;
    return n;
}

/* local field of site i: C = sum_j cos(q phi_j), S = sum_j sin(q phi_j) */
void orc_local_field(int64_t H, int64_t W, const double* phi, int32_t boundary, double q,
                     int64_t y, int64_t x, double* C, double* S)
{
    int64_t nb[4];
    int n = neighbours(H, W, boundary, y, x, nb);
    double c = 0.0, s = 0.0;
    for (int k = 0; k < n; ++k) { c += cos(q * phi[nb[k]]); s += sin(q * phi[nb[k]]); }
    *C = c;
    *S = s;
}

/* energy of the bonds of site i when its angle is phi_i: -J sum_j cos[q(phi_i - phi_j)] */
double orc_site_energy(int64_t H, int64_t W, const double* phi, int32_t boundary, double q,
                       double J, int64_t y, int64_t x, double phi_i)
{
    int64_t nb[4];
    int n = neighbours(H, W, boundary, y, x, nb);
    double e = 0.0;
    for (int k = 0; k < n; ++k) e += cos(q * (phi_i - phi[nb[k]]));
    return -J * e;
}

/* ------------------------------------------------------------------ hybrid update */
/* Over-relaxation: the site energy is -J R cos(q phi - psi); reflecting q phi about psi
 * keeps it.  The reflected angle is used only when it lies in [0, 2 pi]. */
double orc_overrelax(double phi_i, double C, double S, double q, int32_t* applied)
{
    *applied = 0;
    if (C == 0.0 && S == 0.0) return phi_i;
    double psi = atan2(S, C);
    double phi_r = 2.0 * psi / q - phi_i;
    if (phi_r >= 0.0 && phi_r <= TWO_PI) { *applied = 1; return phi_r; }
    return phi_i;
}

int32_t orc_site_update(int64_t H, int64_t W, double* phi, int32_t boundary, double q,
                        double J, double T, double alpha, int64_t y, int64_t x,
                        uint32_t wa, uint32_t wb)
{
    int64_t i = y * W + x;
    int32_t dec = 0;
    /* over-relaxation step */
    double C, S;
    int32_t applied;
    orc_local_field(H, W, phi, boundary, q, y, x, &C, &S);
    phi[i] = orc_overrelax(phi[i], C, S, q, &applied);
    if (applied) dec |= ORC_DEC_OR;
    /* restricted Metropolis step */
    double phi_p = phi[i] + TWO_PI * alpha * (orc_uniform(wa) - 0.5);
    if (phi_p < 0.0 || phi_p > TWO_PI) return dec | ORC_DEC_OUTSIDE;
    double dE = orc_site_energy(H, W, phi, boundary, q, J, y, x, phi_p)
              - orc_site_energy(H, W, phi, boundary, q, J, y, x, phi[i]);
    if (orc_uniform(wb) < exp(-dE / T)) {
        phi[i] = phi_p;
        dec |= ORC_DEC_ACCEPT;
    }
    return dec;
}

/* one hybrid sweep: all prediction sites of colour 0, then of colour 1 */
int64_t orc_sweep(int64_t H, int64_t W, double* phi, const uint8_t* mask, int32_t boundary,
                  double q, double J, double T, double alpha, uint64_t seed, uint32_t sweep,
                  uint32_t chain, int32_t n_threads, uint8_t* decisions)
{
    int64_t accepts = 0;
#ifdef _OPENMP
    int nt = n_threads > 0 ? n_threads : omp_get_max_threads();
#else
    (void)n_threads;
#endif
    for (int colour = 0; colour < 2; ++colour) {
#ifdef _OPENMP
#pragma omp parallel for schedule(static) reduction(+ : accepts) num_threads(nt)
#endif
        for (int64_t y = 0; y < H; ++y) {
            for (int64_t x = 0; x < W; ++x) {
                if (((x + y) & 1) != colour) continue;
                int64_t i = y * W + x;
                if (mask[i]) continue;
                uint32_t wa, wb;
                orc_site_words(seed, W, y, x, sweep, chain, 0, &wa, &wb);
                int32_t dec = orc_site_update(H, W, phi, boundary, q, J, T, alpha, y, x, wa, wb);
                if (dec & ORC_DEC_ACCEPT) ++accepts;
                if (decisions) decisions[i] = (uint8_t)dec;
            }
        }
    }
    return accepts;
}

/* initial state of the prediction sites: uniform on [0, 2 pi) from the tag-1 counter */
void orc_init_chain(int64_t H, int64_t W, double* phi, const uint8_t* mask, uint64_t seed,
                    uint32_t chain)
{
    for (int64_t y = 0; y < H; ++y)
        for (int64_t x = 0; x < W; ++x) {
            int64_t i = y * W + x;
            if (mask[i]) continue;
            uint32_t wa, wb;
            orc_site_words(seed, W, y, x, 0, chain, 1, &wa, &wb);
            phi[i] = TWO_PI * orc_uniform(wa);
        }
}

/* ------------------------------------------------------------------ context */
enum { PH_EMPTY = 0, PH_LOADED = 1, PH_TEMPERED = 2, PH_AVERAGED = 3 };

struct orc_ctx {
    orc_config cfg;
    int64_t H, W, n;
    double* z;
    uint8_t* mask;
    double zmin, zmax;
    double* phi;       /* [n_chains][n] */
    double* acc;       /* [n_chains][n] */
    double* T;         /* [n_chains] */
    double* alpha;     /* [n_chains] */
    double* e_sim;     /* [n_chains] last measured */
    double* acc_rate;  /* [n_chains] last sweep */
    double* trace;     /* [n_chains][trace_cap][4] */
    int32_t trace_cap, trace_len;
    double e_smp;
    int64_t n_pred, n_bonds, n_sample_bonds;
    int64_t next_sweep, n_avg;
    int32_t phase;
};

static int check_config(const orc_config* c)
{
    if (!(c->q > 0.0 && c->q <= 0.5)) return ORC_EINVAL;
    if (!(c->J > 0.0) || !isfinite(c->J)) return ORC_EINVAL;
    if (c->boundary != ORC_OPEN && c->boundary != ORC_PERIODIC) return ORC_EINVAL;
    if (c->n_chains < 1) return ORC_EINVAL;
    if (!(c->alpha0 > 0.0 && c->alpha0 <= 1.0)) return ORC_EINVAL;
    if (!(c->acc_target > 0.0 && c->acc_target < 1.0)) return ORC_EINVAL;
    if (!(c->T_min > 0.0) || !(c->T_max >= c->T_min) || !isfinite(c->T_max)) return ORC_EINVAL;
    if (c->grid_id < 0) return ORC_EINVAL;
    return ORC_OK;
}

static void free_arrays(orc_ctx* c)
{
    free(c->z); free(c->mask); free(c->phi); free(c->acc); free(c->T); free(c->alpha);
    free(c->e_sim); free(c->acc_rate); free(c->trace);
    c->z = NULL; c->mask = NULL; c->phi = NULL; c->acc = NULL; c->T = NULL; c->alpha = NULL;
    c->e_sim = NULL; c->acc_rate = NULL; c->trace = NULL;
}

int orc_create(const orc_config* cfg, orc_ctx** out)
{
    if (!cfg || !out) return ORC_EINVAL;
    int rc = check_config(cfg);
    if (rc) return rc;
    orc_ctx* c = (orc_ctx*)calloc(1, sizeof(orc_ctx));
    if (!c) return ORC_ENOMEM;
    c->cfg = *cfg;
    *out = c;
    return ORC_OK;
}

void orc_destroy(orc_ctx* ctx)
{
    if (!ctx) return;
    free_arrays(ctx);
    free(ctx);
}

static uint32_t chain_word(const orc_ctx* c, int32_t chain)
{
    return (uint32_t)(c->cfg.grid_id * c->cfg.n_chains + chain);
}

int orc_load(orc_ctx* c, int64_t H, int64_t W, const double* z, const uint8_t* mask)
{
    if (!c || !z || !mask) return ORC_EINVAL;
    if (H < 2 || W < 2) return ORC_EINVAL;
    if (c->cfg.boundary == ORC_PERIODIC && ((H & 1) || (W & 1))) return ORC_EBIPARTITE;
    int64_t n = H * W;
    double* phi0 = (double*)malloc((size_t)n * sizeof(double));
    if (!phi0) return ORC_ENOMEM;
    double zmin, zmax;
    int rc = orc_map(n, z, mask, &zmin, &zmax, phi0);
    if (rc) { free(phi0); return rc; }
    int64_t nsb = 0;
    double ssum = orc_bond_sum(H, W, phi0, mask, c->cfg.boundary, c->cfg.q, &nsb,
                               c->cfg.n_threads);
    if (nsb == 0) { free(phi0); return ORC_ENOSAMPLE; }

    free_arrays(c);
    int C = c->cfg.n_chains;
    c->H = H; c->W = W; c->n = n;
    c->z = (double*)malloc((size_t)n * sizeof(double));
    c->mask = (uint8_t*)malloc((size_t)n);
    c->phi = (double*)malloc((size_t)n * C * sizeof(double));
    c->acc = (double*)calloc((size_t)n * C, sizeof(double));
    c->T = (double*)calloc((size_t)C, sizeof(double));
    c->alpha = (double*)calloc((size_t)C, sizeof(double));
    c->e_sim = (double*)calloc((size_t)C, sizeof(double));
    c->acc_rate = (double*)calloc((size_t)C, sizeof(double));
    if (!c->z || !c->mask || !c->phi || !c->acc || !c->T || !c->alpha || !c->e_sim ||
        !c->acc_rate) { free(phi0); free_arrays(c); return ORC_ENOMEM; }
    memcpy(c->z, z, (size_t)n * sizeof(double));
    memcpy(c->mask, mask, (size_t)n);
    c->zmin = zmin; c->zmax = zmax;
    c->n_pred = 0;
    for (int64_t i = 0; i < n; ++i) c->n_pred += mask[i] == 0;
    orc_bond_sum(H, W, phi0, NULL, c->cfg.boundary, c->cfg.q, &c->n_bonds, 1);
    c->n_sample_bonds = nsb;
    c->e_smp = -c->cfg.J * ssum / (double)nsb;
    for (int ch = 0; ch < C; ++ch) {
        double* p = c->phi + (size_t)ch * n;
        memcpy(p, phi0, (size_t)n * sizeof(double));
        orc_init_chain(H, W, p, mask, c->cfg.seed, chain_word(c, ch));
        c->alpha[ch] = c->cfg.alpha0;
        c->T[ch] = 0.0;
    }
    free(phi0);
    c->trace_cap = 0; c->trace_len = 0;
    c->next_sweep = 0; c->n_avg = 0;
    c->phase = PH_LOADED;
    return ORC_OK;
}

static double clampd(double v, double lo, double hi) { return v < lo ? lo : (v > hi ? hi : v); }

/* n conditional sweeps per chain with the control and the per-sweep trace.  fixed = 0: the
 * temperature follows the energy matching from T_0 and the window the acceptance; FIX_T: the
 * temperature stays at each chain's current value; FIX_T | FIX_ALPHA: the window stays too.
 * T_hat = mean of the temperatures used in sweeps floor(n/2) .. n-1 (with a fixed T, that T
 * itself). */
enum { FIX_T = 1, FIX_ALPHA = 2 };
static int sweep_loop(orc_ctx* c, int32_t n_equil, int fixed, double* T_out)
{
    const orc_config* g = &c->cfg;
    int C = g->n_chains;
    free(c->trace);
    c->trace_cap = n_equil;
    c->trace_len = 0;
    c->trace = (double*)calloc((size_t)C * (n_equil > 0 ? n_equil : 1) * 4, sizeof(double));
    if (!c->trace) return ORC_ENOMEM;
    double T0 = clampd(4.0 * (c->e_smp + g->J), g->T_min, g->T_max);
    for (int ch = 0; ch < C; ++ch) {
        double* p = c->phi + (size_t)ch * c->n;
        double T = (fixed & FIX_T) ? c->T[ch] : T0, a = c->alpha[ch], Tsum = 0.0;
        int64_t Tcnt = 0;
        for (int32_t s = 0; s < n_equil; ++s) {
            int64_t acc = orc_sweep(c->H, c->W, p, c->mask, g->boundary, g->q, g->J, T, a,
                                    g->seed, (uint32_t)(c->next_sweep + s), chain_word(c, ch),
                                    g->n_threads, NULL);
            int64_t nb;
            double e_sim = -g->J * orc_bond_sum(c->H, c->W, p, NULL, g->boundary, g->q, &nb,
                                                g->n_threads) / (double)nb;
            double A = c->n_pred > 0 ? (double)acc / (double)c->n_pred : g->acc_target;
            double* tr = c->trace + ((size_t)ch * n_equil + s) * 4;
            tr[0] = e_sim; tr[1] = T; tr[2] = a; tr[3] = A;
            if (s >= n_equil / 2) { Tsum += T; ++Tcnt; }
            if (!(fixed & FIX_T)) {
                /* temperature control: multiplicative energy matching */
                double num = c->e_smp + g->J, den = e_sim + g->J;
                double r = den <= 1e-300 ? 2.0 : num / den;
                r = clampd(r, 0.5, 2.0);
                T = clampd(T * r, g->T_min, g->T_max);
            }
            /* Metropolis window control */
            if (!(fixed & FIX_ALPHA)) a = clampd(a * A / g->acc_target, 1e-3, 1.0);
            c->e_sim[ch] = e_sim;
            c->acc_rate[ch] = A;
        }
        if (!(fixed & FIX_T)) c->T[ch] = Tcnt > 0 ? Tsum / (double)Tcnt : T0;
        c->alpha[ch] = a;
        if (T_out) T_out[ch] = c->T[ch];
    }
    c->trace_len = n_equil;
    c->next_sweep += n_equil;
    c->phase = PH_TEMPERED;
    return ORC_OK;
}

int orc_infer_temperature(orc_ctx* c, int32_t n_equil, double* T_out)
{
    if (!c) return ORC_EINVAL;
    if (c->phase < PH_LOADED) return ORC_ESTATE;
    if (n_equil < 0) return ORC_EINVAL;
    return sweep_loop(c, n_equil, 0, T_out);
}

int orc_equilibrate(orc_ctx* c, int32_t n, double* T_out)
{
    if (!c) return ORC_EINVAL;
    if (c->phase < PH_TEMPERED) return ORC_ESTATE;
    if (n < 0) return ORC_EINVAL;
    return sweep_loop(c, n, FIX_T, T_out);
}

/* ------------------------------------------------------------------ energy-temperature curve */
int orc_energy_curve(const orc_config* cfg, int64_t side, int32_t n_T, const double* T,
                     int32_t n_burn, int32_t n_meas, double* e_out, double* trace_out)
{
    if (!cfg || !T || !e_out || n_T < 1 || n_burn < 0 || n_meas < 1) return ORC_EINVAL;
    if (side < 2 || (side & 1)) return ORC_EBIPARTITE;
    for (int32_t i = 0; i < n_T; ++i)
        if (!(T[i] > 0.0) || !isfinite(T[i])) return ORC_EINVAL;
    orc_config g = *cfg;
    g.boundary = ORC_PERIODIC;
    g.n_chains = n_T;
    orc_ctx* c = NULL;
    int rc = orc_create(&g, &c);
    if (rc) return rc;
    int64_t n = side * side;
    c->H = side; c->W = side; c->n = n;
    c->z = (double*)calloc((size_t)n, sizeof(double));
    c->mask = (uint8_t*)calloc((size_t)n, 1);               /* no data: every site free */
    c->phi = (double*)calloc((size_t)n * n_T, sizeof(double));
    c->acc = (double*)calloc((size_t)n * n_T, sizeof(double));
    c->T = (double*)calloc((size_t)n_T, sizeof(double));
    c->alpha = (double*)calloc((size_t)n_T, sizeof(double));
    c->e_sim = (double*)calloc((size_t)n_T, sizeof(double));
    c->acc_rate = (double*)calloc((size_t)n_T, sizeof(double));
    if (!c->z || !c->mask || !c->phi || !c->acc || !c->T || !c->alpha || !c->e_sim ||
        !c->acc_rate) { orc_destroy(c); return ORC_ENOMEM; }
    c->n_pred = n;
    c->n_bonds = 2 * n;
    for (int32_t i = 0; i < n_T; ++i) {
        orc_init_chain(side, side, c->phi + (size_t)i * n, c->mask, g.seed, chain_word(c, i));
        c->alpha[i] = g.alpha0;
        c->T[i] = T[i];
    }
    c->phase = PH_TEMPERED;
    /* burn-in with the window control, then measurement at a fixed window: a window that
     * follows the chain's own acceptance makes the transition kernel depend on its past */
    const int32_t total = n_burn + n_meas;
    rc = sweep_loop(c, n_burn, FIX_T, NULL);
    if (!rc && trace_out)
        for (int32_t i = 0; i < n_T; ++i)
            memcpy(trace_out + (size_t)i * total * 4, c->trace + (size_t)i * n_burn * 4,
                   (size_t)n_burn * 4 * sizeof(double));
    if (!rc) rc = sweep_loop(c, n_meas, FIX_T | FIX_ALPHA, NULL);
    if (rc) { orc_destroy(c); return rc; }
    for (int32_t i = 0; i < n_T; ++i) {
        double s = 0.0;
        for (int32_t k = 0; k < n_meas; ++k) s += c->trace[((size_t)i * n_meas + k) * 4];
        e_out[i] = s / (double)n_meas;
        if (trace_out)
            memcpy(trace_out + ((size_t)i * total + n_burn) * 4, c->trace + (size_t)i * n_meas * 4,
                   (size_t)n_meas * 4 * sizeof(double));
    }
    orc_destroy(c);
    return ORC_OK;
}

double orc_curve_temperature(int32_t n_T, const double* T, const double* e, double e_target)
{
    if (n_T < 2 || e_target <= e[0]) return T[0];
    for (int32_t i = 0; i + 1 < n_T; ++i)
        if (e_target <= e[i + 1]) {
            const double de = e[i + 1] - e[i];
            if (!(de > 0.0)) return T[i];
            return T[i] + (T[i + 1] - T[i]) * ((e_target - e[i]) / de);
        }
    return T[n_T - 1];
}

int orc_set_temperature_curve(orc_ctx* c, int32_t n_T, const double* T, const double* e,
                              double* T_out)
{
    if (!c || !T || !e || n_T < 1) return ORC_EINVAL;
    if (c->phase < PH_LOADED) return ORC_ESTATE;
    for (int32_t i = 0; i < n_T; ++i)
        if (!(T[i] > 0.0) || (i > 0 && !(T[i] > T[i - 1]))) return ORC_EINVAL;
    const double Th = orc_curve_temperature(n_T, T, e, c->e_smp);
    for (int ch = 0; ch < c->cfg.n_chains; ++ch) {
        c->T[ch] = Th;
        if (T_out) T_out[ch] = Th;
    }
    if (c->phase < PH_TEMPERED) c->phase = PH_TEMPERED;
    return ORC_OK;
}

int orc_set_temperature(orc_ctx* c, double T)
{
    if (!c) return ORC_EINVAL;
    if (c->phase < PH_LOADED) return ORC_ESTATE;
    if (!(T > 0.0) || !isfinite(T)) return ORC_EINVAL;
    for (int ch = 0; ch < c->cfg.n_chains; ++ch) c->T[ch] = T;
    if (c->phase < PH_TEMPERED) c->phase = PH_TEMPERED;
    return ORC_OK;
}

int orc_run(orc_ctx* c, int32_t n_avg)
{
    if (!c) return ORC_EINVAL;
    if (n_avg < 0) return ORC_EINVAL;
    if (c->phase < PH_TEMPERED) return ORC_ESTATE;
    const orc_config* g = &c->cfg;
    for (int ch = 0; ch < g->n_chains; ++ch) {
        double* p = c->phi + (size_t)ch * c->n;
        double* a = c->acc + (size_t)ch * c->n;
        for (int32_t s = 0; s < n_avg; ++s) {
            int64_t acc = orc_sweep(c->H, c->W, p, c->mask, g->boundary, g->q, g->J, c->T[ch],
                                    c->alpha[ch], g->seed, (uint32_t)(c->next_sweep + s),
                                    chain_word(c, ch), g->n_threads, NULL);
            c->acc_rate[ch] = c->n_pred > 0 ? (double)acc / (double)c->n_pred : 0.0;
            for (int64_t i = 0; i < c->n; ++i)
                if (!c->mask[i]) a[i] += p[i];
        }
    }
    c->next_sweep += n_avg;
    c->n_avg += n_avg;
    if (n_avg > 0) c->phase = PH_AVERAGED;
    return ORC_OK;
}

int orc_get_predictions(orc_ctx* c, double* zhat)
{
    if (!c || !zhat) return ORC_EINVAL;
    if (c->phase < PH_AVERAGED || c->n_avg == 0) return ORC_ESTATE;
    int C = c->cfg.n_chains;
    for (int64_t i = 0; i < c->n; ++i) {
        if (c->mask[i]) { zhat[i] = c->z[i]; continue; }
        double m = 0.0;
        for (int ch = 0; ch < C; ++ch) m += c->acc[(size_t)ch * c->n + i] / (double)c->n_avg;
        m /= (double)C;
        zhat[i] = c->zmin + (c->zmax - c->zmin) * (m / TWO_PI);
    }
    return ORC_OK;
}

int orc_get_stats(orc_ctx* c, orc_chain_stats* out)
{
    if (!c || !out) return ORC_EINVAL;
    if (c->phase < PH_LOADED) return ORC_ESTATE;
    for (int ch = 0; ch < c->cfg.n_chains; ++ch) {
        orc_chain_stats* s = out + ch;
        s->T = c->T[ch]; s->alpha = c->alpha[ch]; s->e_sample = c->e_smp;
        s->e_sim = c->e_sim[ch]; s->acc_rate = c->acc_rate[ch];
        s->n_pred = c->n_pred; s->n_bonds = c->n_bonds; s->n_sample_bonds = c->n_sample_bonds;
        s->zmin = c->zmin; s->zmax = c->zmax;
    }
    return ORC_OK;
}

int orc_get_trace(orc_ctx* c, int32_t chain, int32_t max_entries, double* out, int32_t* n_out)
{
    if (!c || !out || chain < 0 || chain >= c->cfg.n_chains || max_entries < 0) return ORC_EINVAL;
    int32_t n = c->trace_len < max_entries ? c->trace_len : max_entries;
    if (n > 0)
        memcpy(out, c->trace + (size_t)chain * c->trace_cap * 4, (size_t)n * 4 * sizeof(double));
    if (n_out) *n_out = n;
    return ORC_OK;
}

int orc_get_state(orc_ctx* c, double* phi, double* acc, double* ctl, int64_t* meta)
{
    if (!c) return ORC_EINVAL;
    if (c->phase < PH_LOADED) return ORC_ESTATE;
    size_t tot = (size_t)c->n * c->cfg.n_chains;
    if (phi) memcpy(phi, c->phi, tot * sizeof(double));
    if (acc) memcpy(acc, c->acc, tot * sizeof(double));
    if (ctl)
        for (int ch = 0; ch < c->cfg.n_chains; ++ch) { ctl[2 * ch] = c->T[ch]; ctl[2 * ch + 1] = c->alpha[ch]; }
    if (meta) { meta[0] = c->next_sweep; meta[1] = c->n_avg; meta[2] = c->phase; }
    return ORC_OK;
}

int orc_set_state(orc_ctx* c, const double* phi, const double* acc, const double* ctl,
                  const int64_t* meta)
{
    if (!c) return ORC_EINVAL;
    if (c->phase < PH_LOADED) return ORC_ESTATE;
    int C = c->cfg.n_chains;
    if (phi) {
        for (int ch = 0; ch < C; ++ch)
            for (int64_t i = 0; i < c->n; ++i) {
                if (c->mask[i]) continue;    /* sample sites stay as loaded */
                double v = phi[(size_t)ch * c->n + i];
                if (!(v >= 0.0 && v <= TWO_PI)) return ORC_EINVAL;
            }
        for (int ch = 0; ch < C; ++ch)
            for (int64_t i = 0; i < c->n; ++i)
                if (!c->mask[i]) c->phi[(size_t)ch * c->n + i] = phi[(size_t)ch * c->n + i];
    }
    if (acc) memcpy(c->acc, acc, (size_t)c->n * C * sizeof(double));
    if (ctl)
        for (int ch = 0; ch < C; ++ch) { c->T[ch] = ctl[2 * ch]; c->alpha[ch] = ctl[2 * ch + 1]; }
    if (meta) {
        if (meta[0] < 0 || meta[1] < 0 || meta[2] < PH_LOADED || meta[2] > PH_AVERAGED)
            return ORC_EINVAL;
        c->next_sweep = meta[0]; c->n_avg = meta[1]; c->phase = (int32_t)meta[2];
    }
    return ORC_OK;
}

int orc_debug_sweep(orc_ctx* c, int32_t sweep, uint8_t* decisions)
{
    if (!c || !decisions || sweep < 0) return ORC_EINVAL;
    if (c->phase < PH_TEMPERED) return ORC_ESTATE;
    const orc_config* g = &c->cfg;
    for (int ch = 0; ch < g->n_chains; ++ch) {
        uint8_t* d = decisions + (size_t)ch * c->n;
        memset(d, 0, (size_t)c->n);
        orc_sweep(c->H, c->W, c->phi + (size_t)ch * c->n, c->mask, g->boundary, g->q, g->J,
                  c->T[ch], c->alpha[ch], g->seed, (uint32_t)sweep, chain_word(c, ch),
                  g->n_threads, d);
    }
    return ORC_OK;
}

int orc_burn_in(orc_ctx* c, int32_t n)
{
    if (!c) return ORC_EINVAL;
    if (n < 0) return ORC_EINVAL;
    if (c->phase < PH_TEMPERED) return ORC_ESTATE;
    const orc_config* g = &c->cfg;
    for (int ch = 0; ch < g->n_chains; ++ch)
        for (int32_t s = 0; s < n; ++s) {
            int64_t acc = orc_sweep(c->H, c->W, c->phi + (size_t)ch * c->n, c->mask,
                                    g->boundary, g->q, g->J, c->T[ch], c->alpha[ch], g->seed,
                                    (uint32_t)(c->next_sweep + s), chain_word(c, ch),
                                    g->n_threads, NULL);
            c->acc_rate[ch] = c->n_pred > 0 ? (double)acc / (double)c->n_pred : 0.0;
        }
    c->next_sweep += n;
    return ORC_OK;
}

int orc_run_record(orc_ctx* c, int32_t n, int32_t n_sites, const int64_t* sites, double* out)
{
    if (!c || !out || !sites || n < 0 || n_sites < 1) return ORC_EINVAL;
    if (c->phase < PH_TEMPERED) return ORC_ESTATE;
    for (int32_t k = 0; k < n_sites; ++k)
        if (sites[k] < 0 || sites[k] >= c->n) return ORC_EINVAL;
    const orc_config* g = &c->cfg;
    for (int32_t s = 0; s < n; ++s) {
        orc_sweep(c->H, c->W, c->phi, c->mask, g->boundary, g->q, g->J, c->T[0], c->alpha[0],
                  g->seed, (uint32_t)(c->next_sweep + s), chain_word(c, 0), g->n_threads, NULL);
        for (int32_t k = 0; k < n_sites; ++k) out[(size_t)s * n_sites + k] = c->phi[sites[k]];
    }
    c->next_sweep += n;
    return ORC_OK;
}

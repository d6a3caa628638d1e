/*
 * FP64 CPU oracle of the vectorial Maxwell-Bloch FDTD step (test
 * infrastructure only; see mb_oracle.h for the equations and units).
 *
 * Written as plain loops over separate arrays, one update after another, in
 * the order the step is defined: a1 (H), energy, a2 (P), a3 (E), a6 (Mur,
 * source), a4 (populations), a7 (monitors).  No fusion, no tiling; OpenMP only
 * splits the outer z loop.  Every floating-point quantity is FP64.  With
 * round_f32 set, each coefficient (and the initial populations) is rounded to
 * binary32 once, so that the oracle evaluates the same recurrence as an FP32
 * implementation that stores those coefficients in binary32; the arithmetic
 * itself stays FP64.
 */
#include "mb_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define ORC_C0 299792458.0
#define ORC_EPS0 8.8541878128e-12
#define ORC_HBAR 1.054571817e-34
#define ORC_PI 3.14159265358979323846

struct orc_sim {
    orc_params p;
    int nx, ny, nz;
    size_t sx, sy, ntot;
    double coef[ORC_C_COUNT];
    double rates[4];           /* dt32, dt21, dt10, dtWp before any freezing */
    double* f[ORC_NFIELDS];
    double* Hn[3];             /* H^{n+1/2} while a step runs */
    double* Eold[3];           /* E^n while a step runs */
    double* eps;               /* per cell, nx*ny*nz */
    double* inv_eps;
    uint8_t* gain;
    int64_t step;
    int src_on, src_kind, src_comp, src_i, src_j, src_k;
    double src_amp, src_ws, src_tp, src_t0;
    double* map;               /* energy density of plane map_k summed over steps */
    int map_k;
    int64_t map_count;
    int n_probes, n_freq;
    int32_t* probes;
    double* omega;
    double* spec;
    int box_on, box[6];
    double loss;
    double W_now, W_int;
    double* hist;
    int64_t hist_len, hist_cap;
    double* plane_sum;         /* per-plane partial sums, summed in order */
    double* prof[3][2];        /* loss profile per axis at integer / half positions */
    int init_kind;             /* initial populations of the last orc_set_pump */
};

static double rnd(const orc_sim* s, double v) { return s->p.round_f32 ? (double)(float)v : v; }

static size_t at(const orc_sim* s, int i, int j, int k) {
    return (size_t)i + s->sx * ((size_t)j + s->sy * (size_t)k);
}

static size_t cell_of(const orc_sim* s, int i, int j, int k) {
    return (size_t)i + (size_t)s->nx * ((size_t)j + (size_t)s->ny * (size_t)k);
}

static int dim(const orc_sim* s, int a) { return a == 0 ? s->nx : (a == 1 ? s->ny : s->nz); }

/* E-site (c; i,j,k) is interior (updated by Ampere's law) when its index along
 * c lies in [0, n_c) and its indices along the two other axes lie in [1, n). */
static int e_interior(const orc_sim* s, int c, int i, int j, int k) {
    int idx[3] = {i, j, k};
    for (int a = 0; a < 3; ++a) {
        if (a == c) {
            if (idx[a] < 0 || idx[a] >= dim(s, a)) return 0;
        } else {
            if (idx[a] < 1 || idx[a] >= dim(s, a)) return 0;
        }
    }
    return 1;
}

/* Loss a = sigma dt / (2 eps) of the graded layer at coordinate x (cells) on
 * axis a: a_max ((L - x)/L)^p near the low wall, a_max ((x - (n - L))/L)^p near
 * the high wall, 0 in between. */
static double layer_profile(const orc_sim* s, int a, double x) {
    if (s->p.bc[a] != ORC_ABSORB || s->p.absorb_cells <= 0) return 0.0;
    const double L = (double)s->p.absorb_cells;
    const double n = (double)dim(s, a);
    double v = 0.0;
    if (x < L) v += pow((L - x) / L, (double)s->p.absorb_order);
    if (x > n - L) v += pow((x - (n - L)) / L, (double)s->p.absorb_order);
    return s->p.absorb_rate * v;
}

/* loss of an E-site (half position along its own axis) or H-site (half
 * positions along the two other axes) */
static double site_loss(const orc_sim* s, int is_h, int c, int i, int j, int k) {
    const int idx[3] = {i, j, k};
    double a = 0.0;
    for (int ax = 0; ax < 3; ++ax) {
        const int half = is_h ? (ax != c) : (ax == c);
        a += s->prof[ax][half][idx[ax]];
    }
    return a;
}

/* Coefficients of the semi-implicit lossy update of a site with loss a:
 * X' = ca X + cb (increment), ca = (1 - a)/(1 + a), cb = 1/(1 + a).  Like
 * every other coefficient they are formed in FP64 and, with round_f32,
 * rounded once to binary32. */
static double layer_ca(const orc_sim* s, double a) { return rnd(s, (1.0 - a) / (1.0 + a)); }
static double layer_cb(const orc_sim* s, double a) { return rnd(s, 1.0 / (1.0 + a)); }

/* ---------------------------------------------------------------- Philox */

/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two 32x32
 * multiplications with the round constants 0xD2511F53 and 0xCD9E8D57, the key
 * advanced by the Weyl increments 0x9E3779B9 and 0xBB67AE85 between rounds. */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)x0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)x2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t y0 = hi1 ^ x1 ^ k0;
        uint32_t y1 = lo1;
        uint32_t y2 = hi0 ^ x3 ^ k1;
        uint32_t y3 = lo0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* Three standard normals for one cell and step: Philox words -> 24-bit
 * uniforms u = (w/256 + 1/2) / 2^24 in (0,1) -> Box-Muller pairs. */
void orc_normals3(uint64_t seed, uint32_t cell, uint32_t step, uint32_t realization,
                  double xi[3]) {
    uint32_t ctr[4] = {cell, step, realization, 0u};
    uint32_t key[2] = {(uint32_t)(seed & 0xFFFFFFFFu), (uint32_t)(seed >> 32)};
    uint32_t w[4];
    orc_philox4x32_10(ctr, key, w);
    double u[4];
    for (int q = 0; q < 4; ++q) u[q] = ((double)(w[q] >> 8) + 0.5) / 16777216.0;
    double r0 = sqrt(-2.0 * log(u[0]));
    double r1 = sqrt(-2.0 * log(u[2]));
    xi[0] = r0 * cos(2.0 * ORC_PI * u[1]);
    xi[1] = r0 * sin(2.0 * ORC_PI * u[1]);
    xi[2] = r1 * cos(2.0 * ORC_PI * u[3]);
}

/* ------------------------------------------------------- site updates */

/* a2: central-difference Lorentz oscillator driven by (N1 - N2) E plus noise */
double orc_p_next(const double* c, double P, double Pprev, double E, double dN, double xi) {
    return c[ORC_C_A] * P + c[ORC_C_B] * Pprev + c[ORC_C_CK] * dN * E + c[ORC_C_CF] * xi;
}

/* a4: forward-Euler four-level rates; N = {N0, N1, N2, N3} */
void orc_pop_next(const double* c, double N[4], double Ebar, double dP) {
    double W = c[ORC_C_BETA] * Ebar * dP;
    double n0 = N[0], n1 = N[1], n2 = N[2], n3 = N[3];
    N[0] = n0 + c[ORC_C_DT10] * n1 - c[ORC_C_DTWP] * n0;
    N[1] = n1 + c[ORC_C_DT21] * n2 - c[ORC_C_DT10] * n1 - W;
    N[2] = n2 + c[ORC_C_DT32] * n3 - c[ORC_C_DT21] * n2 + W;
    N[3] = n3 + c[ORC_C_DTWP] * n0 - c[ORC_C_DT32] * n3;
}

void orc_p_series(const double* coef, const double* E, const double* dN, int64_t n,
                  double* P_out) {
    double P = 0.0, Pprev = 0.0;
    for (int64_t t = 0; t < n; ++t) {
        double Pn = orc_p_next(coef, P, Pprev, E[t], dN[t], 0.0);
        Pprev = P;
        P = Pn;
        P_out[t] = P;
    }
}

void orc_pop_series(const double* coef, double N[4], const double* Ebar, const double* dP,
                    int64_t n, double* N_out) {
    for (int64_t t = 0; t < n; ++t) {
        orc_pop_next(coef, N, Ebar[t], dP[t]);
        for (int q = 0; q < 4; ++q) N_out[4 * t + q] = N[q];
    }
}

/* --------------------------------------------------------- lifecycle */

static void compute_coefficients(orc_sim* s) {
    const orc_params* p = &s->p;
    double dt = p->courant * p->dx / (ORC_C0 * sqrt(3.0));
    double S = ORC_C0 * dt / p->dx;
    double wa = 2.0 * ORC_PI * ORC_C0 / p->lambda0;
    double dwa = 2.0 * ORC_PI * ORC_C0 * p->dlambda / (p->lambda0 * p->lambda0);
    double kappa = 6.0 * ORC_PI * ORC_EPS0 * ORC_C0 * ORC_C0 * ORC_C0 / (wa * wa * p->tau21);
    double omp2 = kappa * p->N_ref / ORC_EPS0;
    double D = 1.0 + 0.5 * dwa * dt;
    double beta = ORC_EPS0 * p->E_ref * p->E_ref / (ORC_HBAR * wa * p->N_ref);
    double* c = s->coef;
    c[ORC_C_DT] = dt;
    c[ORC_C_S] = rnd(s, S);
    c[ORC_C_A] = rnd(s, (2.0 - wa * wa * dt * dt) / D);
    c[ORC_C_B] = rnd(s, -(1.0 - 0.5 * dwa * dt) / D);
    c[ORC_C_CK] = rnd(s, dt * dt * omp2 / D);
    c[ORC_C_WA] = wa;
    c[ORC_C_DWA] = dwa;
    c[ORC_C_OMP2] = omp2;
    s->rates[0] = rnd(s, dt / p->tau32);
    s->rates[1] = rnd(s, dt / p->tau21);
    s->rates[2] = rnd(s, dt / p->tau10);
    s->rates[3] = rnd(s, dt * p->Wp);
    if (p->frozen_pop) {
        c[ORC_C_BETA] = 0.0;
        c[ORC_C_DT32] = c[ORC_C_DT21] = c[ORC_C_DT10] = c[ORC_C_DTWP] = 0.0;
    } else {
        c[ORC_C_BETA] = rnd(s, beta);
        c[ORC_C_DT32] = s->rates[0];
        c[ORC_C_DT21] = s->rates[1];
        c[ORC_C_DT10] = s->rates[2];
        c[ORC_C_DTWP] = s->rates[3];
    }
    c[ORC_C_NA] = 0.0;
    c[ORC_C_CF] = 0.0;
}

orc_sim* orc_create(const orc_params* p) {
    if (!p || p->nx < 2 || p->ny < 2 || p->nz < 2) return NULL;
    if (!(p->courant > 0.0 && p->courant <= 1.0)) return NULL;
    orc_sim* s = (orc_sim*)calloc(1, sizeof(orc_sim));
    if (!s) return NULL;
    s->p = *p;
    s->nx = p->nx; s->ny = p->ny; s->nz = p->nz;
    s->sx = (size_t)p->nx + 1;
    s->sy = (size_t)p->ny + 1;
    s->ntot = s->sx * s->sy * ((size_t)p->nz + 1);
    for (int q = 0; q < ORC_NFIELDS; ++q) s->f[q] = (double*)calloc(s->ntot, sizeof(double));
    for (int q = 0; q < 3; ++q) {
        s->Hn[q] = (double*)calloc(s->ntot, sizeof(double));
        s->Eold[q] = (double*)calloc(s->ntot, sizeof(double));
    }
    size_t ncell = (size_t)p->nx * p->ny * p->nz;
    s->eps = (double*)malloc(ncell * sizeof(double));
    s->inv_eps = (double*)malloc(ncell * sizeof(double));
    s->gain = (uint8_t*)calloc(ncell, 1);
    s->plane_sum = (double*)calloc((size_t)p->nz + 1, sizeof(double));
    for (size_t q = 0; q < ncell; ++q) { s->eps[q] = 1.0; s->inv_eps[q] = 1.0; }
    for (int a = 0; a < 3; ++a)
        for (int h = 0; h < 2; ++h) {
            const int n = dim(s, a);
            s->prof[a][h] = (double*)calloc((size_t)n + 1, sizeof(double));
            for (int q = 0; q <= n; ++q)
                s->prof[a][h][q] = rnd(s, layer_profile(s, a, (double)q + (h ? 0.5 : 0.0)));
        }
    compute_coefficients(s);
    return s;
}

void orc_destroy(orc_sim* s) {
    if (!s) return;
    for (int q = 0; q < ORC_NFIELDS; ++q) free(s->f[q]);
    for (int q = 0; q < 3; ++q) { free(s->Hn[q]); free(s->Eold[q]); }
    free(s->eps); free(s->inv_eps); free(s->gain); free(s->plane_sum);
    for (int a = 0; a < 3; ++a) { free(s->prof[a][0]); free(s->prof[a][1]); }
    free(s->probes); free(s->omega); free(s->spec); free(s->hist); free(s->map);
    free(s);
}

void orc_coefficients(const orc_sim* s, double* out) {
    memcpy(out, s->coef, sizeof(double) * ORC_C_COUNT);
}

int orc_set_material(orc_sim* s, const float* eps_r, const uint8_t* gain) {
    size_t ncell = (size_t)s->nx * s->ny * s->nz;
    for (size_t q = 0; q < ncell; ++q) {
        double e = (double)eps_r[q];
        if (!(e > 0.0)) return -1;
        s->eps[q] = e;
        s->inv_eps[q] = rnd(s, 1.0 / e);
        s->gain[q] = gain[q] ? 1 : 0;
    }
    return 0;
}

static void reset_monitors(orc_sim* s) {
    s->step = 0;
    s->W_now = s->W_int = 0.0;
    s->hist_len = 0;
    s->loss = 0.0;
    if (s->spec) memset(s->spec, 0, sizeof(double) * 2 * (size_t)s->n_probes * s->n_freq);
    if (s->map) memset(s->map, 0, sizeof(double) * (size_t)s->nx * s->ny);
    s->map_count = 0;
}

int orc_set_pump(orc_sim* s, double Na_si, int init) {
    double Na = Na_si / s->p.N_ref;
    s->coef[ORC_C_NA] = rnd(s, Na);
    {
        /* cF = ck * Na * E_sp from unrounded FP64 factors, then rounded once */
        double dt = s->coef[ORC_C_DT];
        double D = 1.0 + 0.5 * s->coef[ORC_C_DWA] * dt;
        double ck = dt * dt * s->coef[ORC_C_OMP2] / D;
        s->coef[ORC_C_CF] = s->p.noise ? rnd(s, ck * Na * s->p.E_sp) : 0.0;
    }
    double N[4] = {0, 0, 0, 0};
    double na = s->coef[ORC_C_NA];
    if (init == ORC_INIT_GROUND) {
        N[0] = na;
    } else if (init == ORC_INIT_PREPUMPED) {
        /* E = 0 fixed point of the discrete rates (null space of the rate
         * matrix): dtWp N0 = dt32 N3 = dt21 N2 = dt10 N1 with N0 = N_a - N1 -
         * N2 - N3.  N2, which holds almost all atoms, is set first; N1 and N3
         * then solve their own equations for the rounded N2 (N3 with N0 =
         * N_a - N1 - N2 - N3, i.e. N3 = dtWp (N_a - N1 - N2)/(dt32 + dtWp)),
         * so that with rounded populations each equation is off by the
         * rounding of its own population only (N3 computed from the unrounded
         * N0 would be off by the rounding of N2, relative to the small N0) */
        double d32 = s->rates[0], d21 = s->rates[1], d10 = s->rates[2], dwp = s->rates[3];
        double n0 = na / (1.0 + dwp / d32 + dwp / d21 + dwp / d10);
        N[2] = rnd(s, dwp * n0 / d21);
        N[1] = rnd(s, d21 * N[2] / d10);
        N[3] = rnd(s, dwp * (na - N[1] - N[2]) / (d32 + dwp));
        N[0] = na - (N[1] + N[2] + N[3]);
    } else {
        return -1;
    }
    s->init_kind = init;
    for (int q = 0; q < 12; ++q) memset(s->f[q], 0, sizeof(double) * s->ntot);
    for (int q = 12; q < 24; ++q) memset(s->f[q], 0, sizeof(double) * s->ntot);
    for (int k = 0; k <= s->nz; ++k)
        for (int j = 0; j <= s->ny; ++j)
            for (int i = 0; i <= s->nx; ++i)
                for (int c = 0; c < 3; ++c) {
                    if (!e_interior(s, c, i, j, k) || !s->gain[cell_of(s, i, j, k)]) continue;
                    size_t x = at(s, i, j, k);
                    s->f[12 + c][x] = N[1];
                    s->f[15 + c][x] = N[2];
                    s->f[18 + c][x] = N[3];
                    s->f[21 + c][x] = N[0];
                }
    reset_monitors(s);
    return 0;
}

int orc_set_source(orc_sim* s, int comp, int i, int j, int k, double amp,
                   double lambda_s, double tau_p, double t0) {
    if (comp < 0 || comp > 2 || !e_interior(s, comp, i, j, k)) return -1;
    s->src_on = 1;
    s->src_kind = 0;
    s->src_comp = comp; s->src_i = i; s->src_j = j; s->src_k = k;
    s->src_amp = amp;
    s->src_ws = 2.0 * ORC_PI * ORC_C0 / lambda_s;
    s->src_tp = tau_p;
    s->src_t0 = t0;
    return 0;
}

int orc_set_cw_source(orc_sim* s, int comp, int i, int j, int k, double amp,
                      double lambda_s, double t_ramp) {
    if (comp < 0 || comp > 2 || !e_interior(s, comp, i, j, k) || !(t_ramp > 0.0)) return -1;
    s->src_on = 1;
    s->src_kind = 1;
    s->src_comp = comp; s->src_i = i; s->src_j = j; s->src_k = k;
    s->src_amp = amp;
    s->src_ws = 2.0 * ORC_PI * ORC_C0 / lambda_s;
    s->src_tp = t_ramp;
    s->src_t0 = 0.0;
    return 0;
}

/* soft source added to E^{n+1} during step n, evaluated at t = (n+1) dt:
 * the Gaussian pulse, or the continuous wave with a Gaussian switch-on */
double orc_source_value(const orc_sim* s, int64_t n) {
    if (!s->src_on) return 0.0;
    if (s->src_kind == 1) {
        double t = (double)(n + 1) * s->coef[ORC_C_DT];
        double ramp = 1.0 - exp(-(t / s->src_tp) * (t / s->src_tp));
        return rnd(s, s->src_amp * ramp * sin(s->src_ws * t));
    }
    double t = (double)(n + 1) * s->coef[ORC_C_DT] - s->src_t0;
    double v = s->src_amp * sin(s->src_ws * t) * exp(-(t / s->src_tp) * (t / s->src_tp));
    return rnd(s, v);
}

int orc_set_plane_monitor(orc_sim* s, int k) {
    if (k < -1 || k >= s->nz) return -1;
    free(s->map);
    s->map = NULL;
    s->map_k = -1;
    s->map_count = 0;
    if (k < 0) return 0;
    s->map = (double*)calloc((size_t)s->nx * s->ny, sizeof(double));
    if (!s->map) return -1;
    s->map_k = k;
    return 0;
}

int64_t orc_read_plane_monitor(const orc_sim* s, double* out) {
    if (!s->map) return -1;
    memcpy(out, s->map, sizeof(double) * (size_t)s->nx * s->ny);
    return s->map_count;
}

/* energy density 1/2 [eps |E^n|^2 + |H^{n+1/2}|^2] of the cells of plane
 * map_k from their own sites (i, j, map_k), added to the sums */
static void plane_monitor(orc_sim* s) {
    if (!s->map) return;
    const int k = s->map_k;
    for (int j = 0; j < s->ny; ++j)
        for (int i = 0; i < s->nx; ++i) {
            size_t x = at(s, i, j, k);
            double e2 = (s->f[0][x] * s->f[0][x] + s->f[1][x] * s->f[1][x]) + s->f[2][x] * s->f[2][x];
            double h2 = (s->Hn[0][x] * s->Hn[0][x] + s->Hn[1][x] * s->Hn[1][x]) + s->Hn[2][x] * s->Hn[2][x];
            s->map[(size_t)i + (size_t)s->nx * j] += 0.5 * (s->eps[cell_of(s, i, j, k)] * e2 + h2);
        }
    s->map_count++;
}

int orc_set_probes(orc_sim* s, const int32_t* sites, int n_probes, const double* omega,
                   int n_freq) {
    for (int q = 0; q < n_probes; ++q) {
        const int32_t* r = sites + 4 * q;
        if (r[0] < 0 || r[0] > 2 || r[1] < 0 || r[1] > s->nx || r[2] < 0 || r[2] > s->ny ||
            r[3] < 0 || r[3] > s->nz)
            return -1;
    }
    free(s->probes); free(s->omega); free(s->spec);
    s->n_probes = n_probes;
    s->n_freq = n_freq;
    s->probes = (int32_t*)malloc(sizeof(int32_t) * 4 * (size_t)(n_probes > 0 ? n_probes : 1));
    s->omega = (double*)malloc(sizeof(double) * (size_t)(n_freq > 0 ? n_freq : 1));
    s->spec = (double*)calloc(2 * (size_t)(n_probes > 0 ? n_probes : 1) * (n_freq > 0 ? n_freq : 1),
                              sizeof(double));
    memcpy(s->probes, sites, sizeof(int32_t) * 4 * (size_t)n_probes);
    memcpy(s->omega, omega, sizeof(double) * (size_t)n_freq);
    return 0;
}

int orc_set_loss_box(orc_sim* s, int i0, int j0, int k0, int i1, int j1, int k1) {
    if (i0 < 0 || j0 < 0 || k0 < 0 || i1 > s->nx || j1 > s->ny || k1 > s->nz || i0 >= i1 ||
        j0 >= j1 || k0 >= k1)
        return -1;
    s->box_on = 1;
    s->box[0] = i0; s->box[1] = j0; s->box[2] = k0;
    s->box[3] = i1; s->box[4] = j1; s->box[5] = k1;
    return 0;
}

int64_t orc_step_index(const orc_sim* s) { return s->step; }

int orc_get_field(const orc_sim* s, int id, double* out) {
    if (id < 0 || id >= ORC_NFIELDS) return -1;
    memcpy(out, s->f[id], sizeof(double) * s->ntot);
    return 0;
}

int orc_set_field(orc_sim* s, int id, const double* in) {
    if (id < 0 || id >= ORC_NFIELDS) return -1;
    memcpy(s->f[id], in, sizeof(double) * s->ntot);
    return 0;
}

void orc_read_energy(const orc_sim* s, double* W_now, double* W_int) {
    *W_now = s->W_now;
    *W_int = s->W_int;
}

int64_t orc_energy_history(const orc_sim* s, double* out, int64_t cap) {
    int64_t n = s->hist_len < cap ? s->hist_len : cap;
    if (out && n > 0) memcpy(out, s->hist, sizeof(double) * (size_t)n);
    return s->hist_len;
}

void orc_read_spectrum(const orc_sim* s, double* re_im) {
    memcpy(re_im, s->spec, sizeof(double) * 2 * (size_t)s->n_probes * s->n_freq);
}

double orc_read_loss(const orc_sim* s) { return s->loss; }

/* ------------------------------------------------------------- step */

/* a1: H^{n+1/2} = H^{n-1/2} - S curl+ E^n on every H-site of [0,n)^3 */
static void update_h(orc_sim* s) {
    const double S = s->coef[ORC_C_S];
    double *Ex = s->f[0], *Ey = s->f[1], *Ez = s->f[2];
    double *Hx = s->f[3], *Hy = s->f[4], *Hz = s->f[5];
#pragma omp parallel for schedule(static)
    for (int k = 0; k < s->nz; ++k)
        for (int j = 0; j < s->ny; ++j)
            for (int i = 0; i < s->nx; ++i) {
                size_t x = at(s, i, j, k);
                size_t xi = at(s, i + 1, j, k), xj = at(s, i, j + 1, k), xk = at(s, i, j, k + 1);
                double cx = (Ez[xj] - Ez[x]) - (Ey[xk] - Ey[x]);
                double cy = (Ex[xk] - Ex[x]) - (Ez[xi] - Ez[x]);
                double cz = (Ey[xi] - Ey[x]) - (Ex[xj] - Ex[x]);
                const double c3[3] = {cx, cy, cz};
                const double* H3[3] = {Hx, Hy, Hz};
                for (int c = 0; c < 3; ++c) {
                    const double a = site_loss(s, 1, c, i, j, k);
                    if (a == 0.0) {
                        s->Hn[c][x] = H3[c][x] - S * c3[c];
                    } else {
                        /* semi-implicit loss: (H' - H) = -S curl - a (H' + H) */
                        s->Hn[c][x] = layer_ca(s, a) * H3[c][x] - layer_cb(s, a) * (S * c3[c]);
                    }
                }
            }
}

/* W^n = 1/2 [ sum_interior-E eps |E^n|^2 + sum_H H^{n-1/2} . H^{n+1/2} ];
 * H-sites on the wall normal to their own component are excluded. */
static double energy(orc_sim* s) {
#pragma omp parallel for schedule(static)
    for (int k = 0; k < s->nz; ++k) {
        double acc = 0.0;
        for (int j = 0; j < s->ny; ++j)
            for (int i = 0; i < s->nx; ++i) {
                size_t x = at(s, i, j, k);
                double e = s->eps[cell_of(s, i, j, k)];
                int idx[3] = {i, j, k};
                for (int c = 0; c < 3; ++c) {
                    if (e_interior(s, c, i, j, k)) acc += e * s->f[c][x] * s->f[c][x];
                    if (idx[c] >= 1) acc += s->f[3 + c][x] * s->Hn[c][x];
                }
            }
        s->plane_sum[k] = acc;
    }
    double W = 0.0;
    for (int k = 0; k < s->nz; ++k) W += s->plane_sum[k];
    return 0.5 * W;
}

/* a2: P^{n+1} at interior gain E-sites; afterwards f[6+c] = P^{n+1} and
 * f[9+c] = P^n. */
static void update_p(orc_sim* s) {
    const double* coef = s->coef;
    const int noise = s->p.noise && coef[ORC_C_CF] != 0.0;
    const uint32_t n = (uint32_t)s->step;
#pragma omp parallel for schedule(static)
    for (int k = 0; k < s->nz; ++k)
        for (int j = 0; j < s->ny; ++j)
            for (int i = 0; i < s->nx; ++i) {
                size_t cell = cell_of(s, i, j, k);
                if (!s->gain[cell]) continue;
                size_t x = at(s, i, j, k);
                double xi[3] = {0.0, 0.0, 0.0};
                if (noise) orc_normals3(s->p.seed, (uint32_t)cell, n, s->p.realization, xi);
                for (int c = 0; c < 3; ++c) {
                    if (!e_interior(s, c, i, j, k)) continue;
                    double P = s->f[6 + c][x], Pp = s->f[9 + c][x];
                    double dN = s->f[12 + c][x] - s->f[15 + c][x];
                    double Pn = orc_p_next(coef, P, Pp, s->f[c][x], dN, xi[c]);
                    s->f[9 + c][x] = P;
                    s->f[6 + c][x] = Pn;
                }
            }
}

/* a3: E^{n+1} at interior E-sites (E^n kept in Eold) */
static void update_e(orc_sim* s) {
    const double S = s->coef[ORC_C_S];
    for (int c = 0; c < 3; ++c) memcpy(s->Eold[c], s->f[c], sizeof(double) * s->ntot);
    double *Hx = s->Hn[0], *Hy = s->Hn[1], *Hz = s->Hn[2];
#pragma omp parallel for schedule(static)
    for (int k = 0; k < s->nz; ++k)
        for (int j = 0; j < s->ny; ++j)
            for (int i = 0; i < s->nx; ++i) {
                size_t x = at(s, i, j, k);
                size_t cell = cell_of(s, i, j, k);
                double ie = s->inv_eps[cell];
                int g = s->gain[cell];
                for (int c = 0; c < 3; ++c) {
                    if (!e_interior(s, c, i, j, k)) continue;
                    double curl;
                    if (c == 0)
                        curl = (Hz[x] - Hz[at(s, i, j - 1, k)]) - (Hy[x] - Hy[at(s, i, j, k - 1)]);
                    else if (c == 1)
                        curl = (Hx[x] - Hx[at(s, i, j, k - 1)]) - (Hz[x] - Hz[at(s, i - 1, j, k)]);
                    else
                        curl = (Hy[x] - Hy[at(s, i - 1, j, k)]) - (Hx[x] - Hx[at(s, i, j - 1, k)]);
                    double dP = g ? s->f[6 + c][x] - s->f[9 + c][x] : 0.0;
                    const double a = site_loss(s, 0, c, i, j, k);
                    if (a == 0.0)
                        s->f[c][x] = s->Eold[c][x] + ie * (S * curl - dP);
                    else
                        s->f[c][x] = layer_ca(s, a) * s->Eold[c][x] +
                                     layer_cb(s, a) * (ie * (S * curl - dP));
                }
            }
    for (int c = 0; c < 3; ++c) memcpy(s->f[3 + c], s->Hn[c], sizeof(double) * s->ntot);
}

static double mur_coef(const orc_sim* s, int i, int j, int k) {
    int ci = i < s->nx ? i : s->nx - 1;
    int cj = j < s->ny ? j : s->ny - 1;
    int ck = k < s->nz ? k : s->nz - 1;
    double e = s->eps[cell_of(s, ci, cj, ck)];
    double sp = (ORC_C0 * s->coef[ORC_C_DT] / s->p.dx) / sqrt(e);
    return rnd(s, (sp - 1.0) / (sp + 1.0));
}

/* a6: first-order Mur on the faces of Mur axes, applied face by face in x, y,
 * z order in place (so an edge keeps the value of its last face).  A site on
 * any PEC wall (or the conducting wall behind a lossy layer) is never written
 * and stays zero. */
static void apply_mur(orc_sim* s) {
    const int n[3] = {s->nx, s->ny, s->nz};
    for (int a = 0; a < 3; ++a) {
        if (s->p.bc[a] != ORC_MUR1) continue;
        for (int c = 0; c < 3; ++c) {
            if (c == a) continue;
            double* E = s->f[c];
            double* Eo = s->Eold[c];
            for (int side = 0; side < 2; ++side) {
                int wall = side ? n[a] : 0;
                int inner = side ? n[a] - 1 : 1;
                int lo[3] = {0, 0, 0}, hi[3] = {n[0] + 1, n[1] + 1, n[2] + 1};
                hi[c] = n[c];
                lo[a] = wall; hi[a] = wall + 1;
                for (int k = lo[2]; k < hi[2]; ++k)
                    for (int j = lo[1]; j < hi[1]; ++j)
                        for (int i = lo[0]; i < hi[0]; ++i) {
                            int idx[3] = {i, j, k};
                            int on_pec = 0;
                            for (int b = 0; b < 3; ++b)   /* PEC and lossy-layer walls conduct */
                                if (b != c && s->p.bc[b] != ORC_MUR1 && (idx[b] == 0 || idx[b] == n[b]))
                                    on_pec = 1;
                            if (on_pec) continue;
                            int jdx[3] = {i, j, k};
                            jdx[a] = inner;
                            size_t xb = at(s, i, j, k);
                            size_t x1 = at(s, jdx[0], jdx[1], jdx[2]);
                            double m = mur_coef(s, i, j, k);
                            E[xb] = Eo[x1] + m * (E[x1] - Eo[xb]);
                        }
            }
        }
    }
}

/* a4: populations at interior gain E-sites */
static void update_pop(orc_sim* s) {
    const double* coef = s->coef;
#pragma omp parallel for schedule(static)
    for (int k = 0; k < s->nz; ++k)
        for (int j = 0; j < s->ny; ++j)
            for (int i = 0; i < s->nx; ++i) {
                if (!s->gain[cell_of(s, i, j, k)]) continue;
                size_t x = at(s, i, j, k);
                for (int c = 0; c < 3; ++c) {
                    if (!e_interior(s, c, i, j, k)) continue;
                    double N[4] = {s->f[21 + c][x], s->f[12 + c][x], s->f[15 + c][x], s->f[18 + c][x]};
                    double Ebar = 0.5 * (s->f[c][x] + s->Eold[c][x]);
                    double dP = s->f[6 + c][x] - s->f[9 + c][x];
                    orc_pop_next(coef, N, Ebar, dP);
                    s->f[21 + c][x] = N[0];
                    s->f[12 + c][x] = N[1];
                    s->f[15 + c][x] = N[2];
                    s->f[18 + c][x] = N[3];
                }
            }
}

static void monitors_after(orc_sim* s) {
    const double dt = s->coef[ORC_C_DT];
    const double tn = (double)(s->step + 1) * dt;
    if (s->box_on) {
        double acc = 0.0;
        for (int k = s->box[2]; k < s->box[5]; ++k)
            for (int j = s->box[1]; j < s->box[4]; ++j)
                for (int i = s->box[0]; i < s->box[3]; ++i)
                    for (int c = 0; c < 3; ++c)
                        if (e_interior(s, c, i, j, k)) {
                            double e = s->f[c][at(s, i, j, k)];
                            acc += e * e;
                        }
        s->loss += acc;
    }
    for (int q = 0; q < s->n_probes; ++q) {
        const int32_t* r = s->probes + 4 * q;
        double e = s->f[r[0]][at(s, r[1], r[2], r[3])];
        for (int w = 0; w < s->n_freq; ++w) {
            double ph = s->omega[w] * tn;
            size_t o = 2 * ((size_t)q * s->n_freq + w);
            s->spec[o] += e * cos(ph);
            s->spec[o + 1] += e * sin(ph);
        }
    }
}

static void push_energy(orc_sim* s, double W) {
    if (s->hist_len == s->hist_cap) {
        int64_t cap = s->hist_cap ? 2 * s->hist_cap : 1024;
        s->hist = (double*)realloc(s->hist, sizeof(double) * (size_t)cap);
        s->hist_cap = cap;
    }
    s->hist[s->hist_len++] = W;
    s->W_now = W;
    s->W_int += W;
}

int orc_step(orc_sim* s, int64_t nsteps) {
    for (int64_t t = 0; t < nsteps; ++t) {
        update_h(s);
        push_energy(s, energy(s));
        plane_monitor(s);
        update_p(s);
        update_e(s);
        apply_mur(s);
        if (s->src_on)
            s->f[s->src_comp][at(s, s->src_i, s->src_j, s->src_k)] += orc_source_value(s, s->step);
        update_pop(s);
        monitors_after(s);
        s->step++;
    }
    return 0;
}

/* ============================================================ adjoint
 * Reverse-mode derivative of the loss-box objective
 *     L = sum over steps n = 1..N of sum over interior E-sites in the box of (E^n)^2
 * with respect to eps_r of every cell and to the pump density N_a, for runs
 * that start from orc_set_pump (step 0).  The state of step n is the 24 site
 * arrays X^n = (E, H, P, P_prev, N1, N2, N3, N0); one step is the map
 * X^{n+1} = F(X^n; eps, N_a) of orc_step, and the adjoint runs the transposed
 * linearisation of F backwards over the stored trajectory.  Mur walls are not
 * supported (their coefficient would make the wall rows depend on eps). */

typedef double* state_t[ORC_NFIELDS];

static int state_alloc(const orc_sim* s, state_t X) {
    for (int q = 0; q < ORC_NFIELDS; ++q) {
        X[q] = (double*)calloc(s->ntot, sizeof(double));
        if (!X[q]) return -1;
    }
    return 0;
}

static void state_free(state_t X) {
    for (int q = 0; q < ORC_NFIELDS; ++q) { free(X[q]); X[q] = NULL; }
}

/* The sim's fields after one more step, computed on a copy. */
static int forward_copy(const orc_sim* s, state_t X1) {
    orc_sim* t = orc_create(&s->p);
    if (!t) return -1;
    size_t ncell = (size_t)s->nx * s->ny * s->nz;
    memcpy(t->eps, s->eps, ncell * sizeof(double));
    memcpy(t->inv_eps, s->inv_eps, ncell * sizeof(double));
    memcpy(t->gain, s->gain, ncell);
    memcpy(t->coef, s->coef, sizeof(s->coef));
    memcpy(t->rates, s->rates, sizeof(s->rates));
    for (int q = 0; q < ORC_NFIELDS; ++q) memcpy(t->f[q], s->f[q], sizeof(double) * s->ntot);
    t->step = s->step;
    t->src_on = s->src_on; t->src_kind = s->src_kind; t->src_comp = s->src_comp;
    t->src_i = s->src_i; t->src_j = s->src_j; t->src_k = s->src_k;
    t->src_amp = s->src_amp; t->src_ws = s->src_ws; t->src_tp = s->src_tp; t->src_t0 = s->src_t0;
    orc_step(t, 1);
    for (int q = 0; q < ORC_NFIELDS; ++q) memcpy(X1[q], t->f[q], sizeof(double) * s->ntot);
    orc_destroy(t);
    return 0;
}

static int has_mur(const orc_sim* s) {
    return s->p.bc[0] == ORC_MUR1 || s->p.bc[1] == ORC_MUR1 || s->p.bc[2] == ORC_MUR1;
}

/* curl- of an H-type array at E-site (c; i,j,k) and curl+ of an E-type array
 * at H-site (c; i,j,k), the stencils of a3 and a1.  Values outside the
 * extended range count as zero. */
static double get0(const orc_sim* s, const double* a, int i, int j, int k) {
    if (i < 0 || j < 0 || k < 0 || i > s->nx || j > s->ny || k > s->nz) return 0.0;
    return a[at(s, i, j, k)];
}

static double curl_minus(const orc_sim* s, double* const* h, int c, int i, int j, int k) {
    if (c == 0) return (get0(s, h[2], i, j, k) - get0(s, h[2], i, j - 1, k)) - (get0(s, h[1], i, j, k) - get0(s, h[1], i, j, k - 1));
    if (c == 1) return (get0(s, h[0], i, j, k) - get0(s, h[0], i, j, k - 1)) - (get0(s, h[2], i, j, k) - get0(s, h[2], i - 1, j, k));
    return (get0(s, h[1], i, j, k) - get0(s, h[1], i - 1, j, k)) - (get0(s, h[0], i, j, k) - get0(s, h[0], i, j - 1, k));
}

static double curl_plus(const orc_sim* s, double* const* e, int c, int i, int j, int k) {
    if (c == 0) return (get0(s, e[2], i, j + 1, k) - get0(s, e[2], i, j, k)) - (get0(s, e[1], i, j, k + 1) - get0(s, e[1], i, j, k));
    if (c == 1) return (get0(s, e[0], i, j, k + 1) - get0(s, e[0], i, j, k)) - (get0(s, e[2], i + 1, j, k) - get0(s, e[2], i, j, k));
    return (get0(s, e[1], i + 1, j, k) - get0(s, e[1], i, j, k)) - (get0(s, e[0], i, j + 1, k) - get0(s, e[0], i, j, k));
}

static int h_updated(const orc_sim* s, int i, int j, int k) {
    return i < s->nx && j < s->ny && k < s->nz;
}

/* Tangent-linear step: dX1 = J(X0) dX0, the derivative of one step taken at
 * X0 (X1 = F(X0) given) with eps and N_a fixed. */
static void tangent_step(const orc_sim* s, state_t X0, state_t X1, double* const* v, double** y) {
    const double* c = s->coef;
    const double S = c[ORC_C_S];
    for (int q = 0; q < ORC_NFIELDS; ++q) memcpy(y[q], v[q], sizeof(double) * s->ntot);
    /* H' = da H - db S curl+ E on [0,n)^3; the step leaves the other H-sites at
     * zero (they are never updated), so their derivative is zero */
    for (int q = 3; q < 6; ++q) memset(y[q], 0, sizeof(double) * s->ntot);
    for (int k = 0; k < s->nz; ++k)
        for (int j = 0; j < s->ny; ++j)
            for (int i = 0; i < s->nx; ++i)
                for (int cc = 0; cc < 3; ++cc) {
                    const double a = site_loss(s, 1, cc, i, j, k);
                    const double da = layer_ca(s, a), db = layer_cb(s, a);
                    y[3 + cc][at(s, i, j, k)] = da * v[3 + cc][at(s, i, j, k)] - db * S * curl_plus(s, (double* const*)v, cc, i, j, k);
                }
    for (int k = 0; k <= s->nz; ++k)
        for (int j = 0; j <= s->ny; ++j)
            for (int i = 0; i <= s->nx; ++i)
                for (int cc = 0; cc < 3; ++cc) {
                    if (!e_interior(s, cc, i, j, k)) continue;
                    const size_t x = at(s, i, j, k), cell = cell_of(s, i, j, k);
                    const double ie = s->inv_eps[cell];
                    const double a = site_loss(s, 0, cc, i, j, k);
                    const double ca = layer_ca(s, a), cb = layer_cb(s, a);
                    double ddP = 0.0;
                    if (s->gain[cell]) {
                        const double E = X0[cc][x], dN = X0[12 + cc][x] - X0[15 + cc][x];
                        const double dPn = c[ORC_C_A] * v[6 + cc][x] + c[ORC_C_B] * v[9 + cc][x] +
                                           c[ORC_C_CK] * (v[12 + cc][x] - v[15 + cc][x]) * E +
                                           c[ORC_C_CK] * dN * v[cc][x];
                        ddP = dPn - v[6 + cc][x];
                        y[6 + cc][x] = dPn;
                        y[9 + cc][x] = v[6 + cc][x];
                    }
                    const double dEn = ca * v[cc][x] + cb * ie * (S * curl_minus(s, y + 3, cc, i, j, k) - ddP);
                    y[cc][x] = dEn;
                    if (s->gain[cell]) {
                        const double dPf = X1[6 + cc][x] - X0[6 + cc][x];
                        const double dW = c[ORC_C_BETA] * 0.5 * ((dEn + v[cc][x]) * dPf + (X1[cc][x] + X0[cc][x]) * ddP);
                        const double n0 = v[21 + cc][x], n1 = v[12 + cc][x], n2 = v[15 + cc][x], n3 = v[18 + cc][x];
                        y[21 + cc][x] = n0 + c[ORC_C_DT10] * n1 - c[ORC_C_DTWP] * n0;
                        y[12 + cc][x] = n1 + c[ORC_C_DT21] * n2 - c[ORC_C_DT10] * n1 - dW;
                        y[15 + cc][x] = n2 + c[ORC_C_DT32] * n3 - c[ORC_C_DT21] * n2 + dW;
                        y[18 + cc][x] = n3 + c[ORC_C_DTWP] * n0 - c[ORC_C_DT32] * n3;
                    }
                }
}

/* Adjoint step: z = J(X0)^T w, plus the parameter terms of this step:
 * g_eps[cell] += dL/d eps_r and *g_na += dL/d(N_a / N_ref) through the noise
 * amplitude (both may be NULL).  step_n is the index of the step X0 -> X1. */
static void adjoint_step(const orc_sim* s, state_t X0, state_t X1, int64_t step_n,
                         double* const* w, double** z, double* g_eps, double* g_na) {
    const double* c = s->coef;
    const double S = c[ORC_C_S];
    const size_t nt = s->ntot;
    double* etot[3];
    double* u[3];
    double* htot[3];
    double* vh[3];
    for (int q = 0; q < 3; ++q) {
        etot[q] = (double*)calloc(nt, sizeof(double));
        u[q] = (double*)calloc(nt, sizeof(double));
        htot[q] = (double*)calloc(nt, sizeof(double));
        vh[q] = (double*)calloc(nt, sizeof(double));
    }
    for (int q = 0; q < ORC_NFIELDS; ++q) memcpy(z[q], w[q], sizeof(double) * nt);   /* identity rows */
    /* E' enters W: the total adjoint of E' and u = cb ie etot at interior sites */
    for (int k = 0; k <= s->nz; ++k)
        for (int j = 0; j <= s->ny; ++j)
            for (int i = 0; i <= s->nx; ++i)
                for (int cc = 0; cc < 3; ++cc) {
                    const size_t x = at(s, i, j, k);
                    etot[cc][x] = w[cc][x];
                    if (!e_interior(s, cc, i, j, k)) continue;
                    const size_t cell = cell_of(s, i, j, k);
                    if (s->gain[cell]) {
                        const double Wh = w[15 + cc][x] - w[12 + cc][x];
                        const double dPf = X1[6 + cc][x] - X0[6 + cc][x];
                        etot[cc][x] += Wh * c[ORC_C_BETA] * 0.5 * dPf;
                    }
                    const double a = site_loss(s, 0, cc, i, j, k);
                    u[cc][x] = layer_cb(s, a) * s->inv_eps[cell] * etot[cc][x];
                }
    /* H: the adjoint of H' collects S curl+ u (the transpose of curl- is curl+) */
    for (int k = 0; k <= s->nz; ++k)
        for (int j = 0; j <= s->ny; ++j)
            for (int i = 0; i <= s->nx; ++i)
                for (int cc = 0; cc < 3; ++cc) {
                    const size_t x = at(s, i, j, k);
                    if (!h_updated(s, i, j, k)) {   /* zeroed by the step */
                        htot[cc][x] = 0.0;
                        z[3 + cc][x] = 0.0;
                        continue;
                    }
                    htot[cc][x] = w[3 + cc][x] + S * curl_plus(s, u, cc, i, j, k);
                    const double a = site_loss(s, 1, cc, i, j, k);
                    z[3 + cc][x] = layer_ca(s, a) * htot[cc][x];
                    vh[cc][x] = layer_cb(s, a) * htot[cc][x];
                }
    /* E: identity or ca etot, minus S curl- (db htot) (the transpose of curl+),
     * and the Bloch terms at interior gain sites */
    double* Hn[3] = {X1[3], X1[4], X1[5]};
    for (int k = 0; k <= s->nz; ++k)
        for (int j = 0; j <= s->ny; ++j)
            for (int i = 0; i <= s->nx; ++i)
                for (int cc = 0; cc < 3; ++cc) {
                    const size_t x = at(s, i, j, k);
                    double e_adj = w[cc][x];
                    const int in = e_interior(s, cc, i, j, k);
                    if (in) {
                        const double a = site_loss(s, 0, cc, i, j, k);
                        e_adj = layer_ca(s, a) * etot[cc][x];
                    }
                    e_adj -= S * curl_minus(s, vh, cc, i, j, k);
                    if (in) {
                        const size_t cell = cell_of(s, i, j, k);
                        const double ie = s->inv_eps[cell];
                        const double a = site_loss(s, 0, cc, i, j, k);
                        const double cb = layer_cb(s, a);
                        double dPf = 0.0;
                        if (s->gain[cell]) {
                            dPf = X1[6 + cc][x] - X0[6 + cc][x];
                            const double E = X0[cc][x], En = X1[cc][x];
                            const double Wh = w[15 + cc][x] - w[12 + cc][x];
                            const double dPh = Wh * c[ORC_C_BETA] * 0.5 * (En + E) - cb * ie * etot[cc][x];
                            const double pn = w[6 + cc][x] + dPh;
                            const double dN = X0[12 + cc][x] - X0[15 + cc][x];
                            e_adj += c[ORC_C_CK] * dN * pn + Wh * c[ORC_C_BETA] * 0.5 * dPf;
                            z[6 + cc][x] = w[9 + cc][x] + c[ORC_C_A] * pn - dPh;
                            z[9 + cc][x] = c[ORC_C_B] * pn;
                            const double n0 = w[21 + cc][x], n1 = w[12 + cc][x], n2 = w[15 + cc][x], n3 = w[18 + cc][x];
                            z[21 + cc][x] = n0 * (1.0 - c[ORC_C_DTWP]) + n3 * c[ORC_C_DTWP];
                            z[12 + cc][x] = n1 * (1.0 - c[ORC_C_DT10]) + n0 * c[ORC_C_DT10] + c[ORC_C_CK] * E * pn;
                            z[15 + cc][x] = n2 * (1.0 - c[ORC_C_DT21]) + n1 * c[ORC_C_DT21] - c[ORC_C_CK] * E * pn;
                            z[18 + cc][x] = n3 * (1.0 - c[ORC_C_DT32]) + n2 * c[ORC_C_DT32];
                            if (g_na && s->p.noise && c[ORC_C_CF] != 0.0) {
                                double xi[3];
                                orc_normals3(s->p.seed, (uint32_t)cell, (uint32_t)step_n, s->p.realization, xi);
                                *g_na += c[ORC_C_CK] * s->p.E_sp * xi[cc] * pn;
                            }
                        }
                        if (g_eps) {
                            /* E' depends on eps through ie = 1/eps: d ie / d eps = -ie^2 */
                            const double rhs = S * curl_minus(s, Hn, cc, i, j, k) - dPf;
                            g_eps[cell] += etot[cc][x] * cb * rhs * (-ie * ie);
                        }
                    }
                    z[cc][x] = e_adj;
                }
    for (int q = 0; q < 3; ++q) { free(etot[q]); free(u[q]); free(htot[q]); free(vh[q]); }
}

int orc_tangent_step(orc_sim* s, double* const* v, double** y) {
    if (has_mur(s)) return -1;
    state_t X0, X1;
    for (int q = 0; q < ORC_NFIELDS; ++q) X0[q] = s->f[q];
    if (state_alloc(s, X1) || forward_copy(s, X1)) { state_free(X1); return -1; }
    tangent_step(s, X0, X1, v, y);
    state_free(X1);
    return 0;
}

int orc_adjoint_step(orc_sim* s, double* const* w, double** z) {
    if (has_mur(s)) return -1;
    state_t X0, X1;
    for (int q = 0; q < ORC_NFIELDS; ++q) X0[q] = s->f[q];
    if (state_alloc(s, X1) || forward_copy(s, X1)) { state_free(X1); return -1; }
    adjoint_step(s, X0, X1, s->step, w, z, NULL, NULL);
    state_free(X1);
    return 0;
}

int orc_adjoint_run(orc_sim* s, int64_t nsteps, double* grad_eps, double* grad_Na, double* loss) {
    if (has_mur(s) || !s->box_on || s->step != 0 || nsteps < 1) return -1;
    const size_t nt = s->ntot;
    const size_t ncell = (size_t)s->nx * s->ny * s->nz;
    state_t* X = (state_t*)calloc((size_t)nsteps + 1, sizeof(state_t));
    if (!X) return -1;
    int rc = 0;
    for (int64_t n = 0; n <= nsteps && !rc; ++n) rc = state_alloc(s, X[n]);
    /* forward, keeping every state */
    double L = 0.0;
    for (int64_t n = 0; n <= nsteps && !rc; ++n) {
        if (n > 0) {
            const double l0 = s->loss;
            orc_step(s, 1);
            L += s->loss - l0;
        }
        for (int q = 0; q < ORC_NFIELDS; ++q) memcpy(X[n][q], s->f[q], sizeof(double) * nt);
    }
    state_t lam, nxt;
    if (!rc) rc = state_alloc(s, lam);
    if (!rc) rc = state_alloc(s, nxt);
    double g_na = 0.0;
    if (!rc) {
        memset(grad_eps, 0, ncell * sizeof(double));
        for (int64_t n = nsteps; n >= 1; --n) {
            /* dL/dE^n = 2 E^n on the interior sites of the box */
            for (int k = s->box[2]; k < s->box[5]; ++k)
                for (int j = s->box[1]; j < s->box[4]; ++j)
                    for (int i = s->box[0]; i < s->box[3]; ++i)
                        for (int cc = 0; cc < 3; ++cc)
                            if (e_interior(s, cc, i, j, k)) {
                                const size_t x = at(s, i, j, k);
                                lam[cc][x] += 2.0 * X[n][cc][x];
                            }
            adjoint_step(s, X[n - 1], X[n], n - 1, lam, nxt, grad_eps, &g_na);
            for (int q = 0; q < ORC_NFIELDS; ++q) memcpy(lam[q], nxt[q], sizeof(double) * nt);
        }
        /* initial populations: N_i^0 = r_i (N_a / N_ref) on interior gain sites */
        double r[4] = {0.0, 0.0, 0.0, 0.0};   /* N0, N1, N2, N3 */
        if (s->init_kind == ORC_INIT_GROUND) {
            r[0] = 1.0;
        } else {
            double d32 = s->rates[0], d21 = s->rates[1], d10 = s->rates[2], dwp = s->rates[3];
            double r0 = 1.0 / (1.0 + dwp / d32 + dwp / d21 + dwp / d10);
            r[0] = r0; r[3] = dwp * r0 / d32; r[2] = dwp * r0 / d21; r[1] = dwp * r0 / d10;
        }
        for (int k = 0; k <= s->nz; ++k)
            for (int j = 0; j <= s->ny; ++j)
                for (int i = 0; i <= s->nx; ++i)
                    for (int cc = 0; cc < 3; ++cc) {
                        if (!e_interior(s, cc, i, j, k) || !s->gain[cell_of(s, i, j, k)]) continue;
                        const size_t x = at(s, i, j, k);
                        g_na += r[0] * lam[21 + cc][x] + r[1] * lam[12 + cc][x] + r[2] * lam[15 + cc][x] +
                                r[3] * lam[18 + cc][x];
                    }
        *grad_Na = g_na / s->p.N_ref;
        *loss = L;
    }
    state_free(lam);
    state_free(nxt);
    for (int64_t n = 0; n <= nsteps; ++n) state_free(X[n]);
    free(X);
    return rc;
}


/*
 * FP64 CPU oracle of the vectorial Maxwell-Bloch FDTD step.
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the plain, slow reference that
 * the GPU library is checked against.  Only the test-suite, the smoke check
 * and the CPU-baseline leg of the benchmark load it; the product path never
 * does.  It shares no source with the GPU library.
 *
 * What it computes (Simulations section of the paper: vectorial Maxwell-Bloch
 * equations, 21 coupled fields, FDTD on a Yee grid, four-level gain confined
 * to the voids between dielectric spheres, pump fixed by the atomic density
 * N_a, spontaneous emission as a stochastic source).  The paper defers the
 * equations to earlier work, so the standard four-level Lorentz-oscillator
 * model is used, in scaled units (x in dx, t in dt, E in E_ref,
 * H in E_ref/eta0, P in eps0*E_ref, N in N_ref).  Per step n:
 *
 *   a1  H^{n+1/2} = H^{n-1/2} - S curl+ E^n                     (Faraday)
 *   a2  P^{n+1}   = a P^n + b P^{n-1} + ck (N1-N2)^n E^n + cF xi^n
 *                                         (Lorentz oscillator, gain E-sites)
 *   a3  E^{n+1}   = E^n + (1/eps_r)(S curl- H^{n+1/2} - (P^{n+1}-P^n))
 *                                                                (Ampere)
 *   a6  boundary (PEC walls, first-order Mur, or a graded impedance-matched
 *       lossy layer backed by PEC) and soft source on E^{n+1}.  In the lossy
 *       layer a1 and a3 become H' = da H - db S curl E and
 *       E' = ca E + cb (1/eps)(S curl H - dP) with ca = da = (1-a)/(1+a),
 *       cb = db = 1/(1+a), a = a_max sum over axes of (depth/L)^p.
 *   a4  four-level rate equations with field work W = beta Ebar (P^{n+1}-P^n)
 *       N3 += dtWp N0 - dt32 N3;  N2 += dt32 N3 - dt21 N2 + W
 *       N1 += dt21 N2 - dt10 N1 - W;  N0 += dt10 N1 - dtWp N0
 *   a7  monitors: discrete energy, probe DFT (e^{+i w t} convention of the
 *       Gross-Pitaevskii section), loss-box integral of |E|^2.
 *
 * All arrays are FP64 over the extended Yee index range
 * (nx+1)*(ny+1)*(nz+1), x fastest.  Each E-site owns its own polarisation
 * and four populations (3 sites x (P, P_prev, N0..N3) + E + H = 24 values per
 * cell; the oracle keeps N0 explicitly).
 */
#ifndef MB_ORACLE_H
#define MB_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_PEC = 0, ORC_MUR1 = 1, ORC_ABSORB = 2 };
enum { ORC_INIT_GROUND = 0, ORC_INIT_PREPUMPED = 1 };

/* field ids: E 0-2, H 3-5, P^n 6-8, P^{n-1} 9-11, N1 12-14, N2 15-17,
 * N3 18-20, N0 21-23 (component x, y, z in each group) */
enum { ORC_NFIELDS = 24 };

typedef struct orc_params {
    int32_t nx, ny, nz;
    int32_t bc[3];          /* per axis: ORC_PEC, ORC_MUR1 or ORC_ABSORB */
    int32_t round_f32;      /* 1: every coefficient rounded to binary32 */
    int32_t frozen_pop;     /* 1: populations held fixed (a4 skipped) */
    double dx;              /* m */
    double courant;         /* c dt sqrt(3) / dx */
    double lambda0, dlambda;/* m */
    double tau32, tau21, tau10; /* s */
    double Wp;              /* 1/s */
    double N_ref, E_ref, E_sp;
    uint64_t seed;
    uint32_t realization;
    int32_t noise;          /* 1: spontaneous-emission source on */
    int32_t absorb_cells;   /* depth L of the graded lossy layer on ORC_ABSORB faces */
    int32_t absorb_order;   /* grading exponent p */
    double absorb_rate;     /* a_max: loss per step sigma dt/(2 eps) at the wall */
} orc_params;

/* coefficient vector layout returned by orc_coefficients */
enum {
    ORC_C_DT, ORC_C_S, ORC_C_A, ORC_C_B, ORC_C_CK, ORC_C_CF, ORC_C_BETA,
    ORC_C_DT32, ORC_C_DT21, ORC_C_DT10, ORC_C_DTWP, ORC_C_NA,
    ORC_C_WA, ORC_C_DWA, ORC_C_OMP2, ORC_C_COUNT
};

typedef struct orc_sim orc_sim;

orc_sim* orc_create(const orc_params* p);
void     orc_destroy(orc_sim* s);
void     orc_coefficients(const orc_sim* s, double* out /* ORC_C_COUNT */);
int      orc_set_material(orc_sim* s, const float* eps_r, const uint8_t* gain);
int      orc_set_pump(orc_sim* s, double Na, int init);
int      orc_set_source(orc_sim* s, int comp, int i, int j, int k, double amp,
                        double lambda_s, double tau_p, double t0);
double   orc_source_value(const orc_sim* s, int64_t n);
/* continuous wave amp (1 - exp(-(t/t_ramp)^2)) sin(w_s t), replacing any source */
int      orc_set_cw_source(orc_sim* s, int comp, int i, int j, int k, double amp,
                           double lambda_s, double t_ramp);
/* energy density of the cells of plane z = k summed over steps (k = -1: off);
 * the read returns the number of steps summed (-1 without a monitor) */
int      orc_set_plane_monitor(orc_sim* s, int k);
int64_t  orc_read_plane_monitor(const orc_sim* s, double* out /* nx*ny */);
int      orc_set_probes(orc_sim* s, const int32_t* sites, int n_probes,
                        const double* omega, int n_freq);
int      orc_set_loss_box(orc_sim* s, int i0, int j0, int k0, int i1, int j1, int k1);
int      orc_step(orc_sim* s, int64_t nsteps);
int64_t  orc_step_index(const orc_sim* s);
int      orc_get_field(const orc_sim* s, int id, double* out);
int      orc_set_field(orc_sim* s, int id, const double* in);
void     orc_read_energy(const orc_sim* s, double* W_now, double* W_int);
int64_t  orc_energy_history(const orc_sim* s, double* out, int64_t cap);
void     orc_read_spectrum(const orc_sim* s, double* re_im);
double   orc_read_loss(const orc_sim* s);

/* Adjoint of the loss-box objective L = sum_{n=1..N} sum_{box} (E^n)^2 over a
 * run of nsteps that starts at orc_set_pump (step 0), with PEC or lossy-layer
 * walls (no Mur).  Advances the sim by nsteps and returns L, dL/d eps_r per
 * cell (grad_eps[nx*ny*nz]) and dL/dN_a (per m^-3).  The whole trajectory is
 * kept in memory (small grids only).  -1 when not applicable. */
int      orc_adjoint_run(orc_sim* s, int64_t nsteps, double* grad_eps, double* grad_Na,
                         double* loss);
/* One step's linearisation at the current state (not advanced), on the 24
 * field arrays in field-id order: tangent y = J v and adjoint z = J^T w. */
int      orc_tangent_step(orc_sim* s, double* const* v, double** y);
int      orc_adjoint_step(orc_sim* s, double* const* w, double** z);

/* building blocks, exported so the tests can pin them in isolation; the grid
 * stepper calls exactly these */
void     orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
void     orc_normals3(uint64_t seed, uint32_t cell, uint32_t step, uint32_t realization,
                      double xi[3]);
double   orc_p_next(const double* coef, double P, double Pprev, double E, double dN, double xi);
void     orc_pop_next(const double* coef, double N[4], double Ebar, double dP);
void     orc_p_series(const double* coef, const double* E, const double* dN, int64_t n,
                      double* P_out);
void     orc_pop_series(const double* coef, double N[4], const double* Ebar, const double* dP,
                        int64_t n, double* N_out /* 4*n */);

#ifdef __cplusplus
}
#endif
#endif

/*
 * mbf -- Maxwell-Bloch FDTD on one MI355X (gfx950).
 *
 * C ABI of the GPU library.  One handle = one simulation: a Yee grid of
 * nx*ny*nz cells carrying the 21 fields of the vectorial Maxwell-Bloch model
 * of the paper's Simulations section (E, H, the polarisation P with its
 * previous value, and populations N1, N2, N3 of a four-level gain medium at
 * every E-site of a gain cell; N0 = N_a - N1 - N2 - N3 is derived), dielectric
 * spheres with gain only in the voids, and spontaneous-emission noise from a
 * counter-based Philox4x32-10 stream keyed by (seed, realization, cell, step).
 *
 * One step n (scaled units: x in dx, t in dt, E in E_ref, H in E_ref/eta0,
 * P in eps0 E_ref, N in N_ref):
 *   a1  H^{n+1/2} = H^{n-1/2} - S curl+ E^n
 *   a2  P^{n+1} = a P^n + b P^{n-1} + ck (N1-N2) E^n + cF xi^n   (gain sites)
 *   a3  E^{n+1} = E^n + (1/eps_r)(S curl- H^{n+1/2} - (P^{n+1} - P^n))
 *   a6  PEC or first-order Mur walls, then the soft source, on E^{n+1}
 *   a4  four-level rates with the field work beta (E^{n+1}+E^n)/2 (P^{n+1}-P^n)
 *   a7  FP64 monitors: energy, running DFT at probe sites, loss-box sum
 *
 * Conventions
 *  - Every call returns an int status: MBF_OK (0) or a negative MBF_E* code.
 *    mbf_last_error(h) returns a message owned by the handle, valid until the
 *    next call on it; mbf_global_error() covers failures before a handle
 *    exists.  No C++ exception crosses this interface.
 *  - The handle owns all device memory it allocates and frees it in
 *    mbf_destroy.  The caller owns every buffer it passes; sizes are implied
 *    by the grid and checked where a size is passed.
 *  - Pointers tagged MBF_MEM_DEVICE are device addresses (for instance a torch
 *    tensor's data_ptr()); MBF_MEM_HOST pointers are ordinary host memory.
 *    The caller keeps device buffers alive until the work queued on the
 *    handle's stream has finished.
 *  - `stream` is a hipStream_t passed as void*.  NULL makes the handle create
 *    and own a stream of default priority.  All work is queued on that stream;
 *    reads into host memory synchronise it.
 *  - Site arrays (mbf_read_field / mbf_write_field) span the extended Yee
 *    index range (nx+1)*(ny+1)*(nz+1), x fastest, in the handle's precision
 *    (float for MBF_FP32, double for MBF_FP64).  E-site (c; i,j,k) of
 *    component c lies at the cell edge (i,j,k) + e_c/2, H-site at the face
 *    (i,j,k) + (1 - e_c)/2.  Cell arrays (material) span nx*ny*nz.
 *  - Handles are not thread-safe; distinct handles are independent.
 */
#ifndef MBF_H
#define MBF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define MBF_OK 0
#define MBF_EINVAL (-1)      /* bad argument or configuration */
#define MBF_ECFL (-2)        /* Courant number outside (0, 1] */
#define MBF_ENOMEM (-3)      /* device or host allocation failed */
#define MBF_EHIP (-4)        /* a HIP runtime call failed */
#define MBF_ENONFINITE (-5)  /* the energy monitor saw a NaN or infinity */
#define MBF_ESTATE (-6)      /* call not valid in the handle's current state */
#define MBF_ENODEV (-7)      /* no usable gfx950 device */

/* boundary per axis */
#define MBF_PEC 0
#define MBF_MUR1 1    /* first-order Mur on the wall E-sites */
#define MBF_ABSORB 2  /* graded impedance-matched lossy layer of absorb_cells
                         cells, backed by a conducting wall: in the layer H and
                         E lose a fraction 2a/(1+a) per step (a = absorb_rate
                         ((depth)/absorb_cells)^absorb_order summed over axes),
                         the same for E and H so that every medium stays matched */

/* initial populations for mbf_set_pump */
#define MBF_INIT_GROUND 0     /* N0 = N_a, N1 = N2 = N3 = 0 */
#define MBF_INIT_PREPUMPED 1  /* E = 0 fixed point of the discrete rates */

/* precision of the fields */
#define MBF_FP32 0
#define MBF_FP64 1

#define MBF_MEM_HOST 0
#define MBF_MEM_DEVICE 1

/* flags */
#define MBF_FLAG_FROZEN_POP 1  /* populations held fixed (row a4 skipped) */

/* field ids for mbf_read_field / mbf_write_field */
#define MBF_EX 0
#define MBF_EY 1
#define MBF_EZ 2
#define MBF_HX 3
#define MBF_HY 4
#define MBF_HZ 5
#define MBF_PX 6        /* P^n */
#define MBF_PPREVX 9    /* P^{n-1} */
#define MBF_N1X 12
#define MBF_N2X 15
#define MBF_N3X 18
#define MBF_NFIELDS 21

/* coefficient vector returned by mbf_coefficients (values as used on the
 * device, promoted to double) */
enum {
    MBF_C_DT, MBF_C_S, MBF_C_A, MBF_C_B, MBF_C_CK, MBF_C_CF, MBF_C_BETA,
    MBF_C_DT32, MBF_C_DT21, MBF_C_DT10, MBF_C_DTWP, MBF_C_NA, MBF_C_COUNT
};

typedef struct mbf_config {
    int32_t nx, ny, nz;        /* cells per axis, each >= 2 */
    int32_t boundary[3];       /* MBF_PEC or MBF_MUR1 per axis */
    int32_t precision;         /* MBF_FP32 or MBF_FP64 */
    int32_t noise;             /* 1: spontaneous-emission source on */
    int32_t flags;             /* MBF_FLAG_* */
    int32_t reserved0;
    double dx;                 /* cell size [m] */
    double courant;            /* c dt sqrt(3)/dx, in (0, 1] */
    double lambda0, dlambda;   /* gain centre wavelength and bandwidth [m] */
    double tau32, tau21, tau10;/* level lifetimes [s]; tau21 also fixes the coupling */
    double Wp;                 /* pump rate 0 -> 3 [1/s] */
    double N_ref, E_ref;       /* scaling density [m^-3] and field [V/m] */
    double E_sp;               /* noise amplitude in units of E_ref */
    uint64_t seed;             /* Philox key */
    uint32_t realization;      /* third Philox counter word */
    int32_t reserved1;
    int64_t energy_history;    /* steps of per-step energy kept on device (0: none) */
    int32_t absorb_cells;      /* depth of the MBF_ABSORB layer in cells (>= 1) */
    int32_t absorb_order;      /* grading exponent of the layer (>= 0) */
    double absorb_rate;        /* loss a at the wall, per step (>= 0) */
} mbf_config;

typedef struct mbf_handle mbf_handle;
typedef struct mbf_batch mbf_batch;

/* Library version string; never fails. */
const char* mbf_version(void);

/* Message of the last failure that happened without a handle (create). */
const char* mbf_global_error(void);

/* Message of the last failure on h (empty string when none). */
const char* mbf_last_error(const mbf_handle* h);

/* Fill *cfg with the workload defaults (dx 20 nm, Courant 0.99, lambda0
 * 590 nm, bandwidth 230 nm, tau32 = tau10 = 100 fs, tau21 = 1 ns,
 * Wp = 1e12 /s, N_ref 1e24 m^-3, E_ref 1e8 V/m, E_sp 1e-6, PEC, FP32, noise
 * on, seed 0, lossy layer 8 cells deep, quadratic, a = 0.25 at the wall).
 * Returns MBF_EINVAL for NULL or sizes < 2. */
int mbf_config_default(mbf_config* cfg, int nx, int ny, int nz);

/* Validate cfg (sizes >= 2, ny and nz < 65535, every site array below 4 GiB,
 * Courant number, finite positive parameters) before any allocation, then
 * allocate E and H on the current device and zero them (the Bloch state is
 * allocated by mbf_set_material, one value per gain cell).  *out receives the
 * handle.  Errors: MBF_EINVAL, MBF_ECFL, MBF_ENODEV, MBF_ENOMEM, MBF_EHIP. */
int mbf_create(const mbf_config* cfg, void* stream, mbf_handle** out);

/* Free everything the handle owns.  NULL is ignored. */
void mbf_destroy(mbf_handle* h);

/* Coefficients as stored on the device (MBF_C_COUNT doubles into out[n]). */
int mbf_coefficients(const mbf_handle* h, double* out, int n);

/* Material map (Simulations section: spheres of index 2.9 in a background,
 * gain only in the voids).  eps_r[nx*ny*nz] relative permittivity (> 0) and
 * gain[nx*ny*nz] (0 or 1) per cell, x fastest; an E-site takes the values of
 * the cell whose edge it lies on.  At most 128 distinct eps_r values among
 * the gain cells and 128 among the others.
 * Copies; the caller's buffers are not retained.  (Re)allocates the Bloch
 * state (15 arrays of one value per gain cell), zeroes it and requires a new
 * mbf_set_pump before stepping. */
int mbf_set_material(mbf_handle* h, const float* eps_r, const uint8_t* gain, int mem_kind);

/* Pump density N_a [m^-3] (Simulations section: the pump is set through the
 * atomic density and is constant over the run).  Zeroes E, H, P and the
 * monitors, sets the populations of every gain E-site per `init`, and resets
 * the step counter to 0. */
int mbf_set_pump(mbf_handle* h, double Na, int init);

/* Soft point source on E-site (comp; i,j,k), which must be interior:
 * amp * sin(w_s (t - t0)) * exp(-((t - t0)/tau_p)^2) with w_s = 2 pi c /
 * lambda_s, added to E^{n+1} at t = (n+1) dt (passive broadband run of the
 * Simulations section: single-cycle ~1 fs pulse at 532 nm).  One source per
 * handle; amp = 0 removes it. */
int mbf_add_point_source(mbf_handle* h, int comp, int i, int j, int k, double amp,
                         double lambda_s, double tau_p, double t0);

/* Continuous-wave soft source on E-site (comp; i,j,k), which must be
 * interior: amp * (1 - exp(-(t/t_ramp)^2)) * sin(w_s t) with w_s = 2 pi c /
 * lambda_s, added to E^{n+1} at t = (n+1) dt (Simulations section: the field
 * distribution of a mode is found by CW excitation at its spectral peak; the
 * Gaussian switch-on over t_ramp keeps the drive narrow-band).  It replaces
 * any source of the handle (one source per handle); amp != 0, lambda_s > 0,
 * t_ramp > 0 (MBF_EINVAL otherwise). */
int mbf_add_cw_source(mbf_handle* h, int comp, int i, int j, int k, double amp, double lambda_s,
                      double t_ramp);

/* Running DFT monitor: F[p][w] += E_c(site_p)^{m} exp(+i omega_w m dt) for
 * every sample m (the Fourier sign of the Gross-Pitaevskii section).
 * sites[4*n_probes] rows (comp, i, j, k); omega[n_freq] in rad/s; samples are
 * buffered `decim` steps on the device (1..1024) and folded into FP64
 * accumulators.  Replaces any previous probe set and zeroes the spectrum. */
int mbf_set_probes(mbf_handle* h, const int32_t* sites, int n_probes, const double* omega,
                   int n_freq, int decim);

/* Loss-box monitor: L += sum of |E|^2 over the interior E-sites of cells in
 * [i0,i1) x [j0,j1) x [k0,k1), every step, in FP64. */
int mbf_set_loss_box(mbf_handle* h, int i0, int j0, int k0, int i1, int j1, int k1);

/* Queue nsteps steps on the handle's stream (asynchronous).  Requires
 * mbf_set_material and mbf_set_pump first (MBF_ESTATE otherwise). */
int mbf_step(mbf_handle* h, int64_t nsteps);

/* Block until the handle's stream is idle. */
int mbf_sync(mbf_handle* h);

/* Steps taken since the last mbf_set_pump. */
int mbf_step_index(const mbf_handle* h, int64_t* out);

/* W_now = energy W^n of the last step, W_int = sum of W over all steps
 * (scaled units; multiply by eps0 E_ref^2 dx^3 for joules).  Synchronises.
 * MBF_ENONFINITE once any step produced a NaN or infinite energy. */
int mbf_read_energy(mbf_handle* h, double* W_now, double* W_int);

/* Per-step energy history (capacity set by cfg.energy_history); *count
 * receives the number of stored steps, min(count, cap) are copied. */
int mbf_read_energy_history(mbf_handle* h, double* out, int64_t cap, int64_t* count);

/* Spectrum re_im[2 * n_probes * n_freq] (probe-major, interleaved re, im). */
int mbf_read_spectrum(mbf_handle* h, double* re_im);

/* Loss-box integral. */
int mbf_read_loss(mbf_handle* h, double* out);

/* Energy density in a section of the sample (Simulations section: the
 * energy density in the middle section under CW excitation, Fig. 1 inset,
 * and in the lasing run, Fig. 2a).  mbf_set_plane_monitor(h, k) with
 * 0 <= k < nz sums, every step n, u(i,j) = 1/2 [eps_r |E^n|^2 +
 * |H^{n+1/2}|^2] over the cell's own E- and H-sites (i, j, k) into an FP64
 * array of nx*ny values (x fastest), starting from zero now; k = -1 removes
 * the monitor.  mbf_reset_plane_monitor zeroes the sums;
 * mbf_read_plane_monitor synchronises and copies them to the host buffer
 * out[nx*ny] (caller-owned) with *count the number of steps summed (divide
 * for the time average).  mbf_set_pump zeroes the sums too; checkpoints and
 * device snapshots carry them (an image saved with a monitor loads only into
 * a handle monitoring the same plane).  MBF_ESTATE without a monitor. */
int mbf_set_plane_monitor(mbf_handle* h, int k);
int mbf_reset_plane_monitor(mbf_handle* h);
int mbf_read_plane_monitor(mbf_handle* h, double* out, int64_t* count);

/* ------------------------------------------------------ spectral statistics
 * Peak and width of an emission spectrum (Results section: the linewidth of
 * the Maxwell-Bloch spectra comes from a Gaussian fit, Fig. 5b; the width of
 * the measured spectra is their standard deviation, Fig. 4).  From complex
 * probe amplitudes F[p][k] (the running DFT of mbf_set_probes):
 *   S_k = sum_p |F[p][k]|^2 (probes added in index order, FP64);
 *   peak_bin = the first k holding the largest S_k (-1 when S is all zero);
 *   mean_omega, std_omega = first moment and standard deviation of omega
 *   under the weight S;
 *   fit_lo..fit_hi = the run of bins around the peak with S_k >= level *
 *   S_peak; over it a weighted least-squares parabola
 *   ln(S_k / S_peak) = a + b x + c x^2, weights (S_k / S_peak)^2,
 *   x = (omega_k - omega_peak) / s with s the mean bin spacing in the run,
 *   gives the Gaussian fit_amplitude * exp(-(omega - fit_center)^2 /
 *   (2 fit_sigma^2)); fit_ok = 1 when the run has at least 3 bins and c < 0
 *   (fit_* are 0 otherwise).  Frequencies in rad/s. */
typedef struct {
    double total;          /* sum_k S_k */
    double peak_omega;     /* omega[peak_bin] */
    double peak_value;     /* S at the peak */
    double mean_omega;
    double std_omega;
    double fit_center;
    double fit_sigma;
    double fit_amplitude;
    int32_t peak_bin;
    int32_t fit_lo, fit_hi;
    int32_t fit_ok;
} mbf_spec_stats;

/* Statistics of the handle's probe spectra (pending DFT work is flushed
 * first); runs on the handle's stream and synchronises.  0 < level < 1
 * (MBF_EINVAL otherwise); MBF_ESTATE without probes. */
int mbf_spectrum_stats(mbf_handle* h, double level, mbf_spec_stats* out);

/* The same statistics of caller data: spec[2 * n_probes * n_freq] (probe-
 * major, interleaved re, im) and omega[n_freq], both host or both device
 * memory per mem_kind (caller-owned, unchanged; a device spec must be 16-byte
 * aligned).  Runs on `stream` (NULL: the null stream) in device memory it
 * allocates and frees; returns when *out holds the result.  n_probes >= 1,
 * n_freq >= 1, 0 < level < 1 (MBF_EINVAL otherwise). */
int mbf_spectral_stats(const double* spec, int n_probes, int n_freq, const double* omega, double level,
                       int mem_kind, void* stream, mbf_spec_stats* out);

/* mbf_spectral_stats for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same kernels and results, but nothing is allocated or
 * freed.  spec[2 * n_probes * n_freq], omega[n_freq] and *out are device
 * memory (caller-owned; spec 16-byte, omega and out 8-byte aligned).  The
 * work is queued on `stream` (NULL: the null stream) and the call returns
 * without waiting; *out holds the result once the stream reaches it.  The
 * intermediate power spectrum lives in a fixed per-device scratch array of
 * 65536 FP64 values held by the library until the process ends:
 * 1 <= n_freq <= 65536 (MBF_EINVAL otherwise), n_probes >= 1, 0 < level < 1.
 * Every call on a device shares that array (each call overwrites the bins it
 * uses before reading them): calls ordered on one stream are safe, calls that
 * overlap on one device (other streams, other threads) race. */
int mbf_spectral_stats_noalloc(const double* spec, int n_probes, int n_freq, const double* omega, double level,
                               void* stream, mbf_spec_stats* out);

/* Spectral peaks (Simulations section: the spectrum after a wide-band pulse
 * shows several peaks, the long-lived modes, Fig. 1).  Of the same S_k: the
 * bins with S_k > 0, S_k >= min_rel * max_k S_k and S_{k-1} < S_k >= S_{k+1}
 * (a band-edge bin compares with its one neighbour; a flat top counts once,
 * at its first bin), by decreasing S_k (equal values: lower k first), at most
 * max_peaks of them into the host buffer bins[max_peaks] (caller-owned),
 * *n_found how many.  0 <= min_rel <= 1, 1 <= max_peaks <= 1024 (MBF_EINVAL
 * otherwise).  mbf_spectrum_peaks works on a handle's spectra (MBF_ESTATE
 * without probes), mbf_spectral_peaks on caller amplitudes as
 * mbf_spectral_stats. */
int mbf_spectrum_peaks(mbf_handle* h, double min_rel, int max_peaks, int32_t* bins, int* n_found);
int mbf_spectral_peaks(const double* spec, int n_probes, int n_freq, double min_rel, int max_peaks, int mem_kind,
                       void* stream, int32_t* bins, int* n_found);

/* Copy one site array out of / into the device state (see field ids), in the
 * packed layout of (nx+1)*(ny+1)*(nz+1) values, x fastest; dst/src are host
 * or device memory per mem_kind, owned by the caller.  Reading P gives P^n,
 * MBF_PPREVX+c gives P^{n-1}.  P and N exist on gain cells only: they read as
 * zero elsewhere and values written elsewhere are dropped.  Before
 * mbf_set_material the Bloch fields give MBF_ESTATE. */
int mbf_read_field(mbf_handle* h, int field_id, void* dst, int mem_kind);
int mbf_write_field(mbf_handle* h, int field_id, const void* src, int mem_kind);

/* Kernel schedule.  All variants give bitwise identical fields; they differ
 * in how the step is cut into kernels.  Workgroups cover 64 x tile_y columns
 * over zseg planes (zseg = 0: 2 for MBF_VARIANT_TWO_PASS_SPLIT, 4 for the
 * others).  xcd_remap chooses which XCD runs which
 * workgroup (the hardware deals launch-order workgroups to the 8 XCDs in
 * turn): 0 launch order; 1 each XCD a contiguous range of (x tile, y tile,
 * z segment) work items; 2 (default) whole z-segment layers dealt to the XCDs
 * in turn, so neighbouring tiles share an L2 and the XCDs stream one window of
 * planes together.  tile_y must be 2, 4, 8 or 16.
 *   MBF_VARIANT_TWO_PASS: a1 in one kernel, a2-a5 in a second.
 *   MBF_VARIANT_TWO_PASS_SPLIT: the same two passes; the second prefetches
 *     only the dense fields of the next plane and loads the Bloch state at the
 *     start of each plane, and the first writes H with streaming (non-
 *     temporal) stores: fewer registers, more waves, faster on grids that
 *     fill the device and exceed its caches (a batch of 320^3 realizations),
 *     slower on small ones.
 *   MBF_VARIANT_FUSED: rows a1-a5 in one z-marching kernel in which every
 *     wave owns a row and forms again the few H^{n+1/2} values of the
 *     neighbouring row, column and plane that it needs (waves exchange no
 *     field values).
 *   MBF_VARIANT_FUSED_LDS: rows a1-a5 in one z-marching kernel whose waves
 *     advance plane by plane together (one barrier per plane) and hand the
 *     H^{n+1/2} of their rows to the neighbouring row's E update through
 *     LDS; only the tile's edges are formed again.  zseg = 0 means 8.
 *   MBF_VARIANT_FUSED_PERSISTENT: the kernel of MBF_VARIANT_FUSED as one
 *     persistent launch per step for all members: a grid sized to what the
 *     device holds at once takes the work items from eight device-side
 *     queues in work-table order (queue x serves the entries the dispatch
 *     order meant for XCD x; workgroup b serves queue b mod 8) until they are
 *     drained, and the last workgroup to finish resets the queues for the
 *     next launch, so it replays in graphs like the others.
 * group_mb (batches only; >= 0): consecutive members whose device state adds
 * up to at most group_mb MiB form a group, and a graph-replayed chunk of
 * steps runs group by group, so that a group's state can stay in the
 * device's last-level cache over the chunk; 0 puts all members in one group.
 * Results do not depend on it.
 * Default schedule (also the autotuner's first candidate): tile_y 4, zseg 0,
 * xcd_remap 2, group_mb 0, MBF_VARIANT_TWO_PASS_SPLIT for a grid of at least
 * 4 Mi cells (for a batch: its largest member), MBF_VARIANT_TWO_PASS below;
 * a single grid below 4 Mi cells takes the longest zseg of 4, 2 and 1 that
 * still cuts it into at least 1024 work items (1 if none does). */
#define MBF_VARIANT_TWO_PASS 0
#define MBF_VARIANT_FUSED 1
#define MBF_VARIANT_TWO_PASS_SPLIT 2
#define MBF_VARIANT_FUSED_LDS 3
#define MBF_VARIANT_FUSED_PERSISTENT 4
typedef struct mbf_tuning {
    int32_t variant;
    int32_t tile_y;
    int32_t zseg;
    int32_t xcd_remap;
    int32_t group_mb;
} mbf_tuning;
int mbf_set_tuning(mbf_handle* h, const mbf_tuning* t);
int mbf_get_tuning(const mbf_handle* h, mbf_tuning* t);

/* Time candidate schedules (every variant, tile_y 2/4/8, zseg 2/4/8; the
 * default first) on the handle's own grid for about budget_ms (at least one
 * candidate), keep the fastest and report it in *chosen (may be NULL).  The
 * simulation state is saved to device memory before the trials and restored
 * after them, so the run continues exactly as if autotune had not been
 * called; this needs one extra copy of the state in device memory
 * (MBF_ENOMEM otherwise).  Needs material and pump (MBF_ESTATE).
 * Persistence: when the environment variable MBF_TUNE_CACHE names a file,
 * the choice is appended to it, keyed by the device architecture, the
 * precision and the grid and walls, and a later call with the same key (in
 * this or another process) applies the stored schedule without timing
 * anything.  mbf_batch_autotune does the same, keyed by every member. */
int mbf_autotune(mbf_handle* h, int budget_ms, mbf_tuning* chosen);

/* Queue nsteps steps without graph capture, bracketing the field kernels of
 * every step with HIP events on the handle's stream.  On return
 * (synchronised) kernel_ms[0] holds the summed duration of the first field
 * kernel (the fused step kernel, or the Faraday pass of the two-pass variant)
 * and kernel_ms[1] that of the second (the Ampere/Bloch pass; 0 for the
 * fused variant); *launches is the number of steps.  Used to time the kernels
 * against their roofline. */
int mbf_step_timed(mbf_handle* h, int64_t nsteps, double* kernel_ms /* [2] */, int64_t* launches);

/* Algorithmic HBM bytes: what must move if every value is read and written
 * exactly once.  bytes[0], the step: per cell E and H read and written
 * (4 x 3 values) and 1 material byte; per interior gain E-site P^n and
 * P^{n-1} read, P^{n+1} written, N1..N3 read and written (9 values).  A value
 * is 4 B in FP32 and 8 B in FP64, so a cell whose three E-sites carry gain
 * costs 157 B in FP32.  bytes[1] and bytes[2]: the same count for the first
 * and second field kernel of the current variant (the two-pass variant reads
 * H^{n+1/2} and the material byte in both passes).  From the current
 * material map. */
int mbf_step_bytes(const mbf_handle* h, double* bytes /* [3] */);

/* Checkpoint: bytes needed, save into / load from a caller buffer.  The
 * image holds all 21 fields, the step index and the monitors, with a
 * checksum; noise needs no state (it is keyed by the step index), so a
 * resumed run is bitwise identical to an uninterrupted one. */
int mbf_state_size(const mbf_handle* h, size_t* out);
int mbf_save_state(mbf_handle* h, void* buf, size_t n);
int mbf_load_state(mbf_handle* h, const void* buf, size_t n);

/* ---------------------------------------------------------------- adjoint
 * Gradient of the loss-box objective (the loss-box monitor summed over the
 * run) L = sum_{n=1..nsteps} sum_{interior E-sites in the box} (E^n)^2 with
 * respect to eps_r of every cell and to the pump density N_a, by reverse-mode
 * differentiation of the discrete step (rows a2-a4 transposed, curl- and
 * curl+ exchanged).  The run starts right after mbf_set_pump (step 0;
 * MBF_ESTATE otherwise) with the loss box set (MBF_ESTATE), PEC or absorbing
 * walls (Mur walls: MBF_EINVAL).  The forward run keeps a device snapshot of
 * the state every K steps; the reverse sweep recomputes each segment of K
 * steps from its snapshot, storing E, P, N1 and N2 of every step, and then
 * runs the K reverse steps, so device memory grows with nsteps/K + K.
 * grad_eps receives nx*ny*nz doubles, x fastest (host or device memory per
 * mem_kind, caller-owned), *grad_Na dL/dN_a in m^3, *loss L.  The handle is
 * left at step nsteps, as after mbf_step(nsteps).  The gradient is the same,
 * bit for bit, for every K. */
int mbf_adjoint_run(mbf_handle* h, int64_t nsteps, int K, void* grad_eps, int mem_kind, double* grad_Na,
                    double* loss);

/* -------------------------------------------- Gross-Pitaevskii / ST law
 * The theory of the Gross-Pitaevskii section: the oscillation condition of
 * the random laser in dimensionless form (Eq. g5),
 *     -phi'' + tau^2 phi + phi^3 = E phi,
 * whose positive bound state exists for E > 1, with E = (p - 1)/(kappa
 * sqrt(p)) (Eq. ee, p the pump relative to the high-Q loss) and the
 * threshold E = 1 at p_th = 1 + kappa^2/2 + kappa sqrt(4 + kappa^2)/2.
 * mbf_gp_solve solves it for n_E eigenvalues at once (one workgroup each) on
 * M interior points tau_i = -L + (i+1) h, h = 2L/(M+1), phi(+-L) = 0,
 * second differences: a semi-implicit gradient flow from the near-threshold
 * Gaussian (E < 3) or the Thomas-Fermi profile, then Newton steps to an update
 * below 1e-13 of max phi.  For each E it returns phi (M values), the spectrum
 * S_k = phit(nu_k)^2 with phit(nu) = (h/2pi) sum_i phi_i cos(nu tau_i), nu_k =
 * k dnu (n_nu values), and 7 statistics: N = h sum phi^2, the spectral waist
 * w = sigma_nu/(2 pi) (sigma_nu^2 the second moment of the even spectrum; a
 * Gaussian exp(-nu^2/(8 pi^2 w^2)) has waist w; w -> 1/(2 sqrt(2) pi) at
 * threshold), the peak S(0), max phi, the largest residual of the discrete
 * equation, the Newton steps taken and a converged flag (1/0).  In real units
 * (Eq. s1 and below) W = w sqrt(kappa) / (p^{1/4} t_g), S_peak = t_g^2 S(0) /
 * gamma_S.  E[n_E], phi[n_E*M], spec[n_E*n_nu], stats[n_E*7]: all host or
 * all device memory per mem_kind, caller-owned; runs on `stream` and returns
 * when the results are in place.  1 <= n_E <= 65535, 3 <= M <= 1023, L > 0,
 * n_nu >= 1, dnu > 0, every E > 1 (MBF_EINVAL otherwise). */
int mbf_gp_solve(const double* E, int n_E, int M, double L, int n_nu, double dnu, int mem_kind, void* stream,
                 double* phi, double* spec, double* stats);
/* E(p) of Eq. ee and the threshold pump p_th (E = 1). */
double mbf_gp_eigenvalue(double p, double kappa);
double mbf_gp_threshold(double kappa);

/* ST-law linewidth fit (Gross-Pitaevskii section, Eqs. ee, s1, wth and the
 * numerical waist of Eq. g5, compared with the Maxwell-Bloch linewidths in
 * Fig. 5b): kappa such that, with p = p_th(kappa) Na[i] / N_th,
 * E = (p - 1)/(kappa sqrt(p)) and the model waist (in frequency omega/2pi)
 * W_model = w(E) sqrt(kappa) / (p^{1/4} t_g), the squared log misfit
 * sum_i (ln W_model_i - ln W[i])^2 is least; w(E) is the waist of the bound
 * state (mbf_gp_solve on M points of [-L, L], n_nu spectrum points of
 * spacing dnu).  Golden-section search over ln kappa in [ln 1e-3, ln 10] to a
 * bracket of 1e-10; a kappa for which some eigenvalue exceeds (0.7 L)^2 (the
 * bound state would not fit the window) or a bound state does not converge
 * counts as no fit.  Na[n] (m^-3, each > N_th) and W[n] (Hz, > 0) are host
 * arrays; *kappa and, when not NULL, W_fit[n] (the model waists at kappa) are
 * host outputs.  Runs on `stream`, returns when done.  MBF_EINVAL for bad
 * sizes, MBF_ENONFINITE when no kappa in the range gives every bound state. */
int mbf_kappa_fit(const double* Na, const double* W, int n, double N_th, double t_g, int M, double L, int n_nu,
                  double dnu, void* stream, double* kappa, double* W_fit);

/* Lasing threshold of a pump sweep (Results section, Fig. 5b: the threshold
 * E = 1 of the theory, located on the simulations themselves).  Each run
 * starts from the pumped state without noise, excited by a small field with
 * no static part (a soft pulse has none; a random field does, and its
 * undamped energy hides the decay below threshold); its energy history W^n
 * (mbf_read_energy_history) grows or decays with the least-damped mode.  rate = least-squares slope of ln W^n over
 * n0 <= n < n1 (per step); the threshold is the root N_th = -a/b of the
 * least-squares line rate = a + b N_a through the runs.  hist[n_runs *
 * stride] (run r at r * stride; host or device per mem_kind, caller-owned),
 * Na[n_runs] host (m^-3); rates[n_runs] and fit[3] = (a, b, N_th) are host
 * outputs.  n_runs >= 2 with distinct N_a, 0 <= n0, n1 - n0 >= 2,
 * stride >= n1 (MBF_EINVAL otherwise); a non-positive W in the window gives
 * MBF_ENONFINITE.  Runs on `stream` and returns when done. */
int mbf_growth_threshold(const double* hist, int n_runs, int64_t stride, int64_t n0, int64_t n1, const double* Na,
                         int mem_kind, void* stream, double* rates, double* fit);

/* Knee of a pump sweep (Results section, Fig. 5b: the linewidth collapses
 * where the sample starts to lase; the theory's threshold E = 1), for y =
 * a width (or its log) against x = N_a: two least-squares lines, one through
 * points [0, s) and one through [s, n) (at least two each), with the split s
 * that leaves the least summed squared residual (the first on ties); the
 * knee is where the two lines cross, kept between x[s-1] and x[s] (their
 * midpoint if the lines do not cross there at a finite point).  x[n], y[n]
 * host or device per mem_kind (caller-owned); out[7] host output: knee, s,
 * aL, bL, aR, bR, residual sum (y = a + b x on each side).  4 <= n <= 1024
 * and x strictly increasing (MBF_EINVAL), finite values (MBF_ENONFINITE).
 * Runs on `stream` and returns when done. */
int mbf_knee_fit(const double* x, const double* y, int n, int mem_kind, void* stream, double* out);

/* ------------------------------------------------------------- packing
 * The sample is a granular packing of dielectric spheres obtained by
 * molecular dynamics (Simulations section; the method is not given there).
 * mbf_pack_md computes such a packing as a compression run of soft spheres in
 * the closed box [0, box[0]] x [0, box[1]] x [0, box[2]] (cell units), in the
 * dissipative (overdamped) limit of granular dynamics.  At scale s the
 * spheres have diameters s d_i and the energy is
 *     U_s = 1/2 sum_{i<j} (s (d_i + d_j)/2 - |x_i - x_j|)_+^2
 *         + 1/2 sum_i sum_a [(s d_i/2 - x_ia)_+^2 + (x_ia + s d_i/2 - L_a)_+^2];
 * a step moves every centre at once, x_i += eta F_i with F_i = -grad_i U_s
 * (coincident centres exert no force on each other).  The scale runs through
 * s_m = s0 + (1 - s0) m / stages, m = 0..stages: `iters` steps at each
 * s_m < 1, then `final_iters` steps at s = 1 (stages = 0: final_iters steps
 * at s = 1).  Steps are stable while eta < 1 / (the most contacts of one
 * sphere); s0 = 0.5, stages = 100, iters = 20, final_iters = 1000, eta = 0.15
 * bring a 0.4 fill of 10%-polydisperse spheres to overlaps below 1e-4 of a
 * diameter.
 *
 * diam[n] (unchanged) and centres[3 n] ((x, y, z) per sphere, replaced by the
 * packed centres) are both host or both device memory per mem_kind, caller-
 * owned; box[3] and the outputs are host memory.  *energy receives U_1 and
 * *max_overlap the largest overlap of a pair or of a sphere with a wall at
 * s = 1 (0 when nothing overlaps).  Runs on `stream` (NULL: the null stream)
 * in device memory it allocates and frees, and returns when the results are
 * in place; the same input gives the same bits on every run.  Errors:
 * MBF_EINVAL for 0 > n > 2^26, box edges or diameters not finite and > 0,
 * centres not finite, s0 outside (0, 1], negative counts, eta not finite and
 * > 0, or a box of more than 2^24 cells of the largest diameter; MBF_ESTATE
 * when more than 32 centres fall into one such cell; MBF_ENONFINITE when the
 * run diverges.  After MBF_ESTATE or MBF_ENONFINITE the centres hold the
 * run's last state.  n = 0 returns at once with zeros. */
#define MBF_PACK_MAX_SPHERES (1 << 26)
typedef struct {
    double s0;            /* starting scale of the diameters, 0 < s0 <= 1 */
    int32_t stages;       /* growth stages from s0 to 1 */
    int32_t iters;        /* steps at each scale below 1 */
    int32_t final_iters;  /* steps at s = 1 */
    int32_t pad;
    double eta;           /* step length */
} mbf_pack_params;
int mbf_pack_md(int n, const double* box, const double* diam, double* centres, const mbf_pack_params* prm,
                int mem_kind, void* stream, double* energy, double* max_overlap);

/* ---------------------------------------------------------------- batches
 * Many realizations advanced together (Simulations section: the emission is
 * studied over several sphere packings and pump levels N_a).  A batch owns R
 * member handles, 1 <= R <= 255, created from cfgs[0..R-1] (any sizes and
 * walls, one precision) on one stream (`stream`, or a new one when NULL).
 * mbf_batch_member returns a member's handle, owned by the batch and valid
 * until mbf_batch_destroy: material, pump, sources, probes, reads and
 * checkpoints go through it, and the member can still be stepped alone.
 * mbf_batch_step advances every member by nsteps with one launch of each
 * step kernel per step for all members (a work table maps workgroups to
 * (member, tile)); chunks of steps are replayed as a hipGraph.  A member's
 * fields, energies and spectra after mbf_batch_step are bitwise those of the
 * same member stepped alone with the same tuning.  Every member needs its
 * material and pump set (MBF_ESTATE otherwise).  mbf_batch_set_tuning sets
 * the schedule of the batch and of every member; batched steps always use the
 * batch's schedule, even for a member whose own schedule was changed later
 * (that one only applies when the member is stepped alone).  Timing and algorithmic
 * bytes as for a handle, summed over the members.  Errors of batch calls are
 * read with mbf_batch_last_error. */
int mbf_batch_create(const mbf_config* cfgs, int R, void* stream, mbf_batch** out);
void mbf_batch_destroy(mbf_batch* b);
const char* mbf_batch_last_error(const mbf_batch* b);
int mbf_batch_size(const mbf_batch* b);
int mbf_batch_member(mbf_batch* b, int r, mbf_handle** out);
int mbf_batch_set_tuning(mbf_batch* b, const mbf_tuning* t);
int mbf_batch_get_tuning(const mbf_batch* b, mbf_tuning* t);
int mbf_batch_step(mbf_batch* b, int64_t nsteps);
int mbf_batch_sync(mbf_batch* b);
int mbf_batch_step_timed(mbf_batch* b, int64_t nsteps, double* kernel_ms /* [2] */, int64_t* launches);
int mbf_batch_step_bytes(const mbf_batch* b, double* bytes /* [3] */);
/* mbf_autotune for a whole batch, timed on graph-replayed batched chunks:
 * group_mb (0, 1, 96, 192) at the default schedule, then the schedules at the
 * best grouping, then the other groupings (32, 64, 128) for the best
 * schedule; the result applies to the batch and every member. */
int mbf_batch_autotune(mbf_batch* b, int budget_ms, mbf_tuning* chosen);
/* mbf_spectrum_stats of every member: out[R], member order (the linewidth
 * and peak against the members' pump levels). */
int mbf_batch_spectrum_stats(mbf_batch* b, double level, mbf_spec_stats* out);

/* mbf_growth_threshold over the members' own energy histories (device) and
 * pump levels: every member needs an energy history of at least n1 steps and
 * to have taken n1 steps (MBF_ESTATE otherwise). */
int mbf_batch_growth_threshold(mbf_batch* b, int64_t n0, int64_t n1, double* rates, double* fit);

#ifdef __cplusplus
}
#endif
#endif

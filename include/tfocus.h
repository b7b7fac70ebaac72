/*
 * tfocus.h -- C ABI of libtfocus, an MI355X (gfx950) implementation of the
 * tight-focusing method of Panova et al., "Optimized computation of tight
 * focusing of short pulses using mapping to periodic space"
 * (arXiv:2010.00409).
 *
 * The calls follow the paper's problem statement: put a pulse on the
 * focusing sphere and map it into a periodic layer (Sec. II.B-II.C), advance
 * it with the dispersion-free spectral step (Sec. II.A), and read the focal
 * field back through the cut-out (Sec. II.C, Eqs. (14)-(16)).
 *
 * Conventions shared by every call
 * --------------------------------
 * Units: c = 1.  Lengths are in any unit; the natural one is the central
 *   wavelength.  Time is length / c.  Fields are in the CGS form of the paper
 *   (E and B share units).
 * Field layout: one contiguous array [6][nz][ny][nx] of the solver's element
 *   type (float for TF_F32, double for TF_F64), components Ex, Ey, Ez, Bx, By,
 *   Bz, x fastest.  Node (i, j, k) sits at (x_min + i dx, y_min + j dy,
 *   z_min + k dz); the grid is periodic on all three axes.
 * Memory: pointers flagged "on_device" are HIP device pointers on the
 *   solver's device (for example a torch tensor's data_ptr()); others are
 *   host pointers.  Caller buffers are borrowed only for the call and, for
 *   device pointers, until the work queued on the solver's stream completes.
 *   Objects own all memory they allocate.
 * Streams: all device work is queued on the stream given at creation (NULL
 *   means the null stream).  Only calls that return data into host memory
 *   synchronise that stream.
 * Errors: every call returns a tf_status; no exception crosses the ABI.
 *   Arguments are validated before any HIP call.  tf_last_error() returns a
 *   message for the last failure on the calling thread.
 * Threading: one object per thread; distinct objects are independent.
 */
#ifndef TFOCUS_H
#define TFOCUS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    TF_OK = 0,
    TF_EINVAL = -1,        /* null pointer, bad size or bad parameter        */
    TF_EUNSUPPORTED = -2,  /* axis length with a prime factor other than 2,3 */
    TF_ENOMEM = -3,        /* device allocation failed or exceeds the cap    */
    TF_EDEVICE = -4,       /* a HIP call failed (message has the HIP error)  */
    TF_ESTATE = -5,        /* call not valid in the object's current state   */
    TF_EDOMAIN = -6,       /* period D = nx dx not larger than the pulse L   */
    TF_ENONFINITE = -7     /* non-finite value found by a checked call       */
} tf_status;

typedef enum { TF_F32 = 0, TF_F64 = 1 } tf_precision;

/* Longitudinal profile u_l of the pulse. */
typedef enum {
    TF_ENV_COS2 = 0,      /* sin(2 pi z/lambda - cep) cos^2(pi z/L), Eq. (7)      */
    TF_ENV_GAUSS = 1,     /* sin(2 pi z/lambda - cep) exp(-z^2 ln4/(n lambda)^2),
                             Sec. III.B.1, cut to |z| <= L/2                     */
    TF_ENV_SPECTRAL = 2   /* Re sum_m a_m exp(i(phi_m - w_m z)), Gaussian spectrum
                             of relative width `bandwidth`, spectral phase
                             cep + pi/2 + gdd (w-w0)^2/2 + tod (w-w0)^3/6 over
                             nfreq samples, max |g| = 1, cut to |z| <= L/2      */
} tf_envelope;

/* Transverse profile u_ts(alpha), alpha = angle from the -x axis. */
typedef enum {
    TF_TS_FLATTOP = 0,    /* Eq. (5): 1 below theta - eps/2, cos^2 edge, 0 above */
    TF_TS_GAUSS = 1       /* exp(-alpha^2/theta^2) for alpha <= pi/2, Sec. III.B.1 */
} tf_transverse;

typedef enum {
    TF_POL_LINEAR = 0,    /* d = (0, cos pol_angle, sin pol_angle); with
                             ellipticity e a second part along (0,-sin,cos) in
                             quadrature, amplitudes 1/sqrt(1+e^2), e/sqrt(1+e^2) */
    TF_POL_RADIAL = 1     /* d = x (along the optical axis)                      */
} tf_polarization;

/* Periodic grid; the layer period along x is D = nx * dx. */
typedef struct {
    int32_t nx, ny, nz;   /* nx even; each length one tf_supported_length
                             accepts                                            */
    int32_t replicate_yz; /* 0: the grid holds the pulse transversely.  1: y and
                             z are periods of the mapping too (transverse
                             duplication, Sec. II.C closing remarks): every
                             node also sums the replicas y + m ny dy,
                             z + l nz dz, and focal windows wrap in y and z   */
    double dx, dy, dz;    /* > 0                                                 */
    double x_min, y_min, z_min;
} tf_grid;

/* Pulse on the focusing sphere, Sec. II.B (flat-top) and Sec. III.B.1
 * (Gaussian beam).  E = u s0, B = u s1 with u(R) = (A/R) u_l(R - R0)
 * u_ts(alpha), s1 = d x R / |d x R|, s0 = R x (d x R) / |R x (d x R)|. */
typedef struct {
    int32_t envelope;      /* tf_envelope                                        */
    int32_t transverse;    /* tf_transverse                                      */
    int32_t polarization;  /* tf_polarization                                    */
    int32_t nfreq;         /* spectral samples (TF_ENV_SPECTRAL), 1..4096         */
    double wavelength;     /* central wavelength lambda > 0                      */
    double R0;             /* radius of the pulse centre                         */
    double L;              /* full support length; R_min,max = R0 -/+ L/2        */
    double ncycles;        /* TF_ENV_GAUSS: intensity FWHM in wavelengths        */
    double f_number;       /* theta = arctan(1/(2 f)) when theta <= 0            */
    double theta;          /* opening half-angle (> 0 overrides f_number)        */
    double eps;            /* flat-top edge width                                 */
    double P0;             /* cycle-averaged power through the cap, Eq. (9)       */
    double pol_angle, ellipticity;
    double cep, gdd, tod;  /* carrier-envelope phase, chirp (time units^2, ^3)   */
    double bandwidth;      /* TF_ENV_SPECTRAL: relative 1/e half-width delta      */
    int32_t nbumps;        /* wavefront phase perturbation (Sec. III.B.3): number
                              of Gaussian bumps, 0..1024                           */
    int32_t reserved;
    const double* bumps;   /* host, nbumps x {ay, az, amplitude, width}: the
                              direction of a point, alpha (y, z) / rho, gets the
                              phase sum_i amplitude_i exp(-|(ay, az) - (ay_i,
                              az_i)|^2 / width_i^2) added to its carrier phase
                              (as cep is); copied by tf_set_pulse /
                              tf_batch_create, not kept                            */
} tf_pulse;

/* Geometry derived from a pulse by tf_pulse_geometry / tf_set_pulse. */
typedef struct {
    double theta;          /* opening angle, Sec. II.B                            */
    double A;              /* amplitude, Eq. (9) (flat-top) or sqrt(4P0/F(theta)) */
    double R_min, R_max;   /* R0 -/+ L/2                                           */
    double L;
    double D_min;          /* Eq. (12) at theta                                    */
    double alpha_max;      /* angular support edge                                 */
    double D;              /* nx dx of the solver (tf_set_pulse only)              */
    int32_t overlap;       /* D < D_min: replicas overlap (allowed, Sec. II.C)     */
    int32_t reserved;
} tf_pulse_info;

/* Node-aligned focal window of wx*wy*wz nodes centred on the node nearest
 * (cx, cy, cz); node i along x is centre + i - wx/2.  x wraps (mapping T,
 * Eq. (13)); y and z must stay inside the grid unless it replicates the pulse
 * transversely (replicate_yz), where they wrap as x does. */
typedef struct {
    int32_t wx, wy, wz, reserved;
    double cx, cy, cz;
} tf_window;

typedef struct tf_solver tf_solver;

/* Version string "tfocus <major>.<minor>". */
const char* tf_version(void);

/* Message of the calling thread's last failure ("" if none). */
const char* tf_last_error(void);

/* 1 if n is a supported axis length: 2^a (8 .. 1024), 3 2^a (24 .. 768),
 * 5 2^a (40 .. 640) or 7 2^a (56 .. 896).  Lengths with a factor 5 or 7
 * (the paper's 112 and 896 node axes, Sec. III.A) take radix-5 and radix-7
 * stages and run the generic y and z kernels. */
int32_t tf_supported_length(int32_t n);

/* Host only.  Opening angle (Sec. II.B), amplitude (Eq. (9); Gaussian
 * transverse: sqrt(4 P0 / F(theta)), F of Sec. III.B.1), radii and D_min
 * (Eq. (12)).  info->D and info->overlap are set to 0. */
tf_status tf_pulse_geometry(const tf_pulse* pulse, tf_pulse_info* info);

/* Host only.  The periodic layer of Sec. II.C for a pulse: D = nx dx,
 * x_min = -R_min - D moved onto the node grid so the origin is a node,
 * y_min = -(ny/2) dy, z_min = -(nz/2) dz.  Writes *out. */
tf_status tf_layer_grid(const tf_pulse* pulse, int32_t nx, int32_t ny, int32_t nz,
                        double dx, double dy, double dz, tf_grid* out);

/* Create a solver on the current HIP device.  Allocates the field state
 * (6 nx ny nz elements) and the half spectrum (6 nz ny nkx complex, nkx =
 * nx/2: the x DC and Nyquist planes share slot 0 as F(0) + i F(nx/2)), so
 * about 12 nx ny nz elements in all.  The state starts at zero with t = 0.
 * hip_stream: hipStream_t or NULL (a stream of that device).  Every later
 * call on the solver must be made with the same device current.  TF_ENOMEM
 * if the environment variable TFOCUS_MAX_DEVICE_BYTES is set below the
 * bytes needed. */
tf_status tf_create(const tf_grid* grid, int32_t precision, void* hip_stream,
                    tf_solver** out);

/* Free everything the solver owns (waits for its stream). NULL is a no-op. */
tf_status tf_destroy(tf_solver* s);

/* Copy a state [6][nz][ny][nx] in, set the time to t.  The state is taken as
 * is (no projection).  Host sources are copied synchronously. */
tf_status tf_set_fields(tf_solver* s, const void* src, int32_t src_on_device, double t);

/* Copy the state out.  A host destination synchronises the stream. */
tf_status tf_get_fields(tf_solver* s, void* dst, int32_t dst_on_device);

/* Borrowed device pointer to the state array (valid until tf_destroy). */
tf_status tf_state_ptr(tf_solver* s, void** dev_ptr);

/* Initialise E and B from the pulse, Eqs. (5)-(11), mapped into the layer:
 * every node sums the pulse over its preimages x + n D (Eq. (13) and the
 * superposition remark after Eq. (12)), and with replicate_yz also over
 * y + m ny dy, z + l nz dz.  Sets t = 0 and the cut-out radii,
 * and makes the next tf_advance remove the longitudinal part of B once
 * (E loses its longitudinal part at every step, Eq. (3)).
 * TF_EDOMAIN if D = nx dx <= L.  info (nullable) receives the geometry. */
tf_status tf_set_pulse(tf_solver* s, const tf_pulse* pulse, tf_pulse_info* info);

/* Cut-out radii R_min, R_max for tf_read_focal when the state was loaded
 * with tf_set_fields. */
tf_status tf_set_cutout(tf_solver* s, double R_min, double R_max);

/* Advance nsteps steps of dt (any sign and size; one step of any length is
 * exact, Sec. II.A).  Each step: forward 3-D real FFT of the six components,
 * per-mode rotation of Eqs. (3)-(4) with C = cos(c|k|dt), S = sin(c|k|dt),
 * inverse FFT.  k-space conventions: forward transform exp(-i k.x); k_hat =
 * 0 at k = 0; Nyquist indices contribute 0 to k.  t += nsteps * dt.
 * Asynchronous on the solver's stream.  Runs of eight steps are replayed
 * from a graph captured on a private stream at the first such call with
 * this dt (and again when dt changes), owned by the solver; the first step
 * after tf_set_pulse, the remainder and all steps while tf_profile is on
 * are launched directly.  Both give the same bits. */
tf_status tf_advance(tf_solver* s, int64_t nsteps, double dt);

/* One step of dt with a current density j held over the step (Sec. II.A,
 * Eqs. (1)-(2), CGS units, c = 1):
 *   E' = C E + i S k_hat x B - (4 pi S / |k|) j + (1 - C) k_hat (k_hat . E)
 *        + 4 pi k_hat (k_hat . j) (S / |k| - dt)
 *   B' = C B - i S k_hat x E + 4 pi i ((1 - C) / |k|) k_hat x j
 * per mode, between the forward and inverse 3-D FFTs, with the conventions
 * of tf_advance.  At |k| = 0 the factors S / |k| and (1 - C) / |k| take
 * their limits dt and 0, so a uniform current gives E' = E - 4 pi dt j.
 * The longitudinal part of E is kept (it changes by -4 pi dt k_hat . j);
 * after tf_set_pulse the longitudinal part of B is removed first, as in
 * tf_advance.  j: 3 nx ny nz elements of the solver's precision, layout
 * [component][z][y][x] (jx, jy, jz), x fastest, on the host (j_on_device =
 * 0; the call then waits for the copy) or on the solver's device (1),
 * borrowed for the call.  The first call allocates a six-component current
 * array and a second half spectrum (12 nx ny nz elements), kept until
 * tf_destroy.  t += dt.  Asynchronous on the solver's stream for device j.
 * TF_EUNSUPPORTED where nine z columns do not fit the LDS (float64 with
 * nz = 1024); TF_ENOMEM above TFOCUS_MAX_DEVICE_BYTES. */
tf_status tf_advance_current(tf_solver* s, const void* j, int32_t j_on_device, double dt);

/* Focal window [6][wz][wy][wx] at the current time: u(R) = u~(T(R)) I_S(t)(R),
 * Eqs. (14)-(16), with the third case of Eq. (15) read as "x >= 0 and
 * R > r(t)".  dst holds 6 wx wy wz elements of the solver's type.
 * TF_ESTATE if no cut-out radii are known; TF_EINVAL if the window leaves
 * the grid transversely. */
tf_status tf_read_focal(tf_solver* s, const tf_window* win, void* dst, int32_t dst_on_device);

/* Synchronous diagnostics of the current state: energy = sum over nodes of
 * E^2 + B^2; max_div_e = max |k_hat . E_hat| / max |E_hat| over modes and
 * likewise for B.  Any pointer may be NULL.  TF_ENONFINITE if the energy is
 * not finite. */
tf_status tf_diagnostics(tf_solver* s, double* energy, double* max_div_e, double* max_div_b);

/* tf_advance followed by tf_diagnostics without the diagnostics' own
 * passes: nsteps >= 1 steps of dt, the last of which runs the generic z
 * kernel with the diagnostics folded into it (Sec. II.A: the energy the
 * rotation of Eqs. (3)-(4) conserves, and the transversality the text after
 * Eq. (2) asks for).  The values describe the state after the call, taken
 * from its spectrum inside that z pass: energy by Parseval (the R2C half
 * spectrum with weight 2 off the packed kx = 0 slot), the same ratios as
 * tf_diagnostics (equal to it up to rounding).  Synchronous.  Any output
 * pointer may be NULL.  TF_EINVAL for nsteps < 1; TF_ENONFINITE if the
 * energy is not finite. */
tf_status tf_advance_diagnosed(tf_solver* s, int64_t nsteps, double dt, double* energy, double* max_div_e,
                               double* max_div_b);

/* Current time t (host bookkeeping, no synchronisation). */
tf_status tf_time(const tf_solver* s, double* t);

/* Grid the solver was created with. */
tf_status tf_get_grid(const tf_solver* s, tf_grid* grid);


/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the steps of
 * tf_advance applied in place to a caller-owned state, with no allocation and
 * no solver object.  state_dev: [6][nz][ny][nx] of the precision's element
 * type, device memory on the current device; advanced by nsteps steps of dt
 * (Eqs. (3)-(4) between forward and inverse 3-D FFTs, the conventions of
 * tf_advance); project_b_first = 1 also removes the longitudinal part of B in
 * the first step, as the first tf_advance after tf_set_pulse does.  Kernel
 * plans as tf_create.  The spectrum and twiddle tables live in a static
 * 128 MiB device array that every call on a device shares (each device holds
 * its own until the process ends): a grid needing more gives TF_ENOMEM before
 * any HIP call (about 5.5 M cells in float32, 2.7 M in float64: 128^3 fits
 * in both).  Nothing in it must start at zero (each call rebuilds the tables
 * and each step rewrites the spectrum), but calls on one device whose work
 * overlaps in time race on it.  Only kernel launches are queued on hip_stream
 * (NULL: the null stream), so the call may be captured into a graph; the
 * first call on a device looks the array up (hipGetSymbolAddress) and should
 * be made outside capture (nsteps = 0 does only that). */
tf_status tf_advance_noalloc(const tf_grid* grid, int32_t precision, void* state_dev, int64_t nsteps, double dt,
                             int32_t project_b_first, void* hip_stream);

/* Pass kinds reported by tf_profile_read. */
typedef enum {
    TF_PASS_X_FORWARD = 0, TF_PASS_Y_FORWARD = 1, TF_PASS_Z_STEP = 2, TF_PASS_Y_INVERSE = 3,
    TF_PASS_X_INVERSE = 4, TF_PASS_INIT = 5, TF_PASS_READOUT = 6, TF_PASS_OTHER = 7,
    TF_NPASS = 8
} tf_pass;

/* Start (enable = 1) or stop (0) timing every kernel launch of the solver
 * with a pair of HIP events on its stream.  Enabling clears earlier records. */
tf_status tf_profile(tf_solver* s, int32_t enable);

/* Synchronise and report, per tf_pass kind, the summed kernel time in ms and
 * the number of launches recorded since profiling was enabled.  Either
 * array (TF_NPASS entries) may be NULL. */
tf_status tf_profile_read(tf_solver* s, double* ms_total, int64_t* launches);

/* ---- batched sweeps (uneven grids) ------------------------------------- */

typedef struct tf_batch tf_batch;

/* n independent instances (grid + pulse), precision for all.  Instances with
 * identical grids share one allocation and run together: every pass of a
 * step is one launch over all active instances of that grid.  Validates
 * every grid and pulse (TF_EDOMAIN if an instance's D <= L) and uploads the
 * pulse tables; the states are initialised by tf_batch_run.  Lives on the
 * current HIP device; later calls need the same device current. */
tf_status tf_batch_create(const tf_grid* grids, const tf_pulse* pulses, int32_t n, int32_t precision,
                          void* hip_stream, tf_batch** out);

/* One sweep: initialise every instance from its pulse (as tf_set_pulse),
 * advance instance i by nsteps[i] steps of dt[i] (the first step removes
 * longitudinal B once, as after tf_set_pulse), and cut out the window
 * (shared shape and centre, Eqs. (14)-(16) at t_i = nsteps[i] dt[i]) into
 * dst_dev + i * 6 * wx * wy * wz (device memory, n windows, solver element
 * type).  use_graph = 1 captures the whole sweep into a hipGraph on first
 * use and replays it while nsteps, dt, the window and dst_dev are unchanged
 * and no other run came between; 0 launches eagerly (and drops a captured
 * graph, whose slot order it may change).  Asynchronous on the batch
 * stream. */
tf_status tf_batch_run(tf_batch* b, const int64_t* nsteps, const double* dt, const tf_window* win,
                       void* dst_dev, int32_t use_graph);

/* Final state [6][nz][ny][nx] of instance i after the last run. */
tf_status tf_batch_get_fields(tf_batch* b, int32_t i, void* dst, int32_t dst_on_device);

tf_status tf_batch_destroy(tf_batch* b);

/* ---- kernel plans and the autotuner ------------------------------------ */

/* Plan file consulted by tf_create and tf_batch_create (also taken from the
 * environment variable TFOCUS_PLAN_FILE).  NULL or "" clears it. */
tf_status tf_set_plan_file(const char* path);

/* Host only.  The kernel plan tf_create and tf_batch_create use for a grid:
 * the y row blocking of the spectrum, whether the fast float32 kernels may
 * run (0 selects the generic kernels; also 0 when the fast z kernel's 32-bit
 * strip offsets would not reach a row of the spectrum), the fast z kernel's
 * strip shape, and the columns per strip of the fast y kernel (64, i.e.
 * 512-byte strips, or 32).  From the plan file, then the environment
 * overrides TFOCUS_ROW_BLOCK, TFOCUS_GENERIC_KERNELS, TFOCUS_ZVARIANT and
 * TFOCUS_YSTRIP.  Any output pointer may be NULL. */
tf_status tf_kernel_plan(const tf_grid* grid, int32_t precision, int32_t* row_block, int32_t* fast,
                         int32_t* zvariant, int32_t* ystrip);

/* For each cube size N in sizes[0..n): time a few steps of every kernel
 * plan (y row blocking 8 or none; generic kernels or the fast float32
 * kernels with each z strip shape of that length and both y strip widths)
 * on the current device with HIP events, on pseudo-random fields, in three
 * interleaved rounds (each plan keeps its fastest round); keep the fastest
 * plan and merge "arch precision N N N row_block fast zvariant ystrip ms"
 * into plan_path.  best_ms (nullable) receives
 * the best ms per step.  Allocates two N^3 six-component states on the
 * current device for the duration of the call. */
tf_status tf_tune(const int32_t* sizes, int32_t n, int32_t precision, const char* plan_path, double* best_ms);

/* ---- learned surrogate (Fourier neural operator) ----------------------- */

/* The paper motivates the method as a fast generator of many focusing runs,
 * for instance as training data for learned models (Sec. I, Sec. III.B.3).
 * This surrogate is trained on the solver's focal windows and maps eight
 * pulse and optics parameters, each normalised to [0, 1], to the
 * six-component field on a 64^3 focal window.  The plain solver stays its
 * fallback and the reference for its error.
 *
 * Architecture (fixed): lift [p, x, y, z] -> 32 channels (x, y, z the node
 * coordinates scaled to [-1, 1)); three Fourier layers
 *   z_l = irfft3(R_l . rfft3(v_l) on the kept modes) + v_l W_l + b_l,
 *   v_{l+1} = GELU(z_l) except after the last layer;
 * kept modes kx in [0, 12), ky, kz in [0, 12) U [52, 64), mode
 * q = (kz_i * 24 + ky_i) * 12 + kx (i: position in the kept list); R_l[q] a
 * complex 32 x 32 matrix; projection o = GELU(v P1 + c1) P2 + c2 to 6 K
 * channels (K basis fields of 6 components) and the output
 * out = sum_k w[k] o[6k .. 6k + 5] with per-sample head weights w.
 * K = 1 (w = 1) is the plain head.  K = 2 and K = 4 use the solver's
 * linearity: the initial field, hence the focal field, is
 * Re[exp(i s CEP) F] / gnorm with a complex F (s = +1 for the spectral
 * envelope, -1 for the sin(k z - CEP) envelopes of Eq. (7) and Sec. III.B.1;
 * gnorm the spectral normalisation), so K = 2 learns Re F and Im F and takes
 * the carrier-envelope phase exactly; K = 4 learns F for polarisation along y
 * and along z and weights them by the polarisation angle and ellipticity
 * (exact on the optical axis, where the direction factor of Sec. II.B is
 * linear in d; the network corrects the rest).  tf_fno_phasor_weights gives w.
 * Loss: mean over the batch of ||out - y|| / ||y||.
 *
 * Parameters are one float32 vector of tf_fno_param_count(K) entries:
 * W0 (11 x 32), b0 (32), then for each layer W (32 x 32), b (32),
 * R (6912 x 32 x 32 complex stored [q][c][o][re, im]), then P1 (32 x 128),
 * c1 (128), P2 (128 x 6K), c2 (6K); matrices row-major, input index first.
 * Every contraction runs on bf16 MFMA with float32 accumulation; learned
 * weights are used as bf16 copies of the float32 master weights.
 *
 * Device layouts: params [B][8]; head_w [B][K] (NULL allowed when K = 1);
 * out and target [B][6][64][64][64] (components Ex Ey Ez Bx By Bz, x
 * fastest); node tensors v, u [B][64 z][64 y][64 x][32 c]; modes
 * [B][24 kz][2 re/im][24 ky][12 kx][32 c]. */

typedef struct tf_fno tf_fno;

/* Parameter count for a head of nbasis (1, 2 or 4) basis fields; -1 otherwise. */
int64_t tf_fno_param_count(int32_t nbasis);

/* Host only.  Head weights w[0..nbasis) of a pulse: nbasis 1: {1}; 2:
 * {Re z, -Im z} / gnorm; 4: {Re za, -Im za, Re zb, -Im zb} / gnorm with
 * z = exp(i s CEP), a = (cos psi - i s e sin psi) / n, b = (sin psi + i s e cos psi) / n,
 * n = sqrt(1 + e^2), psi the polarisation angle and e the ellipticity
 * (radial polarisation: a = 1, b = 0). */
tf_status tf_fno_phasor_weights(const tf_pulse* pulse, int32_t nbasis, double* w);

/* Allocate a surrogate for batches up to max_batch (1..128) with a head of
 * nbasis basis fields on the current device.  training = 0 allocates only
 * what inference needs (about 80 MB per sample); training = 1 also keeps
 * activations, gradients and Adam state (about 0.45 GB per sample plus
 * 0.8 GB).  Parameters start at 0. */
tf_status tf_fno_create(int32_t max_batch, int32_t training, int32_t nbasis, void* hip_stream, tf_fno** out);

/* Period P of the surrogate's spectral transform, 64 (the plain transform
 * over the 64^3 window, the default) to 256.  With P > 64 the window is
 * extended by zeros to P nodes per axis, the kept modes are those of the
 * period-P transform ([0, 12) along x, [0, 12) U [P - 12, P) along y and
 * z) and the inverse is cut back to the window: the usual padding of
 * Fourier neural operators, for windows whose fields do not match across
 * opposite faces.  Only the truncated-DFT tables change (rebuilt in float64
 * and uploaded, synchronously); weights, shapes and kernels stay.  Changing
 * the period changes what existing weights compute.  TF_EINVAL outside
 * [64, 256]. */
tf_status tf_fno_set_period(tf_fno* f, int32_t period);
tf_status tf_fno_get_period(const tf_fno* f, int32_t* period);
tf_status tf_fno_destroy(tf_fno* f);

/* Copy the flat parameter vector in or out.  Setting resets Adam. */
tf_status tf_fno_set_params(tf_fno* f, const float* src, int32_t src_on_device);
tf_status tf_fno_get_params(tf_fno* f, float* dst, int32_t dst_on_device);

/* Inference: out <- surrogate(params) for batch samples (device pointers).
 * Asynchronous on the surrogate's stream. */
tf_status tf_fno_forward(tf_fno* f, const float* params, const float* head_w, int32_t batch, float* out);

/* Inference as one graph replay: the whole forward pass is captured into a
 * hipGraph on first use and replayed while params, head_w, out and batch are
 * the same pointers and size (new values in them, and new parameters, are
 * picked up; bf16 working copies are refreshed before the replay).  Results
 * equal tf_fno_forward bit for bit.  Asynchronous on the surrogate's stream. */
tf_status tf_fno_infer(tf_fno* f, const float* params, const float* head_w, int32_t batch, float* out);

/* Loss and gradient of the batch (device params, head weights and target).
 * loss (host, nullable) receives the loss; grad (host, nullable) receives the
 * gradient in the flat parameter layout.  Either pointer synchronises.
 * TF_ESTATE for an inference-only surrogate. */
tf_status tf_fno_loss_grad(tf_fno* f, const float* params, const float* head_w, const float* target, int32_t batch,
                           double* loss, float* grad);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected) with
 * learning rate lr on the batch loss.  loss (host, nullable) as above. */
tf_status tf_fno_train_step(tf_fno* f, const float* params, const float* head_w, const float* target,
                            int32_t batch, double lr, double* loss);

/* Configuration of a whole training run (tf_fno_train). */
typedef struct {
    int32_t epochs;          /* passes over the n samples, >= 1                      */
    int32_t batch;           /* minibatch size, 1..max_batch, <= n                   */
    double lr;               /* peak learning rate                                    */
    double lr_min_frac;      /* cosine decay from lr to lr * lr_min_frac, in [0, 1]   */
    uint64_t seed;           /* seed of the per-epoch shuffles (splitmix64)           */
    int32_t scale_targets;   /* 1: train on targets / RMS(all targets), then fold the
                                RMS into P2 and c2 so the operator predicts the
                                targets (the Adam state is reset afterwards)          */
    int32_t reserved;
    double* epoch_loss;      /* host, nullable: epochs entries, the mean batch loss
                                of each epoch                                          */
    void (*progress)(int32_t epoch, double loss, void* user);
                             /* nullable: called on the calling thread after each
                                epoch with its mean loss (for logs of long runs)      */
    void* progress_user;     /* passed to progress                                   */
} tf_train_cfg;

/* A whole training run on the device: per epoch a Fisher-Yates shuffle of the
 * n samples (host, splitmix64 from seed), then n / batch steps, each a
 * minibatch gather (device), tf_fno_train_step's loss, gradient and Adam
 * update with the step's cosine learning rate, and the loss logged on the
 * device; the log is read back once per epoch.  params_dev [n][8], head_w_dev
 * [n][K] (NULL when K = 1) and targets_dev [n][6][64][64][64] are device
 * memory and are not modified.  final_loss (nullable) receives the last
 * epoch's mean loss.  Synchronous.  TF_ESTATE for an inference-only
 * surrogate; TF_ENONFINITE if the loss or the target RMS is not finite. */
tf_status tf_fno_train(tf_fno* f, const float* params_dev, const float* head_w_dev, const float* targets_dev,
                       int64_t n, const tf_train_cfg* cfg, double* final_loss);

/* Held-out error: rel_l2 (host, n entries) receives ||out_i - y_i|| / ||y_i||
 * for the surrogate's prediction out_i of every sample (device inputs as for
 * tf_fno_train), in batches of max_batch.  Synchronous. */
tf_status tf_fno_eval(tf_fno* f, const float* params_dev, const float* head_w_dev, const float* targets_dev,
                      int64_t n, double* rel_l2);

/* The operator's truncated transforms on their own (device pointers):
 * modes <- rfft3(v) on the kept modes; u <- irfft3 of the kept modes with
 * zeros elsewhere (scipy / numpy normalisation: the inverse carries 1/64^3). */
tf_status tf_fno_spectral_forward(tf_fno* f, const float* v, int32_t batch, float* modes);
tf_status tf_fno_spectral_inverse(tf_fno* f, const float* modes, int32_t batch, float* u);

/* Checkpoint the float32 parameters (and, for a training surrogate, the Adam
 * moments and step) to a file, and read one back.  A surrogate with a
 * padded transform records its period, and loading restores it.  TF_EINVAL
 * for a file of another architecture or head. */
tf_status tf_fno_save(tf_fno* f, const char* path);
tf_status tf_fno_load(tf_fno* f, const char* path);

#ifdef __cplusplus
}
#endif

#endif /* TFOCUS_H */

/*
 * libmhd: MI355X (gfx950) pseudo-spectral compressible-MHD hot path.
 *
 * The library evolves the eight conserved fields of the paper's compressible
 * MHD system (Section III, Eqs. MHD1-MHD4: mass, momentum, total energy,
 * induction), in the normalised Heaviside-Lorentz units of Section V
 * (magnetic pressure |B|^2/2, Lorentz stress B B), on the periodic box
 * [0, 2*pi)^3 with an n^3 grid.  Spatial derivatives are pseudo-spectral
 * (Section II: transform, multiply by i k, transform back; nonlinear products
 * in real space), dealiased by the cubic 2/3 rule, and time advances with the
 * second-order Adams-Bashforth scheme (Sections II and IV) started by one
 * Euler step.  The closure is the ideal gas P = (gamma-1)(E - m.u/2 - |B|^2/2)
 * with the energy equation MHD3.
 *
 * Conventions shared by every entry point
 *  - Real field sets are device arrays [8][n][n][n], x fastest, field order
 *    rho, m_x, m_y, m_z, B_x, B_y, B_z, E; element type given by `dtype`
 *    (MHD_FP64 = double, MHD_FP32 = float).
 *  - Forward DFT f^(k) = sum_x f(x) exp(-i k.x) (unnormalised); inverse with
 *    1/n^3.  Wavenumber of index i is i for 2i < n, else i - n.
 *  - A mode is retained iff 3|k| < n on all three axes; K = (n-1)/3 is the
 *    largest retained |k| per axis.
 *  - Compact spectra (the state and the mhd_fft3d hook) are complex arrays
 *    [kz][ky][kx] of (2K+1) x (2K+1) x P interleaved (re, im) pairs in the
 *    working precision, P = mhd_spectrum_pitch(n) = K+1 rounded up to a
 *    multiple of 8; kz and ky run 0..K then -K..-1, kx runs 0..K, and the
 *    entries kx = K+1..P-1 are padding that is neither read nor written.
 *  - Every call enqueues work on the stream given to mhd_init and returns
 *    without waiting, except where a function says it synchronises.
 *  - All device memory belongs to the caller: the workspace passed to
 *    mhd_init and the field arrays of each call.  The library never calls
 *    hipMalloc or hipFree.  A context keeps pointers into its workspace, so
 *    the workspace must outlive it.
 *  - Functions return MHD_OK (0) or a negative MHD_E_* status; nothing throws
 *    or exits.  After MHD_E_HIP, mhd_last_error gives the HIP error text.
 *  - One context per stream; a context is not thread-safe.
 *
 * Supported sizes: n in {8, 12, 16, 24, 32, 48, 64, 96, 128, 192, 256, 384,
 * 512} for MHD_FP64 and additionally 768 and 1024 for MHD_FP32 and MHD_MIXED
 * (mhd_supported_size).
 */
#ifndef MHD_H
#define MHD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    MHD_OK = 0,
    MHD_E_ARG = -1,       /* null pointer, bad enum, non-positive dt, ... */
    MHD_E_SIZE = -2,      /* n not supported for this precision */
    MHD_E_WORKSPACE = -3, /* workspace null, misaligned (256 B) or too small */
    MHD_E_HIP = -4,       /* a HIP runtime call failed (see mhd_last_error) */
    MHD_E_NONFINITE = -5, /* a non-finite value was found in the state */
    MHD_E_CFL = -6,       /* dt exceeded the CFL limit (only with MHD_FLAG_CHECK_CFL) */
    MHD_E_STATE = -7      /* no state has been set yet, or a blob is not a valid checkpoint */
};

/* Working precision (mhd_params.precision) and real-field element types
 * (dtype arguments take MHD_FP64 or MHD_FP32 only).  MHD_MIXED stores and
 * computes in FP32 but runs every radix-16 FFT stage that goes LDS to LDS as
 * a matrix product on the MFMA units: the DFT matrix and the data are split
 * into BF16 high and low parts and three products are accumulated in FP32
 * (the low*low product is dropped); twiddles stay FP32.  Real fields and
 * compact spectra of an MHD_MIXED context are FP32. */
enum { MHD_FP64 = 0, MHD_FP32 = 1, MHD_MIXED = 2 };

/* mhd_params.flags */
enum {
    MHD_FLAG_CHECK_CFL = 1,      /* mhd_diagnostics reports MHD_E_CFL when dt > dt_cfl seen by a step */
    MHD_FLAG_NO_GRAPH = 2,       /* mhd_step launches every kernel itself instead of replaying a HIP graph */
    MHD_FLAG_VISC_LAPLACIAN = 4, /* viscous force nu lap u (Section V's momentum equation) instead of
                                    div(2 nu rho S) (Eq. MHD2); the energy gains nu lap(|u|^2/2), its work
                                    plus heating, so <E> stays conserved */
    MHD_FLAG_KINEMATIC = 8,      /* kinematic dynamo (Section V-B): rho, m and E are frozen and only the
                                    induction equation evolves, under the frozen flow */
    MHD_FLAG_SCHEDULE_ALT = 16   /* run the alternative kernel schedule (radix plans with one radix-16
                                    stage, 8-column tiles), built for MHD_FP32 at n = 32, 64, 96, 128 only
                                    (MHD_E_SIZE elsewhere); the ensemble autotuner chooses between the two
                                    schedules per group, and a single run with this flag reproduces a
                                    member run on that schedule bit for bit */
};

/* Time integrators (mhd_params.scheme); Section II names all three and finds
 * that they agree.  MHD_AB2: U^{n+1} = U^n + dt (3/2 R^n - 1/2 R^{n-1}), Euler
 * first (one right-hand side per step).  MHD_RK4: the classical four-stage
 * Runge-Kutta scheme (four).  MHD_PC: the AB2 step as predictor U*, then the
 * trapezoidal corrector U^{n+1} = U^n + dt/2 (R^n + R(U*)) (two). */
enum { MHD_AB2 = 0, MHD_RK4 = 1, MHD_PC = 2 };

typedef struct {
    int32_t n;         /* grid points per side */
    int32_t precision; /* MHD_FP64, MHD_FP32 or MHD_MIXED */
    int32_t flags;     /* MHD_FLAG_* */
    int32_t scheme;    /* MHD_AB2 (0), MHD_RK4 or MHD_PC */
    double gamma;      /* ratio of specific heats, > 1 */
    double nu;         /* kinematic viscosity, >= 0 (Eq. MHD2: div(2 nu rho S); with
                          MHD_FLAG_VISC_LAPLACIAN the coefficient of nu lap u) */
    double eta;        /* magnetic diffusivity, >= 0 (Eq. MHD4: eta lap B) */
    double dt;         /* fixed time step, > 0 */
    double cfl;        /* Courant number of the dt_cfl diagnostic, > 0 (e.g. 0.1) */
    double force;      /* amplitude F0 of the ABC body force rho f of Section V-B, f = F0 (sin z + cos y,
                          sin x + cos z, sin y + cos x) (A = B = C = 1, k_f = 1): the momentum gains
                          rho f and the energy its work m.f; 0 = unforced */
} mhd_params;

/* FP64 volume-mean diagnostics of the current state (Section III: dynamic
 * sound speed c_s = sqrt(gamma <P>/<rho>), Alfven speed and Mach numbers;
 * Section V: energies per grid point). */
typedef struct {
    double t;          /* simulated time */
    int64_t step;      /* steps taken since mhd_set_state */
    double mass;       /* <rho> */
    double mom[3];     /* <m> */
    double e_kin;      /* <m.u/2> */
    double e_mag;      /* <|B|^2/2> */
    double e_int;      /* <P>/(gamma-1) */
    double e_tot;      /* <E> */
    double h_cross;    /* <u.B> */
    double h_mag;      /* <A.B>, Coulomb gauge, k = 0 excluded */
    double divb_rms;   /* <(div B)^2>^(1/2) (Parseval) */
    double divb_max;   /* max |div B| over the grid */
    double divb_rel;   /* divb_rms / <|curl B|^2>^(1/2) */
    double j_rms;      /* <|curl B|^2>^(1/2) */
    double dt_cfl;     /* cfl * (2 pi/n) / max(max_i |u_i| + c_f), c_f^2 = (gamma P + |B|^2)/rho */
    double c_s;        /* sqrt(gamma <P> / <rho>) */
    double v_a;        /* <|B|> / sqrt(<rho>) */
    double mach_s;     /* <|u|> / c_s */
    double mach_a;     /* <|u|> / v_a */
    int64_t nonfinite; /* non-finite values in the real-space state */
} mhd_diag;

typedef struct mhd_ctx mhd_ctx;

/* 1 if n is supported for `precision`, else 0.  (Section II: the periodic
 * box is discretised on n^3 points for the FFT; sizes are n = 2^a 3^b.) */
int mhd_supported_size(int32_t n, int32_t precision);

/* Bytes of device workspace mhd_init needs for these parameters, or 0 if the
 * parameters are invalid. */
size_t mhd_workspace_bytes(const mhd_params* p);

/* Creates a context for one run of Eqs. MHD1-MHD4 (Section III) with the
 * transport coefficients nu, eta of Eqs. MHD2-MHD4 and the time step of the
 * Adams-Bashforth scheme (Sections II and IV).  d_workspace: caller-owned
 * device memory of at least mhd_workspace_bytes(p) bytes, 256-byte aligned
 * (MHD_E_WORKSPACE otherwise).  hip_stream: the hipStream_t every later call
 * enqueues on (NULL = default stream).  Uploads the twiddle tables
 * (synchronously).  *out receives the context; MHD_E_ARG / MHD_E_SIZE for
 * invalid parameters. */
int mhd_init(const mhd_params* p, void* d_workspace, size_t ws_bytes, void* hip_stream, mhd_ctx** out);

/* Sets the state to D F[U] for the real fields U = d_fields ([8][n][n][n],
 * element type dtype; caller-owned, read only) -- the spectral representation
 * of the conserved variables of Eqs. MHD1-MHD4 that the pseudo-spectral method
 * of Section II evolves -- and resets t, the step count and the AB2 history
 * (the next step is an Euler step).  Inputs are rounded to the working
 * precision.  MHD_E_ARG for a null pointer or a bad dtype. */
int mhd_set_state(mhd_ctx* ctx, const void* d_fields, int32_t dtype);

/* Writes F^-1 of the state (the conserved fields of Eqs. MHD1-MHD4 on the
 * grid, Section II's inverse transform) to the caller-owned d_fields
 * ([8][n][n][n], element type dtype).  MHD_E_STATE if no state is set. */
int mhd_get_state(mhd_ctx* ctx, void* d_fields, int32_t dtype);

/* Pure right-hand side (Eqs. MHD1-MHD4 of Section III, evaluated by the
 * pseudo-spectral method of Section II): d_rhs_out = F^-1 R(D F[U]) for the
 * real fields U = d_fields_in; the context's state, history and status are
 * untouched.  Both arrays caller-owned, [8][n][n][n] of element type dtype;
 * they may not overlap.  MHD_E_ARG for a null pointer or a bad dtype. */
int mhd_rhs(mhd_ctx* ctx, const void* d_fields_in, void* d_rhs_out, int32_t dtype);

/* Allocation-free right-hand side, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc): the same result as mhd_init + mhd_rhs with parameters p
 * (bit for bit: the same kernels and launch geometry), but the workspace is
 * a file-scope device array of the library (64 MiB; each GPU holds its own
 * copy until the process ends) and the context lives on the caller's stack,
 * so nothing is allocated on the device or the host.  d_fields_in /
 * d_rhs_out: caller-owned [8][n][n][n] arrays of element type dtype, on the
 * current device; the work is enqueued on hip_stream (NULL = default stream)
 * after one synchronous upload of the twiddle table.  Sizes whose workspace
 * exceeds 64 MiB (mhd_workspace_bytes(p) > 64 MiB: n <= 64 fits in every
 * precision) return MHD_E_WORKSPACE.  Every call on a GPU shares that GPU's
 * array and leaves its contents behind; nothing in it needs to start at zero
 * (every array the right-hand side reads is written earlier in the same
 * call).  Calls that overlap on one GPU (other streams, other host threads)
 * race on the array and must be serialised by the caller. */
int mhd_rhs_noalloc(const mhd_params* p, const void* d_fields_in, void* d_rhs_out, int32_t dtype,
                    void* hip_stream);

/* Switches the kernel schedule of the context's later right-hand sides and
 * steps (0 = default build, 1 = the MHD_FLAG_SCHEDULE_ALT build); the state,
 * the history and the transforms of set/get/diagnostics are unaffected (both
 * builds lay out the compact spectra identically).  A run whose state was set
 * on the default build and then switched reproduces an ensemble member on
 * that schedule bit for bit (members get their states before the tuner
 * runs).  MHD_E_SIZE where the build does not exist (the context keeps its
 * schedule); MHD_E_ARG for other values. */
int mhd_set_schedule(mhd_ctx* ctx, int32_t schedule);

/* Advances the state by nsteps >= 0 steps of the Adams-Bashforth scheme
 * (Sections II and IV; second order, fixed dt):
 * U^{n+1} = U^n + dt (3/2 R^n - 1/2 R^{n-1}); the first step after
 * mhd_set_state is Euler.  The first call launches the steady step's
 * kernels once under stream capture and every later step replays that HIP
 * graph (unless MHD_FLAG_NO_GRAPH is set or mhd_profile is recording); the
 * arithmetic is the same either way.  Returns MHD_E_STATE if no state is
 * set, MHD_E_ARG for nsteps < 0. */
int mhd_step(mhd_ctx* ctx, int32_t nsteps);

/* Computes the diagnostics of the current state (Section III: c_s, V_A,
 * M_s, M_A; Section V: energies per grid point, cross and magnetic helicity)
 * into *h_out (host memory), with FP64 compensated (Neumaier) reductions, and
 * synchronises the stream.  Returns MHD_E_NONFINITE if the state holds a
 * non-finite value or a step met one, MHD_E_CFL if MHD_FLAG_CHECK_CFL is set
 * and some step since mhd_set_state ran with dt above its CFL limit (the
 * steps' largest signal speed is kept and reduced in FP64); *h_out is filled
 * either way.  MHD_E_STATE if no state is set. */
int mhd_diagnostics(mhd_ctx* ctx, mhd_diag* h_out);

/* Turbulence diagnostics of Section V (its decaying-turbulence and MHD
 * runs): shell spectra and velocity-gradient statistics of the current state,
 * in FP64 from the compact spectra, with u = m/rho formed on the grid and
 * u^ = D F[u] as the right-hand side forms them.  Shell s holds the retained
 * modes with floor(|k| + 1/2) = s, s = 0 .. mhd_spectra_shells(n) - 1.
 *   h_eu[s] = sum over shell s of |u^|^2 / (2 n^6)  (kinetic spectrum per unit mass)
 *   h_eb[s] = sum over shell s of |B^|^2 / (2 n^6)  (sums to <|B|^2>/2)
 *   h_mom[0] = theta' = <(div u)^2>^(1/2)  (Parseval)
 *   h_mom[1] = S_3 = <d^3> / <d^2>^(3/2), d = du_x/dx on the grid
 *   h_mom[2] = <d^2>^(1/2)
 * Host arrays of mhd_spectra_shells(n) (h_eu, h_eb) and 3 (h_mom) doubles.
 * Synchronises the stream; uses the workspace's scratch (not the state).
 * MHD_E_STATE if no state is set. */
int32_t mhd_spectra_shells(int32_t n);
int mhd_spectra(mhd_ctx* ctx, double* h_eu, double* h_eb, double* h_mom);

/* Tracer particles (Section VI): passive particles sprinkled in the box,
 * moved by the magnetic field of the grid.  d_pos, d_vel: caller-owned FP64
 * device arrays [np][3] of (x, y, z) components; positions are taken modulo
 * the period 2 pi.  Grid fields are interpolated to a particle by
 * cloud-in-cell weights (Section VI's eight-corner volume weighting,
 * normalised by the cell volume: the trilinear interpolant; the paper's
 * extra factor dt in those weights is dropped).  Both calls use the current
 * state (synthesised to real space in the workspace's scratch) and enqueue
 * on the context's stream.
 * mhd_tracers_velocity: d_vel = the grid velocity u = m/rho interpolated at
 *   d_pos (the tracers' initial velocity, Section VI).
 * mhd_tracers_push: nsteps Boris steps of length dt with q = M = 1:
 *   t = B_p dt/2, s = 2t/(1 + |t|^2), v' = v + v x t, v <- v + v' x s,
 *   x <- x + v dt, wrapped into [0, 2 pi); B_p is the field interpolated at
 *   each step's start position.  The field is the current state's, held fixed
 *   over the call; interleave with mhd_step to follow an evolving flow.
 * MHD_E_STATE if no state is set; MHD_E_ARG for null arrays with np > 0,
 * np < 0, nsteps < 0 or a non-finite dt. */
int mhd_tracers_velocity(mhd_ctx* ctx, const double* d_pos, double* d_vel, int64_t np);
int mhd_tracers_push(mhd_ctx* ctx, double* d_pos, double* d_vel, int64_t np, double dt, int32_t nsteps);

/* Checkpoint/restart of the multistep state.  The AB2 scheme (Sections II
 * and IV) carries the previous right-hand side R^{n-1} besides U^n, so a
 * restart needs both: a checkpoint blob holds a 256-byte header (format
 * version, n, precision, step, t, dt, sizes and a 64-bit checksum of every
 * other word), the compact state U^n, the history R^{n-1} and the CFL /
 * non-finite status of the steps taken so far.  The blob is caller-owned
 * device memory of mhd_checkpoint_bytes(ctx) bytes, 256-byte aligned.
 *
 * mhd_checkpoint_bytes: blob size for this context (0 for a null context).
 * mhd_save: enqueues the copy and the checksum on the context's stream
 *   (asynchronous); MHD_E_STATE if no state is set, MHD_E_ARG for a null or
 *   misaligned blob.
 * mhd_load: synchronises the stream, checks the header and the checksum and,
 *   if they hold, enqueues the copies into the context: a run continued from
 *   a blob is bit for bit the run that saved it.  MHD_E_STATE for a blob that
 *   is not a valid checkpoint (wrong format or size, checksum mismatch: the
 *   context is left unchanged); MHD_E_ARG for a valid checkpoint of a
 *   different n, precision or dt. */
size_t mhd_checkpoint_bytes(const mhd_ctx* ctx);
int mhd_save(mhd_ctx* ctx, void* d_blob);
int mhd_load(mhd_ctx* ctx, const void* d_blob);

/* Test hook with the transform conventions above (Section II: the forward
 * and inverse FFTs of the pseudo-spectral method).  dir = -1: d_in is one real
 * n^3 field, d_out its compact spectrum D F[f].  dir = +1: d_in a compact
 * spectrum, d_out the real field F^-1 (n^-3 normalised).  Both in the working
 * precision; the arrays may not overlap.  Uses the context's workspace. */
int mhd_fft3d(mhd_ctx* ctx, int32_t dir, const void* d_in, void* d_out);

/* Number of complex values of one compact spectrum, (2K+1)^2 P. */
int64_t mhd_spectrum_size(int32_t n);

/* kx pitch P of the compact spectrum (K+1 rounded up to a multiple of 8). */
int32_t mhd_spectrum_pitch(int32_t n);

/* Launch classes of one step, for mhd_profile_read.  Suffix _A: phase A
 * (u^ = D F[m/rho]); _B: phase B (fluxes and update); ZRHS: forward z with
 * the momentum, induction and energy right-hand sides and their update; RHO:
 * the density right-hand side -i k.m^ and its update. */
enum {
    MHD_PASS_ZINV_A = 0, MHD_PASS_YINV_A, MHD_PASS_XA, MHD_PASS_YFWD_A, MHD_PASS_ZFWD_A,
    MHD_PASS_ZINV_B, MHD_PASS_YINV_B, MHD_PASS_XB, MHD_PASS_YFWD_B, MHD_PASS_ZRHS,
    MHD_PASS_RHO, MHD_PASS_REDUCE, MHD_PASS_COUNT
};

/* Benchmark hook (not physics).  class_mask != 0 clears the counters and
 * brackets every later kernel launch of mhd_step whose launch class cls has
 * bit (1 << cls) set in class_mask with a pair of HIP events on the
 * context's stream (-1 selects every class; at most 4096 launches are
 * recorded, later ones are counted as dropped); class_mask = 0 stops
 * recording.  Each event pair adds a little time between launches, so a
 * throughput measurement should select only the classes it needs.  Creates
 * its events on first use (no device memory). */
int mhd_profile(mhd_ctx* ctx, int32_t class_mask);

/* Synchronises the stream and writes, per launch class (MHD_PASS_*), the
 * summed kernel time in milliseconds, the number of launches timed and the
 * summed algorithmic HBM bytes of those launches (each input and output
 * array counted once).  Any pointer may be NULL.  Returns the number of
 * dropped launches through *dropped when non-NULL. */
int mhd_profile_read(mhd_ctx* ctx, double* ms, int64_t* launches, double* bytes, int64_t* dropped);

/* Algorithmic HBM bytes of one mhd_step of this context (sum over its
 * launches, each array read or written once), or 0 for a null context. */
double mhd_step_bytes(const mhd_ctx* ctx);

/* Benchmark hook (not physics): enqueues one streaming copy of `bytes`
 * (a multiple of 16; both pointers 16-byte aligned, caller-owned device
 * memory) from d_src to d_dst on hip_stream, with the library's own copy
 * kernel.  Its rate is the practical HBM ceiling the passes are compared
 * with.  MHD_E_ARG for bad sizes or alignment. */
int mhd_bench_copy(const void* d_src, void* d_dst, size_t bytes, void* hip_stream);

/* Releases the host-side context (not the caller's workspace). */
int mhd_destroy(mhd_ctx* ctx);

/* Static text of a status code. */
const char* mhd_status_string(int status);

/* Text of the last HIP error seen by ctx ("" if none). */
const char* mhd_last_error(const mhd_ctx* ctx);

/* ---------------------------------------------------------------- ensembles
 *
 * An ensemble advances `count` independent runs of the same equations
 * (Eqs. MHD1-MHD4, AB2 stepping as in mhd_step), each with its own grid size,
 * precision, nu, eta, gamma and dt.  Members with equal (n, precision) form a
 * group of at most 64 whose passes run as one persistent launch per pass over
 * all of the group's members; groups run as parallel branches of one HIP
 * graph, replayed once per step.  Each member's arithmetic is exactly that of
 * a single context with the same parameters, so a member's state matches a
 * solo run bit for bit, and a non-finite value in one member never reaches
 * another.  The paper runs one simulation at a time; the ensemble is an
 * extension of the same per-step operator.  Members use the AB2 scheme
 * without the Section V variants (scheme MHD_AB2, no force, neither
 * MHD_FLAG_VISC_LAPLACIAN nor MHD_FLAG_KINEMATIC; MHD_E_ARG otherwise). */
typedef struct mhd_ens mhd_ens;

/* Bytes of device workspace for the members p[0..count-1] (count >= 1), or 0
 * if any member's parameters are invalid. */
size_t mhd_ens_workspace_bytes(const mhd_params* p, int32_t count);

/* Creates an ensemble.  d_workspace: caller-owned device memory of at least
 * mhd_ens_workspace_bytes(p, count) bytes, 256-byte aligned; every call
 * enqueues on hip_stream (NULL = default stream).  The ensemble creates one
 * extra stream per group (default priority) for the graph's branches.
 * tune_cache_path: text file of tuned launch geometries (read at init,
 * appended to after tuning); NULL keeps tuning results in memory only; an
 * empty string "" turns tuning off (every pass uses its resident-occupancy
 * grid).  Tuning runs at the first mhd_ens_step with all states set and
 * evaluates right-hand sides only, so it leaves every state unchanged. */
int mhd_ens_init(const mhd_params* p, int32_t count, void* d_workspace, size_t ws_bytes, void* hip_stream,
                 const char* tune_cache_path, mhd_ens** out);

/* Sets member `member`'s state from real fields ([8][n][n][n], element type
 * dtype) exactly as mhd_set_state does for a context. */
int mhd_ens_set_state(mhd_ens* ens, int32_t member, const void* d_fields, int32_t dtype);

/* Writes member `member`'s state as real fields, as mhd_get_state. */
int mhd_ens_get_state(mhd_ens* ens, int32_t member, void* d_fields, int32_t dtype);

/* Advances every member by nsteps >= 0 steps (MHD_E_STATE unless every
 * member has a state).  A step in which some member takes its first (Euler)
 * step runs eagerly; every other step replays the captured graph. */
int mhd_ens_step(mhd_ens* ens, int32_t nsteps);

/* Diagnostics of every member into h_out[count] (host) and each member's
 * status (as mhd_diagnostics would return it) into h_status[count] (host,
 * may be NULL); synchronises the stream.  Returns MHD_OK when every member
 * is finite and within its CFL limit, else the first member's failing
 * status. */
int mhd_ens_diagnostics(mhd_ens* ens, mhd_diag* h_out, int32_t* h_status);

/* Number of member groups (equal n and precision, at most 64 members). */
int32_t mhd_ens_num_groups(const mhd_ens* ens);

/* Group g's grid size, precision, member count, tuned persistent-grid
 * scales (column passes, row passes; 1 = resident-occupancy grid) and tuned
 * kernel schedule (0 = default, 1 = the MHD_FLAG_SCHEDULE_ALT build).  Any
 * output pointer may be NULL. */
int mhd_ens_group_info(const mhd_ens* ens, int32_t g, int32_t* n, int32_t* precision, int32_t* members,
                       double* col_scale, double* row_scale, int32_t* schedule);

/* Algorithmic HBM bytes of one mhd_ens_step over all members. */
double mhd_ens_step_bytes(const mhd_ens* ens);

/* Releases the ensemble's host state, streams, events and graph (not the
 * caller's workspace). */
int mhd_ens_destroy(mhd_ens* ens);

/* Text of the last HIP error seen by the ensemble ("" if none). */
const char* mhd_ens_last_error(const mhd_ens* ens);

#ifdef __cplusplus
}
#endif

#endif /* MHD_H */

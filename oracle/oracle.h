/*
 * FP64 CPU oracle for the pseudo-spectral compressible-MHD right-hand side.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path links, loads or calls
 * this code: only the test suite, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no source with the HIP library: its own FFT,
 * its own spectral operators, its own flux arithmetic.
 *
 * What it computes (paper: Section III, Eqs. MHD1-MHD4 and their component
 * form; Section V, Eqs. density/velocity/Bfield for the normalised units):
 *   - a periodic box [0, 2*pi)^3 on an n^3 grid, arrays [z][y][x], x fastest;
 *   - the unnormalised forward DFT  f^(k) = sum_x f(x) exp(-i k.x) and the
 *     inverse with 1/n^3;
 *   - the cubic 2/3 dealiasing mask D(k) = [3|kx|<n][3|ky|<n][3|kz|<n];
 *   - the spectral right-hand side R(U^) of the eight conserved fields
 *     (rho, m_x, m_y, m_z, B_x, B_y, B_z, E), Heaviside-Lorentz units
 *     (4*pi -> 1, c -> 1), ideal-gas closure P = (gamma-1)(E - m.u/2 - |B|^2/2);
 *   - second-order Adams-Bashforth stepping, Euler on the first step; the
 *     classical Runge-Kutta 4 and a second-order Adams-Bashforth-Moulton
 *     predictor-corrector (Section II names all three);
 *   - the variants of Section V: viscous force nu lap u instead of the stress
 *     form, the ABC body force rho f, and the kinematic mode (rho, m, E
 *     frozen, B evolving);
 *   - FP64 volume-mean diagnostics with Neumaier compensated sums.
 *
 * Every function returns 0 on success and a negative value on a bad argument
 * or an allocation failure.  All arrays are caller-owned host memory.
 */
#ifndef MHD_ORACLE_H
#define MHD_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ORC_NFIELDS 8

/* Time integrators (orc_params.scheme) and options (orc_params.options). */
enum { ORC_AB2 = 0, ORC_RK4 = 1, ORC_PC = 2 };
enum { ORC_VISC_LAPLACIAN = 1, ORC_KINEMATIC = 2 };

typedef struct {
    int32_t n;      /* grid points per side */
    double gamma;   /* ratio of specific heats */
    double nu;      /* kinematic viscosity (with ORC_VISC_LAPLACIAN: the coefficient of nu lap u) */
    double eta;     /* magnetic diffusivity */
    double dt;      /* fixed time step */
    double cfl;     /* Courant number used by the dt_cfl diagnostic */
    int32_t scheme; /* ORC_AB2, ORC_RK4 or ORC_PC (orc_run) */
    int32_t options;/* ORC_VISC_LAPLACIAN, ORC_KINEMATIC */
    double force;   /* amplitude of the ABC body force (0 = unforced) */
} orc_params;

/* Indices of the diagnostic vector written by orc_diag. */
enum {
    ORC_MASS = 0, ORC_MOMX, ORC_MOMY, ORC_MOMZ,
    ORC_EKIN, ORC_EMAG, ORC_EINT, ORC_ETOT,
    ORC_HCROSS, ORC_HMAG,
    ORC_DIVB_RMS, ORC_DIVB_MAX, ORC_DIVB_REL,
    ORC_DTCFL, ORC_CS, ORC_VA, ORC_MACHS, ORC_MACHA,
    ORC_NONFINITE, ORC_JRMS,
    ORC_NDIAG
};

/* 1D complex DFT of length n (any n >= 1), unnormalised, interleaved re/im.
 * sign = -1 forward, +1 inverse.  in and out may not alias. */
int orc_fft1d(int32_t n, const double* in, double* out, int32_t sign);

/* In-place 3D complex DFT of an n^3 interleaved array [z][y][x], unnormalised. */
int orc_fft3d(int32_t n, double* a, int32_t sign);

/* f <- F^-1 D F f for one real n^3 field (projection onto the retained band). */
int orc_project(int32_t n, double* f);

/* Real-space right-hand side: U[8][n^3] -> R[8][n^3], with U^ = D F U first. */
int orc_rhs(const orc_params* p, const double* U, double* R);

/* Advance U[8][n^3] in place by nsteps steps of p->scheme (AB2 and PC start
 * with an Euler predictor), starting from U^ = D F U.  On return U holds
 * F^-1 of the final spectral state. */
int orc_run(const orc_params* p, double* U, int32_t nsteps);

/* Diagnostics of the state U^ = D F U (see the ORC_* indices). */
int orc_diag(const orc_params* p, const double* U, double* out);

/* Turbulence diagnostics (Section V) of the state U^ = D F U, with
 * u = m / rho and u^ = D F u: kinetic and magnetic shell spectra
 * eu[s], eb[s] (shell s: floor(|k| + 1/2) = s, s < nshell; sum |.|^2 / 2n^6),
 * and mom = {theta' = <(div u)^2>^(1/2), S_3 = <d^3>/<d^2>^(3/2),
 * <d^2>^(1/2)} with d = du_x/dx. */
int orc_spectra(const orc_params* p, const double* U, int32_t nshell, double* eu, double* eb, double* mom);

/* Tracer particles (Section VI).  Positions pos[np][3] = (x, y, z) in
 * [0, 2 pi) (any real value is taken modulo the period).
 * orc_cic: cloud-in-cell interpolation of the real fields f[nc][n^3] at the
 *   positions into out[np][nc] (the trilinear interpolant of the grid values).
 * orc_tracer_push: nsteps Boris steps (q = M = 1) in the magnetic field
 *   B[3][n^3], interpolated by cloud-in-cell at each step's start position;
 *   positions advance by v dt and wrap into [0, 2 pi). */
int orc_cic(int32_t n, const double* f, int32_t nc, const double* pos, int64_t np, double* out);
int orc_tracer_push(int32_t n, const double* B, double* pos, double* vel, int64_t np, double dt, int32_t nsteps);

/* Neumaier compensated sum (exposed so tests can pin it against math.fsum). */
double orc_neumaier_sum(const double* x, int64_t n);

/* Number of OpenMP threads the oracle uses (1 if built without OpenMP). */
int32_t orc_num_threads(void);

/* Sets the number of OpenMP threads of later calls (threads > 0). */
void orc_set_num_threads(int32_t threads);

#ifdef __cplusplus
}
#endif

#endif /* MHD_ORACLE_H */

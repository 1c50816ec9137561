/*
 * FP64 CPU oracle: FFT, spectral operators, MHD right-hand side, AB2 stepping
 * and diagnostics.  TEST INFRASTRUCTURE ONLY (see oracle.h): no product code
 * calls it, and it shares no source with the HIP library.
 *
 * It is written to be read against the paper, not to be fast: full complex
 * n^3 arrays, one 3D transform per derivative, the fluxes written out term by
 * term in the order of the paper's component equations.
 */
#include "oracle.h"

#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;

static const double TWO_PI = 6.28318530717958647692528676655900577;

/* ------------------------------------------------------------------------- */
/* FFT: recursive mixed-radix decimation in time.                             */
/* X[k + q*m] = sum_r W_n^{r(k+q*m)} Y_r[k], Y_r = DFT_m of x[j*p + r],       */
/* p the smallest prime factor of n, m = n/p (any n; a prime n is a direct    */
/* DFT).  Roots come from a table of exp(sign*2*pi*i*j/n0), j < n0, built     */
/* with libm cos/sin of an exactly reduced integer argument.                  */
/* ------------------------------------------------------------------------- */

static int smallest_factor(int n) {
    if (n % 2 == 0) return 2;
    for (int p = 3; p * p <= n; p += 2)
        if (n % p == 0) return p;
    return n;
}

static cplx* root_table(int n, int sign) {
    cplx* tw = (cplx*)malloc((size_t)n * sizeof(cplx));
    if (!tw) return NULL;
    for (int j = 0; j < n; ++j) {
        double a = TWO_PI * (double)j / (double)n;
        tw[j] = cos(a) + (double)sign * I * sin(a);
    }
    return tw;
}

/* out[0..n) = DFT_n of in[0], in[s], in[2s], ...; W_n^j = tw[(j*ts) mod n0]. */
static void fft_rec(int n, const cplx* in, long s, cplx* out,
                    const cplx* tw, long ts, long n0) {
    if (n == 1) { out[0] = in[0]; return; }
    int p = smallest_factor(n), m = n / p;
    for (int r = 0; r < p; ++r)
        fft_rec(m, in + (long)r * s, s * p, out + (long)r * m, tw, ts * p, n0);
    cplx t[p], y[p];
    for (int k = 0; k < m; ++k) {
        for (int r = 0; r < p; ++r)
            t[r] = out[r * m + k] * tw[(((long)r * k) % n) * ts % n0];
        for (int q = 0; q < p; ++q) {
            cplx acc = 0;
            for (int r = 0; r < p; ++r)
                acc += t[r] * tw[(((long)r * q) % p) * (ts * m) % n0];
            y[q] = acc;
        }
        for (int q = 0; q < p; ++q) out[k + q * m] = y[q];
    }
}

int orc_fft1d(int32_t n, const double* in, double* out, int32_t sign) {
    if (n < 1 || (sign != 1 && sign != -1) || !in || !out) return -1;
    cplx* tw = root_table(n, sign);
    if (!tw) return -2;
    fft_rec(n, (const cplx*)in, 1, (cplx*)out, tw, 1, n);
    free(tw);
    return 0;
}

/* One 1D transform along `axis` (0 = x, 1 = y, 2 = z) of every line. */
static int fft_axis(int n, cplx* a, int axis, const cplx* tw) {
    const long N = n;
    const long stride = axis == 0 ? 1 : (axis == 1 ? N : N * N);
    int err = 0;
#pragma omp parallel
    {
        cplx* buf = (cplx*)malloc(2 * (size_t)N * sizeof(cplx));
        if (!buf) {
#pragma omp atomic write
            err = -2;
        }
#pragma omp for schedule(static)
        for (long line = 0; line < N * N; ++line) {
            if (!buf) continue;
            long base;
            if (axis == 0) base = line * N;
            else if (axis == 1) base = (line / N) * N * N + line % N;
            else base = line;
            for (long i = 0; i < N; ++i) buf[i] = a[base + i * stride];
            fft_rec(n, buf, 1, buf + N, tw, 1, N);
            for (long i = 0; i < N; ++i) a[base + i * stride] = buf[N + i];
        }
        free(buf);
    }
    return err;
}

int orc_fft3d(int32_t n, double* a, int32_t sign) {
    if (n < 1 || (sign != 1 && sign != -1) || !a) return -1;
    cplx* tw = root_table(n, sign);
    if (!tw) return -2;
    int err = 0;
    for (int axis = 0; axis < 3 && !err; ++axis) err = fft_axis(n, (cplx*)a, axis, tw);
    free(tw);
    return err;
}

/* ------------------------------------------------------------------------- */
/* Grid, wavenumbers, mask.                                                   */
/* ------------------------------------------------------------------------- */

typedef struct {
    int n;
    long n3;
    double gamma, nu, eta, dt, cfl;
    int scheme;      /* ORC_AB2, ORC_RK4, ORC_PC */
    int visc_lap;    /* 1: viscous force nu lap u (Section V) instead of div(2 nu rho S) */
    int kinematic;   /* 1: rho, m, E frozen; only the induction equation evolves */
    double force;    /* amplitude of the ABC body force rho f (Section V-B), 0 = none */
} grid;

/* Integer wavenumber of DFT index i on a box of length 2*pi. */
static inline int wavenumber(int i, int n) { return (2 * i < n) ? i : i - n; }

/* Cubic 2/3 rule: keep a mode iff 3|k| < n along every axis. */
static inline int in_band(int k, int n) { return 3 * abs(k) < n; }

static void* xmalloc(size_t bytes) { return malloc(bytes ? bytes : 1); }

/* F: real field -> full complex spectrum (unnormalised). */
static int forward(const grid* g, const double* f, cplx* out) {
    for (long i = 0; i < g->n3; ++i) out[i] = f[i];
    return orc_fft3d(g->n, (double*)out, -1);
}

/* F^-1: complex spectrum -> real part of the normalised inverse.  `tmp` is a
 * complex scratch array; `in` is left untouched. */
static int inverse(const grid* g, const cplx* in, cplx* tmp, double* out) {
    memcpy(tmp, in, (size_t)g->n3 * sizeof(cplx));
    int err = orc_fft3d(g->n, (double*)tmp, 1);
    const double s = 1.0 / (double)g->n3;
    for (long i = 0; i < g->n3; ++i) out[i] = creal(tmp[i]) * s;
    return err;
}

/* a <- D a */
static void apply_mask(const grid* g, cplx* a) {
    const int n = g->n;
    for (int iz = 0; iz < n; ++iz)
        for (int iy = 0; iy < n; ++iy)
            for (int ix = 0; ix < n; ++ix) {
                int keep = in_band(wavenumber(iz, n), n) && in_band(wavenumber(iy, n), n) &&
                           in_band(wavenumber(ix, n), n);
                if (!keep) a[((long)iz * n + iy) * n + ix] = 0;
            }
}

/* out = c * (i k_axis) * in  (axis 0 = x, 1 = y, 2 = z) */
static void times_ik(const grid* g, const cplx* in, int axis, double c, cplx* out) {
    const int n = g->n;
    for (int iz = 0; iz < n; ++iz)
        for (int iy = 0; iy < n; ++iy)
            for (int ix = 0; ix < n; ++ix) {
                int i3[3] = {ix, iy, iz};
                long id = ((long)iz * n + iy) * n + ix;
                out[id] = c * I * (double)wavenumber(i3[axis], n) * in[id];
            }
}

/* acc += c * D * (i k_axis) * in */
static void accum_ik(const grid* g, const cplx* in, int axis, double c, cplx* acc) {
    const int n = g->n;
    for (int iz = 0; iz < n; ++iz)
        for (int iy = 0; iy < n; ++iy)
            for (int ix = 0; ix < n; ++ix) {
                int kx = wavenumber(ix, n), ky = wavenumber(iy, n), kz = wavenumber(iz, n);
                if (!(in_band(kx, n) && in_band(ky, n) && in_band(kz, n))) continue;
                int k3[3] = {kx, ky, kz};
                long id = ((long)iz * n + iy) * n + ix;
                acc[id] += c * I * (double)k3[axis] * in[id];
            }
}

int orc_project(int32_t n, double* f) {
    if (n < 1 || !f) return -1;
    grid g = {n, (long)n * n * n, 0, 0, 0, 0, 0, ORC_AB2, 0, 0, 0.0};
    cplx* a = (cplx*)xmalloc((size_t)g.n3 * sizeof(cplx));
    cplx* t = (cplx*)xmalloc((size_t)g.n3 * sizeof(cplx));
    int err = (!a || !t) ? -2 : 0;
    if (!err) err = forward(&g, f, a);
    if (!err) { apply_mask(&g, a); err = inverse(&g, a, t, f); }
    free(a); free(t);
    return err;
}

/* ------------------------------------------------------------------------- */
/* Right-hand side of MHD1-MHD4 in conservative form.                         */
/* Field order: 0 rho, 1-3 m, 4-6 B, 7 E.                                     */
/* ------------------------------------------------------------------------- */

enum { F_RHO = 0, F_MX = 1, F_BX = 4, F_E = 7 };

typedef struct {
    double* U[8];     /* real state fields */
    double* u[3];     /* velocity */
    double* G[9];     /* G[3*i + j] = d_j u_i */
    double* S[9];     /* traceless strain, full symmetric 3x3 */
    double* J[3];     /* current density = curl B */
    double* flux;     /* one real flux component at a time */
    cplx* uh[3];      /* D F u */
    cplx* c0;         /* complex scratch */
    cplx* c1;         /* complex scratch */
} rhs_work;

static void free_work(rhs_work* w) {
    for (int i = 0; i < 8; ++i) free(w->U[i]);
    for (int i = 0; i < 3; ++i) { free(w->u[i]); free(w->J[i]); free(w->uh[i]); }
    for (int i = 0; i < 9; ++i) { free(w->G[i]); free(w->S[i]); }
    free(w->flux); free(w->c0); free(w->c1);
    memset(w, 0, sizeof(*w));
}

static int alloc_work(const grid* g, rhs_work* w) {
    memset(w, 0, sizeof(*w));
    size_t rb = (size_t)g->n3 * sizeof(double), cb = (size_t)g->n3 * sizeof(cplx);
    int ok = 1;
    for (int i = 0; i < 8; ++i) ok &= (w->U[i] = (double*)xmalloc(rb)) != NULL;
    for (int i = 0; i < 3; ++i) {
        ok &= (w->u[i] = (double*)xmalloc(rb)) != NULL;
        ok &= (w->J[i] = (double*)xmalloc(rb)) != NULL;
        ok &= (w->uh[i] = (cplx*)xmalloc(cb)) != NULL;
    }
    for (int i = 0; i < 9; ++i) {
        ok &= (w->G[i] = (double*)xmalloc(rb)) != NULL;
        ok &= (w->S[i] = (double*)xmalloc(rb)) != NULL;
    }
    ok &= (w->flux = (double*)xmalloc(rb)) != NULL;
    ok &= (w->c0 = (cplx*)xmalloc(cb)) != NULL;
    ok &= (w->c1 = (cplx*)xmalloc(cb)) != NULL;
    if (!ok) { free_work(w); return -2; }
    return 0;
}

/* Rh[target] += c * D * i k_axis * F[w->flux] */
static int add_divergence_term(const grid* g, rhs_work* w, int axis, double c, cplx* target) {
    int err = forward(g, w->flux, w->c0);
    accum_ik(g, w->c0, axis, c, target);
    return err;
}

/* Uh: 8 band-limited spectra; Rh: 8 output spectra. */
static int rhs_spectral(const grid* g, const cplx* const* Uh, cplx* const* Rh, rhs_work* w) {
    const long n3 = g->n3;
    const double gm1 = g->gamma - 1.0, nu = g->nu, eta = g->eta;
    /* coefficient of the stress form div(2 nu rho S) (Eqs. MHD2-MHD3); zero
     * when the viscous force is nu lap u instead (added below) */
    const double nu_s = g->visc_lap ? 0.0 : 2.0 * nu;
    int err = 0;

    /* (i) the state in real space */
    for (int f = 0; f < 8 && !err; ++f) err = inverse(g, Uh[f], w->c0, w->U[f]);
    double* rho = w->U[F_RHO];
    double* m[3] = {w->U[F_MX], w->U[F_MX + 1], w->U[F_MX + 2]};
    double* B[3] = {w->U[F_BX], w->U[F_BX + 1], w->U[F_BX + 2]};
    double* E = w->U[F_E];

    /* (ii) u = m / rho */
    for (int i = 0; i < 3; ++i)
        for (long p = 0; p < n3; ++p) w->u[i][p] = m[i][p] / rho[p];

    /* (iii) u^ = D F u, G_ij = F^-1[i k_j u^_i], S = sym(G) - (1/3) I div u  (Eqs. 3-4) */
    for (int i = 0; i < 3 && !err; ++i) {
        err = forward(g, w->u[i], w->uh[i]);
        apply_mask(g, w->uh[i]);
    }
    for (int i = 0; i < 3 && !err; ++i)
        for (int j = 0; j < 3 && !err; ++j) {
            times_ik(g, w->uh[i], j, 1.0, w->c1);
            err = inverse(g, w->c1, w->c0, w->G[3 * i + j]);
        }
    for (long p = 0; p < n3 && !err; ++p) {
        double theta = w->G[0][p] + w->G[4][p] + w->G[8][p];
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j)
                w->S[3 * i + j][p] = 0.5 * (w->G[3 * i + j][p] + w->G[3 * j + i][p]) -
                                     (i == j ? theta / 3.0 : 0.0);
    }

    /* (iv) J = curl B, spectrally: J^ = i k x B^ */
    for (int i = 0; i < 3 && !err; ++i) {
        int a = (i + 1) % 3, b = (i + 2) % 3;  /* J_i = d_a B_b - d_b B_a */
        times_ik(g, Uh[F_BX + b], a, 1.0, w->c1);
        for (long p = 0; p < n3; ++p) w->c0[p] = w->c1[p];
        times_ik(g, Uh[F_BX + a], b, 1.0, w->c1);
        for (long p = 0; p < n3; ++p) w->c1[p] = w->c0[p] - w->c1[p];
        err = inverse(g, w->c1, w->c0, w->J[i]);
    }

    for (int f = 0; f < 8; ++f) memset(Rh[f], 0, (size_t)n3 * sizeof(cplx));

    /* MHD1: R_rho = -i k . m^ (m^ is a state field, already band-limited) */
    for (int j = 0; j < 3; ++j) accum_ik(g, Uh[F_MX + j], j, -1.0, Rh[F_RHO]);

    /* MHD2: R_m_i = -D sum_j i k_j F[Pi_ij],
     * Pi_ij = m_i u_j + P_tot delta_ij - B_i B_j - 2 nu rho S_ij,
     * P = (gamma-1)(E - m.u/2 - |B|^2/2), P_tot = P + |B|^2/2. */
    for (int i = 0; i < 3 && !err; ++i)
        for (int j = 0; j < 3 && !err; ++j) {
            for (long p = 0; p < n3; ++p) {
                double B2 = B[0][p] * B[0][p] + B[1][p] * B[1][p] + B[2][p] * B[2][p];
                double mu = m[0][p] * w->u[0][p] + m[1][p] * w->u[1][p] + m[2][p] * w->u[2][p];
                double P = gm1 * (E[p] - 0.5 * mu - 0.5 * B2);
                double Ptot = P + 0.5 * B2;
                w->flux[p] = m[i][p] * w->u[j][p] + (i == j ? Ptot : 0.0) - B[i][p] * B[j][p] -
                             nu_s * rho[p] * w->S[3 * i + j][p];
            }
            err = add_divergence_term(g, w, j, -1.0, Rh[F_MX + i]);
        }

    /* MHD3: R_E = -D sum_j i k_j F[F^E_j],
     * F^E_j = (E + P_tot) u_j - (u.B) B_j - 2 nu rho (u.S)_j - eta (B x J)_j */
    for (int j = 0; j < 3 && !err; ++j) {
        int a = (j + 1) % 3, b = (j + 2) % 3;
        for (long p = 0; p < n3; ++p) {
            double u0 = w->u[0][p], u1 = w->u[1][p], u2 = w->u[2][p];
            double B2 = B[0][p] * B[0][p] + B[1][p] * B[1][p] + B[2][p] * B[2][p];
            double mu = m[0][p] * u0 + m[1][p] * u1 + m[2][p] * u2;
            double P = gm1 * (E[p] - 0.5 * mu - 0.5 * B2);
            double Ptot = P + 0.5 * B2;
            double uB = u0 * B[0][p] + u1 * B[1][p] + u2 * B[2][p];
            double uS = u0 * w->S[0 * 3 + j][p] + u1 * w->S[1 * 3 + j][p] + u2 * w->S[2 * 3 + j][p];
            double BxJ = B[a][p] * w->J[b][p] - B[b][p] * w->J[a][p];
            w->flux[p] = (E[p] + Ptot) * w->u[j][p] - uB * B[j][p] - nu_s * rho[p] * uS - eta * BxJ;
        }
        err = add_divergence_term(g, w, j, -1.0, Rh[F_E]);
    }

    /* MHD4: R_B = D (i k x F[u x B]) - eta |k|^2 B^ ;
     * (curl e)_i = d_a e_b - d_b e_a with (i, a, b) cyclic. */
    for (int c = 0; c < 3 && !err; ++c) {
        int a = (c + 1) % 3, b = (c + 2) % 3;  /* e_c = u_a B_b - u_b B_a */
        for (long p = 0; p < n3; ++p)
            w->flux[p] = w->u[a][p] * B[b][p] - w->u[b][p] * B[a][p];
        /* e_c enters (curl e)_b = d_c e_a - d_a e_c  and  (curl e)_a = d_b e_c - d_c e_b */
        err = forward(g, w->flux, w->c0);
        accum_ik(g, w->c0, a, -1.0, Rh[F_BX + b]);
        accum_ik(g, w->c0, b, +1.0, Rh[F_BX + a]);
    }
    {
        const int n = g->n;
        for (int iz = 0; iz < n; ++iz)
            for (int iy = 0; iy < n; ++iy)
                for (int ix = 0; ix < n; ++ix) {
                    double kx = wavenumber(ix, n), ky = wavenumber(iy, n), kz = wavenumber(iz, n);
                    long id = ((long)iz * n + iy) * n + ix;
                    for (int i = 0; i < 3; ++i)
                        Rh[F_BX + i][id] -= eta * (kx * kx + ky * ky + kz * kz) * Uh[F_BX + i][id];
                }
    }

    /* Viscous force nu lap u (the momentum equation of Section V) in place of
     * the stress form: R_m += -nu |k|^2 u^.  Its work plus the viscous heating
     * is nu lap(|u|^2/2), so R_E += -nu |k|^2 D F[|u|^2/2] keeps <E> conserved. */
    if (g->visc_lap && !err) {
        for (long p = 0; p < n3; ++p)
            w->flux[p] = 0.5 * (w->u[0][p] * w->u[0][p] + w->u[1][p] * w->u[1][p] + w->u[2][p] * w->u[2][p]);
        err = forward(g, w->flux, w->c0);
        apply_mask(g, w->c0);
        const int n = g->n;
        for (int iz = 0; iz < n; ++iz)
            for (int iy = 0; iy < n; ++iy)
                for (int ix = 0; ix < n; ++ix) {
                    double kx = wavenumber(ix, n), ky = wavenumber(iy, n), kz = wavenumber(iz, n);
                    double k2 = kx * kx + ky * ky + kz * kz;
                    long id = ((long)iz * n + iy) * n + ix;
                    for (int i = 0; i < 3; ++i) Rh[F_MX + i][id] -= nu * k2 * w->uh[i][id];
                    Rh[F_E][id] -= nu * k2 * w->c0[id];
                }
    }

    /* ABC body force (Section V-B) with A = B = C = 1, k_f = 1, amplitude F0:
     * f = F0 (sin z + cos y, sin x + cos z, sin y + cos x).  Momentum gains
     * rho f, the total energy the work rho f.u = m.f; both dealiased. */
    if (g->force != 0.0 && !err) {
        const int n = g->n;
        double* fx = (double*)xmalloc((size_t)n3 * sizeof(double));
        if (!fx) return -2;
        for (int c = 0; c < 3 && !err; ++c) {
            for (int iz = 0; iz < n; ++iz)
                for (int iy = 0; iy < n; ++iy)
                    for (int ix = 0; ix < n; ++ix) {
                        double x = TWO_PI * ix / n, y = TWO_PI * iy / n, z = TWO_PI * iz / n;
                        double f = c == 0 ? sin(z) + cos(y) : (c == 1 ? sin(x) + cos(z) : sin(y) + cos(x));
                        fx[((long)iz * n + iy) * n + ix] = g->force * f;
                    }
            for (long p = 0; p < n3; ++p) w->flux[p] = rho[p] * fx[p];
            err = forward(g, w->flux, w->c0);
            apply_mask(g, w->c0);
            for (long p = 0; p < n3; ++p) Rh[F_MX + c][p] += w->c0[p];
            for (long p = 0; p < n3 && !err; ++p) w->flux[p] = m[c][p] * fx[p];
            if (!err) err = forward(g, w->flux, w->c0);
            apply_mask(g, w->c0);
            for (long p = 0; p < n3; ++p) Rh[F_E][p] += w->c0[p];
        }
        free(fx);
    }

    /* Kinematic mode (Section V-B, the dynamo runs with the density and
     * velocity equations turned off): only B evolves, under the given flow. */
    if (g->kinematic) {
        memset(Rh[F_RHO], 0, (size_t)n3 * sizeof(cplx));
        for (int i = 0; i < 3; ++i) memset(Rh[F_MX + i], 0, (size_t)n3 * sizeof(cplx));
        memset(Rh[F_E], 0, (size_t)n3 * sizeof(cplx));
    }
    return err;
}

static int make_grid(const orc_params* p, grid* g) {
    if (!p || p->n < 1 || p->n > 4096) return -1;
    g->n = p->n;
    g->n3 = (long)p->n * p->n * p->n;
    g->gamma = p->gamma; g->nu = p->nu; g->eta = p->eta; g->dt = p->dt; g->cfl = p->cfl;
    if (p->scheme < ORC_AB2 || p->scheme > ORC_PC) return -1;
    g->scheme = p->scheme;
    g->visc_lap = (p->options & ORC_VISC_LAPLACIAN) != 0;
    g->kinematic = (p->options & ORC_KINEMATIC) != 0;
    g->force = p->force;
    return 0;
}

static cplx** alloc_spectra(const grid* g, int count) {
    cplx** s = (cplx**)calloc((size_t)count, sizeof(cplx*));
    if (!s) return NULL;
    for (int f = 0; f < count; ++f) {
        s[f] = (cplx*)xmalloc((size_t)g->n3 * sizeof(cplx));
        if (!s[f]) {
            for (int h = 0; h < f; ++h) free(s[h]);
            free(s);
            return NULL;
        }
    }
    return s;
}

static void free_spectra(cplx** s, int count) {
    if (!s) return;
    for (int f = 0; f < count; ++f) free(s[f]);
    free(s);
}

/* U^ = D F U for the eight fields. */
static int to_state(const grid* g, const double* U, cplx** Uh) {
    int err = 0;
    for (int f = 0; f < 8 && !err; ++f) {
        err = forward(g, U + (long)f * g->n3, Uh[f]);
        apply_mask(g, Uh[f]);
    }
    return err;
}

int orc_rhs(const orc_params* p, const double* U, double* R) {
    grid g;
    if (make_grid(p, &g) || !U || !R) return -1;
    cplx** Uh = alloc_spectra(&g, 8);
    cplx** Rh = alloc_spectra(&g, 8);
    rhs_work w;
    int err = (!Uh || !Rh) ? -2 : alloc_work(&g, &w);
    if (!err) err = to_state(&g, U, Uh);
    if (!err) err = rhs_spectral(&g, (const cplx* const*)Uh, Rh, &w);
    for (int f = 0; f < 8 && !err; ++f) err = inverse(&g, Rh[f], w.c0, R + (long)f * g.n3);
    if (Uh && Rh) free_work(&w);
    free_spectra(Uh, 8); free_spectra(Rh, 8);
    return err;
}

/* Time integrators with a fixed step (Section II lists Adams-Bashforth,
 * Runge-Kutta 4 and predictor-corrector and finds that they agree):
 *   ORC_AB2: U^{n+1} = U^n + dt (3/2 R^n - 1/2 R^{n-1}); the first step is
 *            Euler (the history R^{-1} is taken equal to R^0);
 *   ORC_RK4: the classical four-stage Runge-Kutta scheme;
 *   ORC_PC:  Adams-Bashforth-Moulton of second order: the AB2 step above as
 *            predictor U*, then the trapezoidal corrector
 *            U^{n+1} = U^n + dt/2 (R^n + R(U*)), history R^{n-1} <- R^n. */
int orc_run(const orc_params* p, double* U, int32_t nsteps) {
    grid g;
    if (make_grid(p, &g) || !U || nsteps < 0) return -1;
    const int scheme = g.scheme;
    const int nsp = scheme == ORC_AB2 ? 3 : 5;
    cplx** Uh = alloc_spectra(&g, 8);
    cplx** Rh = alloc_spectra(&g, 8);
    cplx** Rp = alloc_spectra(&g, 8);                       /* history (AB2, PC) or stage sum (RK4) */
    cplx** Us = nsp > 3 ? alloc_spectra(&g, 8) : NULL;      /* stage / predicted state */
    cplx** Rs = nsp > 3 ? alloc_spectra(&g, 8) : NULL;      /* RHS of the stage state */
    rhs_work w;
    int err = (!Uh || !Rh || !Rp || (nsp > 3 && (!Us || !Rs))) ? -2 : alloc_work(&g, &w);
    const long n3 = g.n3;
    const double dt = g.dt;
    if (!err) err = to_state(&g, U, Uh);
    for (int s = 0; s < nsteps && !err; ++s) {
        err = rhs_spectral(&g, (const cplx* const*)Uh, Rh, &w);
        if (err) break;
        if (scheme == ORC_AB2) {
            for (int f = 0; f < 8; ++f) {
                if (s == 0) memcpy(Rp[f], Rh[f], (size_t)n3 * sizeof(cplx));
                for (long q = 0; q < n3; ++q) {
                    Uh[f][q] += dt * (1.5 * Rh[f][q] - 0.5 * Rp[f][q]);
                    Rp[f][q] = Rh[f][q];
                }
            }
        } else if (scheme == ORC_RK4) {
            /* k1 = Rh; Rp accumulates k1 + 2 k2 + 2 k3 + k4 */
            static const double c_stage[3] = {0.5, 0.5, 1.0}, w_stage[3] = {2.0, 2.0, 1.0};
            for (int f = 0; f < 8; ++f)
                for (long q = 0; q < n3; ++q) {
                    Rp[f][q] = Rh[f][q];
                    Us[f][q] = Uh[f][q] + c_stage[0] * dt * Rh[f][q];
                }
            for (int st = 0; st < 3 && !err; ++st) {
                err = rhs_spectral(&g, (const cplx* const*)Us, Rs, &w);
                for (int f = 0; f < 8 && !err; ++f)
                    for (long q = 0; q < n3; ++q) {
                        Rp[f][q] += w_stage[st] * Rs[f][q];
                        if (st < 2) Us[f][q] = Uh[f][q] + c_stage[st + 1] * dt * Rs[f][q];
                    }
            }
            for (int f = 0; f < 8 && !err; ++f)
                for (long q = 0; q < n3; ++q) Uh[f][q] += dt / 6.0 * Rp[f][q];
        } else {
            /* predictor (AB2, Euler on the first step), then the trapezoidal corrector */
            for (int f = 0; f < 8; ++f) {
                if (s == 0) memcpy(Rp[f], Rh[f], (size_t)n3 * sizeof(cplx));
                for (long q = 0; q < n3; ++q) Us[f][q] = Uh[f][q] + dt * (1.5 * Rh[f][q] - 0.5 * Rp[f][q]);
            }
            err = rhs_spectral(&g, (const cplx* const*)Us, Rs, &w);
            for (int f = 0; f < 8 && !err; ++f)
                for (long q = 0; q < n3; ++q) {
                    Uh[f][q] += 0.5 * dt * (Rh[f][q] + Rs[f][q]);
                    Rp[f][q] = Rh[f][q];
                }
        }
    }
    for (int f = 0; f < 8 && !err; ++f) err = inverse(&g, Uh[f], w.c0, U + (long)f * g.n3);
    if (Uh && Rh && Rp && (nsp == 3 || (Us && Rs))) free_work(&w);
    free_spectra(Uh, 8); free_spectra(Rh, 8); free_spectra(Rp, 8);
    if (Us) free_spectra(Us, 8);
    if (Rs) free_spectra(Rs, 8);
    return err;
}

/* ------------------------------------------------------------------------- */
/* Turbulence diagnostics of Section V: shell spectra, theta', S_3.           */
/* ------------------------------------------------------------------------- */

/* Of the state U^ = D F U: u = m / rho on the grid and u^ = D F u (as the
 * right-hand side forms them).  Shell s holds the modes with
 * floor(|k| + 1/2) = s;  E_u(s) = sum over the shell of |u^|^2 / (2 n^6) and
 * E_B(s) likewise of B^ (so sum_s E_B(s) = <|B|^2> / 2 by Parseval).
 * theta' = <(div u)^2>^(1/2) with div u = F^-1[i k . u^] (Parseval sum);
 * S_3 = <d^3> / <d^2>^(3/2) with d = du_x/dx = F^-1[i k_x u^_x] on the grid. */
int orc_spectra(const orc_params* p, const double* Uin, int32_t nshell, double* eu, double* eb, double* mom) {
    grid g;
    if (make_grid(p, &g) || !Uin || nshell < 1 || !eu || !eb || !mom) return -1;
    const int n = g.n;
    const long n3 = g.n3;
    cplx** Uh = alloc_spectra(&g, 8);
    rhs_work w;
    int err = !Uh ? -2 : alloc_work(&g, &w);
    if (!err) err = to_state(&g, Uin, Uh);
    for (int f = 0; f < 8 && !err; ++f) err = inverse(&g, Uh[f], w.c0, w.U[f]);
    for (int i = 0; i < 3 && !err; ++i) {
        for (long q = 0; q < n3; ++q) w.u[i][q] = w.U[F_MX + i][q] / w.U[F_RHO][q];
        err = forward(&g, w.u[i], w.uh[i]);
        apply_mask(&g, w.uh[i]);
    }
    for (int s = 0; s < nshell; ++s) eu[s] = eb[s] = 0.0;
    double div2 = 0.0;
    const double inv6 = 1.0 / ((double)n3 * (double)n3);
    for (int iz = 0; iz < n && !err; ++iz)
        for (int iy = 0; iy < n; ++iy)
            for (int ix = 0; ix < n; ++ix) {
                const double kx = wavenumber(ix, n), ky = wavenumber(iy, n), kz = wavenumber(iz, n);
                const long id = ((long)iz * n + iy) * n + ix;
                const int s = (int)floor(sqrt(kx * kx + ky * ky + kz * kz) + 0.5);
                double a = 0.0, b = 0.0;
                for (int i = 0; i < 3; ++i) {
                    a += creal(w.uh[i][id] * conj(w.uh[i][id]));
                    b += creal(Uh[F_BX + i][id] * conj(Uh[F_BX + i][id]));
                }
                if (s < nshell) {
                    eu[s] += 0.5 * a * inv6;
                    eb[s] += 0.5 * b * inv6;
                }
                const cplx d = I * (kx * w.uh[0][id] + ky * w.uh[1][id] + kz * w.uh[2][id]);
                div2 += creal(d * conj(d)) * inv6;
            }
    if (!err) {
        times_ik(&g, w.uh[0], 0, 1.0, w.c1);
        err = inverse(&g, w.c1, w.c0, w.flux);
    }
    if (!err) {
        double* d2 = w.G[0];
        double* d3 = w.G[1];
        for (long q = 0; q < n3; ++q) {
            d2[q] = w.flux[q] * w.flux[q];
            d3[q] = d2[q] * w.flux[q];
        }
        const double m2 = orc_neumaier_sum(d2, n3) / (double)n3, m3 = orc_neumaier_sum(d3, n3) / (double)n3;
        mom[0] = sqrt(div2);
        mom[1] = m2 > 0 ? m3 / pow(m2, 1.5) : 0.0;
        mom[2] = sqrt(m2);
    }
    if (Uh) free_work(&w);
    free_spectra(Uh, 8);
    return err;
}

/* ------------------------------------------------------------------------- */
/* Tracer particles (Section VI): cloud-in-cell interpolation of grid fields  */
/* to particle positions and the Boris push in the magnetic field.            */
/* ------------------------------------------------------------------------- */

/* Grid point j of an axis sits at x_j = 2 pi j / n.  A particle at x lies in
 * the cell with lower corner i = floor(x / dx) (periodic), at fraction
 * f = x / dx - i; each of the eight corners weighs the product over the axes
 * of f (upper corner) or 1 - f (lower corner): the volume of the opposite
 * sub-box, normalised by the cell volume. */
static void cic_setup(int n, double x, int* i0, int* i1, double* f) {
    const double dx = TWO_PI / n;
    double s = x / dx;
    double fl = floor(s);
    *f = s - fl;
    long i = (long)fl % n;
    if (i < 0) i += n;
    *i0 = (int)i;
    *i1 = (int)((i + 1) % n);
}

int orc_cic(int32_t n, const double* f, int32_t nc, const double* pos, int64_t np, double* out) {
    if (n < 1 || !f || nc < 1 || !pos || np < 0 || !out) return -1;
    const long n3 = (long)n * n * n;
    for (int64_t p = 0; p < np; ++p) {
        int ix0, ix1, iy0, iy1, iz0, iz1;
        double fx, fy, fz;
        cic_setup(n, pos[3 * p + 0], &ix0, &ix1, &fx);
        cic_setup(n, pos[3 * p + 1], &iy0, &iy1, &fy);
        cic_setup(n, pos[3 * p + 2], &iz0, &iz1, &fz);
        const int ix[2] = {ix0, ix1}, iy[2] = {iy0, iy1}, iz[2] = {iz0, iz1};
        const double wx[2] = {1.0 - fx, fx}, wy[2] = {1.0 - fy, fy}, wz[2] = {1.0 - fz, fz};
        for (int c = 0; c < nc; ++c) {
            double acc = 0.0;
            for (int a = 0; a < 2; ++a)
                for (int b = 0; b < 2; ++b)
                    for (int d = 0; d < 2; ++d)
                        acc += wz[a] * wy[b] * wx[d] * f[c * n3 + ((long)iz[a] * n + iy[b]) * n + ix[d]];
            out[p * nc + c] = acc;
        }
    }
    return 0;
}

/* Boris push with q = M = 1 (Section VI, Eqs. for t, s, v_d, v and x):
 * t = B dt / 2, s = 2 t / (1 + |t|^2), v' = v + v x t, v+ = v + v' x s,
 * x+ = x + v+ dt, wrapped into [0, 2 pi).  B is interpolated at the particle's
 * position at the start of each step. */
int orc_tracer_push(int32_t n, const double* B, double* pos, double* vel, int64_t np, double dt, int32_t nsteps) {
    if (n < 1 || !B || !pos || !vel || np < 0 || nsteps < 0) return -1;
    for (int s = 0; s < nsteps; ++s) {
        for (int64_t p = 0; p < np; ++p) {
            double Bp[3];
            orc_cic(n, B, 3, pos + 3 * p, 1, Bp);
            double t[3] = {0.5 * dt * Bp[0], 0.5 * dt * Bp[1], 0.5 * dt * Bp[2]};
            const double t2 = t[0] * t[0] + t[1] * t[1] + t[2] * t[2];
            double sv[3] = {2.0 * t[0] / (1.0 + t2), 2.0 * t[1] / (1.0 + t2), 2.0 * t[2] / (1.0 + t2)};
            double* v = vel + 3 * p;
            double vd[3] = {v[0] + (v[1] * t[2] - v[2] * t[1]), v[1] + (v[2] * t[0] - v[0] * t[2]),
                            v[2] + (v[0] * t[1] - v[1] * t[0])};
            double vn[3] = {v[0] + (vd[1] * sv[2] - vd[2] * sv[1]), v[1] + (vd[2] * sv[0] - vd[0] * sv[2]),
                            v[2] + (vd[0] * sv[1] - vd[1] * sv[0])};
            for (int c = 0; c < 3; ++c) {
                v[c] = vn[c];
                double x = pos[3 * p + c] + vn[c] * dt;
                x = fmod(x, TWO_PI);
                if (x < 0) x += TWO_PI;
                pos[3 * p + c] = x;
            }
        }
    }
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Diagnostics (volume means, Neumaier sums).                                 */
/* ------------------------------------------------------------------------- */

double orc_neumaier_sum(const double* x, int64_t n) {
    double s = 0.0, c = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double t = s + x[i];
        if (fabs(s) >= fabs(x[i])) c += (s - t) + x[i];
        else c += (x[i] - t) + s;
        s = t;
    }
    return s + c;
}

static double mean_of(const grid* g, const double* x) {
    return orc_neumaier_sum(x, g->n3) / (double)g->n3;
}

int orc_diag(const orc_params* p, const double* Uin, double* out) {
    grid g;
    if (make_grid(p, &g) || !Uin || !out) return -1;
    const long n3 = g.n3;
    const int n = g.n;
    const double gm1 = g.gamma - 1.0;
    cplx** Uh = alloc_spectra(&g, 8);
    rhs_work w;
    int err = !Uh ? -2 : alloc_work(&g, &w);
    int64_t nonfinite = 0;
    for (long q = 0; q < 8 * n3; ++q) nonfinite += !isfinite(Uin[q]);
    if (!err) err = to_state(&g, Uin, Uh);
    for (int f = 0; f < 8 && !err; ++f) err = inverse(&g, Uh[f], w.c0, w.U[f]);
    if (err) {
        if (Uh) free_work(&w);
        free_spectra(Uh, 8);
        return err;
    }
    double* rho = w.U[0];
    double* m[3] = {w.U[1], w.U[2], w.U[3]};
    double* B[3] = {w.U[4], w.U[5], w.U[6]};
    double* E = w.U[7];
    double* t = w.flux;
    double* P = w.G[0];
    double* Babs = w.G[1];
    double* uabs = w.G[2];

    for (int i = 0; i < 3; ++i)
        for (long q = 0; q < n3; ++q) w.u[i][q] = m[i][q] / rho[q];
    double cmax = 0.0;
    for (long q = 0; q < n3; ++q) {
        double u0 = w.u[0][q], u1 = w.u[1][q], u2 = w.u[2][q];
        double B2 = B[0][q] * B[0][q] + B[1][q] * B[1][q] + B[2][q] * B[2][q];
        double mu = m[0][q] * u0 + m[1][q] * u1 + m[2][q] * u2;
        P[q] = gm1 * (E[q] - 0.5 * mu - 0.5 * B2);
        Babs[q] = sqrt(B2);
        uabs[q] = sqrt(u0 * u0 + u1 * u1 + u2 * u2);
        double umax = fmax(fabs(u0), fmax(fabs(u1), fabs(u2)));
        double cf = sqrt((g.gamma * P[q] + B2) / rho[q]);
        double c = umax + cf;
        if (!(c <= cmax)) cmax = c;  /* NaN propagates */
    }
    out[ORC_MASS] = mean_of(&g, rho);
    for (int i = 0; i < 3; ++i) out[ORC_MOMX + i] = mean_of(&g, m[i]);
    for (long q = 0; q < n3; ++q)
        t[q] = 0.5 * (m[0][q] * w.u[0][q] + m[1][q] * w.u[1][q] + m[2][q] * w.u[2][q]);
    out[ORC_EKIN] = mean_of(&g, t);
    for (long q = 0; q < n3; ++q) t[q] = 0.5 * Babs[q] * Babs[q];
    out[ORC_EMAG] = mean_of(&g, t);
    double Pmean = mean_of(&g, P);
    out[ORC_EINT] = Pmean / gm1;
    out[ORC_ETOT] = mean_of(&g, E);
    for (long q = 0; q < n3; ++q)
        t[q] = w.u[0][q] * B[0][q] + w.u[1][q] * B[1][q] + w.u[2][q] * B[2][q];
    out[ORC_HCROSS] = mean_of(&g, t);

    /* Spectral sums over the full spectrum (Parseval: <f g> = n^-6 sum f^ conj g^). */
    double* hm = w.G[3];
    double* db = w.G[4];
    double* jj = w.G[5];
    {
        const double inv = 1.0 / ((double)n3 * (double)n3);
        long id = 0;
        for (int iz = 0; iz < n; ++iz)
            for (int iy = 0; iy < n; ++iy)
                for (int ix = 0; ix < n; ++ix, ++id) {
                    double kx = wavenumber(ix, n), ky = wavenumber(iy, n), kz = wavenumber(iz, n);
                    double k2 = kx * kx + ky * ky + kz * kz;
                    cplx bx = Uh[4][id], by = Uh[5][id], bz = Uh[6][id];
                    /* J^ = i k x B^, A^ = J^ / |k|^2 (Coulomb gauge, A^(0) = 0) */
                    cplx jx = I * (ky * bz - kz * by);
                    cplx jy = I * (kz * bx - kx * bz);
                    cplx jz = I * (kx * by - ky * bx);
                    cplx dv = I * (kx * bx + ky * by + kz * bz);
                    hm[id] = k2 > 0 ? creal((jx * conj(bx) + jy * conj(by) + jz * conj(bz)) / k2) * inv : 0.0;
                    db[id] = creal(dv * conj(dv)) * inv;
                    jj[id] = creal(jx * conj(jx) + jy * conj(jy) + jz * conj(jz)) * inv;
                }
    }
    out[ORC_HMAG] = orc_neumaier_sum(hm, n3);
    double divb2 = orc_neumaier_sum(db, n3);
    double j2 = orc_neumaier_sum(jj, n3);
    out[ORC_DIVB_RMS] = sqrt(divb2);
    out[ORC_JRMS] = sqrt(j2);
    out[ORC_DIVB_REL] = j2 > 0 ? sqrt(divb2 / j2) : 0.0;
    {
        /* max |div B| in real space */
        for (long q = 0; q < n3; ++q) w.c1[q] = 0;
        for (int j = 0; j < 3; ++j) accum_ik(&g, Uh[4 + j], j, 1.0, w.c1);
        err = inverse(&g, w.c1, w.c0, t);
        double mx = 0.0;
        for (long q = 0; q < n3; ++q) mx = fmax(mx, fabs(t[q]));
        out[ORC_DIVB_MAX] = mx;
    }
    double rho_mean = out[ORC_MASS];
    out[ORC_CS] = sqrt(g.gamma * Pmean / rho_mean);
    double Bmean = mean_of(&g, Babs);
    double umean = mean_of(&g, uabs);
    out[ORC_VA] = Bmean / sqrt(rho_mean);
    out[ORC_MACHS] = umean / out[ORC_CS];
    out[ORC_MACHA] = out[ORC_VA] > 0 ? umean / out[ORC_VA] : INFINITY;
    out[ORC_DTCFL] = g.cfl * (TWO_PI / (double)n) / cmax;
    out[ORC_NONFINITE] = (double)nonfinite;

    free_work(&w);
    free_spectra(Uh, 8);
    return err;
}

int32_t orc_num_threads(void) {
#ifdef _OPENMP
    return (int32_t)omp_get_max_threads();
#else
    return 1;
#endif
}

void orc_set_num_threads(int32_t threads) {
#ifdef _OPENMP
    if (threads > 0) omp_set_num_threads(threads);
#else
    (void)threads;
#endif
}

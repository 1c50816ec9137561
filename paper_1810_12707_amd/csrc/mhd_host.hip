// libmhd host side: the C-ABI of include/mhd.h, workspace carving, twiddle
// tables, the pass pipelines of the right-hand side and the FP64 reductions.
//
// One right-hand-side evaluation (Eqs. MHD1-MHD4) runs as two phases:
//   A: rho^, m^ --inverse z, y--> x-pass (u = m/rho, forward x) --forward y, z--> u^ = D F[u]
//   B: B^, E^, u^ --inverse z with the spectral multipliers for S and J = curl B--> inverse y
//      --> x-pass (all fluxes at every grid point) --> forward y
//      --> forward z with divergence / curl, resistive term and the AB2 update.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <type_traits>
#include <string>
#include <vector>

#include "../../include/mhd.h"
#include "mhd_internal.h"
#include "mhd_registry.h"

namespace mhd {

Registry& registry() {
  static Registry* r = [] {
    Registry* reg = new Registry();
#define MHD_CALL_REGISTER(NN) register_##NN(*reg);
    MHD_SIZES(MHD_CALL_REGISTER)
#undef MHD_CALL_REGISTER
#define MHD_CALL_REGISTER_S1(NN) register_s1_##NN(*reg);
    MHD_SCHED1_SIZES(MHD_CALL_REGISTER_S1)
#undef MHD_CALL_REGISTER_S1
    return reg;
  }();
  return *r;
}

// ------------------------------------------------------------------ reductions

// One launch for both record sets of the diagnostics.  Block q reduces
// column q of p1[n1][nq1] into out1[q] for q < nq1, else column q - nq1 of
// p2[n2][nq2] into out2[q - nq1].  Thread t takes records t, t + 256, ... with
// a Neumaier sum (or a NaN-propagating max when bit q of max_mask is set; the
// mask applies to the first set), and the 256 (sum, compensation) pairs are
// combined pairwise in a fixed tree.  Deterministic for given record counts.
__device__ __forceinline__ void two_sum_into(double& s, double& c, double x) {
  const double t = s + x;
  if (fabs(s) >= fabs(x)) c += (s - t) + x;
  else c += (x - t) + s;
  s = t;
}

__global__ void __launch_bounds__(kThreads)
k_reduce(const double* __restrict__ p1, int64_t n1, int nq1, unsigned max_mask, const double* __restrict__ p2,
         int64_t n2, int nq2, double* __restrict__ out1, double* __restrict__ out2) {
  __shared__ double s_s[kThreads];
  __shared__ double s_c[kThreads];
  const bool first = (int)blockIdx.x < nq1;
  const int q = first ? (int)blockIdx.x : (int)blockIdx.x - nq1;
  const double* part = first ? p1 : p2;
  const int64_t nrec = first ? n1 : n2;
  const int nq = first ? nq1 : nq2;
  const int tid = threadIdx.x;
  const bool is_max = first && ((max_mask >> q) & 1u);
  double s = 0.0, c = 0.0;
  for (int64_t r = tid; r < nrec; r += kThreads) {
    const double x = part[r * nq + q];
    if (is_max) {
      if (!(x <= s)) s = x;
    } else {
      two_sum_into(s, c, x);
    }
  }
  s_s[tid] = s;
  s_c[tid] = c;
  __syncthreads();
  for (int w = kThreads / 2; w > 0; w >>= 1) {
    if (tid < w) {
      if (is_max) {
        if (!(s_s[tid + w] <= s_s[tid])) s_s[tid] = s_s[tid + w];
      } else {
        double a = s_s[tid], ca = s_c[tid] + s_c[tid + w];
        two_sum_into(a, ca, s_s[tid + w]);
        s_s[tid] = a;
        s_c[tid] = ca;
      }
    }
    __syncthreads();
  }
  if (tid == 0) {
    const double r = is_max ? s_s[0] : s_s[0] + s_c[0];
    (first ? out1 : out2)[q] = r;
  }
}

// Spectral sums over the compact B^ (half spectrum: kx > 0 modes count twice):
// sum Re(J^ . conj B^)/|k|^2, sum |i k.B^|^2, sum |J^|^2 with J^ = i k x B^.
// Eq. MHD1 in spectral form, R_rho = -i k . m^, with the density's AB2
// update U_rho += dt (a_cur R + a_prev R_prev), R_prev <- R, or the store of
// R into rout.  One thread per compact entry (padding skipped) of member
// blockIdx.y.  Launched before the forward-z pass that forms the other seven
// right-hand sides, since that pass overwrites m^ with its next time level.
template <typename T>
__global__ void __launch_bounds__(kThreads) k_rho_rhs(const RhsArgs<T> a) {
  using V2 = typename std::conditional<sizeof(T) == 4, float2, double2>::type;
  const Geo& g = a.g;
  const int mem = blockIdx.y;
  const int64_t idx = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  const int64_t plane = (int64_t)g.nb * g.nhp;
  const int lz = (int)(idx / plane);
  const int rem = (int)(idx - (int64_t)lz * plane);
  const int ly = rem / g.nhp, kx = rem - ly * g.nhp;
  if (idx >= g.sc || kx >= g.nh) return;
  const int kz = lz <= g.K ? lz : lz - g.nb;
  const int ky = ly <= g.K ? ly : ly - g.nb;
  const int64_t ms = a.bt.mstride;
  V2* const state = reinterpret_cast<V2*>(member_ptr(a.state, mem, ms));
  const V2 mx = state[g.sc + idx], my = state[2 * g.sc + idx], mz = state[3 * g.sc + idx];
  const T dx = T(kx) * mx.x + T(ky) * my.x + T(kz) * mz.x;
  const T dy = T(kx) * mx.y + T(ky) * my.y + T(kz) * mz.y;
  V2 R;
  R.x = a.kinematic ? T(0) : dy;  // -i (dx + i dy); zero with the density frozen
  R.y = a.kinematic ? T(0) : -dx;
  if (a.rout) {
    reinterpret_cast<V2*>(member_ptr(a.rout, mem, ms))[idx] = R;
    return;
  }
  V2* const rprev = reinterpret_cast<V2*>(member_ptr(a.rprev, mem, ms));
  const T dt = T(a.dt[mem]), ac = T(a.a_cur[mem]), ap = T(a.a_prev[mem]);
  T ir = R.x * ac, ii = R.y * ac;
  if (a.a_prev[mem] != 0.0) {
    const V2 p = rprev[idx];
    ir += p.x * ap;
    ii += p.y * ap;
  }
  V2 u = state[idx];
  u.x += dt * ir;
  u.y += dt * ii;
  state[idx] = u;
  rprev[idx] = R;
}

// ABC body force of Section V-B in spectral form.  With f = F0 (sin z + cos y,
// sin x + cos z, sin y + cos x), the product of a band-limited field g with
// one term is a shift of its spectrum: F[g sin z](k) = (g^(k - e_z) -
// g^(k + e_z)) / 2i, F[g cos y](k) = (g^(k - e_y) + g^(k + e_y)) / 2.  The
// products have modes up to K + 1 < n/2, so this is exactly the dealiased
// pseudo-spectral product D F[g f].  Writes force [4][sc]: D F[rho f_x],
// D F[rho f_y], D F[rho f_z] and the work D F[m.f].  One thread per compact
// entry; kx < 0 neighbours come from Hermitian symmetry, out-of-band ones are
// zero.  Reads the state before anything of this step overwrites it.
template <typename T>
__global__ void __launch_bounds__(kThreads) k_force_abc(const T* __restrict__ state, T* __restrict__ force, Geo g,
                                                       double f0) {
  using V2 = typename std::conditional<sizeof(T) == 4, float2, double2>::type;
  const int64_t idx = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  const int64_t plane = (int64_t)g.nb * g.nhp;
  const int lz = (int)(idx / plane);
  const int rem = (int)(idx - (int64_t)lz * plane);
  const int ly = rem / g.nhp, kx = rem - ly * g.nhp;
  if (idx >= g.sc || kx >= g.nh) return;
  const int kz = lz <= g.K ? lz : lz - g.nb;
  const int ky = ly <= g.K ? ly : ly - g.nb;
  const V2* S = reinterpret_cast<const V2*>(state);
  // spectrum of state field fld at (qx, qy, qz), any signs
  auto at = [&](int fld, int qx, int qy, int qz) -> V2 {
    V2 z;
    z.x = T(0);
    z.y = T(0);
    bool conj = false;
    if (qx < 0) {
      qx = -qx;
      qy = -qy;
      qz = -qz;
      conj = true;
    }
    if (qx > g.K || qy > g.K || qy < -g.K || qz > g.K || qz < -g.K) return z;
    const int by = qy >= 0 ? qy : qy + g.nb, bz = qz >= 0 ? qz : qz + g.nb;
    z = S[fld * g.sc + ((int64_t)bz * g.nb + by) * g.nhp + qx];
    if (conj) z.y = -z.y;
    return z;
  };
  // (g^(k - e) - g^(k + e)) / 2i and (g^(k - e) + g^(k + e)) / 2 along axis e
  auto sin_term = [&](int fld, int ax) -> V2 {
    const int dx = ax == 0, dy = ax == 1, dz = ax == 2;
    const V2 m = at(fld, kx - dx, ky - dy, kz - dz), p = at(fld, kx + dx, ky + dy, kz + dz);
    V2 r;
    r.x = T(0.5) * (m.y - p.y);  // (a) / 2i = -i a / 2
    r.y = T(-0.5) * (m.x - p.x);
    return r;
  };
  auto cos_term = [&](int fld, int ax) -> V2 {
    const int dx = ax == 0, dy = ax == 1, dz = ax == 2;
    const V2 m = at(fld, kx - dx, ky - dy, kz - dz), p = at(fld, kx + dx, ky + dy, kz + dz);
    V2 r;
    r.x = T(0.5) * (m.x + p.x);
    r.y = T(0.5) * (m.y + p.y);
    return r;
  };
  // f_x = sin z + cos y, f_y = sin x + cos z, f_z = sin y + cos x
  const int s_ax[3] = {2, 0, 1}, c_ax[3] = {1, 2, 0};
  V2* F = reinterpret_cast<V2*>(force);
  V2 work;
  work.x = T(0);
  work.y = T(0);
  const T a = T(f0);
  for (int c = 0; c < 3; ++c) {
    const V2 s1 = sin_term(0, s_ax[c]), c1 = cos_term(0, c_ax[c]);
    V2 v;
    v.x = a * (s1.x + c1.x);
    v.y = a * (s1.y + c1.y);
    F[c * g.sc + idx] = v;
    const V2 s2 = sin_term(1 + c, s_ax[c]), c2 = cos_term(1 + c, c_ax[c]);
    work.x += a * (s2.x + c2.x);
    work.y += a * (s2.y + c2.y);
  }
  F[3 * g.sc + idx] = work;
}

// Stage arithmetic of the Runge-Kutta and predictor-corrector schemes over the
// eight compact fields (one thread per entry, padding skipped):
//   CB_RK_FIRST:  acc = R;          us = u + c R
//   CB_RK_MID:    acc += w R;       us = u + c R
//   CB_RK_LAST:   u += c (acc + R)
//   CB_PC_PRED:   us = u + dt (a_cur R + a_prev acc); acc = R   (acc = history)
//   CB_PC_CORR:   u += c (acc + R)                              (acc = R^n)
enum { CB_RK_FIRST = 0, CB_RK_MID, CB_RK_LAST, CB_PC_PRED, CB_PC_CORR };
template <typename T>
__global__ void __launch_bounds__(kThreads) k_combine(T* __restrict__ u, const T* __restrict__ R,
                                                     T* __restrict__ acc, T* __restrict__ us, Geo g, int op,
                                                     double c, double w, double a_cur, double a_prev) {
  const int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x;  // entry of the 8 fields
  if (e >= 8 * g.sc) return;
  const int64_t idx = e % g.sc;
  if (idx % g.nhp >= g.nh) return;  // kx padding: never read or written
  const int64_t j = 2 * e;
  for (int h = 0; h < 2; ++h) {
    const T r = R[j + h];
    switch (op) {
      case CB_RK_FIRST: acc[j + h] = r; us[j + h] = u[j + h] + T(c) * r; break;
      case CB_RK_MID: acc[j + h] += T(w) * r; us[j + h] = u[j + h] + T(c) * r; break;
      case CB_PC_PRED: {
        // the Euler start (a_prev = 0) never reads the history, which may not exist yet
        const T hist = a_prev != 0.0 ? T(a_prev) * acc[j + h] : T(0);
        us[j + h] = u[j + h] + T(c) * (T(a_cur) * r + hist);
        acc[j + h] = r;
        break;
      }
      default: u[j + h] += T(c) * (acc[j + h] + r); break;  // CB_RK_LAST, CB_PC_CORR
    }
  }
}

// ------------------------------------------------------------------ tracers
// Tracer particles of Section VI.  Positions and velocities are FP64 device
// arrays [np][3] (x, y, z); the grid fields are real-space fields in the
// working precision, [nf][n^3] with x fastest; interpolation and push are FP64.
//
// Cloud-in-cell: a particle at x lies in the cell whose lower corner is grid
// point i = floor(x / dx) (periodic, dx = 2 pi / n), at fraction f = x/dx - i
// of the cell; corner i weighs 1 - f and corner i + 1 weighs f per axis, and a
// corner's weight is the product over the axes: the volume of the opposite
// sub-box over the cell volume (trilinear interpolation).
struct CicAxis {
  int i0, i1;
  double w0, w1;
};
__device__ __forceinline__ CicAxis cic_axis(int n, double x) {
  const double dx = 6.28318530717958647692528676655900577 / n;
  const double s = x / dx;
  const double fl = floor(s);
  long long i = (long long)fl % n;
  if (i < 0) i += n;
  CicAxis a;
  a.i0 = (int)i;
  a.i1 = (int)((i + 1) % n);
  a.w1 = s - fl;
  a.w0 = 1.0 - a.w1;
  return a;
}

// Interpolated value of `nc` fields (field c at base + c * n^3) at p; the
// callback receives the eight corner indices and weights.
template <typename F>
__device__ __forceinline__ void cic_corners(int n, const double* p, F&& visit) {
  const CicAxis ax = cic_axis(n, p[0]), ay = cic_axis(n, p[1]), az = cic_axis(n, p[2]);
  const int xi[2] = {ax.i0, ax.i1}, yi[2] = {ay.i0, ay.i1}, zi[2] = {az.i0, az.i1};
  const double xw[2] = {ax.w0, ax.w1}, yw[2] = {ay.w0, ay.w1}, zw[2] = {az.w0, az.w1};
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int d = 0; d < 2; ++d)
        visit(((int64_t)zi[a] * n + yi[b]) * n + xi[d], zw[a] * yw[b] * xw[d]);
}

// Initial tracer velocity: the grid velocity u = m / rho (at the grid points,
// from the real-space rho and m: fields 0..3 of `f`) interpolated by CIC.
template <typename T>
__global__ void __launch_bounds__(kThreads) k_tracer_velocity(const T* __restrict__ f, int n,
                                                             const double* __restrict__ pos, double* __restrict__ vel,
                                                             int64_t np) {
  const int64_t p = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (p >= np) return;
  const int64_t n3 = (int64_t)n * n * n;
  double acc[3] = {0.0, 0.0, 0.0};
  cic_corners(n, pos + 3 * p, [&](int64_t g, double w) {
    const double rho = double(f[g]);
#pragma unroll
    for (int c = 0; c < 3; ++c) acc[c] += w * (double(f[(1 + c) * n3 + g]) / rho);
  });
#pragma unroll
  for (int c = 0; c < 3; ++c) vel[3 * p + c] = acc[c];
}

// nsteps Boris steps (q = M = 1) in the magnetic field B (fields 0..2 of `b`):
// t = B dt / 2, s = 2 t / (1 + |t|^2), v' = v + v x t, v <- v + v' x s,
// x <- x + v dt wrapped into [0, 2 pi); B is interpolated at each step's
// start position.  One thread per particle.
template <typename T>
__global__ void __launch_bounds__(kThreads) k_tracer_push(const T* __restrict__ b, int n, double* __restrict__ pos,
                                                         double* __restrict__ vel, int64_t np, double dt,
                                                         int nsteps) {
  const int64_t p = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (p >= np) return;
  const double two_pi = 6.28318530717958647692528676655900577;
  const int64_t n3 = (int64_t)n * n * n;
  double x[3] = {pos[3 * p], pos[3 * p + 1], pos[3 * p + 2]};
  double v[3] = {vel[3 * p], vel[3 * p + 1], vel[3 * p + 2]};
  for (int s = 0; s < nsteps; ++s) {
    double B[3] = {0.0, 0.0, 0.0};
    cic_corners(n, x, [&](int64_t g, double w) {
#pragma unroll
      for (int c = 0; c < 3; ++c) B[c] += w * double(b[c * n3 + g]);
    });
    const double t[3] = {0.5 * dt * B[0], 0.5 * dt * B[1], 0.5 * dt * B[2]};
    const double t2 = t[0] * t[0] + t[1] * t[1] + t[2] * t[2];
    const double sv[3] = {2.0 * t[0] / (1.0 + t2), 2.0 * t[1] / (1.0 + t2), 2.0 * t[2] / (1.0 + t2)};
    const double vd[3] = {v[0] + (v[1] * t[2] - v[2] * t[1]), v[1] + (v[2] * t[0] - v[0] * t[2]),
                          v[2] + (v[0] * t[1] - v[1] * t[0])};
    const double vn[3] = {v[0] + (vd[1] * sv[2] - vd[2] * sv[1]), v[1] + (vd[2] * sv[0] - vd[0] * sv[2]),
                          v[2] + (vd[0] * sv[1] - vd[1] * sv[0])};
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      v[c] = vn[c];
      double xc = fmod(x[c] + vn[c] * dt, two_pi);
      if (xc < 0) xc += two_pi;
      x[c] = xc;
    }
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    pos[3 * p + c] = x[c];
    vel[3 * p + c] = v[c];
  }
}

// ------------------------------------------------------------------ spectra
// Turbulence diagnostics of Section V over the compact spectra.  Shell s holds
// the modes with floor(|k| + 1/2) = s.  Block b takes entries b, b + G, ...
// (padding skipped); a kx > 0 entry stands for itself and its conjugate (x2).
// Per block: raw shell sums sum |u^|^2 and sum |B^|^2 and sum |k.u^|^2 in LDS
// (FP64 LDS atomics: the order of additions inside a block is not fixed, so
// a block's sums are reproducible to FP64 rounding), written to
// part[b][2 nsh + 1] and reduced over blocks by k_reduce.
constexpr int kSpecBlocks = 256;
template <typename T>
__global__ void __launch_bounds__(kThreads) k_spectra(const T* __restrict__ uh, const T* __restrict__ bh, Geo g,
                                                     int nsh, double* __restrict__ part) {
  extern __shared__ double bins[];  // 2 nsh + 1
  const int nb = 2 * nsh + 1;
  for (int i = threadIdx.x; i < nb; i += kThreads) bins[i] = 0.0;
  __syncthreads();
  const int64_t plane = (int64_t)g.nb * g.nhp;
  for (int64_t idx = (int64_t)blockIdx.x * kThreads + threadIdx.x; idx < g.sc;
       idx += (int64_t)gridDim.x * kThreads) {
    const int lz = (int)(idx / plane);
    const int rem = (int)(idx - (int64_t)lz * plane);
    const int ly = rem / g.nhp, kx = rem - ly * g.nhp;
    if (kx >= g.nh) continue;
    const int kz = lz <= g.K ? lz : lz - g.nb;
    const int ky = ly <= g.K ? ly : ly - g.nb;
    const double w = kx == 0 ? 1.0 : 2.0;
    const double k2 = double(kx) * kx + double(ky) * ky + double(kz) * kz;
    const int s = (int)floor(sqrt(k2) + 0.5);
    double a = 0.0, b = 0.0, dr = 0.0, di = 0.0;
    const double kv[3] = {double(kx), double(ky), double(kz)};
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const double ur = uh[2 * (i * g.sc + idx)], ui = uh[2 * (i * g.sc + idx) + 1];
      const double br = bh[2 * (i * g.sc + idx)], bi = bh[2 * (i * g.sc + idx) + 1];
      a += ur * ur + ui * ui;
      b += br * br + bi * bi;
      dr += kv[i] * ur;
      di += kv[i] * ui;
    }
    if (s < nsh) {
      atomicAdd(&bins[s], w * a);
      atomicAdd(&bins[nsh + s], w * b);
    }
    atomicAdd(&bins[2 * nsh], w * (dr * dr + di * di));
  }
  __syncthreads();
  for (int i = threadIdx.x; i < nb; i += kThreads) part[(int64_t)blockIdx.x * nb + i] = bins[i];
}

// Per-thread Neumaier sums of d^2 and d^3 over a real field d[n3] (grid-stride);
// thread t of block b writes its compensated pair sums to part[(b T + t)][2].
template <typename T>
__global__ void __launch_bounds__(kThreads) k_moments(const T* __restrict__ d, int64_t n3, double* __restrict__ part) {
  double s2 = 0.0, c2 = 0.0, s3 = 0.0, c3 = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n3; i += (int64_t)gridDim.x * kThreads) {
    const double v = double(d[i]);
    two_sum_into(s2, c2, v * v);
    two_sum_into(s3, c3, v * v * v);
  }
  const int64_t r = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  part[2 * r] = s2 + c2;
  part[2 * r + 1] = s3 + c3;
}

template <typename T>
__global__ void __launch_bounds__(kThreads)
k_spec_diag(const T* __restrict__ bx, const T* __restrict__ by, const T* __restrict__ bz, Geo g,
            double* __restrict__ part) {
  __shared__ double s[kThreads];
  const int tid = threadIdx.x;
  const int64_t idx = (int64_t)blockIdx.x * kThreads + tid;
  double q[kSpecQ] = {0.0, 0.0, 0.0};
  const int64_t plane = (int64_t)g.nb * g.nhp;
  const int lz = (int)(idx / plane);
  const int rem = (int)(idx - (int64_t)lz * plane);
  const int ly = rem / g.nhp, kx = rem - ly * g.nhp;
  if (idx < g.sc && kx < g.nh) {  // padding columns hold no data and are not read
    const int kz = lz <= g.K ? lz : lz - g.nb;
    const int ky = ly <= g.K ? ly : ly - g.nb;
    const double w = kx == 0 ? 1.0 : 2.0;
    const double Xr = bx[2 * idx], Xi = bx[2 * idx + 1];
    const double Yr = by[2 * idx], Yi = by[2 * idx + 1];
    const double Zr = bz[2 * idx], Zi = bz[2 * idx + 1];
    // c = k x B (real cross product of k with re and im parts); J^ = i c
    const double cxr = ky * Zr - kz * Yr, cxi = ky * Zi - kz * Yi;
    const double cyr = kz * Xr - kx * Zr, cyi = kz * Xi - kx * Zi;
    const double czr = kx * Yr - ky * Xr, czi = kx * Yi - ky * Xi;
    const double k2 = double(kx) * kx + double(ky) * ky + double(kz) * kz;
    // Re(i c . conj B) = -(Im c . Re B) + (Re c . Im B)
    const double jb = -(cxi * Xr + cyi * Yr + czi * Zr) + (cxr * Xi + cyr * Yi + czr * Zi);
    q[SQ_HM] = k2 > 0 ? w * jb / k2 : 0.0;
    const double dr = kx * Xr + ky * Yr + kz * Zr, di = kx * Xi + ky * Yi + kz * Zi;
    q[SQ_DIVB2] = w * (dr * dr + di * di);
    q[SQ_J2] = w * (cxr * cxr + cxi * cxi + cyr * cyr + cyi * cyi + czr * czr + czi * czi);
  }
  for (int i = 0; i < kSpecQ; ++i) {
    __syncthreads();
    s[tid] = q[i];
    __syncthreads();
    for (int w = kThreads / 2; w > 0; w >>= 1) {
      if (tid < w) s[tid] += s[tid + w];
      __syncthreads();
    }
    if (tid == 0) part[(int64_t)blockIdx.x * kSpecQ + i] = s[0];
  }
}

// Streaming copy of n 16-byte words (the benchmark's practical HBM
// ceiling): one 16-byte load and store per thread and iteration of a
// grid-stride loop over four resident workgroups per CU.  Measured on 1 GiB
// against unrolled (four and eight loads in flight), nontemporal and
// contiguous-chunk variants and more workgroups per CU, this plain form was
// the fastest (5.66 TB/s read + write; hipMemcpy 5.08).
__global__ void __launch_bounds__(kThreads) k_stream_copy(const uint4* __restrict__ src, uint4* __restrict__ dst,
                                                         int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * kThreads;
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += stride) dst[i] = src[i];
}

__global__ void k_fill_u32(unsigned* p, int n, unsigned v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// Checkpoint blob header (256 bytes at the start of the blob).
struct CkptHeader {
  char magic[8];           // "MHDCKPT"
  uint32_t version;        // kCkptVersion
  int32_t n, precision;    // grid and working precision of the saving context
  int32_t first_step;      // 1: the next step is the Euler start (no history yet)
  int64_t step;            // steps since the state was set
  double t, dt;            // simulated time; the fixed step of the AB2 history
  uint64_t payload_bytes;  // bytes after the header
  uint64_t sc;             // complex values per compact spectrum
  uint64_t pad[23];
  uint64_t checksum;       // hash of every other word of the blob
};
static_assert(sizeof(CkptHeader) == 256, "checkpoint header is 256 bytes");
constexpr uint32_t kCkptVersion = 1;
constexpr int kCkptSumWord = 31;  // index of `checksum` among the header's 64-bit words

// Writes the header (passed by value, so the launch captures it) to dst.
__global__ void k_write_header(CkptHeader h, CkptHeader* dst) {
  const uint64_t* src = reinterpret_cast<const uint64_t*>(&h);
  uint64_t* d = reinterpret_cast<uint64_t*>(dst);
  const int i = threadIdx.x;
  if (i < 32) d[i] = i == kCkptSumWord ? 0ull : src[i];
}

// Order-independent 64-bit hash of words[0..nwords) with word `skip` taken as
// zero: the sum (mod 2^64) of the SplitMix64 finaliser applied to each word
// offset by its index, so a changed word or two swapped words change it.
// Block sums are added into *out with one atomic per block (addition mod 2^64
// commutes, so the result does not depend on block order).
__device__ __forceinline__ uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
__global__ void __launch_bounds__(kThreads)
k_blob_hash(const uint64_t* __restrict__ words, int64_t nwords, int64_t skip, unsigned long long* out) {
  __shared__ uint64_t s[kThreads];
  uint64_t acc = 0;
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < nwords; i += (int64_t)gridDim.x * kThreads) {
    const uint64_t w = i == skip ? 0ull : words[i];
    acc += mix64(w + (uint64_t)(i + 1) * 0x9E3779B97F4A7C15ull);
  }
  s[threadIdx.x] = acc;
  __syncthreads();
  for (int w = kThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicAdd(out, (unsigned long long)s[0]);
}

}  // namespace mhd

using namespace mhd;

// ------------------------------------------------------------------ context

namespace {

constexpr int kResWords = 32;    // reduced diagnostics: [0, kDiagQ) real-space, [16, 16 + kSpecQ) spectral,
                                 // [24] max signal speed seen by steps, [25] their non-finite count
constexpr int kResStatus = 24;

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

bool size_ok(int32_t n, int32_t prec) {
  if (n < 8 || n > 1024) return false;
  bool listed = false;
#define MHD_LISTED(NN) listed = listed || (n == NN);
  MHD_SIZES(MHD_LISTED)
#undef MHD_LISTED
  if (!listed) return false;
  if (prec == MHD_FP64 && n > 512) return false;
  return prec == MHD_FP64 || prec == MHD_FP32 || prec == MHD_MIXED;
}

Geo make_geo(int n) {
  Geo g;
  g.n = n;
  g.K = (n - 1) / 3;
  g.nh = g.K + 1;
  g.nb = 2 * g.K + 1;
  g.nhp = (g.nh + 7) / 8 * 8;
  g.sc = (int64_t)g.nb * g.nb * g.nhp;
  g.iz = (int64_t)n * g.nb * g.nhp;
  g.iy = (int64_t)n * n * g.nhp;
  g.n3 = (int64_t)n * n * n;
  return g;
}

// Shells of the retained modes: floor(|k| + 1/2) <= floor(sqrt(3) K + 1/2).
int spectrum_shells(int K) { return (int)std::floor(std::sqrt(3.0) * K + 0.5) + 1; }

struct Layout {
  size_t tw, state, rprev, uhat, tstate, trhs, force, iz, iy, part, spart, status, res, hash, shpart, shres, total;
};

Layout make_layout(const Geo& g, size_t tsize) {
  Layout L;
  size_t off = 0;
  auto take = [&](size_t bytes) { size_t o = off; off += align256(bytes); return o; };
  const size_t cplx = 2 * tsize;
  L.tw = take((size_t)g.n * cplx);
  L.state = take(8 * (size_t)g.sc * cplx);
  L.rprev = take(8 * (size_t)g.sc * cplx);
  L.uhat = take(4 * (size_t)g.sc * cplx);
  L.tstate = take(8 * (size_t)g.sc * cplx);
  L.trhs = take(8 * (size_t)g.sc * cplx);
  L.force = take(4 * (size_t)g.sc * cplx);
  L.iz = take(12 * (size_t)g.iz * cplx);
  L.iy = take(16 * (size_t)g.iy * cplx);
  const size_t rows = (size_t)g.n * g.n / 2;
  const size_t spec_blocks = (size_t)((g.sc + kThreads - 1) / kThreads);
  L.part = take(rows * kDiagQ * sizeof(double));
  L.spart = take(spec_blocks * kSpecQ * sizeof(double));
  L.status = take((size_t)kStatusSlots * 2 * sizeof(double));
  L.res = take(kResWords * sizeof(double));
  L.hash = take(sizeof(uint64_t));
  const size_t nbins = 2 * (size_t)spectrum_shells(g.K) + 1;
  L.shpart = take(std::max(nbins * kSpecBlocks, (size_t)2 * kSpecBlocks * kThreads) * sizeof(double));
  L.shres = take((nbins + 2) * sizeof(double));
  L.total = off;
  return L;
}

}  // namespace

struct mhd_ctx {
  mhd_params p;
  Geo g;
  Layout L;
  hipStream_t stream;
  char* ws;
  size_t ws_bytes;
  bool has_state;
  bool first_step;
  int64_t step;
  double t;
  int num_cus = 0;
  int row_blocks[5] = {0, 0, 0, 0, 0};  // resident workgroups of each row-pass mode
  int col_blocks[3] = {0, 0, 0};        // column passes: forward, inverse (1 term), inverse (3 terms)
  std::string last_err;
  // benchmark timing (mhd_profile)
  bool prof_on = false;
  uint32_t prof_mask = 0;     // launch classes bracketed with events (bit cls)
  std::vector<hipEvent_t> ev;  // 2 per recorded launch
  std::vector<int> rec_cls;
  std::vector<double> rec_bytes;
  int nrec = 0;
  int64_t dropped = 0;
  // the steady AB2 step as a HIP graph (captured at the first graph step)
  hipStream_t cap = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace {

int hip_fail(mhd_ctx* c, hipError_t e, const char* what) {
  if (c) {
    c->last_err = std::string(what) + ": " + hipGetErrorString(e);
  }
  return MHD_E_HIP;
}

int check_launch(mhd_ctx* c, const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(c, e, what);
  return MHD_OK;
}

Term term(int src, int axis, double coef) {
  Term t;
  t.src = src;
  t.axis = axis;
  t.coef = coef;
  return t;
}

OutSpec spec(std::initializer_list<Term> ts) {
  OutSpec s;
  std::memset(&s, 0, sizeof(s));
  s.nterms = 0;
  for (const Term& t : ts) s.t[s.nterms++] = t;
  return s;
}

OutSpec copy_spec(int src, double coef) { return spec({term(src, -1, coef)}); }

// The members one engine runs per launch: member 0 is the engine's context,
// member m sits at byte offset m * stride; per-member physical parameters,
// AB2 coefficients of the current step, and the launch-geometry scales picked
// by the ensemble autotuner.
struct MemberSet {
  int n = 1;
  int64_t stride = 0;
  double gamma[kMaxMem], nu[kMaxMem], eta[kMaxMem], dt[kMaxMem];
  double a_cur[kMaxMem], a_prev[kMaxMem];
  double col_scale = 1.0, row_scale = 1.0;
};

MemberSet single_member(const mhd_ctx* c) {
  MemberSet m;
  m.gamma[0] = c->p.gamma;
  m.nu[0] = c->p.nu;
  m.eta[0] = c->p.eta;
  m.dt[0] = c->p.dt;
  m.a_cur[0] = 1.0;
  m.a_prev[0] = 0.0;
  return m;
}

template <typename T>
struct Engine {
  mhd_ctx* c;
  const Kern<T>& k;
  const Geo& g;
  MemberSet ms;

  Engine(mhd_ctx* ctx, const Kern<T>& kern) : c(ctx), k(kern), g(ctx->g), ms(single_member(ctx)) {}
  Engine(mhd_ctx* ctx, const Kern<T>& kern, const MemberSet& m) : c(ctx), k(kern), g(ctx->g), ms(m) {}

  T* at(size_t off) const { return reinterpret_cast<T*>(c->ws + off); }
  T* state() const { return at(c->L.state); }
  T* rprev() const { return at(c->L.rprev); }
  T* uhat() const { return at(c->L.uhat); }
  T* tstate() const { return at(c->L.tstate); }
  T* trhs() const { return at(c->L.trhs); }
  T* force() const { return at(c->L.force); }
  T* tw() const { return at(c->L.tw); }
  T* iz(int slot) const { return at(c->L.iz) + 2 * (size_t)slot * g.iz; }
  T* iy(int slot) const { return at(c->L.iy) + 2 * (size_t)slot * g.iy; }
  T* spec_field(T* base, int f) const { return base + 2 * (size_t)f * g.sc; }
  double* part() const { return reinterpret_cast<double*>(c->ws + c->L.part); }
  double* spart() const { return reinterpret_cast<double*>(c->ws + c->L.spart); }
  double* status() const { return reinterpret_cast<double*>(c->ws + c->L.status); }
  double* res() const { return reinterpret_cast<double*>(c->ws + c->L.res); }

  // Algorithmic HBM bytes of one launch: each array read or written once,
  // counting data entries only (the kx padding is never touched).
  double cbytes(double n_sc, double n_iz, double n_iy) const {
    const double nb = g.nb, nh = g.nh, n = g.n;
    return (n_sc * nb * nb * nh + n_iz * n * nb * nh + n_iy * n * n * nh) * 2.0 * sizeof(T);
  }
  double class_bytes(int cls) const {
    const double a4 = (c->p.flags & MHD_FLAG_VISC_LAPLACIAN) ? 1 : 0;  // q = |u|^2/2 beside u
    const double fo = c->p.force != 0.0 ? 4 : 0;                       // body-force spectra
    switch (cls) {
      case MHD_PASS_ZINV_A: return cbytes(4, 4, 0);
      case MHD_PASS_YINV_A: return cbytes(0, 4, 4);
      case MHD_PASS_XA: return cbytes(0, 0, 7 + a4);
      case MHD_PASS_YFWD_A: return cbytes(0, 3 + a4, 3 + a4);
      case MHD_PASS_ZFWD_A: return cbytes(3 + a4, 3 + a4, 0);
      case MHD_PASS_ZINV_B: return cbytes(7, 12, 0);
      case MHD_PASS_YINV_B: return cbytes(0, 12, 12);
      case MHD_PASS_XB: return cbytes(0, 0, 28);
      case MHD_PASS_YFWD_B: return cbytes(0, 12, 12);
      case MHD_PASS_ZRHS: return cbytes(28 + 4 * a4 + fo, 12, 0);
      case MHD_PASS_RHO: return cbytes(7 + 2 * fo, 0, 0);
      case MHD_PASS_REDUCE: return 0.0;
      default: return 0.0;
    }
  }

  // Runs `launch`; while profiling, brackets it with a pair of events.
  template <typename F>
  void timed(int cls, F&& launch) {
    const bool want = c->prof_on && ((c->prof_mask >> cls) & 1u);
    if (want && c->nrec < (int)c->rec_cls.size()) {
      const int r = c->nrec++;
      (void)hipEventRecord(c->ev[2 * r], c->stream);
      launch();
      (void)hipEventRecord(c->ev[2 * r + 1], c->stream);
      c->rec_cls[r] = cls;
      c->rec_bytes[r] = class_bytes(cls);
    } else {
      if (want) ++c->dropped;
      launch();
    }
  }

  int ztiles() const { return (int)(((int64_t)g.nb * g.nhp + k.col_width - 1) / k.col_width); }
  int rtiles() const { return (int)(((int64_t)g.nb * g.nhp + k.rhs_width - 1) / k.rhs_width); }
  int ytiles() const { return (g.nh + k.col_width - 1) / k.col_width; }

  Batch batch() const {
    Batch b;
    b.nmem = ms.n;
    b.pad = 0;
    b.mstride = ms.stride;
    return b;
  }

  ColArgs<T> col_args(int kind, int nout) const {
    ColArgs<T> a;
    std::memset(&a, 0, sizeof(a));
    a.kind = kind;
    a.nout = nout;
    a.tw = tw();
    a.g = g;
    a.bt = batch();
    return a;
  }

  // Launch a column pass; ins/outs are per-launch slot lists.  Persistent
  // grid: resident workgroups, capped by the item count.
  void col(int kind, int nout, const T* const* ins, int nin, T* const* outs, const OutSpec* specs) {
    ColArgs<T> a = col_args(kind, nout);
    for (int i = 0; i < nin; ++i) a.in[i] = ins[i];
    int maxt = 1;
    for (int f = 0; f < nout; ++f) {
      a.out[f] = outs[f];
      a.spec[f] = specs[f];
      if (specs[f].nterms > maxt) maxt = specs[f].nterms;
    }
    const bool z = (kind == PK_ZINV || kind == PK_ZFWD);
    const bool inv = (kind == PK_ZINV || kind == PK_YINV);
    const int64_t items = (int64_t)(z ? ztiles() : g.n * ytiles()) * nout * ms.n;
    int64_t blocks = (int64_t)(c->col_blocks[inv ? (maxt > 1 ? 2 : 1) : 0] * ms.col_scale);
    // at least one workgroup per XCD range of the item walk (or one per item)
    if (blocks < 8) blocks = 8;
    if (blocks > items) blocks = items;
    dim3 grid((unsigned)blocks);
    if (inv) k.col_inv(maxt, a, grid, c->stream);
    else k.col_fwd(a, grid, c->stream);
  }

  // Copy-only y passes of `count` fields from slot lists.
  // y pass that copies (transforms) each field.  The row passes leave their
  // r2c outputs doubled, and the forward y pass, their only reader, halves
  // them.
  void y_copy(int kind, int count, T* const* ins, T* const* outs) {
    OutSpec sp[kMaxOut];
    const double coef = kind == PK_YFWD ? 0.5 : 1.0;
    for (int f = 0; f < count; ++f) sp[f] = copy_spec(f, coef);
    col(kind, count, ins, count, outs, sp);
  }

  RowArgs<T> row_args() const {
    RowArgs<T> a;
    std::memset(&a, 0, sizeof(a));
    for (int m = 0; m < ms.n; ++m) {
      a.gamma[m] = ms.gamma[m];
      a.nu[m] = ms.nu[m];
      a.eta[m] = ms.eta[m];
    }
    a.tw = tw();
    a.g = g;
    a.bt = batch();
    return a;
  }

  // Persistent row passes: as many workgroups as can be resident at once
  // (scaled by the tuned factor), capped by the number of row pairs.
  dim3 row_grid(int mode) const {
    int64_t blocks = (int64_t)(c->row_blocks[mode] * ms.row_scale);
    const int64_t items = (int64_t)g.n * g.n / 2 * ms.n;
    if (blocks < 1) blocks = 1;
    if (blocks > items) blocks = items;
    if (blocks > kStatusSlots) blocks = kStatusSlots;  // one status slot per flux-pass workgroup
    return dim3((unsigned)blocks);
  }

  // Row passes address consecutive I_y slots from a first slot and a stride.
  void set_in(RowArgs<T>& r, int first_slot) const {
    r.in0 = iy(first_slot);
    r.in_stride = g.iy;
  }
  void set_out(RowArgs<T>& r, int first_slot) const {
    r.out0 = iy(first_slot);
    r.out_stride = g.iy;
  }

  double inv_n3() const { return 1.0 / (double)g.n3; }

  // Real fields [nf][n^3] (dtype) -> compact spectra D F[f] at dst.
  void forward_real(const void* real, int dtype, int nf, T* dst) {
    RowArgs<T> r = row_args();
    r.real_in = real;
    r.real_dtype = dtype == MHD_FP64 ? 0 : 1;
    r.nf = nf;
    set_out(r, 0);
    k.row(RM_XFWD_REAL, r, row_grid(RM_XFWD_REAL), c->stream);
    T* yi[kMaxOut];
    T* yo[kMaxOut];
    for (int f = 0; f < nf; ++f) { yi[f] = iy(f); yo[f] = iz(f); }
    y_copy(PK_YFWD, nf, yi, yo);
    T* zo[kMaxOut];
    for (int f = 0; f < nf; ++f) zo[f] = spec_field(dst, f);
    OutSpec sp[kMaxOut];
    for (int f = 0; f < nf; ++f) sp[f] = copy_spec(f, 1.0);
    col(PK_ZFWD, nf, yo, nf, zo, sp);
  }

  // Compact spectra at src (nf fields) -> real fields [nf][n^3] (dtype).
  void inverse_real(const T* src, int nf, void* real, int dtype) {
    const T* zi[kMaxIn];
    T* zo[kMaxOut];
    OutSpec sp[kMaxOut];
    for (int f = 0; f < nf; ++f) {
      zi[f] = src + 2 * (size_t)f * g.sc;
      zo[f] = iz(f);
      sp[f] = copy_spec(f, inv_n3());
    }
    col(PK_ZINV, nf, zi, nf, zo, sp);
    T* yo[kMaxOut];
    for (int f = 0; f < nf; ++f) yo[f] = iy(f);
    y_copy(PK_YINV, nf, zo, yo);
    RowArgs<T> r = row_args();
    r.real_out = real;
    r.real_dtype = dtype == MHD_FP64 ? 0 : 1;
    r.nf = nf;
    set_in(r, 0);
    k.row(RM_XINV_REAL, r, row_grid(RM_XINV_REAL), c->stream);
  }

  // Outputs of phase A: u^ (3), and q^ = D F[|u|^2/2] with the viscous-force variant.
  int na() const { return (c->p.flags & MHD_FLAG_VISC_LAPLACIAN) ? 4 : 3; }

  // Phase A: u^ = D F[m / rho] from the state U.
  void phase_a(T* U) {
    const T* zi[4];
    T* zo[4];
    OutSpec sp[4];
    for (int f = 0; f < 4; ++f) {
      zi[f] = spec_field(U, f);
      zo[f] = iz(f);
      sp[f] = copy_spec(f, inv_n3());
    }
    timed(MHD_PASS_ZINV_A, [&] { col(PK_ZINV, 4, zi, 4, zo, sp); });
    T* yo[4] = {iy(0), iy(1), iy(2), iy(3)};
    timed(MHD_PASS_YINV_A, [&] { y_copy(PK_YINV, 4, zo, yo); });
    RowArgs<T> r = row_args();
    set_in(r, 0);
    set_out(r, 4);
    r.nf = na();
    timed(MHD_PASS_XA, [&] { k.row(RM_XA, r, row_grid(RM_XA), c->stream); });
    const int nu_ = na();
    T* ui[4] = {iy(4), iy(5), iy(6), iy(7)};
    T* uo[4] = {iz(0), iz(1), iz(2), iz(3)};
    timed(MHD_PASS_YFWD_A, [&] { y_copy(PK_YFWD, nu_, ui, uo); });
    T* ho[4] = {spec_field(uhat(), 0), spec_field(uhat(), 1), spec_field(uhat(), 2), spec_field(uhat(), 3)};
    OutSpec cp[4] = {copy_spec(0, 1.0), copy_spec(1, 1.0), copy_spec(2, 1.0), copy_spec(3, 1.0)};
    timed(MHD_PASS_ZFWD_A, [&] { col(PK_ZFWD, nu_, uo, nu_, ho, cp); });
  }

  // Phase B: fluxes and the spectral RHS of state U.  rout == nullptr: AB2
  // update of U and the history with the members' coefficients ms.a_cur,
  // ms.a_prev.  record_status: fold the flux pass's CFL speed and
  // non-finite count into the status slots (steps do; pure right-hand sides
  // and the later stages of a multistage step do not).
  void phase_b(T* U, T* rout) { phase_b(U, rout, rout == nullptr); }
  void phase_b(T* U, T* rout, bool record_status) {
    const double s = inv_n3();
    // inputs: 0-2 B^, 3 E^, 4-6 u^
    const T* zi[7] = {spec_field(U, 4), spec_field(U, 5), spec_field(U, 6), spec_field(U, 7),
                      spec_field(uhat(), 0), spec_field(uhat(), 1), spec_field(uhat(), 2)};
    enum { X = 0, Y = 1, Z = 2 };
    const double t3 = s / 3.0, h = 0.5 * s;
    OutSpec sp[12] = {
        copy_spec(0, s), copy_spec(1, s), copy_spec(2, s), copy_spec(3, s),
        // traceless strain (Eqs. 3-4): S_ij = (d_i u_j + d_j u_i)/2 - delta_ij div u / 3
        spec({term(4, X, 2 * t3), term(5, Y, -t3), term(6, Z, -t3)}),  // S_xx
        spec({term(4, X, -t3), term(5, Y, 2 * t3), term(6, Z, -t3)}),  // S_yy
        spec({term(4, Y, h), term(5, X, h)}),                          // S_xy
        spec({term(4, Z, h), term(6, X, h)}),                          // S_xz
        spec({term(5, Z, h), term(6, Y, h)}),                          // S_yz
        // J = curl B
        spec({term(2, Y, s), term(1, Z, -s)}),  // J_x
        spec({term(0, Z, s), term(2, X, -s)}),  // J_y
        spec({term(1, X, s), term(0, Y, -s)}),  // J_z
    };
    T* zo[12];
    for (int f = 0; f < 12; ++f) zo[f] = iz(f);
    timed(MHD_PASS_ZINV_B, [&] { col(PK_ZINV, 12, zi, 7, zo, sp); });
    T* yo[12];
    for (int f = 0; f < 12; ++f) yo[f] = iy(4 + f);
    timed(MHD_PASS_YINV_B, [&] { y_copy(PK_YINV, 12, zo, yo); });
    RowArgs<T> r = row_args();
    set_in(r, 0);
    set_out(r, 0);
    if (c->p.flags & MHD_FLAG_VISC_LAPLACIAN)
      for (int m = 0; m < ms.n; ++m) r.nu[m] = 0.0;  // no stress-form terms: the force is added spectrally
    r.status = record_status ? status() : nullptr;
    timed(MHD_PASS_XB, [&] { k.row(RM_XB, r, row_grid(RM_XB), c->stream); });
    T* fi[12];
    T* fo[12];
    for (int f = 0; f < 12; ++f) { fi[f] = iy(f); fo[f] = iz(f); }
    timed(MHD_PASS_YFWD_B, [&] { y_copy(PK_YFWD, 12, fi, fo); });
    RhsArgs<T> q;
    std::memset(&q, 0, sizeof(q));
    for (int f = 0; f < 12; ++f) q.flux[f] = iz(f);
    // flux slots: 0 Pi_xx, 1 Pi_yy, 2 Pi_zz, 3 Pi_xy, 4 Pi_xz, 5 Pi_yz, 6-8 F^E, 9-11 e = u x B
    // R_f = F_z[A_f] + i kz F_z[Z_f]
    q.A[1] = spec({term(0, X, -1), term(3, Y, -1)});  // MHD2: -i k_j Pi_xj
    q.Z[1] = spec({term(4, -1, -1)});
    q.A[2] = spec({term(3, X, -1), term(1, Y, -1)});
    q.Z[2] = spec({term(5, -1, -1)});
    q.A[3] = spec({term(4, X, -1), term(5, Y, -1)});
    q.Z[3] = spec({term(2, -1, -1)});
    q.A[4] = spec({term(11, Y, 1)});                   // MHD4: i k x e
    q.Z[4] = spec({term(10, -1, -1)});
    q.A[5] = spec({term(11, X, -1)});
    q.Z[5] = spec({term(9, -1, 1)});
    q.A[6] = spec({term(10, X, 1), term(9, Y, -1)});
    q.A[7] = spec({term(6, X, -1), term(7, Y, -1)});  // MHD3: -i k . F^E
    q.Z[7] = spec({term(8, -1, -1)});
    q.state = U;
    q.rprev = rprev();
    q.rout = rout;
    q.tw = tw();
    q.uhat = uhat();
    q.mu = (c->p.flags & MHD_FLAG_VISC_LAPLACIAN) ? c->p.nu : 0.0;
    q.kinematic = (c->p.flags & MHD_FLAG_KINEMATIC) ? 1 : 0;
    q.force = c->p.force != 0.0 ? force() : nullptr;
    for (int m = 0; m < ms.n; ++m) {
      q.dt[m] = ms.dt[m];
      q.a_cur[m] = ms.a_cur[m];
      q.a_prev[m] = ms.a_prev[m];
      q.eta[m] = ms.eta[m];
    }
    q.g = g;
    q.bt = batch();
    const unsigned sblocks = (unsigned)((g.sc + kThreads - 1) / kThreads);
    timed(MHD_PASS_RHO, [&] {
      // the body force reads rho^ and m^ of this step before either is updated
      if (q.force)
        hipLaunchKernelGGL((k_force_abc<T>), dim3(sblocks), dim3(kThreads), 0, c->stream, U, force(), g,
                           c->p.force);
      hipLaunchKernelGGL((k_rho_rhs<T>), dim3(sblocks, (unsigned)ms.n), dim3(kThreads), 0, c->stream, q);
    });
    timed(MHD_PASS_ZRHS, [&] { k.rhs(q, dim3((unsigned)(rtiles() * 7 * ms.n)), c->stream); });
  }

  double step_bytes() const {
    double b = 0.0;
    for (int cls = 0; cls < MHD_PASS_COUNT; ++cls) b += class_bytes(cls);
    const double evals = c->p.scheme == MHD_RK4 ? 4 : (c->p.scheme == MHD_PC ? 2 : 1);
    // a multistage step: its right-hand sides plus the stage arithmetic over the 8-field sets
    const double stage = c->p.scheme == MHD_RK4 ? 4 * cbytes(24, 0, 0) + cbytes(8, 0, 0)
                                                 : (c->p.scheme == MHD_PC ? 2 * cbytes(24, 0, 0) : 0.0);
    return b * evals + stage;
  }

  void combine(int op, double cc, double w, double a_cur = 0.0, double a_prev = 0.0) {
    const unsigned blocks = (unsigned)((8 * g.sc + kThreads - 1) / kThreads);
    hipLaunchKernelGGL((k_combine<T>), dim3(blocks), dim3(kThreads), 0, c->stream, state(), trhs(), rprev(),
                       tstate(), g, op, cc, w, a_cur, a_prev);
  }

  // One step of the context's scheme (single runs).  AB2: one right-hand
  // side with the update fused into its last pass.  RK4 and PC: right-hand
  // sides into trhs, stage states in tstate, and rprev as the RK4 stage sum
  // or the PC history.  The flux pass of the first evaluation (the state at
  // t_n) records the CFL / non-finite status.
  void step_once(bool first) {
    const double dt = c->p.dt;
    if (c->p.scheme == MHD_RK4) {
      phase_a(state());
      phase_b(state(), trhs(), true);
      combine(CB_RK_FIRST, 0.5 * dt, 0.0);
      const double cs[3] = {0.5 * dt, dt, dt / 6.0};
      for (int st = 0; st < 3; ++st) {
        phase_a(tstate());
        phase_b(tstate(), trhs(), false);
        combine(st < 2 ? CB_RK_MID : CB_RK_LAST, cs[st], st < 2 ? 2.0 : 1.0);
      }
      return;
    }
    if (c->p.scheme == MHD_PC) {
      phase_a(state());
      phase_b(state(), trhs(), true);
      combine(CB_PC_PRED, dt, 0.0, first ? 1.0 : 1.5, first ? 0.0 : -0.5);
      phase_a(tstate());
      phase_b(tstate(), trhs(), false);
      combine(CB_PC_CORR, 0.5 * dt, 0.0);
      return;
    }
    ms.a_cur[0] = first ? 1.0 : 1.5;
    ms.a_prev[0] = first ? 0.0 : -0.5;
    phase_a(state());
    phase_b(state(), nullptr);
  }

  void reset_status() {
    const int words = kStatusSlots * 2 * 2;  // doubles as u32 words; +0.0 is all-zero bits
    hipLaunchKernelGGL(k_fill_u32, dim3((words + kThreads - 1) / kThreads), dim3(kThreads), 0, c->stream,
                       reinterpret_cast<unsigned*>(status()), words, 0u);
  }

  // Diagnostics pass over the state: real-space partials and spectral sums.
  void diagnostics() {
    const double s = inv_n3();
    T* U = state();
    const T* zi[8];
    for (int f = 0; f < 8; ++f) zi[f] = spec_field(U, f);
    enum { X = 0, Y = 1, Z = 2 };
    constexpr int NF = kDiagFields;  // the state and div B
    OutSpec sp[NF];
    for (int f = 0; f < 8; ++f) sp[f] = copy_spec(f, s);
    sp[8] = spec({term(4, X, s), term(5, Y, s), term(6, Z, s)});  // div B
    T* zo[NF];
    for (int f = 0; f < NF; ++f) zo[f] = iz(f);
    col(PK_ZINV, NF, zi, 8, zo, sp);
    T* yo[NF];
    for (int f = 0; f < NF; ++f) yo[f] = iy(f);
    y_copy(PK_YINV, NF, zo, yo);
    RowArgs<T> r = row_args();
    set_in(r, 0);
    r.partials = part();
    const dim3 grid = row_grid(RM_XDIAG);  // one partial record per workgroup (<= n^2/2)
    k.row(RM_XDIAG, r, grid, c->stream);
    const int sblocks = (int)((g.sc + kThreads - 1) / kThreads);
    hipLaunchKernelGGL((k_spec_diag<T>), dim3(sblocks), dim3(kThreads), 0, c->stream, spec_field(U, 4),
                       spec_field(U, 5), spec_field(U, 6), g, spart());
    const unsigned maxmask = (1u << DQ_DIVB_MAX) | (1u << DQ_CFL_MAX);
    hipLaunchKernelGGL(k_reduce, dim3(kDiagQ + kSpecQ), dim3(kThreads), 0, c->stream, part(), (int64_t)grid.x,
                       kDiagQ, maxmask, spart(), (int64_t)sblocks, kSpecQ, res(), res() + 16);
    // the steps' status slots: FP64 max of the signal speeds, sum of the non-finite counts
    hipLaunchKernelGGL(k_reduce, dim3(2), dim3(kThreads), 0, c->stream, status(), (int64_t)kStatusSlots, 2, 1u,
                       status(), (int64_t)0, 0, res() + kResStatus, res() + kResStatus);
  }
};

// Working precision -> element type of the state and of real fields.
bool is_fp32(int32_t prec) { return prec == MHD_FP32 || prec == MHD_MIXED; }

const void* kern_for(const mhd_ctx* c) {
  Registry& r = registry();
  if (c->p.flags & MHD_FLAG_SCHEDULE_ALT) {
    if (c->p.precision != MHD_FP32) return nullptr;
    return r.f32s1[c->p.n].row ? &r.f32s1[c->p.n] : nullptr;
  }
  if (c->p.precision == MHD_FP32) return r.f32[c->p.n].row ? &r.f32[c->p.n] : nullptr;
  if (c->p.precision == MHD_MIXED) return r.mx[c->p.n].row ? &r.mx[c->p.n] : nullptr;
  return r.f64[c->p.n].row ? &r.f64[c->p.n] : nullptr;
}

template <typename F>
int with_engine(mhd_ctx* c, F&& fn) {
  const void* k = kern_for(c);
  if (!k) return MHD_E_SIZE;
  if (is_fp32(c->p.precision)) {
    Engine<float> e(c, *static_cast<const Kern<float>*>(k));
    return fn(e);
  }
  Engine<double> e(c, *static_cast<const Kern<double>*>(k));
  return fn(e);
}

int validate(const mhd_params* p) {
  if (!p) return MHD_E_ARG;
  if (p->precision != MHD_FP32 && p->precision != MHD_FP64 && p->precision != MHD_MIXED) return MHD_E_ARG;
  if (p->scheme != MHD_AB2 && p->scheme != MHD_RK4 && p->scheme != MHD_PC) return MHD_E_ARG;
  if (!std::isfinite(p->force)) return MHD_E_ARG;
  if (!(p->gamma > 1.0) || !(p->nu >= 0.0) || !(p->eta >= 0.0) || !(p->dt > 0.0) || !(p->cfl > 0.0)) return MHD_E_ARG;
  if (!std::isfinite(p->gamma) || !std::isfinite(p->nu) || !std::isfinite(p->eta) || !std::isfinite(p->dt) ||
      !std::isfinite(p->cfl))
    return MHD_E_ARG;
  if (!size_ok(p->n, p->precision)) return MHD_E_SIZE;
  return MHD_OK;
}

bool dtype_ok(int32_t d) { return d == MHD_FP32 || d == MHD_FP64; }

// Ensemble members: AB2 without the Section V variants (their batched
// launches carry per-member AB2 coefficients only).
int validate_member(const mhd_params* p) {
  const int v = validate(p);
  if (v != MHD_OK) return v;
  if (p->scheme != MHD_AB2 || p->force != 0.0 || (p->flags & (MHD_FLAG_VISC_LAPLACIAN | MHD_FLAG_KINEMATIC)))
    return MHD_E_ARG;
  return MHD_OK;
}

}  // namespace

static int ctx_geometry(mhd_ctx* c);

// Sets up a context in place (no allocation): parameters, layout, launch
// geometry and the twiddle table, uploaded through a host buffer on the stack
// (synchronously).  The workspace must have been checked by the caller.
static int ctx_setup(mhd_ctx* c, const mhd_params* p, void* d_workspace, size_t ws_bytes, hipStream_t stream) {
  c->p = *p;
  c->g = make_geo(p->n);
  const size_t ts = is_fp32(p->precision) ? sizeof(float) : sizeof(double);
  c->L = make_layout(c->g, ts);
  c->stream = stream;
  c->ws = static_cast<char*>(d_workspace);
  c->ws_bytes = ws_bytes;
  c->has_state = false;
  c->first_step = true;
  c->step = 0;
  c->t = 0.0;
  const int rg = ctx_geometry(c);
  if (rg != MHD_OK) return rg;
  // twiddles exp(-2 pi i j / n) in FP64, rounded once to the working precision
  const int n = p->n;
  const double two_pi = 6.28318530717958647692528676655900577;
  double h64[2 * 1024];
  float h32[2 * 1024];
  for (int j = 0; j < n; ++j) {
    const double cr = std::cos(two_pi * j / n), ci = -std::sin(two_pi * j / n);
    h64[2 * j] = cr;
    h64[2 * j + 1] = ci;
    h32[2 * j] = (float)cr;
    h32[2 * j + 1] = (float)ci;
  }
  const void* src = is_fp32(p->precision) ? static_cast<const void*>(h32) : static_cast<const void*>(h64);
  hipError_t e = hipMemcpyAsync(c->ws + c->L.tw, src, 2 * (size_t)n * ts, hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);  // the host buffer dies with this frame
  return e == hipSuccess ? MHD_OK : MHD_E_HIP;
}

// Launch geometry of the context's kernels (their resident workgroups per CU
// times the CU count); redone when an ensemble group switches schedule.
static int ctx_geometry(mhd_ctx* c) {
  const mhd_params* p = &c->p;
  const void* kv = kern_for(c);
  if (!kv) return MHD_E_SIZE;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&c->num_cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess || c->num_cus <= 0) return MHD_E_HIP;
  const bool f32 = is_fp32(p->precision);
  for (int m = 0; m < 5; ++m) {
    const int occ = f32 ? static_cast<const Kern<float>*>(kv)->row_occupancy(m)
                        : static_cast<const Kern<double>*>(kv)->row_occupancy(m);
    c->row_blocks[m] = occ * c->num_cus;
  }
  const int cocc[3] = {f32 ? static_cast<const Kern<float>*>(kv)->col_occupancy(-1, 1)
                           : static_cast<const Kern<double>*>(kv)->col_occupancy(-1, 1),
                       f32 ? static_cast<const Kern<float>*>(kv)->col_occupancy(1, 1)
                           : static_cast<const Kern<double>*>(kv)->col_occupancy(1, 1),
                       f32 ? static_cast<const Kern<float>*>(kv)->col_occupancy(1, 3)
                           : static_cast<const Kern<double>*>(kv)->col_occupancy(1, 3)};
  for (int m = 0; m < 3; ++m) c->col_blocks[m] = cocc[m] * c->num_cus;
  return MHD_OK;
}

static int ctx_check(const mhd_params* p, void* d_workspace, size_t ws_bytes) {
  const int v = validate(p);
  if (v != MHD_OK) return v;
  const size_t need = mhd_workspace_bytes(p);
  if (!d_workspace || ws_bytes < need || (reinterpret_cast<uintptr_t>(d_workspace) & 255u) != 0)
    return MHD_E_WORKSPACE;
  return MHD_OK;
}

static int ctx_create(const mhd_params* p, void* d_workspace, size_t ws_bytes, hipStream_t stream, mhd_ctx** out) {
  if (!out) return MHD_E_ARG;
  *out = nullptr;
  int rc = ctx_check(p, d_workspace, ws_bytes);
  if (rc != MHD_OK) return rc;
  mhd_ctx* c = new (std::nothrow) mhd_ctx();
  if (!c) return MHD_E_ARG;
  rc = ctx_setup(c, p, d_workspace, ws_bytes, stream);
  if (rc != MHD_OK) {
    delete c;
    return rc;
  }
  *out = c;
  return MHD_OK;
}

static int ctx_diag(mhd_ctx* c, mhd_diag* h) {
  if (!c || !h) return MHD_E_ARG;
  if (!c->has_state) return MHD_E_STATE;
  int rc = with_engine(c, [&](auto& e) {
    e.diagnostics();
    return check_launch(c, "mhd_diagnostics");
  });
  if (rc != MHD_OK) return rc;
  double res[kResWords];
  hipError_t err = hipMemcpyAsync(res, c->ws + c->L.res, sizeof(res), hipMemcpyDeviceToHost, c->stream);
  if (err == hipSuccess) err = hipStreamSynchronize(c->stream);
  if (err != hipSuccess) return hip_fail(c, err, "mhd_diagnostics copy");
  const Geo& g = c->g;
  const double n3 = (double)g.n3;
  const double inv6 = 1.0 / (n3 * n3);
  const double gm1 = c->p.gamma - 1.0;
  std::memset(h, 0, sizeof(*h));
  h->t = c->t;
  h->step = c->step;
  h->mass = res[DQ_RHO] / n3;
  h->mom[0] = res[DQ_MX] / n3;
  h->mom[1] = res[DQ_MY] / n3;
  h->mom[2] = res[DQ_MZ] / n3;
  h->e_kin = res[DQ_EKIN] / n3;
  h->e_mag = res[DQ_EMAG] / n3;
  const double pmean = res[DQ_P] / n3;
  h->e_int = pmean / gm1;
  h->e_tot = res[DQ_E] / n3;
  h->h_cross = res[DQ_HC] / n3;
  h->h_mag = res[16 + SQ_HM] * inv6;
  const double divb2 = res[16 + SQ_DIVB2] * inv6;
  const double j2 = res[16 + SQ_J2] * inv6;
  h->divb_rms = std::sqrt(divb2);
  h->j_rms = std::sqrt(j2);
  h->divb_rel = j2 > 0 ? std::sqrt(divb2 / j2) : 0.0;
  h->divb_max = res[DQ_DIVB_MAX];
  const double two_pi = 6.28318530717958647692528676655900577;
  h->dt_cfl = c->p.cfl * (two_pi / g.n) / res[DQ_CFL_MAX];
  h->c_s = std::sqrt(c->p.gamma * pmean / h->mass);
  const double umean = res[DQ_UABS] / n3;
  h->v_a = (res[DQ_BABS] / n3) / std::sqrt(h->mass);
  h->mach_s = umean / h->c_s;
  h->mach_a = h->v_a > 0 ? umean / h->v_a : INFINITY;
  h->nonfinite = (int64_t)res[DQ_NONFINITE];
  const double cmax_seen = res[kResStatus], bad_seen = res[kResStatus + 1];
  if (h->nonfinite > 0 || bad_seen > 0 || !(cmax_seen == cmax_seen)) return MHD_E_NONFINITE;
  if ((c->p.flags & MHD_FLAG_CHECK_CFL) && cmax_seen > 0) {
    const double dt_lim = c->p.cfl * (two_pi / g.n) / cmax_seen;
    if (c->p.dt > dt_lim) return MHD_E_CFL;
  }
  return MHD_OK;
}

// The steady AB2 step (coefficients 3/2, -1/2) captured once as a graph on a
// private stream (the caller's stream may be the legacy default stream, which
// cannot be captured) and replayed by mhd_step.  The step's launches never
// change: the workspace, the parameters and the launch geometry are fixed for
// the context's lifetime.
static int ctx_capture(mhd_ctx* c) {
  hipError_t e = hipSuccess;
  if (!c->cap) e = hipStreamCreateWithFlags(&c->cap, hipStreamNonBlocking);
  if (e != hipSuccess) return hip_fail(c, e, "graph stream");
  e = hipStreamBeginCapture(c->cap, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return hip_fail(c, e, "hipStreamBeginCapture");
  hipStream_t saved = c->stream;
  c->stream = c->cap;
  (void)with_engine(c, [&](auto& eng) {
    eng.step_once(false);
    return MHD_OK;
  });
  c->stream = saved;
  hipGraph_t g = nullptr;
  const hipError_t le = hipGetLastError();
  e = hipStreamEndCapture(c->cap, &g);
  if (le != hipSuccess || e != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return hip_fail(c, le != hipSuccess ? le : e, "step capture");
  }
  hipGraphExec_t x = nullptr;
  e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    (void)hipGraphDestroy(g);
    return hip_fail(c, e, "hipGraphInstantiate");
  }
  c->graph = g;
  c->exec = x;
  return MHD_OK;
}

// Checkpoint blob: header, then the compact state U^n, the AB2 history
// R^{n-1} and the status slots, each at a 256-byte boundary.
struct CkptLayout {
  size_t state, rprev, status, total, spec_bytes, status_bytes;
};
static CkptLayout ckpt_layout(const mhd_ctx* c) {
  CkptLayout B;
  const size_t ts = is_fp32(c->p.precision) ? sizeof(float) : sizeof(double);
  B.spec_bytes = 8 * (size_t)c->g.sc * 2 * ts;
  B.status_bytes = (size_t)kStatusSlots * 2 * sizeof(double);
  size_t off = sizeof(CkptHeader);
  B.state = off;
  off += align256(B.spec_bytes);
  B.rprev = off;
  off += align256(B.spec_bytes);
  B.status = off;
  off += align256(B.status_bytes);
  B.total = off;
  return B;
}

// *out += hash of the blob's 64-bit words (the checksum word read as zero);
// the caller zeroes *out first where it starts a new hash.
static void blob_hash(mhd_ctx* c, const char* blob, size_t bytes, unsigned long long* out) {
  const int64_t words = (int64_t)(bytes / sizeof(uint64_t));
  int64_t blocks = (words + kThreads * 8 - 1) / (kThreads * 8);
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_blob_hash, dim3((unsigned)blocks), dim3(kThreads), 0, c->stream,
                     reinterpret_cast<const uint64_t*>(blob), words, (int64_t)kCkptSumWord, out);
}

// Device scratch of mhd_rhs_noalloc: a file-scope device array (each GPU the
// library runs on holds its own copy until the process ends).  Host code
// never passes the array's name to a kernel: scratch_address resolves each
// device's copy once, with that device current, and every later use goes
// through that address.
constexpr size_t kScratchBytes = size_t(64) << 20;
static __device__ __align__(256) char scratch[kScratchBytes];
constexpr int kMaxDevices = 64;

static int scratch_address(void** out) {
  static std::mutex mu;
  static void* addr[kMaxDevices] = {nullptr};
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return MHD_E_HIP;
  if (dev < 0 || dev >= kMaxDevices) return MHD_E_ARG;
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[dev]) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) return MHD_E_HIP;
    addr[dev] = ptr;
  }
  *out = addr[dev];
  return MHD_OK;
}

// ------------------------------------------------------------------ ensembles

// Members with equal (n, precision), at most kMaxMem of them, share one
// launch per pass: their workspaces sit at a uniform stride from the group's
// base, and `lead` is a context over the first slot whose stream is the
// group's branch stream.
struct EnsGroup {
  int32_t n = 0, precision = 0;
  std::vector<int> members;  // ensemble member index of each slot
  size_t stride = 0;         // bytes between consecutive slots' workspaces
  char* base = nullptr;
  mhd_ctx* lead = nullptr;
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  double col_scale = 1.0, row_scale = 1.0;  // persistent-grid scales (tuned)
  int sched = 0;                            // kernel schedule (tuned): 0 default, 1 MHD_FLAG_SCHEDULE_ALT
  bool tuned = false;
};

struct mhd_ens {
  int32_t count = 0;
  hipStream_t stream = nullptr;
  std::vector<mhd_ctx*> mem;  // one context per member, on the ensemble stream
  std::vector<int> grp_of;
  std::vector<EnsGroup> groups;
  hipStream_t cap = nullptr;  // capture origin (the caller's stream may be the legacy default stream)
  hipEvent_t fork = nullptr, t0 = nullptr, t1 = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int tune_mode = 1;  // 0: off, 1: in memory, 2: in memory and the cache file
  std::string tune_path;
  std::string last_err;
  int num_cus = 0;
};

namespace {

int ens_fail(mhd_ens* E, hipError_t e, const char* what) {
  E->last_err = std::string(what) + ": " + hipGetErrorString(e);
  return MHD_E_HIP;
}

// One pass sequence of group G: a step (AB2 coefficients from each member's
// history) or, with rhs_only, right-hand sides into the members' scratch
// slots, leaving states and histories unchanged.
template <typename T>
void group_launch(mhd_ens* E, EnsGroup& G, const Kern<T>& k, bool rhs_only) {
  MemberSet ms;
  ms.n = (int)G.members.size();
  ms.stride = (int64_t)G.stride;
  ms.col_scale = G.col_scale;
  ms.row_scale = G.row_scale;
  for (int s = 0; s < ms.n; ++s) {
    const mhd_ctx* mc = E->mem[G.members[s]];
    ms.gamma[s] = mc->p.gamma;
    ms.nu[s] = mc->p.nu;
    ms.eta[s] = mc->p.eta;
    ms.dt[s] = mc->p.dt;
    ms.a_cur[s] = mc->first_step ? 1.0 : 1.5;
    ms.a_prev[s] = mc->first_step ? 0.0 : -0.5;
  }
  Engine<T> e(G.lead, k, ms);
  e.phase_a(e.state());
  e.phase_b(e.state(), rhs_only ? e.trhs() : nullptr);
}

// Every group as a parallel branch forked from and joined into `origin` (the
// ensemble stream, or the capture stream while the graph is recorded).
int ens_launch(mhd_ens* E, hipStream_t origin, bool rhs_only) {
  hipError_t e = hipEventRecord(E->fork, origin);
  for (EnsGroup& G : E->groups) {
    if (e == hipSuccess) e = hipStreamWaitEvent(G.stream, E->fork, 0);
    if (e != hipSuccess) break;
    const void* kv = kern_for(G.lead);
    if (is_fp32(G.precision)) group_launch(E, G, *static_cast<const Kern<float>*>(kv), rhs_only);
    else group_launch(E, G, *static_cast<const Kern<double>*>(kv), rhs_only);
    e = hipEventRecord(G.done, G.stream);
    if (e == hipSuccess) e = hipStreamWaitEvent(origin, G.done, 0);
  }
  if (e == hipSuccess) e = hipGetLastError();
  return e == hipSuccess ? MHD_OK : ens_fail(E, e, "ensemble launch");
}

// Switches group G's launches to kernel schedule `sched` (the lead context
// takes that build's kernels and launch geometry; the members' own contexts,
// used for set/get/diagnostics, keep the default build: both lay out the
// compact spectra identically).  MHD_E_SIZE if the build does not exist.
int set_schedule(EnsGroup& G, int sched) {
  const int rc = mhd_set_schedule(G.lead, sched);
  if (rc == MHD_OK) G.sched = sched;
  return rc;
}

std::string tune_key(const EnsGroup& G, int cus) {
  char b[96];
  std::snprintf(b, sizeof(b), "%d %d %d %d", G.n, G.precision, (int)G.members.size(), cus);
  return b;
}

// Cache lines: "mhd-ens-tune <n> <precision> <members> <CUs> <col_scale> <row_scale> <schedule>".
void tune_read(mhd_ens* E) {
  FILE* f = std::fopen(E->tune_path.c_str(), "r");
  if (!f) return;
  char line[256];
  while (std::fgets(line, sizeof(line), f)) {
    int n, pr, nm, cus, sc = 0;
    double cs, rs;
    const int got = std::sscanf(line, "mhd-ens-tune %d %d %d %d %lf %lf %d", &n, &pr, &nm, &cus, &cs, &rs, &sc);
    if (got < 6) continue;
    if (!(cs > 0.0 && cs <= 4.0 && rs > 0.0 && rs <= 4.0) || sc < 0 || sc > 1) continue;
    for (EnsGroup& G : E->groups) {
      if (G.n == n && G.precision == pr && (int)G.members.size() == nm && E->num_cus == cus) {
        if (sc == 1 && set_schedule(G, 1) != MHD_OK) continue;  // no such build: keep tuning
        G.col_scale = cs;
        G.row_scale = rs;
        G.tuned = true;
      }
    }
  }
  std::fclose(f);
}

void tune_write(mhd_ens* E, const EnsGroup& G) {
  FILE* f = std::fopen(E->tune_path.c_str(), "a");
  if (!f) return;  // an unwritable cache only costs a re-tune next time
  std::fprintf(f, "mhd-ens-tune %s %.4f %.4f %d\n", tune_key(G, E->num_cus).c_str(), G.col_scale, G.row_scale,
               G.sched);
  std::fclose(f);
}

// Times right-hand-side evaluations of the whole ensemble (all branches
// running together), in milliseconds per evaluation.
int ens_time(mhd_ens* E, int reps, double* ms) {
  int rc = ens_launch(E, E->stream, true);  // warm-up
  hipError_t e = hipSuccess;
  if (rc == MHD_OK) e = hipEventRecord(E->t0, E->stream);
  for (int r = 0; rc == MHD_OK && e == hipSuccess && r < reps; ++r) rc = ens_launch(E, E->stream, true);
  if (rc != MHD_OK) return rc;
  if (e == hipSuccess) e = hipEventRecord(E->t1, E->stream);
  if (e == hipSuccess) e = hipEventSynchronize(E->t1);
  float t = 0.f;
  if (e == hipSuccess) e = hipEventElapsedTime(&t, E->t0, E->t1);
  if (e != hipSuccess) return ens_fail(E, e, "ensemble tuning");
  *ms = (double)t / reps;
  return MHD_OK;
}

// One sweep of coordinate search over the groups: for each untuned group,
// the kernel schedule (the default build, or the alternative one where it
// exists) and the persistent-grid scales of its column and row passes that
// give the fastest whole-ensemble evaluation, the other groups held at their
// current choices.  A choice other than the default (default build, full
// grids) must beat the default by kTuneMargin, so that timing noise between
// near-equal choices does not change the pick from run to run.
constexpr double kTuneMargin = 0.03;
int ens_tune(mhd_ens* E) {
  static const double kScales[] = {0.25, 0.5, 1.0};
  for (EnsGroup& G : E->groups) {
    if (G.tuned) continue;
    double best = 1e300, bc = 1.0, br = 1.0, t_default = 1e300;
    int bs = 0;
    for (int sched = 0; sched < 2; ++sched) {
      if (set_schedule(G, sched) != MHD_OK) continue;  // no alternative build for this (n, precision)
      for (double cs : kScales) {
        for (double rs : kScales) {
          G.col_scale = cs;
          G.row_scale = rs;
          double t = 0.0;
          int rc = ens_time(E, 3, &t);
          if (rc != MHD_OK) return rc;
          if (sched == 0 && cs == 1.0 && rs == 1.0) t_default = t;
          if (t < best) {
            best = t;
            bc = cs;
            br = rs;
            bs = sched;
          }
        }
      }
    }
    if (!(best < (1.0 - kTuneMargin) * t_default)) {
      bs = 0;
      bc = 1.0;
      br = 1.0;
    }
    const int rc = set_schedule(G, bs);
    if (rc != MHD_OK) return rc;
    G.col_scale = bc;
    G.row_scale = br;
    G.tuned = true;
    if (E->tune_mode == 2) tune_write(E, G);
  }
  return MHD_OK;
}

int ens_capture(mhd_ens* E) {
  hipError_t e = hipStreamBeginCapture(E->cap, hipStreamCaptureModeRelaxed);
  if (e != hipSuccess) return ens_fail(E, e, "hipStreamBeginCapture");
  int rc = ens_launch(E, E->cap, false);
  hipGraph_t g = nullptr;
  e = hipStreamEndCapture(E->cap, &g);
  if (rc != MHD_OK) {
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }
  if (e != hipSuccess) return ens_fail(E, e, "hipStreamEndCapture");
  hipGraphExec_t x = nullptr;
  e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    (void)hipGraphDestroy(g);
    return ens_fail(E, e, "hipGraphInstantiate");
  }
  E->graph = g;
  E->exec = x;
  return MHD_OK;
}

void ens_free(mhd_ens* E) {
  if (!E) return;
  if (E->exec) (void)hipGraphExecDestroy(E->exec);
  if (E->graph) (void)hipGraphDestroy(E->graph);
  for (EnsGroup& G : E->groups) {
    if (G.done) (void)hipEventDestroy(G.done);
    if (G.stream) (void)hipStreamDestroy(G.stream);
    delete G.lead;
  }
  for (mhd_ctx* c : E->mem) mhd_destroy(c);
  if (E->cap) (void)hipStreamDestroy(E->cap);
  if (E->fork) (void)hipEventDestroy(E->fork);
  if (E->t0) (void)hipEventDestroy(E->t0);
  if (E->t1) (void)hipEventDestroy(E->t1);
  delete E;
}

// Group members by (n, precision) in order of first appearance, at most
// kMaxMem per group; returns the workspace offset of each group.
size_t ens_plan(const mhd_params* p, int32_t count, std::vector<EnsGroup>& groups, std::vector<int>& grp_of) {
  groups.clear();
  grp_of.assign(count, -1);
  for (int i = 0; i < count; ++i) {
    int gi = -1;
    for (int j = 0; j < (int)groups.size(); ++j) {
      if (groups[j].n == p[i].n && groups[j].precision == p[i].precision && (int)groups[j].members.size() < kMaxMem) {
        gi = j;
        break;
      }
    }
    if (gi < 0) {
      EnsGroup G;
      G.n = p[i].n;
      G.precision = p[i].precision;
      G.stride = align256(mhd_workspace_bytes(&p[i]));
      groups.push_back(G);
      gi = (int)groups.size() - 1;
    }
    groups[gi].members.push_back(i);
    grp_of[i] = gi;
  }
  size_t total = 0;
  for (const EnsGroup& G : groups) total += G.stride * G.members.size();
  return total;
}

}  // namespace

// ------------------------------------------------------------------ C-ABI

extern "C" {

int mhd_supported_size(int32_t n, int32_t precision) { return size_ok(n, precision) ? 1 : 0; }

int64_t mhd_spectrum_size(int32_t n) {
  if (n < 1) return 0;
  return make_geo(n).sc;
}

int32_t mhd_spectrum_pitch(int32_t n) {
  if (n < 1) return 0;
  return make_geo(n).nhp;
}

size_t mhd_workspace_bytes(const mhd_params* p) {
  if (validate(p) != MHD_OK) return 0;
  const size_t ts = is_fp32(p->precision) ? sizeof(float) : sizeof(double);
  return make_layout(make_geo(p->n), ts).total;
}

int mhd_init(const mhd_params* p, void* d_workspace, size_t ws_bytes, void* hip_stream, mhd_ctx** out) {
  return ctx_create(p, d_workspace, ws_bytes, static_cast<hipStream_t>(hip_stream), out);
}

int mhd_set_state(mhd_ctx* c, const void* d_fields, int32_t dtype) {
  if (!c || !d_fields || !dtype_ok(dtype)) return MHD_E_ARG;
  int rc = with_engine(c, [&](auto& e) {
    e.forward_real(d_fields, dtype, 8, e.state());
    e.reset_status();
    return check_launch(c, "mhd_set_state");
  });
  if (rc == MHD_OK) {
    c->has_state = true;
    c->first_step = true;
    c->step = 0;
    c->t = 0.0;
  }
  return rc;
}

int mhd_get_state(mhd_ctx* c, void* d_fields, int32_t dtype) {
  if (!c || !d_fields || !dtype_ok(dtype)) return MHD_E_ARG;
  if (!c->has_state) return MHD_E_STATE;
  return with_engine(c, [&](auto& e) {
    e.inverse_real(e.state(), 8, d_fields, dtype);
    return check_launch(c, "mhd_get_state");
  });
}

int mhd_rhs(mhd_ctx* c, const void* d_in, void* d_out, int32_t dtype) {
  if (!c || !d_in || !d_out || !dtype_ok(dtype)) return MHD_E_ARG;
  return with_engine(c, [&](auto& e) {
    e.forward_real(d_in, dtype, 8, e.tstate());
    e.phase_a(e.tstate());
    e.phase_b(e.tstate(), e.trhs());
    e.inverse_real(e.trhs(), 8, d_out, dtype);
    return check_launch(c, "mhd_rhs");
  });
}

int mhd_rhs_noalloc(const mhd_params* p, const void* d_in, void* d_out, int32_t dtype, void* hip_stream) {
  if (!p || !d_in || !d_out || !dtype_ok(dtype)) return MHD_E_ARG;
  const int v = validate(p);
  if (v != MHD_OK) return v;
  if (mhd_workspace_bytes(p) > kScratchBytes) return MHD_E_WORKSPACE;  // beyond the static scratch
  void* ws = nullptr;
  int rc = scratch_address(&ws);
  if (rc != MHD_OK) return rc;
  // a context on the stack over the scratch: nothing is allocated, on the
  // device or the host (its string and vectors stay empty)
  mhd_ctx c;
  rc = ctx_setup(&c, p, ws, kScratchBytes, static_cast<hipStream_t>(hip_stream));
  if (rc != MHD_OK) return rc;
  return mhd_rhs(&c, d_in, d_out, dtype);  // every launch is enqueued (arguments copied) when this returns
}

int mhd_set_schedule(mhd_ctx* c, int32_t schedule) {
  if (!c || schedule < 0 || schedule > 1) return MHD_E_ARG;
  const int32_t old = c->p.flags;
  c->p.flags = schedule ? (old | MHD_FLAG_SCHEDULE_ALT) : (old & ~MHD_FLAG_SCHEDULE_ALT);
  const int rc = ctx_geometry(c);
  if (rc != MHD_OK) {
    c->p.flags = old;
    (void)ctx_geometry(c);
    return rc;
  }
  // the captured step belongs to the other build
  if (c->exec) (void)hipGraphExecDestroy(c->exec);
  if (c->graph) (void)hipGraphDestroy(c->graph);
  c->exec = nullptr;
  c->graph = nullptr;
  return MHD_OK;
}

int mhd_step(mhd_ctx* c, int32_t nsteps) {
  if (!c || nsteps < 0) return MHD_E_ARG;
  if (!c->has_state) return MHD_E_STATE;
  // Eager launches for the Euler start, while profiling (events bracket single
  // launches) or with graphs turned off; every other step replays the graph.
  int done = 0;
  int rc = with_engine(c, [&](auto& e) {
    for (; done < nsteps; ++done) {
      const bool first = c->first_step && done == 0;
      if (!first && !c->prof_on && !(c->p.flags & MHD_FLAG_NO_GRAPH)) break;
      e.step_once(first);
    }
    return check_launch(c, "mhd_step");
  });
  if (rc == MHD_OK && done < nsteps) {
    if (!c->exec) rc = ctx_capture(c);
    for (int s = done; rc == MHD_OK && s < nsteps; ++s) {
      const hipError_t e = hipGraphLaunch(c->exec, c->stream);
      if (e != hipSuccess) rc = hip_fail(c, e, "hipGraphLaunch");
    }
  }
  if (rc == MHD_OK && nsteps > 0) {
    c->first_step = false;
    c->step += nsteps;
    c->t += nsteps * c->p.dt;
  }
  return rc;
}

size_t mhd_checkpoint_bytes(const mhd_ctx* c) {
  if (!c) return 0;
  return ckpt_layout(c).total;
}

int mhd_save(mhd_ctx* c, void* d_blob) {
  if (!c || !d_blob || (reinterpret_cast<uintptr_t>(d_blob) & 255u) != 0) return MHD_E_ARG;
  if (!c->has_state) return MHD_E_STATE;
  const CkptLayout B = ckpt_layout(c);
  CkptHeader h;
  std::memset(&h, 0, sizeof(h));
  std::memcpy(h.magic, "MHDCKPT", 8);
  h.version = kCkptVersion;
  h.n = c->p.n;
  h.precision = c->p.precision;
  h.first_step = c->first_step ? 1 : 0;
  h.step = c->step;
  h.t = c->t;
  h.dt = c->p.dt;
  h.payload_bytes = B.total - sizeof(CkptHeader);
  h.sc = (uint64_t)c->g.sc;
  char* blob = static_cast<char*>(d_blob);
  hipLaunchKernelGGL(k_write_header, dim3(1), dim3(64), 0, c->stream, h, reinterpret_cast<CkptHeader*>(blob));
  hipError_t e = hipMemcpyAsync(blob + B.state, c->ws + c->L.state, B.spec_bytes, hipMemcpyDeviceToDevice, c->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(blob + B.rprev, c->ws + c->L.rprev, B.spec_bytes, hipMemcpyDeviceToDevice, c->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(blob + B.status, c->ws + c->L.status, B.status_bytes, hipMemcpyDeviceToDevice, c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "mhd_save copy");
  blob_hash(c, blob, B.total, reinterpret_cast<unsigned long long*>(blob) + kCkptSumWord);
  return check_launch(c, "mhd_save");
}

int mhd_load(mhd_ctx* c, const void* d_blob) {
  if (!c || !d_blob || (reinterpret_cast<uintptr_t>(d_blob) & 255u) != 0) return MHD_E_ARG;
  const CkptLayout B = ckpt_layout(c);
  const char* blob = static_cast<const char*>(d_blob);
  CkptHeader h;
  unsigned long long* hash = reinterpret_cast<unsigned long long*>(c->ws + c->L.hash);
  hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(2), 0, c->stream, reinterpret_cast<unsigned*>(hash), 2, 0u);
  hipError_t e = hipMemcpyAsync(&h, blob, sizeof(h), hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "mhd_load header");
  if (std::memcmp(h.magic, "MHDCKPT", 8) != 0 || h.version != kCkptVersion ||
      h.payload_bytes != B.total - sizeof(CkptHeader) || h.sc != (uint64_t)c->g.sc)
    return MHD_E_STATE;
  blob_hash(c, blob, B.total, hash);
  unsigned long long sum = 0;
  e = hipGetLastError();
  if (e == hipSuccess) e = hipMemcpyAsync(&sum, hash, sizeof(sum), hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "mhd_load checksum");
  if (sum != h.checksum) return MHD_E_STATE;
  // a valid blob of another configuration
  if (h.n != c->p.n || h.precision != c->p.precision || h.dt != c->p.dt) return MHD_E_ARG;
  e = hipMemcpyAsync(c->ws + c->L.state, blob + B.state, B.spec_bytes, hipMemcpyDeviceToDevice, c->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(c->ws + c->L.rprev, blob + B.rprev, B.spec_bytes, hipMemcpyDeviceToDevice, c->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(c->ws + c->L.status, blob + B.status, B.status_bytes, hipMemcpyDeviceToDevice, c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "mhd_load copy");
  c->has_state = true;
  c->first_step = h.first_step != 0;
  c->step = h.step;
  c->t = h.t;
  return MHD_OK;
}

int mhd_diagnostics(mhd_ctx* c, mhd_diag* h) { return ctx_diag(c, h); }

int32_t mhd_spectra_shells(int32_t n) {
  if (n < 1) return 0;
  return spectrum_shells((n - 1) / 3);
}

int mhd_spectra(mhd_ctx* c, double* h_eu, double* h_eb, double* h_mom) {
  if (!c || !h_eu || !h_eb || !h_mom) return MHD_E_ARG;
  if (!c->has_state) return MHD_E_STATE;
  const Geo& g = c->g;
  const int nsh = spectrum_shells(g.K);
  const int nb = 2 * nsh + 1;
  double* shpart = reinterpret_cast<double*>(c->ws + c->L.shpart);
  double* shres = reinterpret_cast<double*>(c->ws + c->L.shres);
  int rc = with_engine(c, [&](auto& e) {
    using T = std::remove_pointer_t<decltype(e.state())>;
    e.phase_a(e.state());  // u^ = D F[m / rho] of the current state
    hipLaunchKernelGGL((k_spectra<T>), dim3(kSpecBlocks), dim3(kThreads), nb * sizeof(double), c->stream,
                       e.uhat(), e.spec_field(e.state(), 4), g, nsh, shpart);
    hipLaunchKernelGGL(k_reduce, dim3(nb), dim3(kThreads), 0, c->stream, shpart, (int64_t)kSpecBlocks, nb, 0u,
                       shpart, (int64_t)0, 0, shres, shres);
    // d = du_x/dx = F^-1[i k_x u^_x] on the grid, then its second and third moments
    const T* zi[1] = {e.uhat()};
    T* zo[1] = {e.iz(0)};
    OutSpec sp[1] = {spec({term(0, 0, e.inv_n3())})};
    e.col(PK_ZINV, 1, zi, 1, zo, sp);
    T* yo[1] = {e.iy(0)};
    e.y_copy(PK_YINV, 1, zo, yo);
    RowArgs<T> r = e.row_args();
    T* real = e.iy(4);
    r.real_out = real;
    r.real_dtype = sizeof(T) == 4 ? 1 : 0;
    r.nf = 1;
    e.set_in(r, 0);
    e.k.row(RM_XINV_REAL, r, e.row_grid(RM_XINV_REAL), c->stream);
    hipLaunchKernelGGL((k_moments<T>), dim3(kSpecBlocks), dim3(kThreads), 0, c->stream, real, g.n3, shpart);
    hipLaunchKernelGGL(k_reduce, dim3(2), dim3(kThreads), 0, c->stream, shpart, (int64_t)kSpecBlocks * kThreads, 2,
                       0u, shpart, (int64_t)0, 0, shres + nb, shres + nb);
    return check_launch(c, "mhd_spectra");
  });
  if (rc != MHD_OK) return rc;
  std::vector<double> res(nb + 2);
  hipError_t err = hipMemcpyAsync(res.data(), shres, (nb + 2) * sizeof(double), hipMemcpyDeviceToHost, c->stream);
  if (err == hipSuccess) err = hipStreamSynchronize(c->stream);
  if (err != hipSuccess) return hip_fail(c, err, "mhd_spectra copy");
  const double n3 = (double)g.n3, inv6 = 1.0 / (n3 * n3);
  for (int s = 0; s < nsh; ++s) {
    h_eu[s] = 0.5 * res[s] * inv6;
    h_eb[s] = 0.5 * res[nsh + s] * inv6;
  }
  const double m2 = res[nb] / n3, m3 = res[nb + 1] / n3;
  h_mom[0] = std::sqrt(res[2 * nsh] * inv6);
  h_mom[1] = m2 > 0 ? m3 / std::pow(m2, 1.5) : 0.0;
  h_mom[2] = std::sqrt(m2);
  return MHD_OK;
}

// Tracers: the real-space fields they need are synthesised from the state
// into the I_y scratch from slot 4 on (at most four fields: 4 n^3 words, at
// most 6 of the 12 free slots), behind the inverse transform's own slots 0-3.
int mhd_tracers_velocity(mhd_ctx* c, const double* d_pos, double* d_vel, int64_t np) {
  if (!c || np < 0 || (np > 0 && (!d_pos || !d_vel))) return MHD_E_ARG;
  if (!c->has_state) return MHD_E_STATE;
  if (np == 0) return MHD_OK;
  return with_engine(c, [&](auto& e) {
    using T = std::remove_pointer_t<decltype(e.state())>;
    T* real = e.iy(4);
    e.inverse_real(e.state(), 4, real, is_fp32(c->p.precision) ? MHD_FP32 : MHD_FP64);  // rho, m
    hipLaunchKernelGGL((k_tracer_velocity<T>), dim3((unsigned)((np + kThreads - 1) / kThreads)), dim3(kThreads), 0,
                       c->stream, real, c->g.n, d_pos, d_vel, np);
    return check_launch(c, "mhd_tracers_velocity");
  });
}

int mhd_tracers_push(mhd_ctx* c, double* d_pos, double* d_vel, int64_t np, double dt, int32_t nsteps) {
  if (!c || np < 0 || nsteps < 0 || !std::isfinite(dt) || (np > 0 && (!d_pos || !d_vel))) return MHD_E_ARG;
  if (!c->has_state) return MHD_E_STATE;
  if (np == 0 || nsteps == 0) return MHD_OK;
  return with_engine(c, [&](auto& e) {
    using T = std::remove_pointer_t<decltype(e.state())>;
    T* real = e.iy(4);
    e.inverse_real(e.spec_field(e.state(), 4), 3, real, is_fp32(c->p.precision) ? MHD_FP32 : MHD_FP64);  // B
    hipLaunchKernelGGL((k_tracer_push<T>), dim3((unsigned)((np + kThreads - 1) / kThreads)), dim3(kThreads), 0,
                       c->stream, real, c->g.n, d_pos, d_vel, np, dt, (int)nsteps);
    return check_launch(c, "mhd_tracers_push");
  });
}

int mhd_fft3d(mhd_ctx* c, int32_t dir, const void* d_in, void* d_out) {
  if (!c || !d_in || !d_out || (dir != 1 && dir != -1)) return MHD_E_ARG;
  return with_engine(c, [&](auto& e) {
    using T = std::remove_pointer_t<decltype(e.state())>;
    const int32_t rd = is_fp32(c->p.precision) ? MHD_FP32 : MHD_FP64;
    if (dir < 0) {
      e.forward_real(d_in, rd, 1, static_cast<T*>(d_out));
    } else {
      e.inverse_real(static_cast<const T*>(d_in), 1, d_out, rd);
    }
    return check_launch(c, "mhd_fft3d");
  });
}

int mhd_profile(mhd_ctx* c, int32_t class_mask) {
  if (!c) return MHD_E_ARG;
  if (class_mask) {
    constexpr int kCap = 4096;
    if (c->ev.empty()) {
      c->ev.resize(2 * kCap);
      for (auto& e : c->ev) {
        hipError_t err = hipEventCreate(&e);
        if (err != hipSuccess) return hip_fail(c, err, "mhd_profile");
      }
      c->rec_cls.assign(kCap, 0);
      c->rec_bytes.assign(kCap, 0.0);
    }
    c->nrec = 0;
    c->dropped = 0;
  }
  c->prof_on = class_mask != 0;
  c->prof_mask = (uint32_t)class_mask;
  return MHD_OK;
}

int mhd_profile_read(mhd_ctx* c, double* ms, int64_t* launches, double* bytes, int64_t* dropped) {
  if (!c) return MHD_E_ARG;
  hipError_t err = hipStreamSynchronize(c->stream);
  if (err != hipSuccess) return hip_fail(c, err, "mhd_profile_read");
  double m[MHD_PASS_COUNT] = {0}, b[MHD_PASS_COUNT] = {0};
  int64_t l[MHD_PASS_COUNT] = {0};
  for (int r = 0; r < c->nrec; ++r) {
    float e = 0.f;
    err = hipEventElapsedTime(&e, c->ev[2 * r], c->ev[2 * r + 1]);
    if (err != hipSuccess) return hip_fail(c, err, "mhd_profile_read elapsed");
    const int cls = c->rec_cls[r];
    m[cls] += e;
    b[cls] += c->rec_bytes[r];
    l[cls] += 1;
  }
  for (int i = 0; i < MHD_PASS_COUNT; ++i) {
    if (ms) ms[i] = m[i];
    if (launches) launches[i] = l[i];
    if (bytes) bytes[i] = b[i];
  }
  if (dropped) *dropped = c->dropped;
  return MHD_OK;
}

double mhd_step_bytes(const mhd_ctx* cc) {
  if (!cc) return 0.0;
  mhd_ctx* c = const_cast<mhd_ctx*>(cc);
  double b = 0.0;
  with_engine(c, [&](auto& e) { b = e.step_bytes(); return MHD_OK; });
  return b;
}

int mhd_destroy(mhd_ctx* c) {
  if (!c) return MHD_OK;
  for (auto& e : c->ev) (void)hipEventDestroy(e);
  if (c->exec) (void)hipGraphExecDestroy(c->exec);
  if (c->graph) (void)hipGraphDestroy(c->graph);
  if (c->cap) (void)hipStreamDestroy(c->cap);
  delete c;
  return MHD_OK;
}

const char* mhd_status_string(int s) {
  switch (s) {
    case MHD_OK: return "ok";
    case MHD_E_ARG: return "invalid argument";
    case MHD_E_SIZE: return "unsupported grid size for this precision";
    case MHD_E_WORKSPACE: return "workspace missing, misaligned or too small";
    case MHD_E_HIP: return "HIP runtime error";
    case MHD_E_NONFINITE: return "non-finite value in the state";
    case MHD_E_CFL: return "time step above the CFL limit";
    case MHD_E_STATE: return "no state set";
    default: return "unknown status";
  }
}

const char* mhd_last_error(const mhd_ctx* c) { return c ? c->last_err.c_str() : ""; }

int mhd_bench_copy(const void* d_src, void* d_dst, size_t bytes, void* hip_stream) {
  if (!d_src || !d_dst || bytes % 16 != 0 || (reinterpret_cast<uintptr_t>(d_src) & 15u) ||
      (reinterpret_cast<uintptr_t>(d_dst) & 15u))
    return MHD_E_ARG;
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
    return MHD_E_HIP;
  const int64_t words = (int64_t)(bytes / 16);
  int64_t blocks = (int64_t)cus * 4;  // four 256-thread workgroups per CU
  const int64_t need = (words + kThreads - 1) / kThreads;
  if (blocks > need) blocks = need < 1 ? 1 : need;
  hipLaunchKernelGGL(k_stream_copy, dim3((unsigned)blocks), dim3(kThreads), 0, static_cast<hipStream_t>(hip_stream),
                     static_cast<const uint4*>(d_src), static_cast<uint4*>(d_dst), words);
  return hipGetLastError() == hipSuccess ? MHD_OK : MHD_E_HIP;
}

size_t mhd_ens_workspace_bytes(const mhd_params* p, int32_t count) {
  if (!p || count < 1) return 0;
  for (int i = 0; i < count; ++i)
    if (validate_member(&p[i]) != MHD_OK) return 0;
  std::vector<EnsGroup> groups;
  std::vector<int> grp_of;
  return ens_plan(p, count, groups, grp_of);
}

int mhd_ens_init(const mhd_params* p, int32_t count, void* d_workspace, size_t ws_bytes, void* hip_stream,
                 const char* tune_cache_path, mhd_ens** out) {
  if (!out) return MHD_E_ARG;
  *out = nullptr;
  if (!p || count < 1) return MHD_E_ARG;
  for (int i = 0; i < count; ++i) {
    const int v = validate_member(&p[i]);
    if (v != MHD_OK) return v;
  }
  mhd_ens* E = new (std::nothrow) mhd_ens();
  if (!E) return MHD_E_ARG;
  E->count = count;
  E->stream = static_cast<hipStream_t>(hip_stream);
  const size_t need = ens_plan(p, count, E->groups, E->grp_of);
  if (!d_workspace || ws_bytes < need || (reinterpret_cast<uintptr_t>(d_workspace) & 255u) != 0) {
    delete E;
    return MHD_E_WORKSPACE;
  }
  if (!tune_cache_path) E->tune_mode = 1;
  else if (tune_cache_path[0] == '\0') E->tune_mode = 0;
  else {
    E->tune_mode = 2;
    E->tune_path = tune_cache_path;
  }
  E->mem.assign(count, nullptr);
  char* base = static_cast<char*>(d_workspace);
  int rc = MHD_OK;
  for (EnsGroup& G : E->groups) {
    G.base = base;
    for (size_t s = 0; s < G.members.size() && rc == MHD_OK; ++s) {
      const int i = G.members[s];
      rc = ctx_create(&p[i], base + s * G.stride, G.stride, E->stream, &E->mem[i]);
    }
    base += G.stride * G.members.size();
    if (rc != MHD_OK) break;
    hipError_t e = hipStreamCreateWithFlags(&G.stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&G.done, hipEventDisableTiming);
    if (e != hipSuccess) {
      rc = ens_fail(E, e, "mhd_ens_init streams");
      break;
    }
    G.lead = new (std::nothrow) mhd_ctx(*E->mem[G.members[0]]);
    if (!G.lead) {
      rc = MHD_E_ARG;
      break;
    }
    G.lead->stream = G.stream;
    G.lead->ev.clear();  // the lead shares no events, graph or stream with member 0
    G.lead->cap = nullptr;
    G.lead->graph = nullptr;
    G.lead->exec = nullptr;
  }
  if (rc == MHD_OK) {
    hipError_t e = hipStreamCreateWithFlags(&E->cap, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&E->fork, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreate(&E->t0);
    if (e == hipSuccess) e = hipEventCreate(&E->t1);
    if (e != hipSuccess) rc = ens_fail(E, e, "mhd_ens_init events");
  }
  if (rc != MHD_OK) {
    ens_free(E);
    return rc;
  }
  E->num_cus = E->mem[0]->num_cus;
  if (E->tune_mode == 0)
    for (EnsGroup& G : E->groups) G.tuned = true;
  if (E->tune_mode == 2) tune_read(E);
  *out = E;
  return MHD_OK;
}

int mhd_ens_set_state(mhd_ens* E, int32_t member, const void* d_fields, int32_t dtype) {
  if (!E || member < 0 || member >= E->count) return MHD_E_ARG;
  return mhd_set_state(E->mem[member], d_fields, dtype);
}

int mhd_ens_get_state(mhd_ens* E, int32_t member, void* d_fields, int32_t dtype) {
  if (!E || member < 0 || member >= E->count) return MHD_E_ARG;
  return mhd_get_state(E->mem[member], d_fields, dtype);
}

int mhd_ens_step(mhd_ens* E, int32_t nsteps) {
  if (!E || nsteps < 0) return MHD_E_ARG;
  for (mhd_ctx* c : E->mem)
    if (!c->has_state) return MHD_E_STATE;
  if (nsteps == 0) return MHD_OK;
  bool untuned = false;
  for (const EnsGroup& G : E->groups) untuned = untuned || !G.tuned;
  if (untuned) {
    const int rc = ens_tune(E);
    if (rc != MHD_OK) return rc;
  }
  for (int s = 0; s < nsteps; ++s) {
    bool any_first = false;
    for (const mhd_ctx* c : E->mem) any_first = any_first || c->first_step;
    if (any_first) {
      const int rc = ens_launch(E, E->stream, false);
      if (rc != MHD_OK) return rc;
      for (mhd_ctx* c : E->mem) c->first_step = false;
    } else {
      if (!E->exec) {
        const int rc = ens_capture(E);
        if (rc != MHD_OK) return rc;
      }
      const hipError_t e = hipGraphLaunch(E->exec, E->stream);
      if (e != hipSuccess) return ens_fail(E, e, "hipGraphLaunch");
    }
    for (mhd_ctx* c : E->mem) {
      c->step += 1;
      c->t += c->p.dt;
    }
  }
  return MHD_OK;
}

int mhd_ens_diagnostics(mhd_ens* E, mhd_diag* h_out, int32_t* h_status) {
  if (!E || !h_out) return MHD_E_ARG;
  int first_bad = MHD_OK;
  for (int i = 0; i < E->count; ++i) {
    const int rc = ctx_diag(E->mem[i], &h_out[i]);
    if (h_status) h_status[i] = rc;
    if (rc == MHD_E_HIP) {
      E->last_err = E->mem[i]->last_err;
      return rc;
    }
    if (rc != MHD_OK && first_bad == MHD_OK) first_bad = rc;
  }
  return first_bad;
}

int32_t mhd_ens_num_groups(const mhd_ens* E) { return E ? (int32_t)E->groups.size() : 0; }

int mhd_ens_group_info(const mhd_ens* E, int32_t g, int32_t* n, int32_t* precision, int32_t* members,
                       double* col_scale, double* row_scale, int32_t* schedule) {
  if (!E || g < 0 || g >= (int32_t)E->groups.size()) return MHD_E_ARG;
  const EnsGroup& G = E->groups[g];
  if (n) *n = G.n;
  if (precision) *precision = G.precision;
  if (members) *members = (int32_t)G.members.size();
  if (col_scale) *col_scale = G.col_scale;
  if (row_scale) *row_scale = G.row_scale;
  if (schedule) *schedule = G.sched;
  return MHD_OK;
}

double mhd_ens_step_bytes(const mhd_ens* E) {
  if (!E) return 0.0;
  double b = 0.0;
  for (const mhd_ctx* c : E->mem) b += mhd_step_bytes(c);
  return b;
}

int mhd_ens_destroy(mhd_ens* E) {
  ens_free(E);
  return MHD_OK;
}

const char* mhd_ens_last_error(const mhd_ens* E) { return E ? E->last_err.c_str() : ""; }

}  // extern "C"

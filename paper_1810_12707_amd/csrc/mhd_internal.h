// Internal definitions shared by the HIP kernels and the host side of libmhd.
//
// Data layout in HBM (per field, working precision T, complex = interleaved
// (re, im) pairs; K = (n-1)/3, nh = K+1, nb = 2K+1, nhp = nh rounded up to a
// multiple of 8 so that every kx row starts on a 64-byte boundary):
//   compact spectrum S  [kz: nb][ky: nb][kx: nhp]  (state, history, u^)
//   z-pass intermediate [z: n][ky: nb][kx: nhp]    ("I_z")
//   y-pass intermediate [z: n][y: n][kx: nhp]      ("I_y")
// Entries with kx >= nh are padding: never read, never written.
// Band indices run 0..K then -K..-1; along a length-n axis, band index l sits
// at position l (l <= K) or l + n - nb (l > K).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

// Kernel schedules.  The pass kernels (mhd_fft.h, mhd_kernels.h) are compiled
// once per grid size with the default schedule and, for the ensemble sizes,
// once more with the alternative schedule (MHD_SCHED = 1: other radix plans
// and narrower column tiles).  Each build lives in its own inline namespace,
// so the two sets of template instances never collide at link time.
#ifndef MHD_SCHED
#define MHD_SCHED 0
#endif
#if MHD_SCHED == 1
#define MHD_SCHED_BEGIN inline namespace sched1 {
#else
#define MHD_SCHED_BEGIN inline namespace sched0 {
#endif
#define MHD_SCHED_END }

namespace mhd {

constexpr int kThreads = 256;  // threads per workgroup of every pass kernel
constexpr int kMaxTerms = 3;   // terms of one spectral linear combination
constexpr int kMaxOut = 12;    // outputs of one column launch
constexpr int kMaxIn = 12;     // inputs of one column launch
constexpr int kRowFields = 16; // fields held by one row (x) pass
constexpr int kDiagQ = 14;     // diagnostic partial sums per block
constexpr int kDiagFields = 9;  // real-space inputs of the diagnostics pass: the state and div B
constexpr int kSpecQ = 3;      // spectral diagnostic partial sums per block
constexpr int kStatusSlots = 2048;  // per-workgroup status slots of the flux pass (grid is capped to this)

// Index of each real-space diagnostic partial.
enum DiagQ {
  DQ_RHO = 0, DQ_MX, DQ_MY, DQ_MZ, DQ_EKIN, DQ_EMAG, DQ_P, DQ_E, DQ_HC,
  DQ_UABS, DQ_BABS, DQ_DIVB_MAX, DQ_CFL_MAX, DQ_NONFINITE
};
// Index of each spectral diagnostic partial.
enum SpecQ { SQ_HM = 0, SQ_DIVB2, SQ_J2 };

// One term of out = sum_t coef_t * (i k_{axis_t} or 1) * in[src_t].
struct Term {
  int32_t src;   // input slot
  int32_t axis;  // -1: no derivative; 0: x; 1: y; 2: z
  double coef;
};

struct OutSpec {
  int32_t nterms;
  int32_t pad;
  Term t[kMaxTerms];
};

enum PassKind { PK_ZINV = 0, PK_YINV = 1, PK_YFWD = 2, PK_ZFWD = 3 };

struct Geo {
  int32_t n, K, nh, nb;
  int32_t nhp;  // kx pitch: nh rounded up to a multiple of 8
  int64_t sc;  // complex values per compact spectrum
  int64_t iz;  // complex values per I_z field
  int64_t iy;  // complex values per I_y field
  int64_t n3;  // real values per field
};

// Members of an ensemble that share a grid size are run by one launch per
// pass: member m's arrays sit at byte offset m * mstride from member 0's.
constexpr int kMaxMem = 64;
struct Batch {
  int32_t nmem;     // members in this launch (1 for a single context)
  int32_t pad;
  int64_t mstride;  // bytes between consecutive members' workspaces
};

// Byte arithmetic on a char pointer (not an integer round trip) keeps the
// pointer's provenance, so the compiler still emits global (not flat) memory
// instructions through the result.
template <typename P>
__host__ __device__ __forceinline__ P* member_ptr(P* p, int m, int64_t stride) {
  using B = typename std::conditional<std::is_const<P>::value, const char, char>::type;
  return reinterpret_cast<P*>(reinterpret_cast<B*>(p) + (int64_t)m * stride);
}

template <typename T>
struct ColArgs {
  const T* in[kMaxIn];  // complex arrays (interleaved) in the pass's input layout
  T* out[kMaxOut];
  OutSpec spec[kMaxOut];
  const T* tw;          // n twiddles exp(-2 pi i j / n), interleaved
  int32_t kind;         // PassKind
  int32_t nout;
  Geo g;
  Batch bt;
};

// Forward-z pass that forms the right-hand side (Eqs. MHD2-MHD4 in spectral
// form) and applies the AB2 update.  Output f = 1..7 is
//   R_f = F_z[A_f] + i kz F_z[Z_f] - eta |k|^2 B^_f (f = 4, 5, 6),
// with A_f, Z_f combinations of the y-transformed fluxes.  The density pass
// (Eq. MHD1, R_rho = -i k.m^) takes the same arguments.
template <typename T>
struct RhsArgs {
  const T* flux[kMaxIn];  // I_z flux slots
  OutSpec A[8];
  OutSpec Z[8];
  T* state;               // compact [8][sc]
  T* rprev;               // compact [8][sc] (R^{n-1}, overwritten with R^n)
  T* rout;                // if non-null: store R here, leave state/rprev untouched
  const T* tw;
  // Section V variants (single runs only, so scalars): mu != 0 adds the
  // viscous force -mu |k|^2 u^ to R_m and -mu |k|^2 q^ to R_E, q = |u|^2/2,
  // from uhat [4][sc] (u^x, u^y, u^z, q^); force: [4][sc] body-force spectra
  // added to R_m and R_E, or null; kinematic: R_rho, R_m, R_E are zero
  const T* uhat;
  const T* force;
  double mu;
  int32_t kinematic;
  int32_t pad2;
  Geo g;
  Batch bt;
  // per member: time step, AB2 coefficients of R^n and R^{n-1}, diffusivity
  double dt[kMaxMem], a_cur[kMaxMem], a_prev[kMaxMem], eta[kMaxMem];
};

enum RowMode { RM_XA = 0, RM_XB = 1, RM_XFWD_REAL = 2, RM_XINV_REAL = 3, RM_XDIAG = 4 };

template <typename T>
struct RowArgs {
  const T* in0;             // first input I_y slot (complex); field f at in0 + 2 f in_stride
  int64_t in_stride;        // complex values between consecutive input fields
  T* out0;                  // first output I_y slot
  int64_t out_stride;
  const void* real_in;      // [nf][n^3] real rows (RM_XFWD_REAL)
  void* real_out;           // [nf][n^3] real rows (RM_XINV_REAL)
  int32_t real_dtype;       // 0 = double, 1 = float
  int32_t nf;               // fields of an I/O pass
  double* partials;         // per-block records (RM_XDIAG, single member)
  double* status;           // RM_XB: status slots [kStatusSlots][2] (max signal speed, non-finite
                            // count), slot = workgroup id; null: no status (pure RHS evaluations)
  const T* tw;
  Geo g;
  Batch bt;
  double gamma[kMaxMem], nu[kMaxMem], eta[kMaxMem];  // per member
};

}  // namespace mhd

// Instantiates every pass kernel for one grid size N = MHD_N, both precisions
// (FP64 only up to N = 512, where the row pass's LDS footprint still fits).
#include "mhd_kernels.h"
#include "mhd_registry.h"

#ifndef MHD_N
#error "compile with -DMHD_N=<grid size>"
#endif

namespace mhd {
namespace {

// Column passes: one instantiation per direction, term count and axis (z or y).
template <typename T, int N, int S, int MAXT, bool MX>
void col_launch(const ColArgs<T>& a, dim3 g, hipStream_t s) {
  constexpr int nt = col_threads<T, N, MX, S, MAXT>();
  if (a.kind == PK_ZINV || a.kind == PK_ZFWD) hipLaunchKernelGGL((k_col<T, N, S, MAXT, MX, true>), g, dim3(nt), 0, s, a);
  else hipLaunchKernelGGL((k_col<T, N, S, MAXT, MX, false>), g, dim3(nt), 0, s, a);
}
template <typename T, int N, bool MX>
void col_inv(int maxt, const ColArgs<T>& a, dim3 g, hipStream_t s) {
  if (maxt <= 1) col_launch<T, N, 1, 1, MX>(a, g, s);
  else col_launch<T, N, 1, kMaxTerms, MX>(a, g, s);
}
template <typename T, int N, bool MX>
void col_fwd(const ColArgs<T>& a, dim3 g, hipStream_t s) {
  col_launch<T, N, -1, 1, MX>(a, g, s);
}
// Resident workgroups per CU of a column-pass class: the smaller of its z and
// y instantiations (the persistent grid is sized once per class).
template <typename T, int N, int S, int MAXT, bool MX>
int col_occ(void) {
  constexpr int nt = col_threads<T, N, MX, S, MAXT>();
  int bz = 0, by = 0;
  const hipError_t ez = hipOccupancyMaxActiveBlocksPerMultiprocessor(&bz, k_col<T, N, S, MAXT, MX, true>, nt, 0);
  const hipError_t ey = hipOccupancyMaxActiveBlocksPerMultiprocessor(&by, k_col<T, N, S, MAXT, MX, false>, nt, 0);
  if (ez != hipSuccess || ey != hipSuccess) return 1;
  const int b = bz < by ? bz : by;
  return b > 0 ? b : 1;
}
template <typename T, int N, bool MX>
int col_occupancy(int dir, int maxt) {
  if (dir < 0) return col_occ<T, N, -1, 1, MX>();
  if (maxt <= 1) return col_occ<T, N, 1, 1, MX>();
  return col_occ<T, N, 1, kMaxTerms, MX>();
}
template <typename T, int N, bool MX>
void rhs(const RhsArgs<T>& a, dim3 g, hipStream_t s) {
  hipLaunchKernelGGL((k_zfwd_rhs<T, N, MX>), g, dim3(rhs_threads<T, N, MX>()), 0, s, a);
}
template <typename T, int N, bool MX>
void row(int mode, const RowArgs<T>& a, dim3 g, hipStream_t s) {
  switch (mode) {
    case RM_XA: hipLaunchKernelGGL((k_row<T, N, RM_XA, MX>), g, dim3(row_threads<T, N, RM_XA, MX>()), 0, s, a); break;
    case RM_XB: hipLaunchKernelGGL((k_row<T, N, RM_XB, MX>), g, dim3(row_threads<T, N, RM_XB, MX>()), 0, s, a); break;
    case RM_XFWD_REAL: hipLaunchKernelGGL((k_row<T, N, RM_XFWD_REAL, MX>), g, dim3(row_threads<T, N, RM_XFWD_REAL, MX>()), 0, s, a); break;
    case RM_XINV_REAL: hipLaunchKernelGGL((k_row<T, N, RM_XINV_REAL, MX>), g, dim3(row_threads<T, N, RM_XINV_REAL, MX>()), 0, s, a); break;
    case RM_XDIAG: hipLaunchKernelGGL((k_row<T, N, RM_XDIAG, MX>), g, dim3(row_threads<T, N, RM_XDIAG, MX>()), 0, s, a); break;
    default: break;
  }
}

template <typename T, int N, bool MX>
int row_occupancy(int mode) {
  int blocks = 0;
  hipError_t e = hipSuccess;
  switch (mode) {
    case RM_XA: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k_row<T, N, RM_XA, MX>,
                                                     row_threads<T, N, RM_XA, MX>(), 0); break;
    case RM_XB: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k_row<T, N, RM_XB, MX>,
                                                     row_threads<T, N, RM_XB, MX>(), 0); break;
    case RM_XFWD_REAL:
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k_row<T, N, RM_XFWD_REAL, MX>,
                                                     row_threads<T, N, RM_XFWD_REAL, MX>(), 0);
      break;
    case RM_XINV_REAL:
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k_row<T, N, RM_XINV_REAL, MX>,
                                                     row_threads<T, N, RM_XINV_REAL, MX>(), 0);
      break;
    case RM_XDIAG: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k_row<T, N, RM_XDIAG, MX>,
                                                     row_threads<T, N, RM_XDIAG, MX>(), 0); break;
    default: break;
  }
  return (e == hipSuccess && blocks > 0) ? blocks : 1;
}

template <typename T, int N, bool MX>
Kern<T> make() {
  Kern<T> k;
  k.n = N;
  k.col_width = col_tile<T, N, MX>();
  k.rhs_width = rhs_tile<T, N, MX>();
  k.col_inv = col_inv<T, N, MX>;
  k.col_fwd = col_fwd<T, N, MX>;
  k.rhs = rhs<T, N, MX>;
  k.row = row<T, N, MX>;
  k.row_occupancy = row_occupancy<T, N, MX>;
  k.col_occupancy = col_occupancy<T, N, MX>;
  return k;
}

}  // namespace

#define MHD_CAT2(a, b) a##b
#define MHD_CAT(a, b) MHD_CAT2(a, b)
#if MHD_SCHED == 1
// the alternative schedule: FP32 only
void MHD_CAT(register_s1_, MHD_N)(Registry& r) { r.f32s1[MHD_N] = make<float, MHD_N, false>(); }
#else
void MHD_CAT(register_, MHD_N)(Registry& r) {
  r.f32[MHD_N] = make<float, MHD_N, false>();
  r.mx[MHD_N] = make<float, MHD_N, true>();
#if MHD_N <= 512
  r.f64[MHD_N] = make<double, MHD_N, false>();
#endif
}
#endif

}  // namespace mhd

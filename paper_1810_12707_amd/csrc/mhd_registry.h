// Per-grid-size kernel launchers, filled in by one translation unit per size
// (mhd_inst.hip compiled with -DMHD_N=<n>).
#pragma once

#include "mhd_internal.h"

namespace mhd {

template <typename T>
struct Kern {
  int n = 0;
  int col_width = 0;  // columns per work item of the column passes
  int rhs_width = 0;  // columns per workgroup of the forward-z RHS pass
  // column passes; maxt = largest number of terms of any output spec (1 or 3)
  void (*col_inv)(int maxt, const ColArgs<T>&, dim3, hipStream_t) = nullptr;
  void (*col_fwd)(const ColArgs<T>&, dim3, hipStream_t) = nullptr;
  int (*col_occupancy)(int dir, int maxt) = nullptr;
  void (*rhs)(const RhsArgs<T>&, dim3, hipStream_t) = nullptr;
  void (*row)(int mode, const RowArgs<T>&, dim3, hipStream_t) = nullptr;
  // resident workgroups per CU of a row-pass mode (persistent grid sizing)
  int (*row_occupancy)(int mode) = nullptr;
};

struct Registry {
  Kern<float> f32[1025];
  Kern<double> f64[1025];
  Kern<float> mx[1025];    // FP32 data, radix-16 stages on MFMA (split BF16 x 3)
  Kern<float> f32s1[1025];  // FP32, alternative schedule (ensemble sizes)
};

Registry& registry();

#define MHD_SIZES(X) X(8) X(12) X(16) X(24) X(32) X(48) X(64) X(96) X(128) X(192) X(256) X(384) X(512) X(768) X(1024)
#define MHD_DECLARE_REGISTER(NN) void register_##NN(Registry&);
MHD_SIZES(MHD_DECLARE_REGISTER)
#undef MHD_DECLARE_REGISTER

// Sizes with an alternative-schedule build (the batched ensemble's sizes).
#define MHD_SCHED1_SIZES(X) X(32) X(64) X(96) X(128)
#define MHD_DECLARE_REGISTER_S1(NN) void register_s1_##NN(Registry&);
MHD_SCHED1_SIZES(MHD_DECLARE_REGISTER_S1)
#undef MHD_DECLARE_REGISTER_S1

}  // namespace mhd

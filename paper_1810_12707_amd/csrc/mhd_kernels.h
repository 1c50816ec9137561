// Pass kernels of the pseudo-spectral MHD right-hand side, templated on the
// working precision T and the grid size N.
//
// Column passes (k_col, k_zfwd_rhs) transform along z or y for a tile of C
// adjacent columns (the contiguous kx or (ky, kx) index), so every global
// access is a run of C consecutive complex values; the tile sits in LDS as
// [N][C].  Row passes (k_row) own two adjacent x rows (z, y) and (z, y+1) of
// every field they touch: the two real rows of one field are packed as one
// complex sequence (row0 + i row1), so one length-N complex FFT does two real
// transforms, and all fields of a row pair are resident in LDS at once for the
// pointwise work.
#pragma once

#include "mhd_fft.h"
#include "mhd_internal.h"

namespace mhd {
MHD_SCHED_BEGIN

template <int N> struct Band {
  static constexpr int K = (N - 1) / 3;
  static constexpr int NH = K + 1;
  static constexpr int NB = 2 * K + 1;
  static constexpr int NHP = (NH + 7) / 8 * 8;  // kx pitch of every layout (64-byte rows)
};

// Position of band index l on a length-N axis, and its wavenumber.
template <int N> __device__ __forceinline__ int band_pos(int l) { return l <= Band<N>::K ? l : l + N - Band<N>::NB; }
template <int N> __device__ __forceinline__ int band_k(int l) { return l <= Band<N>::K ? l : l - Band<N>::NB; }

// Default column tile: 16 columns while the LDS tile stays within 32 KiB,
// else 8.  The alternative schedule takes 8-column tiles (twice the work
// items, half the LDS per workgroup).
template <typename T, int N> constexpr int col_width() {
  constexpr int bytes = N * 2 * (int)sizeof(T);
  if (MHD_SCHED == 1) return 8;
  return 32768 / bytes >= 16 ? 16 : 8;
}

// Threads and tile width of the forward-z RHS pass.  It is latency-bound
// (dependent memory phases per workgroup: the first flux group, the second,
// the state and history), so it wants many resident waves: FP32 at N >= 256
// runs one first-pass butterfly per thread, which keeps registers low -- 512
// threads on 16 columns at N = 256, 1024 threads on 16 columns at N = 512
// (whole 128-byte row segments; 3% faster than 512 threads on 8), 1024
// threads on 8 columns at N = 1024 (FP32 228 -> 106 registers, mixed 196 ->
// 116: four waves per SIMD instead of two, 28.0 -> 21.4 and 35.4 -> 24.0 ms
// per step), and 512 threads on 8 columns for the mixed path below that.
// FP64 at N = 512 takes 512 threads on its 8-column tiles, one butterfly
// each (146 registers instead of 256 with 256 threads, three waves per SIMD
// instead of one: 6.89 -> 4.35 ms per step).
template <typename T, int N, bool MX> constexpr bool rhs_wide() { return sizeof(T) == 4 && N >= 256; }
template <typename T, int N, bool MX> constexpr int rhs_threads() {
  if (sizeof(T) == 8 && N == 512) return 2 * kThreads;
  if (sizeof(T) == 4 && ((!MX && N == 512) || N == 1024)) return 4 * kThreads;
  return rhs_wide<T, N, MX>() ? 2 * kThreads : kThreads;
}
template <typename T, int N, bool MX> constexpr int rhs_tile() {
  if (sizeof(T) == 4 && !MX && N == 512) return 16;
  return rhs_wide<T, N, MX>() ? (N == 256 ? 16 : 8) : col_width<T, N>();
}
// Minimum resident waves per SIMD asked of the compiler (register cap).
template <typename T, int N, bool MX> constexpr int rhs_min_waves() {
  return rhs_wide<T, N, MX>() || (sizeof(T) == 8 && N == 512) ? 1 : 3;
}

// Threads and tile width of the column passes (S = +1 inverse, -1 forward;
// MAXT input terms per element).  Long FP32 columns take 16-column tiles, so
// that every row segment is a whole 128-byte line (8 FP32 columns would read
// half lines, whose other halves another workgroup reads later, often after
// eviction), and enough threads that each holds one or two first-pass
// butterflies.  Measured per pass class: one butterfly per thread (fewer
// registers, more resident waves) pays for the inverse passes at N = 256 and
// 512 and for the forward passes at N = 512; the forward passes at N = 256
// run best with two.  At N = 1024 the passes take 8-column tiles with 1024
// threads, one first-pass butterfly each (98-126 registers, four waves per
// SIMD; with 512 threads they held 162-222 and ran two: 8-15% slower per
// pass, FP32 and mixed).  FP64 at N = 512 (8-column tiles) takes 512 threads,
// one butterfly each (144-202 registers instead of 242-256 and one wave per
// SIMD with 256 threads; the three-term pass 3.02 -> 2.38 ms per step), other
// FP64 sizes 256.  The MFMA variant follows the FP32 rule from N = 256 up
// (its one-term inverse passes at 256 hold 112 registers with 512 threads,
// 180 with 256: 8-12% faster) and keeps 256 threads below.
template <typename T, int N, bool MX, int S, int MAXT> constexpr int col_threads() {
  if (sizeof(T) == 8 && N == 512) return 2 * kThreads;
  if (sizeof(T) != 4 || (MX && N < 256)) return kThreads;
  if (N == 256) return (MAXT > 1 || S > 0) ? 2 * kThreads : kThreads;
  if (N == 512 || N == 1024) return 4 * kThreads;
  return N > 512 ? 2 * kThreads : kThreads;
}
template <typename T, int N, bool MX> constexpr int col_tile() {
  return (sizeof(T) == 4 && N >= 256 && N <= 512) ? 16 : col_width<T, N>();
}

template <typename T>
__device__ __forceinline__ cx<T> ld(const T* base, int64_t idx) {
  return reinterpret_cast<const cx<T>*>(base)[idx];
}
template <typename T>
__device__ __forceinline__ void st(T* base, int64_t idx, cx<T> v) {
  reinterpret_cast<cx<T>*>(base)[idx] = v;
}

template <typename T, int N, int NT = kThreads>
__device__ __forceinline__ void load_twiddles(cx<T>* stw, const T* tw, int tid) {
  for (int i = tid; i < N; i += NT) stw[i] = ld(tw, i);
}

// Band index of position q on a length-N axis, or -1 in the dropped gap.
template <int N> __device__ __forceinline__ int pos_band(int q) {
  return q <= Band<N>::K ? q : (q >= N - Band<N>::K ? q - N + Band<N>::NB : -1);
}

// Decode a flat workgroup id into (tile, field) with the field fastest, after
// the XCD remap: the outputs of one column tile run back to back on one XCD and
// share the L2 copies of the inputs they have in common.
struct TileField {
  int tile, field;
};
__device__ __forceinline__ TileField tile_field(int nfields) {
  const int L = xcd_remap(blockIdx.x, gridDim.x);
  TileField t;
  t.tile = L / nfields;
  t.field = L - t.tile * nfields;
  return t;
}

// ------------------------------------------------------------------ k_col
// S = +1: inverse pass, band (nb) in -> N out.  S = -1: forward, N in -> band out.
// Persistent: items (outer, tile, field), field fastest, walked in XCD-blocked
// order (xcd_item), so the outputs of one tile -- which share inputs -- run
// together on one XCD.  The first FFT pass reads its inputs from registers
// that were loaded from HBM while the previous item was being transformed
// (up to MAXT input terms per element; the zero gap of a band input is never
// loaded); the last pass stores straight to HBM (dropped modes skipped).
// Z: a z pass (else a y pass), fixed at compile time so that the column
// geometry, the strides and the wavenumbers of the multipliers are constants
// rather than uniform branches per element.
template <typename T, int N, int S, int MAXT, bool MX, bool Z>
__global__ void __launch_bounds__((col_threads<T, N, MX, S, MAXT>())) k_col(const ColArgs<T> a) {
  using PL = PlanOf<N, MX>;
  constexpr int C = col_tile<T, N, MX>();
  constexpr int NT = col_threads<T, N, MX, S, MAXT>();
  constexpr int NH = Band<N>::NH, NHP = Band<N>::NHP, NBB = Band<N>::NB;
  using FP = FirstPass<PL, C, NT>;
  __shared__ cx<T> tile[N * C];
  __shared__ cx<T> stw[N];
  const int tid = threadIdx.x;
  constexpr bool zpass = Z;
  // z passes: columns are (ky, kx) flattened over the padded pitch; padding
  // columns (kx >= NH) are never read or written
  constexpr int ncols = zpass ? NBB * NHP : NH;
  constexpr int ntiles = (ncols + C - 1) / C;
  const int per_mem = ntiles * (zpass ? 1 : N) * a.nout;
  const int total = per_mem * a.bt.nmem;  // < 2^31 for every supported size and member count
  // strides (complex elements) of the input and output layouts: z passes
  // (either direction) map [kz][ky][kx] onto itself; the inverse y pass reads
  // [kz][ky band][kx] and writes [kz][y][kx], the forward one the reverse
  constexpr int64_t os_in = zpass ? 0 : (S > 0 ? (int64_t)NBB * NHP : (int64_t)N * NHP);
  constexpr int64_t ls_in = zpass ? (int64_t)NBB * NHP : NHP;
  constexpr int64_t os_out = zpass ? 0 : (S > 0 ? (int64_t)N * NHP : (int64_t)NBB * NHP);
  constexpr int64_t ls_out = ls_in;
  load_twiddles<T, N, NT>(stw, a.tw, tid);
  auto col_ok = [&](int col) { return col < ncols && (!zpass || col - (col / NHP) * NHP < NH); };

  struct Item {
    int m, f, outer, c0;
  };
  auto decode = [&](int item) {
    Item it;
    it.m = item / per_mem;
    const int rest = item - it.m * per_mem;
    const int t = rest / a.nout;
    it.f = rest - t * a.nout;
    it.outer = t / ntiles;
    it.c0 = (t - it.outer * ntiles) * C;
    return it;
  };
  // raw first-pass loads of one item, one set per input term
  cx<T> px[MAXT][FP::CNT][FP::R];
  auto issue = [&](const Item& it) {
    // the item's input pointers, once per item (uniform: scalar registers)
    // rather than once per element under the element's predicate
    const OutSpec& sp = a.spec[it.f];
    const int nt = sp.nterms;
    const T* src[MAXT];
#pragma unroll
    for (int t = 0; t < MAXT; ++t) src[t] = member_ptr(a.in[t < nt ? sp.t[t].src : 0], it.m, a.bt.mstride);
    const int64_t base_in = it.outer * os_in + it.c0;
#pragma unroll
    for (int i = 0; i < FP::CNT; ++i) {
      const int w = tid + i * NT;
      int c, j;
      lane_map<C, FP::NBF, 0>(w, c, j);
      const bool ok = (FP::TOT % NT == 0 || w < FP::TOT) && col_ok(it.c0 + c);
#pragma unroll
      for (int r = 0; r < FP::R; ++r) {
        const int q = j + r * FP::NBF;
        const int l = S > 0 ? pos_band<N>(q) : q;
        // the previous item's values are dead: say so, so that the compiler
        // need not keep them (and wait on loads in flight) when a load below
        // is predicated off
#pragma unroll
        for (int t = 0; t < MAXT; ++t) px[t][i][r] = mk<T>(0, 0);
        if (ok && l >= 0) {
          const int64_t idx = base_in + l * ls_in + c;
#pragma unroll
          for (int t = 0; t < MAXT; ++t)
            if (t < nt) px[t][i][r] = ld(src[t], idx);
        }
      }
    }
  };

  const int G = gridDim.x;
  int item = (int)xcd_item(blockIdx.x, G, 0, total);
  if (item >= 0) issue(decode(item));
  for (int k = 0; item >= 0; ++k) {
    const Item it = decode(item);
    // the item's multipliers, once per item
    const OutSpec& sp = a.spec[it.f];
    // Each term is re * x or dk * (i k_axis) * x.  The three-term pass and
    // the mixed path set the factor that does not apply to zero and combine
    // without a branch per element (absent terms have both zero and zeroed
    // prefetch registers): 4.6% faster for the three-term pass at 512.  The
    // FP32 and FP64 one-term passes keep the branch on the term's kind
    // (uniform), which measured faster there.
    const int nt = sp.nterms;
    T re[MAXT], dk[MAXT];
    int ax[MAXT];
#pragma unroll
    for (int t = 0; t < MAXT; ++t) {
      const int axis = t < nt ? sp.t[t].axis : -1;
      const T cf = t < nt ? T(sp.t[t].coef) : T(0);
      re[t] = axis < 0 ? cf : T(0);
      dk[t] = axis < 0 ? T(0) : cf;
      ax[t] = axis;
    }
    // combine the prefetched terms with their spectral multipliers
    cx<T> v[FP::CNT][FP::R];
#pragma unroll
    for (int i = 0; i < FP::CNT; ++i) {
      const int w = tid + i * NT;
      int c, j;
      lane_map<C, FP::NBF, 0>(w, c, j);
      const int col = it.c0 + c;
      const bool ok = (FP::TOT % NT == 0 || w < FP::TOT) && col_ok(col);
      int kx, ky = 0;
      if (zpass) {
        ky = band_k<N>(col / NHP);
        kx = col - (col / NHP) * NHP;
      } else {
        kx = col;
      }
#pragma unroll
      for (int r = 0; r < FP::R; ++r) {
        const int q = j + r * FP::NBF;
        const int l = S > 0 ? pos_band<N>(q) : q;
        cx<T> acc = mk<T>(0, 0);
        if (ok && l >= 0) {
          int kyy = ky, kz = 0;
          if (S > 0) {
            if (zpass) kz = band_k<N>(l);
            else kyy = band_k<N>(l);
          }
#pragma unroll
          for (int t = 0; t < MAXT; ++t) {
            const cx<T> xv = px[t][i][r];
            if constexpr (MAXT > 1 || MX) {
              const T ck = dk[t] * T(ax[t] == 1 ? kyy : (ax[t] == 2 ? kz : kx));
              acc.x += re[t] * xv.x;
              acc.x -= ck * xv.y;
              acc.y += re[t] * xv.y;
              acc.y += ck * xv.x;
            } else if (t < nt) {
              if (ax[t] < 0) {
                acc.x += re[t] * xv.x;
                acc.y += re[t] * xv.y;
              } else {
                const T ck = dk[t] * T(ax[t] == 0 ? kx : (ax[t] == 1 ? kyy : kz));
                acc.x -= ck * xv.y;
                acc.y += ck * xv.x;
              }
            }
          }
        }
        v[i][r] = acc;
      }
    }
    // The next item's loads go out before this item's first pass where that
    // measured faster (FP32 forward and three-term passes from N = 256: 3-6%
    // at 512), else after it; either way they are in flight during the LDS
    // passes.
    constexpr bool EARLY = sizeof(T) == 4 && !MX && N >= 256 && (S < 0 || MAXT > 1);
    const int next = (int)xcd_item(blockIdx.x, G, k + 1, total);
    if constexpr (EARLY) {
      if (next >= 0) issue(decode(next));
    }
    __syncthreads();  // the previous item's last pass is done reading the tile
    T* out = member_ptr(a.out[it.f], it.m, a.bt.mstride);
    const int64_t base_out = it.outer * os_out + it.c0;
    auto store = [&](int, int, int c, int q, cx<T> val) {
      if (!col_ok(it.c0 + c)) return;
      int l = q;
      if constexpr (S < 0) {
        l = pos_band<N>(q);
        if (l < 0) return;
      }
      st(out, base_out + l * ls_out + c, val);
    };
    fft_first_regs<T, PL, C, NT, C, 1, S, 0, 0>(tile, v, tid, C, store);
    if constexpr (!EARLY) {
      if (next >= 0) issue(decode(next));
    }
    // mixed plans: one-term passes overlap two MFMA groups (the three-term
    // inverse pass would spill)
    fft_rest<T, PL, C, NT, C, 1, S, 0, 0, false, false, (MAXT == 1 ? 2 : 1)>(tile, stw, tid, C, store);
    item = next;
  }
}

// ------------------------------------------------------------------ k_zfwd_rhs
// Flat grid over (member, column tile of (ky, kx), output field f = 1..7),
// field fastest.
template <typename T, int N, bool MX>
__global__ void __launch_bounds__((rhs_threads<T, N, MX>()), (rhs_min_waves<T, N, MX>())) k_zfwd_rhs(const RhsArgs<T> a) {
  using PL = PlanOf<N, MX>;
  constexpr int C = rhs_tile<T, N, MX>();
  constexpr int NT = rhs_threads<T, N, MX>();
  constexpr int NH = Band<N>::NH, NHP = Band<N>::NHP, NBB = Band<N>::NB;
  constexpr int NCOLS = NBB * NHP;  // flattened (ky, kx) over the padded pitch
  using LP = LastPass<PL, C, NT>;
  __shared__ cx<T> tile[N * C];
  __shared__ cx<T> stw[N];
  const int tid = threadIdx.x;
  // fields 1..7; R_rho is formed by its own pass before this one, because
  // this pass overwrites m^ (which R_rho = -i k . m^ reads) with its next level
  const TileField tf = tile_field(7);
  const int f = tf.field + 1;
  constexpr int ZT = (NCOLS + C - 1) / C;  // column tiles per member
  const int mem = tf.tile / ZT;
  const int c0 = (tf.tile - mem * ZT) * C;
  const int64_t sc = a.g.sc;
  const int64_t LS = NCOLS;  // row stride of I_z (z) and of compact (kz)
  const T dt = T(a.dt[mem]), ac = T(a.a_cur[mem]), ap = T(a.a_prev[mem]);
  const bool use_prev = a.a_prev[mem] != 0.0;
  const int64_t ms = a.bt.mstride;
  T* const state = member_ptr(a.state, mem, ms);
  T* const rprev = member_ptr(a.rprev, mem, ms);
  T* const rout = a.rout ? member_ptr(a.rout, mem, ms) : nullptr;

  // Output (i, r) of this thread's last-pass slots: compact index, or -1 for
  // a slot that is idle, a padding column or a dealiased kz.
  auto out_index = [&](int i, int r, int& kx, int& ky, int& kz) -> int64_t {
    int c, q;
    if (!last_slot<PL, C, NT, 0>(tid, i, r, c, q)) return -1;
    const int col = c0 + c;
    kx = col - (col / NHP) * NHP;
    if (col >= NCOLS || kx >= NH) return -1;
    ky = band_k<N>(col / NHP);
    const int l = pos_band<N>(q);
    if (l < 0) return -1;
    kz = band_k<N>(l);
    return f * sc + (int64_t)l * LS + col;
  };
  // The state (for the update, and B^ for the resistive term) and the
  // previous RHS: FP32 from N = 512 loads them before the transforms, so that
  // these loads are in flight while the flux groups are transformed (5%
  // faster).  FP32 at N = 256 (a resident workgroup lost to registers, 4%
  // slower), the mixed path (its MFMA stage needs the registers: 139-140 ->
  // 108 without the early loads, two workgroups per CU instead of one,
  // 0.458 -> 0.372 ms at 256, 3.35 -> 2.59 ms at 512) and the narrow shapes
  // load them last.
  constexpr bool PRE = rhs_wide<T, N, MX>() && !MX && N >= 512;
  const bool need_state = !rout || (f >= 4 && f <= 6);
  const bool need_prev = !rout && use_prev;
  cx<T> u_pre[LP::CNT][LP::R], r_pre[LP::CNT][LP::R];
  auto load_old = [&](int i, int r) {
    u_pre[i][r] = mk<T>(0, 0);
    r_pre[i][r] = mk<T>(0, 0);
    int kx, ky, kz;
    const int64_t idx = out_index(i, r, kx, ky, kz);
    if (idx < 0) return;
    if (need_state) u_pre[i][r] = ld(state, idx);
    if (need_prev) r_pre[i][r] = ld(rprev, idx);
  };
  if constexpr (PRE) {
#pragma unroll
    for (int i = 0; i < LP::CNT; ++i)
#pragma unroll
      for (int r = 0; r < LP::R; ++r) load_old(i, r);
  }

  // R_f -> store, or the AB2 update U += dt (a_cur R^n + a_prev R^{n-1}), R^{n-1} <- R^n
  auto finish = [&](int64_t idx, cx<T> R, cx<T> u, cx<T> rp) {
    if (rout) {
      st(rout, idx, R);
    } else {
      cx<T> inc = cscale(R, ac);
      if (use_prev) inc = cadd(inc, cscale(rp, ap));
      u.x += dt * inc.x;
      u.y += dt * inc.y;
      st(state, idx, u);
      st(rprev, idx, R);
    }
  };

  load_twiddles<T, N, NT>(stw, a.tw, tid);
  cx<T> acc[LP::CNT][LP::R];
#pragma unroll
  for (int i = 0; i < LP::CNT; ++i)
#pragma unroll
    for (int r = 0; r < LP::R; ++r) acc[i][r] = mk<T>(0, 0);

  for (int grp = 0; grp < 2; ++grp) {
    const OutSpec& sp = grp == 0 ? a.A[f] : a.Z[f];
    const int nt = sp.nterms;
    if (nt == 0) continue;           // uniform across the block
    if (grp == 1) __syncthreads();   // the LDS tile is about to be rewritten
    const T* p0 = member_ptr(a.flux[sp.t[0].src], mem, ms);
    const T* p1 = nt > 1 ? member_ptr(a.flux[sp.t[1].src], mem, ms) : p0;
    // the multipliers, converted once per group rather than once per element
    T cf[2];
    int ax[2];
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      cf[t] = t < nt ? T(sp.t[t].coef) : T(0);
      ax[t] = t < nt ? sp.t[t].axis : -1;
    }
    auto load = [&](int c, int q) -> cx<T> {
      const int col = c0 + c;
      cx<T> v = mk<T>(0, 0);
      const int kx = col - (col / NHP) * NHP;
      if (col >= NCOLS || kx >= NH) return v;
      const int ky = band_k<N>(col / NHP);
      const int64_t idx = (int64_t)q * LS + col;
      const cx<T> x0 = ld(p0, idx);
      const cx<T> x1 = nt > 1 ? ld(p1, idx) : mk<T>(0, 0);
      const cx<T> xs[2] = {x0, x1};
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        if constexpr (MX) {
          // branch-free, as in the column passes (faster on the mixed path
          // only): absent terms have zero factors and a zero second input
          const T re = ax[t] < 0 ? cf[t] : T(0);
          const T ck = (ax[t] < 0 ? T(0) : cf[t]) * T(ax[t] == 1 ? ky : kx);
          v.x += re * xs[t].x;
          v.x -= ck * xs[t].y;
          v.y += re * xs[t].y;
          v.y += ck * xs[t].x;
        } else if (t < nt) {
          if (ax[t] < 0) {
            v.x += cf[t] * xs[t].x;
            v.y += cf[t] * xs[t].y;
          } else {
            const T ck = cf[t] * T(ax[t] == 0 ? kx : ky);
            v.x -= ck * xs[t].y;
            v.y += ck * xs[t].x;
          }
        }
      }
      return v;
    };
    auto store = [&](int i, int r, int, int q, cx<T> v) {
      if (grp == 0) {
        acc[i][r] = cadd(acc[i][r], v);
      } else {  // + i kz v
        const int l = pos_band<N>(q);
        const T kz = T(l < 0 ? 0 : band_k<N>(l));
        acc[i][r].x -= kz * v.y;
        acc[i][r].y += kz * v.x;
      }
    };
    fft_reg<T, PL, C, NT, C, 1, -1, 0, 0, true>(tile, stw, tid, C, load, store);
  }
  // epilogue over this thread's last-pass positions: resistive term, the
  // Section V variants (block-uniform branches), update
  const T eta = T(a.eta[mem]);
  const bool induction = f >= 4 && f <= 6;
  const int vslot = f <= 3 ? f - 1 : 3;  // u^_{f-1} for the momentum, q^ for the energy
#pragma unroll
  for (int i = 0; i < LP::CNT; ++i) {
#pragma unroll
    for (int r = 0; r < LP::R; ++r) {
      int kx, ky, kz;
      const int64_t idx = out_index(i, r, kx, ky, kz);
      if (idx < 0) continue;
      if constexpr (!PRE) load_old(i, r);
      cx<T> R = acc[i][r];
      const T k2 = T(kx * kx + ky * ky + kz * kz);
      if (induction) {
        // MHD4 resistive term: - eta |k|^2 B^
        const cx<T> b = u_pre[i][r];
        R.x -= eta * k2 * b.x;
        R.y -= eta * k2 * b.y;
      } else {
        const int64_t off = idx - f * sc;  // position inside one compact field
        if (a.mu != 0.0) {
          // viscous force mu lap u, and mu lap(|u|^2/2) in the energy
          const cx<T> v = ld(member_ptr(a.uhat, mem, ms), vslot * sc + off);
          R.x -= T(a.mu) * k2 * v.x;
          R.y -= T(a.mu) * k2 * v.y;
        }
        if (a.force) R = cadd(R, ld(member_ptr(a.force, mem, ms), vslot * sc + off));
        if (a.kinematic) R = mk<T>(0, 0);  // frozen rho u and E
      }
      finish(idx, R, u_pre[i][r], r_pre[i][r]);
    }
  }
}

// ------------------------------------------------------------------ k_row
// blockIdx.x = row pair p: rows (z, 2y') and (z, 2y'+1), z = p / (N/2).
template <int MODE> struct RowShape;
template <> struct RowShape<RM_XA> { static constexpr int NIN = 4, NOUT = 3, NB = 4; };
template <> struct RowShape<RM_XB> { static constexpr int NIN = 16, NOUT = 12, NB = 16; };
template <> struct RowShape<RM_XFWD_REAL> { static constexpr int NIN = 8, NOUT = 8, NB = 8; };
template <> struct RowShape<RM_XINV_REAL> { static constexpr int NIN = 8, NOUT = 8, NB = 8; };
template <> struct RowShape<RM_XDIAG> { static constexpr int NIN = kDiagFields, NOUT = 0, NB = kDiagFields; };

template <typename T>
__device__ __forceinline__ bool finite_(T v) { return isfinite(v); }

// 1/x and sqrt(x) of the pointwise stages.  FP32: the hardware v_rcp_f32 and
// v_sqrt_f32 (1 ulp) instead of the correctly rounded sequences (about ten
// instructions each), in the VALU-bound flux and velocity passes; the
// difference is at the level of FP32 rounding.  FP64: correctly rounded.
template <typename T> __device__ __forceinline__ T recip_(T x) { return T(1) / x; }
template <> __device__ __forceinline__ float recip_<float>(float x) { return __builtin_amdgcn_rcpf(x); }
template <typename T> __device__ __forceinline__ T sqrt_(T x) { return sqrt(x); }
template <> __device__ __forceinline__ float sqrt_<float>(float x) { return __builtin_amdgcn_sqrtf(x); }

// Fixed-order tree reduction over the block (sum, or NaN-propagating max);
// the result is valid in thread 0.  Deterministic for a given launch shape.
template <int NT = kThreads>
__device__ __forceinline__ double block_reduce(double v, bool is_max, double* s, int tid) {
  __syncthreads();
  s[tid] = v;
  __syncthreads();
  for (int w = NT / 2; w > 0; w >>= 1) {
    if (tid < w) {
      const double o = s[tid + w];
      if (is_max) {
        if (!(o <= s[tid])) s[tid] = o;
      } else {
        s[tid] += o;
      }
    }
    __syncthreads();
  }
  return s[0];
}

// Error-free sum of s and x (Neumaier's two-sum): s <- fl(s + x), the
// rounding error of that addition added to the compensation c.
__device__ __forceinline__ void neumaier_add(double& s, double& c, double x) {
  const double t = s + x;
  if (fabs(s) >= fabs(x)) c += (s - t) + x;
  else c += (x - t) + s;
  s = t;
}

// Compensated fixed-order tree sum over the block of per-thread (sum,
// compensation) pairs; every level adds with neumaier_add, so the block
// result carries the same compensation as a serial Neumaier sum.  s: 2 NT
// doubles of LDS scratch.  The result (s + c) is valid in thread 0.
template <int NT = kThreads>
__device__ __forceinline__ double block_sum_comp(double v, double cv, double* s, int tid) {
  __syncthreads();
  s[tid] = v;
  s[NT + tid] = cv;
  __syncthreads();
  for (int w = NT / 2; w > 0; w >>= 1) {
    if (tid < w) {
      double a = s[tid], ca = s[NT + tid] + s[NT + tid + w];
      neumaier_add(a, ca, s[tid + w]);
      s[tid] = a;
      s[NT + tid] = ca;
    }
    __syncthreads();
  }
  return s[0] + s[NT];
}

// Persistent: workgroup w handles row pairs w, w + G, w + 2G, ... (G = grid
// size, sized by the host to the number of resident workgroups).  For the
// spectral-input modes the global loads of the next row pair's first FFT pass
// are issued right after the current pair's first pass, so they are in flight
// during the current pair's LDS passes, pointwise work and stores.
// Fold a workgroup's CFL speed and non-finite count into its own status slot
// of a member (slot = workgroup id; kStatusSlots slots of two doubles: the
// largest signal speed seen by any step since the state was set, and the
// count of non-finite points).  The speed is reduced in FP64 (a max, exact in
// any precision, NaN propagating) and kept as a running max over steps; each
// slot has a single writer, so no atomics are needed and the result does not
// depend on workgroup order.  Block-uniform call.  s_red: NT doubles of LDS
// scratch, which may alias the caller's row buffer (the reductions begin and
// end with a barrier).
template <int NT>
__device__ __forceinline__ void flush_status(double cfl, int bad, double* slots, double* s_red) {
  const int tid = threadIdx.x;
  const double cfl_b = block_reduce<NT>(cfl, true, s_red, tid);
  const double bad_b = block_reduce<NT>(double(bad), false, s_red, tid);
  __syncthreads();  // every thread has read the results before the scratch is reused
  if (tid == 0) {
    double* const slot = slots + 2 * (int64_t)blockIdx.x;
    const double old = slot[0];
    slot[0] = !(cfl_b <= old) ? cfl_b : old;
    slot[1] = slot[1] + bad_b;
  }
}

// Threads of a row pass: FP32 rows of N >= 1024 take 512, which keeps the
// per-thread first-pass work (and registers) of N = 512 on 256 threads.  The
// FP32 flux pass at N = 512 and 256 also takes 512: with wave maps each wave
// then owns two fields instead of four, the registers fit 128, and its LDS
// tile still allows two workgroups per CU, so four waves per SIMD run instead
// of two (13% faster at 512) or three (3% at 256).  The FP32 velocity pass at
// N = 256 takes 128: two waves of two fields each, whose 32-butterfly radix-8
// passes then fill every lane (256 threads left half of them idle; 19%).
// The FP64 flux pass at N = 512 takes 512 too (its 156 KB LDS tile allows
// one workgroup per CU: two waves per SIMD instead of one, 6.78 -> 5.63 ms).
template <typename T, int N, int MODE, bool MX> constexpr int row_threads() {
  if (sizeof(T) == 4 && !MX && MODE == RM_XB && (N == 512 || N == 256)) return 2 * kThreads;
  if (sizeof(T) == 8 && MODE == RM_XB && N == 512) return 2 * kThreads;
  if (sizeof(T) == 4 && !MX && MODE == RM_XA && N == 256) return kThreads / 2;
  return (sizeof(T) == 4 && N >= 1024) ? 2 * kThreads : kThreads;
}

// Register caps of the FP32 row passes (MFMA variant included), as resident
// workgroups per CU: two, i.e. two waves per SIMD at 256 threads and four for
// the 512-thread flux pass at N = 256 and 512 (128 registers), which is what
// their LDS allows.  Left free, the flux pass can take more than 256 registers
// and then runs one wave per SIMD (the MFMA variant at N = 512 was 1.3x
// slower so than capped).
template <typename T, int N, int MODE, bool MX> constexpr int row_min_blocks() {
  if (sizeof(T) == 4 && !MX && MODE == RM_XB && (N == 512 || N == 256)) return 2;
  return sizeof(T) == 4 ? 2 * kThreads / row_threads<T, N, MODE, MX>() : 1;
}

template <typename T, int N, int MODE, bool MX>
__global__ void __launch_bounds__((row_threads<T, N, MODE, MX>()), (row_min_blocks<T, N, MODE, MX>()))
    k_row(const RowArgs<T> a) {
  using PL = PlanOf<N, MX>;
  constexpr int NT = row_threads<T, N, MODE, MX>();
  constexpr int K = Band<N>::K, NHP = Band<N>::NHP;
  constexpr int NH = Band<N>::NH;
  constexpr int NB = RowShape<MODE>::NB;
  // LDS row layout, chosen per pass by measurement.  Linear addressing where
  // the precomputed addresses would push a pass past 256 registers into
  // spills (the flux pass from N = 512 mixed and N = 1024 FP32, the
  // diagnostics pass at N = 1024).  The stage swizzle (conflict-free LDS
  // access, but more address arithmetic) where it measured faster: the FP32
  // flux pass below N = 512 (3%) and the FP32 velocity pass from N = 512 (2%);
  // it made the mixed passes slower.  Otherwise one padding slot per 8
  // elements.
  constexpr bool LIN = (MODE == RM_XB && N >= (MX ? 512 : 1024)) || (MODE == RM_XDIAG && N >= 1024);
  constexpr bool SWZ = !MX && !LIN && N % 16 == 0 && N >= 128 &&
                       ((MODE == RM_XB && N < 512) || (MODE == RM_XA && N >= 512));
  constexpr int PADSH = 3;
  constexpr int LAY = SWZ ? kSwizzle : (PADSH | (LIN ? kLinear : 0));
  // row pitch in LDS: swizzled rows are shifted by 16 elements from row to
  // row, so that a 32-lane read spanning two rows of N = 128 uses all banks
  constexpr int BS = SWZ ? N + 16 : N + (N >> PADSH) + 1;
  constexpr bool SPEC_IN = MODE != RM_XFWD_REAL;
  // Wave maps: each field's transforms stay inside one wave, so a wave-level
  // fence replaces the workgroup barrier between passes and only the
  // pointwise stage, which reads every field at one point, is bracketed by
  // barriers.  Used (measured) by the velocity and flux passes from N = 512
  // (12% and 5% faster), the FP32 velocity and flux passes at 256 (with 128
  // and 512 threads) and the mixed velocity pass from 512, whose last-pass
  // MFMA groups then take the wave's own butterflies (7%); not by the mixed
  // flux pass (slower) or with fewer fields than waves.
  constexpr bool WAVE = (MX ? (MODE == RM_XA && !mid_mfma<PL>()) : (MODE == RM_XA || MODE == RM_XB)) &&
                       (N >= 512 || (!MX && N == 256)) && NB >= NT / 64;
  // MFMA groups overlapped in the mixed last pass (measured: the velocity
  // pass 2, the flux pass 4 at N = 256; the others spill or slow down)
  constexpr int UNR = MODE == RM_XA ? 2 : ((MODE == RM_XB && N <= 256) ? 4 : 1);
  constexpr int RMAP = WAVE ? 3 : 1;
  using FP = FirstPass<PL, NB, NT, RMAP>;
  auto at = [](int b, int pos) { return lds_at<1, BS, LAY, PL, 0>(b, pos); };
  __shared__ cx<T> buf[NB * BS];
  __shared__ cx<T> stw[N];
  // block reductions (status words, diagnostics) use the row buffer as scratch
  // when it is large enough (each begins with a barrier, after which no row
  // work touches the buffer); small sizes get their own array
  constexpr bool RED_IN_BUF = sizeof(cx<T>) * NB * BS >= 2 * NT * sizeof(double);
  __shared__ double red_own[RED_IN_BUF ? 1 : 2 * NT];
  double* const red = RED_IN_BUF ? reinterpret_cast<double*>(buf) : red_own;
  const int tid = threadIdx.x;
  const int64_t rows_per_mem = (int64_t)N * N / 2;
  const int64_t nitems = rows_per_mem * a.bt.nmem;
  const int nin = (MODE == RM_XFWD_REAL || MODE == RM_XINV_REAL) ? a.nf : RowShape<MODE>::NIN;
  const int nout = (MODE == RM_XFWD_REAL || MODE == RM_XINV_REAL)
                       ? a.nf
                       : ((MODE == RM_XA && a.nf == 4) ? 4 : RowShape<MODE>::NOUT);
  load_twiddles<T, N, NT>(stw, a.tw, tid);
  auto lds_store = [&](int, int, int fld, int q, cx<T> v) { buf[at(fld, q)] = v; };

  // Prefetch registers for the next row pair: the two rows' Hermitian
  // half-spectrum entries X0[q], X1[q] behind the first-pass elements in the
  // lower half (q < N/2, r < R/2).  Elements q >= N-K use X[N-q]: with paired
  // first-pass slots (FMAP 2) that is a lower-half element of the thread's
  // partner butterfly, already in these registers; with FMAP 3 it is in a
  // partner lane's registers; otherwise (FMAP 1) a mirror lane prefetched it
  // and it is read again when used.
  // FMAP 3: plain slots, but when NBF divides the wave width the partner
  // butterfly NBF - j sits in the same wave and the mirror comes by a lane
  // shuffle of its register.
  constexpr int RH = FP::R / 2;
  constexpr int FMAP = (FP::CNT % 2 == 0 && FP::NBF % 2 == 0) ? 2 : ((FP::NBF >= 2 && 64 % FP::NBF == 0) ? 3 : 1);
  constexpr int HC = FP::CNT / 2;
  constexpr int FM1 = FMAP == 2 ? (WAVE ? 4 : 2) : RMAP;  // lane map of the first pass
  // first-pass rows r whose positions j + r NBF all lie in the dealiased gap:
  // known zeros, neither loaded nor assembled, and pruned from the DFT
  constexpr unsigned ZROWS = gap_rows<N, FP::NBF, FP::R, K>();
  cx<T> p0[FP::CNT][RH], p1[FP::CNT][RH];
  auto issue = [&](int64_t item) {
    const int mi = (int)(item / rows_per_mem);
    const int64_t row0 = 2 * (item - mi * rows_per_mem);
    const T* in0 = member_ptr(a.in0, mi, a.bt.mstride);
#pragma unroll
    for (int i = 0; i < FP::CNT; ++i) {
      int b, j;
      const bool ok = first_slot<NB, FP::NBF, NT, FM1>(tid, i, b, j) && b < nin;
      const T* src = in0 + 2 * b * a.in_stride;
#pragma unroll
      for (int r = 0; r < RH; ++r) {
        const int q = j + r * FP::NBF;
        p0[i][r] = mk<T>(0, 0);  // the previous pair's values are dead
        p1[i][r] = mk<T>(0, 0);
        if ((ZROWS >> r) & 1u) continue;
        if (ok && q <= K) {
          p0[i][r] = ld(src, row0 * NHP + q);
          p1[i][r] = ld(src, (row0 + 1) * NHP + q);
        }
      }
    }
  };
  // per-workgroup accumulators of the diagnostic / status modes: the largest
  // signal speed (each point's speed is formed in T, and the thread's maximum
  // of T values is exact in T; it goes to FP64 at the workgroup's flush) and
  // the non-finite count of the flux pass; Neumaier (sum, compensation) pairs
  // of the diagnostics pass
  T cfl = T(0);
  int bad = 0;
  double q[kDiagQ], qc[kDiagQ];
#pragma unroll
  for (int i = 0; i < kDiagQ; ++i) {
    q[i] = 0.0;
    qc[i] = 0.0;
  }

  int64_t item = blockIdx.x;
  if constexpr (SPEC_IN) {
    if (item < nitems) issue(item);
  }
  int cur_m = -1;  // member whose CFL / non-finite status is being accumulated
  for (; item < nitems; item += gridDim.x) {
    const int mem = (int)(item / rows_per_mem);
    const int64_t row0 = 2 * (item - mem * rows_per_mem);  // flattened row z*N + y of the first row
    if constexpr (MODE == RM_XB) {
      if (mem != cur_m) {  // uniform across the workgroup
        if (cur_m >= 0 && a.status) {
          flush_status<NT>(double(cfl), bad, member_ptr(a.status, cur_m, a.bt.mstride), red);
          cfl = T(0);
          bad = 0;
        }
        cur_m = mem;
      }
    }
    // the previous row pair is done with the LDS (with wave maps a wave only
    // writes its own fields before the next barrier, and it is the only one
    // that still reads them)
    if constexpr (!WAVE) __syncthreads();
    if constexpr (!SPEC_IN) {
      // real rows -> packed complex row0 + i row1
      for (int e = tid; e < nin * N; e += NT) {
        const int fld = e / N, x = e - (e / N) * N;
        const int64_t base = fld * a.g.n3 + row0 * N + x;
        T r0, r1;
        if (a.real_dtype == 0) {
          r0 = T(static_cast<const double*>(a.real_in)[base]);
          r1 = T(static_cast<const double*>(a.real_in)[base + N]);
        } else {
          r0 = T(static_cast<const float*>(a.real_in)[base]);
          r1 = T(static_cast<const float*>(a.real_in)[base + N]);
        }
        buf[at(fld, x)] = mk<T>(r0, r1);
      }
    } else {
      // inverse x transform: first pass from the prefetched registers
      // first-pass inputs Z[q] = X0[q] + i X1[q] (q <= K),
      // Z[N-k] = conj(X0[k]) + i conj(X1[k]) (k <= K), zero in the gap.
      // Rows r < R/2 hold q < N/2, rows r >= R/2 hold q > N/2 (mirrors of
      // q < N/2).  The prefetch registers are zero wherever nothing was loaded
      // (q > K, or an idle slot), so both formulas give zero in the gap with no
      // case analysis.  (At q = 0 the formula also adds the imaginary parts of
      // the two rows' DC terms, which are zero up to rounding.)
      cx<T> v[FP::CNT][FP::R];
#pragma unroll
      for (int i = 0; i < FP::CNT; ++i) {
        int b, j;
        const bool ok = first_slot<NB, FP::NBF, NT, FM1>(tid, i, b, j) && b < nin;
        const T* src = member_ptr(a.in0, mem, a.bt.mstride) + 2 * b * a.in_stride;
        // FMAP 3: lane of butterfly NBF - j (j = tid mod NBF since NBF divides 64)
        const int plane = (tid & 63) - j + (FP::NBF - j) % FP::NBF;
#pragma unroll
        for (int r = 0; r < FP::R; ++r) {
          if ((ZROWS >> r) & 1u) {
            v[i][r] = mk<T>(0, 0);
            continue;
          }
          if (r < RH) {
            const cx<T> x0 = p0[i][r < RH ? r : 0], x1 = p1[i][r < RH ? r : 0];
            v[i][r] = mk<T>(x0.x - x1.y, x0.y + x1.x);
            continue;
          }
          // mirror element X[N - q]: element R-r-1 of butterfly NBF-j, or, for
          // j = 0, element R-r of the same butterfly (none for r = R/2: that is
          // q = N/2, in the gap)
          const int r1 = (FP::R - 1 - r) < RH ? (FP::R - 1 - r) : 0;
          const bool self_ok = (FP::R - r) < RH;
          const int r0 = self_ok ? (FP::R - r) : 0;
          const cx<T> zero = mk<T>(0, 0);
          const cx<T> self0 = self_ok ? p0[i][r0] : zero, self1 = self_ok ? p1[i][r0] : zero;
          cx<T> x0 = zero, x1 = zero;
          if constexpr (FMAP == 3) {
            // uniform: every lane takes part in the shuffles
            const cx<T> s0 = mk<T>(__shfl(p0[i][r1].x, plane), __shfl(p0[i][r1].y, plane));
            const cx<T> s1 = mk<T>(__shfl(p1[i][r1].x, plane), __shfl(p1[i][r1].y, plane));
            x0 = j == 0 ? self0 : s0;
            x1 = j == 0 ? self1 : s1;
          } else if constexpr (FMAP == 2) {
            // the partner butterfly is the partner slot, except j = 0 (see
            // above) and j = NBF/2, its own partner
            const int ip = i < HC ? i + HC : i - HC;
            if (j == 0) {
              x0 = self0;
              x1 = self1;
            } else if (j == FP::NBF / 2) {
              x0 = p0[i][r1];
              x1 = p1[i][r1];
            } else {
              x0 = p0[ip][r1];
              x1 = p1[ip][r1];
            }
          } else {
            const int q = j + r * FP::NBF;
            if (ok && q >= N - K) {
              x0 = ld(src, row0 * NHP + (N - q));
              x1 = ld(src, (row0 + 1) * NHP + (N - q));
            }
          }
          v[i][r] = mk<T>(x0.x + x1.y, x1.x - x0.y);
        }
      }
      fft_first_regs<T, PL, NB, NT, 1, BS, +1, FM1, LAY, ZROWS>(buf, v, tid, nin, lds_store);
      if (item + gridDim.x < nitems) issue(item + gridDim.x);  // next pair's loads overlap the rest
      fft_rest<T, PL, NB, NT, 1, BS, +1, RMAP, LAY, false, true, UNR>(buf, stw, tid, nin, lds_store);
    }
    __syncthreads();

    if constexpr (MODE == RM_XINV_REAL) {
      for (int e = tid; e < nout * N; e += NT) {
        const int fld = e / N, x = e - (e / N) * N;
        const cx<T> z = buf[at(fld, x)];
        const int64_t base = fld * a.g.n3 + row0 * N + x;
        if (a.real_dtype == 0) {
          static_cast<double*>(a.real_out)[base] = double(z.x);
          static_cast<double*>(a.real_out)[base + N] = double(z.y);
        } else {
          static_cast<float*>(a.real_out)[base] = float(z.x);
          static_cast<float*>(a.real_out)[base + N] = float(z.y);
        }
      }
      continue;
    }

    if constexpr (MODE == RM_XA) {
      // u = m / rho, both rows at once; with four outputs also q = |u|^2/2
      // (the viscous-force variant's energy term) into the slot m_z vacated
      for (int x = tid; x < N; x += NT) {
        const cx<T> rho = buf[at(0, x)];
        const T i0 = recip_(rho.x), i1 = recip_(rho.y);
        cx<T> u[3];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
          const cx<T> m = buf[at(1 + i, x)];
          u[i] = mk<T>(m.x * i0, m.y * i1);
          buf[at(i, x)] = u[i];
        }
        if (nout == 4)
          buf[at(3, x)] = mk<T>(T(0.5) * (u[0].x * u[0].x + u[1].x * u[1].x + u[2].x * u[2].x),
                                T(0.5) * (u[0].y * u[0].y + u[1].y * u[1].y + u[2].y * u[2].y));
      }
    }

    if constexpr (MODE == RM_XB) {
      // Real-space fluxes of Eqs. MHD2-MHD4 at every point of both rows.
      // Inputs: 0 rho, 1-3 m, 4-6 B, 7 E, 8 S_xx, 9 S_yy, 10 S_xy, 11 S_xz,
      // 12 S_yz, 13-15 J.  Outputs: 0 Pi_xx, 1 Pi_yy, 2 Pi_zz, 3 Pi_xy,
      // 4 Pi_xz, 5 Pi_yz, 6-8 F^E, 9-11 e = u x B.
      const T gm1 = T(a.gamma[mem] - 1.0), gam = T(a.gamma[mem]), two_nu = T(2.0 * a.nu[mem]),
              eta = T(a.eta[mem]);
      for (int x = tid; x < N; x += NT) {
        cx<T> v[16];
#pragma unroll
        for (int f = 0; f < 16; ++f) v[f] = buf[at(f, x)];
        cx<T> o[12];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          auto g = [&](int f) -> T { return h == 0 ? v[f].x : v[f].y; };
          const T rho = g(0), mx = g(1), my = g(2), mz = g(3);
          const T Bx = g(4), By = g(5), Bz = g(6), E = g(7);
          const T Sxx = g(8), Syy = g(9), Sxy = g(10), Sxz = g(11), Syz = g(12);
          const T Szz = -(Sxx + Syy);
          const T Jx = g(13), Jy = g(14), Jz = g(15);
          const T ir = recip_(rho);
          const T ux = mx * ir, uy = my * ir, uz = mz * ir;
          const T B2 = Bx * Bx + By * By + Bz * Bz;
          const T P = gm1 * (E - T(0.5) * (mx * ux + my * uy + mz * uz) - T(0.5) * B2);
          const T Pt = P + T(0.5) * B2;
          const T vr = two_nu * rho;
          T out[12];
          out[0] = mx * ux + Pt - Bx * Bx - vr * Sxx;
          out[1] = my * uy + Pt - By * By - vr * Syy;
          out[2] = mz * uz + Pt - Bz * Bz - vr * Szz;
          out[3] = mx * uy - Bx * By - vr * Sxy;
          out[4] = mx * uz - Bx * Bz - vr * Sxz;
          out[5] = my * uz - By * Bz - vr * Syz;
          const T uB = ux * Bx + uy * By + uz * Bz;
          const T EP = E + Pt;
          const T uSx = ux * Sxx + uy * Sxy + uz * Sxz;
          const T uSy = ux * Sxy + uy * Syy + uz * Syz;
          const T uSz = ux * Sxz + uy * Syz + uz * Szz;
          out[6] = EP * ux - uB * Bx - vr * uSx - eta * (By * Jz - Bz * Jy);
          out[7] = EP * uy - uB * By - vr * uSy - eta * (Bz * Jx - Bx * Jz);
          out[8] = EP * uz - uB * Bz - vr * uSz - eta * (Bx * Jy - By * Jx);
          out[9] = uy * Bz - uz * By;
          out[10] = uz * Bx - ux * Bz;
          out[11] = ux * By - uy * Bx;
#pragma unroll
          for (int k = 0; k < 12; ++k) {
            if (h == 0) o[k].x = out[k];
            else o[k].y = out[k];
          }
          // fastest signal speed for the CFL limit, and a non-finite check
          const T umax = fmax(fabs(ux), fmax(fabs(uy), fabs(uz)));
          const T c = umax + sqrt_((gam * P + B2) * ir);
          if (!(c <= cfl)) cfl = c;  // NaN propagates
          const bool fin = finite_(rho) && finite_(mx) && finite_(my) && finite_(mz) && finite_(Bx) &&
                           finite_(By) && finite_(Bz) && finite_(E);
          bad += fin ? 0 : 1;
        }
#pragma unroll
        for (int k = 0; k < 12; ++k) buf[at(k, x)] = o[k];
      }
    }

    if constexpr (MODE == RM_XDIAG) {
      // Inputs: 0 rho, 1-3 m, 4-6 B, 7 E, 8 div B.  (The current's mean square is
      // a spectral sum, exact by Parseval for the band-limited B^.)
      const double gm1 = a.gamma[mem] - 1.0, gam = a.gamma[mem];
      for (int x = tid; x < N; x += NT) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          auto g = [&](int f) -> double { const cx<T> v = buf[at(f, x)]; return double(h == 0 ? v.x : v.y); };
          const double rho = g(0), mx = g(1), my = g(2), mz = g(3), Bx = g(4), By = g(5), Bz = g(6), E = g(7);
          const double dB = g(8);
          const double ux = mx / rho, uy = my / rho, uz = mz / rho;
          const double B2 = Bx * Bx + By * By + Bz * Bz;
          const double mu = mx * ux + my * uy + mz * uz;
          const double P = gm1 * (E - 0.5 * mu - 0.5 * B2);
          auto acc = [&](int i, double x) { neumaier_add(q[i], qc[i], x); };
          acc(DQ_RHO, rho);
          acc(DQ_MX, mx);
          acc(DQ_MY, my);
          acc(DQ_MZ, mz);
          acc(DQ_EKIN, 0.5 * mu);
          acc(DQ_EMAG, 0.5 * B2);
          acc(DQ_P, P);
          acc(DQ_E, E);
          acc(DQ_HC, ux * Bx + uy * By + uz * Bz);
          acc(DQ_UABS, sqrt(ux * ux + uy * uy + uz * uz));
          acc(DQ_BABS, sqrt(B2));
          const double adb = fabs(dB);
          if (!(adb <= q[DQ_DIVB_MAX])) q[DQ_DIVB_MAX] = adb;
          const double c = fmax(fabs(ux), fmax(fabs(uy), fabs(uz))) + sqrt((gam * P + B2) / rho);
          if (!(c <= q[DQ_CFL_MAX])) q[DQ_CFL_MAX] = c;
          const bool fin = isfinite(rho) && isfinite(mx) && isfinite(my) && isfinite(mz) && isfinite(Bx) &&
                           isfinite(By) && isfinite(Bz) && isfinite(E);
          q[DQ_NONFINITE] += fin ? 0.0 : 1.0;
        }
      }
      continue;
    }

    if constexpr (MODE == RM_XA || MODE == RM_XB || MODE == RM_XFWD_REAL) {
      __syncthreads();
      lds_fft<T, PL, NB, NT, 1, BS, -1, RMAP, LAY, K, UNR>(buf, stw, tid, nout);  // only k <= K and N - k are read
      // unpack: X0[k] = (Z[k] + conj Z[N-k]) / 2, X1[k] = -i (Z[k] - conj Z[N-k]) / 2, k = 0..K,
      // stored doubled (2 X0, 2 X1): the forward y pass that reads these rows
      // applies the 1/2 with its copy coefficient (an exact power-of-two
      // scaling, so the values are the same)
      T* out0 = member_ptr(a.out0, mem, a.bt.mstride);
      const int64_t ost = a.out_stride;
      auto unpack = [&](int fld, int k) {
        const cx<T> zk = buf[at(fld, k)];
        const cx<T> zm = buf[at(fld, k == 0 ? 0 : N - k)];
        const cx<T> x0 = mk<T>(zk.x + zm.x, zk.y - zm.y);
        const cx<T> x1 = mk<T>(zk.y + zm.y, zm.x - zk.x);
        T* dst = out0 + 2 * fld * ost;
        st(dst, row0 * NHP + k, x0);
        st(dst, (row0 + 1) * NHP + k, x1);
      };
      // the same with the field's output row as one wave-uniform pointer
      auto unpack_row = [&](cx<T>* dst, int fld, int k) {
        const cx<T> zk = buf[at(fld, k)];
        const cx<T> zm = buf[at(fld, k == 0 ? 0 : N - k)];
        dst[k] = mk<T>(zk.x + zm.x, zk.y - zm.y);
        dst[NHP + k] = mk<T>(zk.y + zm.y, zm.x - zk.x);
      };
      if constexpr (WAVE) {
        // Each wave unpacks the fields it transformed, field by field: the
        // field and its output row are wave-uniform (scalar registers), so an
        // element costs its two LDS addresses and the store offset.  The flux
        // pass at N <= 256 (at most two 64-wide sweeps of a field) also
        // unrolls the sweeps, keeping the LDS addresses in registers across
        // row pairs; elsewhere that would cost occupancy.
        constexpr int W = NT / 64;
        constexpr int KIT = (NH + 63) / 64;
        const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
        cx<T>* const row_out = reinterpret_cast<cx<T>*>(out0) + row0 * NHP;
#pragma unroll 1
        for (int fl = 0; fl < seqs_per_wave<NB, NT>(); ++fl) {
          const int fld = fl * W + wv;
          if (fld >= nout) break;
          cx<T>* const dst = row_out + fld * ost;
          if constexpr (MODE == RM_XB && KIT <= 2) {
#pragma unroll
            for (int it = 0; it < KIT; ++it) {
              const int k = (tid & 63) + 64 * it;
              if ((it + 1) * 64 <= NH || k < NH) unpack_row(dst, fld, k);
            }
          } else {
#pragma unroll 1
            for (int k = tid & 63; k < NH; k += 64) unpack_row(dst, fld, k);
          }
        }
      } else {
        for (int e = tid; e < nout * NH; e += NT) unpack(e / NH, e - (e / NH) * NH);
      }
    }
  }

  if constexpr (MODE == RM_XB) {
    if (cur_m >= 0 && a.status) flush_status<NT>(double(cfl), bad, member_ptr(a.status, cur_m, a.bt.mstride), red);
  }
  if constexpr (MODE == RM_XDIAG) {
    for (int i = 0; i < kDiagQ; ++i) {
      const bool is_max = i == DQ_DIVB_MAX || i == DQ_CFL_MAX;
      const double r = is_max ? block_reduce<NT>(q[i], true, red, tid) : block_sum_comp<NT>(q[i], qc[i], red, tid);
      if (tid == 0) a.partials[(int64_t)blockIdx.x * kDiagQ + i] = r;
    }
  }
}

MHD_SCHED_END
}  // namespace mhd

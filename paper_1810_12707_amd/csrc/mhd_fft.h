// Batched in-LDS FFTs for gfx950.
//
// A workgroup holds NB sequences of length N in LDS, element (b, l) at
// buf[b*BS + l*ES].  Each radix-R pass of the Stockham autosort (decimation
// in time) lets every thread read R elements of one butterfly into registers,
// twiddle them, do an R-point DFT in registers, and, after a barrier, write
// them to their sorted positions; the output ends in natural order, so no
// bit-reversal pass is needed.  Butterflies are assigned batch-fastest across
// lanes so that a column tile (ES = C, BS = 1) gives unit-stride LDS access.
//
// Twiddles come from a table of exp(-2 pi i j / N), j < N, computed in FP64
// on the host and rounded once to T; the inverse uses the conjugates.
#pragma once

#include <hip/hip_runtime.h>

namespace mhd {

template <typename T> struct V2;
template <> struct V2<float> { using t = float2; };
template <> struct V2<double> { using t = double2; };
template <typename T> using cx = typename V2<T>::t;

template <typename T> __device__ __forceinline__ cx<T> mk(T a, T b) { cx<T> r; r.x = a; r.y = b; return r; }
template <typename X> __device__ __forceinline__ X cadd(X a, X b) { X r; r.x = a.x + b.x; r.y = a.y + b.y; return r; }
template <typename X> __device__ __forceinline__ X csub(X a, X b) { X r; r.x = a.x - b.x; r.y = a.y - b.y; return r; }
template <typename X> __device__ __forceinline__ X cmul(X a, X b) {
  X r; r.x = a.x * b.x - a.y * b.y; r.y = a.x * b.y + a.y * b.x; return r;
}
// a * conj(b)
template <typename X> __device__ __forceinline__ X cmulc(X a, X b) {
  X r; r.x = a.x * b.x + a.y * b.y; r.y = a.y * b.x - a.x * b.y; return r;
}
template <typename X> __device__ __forceinline__ X cconj(X a) { X r; r.x = a.x; r.y = -a.y; return r; }
template <typename X, typename S> __device__ __forceinline__ X cscale(X a, S s) { X r; r.x = a.x * s; r.y = a.y * s; return r; }
// i * a and -i * a
template <typename X> __device__ __forceinline__ X ctimes_i(X a) { X r; r.x = -a.y; r.y = a.x; return r; }
template <typename X> __device__ __forceinline__ X ctimes_mi(X a) { X r; r.x = a.y; r.y = -a.x; return r; }
// multiply by i^s: sign s = -1 gives -i (forward), +1 gives +i (inverse)
template <int S, typename X> __device__ __forceinline__ X ctimes_si(X a) { return S < 0 ? ctimes_mi(a) : ctimes_i(a); }

// ---------------------------------------------------------------- small DFTs
// In place, natural order in and out; S = -1 forward, +1 inverse.

template <int S, typename X> __device__ __forceinline__ void dft2(X* v) {
  X t = csub(v[0], v[1]);
  v[0] = cadd(v[0], v[1]);
  v[1] = t;
}

template <int S, typename X> __device__ __forceinline__ void dft3(X* v) {
  using T = decltype(v[0].x);
  const T h = T(0.86602540378443864676372317075294);  // sin(pi/3)
  X t = cadd(v[1], v[2]);
  X d = csub(v[1], v[2]);
  X m = csub(v[0], cscale(t, T(0.5)));
  v[0] = cadd(v[0], t);
  X sd = ctimes_si<S>(cscale(d, h));  // S * i * sin(pi/3) * (v1 - v2)
  v[1] = cadd(m, sd);
  v[2] = csub(m, sd);
}

template <int S, typename X> __device__ __forceinline__ void dft4(X* v) {
  X t0 = cadd(v[0], v[2]), t1 = csub(v[0], v[2]);
  X t2 = cadd(v[1], v[3]), t3 = ctimes_si<S>(csub(v[1], v[3]));
  v[0] = cadd(t0, t2);
  v[2] = csub(t0, t2);
  v[1] = cadd(t1, t3);
  v[3] = csub(t1, t3);
}

template <int S, typename X> __device__ __forceinline__ void dft8(X* v) {
  using T = decltype(v[0].x);
  const T h = T(0.70710678118654752440084436210485);
  X e[4] = {v[0], v[2], v[4], v[6]};
  X o[4] = {v[1], v[3], v[5], v[7]};
  dft4<S>(e);
  dft4<S>(o);
  // o[q] *= exp(S * i * pi * q / 4)
  X o1 = o[1], o3 = o[3];
  if (S < 0) {
    o[1].x = (o1.x + o1.y) * h; o[1].y = (o1.y - o1.x) * h;
    o[3].x = (o3.y - o3.x) * h; o[3].y = -(o3.x + o3.y) * h;
  } else {
    o[1].x = (o1.x - o1.y) * h; o[1].y = (o1.x + o1.y) * h;
    o[3].x = -(o3.x + o3.y) * h; o[3].y = (o3.x - o3.y) * h;
  }
  o[2] = ctimes_si<S>(o[2]);
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    v[q] = cadd(e[q], o[q]);
    v[q + 4] = csub(e[q], o[q]);
  }
}

template <int R, int S, typename X> __device__ __forceinline__ void dft(X* v) {
  if constexpr (R == 2) dft2<S>(v);
  else if constexpr (R == 3) dft3<S>(v);
  else if constexpr (R == 4) dft4<S>(v);
  else if constexpr (R == 8) dft8<S>(v);
  else static_assert(R == 2 || R == 3 || R == 4 || R == 8, "unsupported radix");
}

// ---------------------------------------------------------------- radix plans

template <int N> struct Plan;
#define MHD_PLAN(NN, ...)                                              \
  template <> struct Plan<NN> {                                        \
    static constexpr int r[] = {__VA_ARGS__};                          \
    static constexpr int np = sizeof(r) / sizeof(int);                 \
  };
MHD_PLAN(8, 8)
MHD_PLAN(12, 4, 3)
MHD_PLAN(16, 4, 4)
MHD_PLAN(24, 8, 3)
MHD_PLAN(32, 8, 4)
MHD_PLAN(48, 4, 4, 3)
MHD_PLAN(64, 8, 8)
MHD_PLAN(96, 8, 4, 3)
MHD_PLAN(128, 8, 4, 4)
MHD_PLAN(192, 8, 8, 3)
MHD_PLAN(256, 8, 8, 4)
MHD_PLAN(384, 8, 4, 4, 3)
MHD_PLAN(512, 8, 8, 8)
MHD_PLAN(768, 8, 8, 4, 3)
MHD_PLAN(1024, 8, 8, 4, 4)
#undef MHD_PLAN

template <int N> constexpr int plan_ns(int p) {
  int ns = 1;
  for (int i = 0; i < p; ++i) ns *= Plan<N>::r[i];
  return ns;
}

template <int N> constexpr bool plan_ok() {
  int prod = 1;
  for (int i = 0; i < Plan<N>::np; ++i) prod *= Plan<N>::r[i];
  return prod == N;
}

// Lane -> (sequence b, butterfly j) assignment of a pass with NBF butterflies
// per sequence: MAP 0 puts the batch fastest (column tiles: lanes touch
// adjacent columns), MAP 1 the butterfly fastest (rows: lanes touch adjacent
// elements of one sequence).
template <int NB, int NBF, int MAP>
__device__ __forceinline__ void lane_map(int w, int& b, int& j) {
  if constexpr (MAP == 0) {
    b = w % NB;
    j = w / NB;
  } else {
    b = w / NBF;
    j = w % NBF;
  }
}

// LDS element address of (sequence b, position pos).  PADSH > 0 inserts one
// padding slot after every 2^PADSH positions, which spreads the strided
// Stockham writes of row-major sequences over the LDS banks.
template <int ES, int BS, int PADSH>
__device__ __forceinline__ int lds_at(int b, int pos) {
  if constexpr (PADSH > 0) return b * BS + pos * ES + (pos >> PADSH);
  else return b * BS + pos * ES;
}

// One Stockham pass.  NB sequences, NT threads; B_ACT (<= NB) of them active.
template <typename T, int N, int NB, int NT, int ES, int BS, int S, int P, int MAP = 0, int PADSH = 0>
__device__ __forceinline__ void fft_pass(cx<T>* buf, const cx<T>* tw, int tid, int b_act) {
  constexpr int R = Plan<N>::r[P];
  constexpr int NS = plan_ns<N>(P);
  constexpr int NBF = N / R;
  constexpr int TOT = NB * NBF;
  constexpr int CNT = (TOT + NT - 1) / NT;
  cx<T> v[CNT][R];
#pragma unroll
  for (int i = 0; i < CNT; ++i) {
    const int w = tid + i * NT;
    int b, j;
    lane_map<NB, NBF, MAP>(w, b, j);
    if ((TOT % NT == 0 || w < TOT) && b < b_act) {
#pragma unroll
      for (int r = 0; r < R; ++r) v[i][r] = buf[lds_at<ES, BS, PADSH>(b, j + r * NBF)];
      if constexpr (NS > 1) {
        const int k = j % NS;
#pragma unroll
        for (int r = 1; r < R; ++r) {
          const cx<T> t = tw[k * r * (N / (NS * R))];
          v[i][r] = (S < 0) ? cmul(v[i][r], t) : cmulc(v[i][r], t);
        }
      }
      dft<R, S>(v[i]);
    }
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < CNT; ++i) {
    const int w = tid + i * NT;
    int b, j;
    lane_map<NB, NBF, MAP>(w, b, j);
    if ((TOT % NT == 0 || w < TOT) && b < b_act) {
      const int k = j % NS;
      const int d = (j / NS) * NS * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) buf[lds_at<ES, BS, PADSH>(b, d + r * NS)] = v[i][r];
    }
  }
  __syncthreads();
}

template <typename T, int N, int NB, int NT, int ES, int BS, int S, int MAP = 0, int PADSH = 0, int P = 0>
__device__ __forceinline__ void lds_fft(cx<T>* buf, const cx<T>* tw, int tid, int b_act) {
  static_assert(plan_ok<N>(), "radix plan does not multiply to N");
  if constexpr (P < Plan<N>::np) {
    fft_pass<T, N, NB, NT, ES, BS, S, P, MAP, PADSH>(buf, tw, tid, b_act);
    lds_fft<T, N, NB, NT, ES, BS, S, MAP, PADSH, P + 1>(buf, tw, tid, b_act);
  }
}

// Passes 1 .. np-2 of a plan, LDS to LDS.
template <typename T, int N, int NB, int NT, int ES, int BS, int S, int MAP, int PADSH, int P>
__device__ __forceinline__ void fft_mid_passes(cx<T>* buf, const cx<T>* tw, int tid, int b_act) {
  if constexpr (P < Plan<N>::np - 1) {
    fft_pass<T, N, NB, NT, ES, BS, S, P, MAP, PADSH>(buf, tw, tid, b_act);
    fft_mid_passes<T, N, NB, NT, ES, BS, S, MAP, PADSH, P + 1>(buf, tw, tid, b_act);
  }
}

// Shape of the first pass of a plan: R0 elements per butterfly, CNT0
// butterflies per thread.
template <int N, int NB, int NT> struct FirstPass {
  static constexpr int R = Plan<N>::r[0];
  static constexpr int NBF = N / R;
  static constexpr int TOT = NB * NBF;
  static constexpr int CNT = (TOT + NT - 1) / NT;
};

// First pass from values already in registers (v[i][r] = element j + r*NBF of
// sequence b for this thread's i-th butterfly): R-point DFTs, then either the
// final outputs (one-pass plans) or the LDS writes of the next pass, followed
// by a barrier.
template <typename T, int N, int NB, int NT, int ES, int BS, int S, int MAP, int PADSH, class Store>
__device__ __forceinline__ void fft_first_regs(cx<T>* buf, cx<T> (&v)[FirstPass<N, NB, NT>::CNT][Plan<N>::r[0]],
                                               int tid, int b_act, Store&& store) {
  using FP = FirstPass<N, NB, NT>;
  constexpr int NP = Plan<N>::np;
#pragma unroll
  for (int i = 0; i < FP::CNT; ++i) {
    const int w = tid + i * NT;
    int b, j;
    lane_map<NB, FP::NBF, MAP>(w, b, j);
    if ((FP::TOT % NT == 0 || w < FP::TOT) && b < b_act) {
      dft<FP::R, S>(v[i]);
      if constexpr (NP == 1) {
#pragma unroll
        for (int r = 0; r < FP::R; ++r) store(i, r, b, r, v[i][r]);
      } else {
#pragma unroll
        for (int r = 0; r < FP::R; ++r) buf[lds_at<ES, BS, PADSH>(b, j * FP::R + r)] = v[i][r];
      }
    }
  }
  if constexpr (NP > 1) __syncthreads();
}

// Middle passes (LDS to LDS) and the last pass (LDS to store()).
template <typename T, int N, int NB, int NT, int ES, int BS, int S, int MAP, int PADSH, class Store>
__device__ __forceinline__ void fft_rest(cx<T>* buf, const cx<T>* tw, int tid, int b_act, Store&& store) {
  constexpr int NP = Plan<N>::np;
  if constexpr (NP > 1) {
    fft_mid_passes<T, N, NB, NT, ES, BS, S, MAP, PADSH, 1>(buf, tw, tid, b_act);
    constexpr int PL = NP - 1;
    constexpr int R = Plan<N>::r[PL];
    constexpr int NS = plan_ns<N>(PL);  // = N / R
    constexpr int NBF = N / R;
    constexpr int TOT = NB * NBF;
    constexpr int CNT = (TOT + NT - 1) / NT;
#pragma unroll
    for (int i = 0; i < CNT; ++i) {
      const int w = tid + i * NT;
      int b, j;
      lane_map<NB, NBF, MAP>(w, b, j);
      if ((TOT % NT == 0 || w < TOT) && b < b_act) {
        cx<T> v[R];
#pragma unroll
        for (int r = 0; r < R; ++r) v[r] = buf[lds_at<ES, BS, PADSH>(b, j + r * NBF)];
#pragma unroll
        for (int r = 1; r < R; ++r) {
          const cx<T> t = tw[j * r];  // k = j mod NS = j; index k r N/(NS R) = j r
          v[r] = (S < 0) ? cmul(v[r], t) : cmulc(v[r], t);
        }
        dft<R, S>(v);
#pragma unroll
        for (int r = 0; r < R; ++r) store(i, r, b, j + r * NS, v[r]);
      }
    }
  }
}

// Register-ended FFT: the first pass takes its inputs from load(b, pos)
// (global memory) and the last pass hands its outputs to
// store(i, r, b, pos, value) from registers; only the passes in between go
// through LDS.  load() is called for all CNT*R elements of a thread before any
// arithmetic, so their memory requests are in flight together.  For one-pass
// plans the inputs go straight from load() through the DFT to store().
// The LDS buffer may be reused after this returns only past a __syncthreads().
template <typename T, int N, int NB, int NT, int ES, int BS, int S, int MAP = 0, int PADSH = 0, class Load,
          class Store>
__device__ __forceinline__ void fft_reg(cx<T>* buf, const cx<T>* tw, int tid, int b_act, Load&& load,
                                        Store&& store) {
  static_assert(plan_ok<N>(), "radix plan does not multiply to N");
  using FP = FirstPass<N, NB, NT>;
  cx<T> v[FP::CNT][FP::R];
#pragma unroll
  for (int i = 0; i < FP::CNT; ++i) {
    const int w = tid + i * NT;
    int b, j;
    lane_map<NB, FP::NBF, MAP>(w, b, j);
    const bool ok = (FP::TOT % NT == 0 || w < FP::TOT) && b < b_act;
#pragma unroll
    for (int r = 0; r < FP::R; ++r) v[i][r] = ok ? load(b, j + r * FP::NBF) : mk<T>(0, 0);
  }
  fft_first_regs<T, N, NB, NT, ES, BS, S, MAP, PADSH>(buf, v, tid, b_act, store);
  fft_rest<T, N, NB, NT, ES, BS, S, MAP, PADSH>(buf, tw, tid, b_act, store);
}

// Per-thread shape of the last pass of fft_reg (for callers that keep its
// outputs in registers).
template <int N, int NB, int NT> struct LastPass {
  static constexpr int R = Plan<N>::r[Plan<N>::np - 1];
  static constexpr int NBF = N / R;
  static constexpr int TOT = NB * NBF;
  static constexpr int CNT = (TOT + NT - 1) / NT;
};

// Workgroup id remap for gfx950's eight XCDs.  Workgroups are handed out
// round-robin (id w runs on XCD w mod 8); the returned logical id makes each
// XCD own one contiguous range, so logically adjacent workgroups share an L2.
__device__ __forceinline__ int xcd_remap(int w, int total) {
  constexpr int X = 8;
  const int per = total / X, rem = total % X;
  const int xcd = w % X, slot = w / X;
  return xcd < rem ? xcd * (per + 1) + slot : rem * (per + 1) + (xcd - rem) * per + slot;
}

// Item order of a persistent grid of G workgroups over `total` items: the
// items are split into eight contiguous ranges, one per XCD, and the
// workgroups resident on an XCD (ids w with w mod 8 = x) walk that XCD's
// range together.  Returns the k-th item of workgroup w, or -1 when done.
__device__ __forceinline__ int64_t xcd_item(int w, int G, int64_t k, int64_t total) {
  constexpr int X = 8;
  const int xcd = w % X, slot = w / X;
  const int per = G / X + (xcd < G % X ? 1 : 0);
  const int64_t base = total / X, rem = total % X;
  const int64_t start = xcd * base + (xcd < rem ? xcd : rem);
  const int64_t len = base + (xcd < rem ? 1 : 0);
  const int64_t idx = k * per + slot;
  return idx < len ? start + idx : -1;
}

}  // namespace mhd

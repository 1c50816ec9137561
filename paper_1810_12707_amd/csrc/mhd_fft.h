// Batched in-LDS FFTs for gfx950.
//
// A workgroup holds NB sequences of length N in LDS, element (b, l) at
// lds_at(b, l).  Each radix-R pass of the Stockham autosort (decimation in
// time) lets every thread read R elements of one butterfly into registers,
// twiddle them, do an R-point DFT, and, after a barrier, write them to their
// sorted positions; the output ends in natural order, so no bit-reversal pass
// is needed.  Lanes are assigned to butterflies batch-fastest (column tiles,
// unit-stride LDS access across adjacent columns) or butterfly-fastest (rows).
//
// A plan (PlanT) is the list of radices.  In a mixed-precision plan
// (MX = true) every radix-16 pass that runs LDS to LDS is a matrix product on
// the MFMA units: the 16-point DFT of 16 butterflies at once is the real
// 32 x 32 matrix [[Re W, -Im W], [Im W, Re W]] times the 32 x 16 matrix of their
// (Re, Im) inputs; W and the inputs are each split into BF16 high and low parts
// (hi = RNE(x), lo = RNE(x - hi)) and Y = W_hi X_hi + W_hi X_lo + W_lo X_hi is
// accumulated in FP32 by v_mfma_f32_16x16x32_bf16 (the lo*lo term, about 2^-16
// relative, is dropped).  Twiddles stay FP32 on the VALU.
//
// Twiddles come from a table of exp(-2 pi i j / N), j < N, computed in FP64
// on the host and rounded once to T; the inverse uses the conjugates.
#pragma once

#include <hip/hip_runtime.h>

#include "mhd_internal.h"

namespace mhd {
MHD_SCHED_BEGIN

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

// cos(2 pi m / 16), m = 0..15 (sin(2 pi m/16) = cos(2 pi (m - 4)/16))
__device__ constexpr double kCos16[16] = {
    1.0, 0.92387953251128675613, 0.70710678118654752440, 0.38268343236508977173,
    0.0, -0.38268343236508977173, -0.70710678118654752440, -0.92387953251128675613,
    -1.0, -0.92387953251128675613, -0.70710678118654752440, -0.38268343236508977173,
    0.0, 0.38268343236508977173, 0.70710678118654752440, 0.92387953251128675613};

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

// Second half of an 8-point DFT from the 4-point DFTs e of the even and o of
// the odd samples.
template <int S, typename X> __device__ __forceinline__ void dft8_combine(X* v, X (&e)[4], X (&o)[4]) {
  using T = decltype(v[0].x);
  const T h = T(0.70710678118654752440084436210485);
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

template <int S, typename X> __device__ __forceinline__ void dft8(X* v) {
  X e[4] = {v[0], v[2], v[4], v[6]};
  X o[4] = {v[1], v[3], v[5], v[7]};
  dft4<S>(e);
  dft4<S>(o);
  dft8_combine<S>(v, e, o);
}

// 8-point DFT of samples with v[3] = v[4] = 0 (a first pass over a band-limited
// input whose rows 3 and 4 fall in the dealiased gap): the 4-point DFTs lose
// two complex additions each.  Equal to dft8 on such input up to the sign of
// zero results.
template <int S, typename X> __device__ __forceinline__ void dft8_z34(X* v) {
  const X a = cadd(v[2], v[6]);
  const X d = ctimes_si<S>(csub(v[2], v[6]));
  X e[4] = {cadd(v[0], a), cadd(v[0], d), csub(v[0], a), csub(v[0], d)};
  const X t0 = cadd(v[1], v[5]), t1 = csub(v[1], v[5]);
  const X w = ctimes_si<S>(v[7]);
  X o[4] = {cadd(t0, v[7]), csub(t1, w), csub(t0, v[7]), cadd(t1, w)};
  dft8_combine<S>(v, e, o);
}

// 16 = 4 x 4: inner 4-point DFTs over stride-4 samples, twiddles
// exp(S 2 pi i n2 k1 / 16), outer 4-point DFTs; output index k1 + 4 k2.
template <int S, typename X> __device__ __forceinline__ void dft16(X* v) {
  using T = decltype(v[0].x);
  X b[4][4];
#pragma unroll
  for (int n2 = 0; n2 < 4; ++n2) {
    X a[4] = {v[n2], v[4 + n2], v[8 + n2], v[12 + n2]};
    dft4<S>(a);
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) {
      const int m = (n2 * k1) & 15;
      X w;
      w.x = T(kCos16[m]);
      w.y = T(S) * T(kCos16[(m + 12) & 15]);
      b[n2][k1] = (m == 0) ? a[k1] : cmul(a[k1], w);
    }
  }
#pragma unroll
  for (int k1 = 0; k1 < 4; ++k1) {
    X c[4] = {b[0][k1], b[1][k1], b[2][k1], b[3][k1]};
    dft4<S>(c);
#pragma unroll
    for (int k2 = 0; k2 < 4; ++k2) v[k1 + 4 * k2] = c[k2];
  }
}

// DFT of samples of which those with bit r of ZM set are known to be zero
// (only the 8-point case with samples 3 and 4 zero is specialised).
template <int R, int S, unsigned ZM, typename X> __device__ __forceinline__ void dft_z(X* v);

template <int R, int S, typename X> __device__ __forceinline__ void dft(X* v) {
  if constexpr (R == 2) dft2<S>(v);
  else if constexpr (R == 3) dft3<S>(v);
  else if constexpr (R == 4) dft4<S>(v);
  else if constexpr (R == 8) dft8<S>(v);
  else if constexpr (R == 16) dft16<S>(v);
  else static_assert(R == 2 || R == 3 || R == 4 || R == 8 || R == 16, "unsupported radix");
}

template <int R, int S, unsigned ZM, typename X> __device__ __forceinline__ void dft_z(X* v) {
  if constexpr (R == 8 && ZM == ((1u << 3) | (1u << 4))) dft8_z34<S>(v);
  else dft<R, S>(v);
}

// ---------------------------------------------------------------- radix plans

template <int NN, bool MXX, int... Rs> struct PlanT {
  static constexpr int N = NN;
  static constexpr bool MX = MXX;  // radix-16 LDS passes on MFMA (split BF16 x 3)
  static constexpr int r[] = {Rs...};
  static constexpr int np = sizeof...(Rs);
};

// FP32 / FP64 plans (VALU only) and mixed plans.  A mixed plan ends in a
// radix-16 stage: the last Stockham pass writes each butterfly onto its own
// inputs, so the MFMA products run group by group with no registers held
// across a barrier.  Radix-16 stages before it would (a middle pass must
// hold every group's products until all groups have read), and a radix-16
// first pass, which reads from global memory, stays on the VALU; measured
// fastest: small radices first, one radix-16 MFMA stage last.
template <int N, bool MX> struct PlanSel;
#define MHD_PLAN(NN, ...) template <> struct PlanSel<NN, false> { using type = PlanT<NN, false, __VA_ARGS__>; };
#define MHD_PLAN_MX(NN, ...) template <> struct PlanSel<NN, true> { using type = PlanT<NN, true, __VA_ARGS__>; };
// The alternative schedule (ensemble sizes only) takes one radix-16 stage:
// fewer LDS passes, more registers per butterfly.
MHD_PLAN(8, 8)
MHD_PLAN(12, 4, 3)
MHD_PLAN(16, 4, 4)
MHD_PLAN(24, 8, 3)
MHD_PLAN(48, 4, 4, 3)
#if MHD_SCHED == 1
MHD_PLAN(32, 2, 16)
MHD_PLAN(64, 4, 16)
MHD_PLAN(96, 2, 3, 16)
MHD_PLAN(128, 8, 16)
#else
MHD_PLAN(32, 8, 4)
MHD_PLAN(64, 8, 8)
MHD_PLAN(96, 8, 4, 3)
MHD_PLAN(128, 8, 4, 4)
#endif
MHD_PLAN(192, 8, 8, 3)
MHD_PLAN(256, 8, 8, 4)
MHD_PLAN(384, 8, 4, 4, 3)
MHD_PLAN(512, 8, 8, 8)
MHD_PLAN(768, 8, 8, 4, 3)
MHD_PLAN(1024, 8, 8, 4, 4)
MHD_PLAN_MX(8, 8)
MHD_PLAN_MX(12, 4, 3)
MHD_PLAN_MX(16, 4, 4)
MHD_PLAN_MX(24, 8, 3)
MHD_PLAN_MX(32, 2, 16)
MHD_PLAN_MX(48, 3, 16)
MHD_PLAN_MX(64, 4, 16)
MHD_PLAN_MX(96, 2, 3, 16)
MHD_PLAN_MX(128, 8, 16)
MHD_PLAN_MX(192, 4, 3, 16)
MHD_PLAN_MX(256, 4, 4, 16)
MHD_PLAN_MX(384, 3, 8, 16)
MHD_PLAN_MX(512, 8, 4, 16)
MHD_PLAN_MX(768, 16, 3, 16)
MHD_PLAN_MX(1024, 8, 8, 16)
#undef MHD_PLAN
#undef MHD_PLAN_MX
template <int N, bool MX = false> using PlanOf = typename PlanSel<N, MX>::type;

template <class PL> constexpr int plan_ns(int p) {
  int ns = 1;
  for (int i = 0; i < p; ++i) ns *= PL::r[i];
  return ns;
}

// A mixed plan with a radix-16 stage before its last (an LDS-to-LDS MFMA pass).
template <class PL> constexpr bool mid_mfma() {
  if (!PL::MX) return false;
  for (int i = 0; i + 1 < PL::np; ++i)
    if (PL::r[i] == 16) return true;
  return false;
}

template <class PL> constexpr bool plan_ok() {
  int prod = 1;
  for (int i = 0; i < PL::np; ++i) prod *= PL::r[i];
  return prod == PL::N;
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

// Row maps that keep each sequence inside one wave.  MAP 3: with W = NT / 64
// waves, sequence b belongs to wave b mod W, which walks its sequences
// b = wave + W f (f = 0, 1, ...) butterfly-fastest, 64 lanes per slot.  Every
// pass then reads and writes only the wave's own sequences, so passes are
// separated by a wave-level fence instead of a workgroup barrier (LDS
// operations of one wave are performed in order).  MAP 4 is MAP 3 with the
// paired first-pass slots of MAP 2.
template <int MAP> constexpr bool wave_map() { return MAP == 3 || MAP == 4; }
template <int NB, int NT> constexpr int seqs_per_wave() { return (NB + NT / 64 - 1) / (NT / 64); }

// Slots per thread of a pass over NB sequences of NBF butterflies.
template <int NB, int NBF, int NT, int MAP> constexpr int slot_count() {
  return wave_map<MAP>() ? (seqs_per_wave<NB, NT>() * NBF + 63) / 64 : (NB * NBF + NT - 1) / NT;
}

// Barrier between two passes: a workgroup barrier, or for the wave maps a
// fence that keeps the compiler from moving LDS accesses across it.
template <int MAP> __device__ __forceinline__ void pass_sync() {
  if constexpr (wave_map<MAP>()) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  } else {
    __syncthreads();
  }
}

// (sequence b, butterfly j) of slot i under a wave map; b >= NB when the slot
// is idle.
template <int NB, int NBF, int NT>
__device__ __forceinline__ void wave_slot(int tid, int i, int& b, int& j) {
  constexpr int W = NT / 64;
  const int u = i * 64 + (tid & 63);
  const int fl = u / NBF;
  j = u - fl * NBF;
  b = fl < seqs_per_wave<NB, NT>() ? fl * W + (tid >> 6) : NB;
}

// Butterfly (sequence b, index j) of first-pass slot i of thread tid, for NB
// sequences of NBF butterflies spread over NT threads; false if the slot is
// idle.  MAP 0 and 1 as lane_map on w = tid + i NT.  MAP 2 puts butterflies j
// and NBF - j of one sequence (j = 0 together with NBF/2) in one thread, as
// slots i and i + CNT/2: the Hermitian mirror X[N - q] that an element q of
// one needs is then an element of the other, already in the thread.
template <int NB, int NBF, int NT, int MAP>
__device__ __forceinline__ bool first_slot(int tid, int i, int& b, int& j) {
  constexpr int TOT = NB * NBF;
  if constexpr (MAP == 4) {
    constexpr int CNT = slot_count<NB, NBF, NT, 4>();
    static_assert(CNT % 2 == 0 && NBF % 2 == 0, "paired slots need an even slot count");
    constexpr int H = CNT / 2, HB = NBF / 2;
    const int u = (tid & 63) + (i % H) * 64;
    const int fl = u / HB;
    const int p = u - fl * HB;
    j = i < H ? p : (p == 0 ? HB : NBF - p);
    b = fl * (NT / 64) + (tid >> 6);
    return fl < seqs_per_wave<NB, NT>() && b < NB;
  } else if constexpr (MAP == 3) {
    wave_slot<NB, NBF, NT>(tid, i, b, j);
    return b < NB;
  } else if constexpr (MAP == 2) {
    constexpr int CNT = (TOT + NT - 1) / NT;
    static_assert(CNT % 2 == 0 && NBF % 2 == 0, "paired slots need an even slot count");
    constexpr int H = CNT / 2, HB = NBF / 2;
    const int u = tid + (i % H) * NT;
    b = u / HB;
    const int p = u - b * HB;
    j = i < H ? p : (p == 0 ? HB : NBF - p);
    return u < TOT / 2;
  } else {
    const int w = tid + i * NT;
    lane_map<NB, NBF, MAP>(w, b, j);
    return TOT % NT == 0 || w < TOT;
  }
}

// Layout code of an LDS sequence buffer (the PADSH template argument of the
// functions below): bits 0-3 give the padding shift s -- one padding slot
// after every 2^s positions, which spreads the strided Stockham writes of
// row-major sequences over the LDS banks (0: no padding); kLinear asks for
// linear addressing (see slot_map); kSwizzle for the stage swizzle below
// (without padding).
constexpr int kLinear = 16;
constexpr int kSwizzle = 32;
template <int PADSH> constexpr int pad_shift() { return (PADSH & kSwizzle) ? 0 : (PADSH & 15); }
template <int PADSH> constexpr bool linear_addr() { return (PADSH & kLinear) != 0; }
template <int PADSH> constexpr bool swizzled() { return (PADSH & kSwizzle) != 0; }

constexpr bool is_pow2(int x) { return x > 0 && (x & (x - 1)) == 0; }
constexpr int ilog2(int x) { return x <= 1 ? 0 : 1 + ilog2(x / 2); }

// Stage swizzle.  Measured on gfx950, a wave's ds_read_b64 is served 32 lanes
// per cycle over 64 four-byte banks and its ds_write_b64 16 lanes per cycle
// over 32, so a read is conflict-free when its 32 lanes hit distinct
// positions mod 32 and a write when its 16 lanes hit distinct positions mod 16
// (8-byte elements).  Padding one slot per 8 positions serves the strided
// Stockham writes but costs every contiguous access a second cycle.  Instead,
// position p of a sequence is stored at p ^ f(p >> 4) (f < 16, so every
// aligned 16-block is permuted in place and contiguous accesses stay
// conflict-free), with f chosen per stage -- the array that pass s - 1
// writes and pass s reads; stage 0, the transform's input, shares the last
// stage's layout -- to spread the writes of pass s - 1: with NS = product of
// the radices before it and R its radix (both powers of two, NS < 16), the 16
// lanes of a write cover 16 / NS butterfly groups, and f gives each group
// its own value in bits log2(NS) .. 3.
template <class PL, int STG> __device__ __forceinline__ int stage_swz(int row) {
  constexpr int st = (STG == 0 || STG >= PL::np) ? PL::np - 1 : STG;
  if constexpr (st == 0) {
    return 0;
  } else {
    constexpr int NSW = plan_ns<PL>(st - 1), RW = PL::r[st - 1];
    if constexpr (NSW >= 16 || !is_pow2(NSW) || !is_pow2(RW) || PL::N % 16 != 0) {
      return 0;
    } else if constexpr (NSW * RW >= 16) {
      // row >= 0: unsigned arithmetic, so the powers of two become shifts and masks
      return (int)((((unsigned)row / (NSW * RW / 16)) % (16 / NSW)) << ilog2(NSW));
    } else {
      return (int)(((unsigned)row % RW) << ilog2(NSW));
    }
  }
}

// LDS element address of (sequence b, position pos) in stage STG of plan PL
// (the stage matters only to a swizzled layout).
template <int ES, int BS, int PADSH, class PL = void, int STG = 0>
__device__ __forceinline__ int lds_at(int b, int pos) {
  constexpr int PS = pad_shift<PADSH>();
  if constexpr (swizzled<PADSH>()) return b * BS + (pos ^ stage_swz<PL, STG>(pos >> 4)) * ES;
  else if constexpr (PS > 0) return b * BS + pos * ES + (pos >> PS);
  else return b * BS + pos * ES;
}

// LDS read that the compiler may not pair with a neighbour into one ds_read2
// instruction: on gfx950 a ds_read2_b64 keeps the LDS busy four times as long
// as a ds_read_b64 (half the read bandwidth), while pairing writes costs
// nothing.  Used where linear addressing or an unpadded (swizzled) layout
// leaves reads a multiple of 8 or 512 bytes apart from a common base.
template <typename X> __device__ __forceinline__ X lds_rd(const X* p) {
  X v = *p;
  asm volatile("" ::: "memory");
  return v;
}

// True when the twiddle index k = j mod NS of a pass is the same in every slot
// w = tid + i NT of a thread (lane_map MAP over NB sequences of NBF
// butterflies): MAP 1 gives j = w mod NBF and NS divides NBF, MAP 0 gives
// j = w / NB.  The thread then reads its R - 1 twiddles once per pass.
template <int MAP, int NB, int NBF, int NT, int NS> constexpr bool slot_invariant_k() {
  if (MAP == 3 || MAP == 4) return 64 % NS == 0 && NBF % NS == 0;
  if (MAP == 1) return NT % NS == 0;
  if (MAP == 0) return NT % NB == 0 && (NT / NB) % NS == 0;
  return false;
}

// Twiddles t[r] = tw[k r N/(NS R)], r = 1..R-1, of butterfly j (k = j mod NS).
template <typename T, int N, int R, int NS>
__device__ __forceinline__ void load_pass_twiddles(cx<T> (&t)[R], const cx<T>* tw, int j) {
  const int k = j % NS;
#pragma unroll
  for (int r = 1; r < R; ++r) t[r] = tw[k * r * (N / (NS * R))];
}

// (sequence b, butterfly j) of slot i of thread tid: lane_map on
// w = tid + i NT.  Linear addressing (LIN): when NT is a multiple of the
// faster-running index's range the slots differ only in the slower index, by
// a constant step; that is written out so that LDS addresses become one base
// plus immediate offsets, which saves the address registers of every slot and
// radix element (at N = 512 the mixed-precision flux pass spilled without
// it).  Without LIN the compiler keeps one precomputed address per element,
// and its reads stay single ds_read_b64s.
template <int NB, int NBF, int NT, int MAP, bool LIN = true>
__device__ __forceinline__ void slot_map(int tid, int i, int& b, int& j) {
  if constexpr (wave_map<MAP>()) {
    wave_slot<NB, NBF, NT>(tid, i, b, j);
  } else if constexpr (LIN && MAP == 1 && NT % NBF == 0) {
    b = tid / NBF + i * (NT / NBF);
    j = tid % NBF;
  } else if constexpr (LIN && MAP == 0 && NT % NB == 0) {
    b = tid % NB;
    j = tid / NB + i * (NT / NB);
  } else {
    lane_map<NB, NBF, MAP>(tid + i * NT, b, j);
  }
}

// With linear addressing: the LDS address step from position p to p + STEP
// when it is the same for every p (no padding, or STEP a multiple of the
// padding period); 0 otherwise, and always 0 without linear addressing.
template <int ES, int PADSH, int STEP> constexpr int lds_step() {
  constexpr int PS = pad_shift<PADSH>();
  if (!linear_addr<PADSH>() || swizzled<PADSH>()) return 0;
  if (PS == 0) return STEP * ES;
  if (STEP % (1 << PS) == 0) return STEP * ES + (STEP >> PS);
  return 0;
}

// Step between the R output positions d + r NS of a Stockham butterfly
// (d = (j / NS) NS R + j mod NS).  In a first pass (NS = 1) d is a multiple of
// R, so when R divides the padding period the R outputs share one padding
// slot count and the step is ES.
template <int ES, int PADSH, int NS, int R> constexpr int lds_write_step() {
  constexpr int PS = pad_shift<PADSH>();
  if (linear_addr<PADSH>() && !swizzled<PADSH>() && NS == 1 && PS > 0 && (1 << PS) % R == 0) return ES;
  return lds_step<ES, PADSH, NS>();
}

// One VALU Stockham pass.  NB sequences, NT threads; B_ACT (<= NB) of them active.
template <typename T, class PL, int NB, int NT, int ES, int BS, int S, int P, int MAP = 0, int PADSH = 0>
__device__ __forceinline__ void fft_pass_valu(cx<T>* buf, const cx<T>* tw, int tid, int b_act) {
  constexpr int N = PL::N;
  constexpr int R = PL::r[P];
  constexpr int NS = plan_ns<PL>(P);
  constexpr int NBF = N / R;
  constexpr int TOT = NB * NBF;
  constexpr int CNT = slot_count<NB, NBF, NT, MAP>();
  constexpr bool TWS = NS > 1 && CNT > 1 && slot_invariant_k<MAP, NB, NBF, NT, NS>();
  constexpr int RSTEP = lds_step<ES, PADSH, NBF>();
  constexpr int WSTEP = lds_write_step<ES, PADSH, NS, R>();
  cx<T> tws[R];
  if constexpr (TWS) {
    int b0, j0;
    slot_map<NB, NBF, NT, MAP, linear_addr<PADSH>()>(tid, 0, b0, j0);
    load_pass_twiddles<T, N, R, NS>(tws, tw, j0);
  }
  cx<T> v[CNT][R];
#pragma unroll
  for (int i = 0; i < CNT; ++i) {
    int b, j;
    slot_map<NB, NBF, NT, MAP, linear_addr<PADSH>()>(tid, i, b, j);
    if ((wave_map<MAP>() || TOT % NT == 0 || tid + i * NT < TOT) && b < b_act) {
      if constexpr (RSTEP > 0) {
        const int a0 = lds_at<ES, BS, PADSH, PL, P>(b, j);
#pragma unroll
        for (int r = 0; r < R; ++r) v[i][r] = lds_rd(&buf[a0 + r * RSTEP]);
      } else {
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const cx<T>* src = &buf[lds_at<ES, BS, PADSH, PL, P>(b, j + r * NBF)];
          v[i][r] = swizzled<PADSH>() ? lds_rd(src) : *src;
        }
      }
      if constexpr (NS > 1) {
        cx<T> t[R];
        if constexpr (TWS) {
#pragma unroll
          for (int r = 1; r < R; ++r) t[r] = tws[r];
        } else {
          load_pass_twiddles<T, N, R, NS>(t, tw, j);
        }
#pragma unroll
        for (int r = 1; r < R; ++r) v[i][r] = (S < 0) ? cmul(v[i][r], t[r]) : cmulc(v[i][r], t[r]);
      }
      dft<R, S>(v[i]);
    }
  }
  pass_sync<MAP>();
#pragma unroll
  for (int i = 0; i < CNT; ++i) {
    int b, j;
    slot_map<NB, NBF, NT, MAP, linear_addr<PADSH>()>(tid, i, b, j);
    if ((wave_map<MAP>() || TOT % NT == 0 || tid + i * NT < TOT) && b < b_act) {
      const int k = j % NS;
      const int d = (j / NS) * NS * R + k;
      if constexpr (WSTEP > 0) {
        const int a0 = lds_at<ES, BS, PADSH, PL, P + 1>(b, d);
#pragma unroll
        for (int r = 0; r < R; ++r) buf[a0 + r * WSTEP] = v[i][r];
      } else {
#pragma unroll
        for (int r = 0; r < R; ++r) buf[lds_at<ES, BS, PADSH, PL, P + 1>(b, d + r * NS)] = v[i][r];
      }
    }
  }
  pass_sync<MAP>();
}

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

// A-operand halves of the 16-point DFT as a real 32 x 32 matrix for this lane.
// The 32 real inputs are ordered with Re and Im interleaved, k = 2 r + c
// (c = 0: Re x_r, c = 1: Im x_r); lane (q = lane mod 16, g = lane / 16) holds
// row q, k = 8 g .. 8 g + 7, i.e. inputs r = 4 g .. 4 g + 3.  Block 0 gives
// Re y_q, block 1 Im y_q.
template <int S>
__device__ __forceinline__ void dft16_operands(int lane, bf16x8& a0h, bf16x8& a0l, bf16x8& a1h, bf16x8& a1l) {
  const int q = lane & 15, g = lane >> 4;
#pragma unroll
  for (int t = 0; t < 8; ++t) {
    const int r = 4 * g + (t >> 1);  // input index
    const bool im_in = (t & 1) != 0;  // Im x_r
    const int m = (q * r) & 15;
    const float re = float(kCos16[m]);
    const float im = float(S) * float(kCos16[(m + 12) & 15]);
    const float w0 = im_in ? -im : re;  // Re y: Re W Re x - Im W Im x
    const float w1 = im_in ? re : im;   // Im y: Im W Re x + Re W Im x
    const __bf16 h0 = (__bf16)w0, h1 = (__bf16)w1;
    a0h[t] = h0;
    a0l[t] = (__bf16)(w0 - (float)h0);
    a1h[t] = h1;
    a1l[t] = (__bf16)(w1 - (float)h1);
  }
}

// Radix-16 Stockham pass on the MFMA units (FP32 data, split BF16 x 3).  Each
// wave takes 16 butterflies at a time: lane (n = lane mod 16, g = lane / 16)
// reads elements 4 g .. 4 g + 3 of butterfly n, twiddles them in FP32 and
// splits their real and imaginary parts into the B operand (k = 2 r + c, as
// in dft16_operands); after the products lane (n, g) holds outputs
// q = 4g .. 4g+3 of butterfly n.
template <class PL, int NB, int NT, int ES, int BS, int S, int P, int MAP, int PADSH>
__device__ __forceinline__ void fft_pass_mfma(float2* buf, const float2* tw, int tid, int b_act) {
  static_assert(!wave_map<MAP>(), "MFMA passes use the workgroup lane maps");
  constexpr int N = PL::N;
  constexpr int R = 16;
  constexpr int NS = plan_ns<PL>(P);
  constexpr int NBF = N / R;
  constexpr int TOT = NB * NBF;
  constexpr int NGRP = (TOT + 15) / 16;
  constexpr int NW = NT / 64;
  constexpr int GPW = (NGRP + NW - 1) / NW;  // groups per wave
  const int lane = tid & 63, wv = tid >> 6;
  const int n = lane & 15, g = lane >> 4;
  bf16x8 a0h, a0l, a1h, a1l;
  dft16_operands<S>(lane, a0h, a0l, a1h, a1l);
  floatx4 yr[GPW], yi[GPW];
#pragma unroll
  for (int s = 0; s < GPW; ++s) {
    const int grp = wv + s * NW;
    const int w = grp * 16 + n;
    int b, j;
    lane_map<NB, NBF, MAP>(w, b, j);
    const bool ok = grp < NGRP && w < TOT && b < b_act;
    const int k = j % NS;
    bf16x8 xh, xl;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int r = 4 * g + e;
      float2 x = ok ? buf[lds_at<ES, BS, PADSH, PL, P>(b, j + r * NBF)] : make_float2(0.f, 0.f);
      if constexpr (NS > 1) {
        if (r > 0) {
          const float2 tv = tw[k * r * (N / (NS * R))];
          x = (S < 0) ? cmul(x, tv) : cmulc(x, tv);
        }
      }
      const __bf16 hr = (__bf16)x.x, hi = (__bf16)x.y;
      xh[2 * e] = hr;
      xl[2 * e] = (__bf16)(x.x - (float)hr);
      xh[2 * e + 1] = hi;
      xl[2 * e + 1] = (__bf16)(x.y - (float)hi);
    }
    floatx4 c0 = {0.f, 0.f, 0.f, 0.f}, c1 = {0.f, 0.f, 0.f, 0.f};
    c0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0h, xh, c0, 0, 0, 0);
    c0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0h, xl, c0, 0, 0, 0);
    c0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0l, xh, c0, 0, 0, 0);
    c1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1h, xh, c1, 0, 0, 0);
    c1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1h, xl, c1, 0, 0, 0);
    c1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1l, xh, c1, 0, 0, 0);
    yr[s] = c0;
    yi[s] = c1;
  }
  __syncthreads();
#pragma unroll
  for (int s = 0; s < GPW; ++s) {
    const int grp = wv + s * NW;
    const int w = grp * 16 + n;
    int b, j;
    lane_map<NB, NBF, MAP>(w, b, j);
    if (grp < NGRP && w < TOT && b < b_act) {
      const int k = j % NS;
      const int d = (j / NS) * NS * R + k;
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int q = 4 * g + t;
        buf[lds_at<ES, BS, PADSH, PL, P + 1>(b, d + q * NS)] = make_float2(yr[s][t], yi[s][t]);
      }
    }
  }
  __syncthreads();
}

// Last radix-16 pass on the MFMA units.  In the last Stockham pass every
// butterfly writes its outputs onto its own input positions (d = j), so the
// groups need no common barrier: each group of 16 butterflies is read,
// multiplied and handed to store(s, t, b, pos, value) (s = group slot of this
// wave, t = 0..3 the lane's four outputs) before the next group is read.
// store() may write the LDS positions in place.
template <class PL, int NB, int NT, int ES, int BS, int S, int P, int MAP, int PADSH, class Store, bool SLOTS = false,
          int UNR = 1>
__device__ __forceinline__ void fft_pass_mfma_last(const float2* buf, const float2* tw, int tid, int b_act,
                                                   Store&& store) {
  constexpr int N = PL::N;
  constexpr int R = 16;
  constexpr int NS = plan_ns<PL>(P);
  static_assert(NS * R == N, "the in-place MFMA pass must be the last pass");
  constexpr int NBF = N / R;
  constexpr int TOT = NB * NBF;
  constexpr int NGRP = (TOT + 15) / 16;
  constexpr int NW = NT / 64;
  // groups per wave: workgroup maps deal the groups round-robin over the
  // waves; wave maps give each wave the groups of its own sequences
  constexpr int GPW = wave_map<MAP>() ? (seqs_per_wave<NB, NT>() * NBF + 15) / 16 : (NGRP + NW - 1) / NW;
  const int lane = tid & 63, wv = tid >> 6;
  const int n = lane & 15, g = lane >> 4;
  bf16x8 a0h, a0l, a1h, a1l;
  dft16_operands<S>(lane, a0h, a0l, a1h, a1l);
  auto group = [&](int s) {
    int b, j;
    bool ok;
    if constexpr (wave_map<MAP>()) {
      const int u = s * 16 + n;  // butterfly index over the wave's sequences
      const int fl = u / NBF;
      j = u - fl * NBF;
      b = fl * NW + wv;
      ok = fl < seqs_per_wave<NB, NT>() && b < b_act;
    } else {
      const int grp = wv + s * NW;
      const int w = grp * 16 + n;
      lane_map<NB, NBF, MAP>(w, b, j);
      ok = grp < NGRP && w < TOT && b < b_act;
    }
    bf16x8 xh, xl;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int r = 4 * g + e;
      float2 x = ok ? buf[lds_at<ES, BS, PADSH, PL, P>(b, j + r * NBF)] : make_float2(0.f, 0.f);
      if (r > 0) {
        const float2 tv = tw[j * r];  // k = j in the last pass
        x = (S < 0) ? cmul(x, tv) : cmulc(x, tv);
      }
      const __bf16 hr = (__bf16)x.x, hi = (__bf16)x.y;
      xh[2 * e] = hr;
      xl[2 * e] = (__bf16)(x.x - (float)hr);
      xh[2 * e + 1] = hi;
      xl[2 * e + 1] = (__bf16)(x.y - (float)hi);
    }
    floatx4 c0 = {0.f, 0.f, 0.f, 0.f}, c1 = {0.f, 0.f, 0.f, 0.f};
    c0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0h, xh, c0, 0, 0, 0);
    c0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0h, xl, c0, 0, 0, 0);
    c0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0l, xh, c0, 0, 0, 0);
    c1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1h, xh, c1, 0, 0, 0);
    c1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1h, xl, c1, 0, 0, 0);
    c1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1l, xh, c1, 0, 0, 0);
    if (ok) {
#pragma unroll
      for (int t = 0; t < 4; ++t) store(s, t, b, j + (4 * g + t) * NS, make_float2(c0[t], c1[t]));
    }
  };
  // The groups run one after another.  The loop is unrolled completely when
  // the store keeps its results in registers indexed by the group slot;
  // otherwise by UNR groups (1, 2 or 4, per kernel by measurement), which
  // overlaps one group's LDS latency and MFMA chain with the next group's
  // work at the cost of registers.
  if constexpr (SLOTS) {
#pragma unroll
    for (int s = 0; s < GPW; ++s) group(s);
  } else if constexpr (UNR >= 4) {
#pragma unroll 4
    for (int s = 0; s < GPW; ++s) group(s);
  } else if constexpr (UNR == 2) {
#pragma unroll 2
    for (int s = 0; s < GPW; ++s) group(s);
  } else {
#pragma unroll 1
    for (int s = 0; s < GPW; ++s) group(s);
  }
}

// Positions r NBF .. r NBF + NBF - 1 of output row r lie strictly between
// KEEP and N - KEEP (bit r set): outputs a caller does not want when KEEP > 0.
template <int N, int NBF, int R, int KEEP> constexpr unsigned gap_rows() {
  unsigned m = 0;
  if (KEEP > 0)
    for (int r = 0; r < R; ++r)
      if (r * NBF > KEEP && r * NBF + NBF - 1 < N - KEEP) m |= 1u << r;
  return m;
}

// Last VALU pass of a plan.  Butterfly j of sequence b reads positions
// j + r NBF and, since NS = NBF in the last pass, its outputs belong at those
// same positions.  INPLACE: they are written back there (no barrier needed in
// between; store is not called); otherwise they go to
// store(i, r, b, j + r NBF, value).  KEEP > 0: positions strictly between KEEP
// and N - KEEP are not wanted; the output rows r that lie wholly there are
// neither computed nor stored.
template <typename T, class PL, int NB, int NT, int ES, int BS, int S, int MAP, int PADSH, int KEEP, bool INPLACE,
          class Store>
__device__ __forceinline__ void fft_last_valu(cx<T>* buf, const cx<T>* tw, int tid, int b_act, Store&& store) {
  constexpr int N = PL::N;
  constexpr int P = PL::np - 1;
  constexpr int R = PL::r[P];
  constexpr int NBF = N / R;
  constexpr int TOT = NB * NBF;
  constexpr int CNT = slot_count<NB, NBF, NT, MAP>();
  constexpr unsigned GAP = gap_rows<N, NBF, R, KEEP>();
  constexpr bool TWS = CNT > 1 && slot_invariant_k<MAP, NB, NBF, NT, NBF>();
  constexpr int RSTEP = lds_step<ES, PADSH, NBF>();
  cx<T> tws[R];
  if constexpr (TWS) {
    int b0, j0;
    slot_map<NB, NBF, NT, MAP, linear_addr<PADSH>()>(tid, 0, b0, j0);
    load_pass_twiddles<T, N, R, NBF>(tws, tw, j0);
  }
#pragma unroll
  for (int i = 0; i < CNT; ++i) {
    int b, j;
    slot_map<NB, NBF, NT, MAP, linear_addr<PADSH>()>(tid, i, b, j);
    if ((wave_map<MAP>() || TOT % NT == 0 || tid + i * NT < TOT) && b < b_act) {
      cx<T> v[R], t[R];
      const int a0 = lds_at<ES, BS, PADSH, PL, P>(b, j);
#pragma unroll
      for (int r = 0; r < R; ++r) {
        if constexpr (RSTEP > 0) v[r] = lds_rd(&buf[a0 + r * RSTEP]);
        else if constexpr (swizzled<PADSH>()) v[r] = lds_rd(&buf[lds_at<ES, BS, PADSH, PL, P>(b, j + r * NBF)]);
        else v[r] = buf[lds_at<ES, BS, PADSH, PL, P>(b, j + r * NBF)];
      }
      if constexpr (TWS) {
#pragma unroll
        for (int r = 1; r < R; ++r) t[r] = tws[r];
      } else {
        load_pass_twiddles<T, N, R, NBF>(t, tw, j);  // k = j in the last pass
      }
#pragma unroll
      for (int r = 1; r < R; ++r) v[r] = (S < 0) ? cmul(v[r], t[r]) : cmulc(v[r], t[r]);
      dft<R, S>(v);
#pragma unroll
      for (int r = 0; r < R; ++r) {
        if ((GAP >> r) & 1u) continue;
        if constexpr (INPLACE) buf[RSTEP > 0 ? a0 + r * RSTEP : lds_at<ES, BS, PADSH, PL, P>(b, j + r * NBF)] = v[r];
        else store(i, r, b, j + r * NBF, v[r]);
      }
    }
  }
}

template <typename T, class PL, int NB, int NT, int ES, int BS, int S, int P, int MAP = 0, int PADSH = 0>
__device__ __forceinline__ void fft_pass(cx<T>* buf, const cx<T>* tw, int tid, int b_act) {
  if constexpr (PL::MX && PL::r[P] == 16) {
    static_assert(sizeof(T) == 4, "the mixed path works on FP32 data");
    fft_pass_mfma<PL, NB, NT, ES, BS, S, P, MAP, PADSH>(reinterpret_cast<float2*>(buf),
                                                        reinterpret_cast<const float2*>(tw), tid, b_act);
  } else {
    fft_pass_valu<T, PL, NB, NT, ES, BS, S, P, MAP, PADSH>(buf, tw, tid, b_act);
  }
}

// All passes LDS to LDS; the last pass runs in place (butterfly by butterfly
// on the VALU, group by group on the MFMA units) and is followed by a barrier.
// KEEP > 0: only positions <= KEEP and >= N - KEEP of the result are wanted
// (the others may be left stale).
template <typename T, class PL, int NB, int NT, int ES, int BS, int S, int MAP = 0, int PADSH = 0, int KEEP = 0,
          int UNR = 1, int P = 0>
__device__ __forceinline__ void lds_fft(cx<T>* buf, const cx<T>* tw, int tid, int b_act) {
  static_assert(plan_ok<PL>(), "radix plan does not multiply to N");
  if constexpr (P < PL::np) {
    if constexpr (PL::MX && PL::r[P] == 16 && P == PL::np - 1 && P > 0) {
      float2* fb = reinterpret_cast<float2*>(buf);
      auto st = [&](int, int, int b, int pos, float2 v) { fb[lds_at<ES, BS, PADSH, PL, P>(b, pos)] = v; };
      fft_pass_mfma_last<PL, NB, NT, ES, BS, S, P, MAP, PADSH, decltype(st)&, false, UNR>(
          fb, reinterpret_cast<const float2*>(tw), tid, b_act, st);
      pass_sync<MAP>();
    } else if constexpr (P == PL::np - 1 && P > 0) {
      fft_last_valu<T, PL, NB, NT, ES, BS, S, MAP, PADSH, KEEP, true>(buf, tw, tid, b_act,
                                                                       [](int, int, int, int, cx<T>) {});
      pass_sync<MAP>();
    } else {
      fft_pass<T, PL, NB, NT, ES, BS, S, P, MAP, PADSH>(buf, tw, tid, b_act);
      lds_fft<T, PL, NB, NT, ES, BS, S, MAP, PADSH, KEEP, UNR, P + 1>(buf, tw, tid, b_act);
    }
  }
}

// Passes 1 .. np-2 of a plan, LDS to LDS.
template <typename T, class PL, int NB, int NT, int ES, int BS, int S, int MAP, int PADSH, int P>
__device__ __forceinline__ void fft_mid_passes(cx<T>* buf, const cx<T>* tw, int tid, int b_act) {
  if constexpr (P < PL::np - 1) {
    fft_pass<T, PL, NB, NT, ES, BS, S, P, MAP, PADSH>(buf, tw, tid, b_act);
    fft_mid_passes<T, PL, NB, NT, ES, BS, S, MAP, PADSH, P + 1>(buf, tw, tid, b_act);
  }
}

// Shape of the first pass of a plan: R elements per butterfly, CNT
// butterflies per thread.
template <class PL, int NB, int NT, int MAP = 1> struct FirstPass {
  static constexpr int R = PL::r[0];
  static constexpr int NBF = PL::N / R;
  static constexpr int TOT = NB * NBF;
  static constexpr int CNT = slot_count<NB, NBF, NT, MAP>();
};

// Per-thread shape of the last pass: outputs are handed to store(i, r, ...)
// for CNT slots i of R outputs r.  VALU last pass: slot i is the thread's i-th
// butterfly and r its R outputs.  MFMA radix-16 last pass: slot i is the
// wave's i-th group of 16 butterflies and r the lane's four outputs.
template <class PL, int NB, int NT> struct LastPass {
  static constexpr int RL = PL::r[PL::np - 1];
  static constexpr bool MFMA = PL::MX && RL == 16 && PL::np > 1;
  static constexpr int NBF = PL::N / RL;
  static constexpr int TOT = NB * NBF;
  static constexpr int NGRP = (TOT + 15) / 16;
  static constexpr int NW = NT / 64;
  static constexpr int CNT = MFMA ? (NGRP + NW - 1) / NW : (TOT + NT - 1) / NT;
  static constexpr int R = MFMA ? 4 : RL;
};

// (sequence b, position pos) of output slot (i, r) of this thread in the last
// pass; false if the slot is idle.
template <class PL, int NB, int NT, int MAP>
__device__ __forceinline__ bool last_slot(int tid, int i, int r, int& b, int& pos) {
  using LP = LastPass<PL, NB, NT>;
  constexpr int NS = PL::N / LP::RL;
  int j;
  if constexpr (LP::MFMA) {
    const int lane = tid & 63, wv = tid >> 6, n = lane & 15, g = lane >> 4;
    const int grp = wv + i * LP::NW;
    const int w = grp * 16 + n;
    lane_map<NB, LP::NBF, MAP>(w, b, j);
    pos = j + (4 * g + r) * NS;
    return grp < LP::NGRP && w < LP::TOT;
  } else {
    const int w = tid + i * NT;
    lane_map<NB, LP::NBF, MAP>(w, b, j);
    pos = j + r * NS;
    return LP::TOT % NT == 0 || w < LP::TOT;
  }
}

// First pass from values already in registers (v[i][r] = element j + r*NBF of
// sequence b for this thread's i-th butterfly): R-point DFTs, then either the
// final outputs (one-pass plans) or the LDS writes of the next pass, followed
// by a barrier.
template <typename T, class PL, int NB, int NT, int ES, int BS, int S, int MAP, int PADSH, unsigned ZM = 0,
          class Store>
__device__ __forceinline__ void fft_first_regs(cx<T>* buf, cx<T> (&v)[FirstPass<PL, NB, NT, MAP>::CNT][PL::r[0]],
                                               int tid, int b_act, Store&& store) {
  using FP = FirstPass<PL, NB, NT, MAP>;
  constexpr int NP = PL::np;
#pragma unroll
  for (int i = 0; i < FP::CNT; ++i) {
    int b, j;
    if (first_slot<NB, FP::NBF, NT, MAP>(tid, i, b, j) && b < b_act) {
      dft_z<FP::R, S, ZM>(v[i]);
      if constexpr (NP == 1) {
#pragma unroll
        for (int r = 0; r < FP::R; ++r) store(i, r, b, r, v[i][r]);
      } else {
        constexpr int WSTEP = lds_write_step<ES, PADSH, 1, FP::R>();
        const int a0 = lds_at<ES, BS, PADSH, PL, 1>(b, j * FP::R);
#pragma unroll
        for (int r = 0; r < FP::R; ++r)
          buf[WSTEP > 0 ? a0 + r * WSTEP : lds_at<ES, BS, PADSH, PL, 1>(b, j * FP::R + r)] = v[i][r];
      }
    }
  }
  if constexpr (NP > 1) pass_sync<MAP>();
}

// Middle passes (LDS to LDS) and the last pass, whose outputs go to
// store(i, r, b, pos, value) with pos = j + r N/R for the thread's i-th
// butterfly j.  On the VALU the last pass computes straight into registers;
// an MFMA last pass writes LDS and the same (i, r, pos) are then read back.
// INPLACE: a VALU last pass writes its outputs back to the LDS positions it
// read instead of calling store (which must then write LDS position pos of
// sequence b, as it is still called by an MFMA last pass).
template <typename T, class PL, int NB, int NT, int ES, int BS, int S, int MAP, int PADSH, bool SLOTS = false,
          bool INPLACE = false, int UNR = 1, class Store>
__device__ __forceinline__ void fft_rest(cx<T>* buf, const cx<T>* tw, int tid, int b_act, Store&& store) {
  constexpr int NP = PL::np;
  if constexpr (NP > 1) {
    fft_mid_passes<T, PL, NB, NT, ES, BS, S, MAP, PADSH, 1>(buf, tw, tid, b_act);
    constexpr int PLAST = NP - 1;
    constexpr int R = PL::r[PLAST];
    if constexpr (PL::MX && R == 16) {
      auto st2 = [&](int i, int r, int b, int pos, float2 v) {
        cx<T> vv;
        vv.x = v.x;
        vv.y = v.y;
        store(i, r, b, pos, vv);
      };
      fft_pass_mfma_last<PL, NB, NT, ES, BS, S, PLAST, MAP, PADSH, decltype(st2)&, SLOTS, UNR>(
          reinterpret_cast<const float2*>(buf), reinterpret_cast<const float2*>(tw), tid, b_act, st2);
    } else {
      fft_last_valu<T, PL, NB, NT, ES, BS, S, MAP, PADSH, 0, INPLACE>(buf, tw, tid, b_act, store);
    }
  }
}

// Register-ended FFT: the first pass takes its inputs from load(b, pos)
// (global memory) and the last pass hands its outputs to
// store(i, r, b, pos, value); only the passes in between go through LDS.
// load() is called for all CNT*R elements of a thread before any arithmetic,
// so their memory requests are in flight together.  For one-pass plans the
// inputs go straight from load() through the DFT to store().  The LDS buffer
// may be reused after this returns only past a __syncthreads().
template <typename T, class PL, int NB, int NT, int ES, int BS, int S, int MAP = 0, int PADSH = 0, bool SLOTS = false, class Load,
          class Store>
__device__ __forceinline__ void fft_reg(cx<T>* buf, const cx<T>* tw, int tid, int b_act, Load&& load,
                                        Store&& store) {
  static_assert(plan_ok<PL>(), "radix plan does not multiply to N");
  using FP = FirstPass<PL, NB, NT, MAP>;
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
  fft_first_regs<T, PL, NB, NT, ES, BS, S, MAP, PADSH>(buf, v, tid, b_act, store);
  fft_rest<T, PL, NB, NT, ES, BS, S, MAP, PADSH, SLOTS>(buf, tw, tid, b_act, store);
}

// Item order of a persistent grid of G workgroups over `total` items: the
// items are split into eight contiguous ranges, one per XCD, and the
// workgroups resident on an XCD (ids w with w mod 8 = x) walk that XCD's
// range together.  Returns the k-th item of workgroup w, or -1 when done.
// A grid of fewer than eight workgroups leaves some XCDs without one, so it
// walks the items with a plain stride instead.
__host__ __device__ __forceinline__ int64_t xcd_item(int w, int G, int64_t k, int64_t total) {
  constexpr int X = 8;
  if (G < X) {
    const int64_t idx = (int64_t)w + k * G;
    return idx < total ? idx : -1;
  }
  const int xcd = w % X, slot = w / X;
  const int per = G / X + (xcd < G % X ? 1 : 0);
  const int64_t base = total / X, rem = total % X;
  const int64_t start = xcd * base + (xcd < rem ? xcd : rem);
  const int64_t len = base + (xcd < rem ? 1 : 0);
  const int64_t idx = k * per + slot;
  return idx < len ? start + idx : -1;
}

// Workgroup id remap for gfx950's eight XCDs (non-persistent grids).
__device__ __forceinline__ int xcd_remap(int w, int total) {
  constexpr int X = 8;
  const int per = total / X, rem = total % X;
  const int xcd = w % X, slot = w / X;
  return xcd < rem ? xcd * (per + 1) + slot : rem * (per + 1) + (xcd - rem) * per + slot;
}

MHD_SCHED_END
}  // namespace mhd

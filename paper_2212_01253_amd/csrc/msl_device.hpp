// Device building blocks of libmsl: compensated complex arithmetic, the
// register/LDS line FFT, the slice transmission and the line-pass program.
//
// Numerical design.  The multislice recurrence (Eq. 1 of arXiv 2212.01253)
// applies the same propagator, FFT twiddles and (for a bar that spans many
// slices) the same transmission value thousands of times.  A constant rounded
// once to float32 therefore contributes the same relative error at every
// slice and the errors add up linearly with the slice count, while the
// rounding of data-dependent sums and products behaves like a random walk.
// The constants of the paraxial passes (FFT twiddles, the radix-8 internal
// factor sqrt(1/2), the one-axis propagator) are therefore single float32
// values that change from pass to pass: each one takes, over a cycle of
// DITHER passes along its axis, its two neighbouring float32 values in the
// order of a first-order sigma-delta modulator, so the running sum of its
// rounding errors stays within about one ulp instead of growing with the
// slice count (pass s uses cycle position tab = (s / 2) mod DITHER, the same
// in the forward sweep, the recompute and the reverse sweep, which is then
// the exact adjoint of the computed forward).  The exact 2-D propagator,
// applied through its own table, stays a two-term (hi + lo) constant applied
// through FMAs.  The transmission is applied as psi + psi * (T - 1) with
// T - 1 evaluated directly, so that its rounding is relative to the small
// quantity T - 1.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace msl {

enum Axis : int { ROW = 0, COL = 1 };  // ROW: line along z (contiguous), COL: along y

enum PreOp : int { PRE_NONE = 0, PRE_PROP = 1, PRE_FFT = 2, PRE_IFFT_N = 3, PRE_IFFT_U = 4 };
enum MidOp : int { MID_NONE = 0, MID_T_FWD = 1, MID_T_ADJ = 2, MID_FF_OUT = 3, MID_FF_SEED = 4 };
enum PostOp : int { POST_NONE = 0, POST_PROP = 1, POST_FFT = 2, POST_PROP2D = 3 };

// One sweep over all lines of one axis.
struct PassDesc {
  int axis;
  int pre, mid, post;
  int conj;             // adjoint: use conj(h) / conj(H)
  int slice;            // slice index of the transmission step
  int tab;              // position in the constants' cycle, 0 .. DITHER - 1
  const float2* src;    // field read
  float2* dst;          // field written (may equal src; nullptr = not written)
  float2* psi_store;    // store the line before the mid step (nullptr = no)
  const float2* psi_load;  // entrance field psi_s for the adjoint step
  // layouts of the four field arrays: LAY_R row-major [ny][nz] (caller
  // arrays), LAY_T 2x2-tiled (working fields; see tile_addr), LAY_C 2x2
  // tiles in column order (fields only column passes touch; see tile_addr_c)
  int src_lay, dst_lay, store_lay, load_lay;
};

enum Layout : int { LAY_R = 0, LAY_T = 1, LAY_C = 2 };

// Everything a pass reads besides the descriptor.
struct Ctx {
  int ny, nz;
  int64_t m;                        // ny * nz
  const float* delta;               // [Ns][ny][nz]
  const float* beta;
  float* gdelta;                    // [Ns][ny][nz] or nullptr
  float* gbeta;
  // Line tables, [DITHER][n] float2: row tab holds the constants of cycle
  // position tab (see above)
  const float2* twz;                // W_nz^e, e < nz
  const float2* twy;                // W_ny^e, e < ny
  const float2* hz;                 // paraxial h_z / nz (DFT order)
  const float2* hy;                 // paraxial h_y / ny
  const float2* H_hi; const float2* H_lo;       // exact H[ky][kz] / ny, two-term
  float kdx_hi, kdx_lo;             // k * dx as a two-term float
  float inv_m;                      // 1 / (ny nz)
  float* intensity;                 // far-field output (fftshifted) or nullptr
  const float* grad_intensity;      // far-field seed input (fftshifted) or nullptr
  // Paraxial schedule: the workspace may hold T - 1 of every slice
  // precomputed, [Ns] 2x2-tiled fields (float2), even slices (row passes) in
  // row tile order, odd slices (column passes) in column tile order, so that
  // each pass reads its slice contiguously and spends no arithmetic on the
  // transmission.  gT stages the odd slices' (dL/d delta, dL/d beta), [Ns/2]
  // fields in column tile order, so those passes write contiguous tiles
  // instead of striding through the caller's row-major gradient stacks.
  const float2* dbT;                // or nullptr
  float2* gT;                       // or nullptr
  // Compact stacks (batched forward): delta, beta and dbT hold a pool of
  // n_pool distinct slices and slice s is pool slice slice_index[s] (device
  // array, values clamped to the pool); dbT then holds T - 1 of every pool
  // slice.  nullptr: slice s is stack slice s.
  const int32_t* slice_index;
  int32_t n_pool;
};

// ---------------------------------------------------------------------------
// constants cycle

constexpr int DITHER = 64;  // passes per axis in one cycle of the constants

// sqrt(1/2) and its float32 neighbours below and above
constexpr double RS2 = 0.70710678118654752440;
constexpr float RS2_DN = 0.70710677f;
constexpr float RS2_UP = 0.70710683f;
static_assert((double)RS2_DN < RS2 && RS2 < (double)RS2_UP, "neighbours of sqrt(1/2)");

// Bit i set: cycle position i uses RS2_UP.  First-order sigma-delta: each
// position takes the neighbour that keeps the running error sum smaller.
constexpr uint64_t rs2_cycle_mask() {
  uint64_t m = 0;
  double e = 0.0;
  for (int i = 0; i < DITHER; ++i) {
    const double dn = e + ((double)RS2_DN - RS2), upv = e + ((double)RS2_UP - RS2);
    if ((upv < 0 ? -upv : upv) < (dn < 0 ? -dn : dn)) {
      m |= 1ull << i;
      e = upv;
    } else {
      e = dn;
    }
  }
  return m;
}
constexpr uint64_t RS2_MASK = rs2_cycle_mask();

__host__ __device__ inline float rs2_at(int tab) { return ((RS2_MASK >> tab) & 1) ? RS2_UP : RS2_DN; }

// ---------------------------------------------------------------------------
// complex helpers

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }

// x * (wh + wl), or x * conj(wh + wl) when CONJ; the small product x*wl is
// formed first and folded into the rounding of the main product.
template <bool CONJ>
__device__ __forceinline__ float2 cmul_comp(float2 x, float2 wh, float2 wl) {
  const float whi = CONJ ? -wh.y : wh.y;
  const float wli = CONJ ? -wl.y : wl.y;
  const float cr = __builtin_fmaf(x.x, wl.x, -(x.y * wli));
  const float ci = __builtin_fmaf(x.x, wli, x.y * wl.x);
  const float re = __builtin_fmaf(x.x, wh.x, __builtin_fmaf(-x.y, whi, cr));
  const float im = __builtin_fmaf(x.x, whi, __builtin_fmaf(x.y, wh.x, ci));
  return make_float2(re, im);
}

__device__ __forceinline__ float2 cmul_comp_dyn(float2 x, float2 wh, float2 wl, bool conj) {
  return conj ? cmul_comp<true>(x, wh, wl) : cmul_comp<false>(x, wh, wl);
}

// x * w, or x * conj(w) when CONJ (single-term constant w).
template <bool CONJ>
__device__ __forceinline__ float2 cmul(float2 x, float2 w) {
  const float wi = CONJ ? -w.y : w.y;
  return make_float2(__builtin_fmaf(x.x, w.x, -(x.y * wi)), __builtin_fmaf(x.x, wi, x.y * w.x));
}

__device__ __forceinline__ float2 cmul_dyn(float2 x, float2 w, bool conj) {
  return conj ? cmul<true>(x, w) : cmul<false>(x, w);
}

// 4-point DFT, forward (W4 = -i) or inverse (W4 = +i), unnormalised.
template <bool INV>
__device__ __forceinline__ void dft4(float2 y0, float2 y1, float2 y2, float2 y3,
                                     float2& Y0, float2& Y1, float2& Y2, float2& Y3) {
  const float2 c0 = cadd(y0, y2), c1 = csub(y0, y2), c2 = cadd(y1, y3), d = csub(y1, y3);
  const float2 c3 = INV ? make_float2(-d.y, d.x) : make_float2(d.y, -d.x);
  Y0 = cadd(c0, c2);
  Y2 = csub(c0, c2);
  Y1 = cadd(c1, c3);
  Y3 = csub(c1, c3);
}

// 8-point DFT in place: v[k] <- sum_n v[n] W8^{+-nk}; rs2 is this pass's
// float32 value of sqrt(1/2).
template <bool INV>
__device__ __forceinline__ void dft8(float2 (&v)[8], float rs2) {
  const float2 a0 = cadd(v[0], v[4]), a1 = cadd(v[1], v[5]), a2 = cadd(v[2], v[6]), a3 = cadd(v[3], v[7]);
  float2 b0 = csub(v[0], v[4]), b1 = csub(v[1], v[5]), b2 = csub(v[2], v[6]), b3 = csub(v[3], v[7]);
  if (!INV) {
    b1 = make_float2((b1.x + b1.y) * rs2, (b1.y - b1.x) * rs2);    // * (1 - i)/sqrt2
    b2 = make_float2(b2.y, -b2.x);                                  // * -i
    b3 = make_float2((b3.y - b3.x) * rs2, -((b3.x + b3.y) * rs2));  // * (-1 - i)/sqrt2
  } else {
    b1 = make_float2((b1.x - b1.y) * rs2, (b1.x + b1.y) * rs2);     // * (1 + i)/sqrt2
    b2 = make_float2(-b2.y, b2.x);                                  // * +i
    b3 = make_float2(-((b3.x + b3.y) * rs2), (b3.x - b3.y) * rs2);  // * (-1 + i)/sqrt2
  }
  dft4<INV>(a0, a1, a2, a3, v[0], v[2], v[4], v[6]);
  dft4<INV>(b0, b1, b2, b3, v[1], v[3], v[5], v[7]);
}

template <bool INV>
__device__ __forceinline__ void dft2(float2& a, float2& b) {
  const float2 s = cadd(a, b), d = csub(a, b);
  a = s;
  b = d;
}

__device__ __forceinline__ int lds_pad(int i) { return i + (i >> 3); }

constexpr int ilog2c(int n) { return n <= 1 ? 0 : 1 + ilog2c(n >> 1); }

// Points per lane of an N-point line: 8 (one radix-8 butterfly per lane per
// stage) or 4 (radix-4), chosen per line length.  A line of N points takes
// L = N / P lanes.
#ifndef MSL_P4_MIN_N
#define MSL_P4_MIN_N 4096  // line length from which lines use 4 points per lane
#endif
#ifndef MSL_P8_MIN_N
#define MSL_P8_MIN_N 512   // shorter lines use 4 points per lane (twice the lanes per line)
#endif
template <int N>
struct LinePts {
  static constexpr int P = (N >= MSL_P4_MIN_N || N < MSL_P8_MIN_N) ? 4 : 8;
  static constexpr int L = N / P;
};

template <int P, bool INV>
__device__ __forceinline__ void dft_p(float2 (&v)[P], float rs2) {
  if constexpr (P == 8) {
    dft8<INV>(v, rs2);
  } else {
    float2 y0, y1, y2, y3;
    dft4<INV>(v[0], v[1], v[2], v[3], y0, y1, y2, y3);
    v[0] = y0;
    v[1] = y1;
    v[2] = y2;
    v[3] = y3;
  }
}

// Per-lane twiddles of one line FFT: lane j of an N-point line needs
// W_N^{(j mod NS) r N / (P NS)}, r = 1..P-1, for every twiddled radix-P stage
// (sub-length NS = R0, P R0, ...).  They are loaded once per pass into
// registers from the pass's row of the twiddle table and serve the forward
// and inverse transforms; rs2 is the pass's value of sqrt(1/2).
template <int N, int P = LinePts<N>::P>
struct LineTw {
  static constexpr int LG = ilog2c(N), LP = ilog2c(P);
  static constexpr int R0LOG = (LG % LP == 0) ? LP : (LG % LP);
  static constexpr int R0 = 1 << R0LOG;     // the one stage radix other than P (R0 = P: none)
  static constexpr int NST = (LG - R0LOG) / LP;
  // R0 = P: a radix-P stage without twiddles, then NST twiddled radix-P stages.
  // R0 < P: a radix-P stage without twiddles, NST - 1 twiddled radix-P stages,
  // and the radix-R0 stage last, where each lane's P / R0 butterflies take
  // R0 - 1 twiddles each (P - P / R0 per lane instead of the P - 1 of a
  // twiddled radix-P stage).
  static constexpr bool R0LAST = R0 < P;
  static constexpr int Q = P / R0;
  static constexpr int NPW = R0LAST ? NST - 1 : NST;  // twiddled radix-P stages
  float2 w[NPW > 0 ? NPW : 1][P - 1];
  float2 wl[R0LAST ? Q : 1][R0LAST ? R0 - 1 : 1];
  float rs2;
};

template <int N, int P = LinePts<N>::P>
__device__ __forceinline__ void load_tw(LineTw<N, P>& tw, const float2* __restrict__ tab_row, int j, int tab) {
  using T = LineTw<N, P>;
  // twiddled radix-P stages: sub-length NS = R0 P^s (R0 = P), or P^(s+1) (radix R0 last)
#pragma unroll
  for (int s = 0, NS = T::R0LAST ? P : T::R0; s < T::NPW; ++s, NS *= P) {
    const int jm = j % NS;
    const int step = N / (P * NS);
#pragma unroll
    for (int r = 1; r < P; ++r) tw.w[s][r - 1] = tab_row[jm * r * step];
  }
  if constexpr (T::R0LAST) {
    // last stage, sub-length N / R0: butterfly i = j + L q takes W_N^(i r)
    constexpr int L = N / P;
#pragma unroll
    for (int q = 0; q < T::Q; ++q)
#pragma unroll
      for (int r = 1; r < T::R0; ++r) tw.wl[q][r - 1] = tab_row[(j + L * q) * r];
  }
  tw.rs2 = rs2_at(tab);
}

// The two LDS exchange buffers of one line.  Consecutive exchanges of a
// workgroup alternate between them, so a stage can write its output while
// other waves still read that stage's input, and each exchange needs one
// barrier (after the writes) instead of two.
struct LineLds {
  float2* a;
  float2* b;
};

// Line FFT of N points held by L = N/P lanes, P points per lane.  On entry
// and on exit lane j holds element j + t*L in v[t] ("t-layout", natural
// order).  Stockham autosort: a first stage of radix R0 <= P without
// twiddles, then radix-P stages; every stage but the last exchanges through
// LDS (padded one slot in eight to spread the strided writes over the
// banks), exchange e in buffer a for even e, b for odd e.  All threads of the
// block call it together (it has block barriers).
//
// Why one barrier per exchange suffices: the writes of exchange e reuse the
// buffer of exchange e - 2, whose reads every wave finished before it wrote
// exchange e - 1 and so before the barrier that follows those writes; the
// writer of exchange e has passed that barrier.  Successive calls keep the
// alternation when the exchange count NST is even; for an odd count every
// call starts on buffer a after a barrier of its own.
// Exchange ordering: a workgroup barrier, or (WAVE: every line held by one
// wavefront) ordering within the wavefront, whose LDS accesses run in order.
template <bool WAVE>
__device__ __forceinline__ void line_sync() {
  if constexpr (WAVE) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  } else {
    __syncthreads();
  }
}

template <int N, bool INV, int P = LinePts<N>::P, bool WAVE = false>
__device__ __forceinline__ void fft_line(float2 (&v)[P], const LineLds& sh, int j, const LineTw<N, P>& tw) {
  constexpr int L = N / P;
  constexpr int R0 = LineTw<N, P>::R0;
  constexpr int NX = LineTw<N, P>::NST;  // exchanges: after every stage but the last
  if constexpr (NX % 2 == 1) line_sync<WAVE>();
  if constexpr (LineTw<N, P>::R0LAST) {
    // ---- radix R0 last: stage 0 radix P, sub-length 1, no twiddles; writes exchange 0 (buffer a)
    constexpr int NPW = LineTw<N, P>::NPW, Q = LineTw<N, P>::Q;
    dft_p<P, INV>(v, tw.rs2);
#pragma unroll
    for (int r = 0; r < P; ++r) sh.a[lds_pad(P * j + r)] = v[r];
    line_sync<WAVE>();
    // ---- twiddled radix-P stages, sub-length NS = P, P^2, ...; stage s reads exchange s, writes s + 1
#pragma unroll
    for (int s = 0, NS = P; s < NPW; ++s, NS *= P) {
      const float2* const rd = (s & 1) ? sh.b : sh.a;
#pragma unroll
      for (int t = 0; t < P; ++t) v[t] = rd[lds_pad(j + t * L)];
#pragma unroll
      for (int r = 1; r < P; ++r) v[r] = cmul<INV>(v[r], tw.w[s][r - 1]);
      dft_p<P, INV>(v, tw.rs2);
      float2* const wr = (s & 1) ? sh.a : sh.b;
      const int base = (j / NS) * NS * P + (j % NS);
#pragma unroll
      for (int r = 0; r < P; ++r) wr[lds_pad(base + r * NS)] = v[r];
      line_sync<WAVE>();
    }
    // ---- radix-R0 stage, sub-length N / R0: butterfly q of the lane is element j + L q and
    // its partners at + r N / R0, i.e. v[q + Q r]; outputs land in the same slots (natural order)
    {
      const float2* const rd = (NPW & 1) ? sh.b : sh.a;
#pragma unroll
      for (int t = 0; t < P; ++t) v[t] = rd[lds_pad(j + t * L)];
#pragma unroll
      for (int q = 0; q < Q; ++q) {
#pragma unroll
        for (int r = 1; r < R0; ++r) v[q + Q * r] = cmul<INV>(v[q + Q * r], tw.wl[q][r - 1]);
        if constexpr (R0 == 4) {
          float2 y0, y1, y2, y3;
          dft4<INV>(v[q], v[q + Q], v[q + 2 * Q], v[q + 3 * Q], y0, y1, y2, y3);
          v[q] = y0;
          v[q + Q] = y1;
          v[q + 2 * Q] = y2;
          v[q + 3 * Q] = y3;
        } else {
          dft2<INV>(v[q], v[q + Q]);
        }
      }
    }
    return;
  }
  // ---- stage 0: radix R0 = P, sub-length 1, trivial twiddles; writes exchange 0 (buffer a)
  float2* const w0 = sh.a;
  if constexpr (R0 == P) {
    dft_p<P, INV>(v, tw.rs2);
#pragma unroll
    for (int r = 0; r < P; ++r) w0[lds_pad(P * j + r)] = v[r];
  } else {
    constexpr int Q = P / R0;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      if constexpr (R0 == 4) {
        float2 y0, y1, y2, y3;
        dft4<INV>(v[q], v[q + Q], v[q + 2 * Q], v[q + 3 * Q], y0, y1, y2, y3);
        const int b = R0 * (j + q * L);
        w0[lds_pad(b)] = y0;
        w0[lds_pad(b + 1)] = y1;
        w0[lds_pad(b + 2)] = y2;
        w0[lds_pad(b + 3)] = y3;
      } else {
        float2 a = v[q], c = v[q + Q];
        dft2<INV>(a, c);
        w0[lds_pad(2 * (j + q * L))] = a;
        w0[lds_pad(2 * (j + q * L) + 1)] = c;
      }
    }
  }
  line_sync<WAVE>();
  // ---- radix-P stages with sub-length NS = R0, P R0, ...; stage s reads exchange s
#pragma unroll
  for (int s = 0, NS = R0; s < NX; ++s, NS *= P) {
    const float2* const rd = (s & 1) ? sh.b : sh.a;
#pragma unroll
    for (int t = 0; t < P; ++t) v[t] = rd[lds_pad(j + t * L)];
#pragma unroll
    for (int r = 1; r < P; ++r) v[r] = cmul<INV>(v[r], tw.w[s][r - 1]);
    dft_p<P, INV>(v, tw.rs2);
    if (s + 1 < NX) {
      float2* const wr = (s & 1) ? sh.a : sh.b;
      const int base = (j / NS) * NS * P + (j % NS);
#pragma unroll
      for (int r = 0; r < P; ++r) wr[lds_pad(base + r * NS)] = v[r];
      line_sync<WAVE>();
    }
  }
}

// ---------------------------------------------------------------------------
// slice transmission

// Returns T - 1 for T = exp(i a - b).  Taylor forms serve |a|, |b| <= 1/8
// (every workload of interest: k dx delta is ~1e-2); the library functions
// run only in waves where some lane is outside that range.
__device__ __forceinline__ float sin_small(float x) {
  // sin x = x (1 - x^2/6 (1 - x^2/20 (1 - x^2/42))), |x| <= 1/8
  const float x2 = x * x;
  return x * __builtin_fmaf(-x2 * (1.0f / 6.0f),
                            __builtin_fmaf(-x2 * (1.0f / 20.0f), __builtin_fmaf(-x2, 1.0f / 42.0f, 1.0f), 1.0f),
                            1.0f);
}

__device__ __forceinline__ float expm1_neg_small(float b) {
  // expm1(-b) = -b (1 - b/2 (1 - b/3 (1 - b/4 (1 - b/5 (1 - b/6 (1 - b/7)))))), |b| <= 1/8
  float p = __builtin_fmaf(-b, 1.0f / 7.0f, 1.0f);
  p = __builtin_fmaf(-b * (1.0f / 6.0f), p, 1.0f);
  p = __builtin_fmaf(-b * (1.0f / 5.0f), p, 1.0f);
  p = __builtin_fmaf(-b * (1.0f / 4.0f), p, 1.0f);
  p = __builtin_fmaf(-b * (1.0f / 3.0f), p, 1.0f);
  p = __builtin_fmaf(-b * 0.5f, p, 1.0f);
  return -b * p;
}

__device__ __forceinline__ float2 transmission_m1(float a, float b) {
  float sa = sin_small(a), sh = sin_small(0.5f * a), em1 = expm1_neg_small(b);
  const bool big = !(fabsf(a) <= 0.125f && fabsf(b) <= 0.125f);
  if (__builtin_expect(__ballot(big) != 0, 0)) {
    if (big) {
      sa = sinf(a);
      sh = sinf(0.5f * a);
      em1 = expm1f(-b);
    }
  }
  const float cm1 = -2.0f * sh * sh;  // cos a - 1
  // T - 1 = (1 + em1)(1 + cm1 + i sa) - 1
  return make_float2(__builtin_fmaf(em1, cm1, cm1 + em1), __builtin_fmaf(em1, sa, sa));
}

// psi * T  = psi + psi (T - 1)
__device__ __forceinline__ float2 apply_t(float2 p, float2 tm1) {
  return make_float2(__builtin_fmaf(p.x, tm1.x, __builtin_fmaf(-p.y, tm1.y, p.x)),
                     __builtin_fmaf(p.x, tm1.y, __builtin_fmaf(p.y, tm1.x, p.y)));
}

// g * conj(T) = g + g conj(T - 1)
__device__ __forceinline__ float2 apply_tconj(float2 g, float2 tm1) {
  return make_float2(__builtin_fmaf(g.x, tm1.x, __builtin_fmaf(g.y, tm1.y, g.x)),
                     __builtin_fmaf(-g.x, tm1.y, __builtin_fmaf(g.y, tm1.x, g.y)));
}

// Element offset of slice s's values in the delta / beta arrays.
__device__ __forceinline__ int64_t slice_offset(const Ctx& c, int s) {
  if (!c.slice_index) return (int64_t)s * c.m;
  int u = c.slice_index[s];
  u = u < 0 ? 0 : (u >= c.n_pool ? c.n_pool - 1 : u);
  return (int64_t)u * c.m;
}

__device__ __forceinline__ float phase_arg(float d, const Ctx& c) {
  return __builtin_fmaf(d, c.kdx_hi, d * c.kdx_lo);
}

// ---------------------------------------------------------------------------
// one line of one pass

// Pass kinds compiled on their own (the executed path only, a fraction of
// the generic kernel's code); KIND_GENERIC follows the descriptor at run time.
enum PassKind : int { KIND_GENERIC = 0, KIND_FWD_MID = 1, KIND_REV_MID = 2 };

__host__ __device__ inline int pass_kind(const PassDesc& pd) {
  if (pd.src_lay != LAY_T || pd.dst_lay != LAY_T || !pd.dst) return KIND_GENERIC;
  if (pd.pre == PRE_PROP && pd.post == POST_PROP && pd.mid == MID_T_FWD && !pd.conj) return KIND_FWD_MID;
  if (pd.pre == PRE_PROP && pd.post == POST_PROP && pd.mid == MID_T_ADJ && pd.conj) return KIND_REV_MID;
  return KIND_GENERIC;
}


// Element offsets within one [ny][nz] field fit in 32 bits (at most 2^20
// elements); slice offsets are added to the (uniform) base pointer instead.

// Offset of element (r, col) in the 2x2-tiled layout: the tile of rows 2a,
// 2a+1 and columns 2b, 2b+1 is 4 consecutive elements (row-major inside the
// tile), tiles row-major over the grid.  A row pass over rows 2a and 2a+1 and
// a column pass over columns 2b and 2b+1 both read whole tiles.
__device__ __forceinline__ uint32_t tile_addr(const Ctx& c, uint32_t r, uint32_t col) {
  return ((((r >> 1) * ((uint32_t)c.nz >> 1)) + (col >> 1)) << 2) + ((r & 1u) << 1) + (col & 1u);
}

// The same 2x2 tiles ordered column by column (tile (a, b) at b ny/2 + a):
// the tiles of a column pass over columns 2b and 2b+1 are contiguous.  Fields
// of one slice that only column passes read and write (the odd slices' packed
// transmissions, stored entrance fields and gradients) use it.
__device__ __forceinline__ uint32_t tile_addr_c(const Ctx& c, uint32_t r, uint32_t col) {
  return ((((col >> 1) * ((uint32_t)c.ny >> 1)) + (r >> 1)) << 2) + ((r & 1u) << 1) + (col & 1u);
}

// The elements j + t L (t = 0 .. P-1) of line `line` of a pass along AXIS in
// layout `lay` are at base + t * stride: in every layout a step of L (even)
// along the line moves by a fixed offset (row-major: L along a row, L nz
// along a column; tiled: 2 L along a row, L nz along a column; tiled in
// column order: L ny along a row, 2 L along a column).
struct LineAddr {
  uint32_t base, stride;
};

template <int N, int AXIS, int P = LinePts<N>::P>
__device__ __forceinline__ LineAddr line_at(const Ctx& c, int lay, int line, int j) {
  constexpr uint32_t L = (uint32_t)(N / P);
  const uint32_t r = AXIS == ROW ? (uint32_t)line : (uint32_t)j;
  const uint32_t col = AXIS == ROW ? (uint32_t)j : (uint32_t)line;
  if (lay == LAY_C) return LineAddr{tile_addr_c(c, r, col), AXIS == ROW ? L * (uint32_t)c.ny : 2 * L};
  const uint32_t base = lay == LAY_T ? tile_addr(c, r, col) : r * (uint32_t)c.nz + col;
  const uint32_t stride = AXIS == ROW ? (lay == LAY_T ? 2 * L : L) : L * (uint32_t)c.nz;
  return LineAddr{base, stride};
}

// Layout of the slice pack: a single stack's pack holds the odd slices (column
// passes) in column tile order, a batch pool (slices of either parity) in row
// tile order.
template <int AXIS>
__device__ __forceinline__ int pack_lay(const Ctx& c) {
  return (AXIS == COL && !c.slice_index) ? (int)LAY_C : (int)LAY_T;
}

// Float2 slots of one line's exchange buffer in LDS: a radix-8 pad every
// eight slots, and an odd length so that neighbouring lines start on
// different banks.
template <int N>
constexpr int line_lds() { return N + N / 8 + 1; }

// Where a pass takes the transmission T - 1 of its slice from: the slice pack
// when the caller built one, else the caller's delta and beta stacks (decided
// at run time), or fixed to the pack at compile time for kernels that serve
// only passes with a pack (the paraxial and batched middle passes), which then
// carry no code for evaluating it.
enum TSource : int { TS_RUNTIME = 0, TS_PACK = 1 };

template <int TS = TS_RUNTIME>
__device__ __forceinline__ bool uses_pack(const Ctx& c) {
  if constexpr (TS == TS_PACK) return true;
  return c.dbT != nullptr;
}

// Everything a line pass reads, gathered in registers.  Loads are issued
// together at the top of the pass (one memory latency instead of one per
// FFT stage); inputs that do not depend on the previous pass can be fetched
// before the grid barrier that separates two passes.
template <int N, int P = LinePts<N>::P>
struct LineIn {
  float2 v[P];            // field
  float dl[P], bt[P];     // delta, beta of the slice
  float2 ps[P];           // psi_s (adjoint)
  float gi[P];            // far-field seed (shifted read)
  float2 hh[P];           // propagator factor (1-D paraxial; 2-D exact: hi part)
  float2 hl[P];           // 2-D exact propagator: lo part
  LineTw<N, P> tw;
};

__device__ __forceinline__ bool uses_h1d(const PassDesc& pd) {
  return pd.pre == PRE_PROP || pd.post == POST_PROP;
}

template <int N, int AXIS, int KIND = KIND_GENERIC, int TS = TS_RUNTIME, int P = LinePts<N>::P>
__device__ __forceinline__ void load_static(const Ctx& c, const PassDesc& pd_, int line, int j, LineIn<N, P>& in) {
  PassDesc pd = pd_;
  if constexpr (KIND != KIND_GENERIC) {
    pd.pre = PRE_PROP;
    pd.post = POST_PROP;
    pd.mid = KIND == KIND_FWD_MID ? MID_T_FWD : MID_T_ADJ;
  }
  constexpr int L = N / P;
  const uint32_t row = (uint32_t)pd.tab * (uint32_t)N;
  load_tw<N, P>(in.tw, (AXIS == ROW ? c.twz : c.twy) + row, j, pd.tab);
  if (uses_h1d(pd)) {
    const float2* hh = (AXIS == ROW ? c.hz : c.hy) + row;
#pragma unroll
    for (int t = 0; t < P; ++t) in.hh[t] = hh[j + t * L];
  } else if (pd.post == POST_PROP2D) {
#pragma unroll
    for (int t = 0; t < P; ++t) {
      const uint32_t e = (uint32_t)(j + t * L) * (uint32_t)c.nz + (uint32_t)line;
      in.hh[t] = c.H_hi[e];
      in.hl[t] = c.H_lo[e];
    }
  }
  if (pd.mid == MID_T_FWD || pd.mid == MID_T_ADJ) {
    if (uses_pack<TS>(c)) {
      // precomputed T - 1 (real part in dl, imaginary part in bt), tiled
      const float2* q = c.dbT + slice_offset(c, pd.slice);
      const LineAddr a = line_at<N, AXIS, P>(c, pack_lay<AXIS>(c), line, j);
#pragma unroll
      for (int t = 0; t < P; ++t) {
        const float2 tm = q[a.base + (uint32_t)t * a.stride];
        in.dl[t] = tm.x;
        in.bt[t] = tm.y;
      }
    } else {
      const int64_t so = slice_offset(c, pd.slice);
      const float* dp = c.delta + so;
      const float* bp = c.beta + so;
      const LineAddr a = line_at<N, AXIS, P>(c, LAY_R, line, j);
#pragma unroll
      for (int t = 0; t < P; ++t) {
        in.dl[t] = dp[a.base + (uint32_t)t * a.stride];
        in.bt[t] = bp[a.base + (uint32_t)t * a.stride];
      }
    }
  }
  if (pd.mid == MID_T_ADJ) {
    const LineAddr a = line_at<N, AXIS, P>(c, pd.load_lay, line, j);
#pragma unroll
    for (int t = 0; t < P; ++t) in.ps[t] = pd.psi_load[a.base + (uint32_t)t * a.stride];
  }
  if (pd.mid == MID_FF_SEED) {
#pragma unroll
    for (int t = 0; t < P; ++t) {
      const int i = j + t * L;
      const int r = AXIS == ROW ? line : i, col = AXIS == ROW ? i : line;
      const int rs = (r + (c.ny >> 1)) & (c.ny - 1), cs = (col + (c.nz >> 1)) & (c.nz - 1);
      in.gi[t] = c.grad_intensity[(uint32_t)rs * (uint32_t)c.nz + (uint32_t)cs];
    }
  }
}

// Field element access.  COH selects device-coherent accesses (agent-scope
// atomics: written through to and read from the coherence point, past the
// per-XCD L2 caches), used when another XCD reads the data within the same
// kernel; plain accesses otherwise.
template <bool COH>
__device__ __forceinline__ float2 field_ld(const float2* p) {
  if constexpr (COH) {
    const unsigned long long u = __hip_atomic_load(reinterpret_cast<const unsigned long long*>(p),
                                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return __builtin_bit_cast(float2, u);
  } else {
    return *p;
  }
}

template <bool COH>
__device__ __forceinline__ void field_st(float2* p, float2 v) {
  if constexpr (COH) {
    __hip_atomic_store(reinterpret_cast<unsigned long long*>(p), __builtin_bit_cast(unsigned long long, v),
                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  } else {
    *p = v;
  }
}

template <int N, int AXIS, bool COH = false, int KIND = KIND_GENERIC, int P = LinePts<N>::P>
__device__ __forceinline__ void load_field(const Ctx& c, const PassDesc& pd, int line, int j, LineIn<N, P>& in) {
  const int lay = KIND != KIND_GENERIC ? (int)LAY_T : pd.src_lay;  // the specialised kinds work on tiled fields
  const LineAddr a = line_at<N, AXIS, P>(c, lay, line, j);
#pragma unroll
  for (int t = 0; t < P; ++t) in.v[t] = field_ld<COH>(pd.src + a.base + (uint32_t)t * a.stride);
}

// FFT, propagator, inverse FFT along the line: the one-axis paraxial factor
// (single-term), or with TWO_TERM the exact 2-D factor (hi + lo).
template <int N, bool TWO_TERM, int P = LinePts<N>::P, bool WAVE = false>
__device__ __forceinline__ void prop_line(float2 (&v)[P], const LineLds& sh, int j, const LineIn<N, P>& in, bool conj) {
  fft_line<N, false, P, WAVE>(v, sh, j, in.tw);
#pragma unroll
  for (int t = 0; t < P; ++t)
    v[t] = TWO_TERM ? cmul_comp_dyn(v[t], in.hh[t], in.hl[t], conj) : cmul_dyn(v[t], in.hh[t], conj);
  fft_line<N, true, P, WAVE>(v, sh, j, in.tw);
}

template <int N, int AXIS, bool COH = false, int KIND = KIND_GENERIC, int TS = TS_RUNTIME, int P = LinePts<N>::P,
          bool WAVE = false>
__device__ __forceinline__ void compute_line(const Ctx& c, const PassDesc& pd_, int line, int j, const LineLds& sh,
                                             LineIn<N, P>& in) {
  constexpr int L = N / P;
  const float inv_n = 1.0f / (float)N;
  float2 (&v)[P] = in.v;
  PassDesc pd = pd_;
  if constexpr (KIND != KIND_GENERIC) {
    pd.pre = PRE_PROP;
    pd.post = POST_PROP;
    pd.mid = KIND == KIND_FWD_MID ? MID_T_FWD : MID_T_ADJ;
    pd.conj = KIND == KIND_REV_MID;
    pd.src_lay = LAY_T;
    pd.dst_lay = LAY_T;
  }

  switch (pd.pre) {
    case PRE_PROP: prop_line<N, false, P, WAVE>(v, sh, j, in, pd.conj != 0); break;
    case PRE_FFT: fft_line<N, false, P>(v, sh, j, in.tw); break;
    case PRE_IFFT_N:
      fft_line<N, true, P>(v, sh, j, in.tw);
#pragma unroll
      for (int t = 0; t < P; ++t) v[t] = make_float2(v[t].x * inv_n, v[t].y * inv_n);
      break;
    case PRE_IFFT_U: fft_line<N, true, P>(v, sh, j, in.tw); break;
    default: break;
  }

  if (pd.psi_store) {
    const LineAddr a = line_at<N, AXIS, P>(c, pd.store_lay, line, j);
#pragma unroll
    for (int t = 0; t < P; ++t) pd.psi_store[a.base + (uint32_t)t * a.stride] = v[t];
  }

  float2 tm1[P];  // T - 1 of the slice at this line's points
  if (pd.mid == MID_T_FWD || pd.mid == MID_T_ADJ) {
    if (uses_pack<TS>(c)) {
#pragma unroll
      for (int t = 0; t < P; ++t) tm1[t] = make_float2(in.dl[t], in.bt[t]);
    } else {
#pragma unroll
      for (int t = 0; t < P; ++t) tm1[t] = transmission_m1(phase_arg(in.dl[t], c), phase_arg(in.bt[t], c));
    }
  }
  if (pd.mid == MID_T_FWD) {
#pragma unroll
    for (int t = 0; t < P; ++t) v[t] = apply_t(v[t], tm1[t]);
  } else if (pd.mid == MID_T_ADJ) {
    const int64_t so = (int64_t)pd.slice * c.m;
    float* const gdp = c.gdelta ? c.gdelta + so : nullptr;
    float* const gbp = c.gbeta ? c.gbeta + so : nullptr;
    float2* const gtp = c.gT ? c.gT + (int64_t)(pd.slice >> 1) * c.m : nullptr;
    const float kdx = c.kdx_hi;
    const LineAddr ar = line_at<N, AXIS, P>(c, LAY_R, line, j);
    const LineAddr at = line_at<N, AXIS, P>(c, LAY_C, line, j);  // gT: odd slices, column passes
#pragma unroll
    for (int t = 0; t < P; ++t) {
      const uint32_t e = ar.base + (uint32_t)t * ar.stride;
      const float2 pt = apply_t(in.ps[t], tm1[t]);  // psi'_s = T_s psi_s
      const float2 g = v[t];                     // cotangent of psi'_s
      // conj(g) * psi' = (gx px + gy py) + i (gx py - gy px)
      const float cre = __builtin_fmaf(g.x, pt.x, g.y * pt.y);
      const float cim = __builtin_fmaf(g.x, pt.y, -(g.y * pt.x));
      if (c.gT && (pd.slice & 1)) {
        gtp[at.base + (uint32_t)t * at.stride] = make_float2(-kdx * cim, -kdx * cre);
      } else {
        if (gdp) gdp[e] = -kdx * cim;
        if (gbp) gbp[e] = -kdx * cre;
      }
      v[t] = apply_tconj(g, tm1[t]);
    }
  } else if (pd.mid == MID_FF_OUT) {
#pragma unroll
    for (int t = 0; t < P; ++t) {
      const int i = j + t * L;
      const int r = AXIS == ROW ? line : i, col = AXIS == ROW ? i : line;
      const int rs = (r + (c.ny >> 1)) & (c.ny - 1), cs = (col + (c.nz >> 1)) & (c.nz - 1);
      const float p = __builtin_fmaf(v[t].x, v[t].x, v[t].y * v[t].y);
      c.intensity[(uint32_t)rs * (uint32_t)c.nz + (uint32_t)cs] = p * c.inv_m;
    }
  } else if (pd.mid == MID_FF_SEED) {
#pragma unroll
    for (int t = 0; t < P; ++t) {
      const float s = 2.0f * c.inv_m * in.gi[t];
      v[t] = make_float2(v[t].x * s, v[t].y * s);
    }
  }

  switch (pd.post) {
    case POST_PROP: prop_line<N, false, P, WAVE>(v, sh, j, in, pd.conj != 0); break;
    case POST_FFT: fft_line<N, false, P>(v, sh, j, in.tw); break;
    case POST_PROP2D: prop_line<N, true, P>(v, sh, j, in, pd.conj != 0); break;  // H[ky][kz] / ny in hh, hl
    default: break;
  }

  if (pd.dst) {
    const LineAddr a = line_at<N, AXIS, P>(c, pd.dst_lay, line, j);
#pragma unroll
    for (int t = 0; t < P; ++t) field_st<COH>(pd.dst + a.base + (uint32_t)t * a.stride, v[t]);
  }
}

// WAVE: each line is held by one wavefront (the caller maps lanes so), and the
// stage exchanges are ordered inside it instead of by workgroup barriers.
template <int N, int AXIS, bool COH = false, int KIND = KIND_GENERIC, int TS = TS_RUNTIME, int P = LinePts<N>::P,
          bool WAVE = false>
__device__ __forceinline__ void run_line(const Ctx& c, const PassDesc& pd, int line, int j, const LineLds& sh) {
  LineIn<N, P> in;
  load_field<N, AXIS, COH, KIND, P>(c, pd, line, j, in);
  load_static<N, AXIS, KIND, TS, P>(c, pd, line, j, in);
  compute_line<N, AXIS, COH, KIND, TS, P, WAVE>(c, pd, line, j, sh, in);
}

// Either axis, chosen per pass at run time (square grids: both line lengths are N).
template <int N, bool COH = false, int P = LinePts<N>::P>
__device__ __forceinline__ void run_line_any(const Ctx& c, const PassDesc& pd, int line, int j, const LineLds& sh) {
  if (pd.axis == ROW) run_line<N, ROW, COH, KIND_GENERIC, TS_RUNTIME, P>(c, pd, line, j, sh);
  else run_line<N, COL, COH, KIND_GENERIC, TS_RUNTIME, P>(c, pd, line, j, sh);
}

// Workgroups are dealt to the XCDs round robin; give each XCD a contiguous
// range of lines so that column passes of one XCD share cache lines in its L2.
__device__ __forceinline__ int xcd_group(int b, int n) {
  return (n % 8 == 0) ? (b % 8) * (n / 8) + b / 8 : b;
}

}  // namespace msl

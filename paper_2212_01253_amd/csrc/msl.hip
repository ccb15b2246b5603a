// libmsl: host entry points of the C ABI declared in include/msl.h, table
// builders and kernel launches.  Multislice forward model, far field,
// amplitude loss and adjoint of arXiv 2212.01253 (Eq. 1, Eq. 4; Sec. 1, 3, 4).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

#include "msl.h"
#include "msl_common.hpp"
#include "msl_device.hpp"
#include "msl_passes.hpp"
#include "msl_persistent.hpp"

using namespace msl_host;
using msl::Ctx;
using msl::PassDesc;
using msl::PhaseSpec;

namespace {

int g_schedule = MSL_SCHED_AUTO;

// Launch shape of the line-pass kernels (msl_set_tuning): lines of length 2^e
// per workgroup, 0 = the default (one wavefront's worth of lanes).
int g_lines_per_group[MSL_TUNE_SLOTS] = {};
int g_points_per_lane[MSL_TUNE_SLOTS] = {};  // 0: default (default_points_per_lane)
int g_batch_streams = 0;  // 0: default (every extra stream)

// Polls of the persistent schedule's bounded barrier wait (msl_set_barrier_spin_limit).
unsigned g_spin_limit = msl::kDefaultSpinLimit;

// LDS of a line-pass workgroup of G n-point lines: two exchange buffers per
// line (msl::LineLds), the first buffers of all G lines, then the second ones.
constexpr int kMaxLdsBytes = 64 * 1024;
int line_pass_lds_bytes(int n, int G) { return 2 * G * (n + n / 8 + 1) * (int)sizeof(float2); }  // msl::line_lds<n>()

template <int N>
__device__ __forceinline__ msl::LineLds line_buffers(float2* lds, int g, int G) {
  return msl::LineLds{lds + g * msl::line_lds<N>(), lds + (G + g) * msl::line_lds<N>()};
}

constexpr size_t kAlign = 256;
size_t up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

// Workspace layout (byte offsets, each region 256-byte aligned).
struct Layout {
  size_t twz, twy, hz, hy;  // line tables, [DITHER][n] float2
  size_t H_hi, H_lo;
  size_t bar, partials, tmp, dbT, W, G, seg, gT;
  size_t total;
};

constexpr int kPartials = 1024;

Layout layout(const msl_geometry& g, int k) {
  Layout L{};
  const size_t m = (size_t)g.ny * g.nz;
  size_t o = 0;
  auto take = [&](size_t bytes) { size_t r = o; o += up(bytes); return r; };
  L.bar = take(8192);  // first, at offset 0: msl_workspace_status finds its status word without the geometry
  L.twz = take((size_t)msl::DITHER * g.nz * 8);
  L.twy = take((size_t)msl::DITHER * g.ny * 8);
  L.hz = take((size_t)msl::DITHER * g.nz * 8);
  L.hy = take((size_t)msl::DITHER * g.ny * 8);
  const bool exact = g.propagator == MSL_PROP_EXACT;
  L.H_hi = take(exact ? m * 8 : 0);
  L.H_lo = take(exact ? m * 8 : 0);
  L.partials = take(kPartials * sizeof(double));
  L.tmp = take(m * 8);  // tiled working field of the forward, the far field and its adjoint
  // paraxial: every slice's transmission T - 1, tiled (the slice pack)
  const size_t odd = exact ? 0 : (size_t)(g.n_slices / 2);
  L.dbT = take((exact ? 0 : (size_t)g.n_slices) * m * 8);
  if (k >= 1) {
    L.W = take(m * 8);  // tiled working field of the segment recompute
    L.G = take(m * 8);  // tiled working field of the reverse sweep (the cotangent)
    L.seg = take((size_t)(k > 1 ? k - 1 : 0) * m * 8 * 2);  // two tiled segment buffers
    L.gT = take(odd * m * 8);  // odd slices' gradients, same layout as dbT
  }
  L.total = o;
  return L;
}

msl_status check_ws(const msl_geometry& g, int k, const void* ws, size_t ws_bytes) {
  const size_t need = layout(g, k).total;
  if (!ws) return fail(MSL_ERR_WORKSPACE, "workspace is NULL");
  if (!aligned(ws, kAlign)) return fail(MSL_ERR_WORKSPACE, "workspace is not 256-byte aligned");
  if (ws_bytes < need)
    return fail(MSL_ERR_WORKSPACE, "workspace too small: need " + std::to_string(need) + " bytes, got " +
                                       std::to_string(ws_bytes));
  return MSL_OK;
}


// ---------------------------------------------------------------------------
// table builders (FP64 arithmetic; line tables as cycles of single float32
// values, the exact propagator split into float32 hi + lo)

// Writes out[i * stride], i < DITHER: the cycle of float32 values that stands
// for x, each one of the two float32 neighbours of x, picked by a first-order
// sigma-delta modulator (the one that keeps the running sum of the errors
// smaller; ties take the lower), so that every partial sum of the errors over
// the cycle stays within one ulp.  A representable x is used as is.
__device__ inline void cycle_store(double x, float* out, int64_t stride) {
  const float f = (float)x;
  if ((double)f == x) {
    for (int i = 0; i < msl::DITHER; ++i) out[i * stride] = f;
    return;
  }
  const float lo = (double)f < x ? f : nextafterf(f, -INFINITY);
  const float hi = nextafterf(lo, INFINITY);
  double e = 0.0;
  for (int i = 0; i < msl::DITHER; ++i) {
    const double el = e + ((double)lo - x), eh = e + ((double)hi - x);
    const bool up = fabs(eh) < fabs(el);
    out[i * stride] = up ? hi : lo;
    e = up ? eh : el;
  }
}

// Element i of an n-element line table [DITHER][n] float2.
__device__ inline void cycle_store2(double re, double im, float2* tab, int n, int i) {
  float* const b = reinterpret_cast<float*>(tab) + 2 * (int64_t)i;
  cycle_store(re, b, 2 * (int64_t)n);
  cycle_store(im, b + 1, 2 * (int64_t)n);
}

__device__ inline void split_store(double re, double im, float2* hi, float2* lo, int64_t i) {
  const float hr = (float)re, hm = (float)im;
  hi[i] = make_float2(hr, hm);
  lo[i] = make_float2((float)(re - (double)hr), (float)(im - (double)hm));
}

// Angular spatial frequency of DFT bin m of an n-point grid with pitch d:
// 2 pi f / (n d) with f = m for m < n/2 and m - n otherwise.
__device__ inline double kfreq(int m, int n, double d) {
  const int f = m < n / 2 ? m : m - n;
  return 2.0 * M_PI * (double)f / ((double)n * d);
}

// Twiddles W_n^e = exp(-2 pi i e / n), e < n, as a [DITHER][n] cycle table.
__global__ void k_twiddles(int n, float2* tab) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  double s, c;
  sincospi(-2.0 * (double)e / (double)n, &s, &c);
  cycle_store2(c, s, tab, n, e);
}

// Paraxial one-axis propagator factor exp(+i dx kq^2 / 2k) / n, as a
// [DITHER][n] cycle table.
__global__ void k_hpar(int n, double d, double dx, double k, float2* tab) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= n) return;
  const double q = kfreq(m, n, d);
  const double ph = dx * q * q / (2.0 * k);
  double s, c;
  sincos(ph, &s, &c);
  cycle_store2(c / n, s / n, tab, n, m);
}

// Exact angular-spectrum propagator H[my][mz] / ny.
__global__ void k_hexact(int ny, int nz, double dy, double dz, double dx, double k, float2* hi, float2* lo) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)ny * nz) return;
  const int my = (int)(i / nz), mz = (int)(i % nz);
  const double ky = kfreq(my, ny, dy), kz = kfreq(mz, nz, dz);
  const double kp2 = ky * ky + kz * kz;
  double re, im;
  if (kp2 < k * k) {
    const double ph = dx * kp2 / (k + sqrt(k * k - kp2));
    sincos(ph, &im, &re);
  } else {
    const double amp = exp(-dx * sqrt(kp2 - k * k));
    double s, c;
    sincos(fmod(k * dx, 2.0 * M_PI), &s, &c);
    re = amp * c;
    im = amp * s;
  }
  split_store(re / ny, im / ny, hi, lo, i);
}

// Tilted plane wave exp(+i k sin(alpha) j dy).
__global__ void k_probe(int ny, int nz, double q, float2* out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)ny * nz) return;
  const int j = (int)(i / nz);
  double s, c;
  sincos(fmod(q * (double)j, 2.0 * M_PI), &s, &c);
  out[i] = make_float2((float)c, (float)s);
}

// Tile (a, b) (rows 2a, 2a+1, columns 2b, 2b+1) handled at work index t of a
// tile kernel, and that tile's index in the output layout.  Row tile order:
// tiles row by row.  Column tile order: each 64-wide wavefront takes an 8 x 8
// block of tiles, a fastest, blocks down the columns, so its row-major
// accesses cover 64-byte runs of 8 rows and its tile accesses 256-byte runs of
// 8 tiles.  Needs ny / 2 and nz / 2 multiples of 8 (grids of 16 and more).
struct TileAt {
  int a, b, out;
};
__device__ __forceinline__ TileAt tile_at(int t, int ny, int nz, bool col_order) {
  if (!col_order) {
    const int tz = nz >> 1;
    return TileAt{t / tz, t % tz, t};
  }
  const int lane = t & 63, blk = t >> 6, nba = ny >> 4;
  const int a = (blk % nba) * 8 + (lane & 7), b = (blk / nba) * 8 + (lane >> 3);
  return TileAt{a, b, b * (ny >> 1) + a};
}

// Slices' transmission minus one, T - 1 = exp(i k dx (delta + i beta)) - 1,
// into 2x2 tiles: slice first + stride * s2 -> out[s2], s2 in [s2b, s2e), in
// column tile order for odd slices when col_odd (a stack's pack: those slices
// are transmitted in column passes), else in row tile order; one thread per
// tile (two 8-byte reads of each stack when VEC, i.e. both stacks 8-byte
// aligned, else four 4-byte reads; two 16-byte writes).  Every slice of a
// stack (first 0, stride 1, col_odd) or of a batch pool (col_odd 0).  Line
// passes without a pack evaluate T - 1 with the same function.
template <bool VEC>
__global__ void __launch_bounds__(256) k_pack_tiled(const float* d, const float* b, float2* out, int ny, int nz,
                                                    int s2b, int s2e, int first, int stride, int col_odd,
                                                    msl::Ctx c) {
  const int64_t m = (int64_t)ny * nz;
  const int tiles = (int)(m >> 2);
  for (int s2 = s2b + blockIdx.y; s2 < s2e; s2 += gridDim.y) {
    const int sl = first + stride * s2;
    const bool col_order = col_odd && (sl & 1);
    const float* ds = d + (int64_t)sl * m;
    const float* bs = b + (int64_t)sl * m;
    float4* o = reinterpret_cast<float4*>(out + (int64_t)s2 * m);
    for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < tiles; t += gridDim.x * blockDim.x) {
      const TileAt ta = tile_at(t, ny, nz, col_order);
      const int64_t e = (int64_t)(2 * ta.a) * nz + 2 * ta.b;
      float2 d0, d1, b0, b1;  // (row 2a, row 2a + 1) x (column 2b, 2b + 1)
      if constexpr (VEC) {
        d0 = *reinterpret_cast<const float2*>(ds + e);
        d1 = *reinterpret_cast<const float2*>(ds + e + nz);
        b0 = *reinterpret_cast<const float2*>(bs + e);
        b1 = *reinterpret_cast<const float2*>(bs + e + nz);
      } else {
        d0 = make_float2(ds[e], ds[e + 1]);
        d1 = make_float2(ds[e + nz], ds[e + nz + 1]);
        b0 = make_float2(bs[e], bs[e + 1]);
        b1 = make_float2(bs[e + nz], bs[e + nz + 1]);
      }
      const float2 t0 = msl::transmission_m1(msl::phase_arg(d0.x, c), msl::phase_arg(b0.x, c));
      const float2 t1 = msl::transmission_m1(msl::phase_arg(d0.y, c), msl::phase_arg(b0.y, c));
      const float2 t2 = msl::transmission_m1(msl::phase_arg(d1.x, c), msl::phase_arg(b1.x, c));
      const float2 t3 = msl::transmission_m1(msl::phase_arg(d1.y, c), msl::phase_arg(b1.y, c));
      o[2 * (int64_t)ta.out] = make_float4(t0.x, t0.y, t1.x, t1.y);
      o[2 * (int64_t)ta.out + 1] = make_float4(t2.x, t2.y, t3.x, t3.y);
    }
  }
}

// Packs slices first + stride * s2, s2 in [s2b, s2e), of (d, b) into out (k_pack_tiled).
hipError_t launch_pack(const float* d, const float* b, float2* out, int ny, int nz, int s2b, int s2e, int first,
                       int stride, int col_odd, const msl::Ctx& c, hipStream_t st);

// gT[s2] (float2 (dL/d delta, dL/d beta) in column tile order) -> gdelta,
// gbeta [s][y][z] row-major for odd slices s = 2 s2 + 1, s2 in [s2b, s2e);
// one thread per tile (two 16-byte reads; 8-byte writes when VEC, i.e. both
// outputs 8-byte aligned, else 4-byte writes).
template <bool VEC>
__global__ void __launch_bounds__(256) k_unpack_tiled(const float2* gT, float* gd, float* gb, int ny, int nz,
                                                      int s2b, int s2e) {
  const int64_t m = (int64_t)ny * nz;
  const int tiles = (int)(m >> 2);
  for (int s2 = s2b + blockIdx.y; s2 < s2e; s2 += gridDim.y) {
    const float4* q = reinterpret_cast<const float4*>(gT + (int64_t)s2 * m);
    const int64_t so = (int64_t)(2 * s2 + 1) * m;
    for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < tiles; t += gridDim.x * blockDim.x) {
      const TileAt ta = tile_at(t, ny, nz, true);
      const int64_t e = so + (int64_t)(2 * ta.a) * nz + 2 * ta.b;
      const float4 u = q[2 * (int64_t)ta.out], w = q[2 * (int64_t)ta.out + 1];  // (d, b) at (0,0), (0,1) | (1,0), (1,1)
      if constexpr (VEC) {
        if (gd) {
          *reinterpret_cast<float2*>(gd + e) = make_float2(u.x, u.z);
          *reinterpret_cast<float2*>(gd + e + nz) = make_float2(w.x, w.z);
        }
        if (gb) {
          *reinterpret_cast<float2*>(gb + e) = make_float2(u.y, u.w);
          *reinterpret_cast<float2*>(gb + e + nz) = make_float2(w.y, w.w);
        }
      } else {
        if (gd) {
          gd[e] = u.x;
          gd[e + 1] = u.z;
          gd[e + nz] = w.x;
          gd[e + nz + 1] = w.z;
        }
        if (gb) {
          gb[e] = u.y;
          gb[e + 1] = u.w;
          gb[e + nz] = w.y;
          gb[e + nz + 1] = w.w;
        }
      }
    }
  }
}

// Launch shape of the tile kernels over n slices of an ny x nz grid.
dim3 tile_grid(int ny, int nz, int n) {
  const int64_t tiles = (int64_t)ny * nz / 4;
  const unsigned gx = (unsigned)std::min<int64_t>((tiles + 255) / 256, 4096);
  return dim3(gx, (unsigned)std::min(n, 8192));
}

hipError_t launch_pack(const float* d, const float* b, float2* out, int ny, int nz, int s2b, int s2e, int first,
                       int stride, int col_odd, const msl::Ctx& c, hipStream_t st) {
  const dim3 grid = tile_grid(ny, nz, s2e - s2b);
  if (aligned(d, 8) && aligned(b, 8))
    hipLaunchKernelGGL(k_pack_tiled<true>, grid, dim3(256), 0, st, d, b, out, ny, nz, s2b, s2e, first, stride,
                       col_odd, c);
  else
    hipLaunchKernelGGL(k_pack_tiled<false>, grid, dim3(256), 0, st, d, b, out, ny, nz, s2b, s2e, first, stride,
                       col_odd, c);
  return hipGetLastError();
}

// Amplitude loss partial sums (FP64) and dL/dI.
__global__ void __launch_bounds__(256) k_amp_loss(const float* I, const float* mamp, float* gI,
                                                  double* partials, int64_t n) {
  __shared__ double red[256];
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const double a = sqrt((double)I[i]);
    const double r = a - (double)mamp[i];
    acc += r * r;
    if (gI) gI[i] = a > 0.0 ? (float)(1.0 - (double)mamp[i] / a) : 0.0f;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) partials[blockIdx.x] = red[0];
}

__global__ void __launch_bounds__(256) k_sum_partials(const double* partials, int n, double* out) {
  __shared__ double red[256];
  double acc = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) acc += partials[i];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = red[0];
}

// ---------------------------------------------------------------------------
// per-pass launches

// Thread t of a workgroup of G lines works on line t mod G at lane t / G:
// neighbouring threads take neighbouring lines, so each load and store of a
// wavefront covers whole 2x2 tiles of the tiled working fields.
// The specialised middle passes take the transmission from the slice pack,
// which launch_pass_tp makes sure exists.
// WAVE_MAP: one line per wavefront also for 512-point lines (the host picks it
// per pass: wave_mapped).
template <int N, int P, int AXIS, int KIND, bool WAVE_MAP = false>
__global__ void __launch_bounds__(256) k_pass(Ctx c, PassDesc pd) {
  extern __shared__ float2 lds[];  // line_pass_lds_bytes(N, G)
  constexpr int L = N / P;
  static_assert(!WAVE_MAP || (L == 64 && KIND != msl::KIND_GENERIC), "one 64-lane line per wavefront");
  constexpr int TS = KIND == msl::KIND_GENERIC ? msl::TS_RUNTIME : msl::TS_PACK;
  const int G = blockDim.x / L;
  const int group = msl::xcd_group(blockIdx.x, gridDim.x);
  if constexpr (WAVE_MAP || (L == 64 && N < 512 && KIND != msl::KIND_GENERIC)) {
    // lines of one wavefront (256 points at 4 per lane): each wavefront takes a
    // whole line and orders its stage exchanges itself (measured faster on the
    // 256-point passes; at 512 points the interleaved mapping below is faster
    // except in the forward sweep's row passes)
    const int g = threadIdx.x / L, j = threadIdx.x % L;
    msl::run_line<N, AXIS, false, KIND, TS, P, true>(c, pd, group * G + g, j, line_buffers<N>(lds, g, G));
  } else {
    const int g = threadIdx.x % G, j = threadIdx.x / G;
    msl::run_line<N, AXIS, false, KIND, TS, P>(c, pd, group * G + g, j, line_buffers<N>(lds, g, G));
  }
}

// Points per lane of the per-pass and batch line kernels for n-point lines:
// the msl_set_tuning choice, else 8 from 512 points up and 4 below (the
// persistent schedule keeps that default).
int default_points_per_lane(int n) { return n >= 512 ? 8 : 4; }
static_assert(msl::LinePts<256>::P == 4 && msl::LinePts<512>::P == 8 && msl::LinePts<1024>::P == 8,
              "the persistent schedule's lines split as default_points_per_lane says");
int points_per_lane(int n) {
  const int p = g_points_per_lane[__builtin_ctz((unsigned)n)];
  return p > 0 ? p : default_points_per_lane(n);
}

// Lines per workgroup of n-point lines at p points per lane: at most 256
// threads (the kernels' launch bound) and at most kMaxLdsBytes of exchange
// buffers.
int max_lines_per_group(int n, int p) {
  const int L = n / p;
  int G = 1;
  while (2 * G * L <= 256 && line_pass_lds_bytes(n, 2 * G) <= kMaxLdsBytes) G *= 2;
  return G;
}

// Default: lines shorter than a wavefront fill one 64-lane wavefront; longer
// lines go two to a workgroup (the two lines of a row or column of tiles)
// when the launch has at least two lines per compute unit, else one, so that
// a launch of few lines still spreads over every compute unit (a 256-line
// pass: 256 one-line workgroups, measured faster than 128 two-line ones; at
// 512 lines two per workgroup are faster).  launch_lines: the lines of every
// instance the launch covers.
constexpr int kComputeUnits = 256;
int lines_per_group(int n, int nlines, int64_t launch_lines) {
  const int p = points_per_lane(n);
  const int L = n / p;
  int G = g_lines_per_group[__builtin_ctz((unsigned)n)];
  if (G <= 0) G = L >= 64 ? (launch_lines >= 2 * kComputeUnits ? 2 : 1) : (L >= 32 ? 2 : 64 / L);
  G = std::min(G, max_lines_per_group(n, p));
  return std::min(G, nlines);
}

// Middle passes over 512-point lines at 8 points per lane that take one line
// per wavefront (no workgroup barriers in their exchanges) instead of two lines
// interleaved over a workgroup (whole 2x2 tiles per load): the forward sweep's
// row passes that store no field for the reverse sweep.  Measured on the
// 512x512x2048 gradient step against the interleaved mapping everywhere: these
// alone 32.20-32.27 ms against 32.46-32.51; with the column passes too 32.34-32.41
// (a column line reads half of every 2x2 tile it touches, so its loads take
// twice the requests); with the recompute's and the reverse sweep's row passes
// too, which run side by side, 32.43-32.58.
template <int N, int P, int AXIS>
constexpr bool wave_mappable() { return N / P == 64 && N >= 512 && AXIS == msl::ROW; }
bool wave_mapped(int kind, const PassDesc& pd) { return kind == msl::KIND_FWD_MID && !pd.psi_store; }

template <int N, int P, int AXIS>
hipError_t launch_pass_tp(const Ctx& c, const PassDesc& pd, hipStream_t st) {
  const int nlines = AXIS == msl::ROW ? c.ny : c.nz;
  constexpr int L = N / P;
  const int G = lines_per_group(N, nlines, nlines);
  const dim3 grid(nlines / G), block(L * G);
  int kind = msl::pass_kind(pd);
  if (!c.dbT) kind = msl::KIND_GENERIC;  // the specialised kinds read the slice pack
  const unsigned lds = (unsigned)line_pass_lds_bytes(N, G);
  switch (kind) {
    case msl::KIND_FWD_MID:
      if constexpr (wave_mappable<N, P, AXIS>()) {
        if (wave_mapped(kind, pd)) {
          hipLaunchKernelGGL((k_pass<N, P, AXIS, msl::KIND_FWD_MID, true>), grid, block, lds, st, c, pd);
          break;
        }
      }
      hipLaunchKernelGGL((k_pass<N, P, AXIS, msl::KIND_FWD_MID>), grid, block, lds, st, c, pd);
      break;
    case msl::KIND_REV_MID: hipLaunchKernelGGL((k_pass<N, P, AXIS, msl::KIND_REV_MID>), grid, block, lds, st, c, pd); break;
    default: hipLaunchKernelGGL((k_pass<N, P, AXIS, msl::KIND_GENERIC>), grid, block, lds, st, c, pd); break;
  }
  return hipGetLastError();
}

// Lines of 64 points and more run at 4 or 8 points per lane, shorter ones at 4.
template <int N, int AXIS>
hipError_t launch_pass_t(const Ctx& c, const PassDesc& pd, hipStream_t st) {
  if constexpr (N >= 64) {
    if (points_per_lane(N) == 8) return launch_pass_tp<N, 8, AXIS>(c, pd, st);
  }
  return launch_pass_tp<N, 4, AXIS>(c, pd, st);
}

template <int AXIS>
hipError_t launch_pass_axis(int n, const Ctx& c, const PassDesc& pd, hipStream_t st) {
  switch (n) {
    case 16: return launch_pass_t<16, AXIS>(c, pd, st);
    case 32: return launch_pass_t<32, AXIS>(c, pd, st);
    case 64: return launch_pass_t<64, AXIS>(c, pd, st);
    case 128: return launch_pass_t<128, AXIS>(c, pd, st);
    case 256: return launch_pass_t<256, AXIS>(c, pd, st);
    case 512: return launch_pass_t<512, AXIS>(c, pd, st);
    case 1024: return launch_pass_t<1024, AXIS>(c, pd, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_pass(const Ctx& c, const PassDesc& pd, hipStream_t st) {
  return pd.axis == msl::ROW ? launch_pass_axis<msl::ROW>(c.nz, c, pd, st)
                             : launch_pass_axis<msl::COL>(c.ny, c, pd, st);
}

// ---------------------------------------------------------------------------
// call setup

struct Call {
  msl_geometry g;
  Layout L;
  Ctx c;
  char* ws;
  hipStream_t st;
};

Call make_call(const msl_geometry& g, const Layout& lay, void* ws, hipStream_t st) {
  Call k_{};
  k_.g = g;
  k_.L = lay;
  k_.ws = static_cast<char*>(ws);
  k_.st = st;
  Ctx& c = k_.c;
  auto P = [&](size_t off) { return reinterpret_cast<float2*>(k_.ws + off); };
  c.ny = g.ny;
  c.nz = g.nz;
  c.m = (int64_t)g.ny * g.nz;
  c.twz = P(k_.L.twz);
  c.twy = P(k_.L.twy);
  c.hz = P(k_.L.hz);
  c.hy = P(k_.L.hy);
  c.H_hi = P(k_.L.H_hi);
  c.H_lo = P(k_.L.H_lo);
  const double kk = 2.0 * M_PI / g.wavelength_nm;
  const double kdx = kk * g.dx_nm;
  c.kdx_hi = (float)kdx;
  c.kdx_lo = (float)(kdx - (double)c.kdx_hi);
  c.inv_m = 1.0f / (float)c.m;
  return k_;
}

Call make_call(const msl_geometry& g, int k, void* ws, hipStream_t st) { return make_call(g, layout(g, k), ws, st); }

msl_status build_tables(const Call& k, bool need_prop) {
  const msl_geometry& g = k.g;
  auto P = [&](size_t off) { return reinterpret_cast<float2*>(k.ws + off); };
  const int tb = 256;
  hipLaunchKernelGGL(k_twiddles, dim3((g.nz + tb - 1) / tb), dim3(tb), 0, k.st, g.nz, P(k.L.twz));
  hipLaunchKernelGGL(k_twiddles, dim3((g.ny + tb - 1) / tb), dim3(tb), 0, k.st, g.ny, P(k.L.twy));
  if (need_prop) {
    const double kk = 2.0 * M_PI / g.wavelength_nm;
    if (g.propagator == MSL_PROP_PARAXIAL) {
      hipLaunchKernelGGL(k_hpar, dim3((g.nz + tb - 1) / tb), dim3(tb), 0, k.st, g.nz, g.dz_nm, g.dx_nm, kk,
                         P(k.L.hz));
      hipLaunchKernelGGL(k_hpar, dim3((g.ny + tb - 1) / tb), dim3(tb), 0, k.st, g.ny, g.dy_nm, g.dx_nm, kk,
                         P(k.L.hy));
    } else {
      const int64_t m = (int64_t)g.ny * g.nz;
      hipLaunchKernelGGL(k_hexact, dim3((unsigned)((m + tb - 1) / tb)), dim3(tb), 0, k.st, g.ny, g.nz, g.dy_nm,
                         g.dz_nm, g.dx_nm, kk, P(k.L.H_hi), P(k.L.H_lo));
    }
  }
  return hip_check(hipGetLastError(), "table kernels");
}

// Helper stream and events of one device.  The adjoint runs side work on it
// beside the reverse sweep on the caller's stream: the segment recompute and
// the unpacking of finished gradient slices.  The batched forward runs its
// grid-size groups side by side on the extra streams.  Created on first use
// and kept for the life of the process (default priority, non-blocking).
// `mu` is held while a call enqueues work that uses the helper, so calls from
// several host threads do not interleave their event records and waits.
constexpr int kBatchStreams = 3;  // extra streams of the batched forward (grid-size groups side by side)

struct Helper {
  std::mutex mu;
  hipStream_t s = nullptr;
  hipEvent_t fork = nullptr, join = nullptr, done = nullptr;
  hipStream_t bs[kBatchStreams] = {};
  hipEvent_t bjoin[kBatchStreams] = {};
};

msl_status helper_for_current_device(Helper*& out) {
  static std::mutex mu;
  static Helper helpers[64];
  int dev = 0;
  MSL_TRY(hip_check(hipGetDevice(&dev), "hipGetDevice"));
  if (dev < 0 || dev >= 64) return fail(MSL_ERR_UNSUPPORTED, "device index out of range");
  std::lock_guard<std::mutex> lock(mu);
  Helper& h = helpers[dev];
  if (!h.s) {
    auto ev = [](hipEvent_t* e) { return hip_check(hipEventCreateWithFlags(e, hipEventDisableTiming), "hipEventCreateWithFlags"); };
    MSL_TRY(hip_check(hipStreamCreateWithFlags(&h.s, hipStreamNonBlocking), "hipStreamCreateWithFlags"));
    MSL_TRY(ev(&h.fork));
    MSL_TRY(ev(&h.join));
    MSL_TRY(ev(&h.done));
    for (int i = 0; i < kBatchStreams; ++i) {
      MSL_TRY(hip_check(hipStreamCreateWithFlags(&h.bs[i], hipStreamNonBlocking), "hipStreamCreateWithFlags"));
      MSL_TRY(ev(&h.bjoin[i]));
    }
  }
  out = &h;
  return MSL_OK;
}

// `dst` waits for the work enqueued on `src` so far.
msl_status stream_after(hipStream_t dst, hipStream_t src, hipEvent_t e) {
  MSL_TRY(hip_check(hipEventRecord(e, src), "hipEventRecord"));
  return hip_check(hipStreamWaitEvent(dst, e, 0), "hipStreamWaitEvent");
}

bool use_persistent(const Call& k, int np) {
  // the persistent kernel serves square grids; other shapes always run per pass
  if (k.c.ny != k.c.nz) return false;
  return g_schedule == MSL_SCHED_PERSISTENT ||
         (g_schedule == MSL_SCHED_AUTO && msl::persistent_preferred(k.c, np));
}

// Runs phase a, and phase b beside it when given (independent fields of a
// square grid), either as one cooperative launch or as launches per pass.
msl_status run_phases(const Call& k, const PhaseSpec& a, const PhaseSpec* b) {
  const int npa = msl::phase_npasses(a);
  const int npb = b ? msl::phase_npasses(*b) : 0;
  const int np = npa > npb ? npa : npb;
  if (np == 0) return MSL_OK;
  unsigned* bar = reinterpret_cast<unsigned*>(k.ws + k.L.bar);
  if (use_persistent(k, np)) {
    hipError_t e = msl::launch_persistent(k.c, a, npa, npb > 0 ? b : nullptr, npb, bar, g_spin_limit, k.st);
    if (e == hipSuccess) return MSL_OK;
    if (g_schedule == MSL_SCHED_PERSISTENT) return hip_check(e, "persistent pass kernel");
    (void)hipGetLastError();  // AUTO: the per-pass schedule below does the same work
  }
  for (int p = 0; p < np; ++p) {
    hipError_t e;
    if (p >= npa) break;
    e = launch_pass(k.c, msl::phase_pass(a, p), k.st);
    if (e != hipSuccess) return hip_check(e, "pass kernel");
  }
  for (int p = 0; p < npb; ++p) {
    hipError_t e = launch_pass(k.c, msl::phase_pass(*b, p), k.st);
    if (e != hipSuccess) return hip_check(e, "pass kernel");
  }
  return MSL_OK;
}

msl_status run_phase(const Call& k, const PhaseSpec& ph) { return run_phases(k, ph, nullptr); }

// Start of a call that runs phases: its workspace status word (msl_workspace_status) restarts at 0.
msl_status clear_status(const Call& k) {
  hipLaunchKernelGGL(msl::k_clear_status, dim3(1), dim3(64), 0, k.st, reinterpret_cast<unsigned*>(k.ws + k.L.bar));
  return hip_check(hipGetLastError(), "status kernel");
}

msl_status copy_field(const Call& k, void* dst, const void* src) {
  return hip_check(hipMemcpyAsync(dst, src, (size_t)k.c.m * 8, hipMemcpyDeviceToDevice, k.st), "hipMemcpyAsync");
}

int odd_slices(const msl_geometry& g) { return g.propagator == MSL_PROP_PARAXIAL ? g.n_slices / 2 : 0; }

// Odd slices among [s0, s1) are 2 s2 + 1 for s2 in [s0 / 2, s1 / 2).
int odd_begin(int s0) { return s0 >> 1; }
int odd_end(int s1) { return s1 >> 1; }

// Packs every slice into dbT (paraxial only: the exact schedule needs no pack).
msl_status pack_slices(Call& k) {
  if (k.g.propagator != MSL_PROP_PARAXIAL) return MSL_OK;
  float2* dbT = reinterpret_cast<float2*>(k.ws + k.L.dbT);
  MSL_TRY(hip_check(launch_pack(k.c.delta, k.c.beta, dbT, k.g.ny, k.g.nz, 0, k.g.n_slices, 0, 1, 1, k.c, k.st),
                    "pack kernel"));
  k.c.dbT = dbT;
  return MSL_OK;
}

// Unpacks the gradients of odd slices 2 s2 + 1, s2 in [s2b, s2e), on stream st.
msl_status unpack_odd_range(const Call& k, int s2b, int s2e, hipStream_t st) {
  if (s2e <= s2b || !k.c.gT) return MSL_OK;
  const dim3 grid = tile_grid(k.g.ny, k.g.nz, s2e - s2b);
  if (aligned(k.c.gdelta, 8) && aligned(k.c.gbeta, 8))   // (a NULL output counts as aligned)
    hipLaunchKernelGGL(k_unpack_tiled<true>, grid, dim3(256), 0, st, k.c.gT, k.c.gdelta, k.c.gbeta, k.g.ny, k.g.nz,
                       s2b, s2e);
  else
    hipLaunchKernelGGL(k_unpack_tiled<false>, grid, dim3(256), 0, st, k.c.gT, k.c.gdelta, k.c.gbeta, k.g.ny, k.g.nz,
                       s2b, s2e);
  return hip_check(hipGetLastError(), "unpack kernel");
}

PhaseSpec blank_phase(const Call& k, int kind) {
  PhaseSpec ph{};
  ph.kind = kind;
  ph.exact = k.g.propagator == MSL_PROP_EXACT;
  ph.ns = k.g.n_slices;
  ph.m = k.c.m;
  return ph;
}

// ---------------------------------------------------------------------------
// batched forward: one launch per (grid size, slice) over every instance of
// that grid size still in its slice loop

struct BatchRec {
  Ctx c;
  float2* field;
  // byte offsets in the batch workspace of the instance's tables, slice pack and working field:
  // the kernel forms those pointers from the workspace base it receives as an argument, so the
  // compiler addresses them as global memory (pointers read from the records are generic)
  uint64_t off_twz, off_twy, off_hz, off_hy, off_pack, off_field;
};

constexpr int kRecChunk = 16;  // records per descriptor-store launch (kernel arguments < 4 KB)

struct RecChunk {
  BatchRec r[kRecChunk];
  int n;
};
static_assert(sizeof(RecChunk) <= 4096, "kernel arguments are limited to 4 KB");

__global__ void k_store_recs(RecChunk chunk, BatchRec* dst) {
  if ((int)threadIdx.x < chunk.n) dst[threadIdx.x] = chunk.r[threadIdx.x];
}

// Middle forward pass (propagate, transmit slice tmpl.slice, propagate) of
// instances recs[0 .. gridDim.x / groups_per_inst): block b handles line
// group b mod groups_per_inst of instance b / groups_per_inst (after the
// XCD-aware renumbering of the whole grid).
template <int N, int P, int AXIS>
__global__ void __launch_bounds__(256) k_pass_batch(const BatchRec* __restrict__ recs, char* __restrict__ wsb,
                                                    int groups_per_inst, PassDesc tmpl) {
  extern __shared__ float2 lds[];  // line_pass_lds_bytes(N, G)
  constexpr int L = N / P;
  const int G = blockDim.x / L;
  const int g = threadIdx.x % G, j = threadIdx.x / G;
  const int gb = msl::xcd_group(blockIdx.x, gridDim.x);
  const int inst = gb / groups_per_inst;
  const BatchRec& r = recs[inst];
  Ctx c = r.c;
  c.twz = reinterpret_cast<const float2*>(wsb + r.off_twz);
  c.twy = reinterpret_cast<const float2*>(wsb + r.off_twy);
  c.hz = reinterpret_cast<const float2*>(wsb + r.off_hz);
  c.hy = reinterpret_cast<const float2*>(wsb + r.off_hy);
  c.dbT = reinterpret_cast<const float2*>(wsb + r.off_pack);
  float2* const field = reinterpret_cast<float2*>(wsb + r.off_field);
  PassDesc pd = tmpl;
  pd.src = field;
  pd.dst = field;
  msl::run_line<N, AXIS, false, msl::KIND_FWD_MID, msl::TS_PACK, P>(c, pd, (gb % groups_per_inst) * G + g, j,
                                                                   line_buffers<N>(lds, g, G));
}

template <int N, int P, int AXIS>
hipError_t launch_pass_batch_tp(const BatchRec* recs, char* wsb, int n_inst, int nlines, const PassDesc& tmpl,
                                hipStream_t st) {
  constexpr int L = N / P;
  const int G = lines_per_group(N, nlines, (int64_t)nlines * n_inst);
  const int gpi = nlines / G;
  hipLaunchKernelGGL((k_pass_batch<N, P, AXIS>), dim3(n_inst * gpi), dim3(L * G), (unsigned)line_pass_lds_bytes(N, G),
                     st, recs, wsb, gpi, tmpl);
  return hipGetLastError();
}

template <int N, int AXIS>
hipError_t launch_pass_batch_t(const BatchRec* recs, char* wsb, int n_inst, int nlines, const PassDesc& tmpl,
                               hipStream_t st) {
  if constexpr (N >= 64) {
    if (points_per_lane(N) == 8) return launch_pass_batch_tp<N, 8, AXIS>(recs, wsb, n_inst, nlines, tmpl, st);
  }
  return launch_pass_batch_tp<N, 4, AXIS>(recs, wsb, n_inst, nlines, tmpl, st);
}

template <int AXIS>
hipError_t launch_pass_batch_axis(int n, const BatchRec* recs, char* wsb, int n_inst, int nlines, const PassDesc& tmpl,
                                  hipStream_t st) {
  switch (n) {
    case 16: return launch_pass_batch_t<16, AXIS>(recs, wsb, n_inst, nlines, tmpl, st);
    case 32: return launch_pass_batch_t<32, AXIS>(recs, wsb, n_inst, nlines, tmpl, st);
    case 64: return launch_pass_batch_t<64, AXIS>(recs, wsb, n_inst, nlines, tmpl, st);
    case 128: return launch_pass_batch_t<128, AXIS>(recs, wsb, n_inst, nlines, tmpl, st);
    case 256: return launch_pass_batch_t<256, AXIS>(recs, wsb, n_inst, nlines, tmpl, st);
    case 512: return launch_pass_batch_t<512, AXIS>(recs, wsb, n_inst, nlines, tmpl, st);
    case 1024: return launch_pass_batch_t<1024, AXIS>(recs, wsb, n_inst, nlines, tmpl, st);
    default: return hipErrorInvalidValue;
  }
}

// Workspace of a batch: the records, then per instance its tables (twiddles,
// propagator factors), a scratch field for the far field and the packed
// transmissions of its pool.
struct BatchInstLayout {
  size_t twz, twy, hz, hy, tmp, pack;
};

struct BatchLayout {
  size_t recs;
  std::vector<BatchInstLayout> inst;
  size_t total;
};

BatchLayout batch_layout(const msl_instance* inst, int n) {
  BatchLayout L;
  size_t o = 0;
  auto take = [&](size_t bytes) { size_t r = o; o += up(bytes); return r; };
  L.recs = take((size_t)n * sizeof(BatchRec));
  L.inst.resize(n);
  for (int i = 0; i < n; ++i) {
    const msl_geometry& g = inst[i].g;
    const size_t m = (size_t)g.ny * g.nz;
    BatchInstLayout& b = L.inst[i];
    b.twz = take((size_t)msl::DITHER * g.nz * 8);
    b.twy = take((size_t)msl::DITHER * g.ny * 8);
    b.hz = take((size_t)msl::DITHER * g.nz * 8);
    b.hy = take((size_t)msl::DITHER * g.ny * 8);
    b.tmp = take(m * 8);
    b.pack = take((size_t)inst[i].n_pool * m * 8);
  }
  L.total = o;
  return L;
}

msl_status check_instances(const msl_instance* inst, int n) {
  if (!inst) return fail(MSL_ERR_ARG, "instance array is NULL");
  if (n < 1) return fail(MSL_ERR_ARG, "instance count must be >= 1");
  for (int i = 0; i < n; ++i) {
    const msl_instance& x = inst[i];
    const std::string at = "instance " + std::to_string(i) + ": ";
    if (check_geometry(&x.g) != MSL_OK) return fail(MSL_ERR_ARG, at + g_last_error);
    if (x.g.propagator != MSL_PROP_PARAXIAL)
      return fail(MSL_ERR_UNSUPPORTED, at + "the batched forward runs the paraxial propagator only");
    if (x.n_pool < 1) return fail(MSL_ERR_ARG, at + "n_pool must be >= 1");
    if (check_ptr(x.pool_delta, 4, "pool_delta") != MSL_OK || check_ptr(x.pool_beta, 4, "pool_beta") != MSL_OK ||
        check_ptr(x.slice_index, 4, "slice_index") != MSL_OK || check_ptr(x.probe, 8, "probe", true) != MSL_OK ||
        check_ptr(x.field_out, 8, "field_out") != MSL_OK || check_ptr(x.intensity_out, 4, "intensity_out", true) != MSL_OK)
      return fail(MSL_ERR_ARG, at + g_last_error);
  }
  return MSL_OK;
}

}  // namespace

// Coordinate search over the launch shape for a unit of work `run` enqueues on
// st: first the number of grid-size groups side by side (when tune_streams),
// then the points per lane and lines per workgroup of each slot in turn, every
// allowed pair;
// each candidate runs once untimed and then `reps` times between two events.
// The fastest setting stays in effect; on an error the previous one returns.
template <class Run>
msl_status autotune_shapes(Run run, hipStream_t st, int reps, const int* slots, int nslots, bool tune_streams,
                           msl_tuning* best, float* best_ms) {
  msl_tuning saved;
  MSL_TRY(msl_get_tuning(&saved));
  hipEvent_t e0 = nullptr, e1 = nullptr;
  MSL_TRY(hip_check(hipEventCreate(&e0), "hipEventCreate"));
  const msl_status ce = hip_check(hipEventCreate(&e1), "hipEventCreate");
  if (ce != MSL_OK) {
    (void)hipEventDestroy(e0);
    return ce;
  }
  auto time_run = [&](float& ms) -> msl_status {
    MSL_TRY(run());
    MSL_TRY(hip_check(hipEventRecord(e0, st), "hipEventRecord"));
    for (int r = 0; r < reps; ++r) MSL_TRY(run());
    MSL_TRY(hip_check(hipEventRecord(e1, st), "hipEventRecord"));
    MSL_TRY(hip_check(hipEventSynchronize(e1), "hipEventSynchronize"));
    MSL_TRY(hip_check(hipEventElapsedTime(&ms, e0, e1), "hipEventElapsedTime"));
    ms /= (float)reps;
    return MSL_OK;
  };
  auto search = [&](float& t_best) -> msl_status {
    MSL_TRY(time_run(t_best));
    if (tune_streams) {
      const int keep = g_batch_streams;
      const int current = keep > 0 ? keep : kBatchStreams + 1;
      int best_v = keep;
      for (int v = 1; v <= kBatchStreams + 1; ++v) {
        if (v == current) continue;
        g_batch_streams = v;
        float t = 0.0f;
        MSL_TRY(time_run(t));
        if (t < t_best) {
          t_best = t;
          best_v = v;
        }
      }
      g_batch_streams = best_v;
    }
    for (int q = 0; q < nslots; ++q) {
      const int e = slots[q], n = 1 << e;
      const int keep_v = g_lines_per_group[e], keep_p = g_points_per_lane[e];
      int best_v = keep_v, best_p = keep_p;
      for (int p : {4, 8}) {
        if (p == 8 && n < 64) continue;
        for (int v = 1; v <= max_lines_per_group(n, p); v *= 2) {
          g_points_per_lane[e] = p;
          g_lines_per_group[e] = v;
          float t = 0.0f;
          MSL_TRY(time_run(t));
          if (t < t_best) {
            t_best = t;
            best_v = v;
            best_p = p;
          }
        }
      }
      g_lines_per_group[e] = best_v;
      g_points_per_lane[e] = best_p;
    }
    return MSL_OK;
  };
  float t_best = 0.0f;
  const msl_status st_search = search(t_best);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st_search != MSL_OK) {
    (void)msl_set_tuning(&saved);
    return st_search;
  }
  if (best) MSL_TRY(msl_get_tuning(best));
  if (best_ms) *best_ms = t_best;
  return MSL_OK;
}

// ---------------------------------------------------------------------------
// Forward without allocation (msl_forward_noalloc): the tables live in a
// fixed-size device array instead of the caller's workspace.  Each GPU the
// library runs on holds its own copy of the array until the process ends; host
// code reaches it only through the address hipGetSymbolAddress returns for the
// current device (the array's name on the host is not a device address).

constexpr size_t kNoAllocLineTable = (size_t)msl::DITHER * 1024 * sizeof(float2);  // a line table, up to 1024 points
constexpr size_t kNoAllocHTable = (size_t)512 * 512 * sizeof(float2);  // exact propagator, up to 512 x 512
constexpr size_t kNoAllocBytes = 4 * kNoAllocLineTable + 2 * kNoAllocHTable;
static_assert(kNoAllocBytes == MSL_NOALLOC_SCRATCH_BYTES, "msl.h states the scratch size");

static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

namespace {

// Table regions of msl_forward_noalloc inside the scratch array (the layout
// fields of the workspace regions it does not use stay 0).
Layout noalloc_layout(const msl_geometry& g) {
  Layout L{};
  size_t o = 0;
  auto take = [&](size_t bytes) { size_t r = o; o += up(bytes); return r; };
  L.twz = take((size_t)msl::DITHER * g.nz * 8);
  L.twy = take((size_t)msl::DITHER * g.ny * 8);
  L.hz = take((size_t)msl::DITHER * g.nz * 8);
  L.hy = take((size_t)msl::DITHER * g.ny * 8);
  const bool exact = g.propagator == MSL_PROP_EXACT;
  const size_t m = (size_t)g.ny * g.nz;
  L.H_hi = take(exact ? m * 8 : 0);
  L.H_lo = take(exact ? m * 8 : 0);
  L.total = o;
  return L;
}

// Device address of the scratch array on the current device, looked up on the
// first call on that device and kept.
msl_status noalloc_scratch(char*& out) {
  static std::mutex mu;
  static void* ptr[64] = {};
  int dev = 0;
  MSL_TRY(hip_check(hipGetDevice(&dev), "hipGetDevice"));
  if (dev < 0 || dev >= 64) return fail(MSL_ERR_UNSUPPORTED, "device index out of range");
  std::lock_guard<std::mutex> lock(mu);
  if (!ptr[dev]) {
    void* p = nullptr;
    MSL_TRY(hip_check(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)"));
    if (!p) return fail(MSL_ERR_HIP, "hipGetSymbolAddress(scratch) returned NULL");
    ptr[dev] = p;
  }
  out = static_cast<char*>(ptr[dev]);
  return MSL_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// C ABI

extern "C" {

int32_t msl_abi_version(void) { return MSL_ABI_VERSION; }

const char* msl_last_error(void) { return g_last_error.c_str(); }

int32_t msl_set_schedule(int32_t schedule) {
  if (schedule != MSL_SCHED_AUTO && schedule != MSL_SCHED_PER_PASS && schedule != MSL_SCHED_PERSISTENT) {
    g_last_error = "unknown schedule " + std::to_string(schedule);
    return MSL_ERR_ARG;
  }
  const int prev = g_schedule;
  g_schedule = schedule;
  return prev;
}

int32_t msl_set_barrier_spin_limit(int32_t polls) {
  if (polls < 0) {
    g_last_error = "spin limit must be >= 0, got " + std::to_string(polls);
    return MSL_ERR_ARG;
  }
  const int32_t prev = (int32_t)std::min<unsigned>(g_spin_limit, 0x7fffffffu);
  g_spin_limit = (unsigned)polls;
  return prev;
}

msl_status msl_workspace_status(void* workspace, size_t ws_bytes, void* hip_stream) {
  if (!workspace) return fail(MSL_ERR_WORKSPACE, "workspace is NULL");
  if (!aligned(workspace, kAlign)) return fail(MSL_ERR_WORKSPACE, "workspace is not 256-byte aligned");
  if (ws_bytes < 8192) return fail(MSL_ERR_WORKSPACE, "workspace too small to hold a status word");
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  MSL_TRY(hip_check(hipStreamSynchronize(st), "hipStreamSynchronize"));
  unsigned w[2] = {0u, 0u};
  MSL_TRY(hip_check(hipMemcpy(w, workspace, sizeof w, hipMemcpyDeviceToHost), "hipMemcpy"));
  if (w[1] != 0u)
    return fail(MSL_ERR_HIP, "a grid barrier of the persistent schedule gave up waiting (bounded spin) in the last "
                             "call on this workspace; its results are not valid (the working field holds NaN)");
  return MSL_OK;
}

msl_status msl_set_tuning(const msl_tuning* t) {
  if (!t) return fail(MSL_ERR_ARG, "tuning is NULL");
  for (int e = 0; e < MSL_TUNE_SLOTS; ++e) {
    const int p = t->points_per_lane[e];
    const bool p_ok = p == 0 || (e >= 4 && p == 4) || (e >= 6 && p == 8);
    if (!p_ok)
      return fail(MSL_ERR_ARG, "points_per_lane[" + std::to_string(e) + "] = " + std::to_string(p) +
                                   ": must be 0, 4 (lines of 16 points and more) or 8 (64 points and more)");
    const int v = t->lines_per_group[e];
    if (v == 0) continue;
    const int hi = e >= 4 ? max_lines_per_group(1 << e, p > 0 ? p : default_points_per_lane(1 << e)) : 0;
    if (v < 0 || (v & (v - 1)) != 0 || v > hi)
      return fail(MSL_ERR_ARG, "lines_per_group[" + std::to_string(e) + "] = " + std::to_string(v) +
                                   ": must be 0 or a power of two <= " + std::to_string(hi) +
                                   " at that points_per_lane");
  }
  if (t->batch_streams < 0 || t->batch_streams > kBatchStreams + 1)
    return fail(MSL_ERR_ARG, "batch_streams must be in [0, " + std::to_string(kBatchStreams + 1) + "]");
  for (int e = 0; e < MSL_TUNE_SLOTS; ++e) {
    g_lines_per_group[e] = t->lines_per_group[e];
    g_points_per_lane[e] = t->points_per_lane[e];
  }
  g_batch_streams = t->batch_streams;
  return MSL_OK;
}

msl_status msl_get_tuning(msl_tuning* t) {
  if (!t) return fail(MSL_ERR_ARG, "tuning is NULL");
  for (int e = 0; e < MSL_TUNE_SLOTS; ++e) {
    t->lines_per_group[e] = g_lines_per_group[e];
    t->points_per_lane[e] = g_points_per_lane[e];
  }
  t->batch_streams = g_batch_streams;
  return MSL_OK;
}

msl_status msl_autotune_forward(const msl_geometry* g, const float* delta, const float* beta, msl_c64* field_scratch,
                                void* workspace, size_t ws_bytes, int32_t reps, void* hip_stream, msl_tuning* best,
                                float* best_ms) {
  MSL_TRY(check_geometry(g));
  if (!field_scratch) return fail(MSL_ERR_ARG, "field_scratch is NULL");
  if (reps < 1 || reps > 1000) return fail(MSL_ERR_ARG, "reps must be in [1, 1000]");
  auto run = [&]() {
    return msl_forward(g, delta, beta, nullptr, field_scratch, nullptr, 0, 0u, workspace, ws_bytes, hip_stream);
  };
  const int slots[2] = {__builtin_ctz((unsigned)g->nz), __builtin_ctz((unsigned)g->ny)};
  return autotune_shapes(run, static_cast<hipStream_t>(hip_stream), reps, slots, 2, false, best, best_ms);
}

msl_status msl_autotune_batch(const msl_instance* inst, int32_t n, void* workspace, size_t ws_bytes, int32_t reps,
                              void* hip_stream, msl_tuning* best, float* best_ms) {
  MSL_TRY(check_instances(inst, n));
  if (reps < 1 || reps > 1000) return fail(MSL_ERR_ARG, "reps must be in [1, 1000]");
  auto run = [&]() { return msl_forward_batch(inst, n, workspace, ws_bytes, hip_stream); };
  std::vector<int> slots;
  for (int i = 0; i < n; ++i)
    for (int d : {inst[i].g.nz, inst[i].g.ny}) {
      const int e = __builtin_ctz((unsigned)d);
      if (std::find(slots.begin(), slots.end(), e) == slots.end()) slots.push_back(e);
    }
  return autotune_shapes(run, static_cast<hipStream_t>(hip_stream), reps, slots.data(), (int)slots.size(), true, best,
                         best_ms);
}

size_t msl_workspace_bytes(const msl_geometry* g, int32_t ckpt_every) {
  if (check_geometry(g) != MSL_OK || ckpt_every < 0) return 0;
  return layout(*g, ckpt_every).total;
}

int32_t msl_checkpoint_count(const msl_geometry* g, int32_t ckpt_every) {
  if (check_geometry(g) != MSL_OK || ckpt_every < 1) return 0;
  return (g->n_slices + ckpt_every - 1) / ckpt_every;
}

msl_status msl_pack_slices(const msl_geometry* g, const float* delta, const float* beta, void* workspace,
                           size_t ws_bytes, void* hip_stream) {
  MSL_TRY(check_geometry(g));
  MSL_TRY(check_ptr(delta, 4, "delta"));
  MSL_TRY(check_ptr(beta, 4, "beta"));
  MSL_TRY(check_ws(*g, 0, workspace, ws_bytes));
  Call k = make_call(*g, 0, workspace, static_cast<hipStream_t>(hip_stream));
  k.c.delta = delta;
  k.c.beta = beta;
  return pack_slices(k);
}

msl_status msl_forward(const msl_geometry* g, const float* delta, const float* beta, const msl_c64* probe,
                       msl_c64* field_out, msl_c64* ckpt, int32_t ckpt_every, uint32_t flags, void* workspace,
                       size_t ws_bytes, void* hip_stream) {
  MSL_TRY(check_geometry(g));
  MSL_TRY(check_ptr(delta, 4, "delta"));
  MSL_TRY(check_ptr(beta, 4, "beta"));
  MSL_TRY(check_ptr(probe, 8, "probe", true));
  MSL_TRY(check_ptr(field_out, 8, "field_out"));
  MSL_TRY(check_ptr(ckpt, 8, "ckpt", true));
  if (ckpt && ckpt_every < 1) return fail(MSL_ERR_ARG, "ckpt given but ckpt_every < 1");
  if (!ckpt && ckpt_every != 0) return fail(MSL_ERR_ARG, "ckpt_every != 0 but ckpt is NULL");
  if (flags & ~MSL_REUSE_SLICE_PACK) return fail(MSL_ERR_ARG, "unknown msl_forward flags");
  MSL_TRY(check_ws(*g, 0, workspace, ws_bytes));
  Call k = make_call(*g, 0, workspace, static_cast<hipStream_t>(hip_stream));
  k.c.delta = delta;
  k.c.beta = beta;
  MSL_TRY(clear_status(k));
  MSL_TRY(build_tables(k, true));
  float2* f = reinterpret_cast<float2*>(field_out);
  const float2* in = reinterpret_cast<const float2*>(probe);
  if (!probe) {
    const double q = 2.0 * M_PI / g->wavelength_nm * std::sin(g->alpha_i_rad) * g->dy_nm;
    hipLaunchKernelGGL(k_probe, dim3((unsigned)((k.c.m + 255) / 256)), dim3(256), 0, k.st, g->ny, g->nz, q, f);
    MSL_TRY(hip_check(hipGetLastError(), "probe kernel"));
    in = f;
  }
  // the first pass reads the probe (row-major), the passes work on the tiled
  // working field, the last one writes the exit wave row-major
  PhaseSpec ph = blank_phase(k, msl::PH_FWD_FULL);
  ph.s0 = 0;
  ph.s1 = g->n_slices;
  ph.field = reinterpret_cast<float2*>(k.ws + k.L.tmp);
  ph.in_rm = in;
  ph.out_rm = f;
  ph.ckpt = reinterpret_cast<float2*>(ckpt);
  ph.ckpt_every = ckpt ? ckpt_every : 0;
  if (flags & MSL_REUSE_SLICE_PACK) {
    if (g->propagator == MSL_PROP_PARAXIAL) k.c.dbT = reinterpret_cast<const float2*>(k.ws + k.L.dbT);
  } else {
    MSL_TRY(pack_slices(k));
  }
  return run_phase(k, ph);
}

msl_status msl_forward_noalloc(const msl_geometry* g, const float* delta, const float* beta, const msl_c64* probe,
                               msl_c64* field_out, msl_c64* ckpt, int32_t ckpt_every, void* hip_stream) {
  MSL_TRY(check_geometry(g));
  MSL_TRY(check_ptr(delta, 4, "delta"));
  MSL_TRY(check_ptr(beta, 4, "beta"));
  MSL_TRY(check_ptr(probe, 8, "probe", true));
  MSL_TRY(check_ptr(field_out, 8, "field_out"));
  MSL_TRY(check_ptr(ckpt, 8, "ckpt", true));
  if (ckpt && ckpt_every < 1) return fail(MSL_ERR_ARG, "ckpt given but ckpt_every < 1");
  if (!ckpt && ckpt_every != 0) return fail(MSL_ERR_ARG, "ckpt_every != 0 but ckpt is NULL");
  const Layout lay = noalloc_layout(*g);
  if (lay.total > kNoAllocBytes)
    return fail(MSL_ERR_UNSUPPORTED, "msl_forward_noalloc: the tables of a " + std::to_string(g->ny) + " x " +
                                         std::to_string(g->nz) + " grid need " + std::to_string(lay.total) +
                                         " bytes, more than its fixed scratch of " + std::to_string(kNoAllocBytes) +
                                         " (the exact propagator's table fits grids up to 512 x 512 points)");
  char* base = nullptr;
  MSL_TRY(noalloc_scratch(base));
  Call k = make_call(*g, lay, base, static_cast<hipStream_t>(hip_stream));
  k.c.delta = delta;
  k.c.beta = beta;
  MSL_TRY(build_tables(k, true));
  float2* f = reinterpret_cast<float2*>(field_out);
  const float2* in = reinterpret_cast<const float2*>(probe);
  if (!probe) {
    const double q = 2.0 * M_PI / g->wavelength_nm * std::sin(g->alpha_i_rad) * g->dy_nm;
    hipLaunchKernelGGL(k_probe, dim3((unsigned)((k.c.m + 255) / 256)), dim3(256), 0, k.st, g->ny, g->nz, q, f);
    MSL_TRY(hip_check(hipGetLastError(), "probe kernel"));
    in = nullptr;
  }
  // No slice pack and no tiled working field (neither would fit a fixed
  // scratch): the passes work on the exit-wave array itself, row-major, and
  // the column passes evaluate the transmission of their slices from the
  // caller's stack, with the same arithmetic as the pack.  Always one launch
  // per pass.
  PhaseSpec ph = blank_phase(k, msl::PH_FWD_FULL);
  ph.s0 = 0;
  ph.s1 = g->n_slices;
  ph.field = f;
  ph.in_rm = in;
  ph.rowmajor = 1;
  ph.ckpt = reinterpret_cast<float2*>(ckpt);
  ph.ckpt_every = ckpt ? ckpt_every : 0;
  const int np = msl::phase_npasses(ph);
  for (int p = 0; p < np; ++p) MSL_TRY(hip_check(launch_pass(k.c, msl::phase_pass(ph, p), k.st), "pass kernel"));
  return MSL_OK;
}

msl_status msl_far_field(const msl_geometry* g, const msl_c64* field, float* intensity, void* workspace,
                         size_t ws_bytes, void* hip_stream) {
  MSL_TRY(check_geometry(g));
  MSL_TRY(check_ptr(field, 8, "field"));
  MSL_TRY(check_ptr(intensity, 4, "intensity"));
  MSL_TRY(check_ws(*g, 0, workspace, ws_bytes));
  Call k = make_call(*g, 0, workspace, static_cast<hipStream_t>(hip_stream));
  k.c.intensity = intensity;
  MSL_TRY(clear_status(k));
  MSL_TRY(build_tables(k, false));
  PhaseSpec ph = blank_phase(k, msl::PH_FF);
  ph.in_rm = reinterpret_cast<const float2*>(field);
  ph.field = reinterpret_cast<float2*>(k.ws + k.L.tmp);
  return run_phase(k, ph);
}

msl_status msl_amp_loss(const msl_geometry* g, const float* intensity, const float* meas_amp, double* loss_out,
                        float* grad_intensity, void* workspace, size_t ws_bytes, void* hip_stream) {
  MSL_TRY(check_geometry(g));
  MSL_TRY(check_ptr(intensity, 4, "intensity"));
  MSL_TRY(check_ptr(meas_amp, 4, "meas_amp"));
  MSL_TRY(check_ptr(loss_out, 8, "loss_out"));
  MSL_TRY(check_ptr(grad_intensity, 4, "grad_intensity", true));
  MSL_TRY(check_ws(*g, 0, workspace, ws_bytes));
  Call k = make_call(*g, 0, workspace, static_cast<hipStream_t>(hip_stream));
  double* partials = reinterpret_cast<double*>(k.ws + k.L.partials);
  const int64_t m = k.c.m;
  int blocks = (int)((m + 255) / 256);
  if (blocks > kPartials) blocks = kPartials;
  hipLaunchKernelGGL(k_amp_loss, dim3(blocks), dim3(256), 0, k.st, intensity, meas_amp, grad_intensity, partials, m);
  hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(256), 0, k.st, partials, blocks, loss_out);
  return hip_check(hipGetLastError(), "loss kernels");
}

msl_status msl_far_field_adjoint(const msl_geometry* g, const msl_c64* field, const float* grad_intensity,
                                 msl_c64* grad_field, void* workspace, size_t ws_bytes, void* hip_stream) {
  MSL_TRY(check_geometry(g));
  MSL_TRY(check_ptr(field, 8, "field"));
  MSL_TRY(check_ptr(grad_intensity, 4, "grad_intensity"));
  MSL_TRY(check_ptr(grad_field, 8, "grad_field"));
  MSL_TRY(check_ws(*g, 0, workspace, ws_bytes));
  Call k = make_call(*g, 0, workspace, static_cast<hipStream_t>(hip_stream));
  k.c.grad_intensity = grad_intensity;
  MSL_TRY(clear_status(k));
  MSL_TRY(build_tables(k, false));
  PhaseSpec ph = blank_phase(k, msl::PH_FFADJ);
  ph.in_rm = reinterpret_cast<const float2*>(field);
  ph.field = reinterpret_cast<float2*>(k.ws + k.L.tmp);
  ph.out_rm = reinterpret_cast<float2*>(grad_field);
  return run_phase(k, ph);
}

msl_status msl_adjoint(const msl_geometry* g, const float* delta, const float* beta, const msl_c64* probe,
                       const msl_c64* ckpt, int32_t ckpt_every, const msl_c64* grad_field, float* grad_delta,
                       float* grad_beta, msl_c64* grad_probe, uint32_t flags, void* workspace,
                       size_t ws_bytes, void* hip_stream) {
  (void)probe;  // the probe is ckpt[0]
  MSL_TRY(check_geometry(g));
  MSL_TRY(check_ptr(delta, 4, "delta"));
  MSL_TRY(check_ptr(beta, 4, "beta"));
  MSL_TRY(check_ptr(probe, 8, "probe", true));
  MSL_TRY(check_ptr(ckpt, 8, "ckpt"));
  if (ckpt_every < 1) return fail(MSL_ERR_ARG, "ckpt_every must be >= 1 for the adjoint");
  MSL_TRY(check_ptr(grad_field, 8, "grad_field"));
  MSL_TRY(check_ptr(grad_delta, 4, "grad_delta", true));
  MSL_TRY(check_ptr(grad_beta, 4, "grad_beta", true));
  MSL_TRY(check_ptr(grad_probe, 8, "grad_probe", true));
  if (flags & ~MSL_REUSE_SLICE_PACK) return fail(MSL_ERR_ARG, "unknown msl_adjoint flags");
  MSL_TRY(check_ws(*g, ckpt_every, workspace, ws_bytes));
  Call k = make_call(*g, ckpt_every, workspace, static_cast<hipStream_t>(hip_stream));
  k.c.delta = delta;
  k.c.beta = beta;
  k.c.gdelta = grad_delta;
  k.c.gbeta = grad_beta;
  MSL_TRY(clear_status(k));
  MSL_TRY(build_tables(k, true));
  if (flags & MSL_REUSE_SLICE_PACK) {
    if (g->propagator == MSL_PROP_PARAXIAL) k.c.dbT = reinterpret_cast<const float2*>(k.ws + k.L.dbT);
  } else {
    MSL_TRY(pack_slices(k));
  }
  const int nodd = odd_slices(*g);
  if (nodd > 0 && (grad_delta || grad_beta)) k.c.gT = reinterpret_cast<float2*>(k.ws + k.L.gT);
  float2* W = reinterpret_cast<float2*>(k.ws + k.L.W);
  float2* G = reinterpret_cast<float2*>(k.ws + k.L.G);
  const float2* gin = reinterpret_cast<const float2*>(grad_field);
  float2* gout = reinterpret_cast<float2*>(grad_probe);
  float2* seg = reinterpret_cast<float2*>(k.ws + k.L.seg);
  const float2* ck = reinterpret_cast<const float2*>(ckpt);
  const int ns = g->n_slices;
  const int nck = (ns + ckpt_every - 1) / ckpt_every;
  const int64_t seg_stride = (int64_t)(ckpt_every > 1 ? ckpt_every - 1 : 0) * k.c.m;
  auto seg_of = [&](int c) { return seg + (c & 1) * seg_stride; };
  auto recomp = [&](int c) {
    PhaseSpec ph = blank_phase(k, msl::PH_FWD_RECOMP);
    ph.s0 = c * ckpt_every;
    ph.s1 = ph.s0 + ckpt_every < ns ? ph.s0 + ckpt_every : ns;
    ph.field = W;
    ph.in_rm = ck + (int64_t)c * k.c.m;  // the first pass reads the checkpoint
    ph.seg = seg_of(c);
    return ph;
  };
  auto reverse = [&](int c) {
    PhaseSpec rv = blank_phase(k, msl::PH_REV);
    rv.s0 = c * ckpt_every;
    rv.s1 = rv.s0 + ckpt_every < ns ? rv.s0 + ckpt_every : ns;
    rv.leading = c == nck - 1;
    rv.field = G;
    rv.in_rm = c == nck - 1 ? gin : nullptr;   // the cotangent of the exit wave enters the first reverse phase
    rv.out_rm = c == 0 ? gout : nullptr;       // the probe's cotangent leaves the last one
    rv.seg = seg_of(c);
    rv.ckpt_c = ck + (int64_t)c * k.c.m;
    return rv;
  };
  if (ckpt_every == 1) {
    // every entrance field is a checkpoint: one reverse sweep reads them
    // directly (row-major), nothing is recomputed
    PhaseSpec rv = blank_phase(k, msl::PH_REV);
    rv.s0 = 0;
    rv.s1 = ns;
    rv.leading = 1;
    rv.field = G;
    rv.in_rm = gin;
    rv.out_rm = gout;
    rv.seg = const_cast<float2*>(ck) + k.c.m;   // slice s >= 1 at ck[s] (only read)
    rv.ckpt_c = ck;
    rv.seg_row_major = 1;
    MSL_TRY(run_phase(k, rv));
    MSL_TRY(unpack_odd_range(k, 0, nodd, k.st));
    return MSL_OK;
  }
  // Segment c-1 is recomputed from its checkpoint while the reverse sweep runs
  // over segment c: the two fields are independent, so on square grids they
  // share passes (and each pass has twice the lines to spread over the chip).
  MSL_TRY(run_phase(k, recomp(nck - 1)));
  const bool persistent = use_persistent(k, ckpt_every + 1);
  auto seg_odd_b = [&](int c) { return odd_begin(c * ckpt_every); };
  auto seg_odd_e = [&](int c) { return odd_end((c + 1) * ckpt_every < ns ? (c + 1) * ckpt_every : ns); };
  if (persistent && g->ny == g->nz) {
    // one cooperative launch carries both fields
    for (int c = nck - 1; c >= 0; --c) {
      PhaseSpec rv = reverse(c);
      if (c >= 1) {
        PhaseSpec nx = recomp(c - 1);
        MSL_TRY(run_phases(k, rv, &nx));
      } else {
        MSL_TRY(run_phase(k, rv));
      }
    }
    MSL_TRY(unpack_odd_range(k, 0, nodd, k.st));
  } else {
    // per-pass launches: the recompute of segment c-1 runs on the helper
    // stream while the reverse sweep over segment c runs on the caller's
    // stream; recompute(c-1) starts after reverse(c+1) (which read the same
    // segment buffer) and reverse(c-1) waits for recompute(c-1).  After
    // recompute(c-1) the helper unpacks the finished gradients of segment c+1.
    Helper* h = nullptr;
    MSL_TRY(helper_for_current_device(h));
    std::lock_guard<std::mutex> lock(h->mu);
    Call kh = k;
    kh.st = h->s;
    for (int c = nck - 1; c >= 0; --c) {
      if (c < nck - 1) MSL_TRY(hip_check(hipStreamWaitEvent(k.st, h->join, 0), "hipStreamWaitEvent"));
      MSL_TRY(stream_after(kh.st, k.st, h->fork));
      if (c >= 1) {
        MSL_TRY(run_phase(kh, recomp(c - 1)));
        MSL_TRY(hip_check(hipEventRecord(h->join, kh.st), "hipEventRecord"));
      }
      if (c < nck - 1) MSL_TRY(unpack_odd_range(k, seg_odd_b(c + 1), seg_odd_e(c + 1), kh.st));
      MSL_TRY(run_phase(k, reverse(c)));
    }
    MSL_TRY(unpack_odd_range(k, seg_odd_b(0), seg_odd_e(0), k.st));
    MSL_TRY(stream_after(k.st, kh.st, h->done));
  }
  return MSL_OK;
}

size_t msl_batch_workspace_bytes(const msl_instance* inst, int32_t n) {
  if (check_instances(inst, n) != MSL_OK) return 0;
  return batch_layout(inst, n).total;
}

msl_status msl_forward_batch(const msl_instance* inst, int32_t n, void* workspace, size_t ws_bytes,
                             void* hip_stream) {
  MSL_TRY(check_instances(inst, n));
  const BatchLayout BL = batch_layout(inst, n);
  if (!workspace) return fail(MSL_ERR_WORKSPACE, "workspace is NULL");
  if (!aligned(workspace, kAlign)) return fail(MSL_ERR_WORKSPACE, "workspace is not 256-byte aligned");
  if (ws_bytes < BL.total)
    return fail(MSL_ERR_WORKSPACE, "workspace too small: need " + std::to_string(BL.total) + " bytes, got " +
                                       std::to_string(ws_bytes));
  char* ws = static_cast<char*>(workspace);
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  BatchRec* drecs = reinterpret_cast<BatchRec*>(ws + BL.recs);
  // order: grouped by grid, slice count descending within a group, so the
  // instances still in their slice loop at any pass are a prefix of the group
  std::vector<int> order(n);
  for (int i = 0; i < n; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    const msl_geometry &ga = inst[a].g, &gb = inst[b].g;
    if (ga.ny != gb.ny) return ga.ny < gb.ny;
    if (ga.nz != gb.nz) return ga.nz < gb.nz;
    return ga.n_slices > gb.n_slices;
  });
  // per instance: tables, probe, pool pack, record
  std::vector<BatchRec> recs(n);
  std::vector<PhaseSpec> phs(n);
  for (int r = 0; r < n; ++r) {
    const int i = order[r];
    const msl_instance& x = inst[i];
    const msl_geometry& g = x.g;
    const BatchInstLayout& b = BL.inst[i];
    auto P = [&](size_t off) { return reinterpret_cast<float2*>(ws + off); };
    Call k{};
    k.g = g;
    k.ws = ws;
    k.st = st;
    Ctx& c = k.c;
    c.ny = g.ny;
    c.nz = g.nz;
    c.m = (int64_t)g.ny * g.nz;
    c.twz = P(b.twz);
    c.twy = P(b.twy);
    c.hz = P(b.hz);
    c.hy = P(b.hy);
    const double kdx = 2.0 * M_PI / g.wavelength_nm * g.dx_nm;
    c.kdx_hi = (float)kdx;
    c.kdx_lo = (float)(kdx - (double)c.kdx_hi);
    c.inv_m = 1.0f / (float)c.m;
    c.delta = x.pool_delta;
    c.beta = x.pool_beta;
    c.slice_index = x.slice_index;
    c.n_pool = x.n_pool;
    c.intensity = x.intensity_out;
    const int tb = 256;
    const double kk = 2.0 * M_PI / g.wavelength_nm;
    hipLaunchKernelGGL(k_twiddles, dim3((g.nz + tb - 1) / tb), dim3(tb), 0, st, g.nz, P(b.twz));
    hipLaunchKernelGGL(k_twiddles, dim3((g.ny + tb - 1) / tb), dim3(tb), 0, st, g.ny, P(b.twy));
    hipLaunchKernelGGL(k_hpar, dim3((g.nz + tb - 1) / tb), dim3(tb), 0, st, g.nz, g.dz_nm, g.dx_nm, kk, P(b.hz));
    hipLaunchKernelGGL(k_hpar, dim3((g.ny + tb - 1) / tb), dim3(tb), 0, st, g.ny, g.dy_nm, g.dx_nm, kk, P(b.hy));
    MSL_TRY(hip_check(hipGetLastError(), "table kernels"));
    float2* f = reinterpret_cast<float2*>(x.field_out);
    const float2* in = reinterpret_cast<const float2*>(x.probe);
    if (!x.probe) {
      const double q = kk * std::sin(g.alpha_i_rad) * g.dy_nm;
      hipLaunchKernelGGL(k_probe, dim3((unsigned)((c.m + 255) / 256)), dim3(256), 0, st, g.ny, g.nz, q, f);
      MSL_TRY(hip_check(hipGetLastError(), "probe kernel"));
      in = f;
    }
    float2* pack = P(b.pack);
    MSL_TRY(hip_check(launch_pack(x.pool_delta, x.pool_beta, pack, g.ny, g.nz, 0, x.n_pool, 0, 1, 0, c, st),
                      "pack kernel"));
    c.dbT = pack;
    recs[r].c = c;
    recs[r].field = P(b.tmp);  // tiled working field
    recs[r].off_twz = b.twz;
    recs[r].off_twy = b.twy;
    recs[r].off_hz = b.hz;
    recs[r].off_hy = b.hy;
    recs[r].off_pack = b.pack;
    recs[r].off_field = b.tmp;
    PhaseSpec& ph = phs[r];
    ph = PhaseSpec{};
    ph.kind = msl::PH_FWD_FULL;
    ph.ns = g.n_slices;
    ph.m = c.m;
    ph.s0 = 0;
    ph.s1 = g.n_slices;
    ph.field = P(b.tmp);
    ph.in_rm = in;
    ph.out_rm = f;
  }
  for (int r0 = 0; r0 < n; r0 += kRecChunk) {
    RecChunk ch{};
    ch.n = std::min(kRecChunk, n - r0);
    for (int q = 0; q < ch.n; ++q) ch.r[q] = recs[r0 + q];
    hipLaunchKernelGGL(k_store_recs, dim3(1), dim3(kRecChunk), 0, st, ch, drecs + r0);
  }
  MSL_TRY(hip_check(hipGetLastError(), "record store kernel"));
  // groups of equal grid; with several groups, each after the first runs on
  // one of the helper's extra streams (forked from and joined back into st)
  std::vector<std::pair<int, int>> groups;
  for (int g0 = 0; g0 < n;) {
    int g1 = g0 + 1;
    while (g1 < n && inst[order[g1]].g.ny == inst[order[g0]].g.ny && inst[order[g1]].g.nz == inst[order[g0]].g.nz) ++g1;
    groups.push_back({g0, g1});
    g0 = g1;
  }
  Helper* h = nullptr;
  std::unique_lock<std::mutex> lock;
  const int nextra = std::min((int)groups.size() - 1, g_batch_streams > 0 ? g_batch_streams - 1 : kBatchStreams);
  if (nextra > 0) {
    MSL_TRY(helper_for_current_device(h));
    lock = std::unique_lock<std::mutex>(h->mu);
    MSL_TRY(hip_check(hipEventRecord(h->fork, st), "hipEventRecord"));
    for (int i = 0; i < nextra; ++i) MSL_TRY(hip_check(hipStreamWaitEvent(h->bs[i], h->fork, 0), "hipStreamWaitEvent"));
  }
  for (size_t gi = 0; gi < groups.size(); ++gi) {
    const int g0 = groups[gi].first, g1 = groups[gi].second;
    const hipStream_t gs = (gi == 0 || nextra == 0) ? st : h->bs[(gi - 1) % nextra];
    const int ny = inst[order[g0]].g.ny, nz = inst[order[g0]].g.nz;
    const int max_ns = inst[order[g0]].g.n_slices;
    for (int r = g0; r < g1; ++r) MSL_TRY(hip_check(launch_pass(recs[r].c, msl::phase_pass(phs[r], 0), gs), "pass kernel"));
    int active = g1 - g0;  // instances with n_slices > p, a prefix of the group
    for (int p = 1; p <= max_ns; ++p) {
      while (active > 0 && inst[order[g0 + active - 1]].g.n_slices <= p) --active;
      if (active > 0) {
        const PassDesc tmpl = msl::phase_pass(phs[g0], p);
        const hipError_t e = tmpl.axis == msl::ROW
                                 ? launch_pass_batch_axis<msl::ROW>(nz, drecs + g0, ws, active, ny, tmpl, gs)
                                 : launch_pass_batch_axis<msl::COL>(ny, drecs + g0, ws, active, nz, tmpl, gs);
        MSL_TRY(hip_check(e, "batched pass kernel"));
      }
      // instances whose slice loop ended at p: their last propagation
      for (int r = g0 + active; r < g1 && inst[order[r]].g.n_slices >= p; ++r)
        if (inst[order[r]].g.n_slices == p)
          MSL_TRY(hip_check(launch_pass(recs[r].c, msl::phase_pass(phs[r], p), gs), "pass kernel"));
    }
  }
  for (int i = 0; i < nextra; ++i) {
    MSL_TRY(hip_check(hipEventRecord(h->bjoin[i], h->bs[i]), "hipEventRecord"));
    MSL_TRY(hip_check(hipStreamWaitEvent(st, h->bjoin[i], 0), "hipStreamWaitEvent"));
  }
  // far fields
  for (int r = 0; r < n; ++r) {
    if (!recs[r].c.intensity) continue;
    PhaseSpec ff{};
    ff.kind = msl::PH_FF;
    ff.m = recs[r].c.m;
    ff.ns = phs[r].ns;
    ff.in_rm = phs[r].out_rm;   // the exit wave (row-major); the working field is free again
    ff.field = phs[r].field;
    for (int p = 0; p < msl::phase_npasses(ff); ++p)
      MSL_TRY(hip_check(launch_pass(recs[r].c, msl::phase_pass(ff, p), st), "far-field kernel"));
  }
  return MSL_OK;
}

}  // extern "C"

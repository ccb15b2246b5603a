// libmsl learned-initialiser kernels (C ABI in include/msl_nn.h): a bfloat16
// matrix-core product with float32 accumulation and the data movement a small
// convolutional network needs around it (3x3 patch extraction and its adjoint,
// upsampling, row pooling, ReLU backward, ADAM, loss).
//
// The product is tiled for CDNA 64-wide wavefronts: a 256-thread workgroup
// owns a 64 x 128 tile of C, each of its four wavefronts a 32 x 64 part as two
// 32 x 32 accumulators of the 32x32x8 bfloat16 MFMA; tiles of A and B pass
// through LDS with k contiguous, so every lane fetches its four k values of an
// MFMA operand with one 8-byte read.
#include <hip/hip_runtime.h>

#include <cmath>
#include <algorithm>
#include <cstdint>
#include <string>

#include "msl.h"
#include "msl_common.hpp"
#include "msl_nn.h"

using namespace msl_host;

namespace {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

// float32 -> bfloat16, round to nearest even (NaN stays NaN)
__device__ __forceinline__ uint16_t to_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

constexpr int TM = 64, TN = 128, TK = 32, KP = TK + 4;

struct GemmArgs {
  int M, N, K, lda, transA, ldb, transB, ldc, relu;
  int kchunk;  // K range of blockIdx.z: [z * kchunk, min(K, (z + 1) * kchunk)); C offset z * M * ldc
  float beta;
  const uint16_t* A;
  const uint16_t* B;
  float* C;
  const float* bias;
  uint16_t* C16;
};

__global__ void __launch_bounds__(256) k_gemm_bf16(GemmArgs g) {
  __shared__ __attribute__((aligned(16))) uint16_t As[TM][KP];  // [m][k]
  __shared__ __attribute__((aligned(16))) uint16_t Bs[TN][KP];  // [n][k]
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int m0 = blockIdx.y * TM, n0 = blockIdx.x * TN;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 64;
  f32x16 acc0 = {}, acc1 = {};
  const int kbeg = blockIdx.z * g.kchunk, kend = min(g.K, kbeg + g.kchunk);
  float* const Cz = g.C + (int64_t)blockIdx.z * g.M * g.ldc;
  for (int k0 = kbeg; k0 < kend; k0 += TK) {
#pragma unroll
    for (int r = 0; r < (TM * TK) / 256; ++r) {
      const int e = tid + 256 * r;
      const int mm = g.transA ? e % TM : e / TK, kk = g.transA ? e / TM : e % TK;
      const int gm = m0 + mm, gk = k0 + kk;
      uint16_t val = 0;
      if (gm < g.M && gk < kend) val = g.A[g.transA ? (int64_t)gk * g.lda + gm : (int64_t)gm * g.lda + gk];
      As[mm][kk] = val;
    }
#pragma unroll
    for (int r = 0; r < (TN * TK) / 256; ++r) {
      const int e = tid + 256 * r;
      const int nn = g.transB ? e / TK : e % TN, kk = g.transB ? e % TK : e / TN;
      const int gk = k0 + kk, gn = n0 + nn;
      uint16_t val = 0;
      if (gk < kend && gn < g.N) val = g.B[g.transB ? (int64_t)gn * g.ldb + gk : (int64_t)gk * g.ldb + gn];
      Bs[nn][kk] = val;
    }
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < TK; ks += 8) {
      const int kq = ks + 4 * (lane >> 5);
      const bf16x4 a = *reinterpret_cast<const bf16x4*>(&As[wm + (lane & 31)][kq]);
      const bf16x4 b0 = *reinterpret_cast<const bf16x4*>(&Bs[wn + (lane & 31)][kq]);
      const bf16x4 b1 = *reinterpret_cast<const bf16x4*>(&Bs[wn + 32 + (lane & 31)][kq]);
      acc0 = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(a, b0, acc0, 0, 0, 0);
      acc1 = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(a, b1, acc1, 0, 0, 0);
    }
    __syncthreads();
  }
  // accumulator element 4i + j of lane l is C[8i + 4(l / 32) + j][l % 32] of the 32 x 32 tile
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int n = n0 + wn + 32 * h + (lane & 31);
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int m = m0 + wm + 8 * i + 4 * (lane >> 5) + j;
        if (m < g.M && n < g.N) {
          float v = h ? acc1[4 * i + j] : acc0[4 * i + j];
          const int64_t o = (int64_t)m * g.ldc + n;
          if (g.beta != 0.0f) v = __builtin_fmaf(g.beta, Cz[o], v);
          if (g.bias) v += g.bias[m];
          if (g.relu) v = fmaxf(v, 0.0f);
          Cz[o] = v;
          if (g.C16) g.C16[o] = to_bf16(v);
        }
      }
  }
}

// ---------------------------------------------------------------------------
// 3x3 convolutions as implicit products: the same tiles, LDS layout and MFMA
// sequence as k_gemm_bf16, with the patch operand formed while it is loaded
// (no patch matrix in memory).  k runs over (channel, tap), tap = 3 (dy + 1) +
// (dx + 1), in the patch matrix's row order, so the forward product is the
// explicit one bit for bit.

struct ConvArgs {
  int Co, C, B, H, W, s, Ho, Wo, relu;
  int K;      // GEMM depth: C * 9 (forward) or Co * 9 (input gradient)
  int64_t N;  // GEMM columns: B * Ho * Wo (forward) or B * H * W (input gradient)
  const uint16_t* w16;  // [Co][C * 9]
  const float* x;       // forward input [C][B][H][W]
  const uint16_t* x16;  // weight gradient: the input as bfloat16 bits instead of x (or nullptr)
  const uint16_t* dy16; // input gradient: output gradient [Co][B][Ho][Wo], bfloat16
  const float* bias;
  float* y;             // forward output [Co][B][Ho][Wo] or input gradient [C][B][H][W]
};

// Stores v[0..3] and v[4..7] as two 8-byte LDS writes.
__device__ __forceinline__ void lds_store8(uint16_t* dst, const uint16_t (&v)[8]) {
  uint2 a, b;
  a.x = (uint32_t)v[0] | ((uint32_t)v[1] << 16);
  a.y = (uint32_t)v[2] | ((uint32_t)v[3] << 16);
  b.x = (uint32_t)v[4] | ((uint32_t)v[5] << 16);
  b.y = (uint32_t)v[6] | ((uint32_t)v[7] << 16);
  *reinterpret_cast<uint2*>(dst) = a;
  *reinterpret_cast<uint2*>(dst + 4) = b;
}

__device__ __forceinline__ void mfma_tile(const uint16_t (&As)[TM][KP], const uint16_t (&Bs)[TN][KP], int wm, int wn,
                                          int lane, f32x16& acc0, f32x16& acc1) {
#pragma unroll
  for (int ks = 0; ks < TK; ks += 8) {
    const int kq = ks + 4 * (lane >> 5);
    const bf16x4 a = *reinterpret_cast<const bf16x4*>(&As[wm + (lane & 31)][kq]);
    const bf16x4 b0 = *reinterpret_cast<const bf16x4*>(&Bs[wn + (lane & 31)][kq]);
    const bf16x4 b1 = *reinterpret_cast<const bf16x4*>(&Bs[wn + 32 + (lane & 31)][kq]);
    acc0 = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(a, b0, acc0, 0, 0, 0);
    acc1 = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(a, b1, acc1, 0, 0, 0);
  }
}

// y = act(conv(x) + bias): M = Co, N = B Ho Wo, K = C 9.  Thread t loads
// weight row m0 + t/4, k 8 (t mod 4) .. +8, and the 16 patch values of
// pixel n0 + t mod 128 at k 16 (t / 128) .. +16.
__global__ void __launch_bounds__(256) k_conv_fwd(ConvArgs a) {
  __shared__ __attribute__((aligned(16))) uint16_t As[TM][KP];
  __shared__ __attribute__((aligned(16))) uint16_t Bs[TN][KP];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int m0 = blockIdx.y * TM;
  const int64_t n0 = (int64_t)blockIdx.x * TN;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 64;
  f32x16 acc0 = {}, acc1 = {};
  const int nl = tid % TN, kh = tid / TN;
  const int64_t n = n0 + nl;
  const bool n_ok = n < a.N;
  int b = 0, i = 0, j = 0;
  if (n_ok) {
    j = (int)(n % a.Wo);
    const int64_t t = n / a.Wo;
    i = (int)(t % a.Ho);
    b = (int)(t / a.Ho);
  }
  const int y0 = a.s * i - 1, x0 = a.s * j - 1;   // window corner (dy = dx = -1)
  const int64_t cstride = (int64_t)a.B * a.H * a.W;
  const float* xb = a.x + (int64_t)b * a.H * a.W;
  const bool w_vec = (a.K & 7) == 0 && (reinterpret_cast<uintptr_t>(a.w16) & 15) == 0;
  for (int k0 = 0; k0 < a.K; k0 += TK) {
    {
      const int m = tid >> 2, kq = (tid & 3) * 8;
      const int gm = m0 + m, gk = k0 + kq;
      uint16_t v[8];
      if (w_vec && gm < a.Co && gk + 8 <= a.K) {
        const uint4 u = *reinterpret_cast<const uint4*>(a.w16 + (int64_t)gm * a.K + gk);
        v[0] = (uint16_t)u.x; v[1] = (uint16_t)(u.x >> 16); v[2] = (uint16_t)u.y; v[3] = (uint16_t)(u.y >> 16);
        v[4] = (uint16_t)u.z; v[5] = (uint16_t)(u.z >> 16); v[6] = (uint16_t)u.w; v[7] = (uint16_t)(u.w >> 16);
      } else {
#pragma unroll
        for (int q = 0; q < 8; ++q) v[q] = (gm < a.Co && gk + q < a.K) ? a.w16[(int64_t)gm * a.K + gk + q] : (uint16_t)0;
      }
      lds_store8(&As[m][kq], v);
    }
    {
      const int kb = k0 + kh * 16;
      int c = kb / 9, tap = kb - 9 * c;
      uint16_t v[16];
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        float val = 0.0f;
        const int yy = y0 + tap / 3, xx = x0 + tap % 3;
        if (n_ok && kb + q < a.K && yy >= 0 && yy < a.H && xx >= 0 && xx < a.W)
          val = xb[(int64_t)c * cstride + (int64_t)yy * a.W + xx];
        v[q] = to_bf16(val);
        if (++tap == 9) {
          tap = 0;
          ++c;
        }
      }
      uint16_t lo[8], hi[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        lo[q] = v[q];
        hi[q] = v[q + 8];
      }
      lds_store8(&Bs[nl][kh * 16], lo);
      lds_store8(&Bs[nl][kh * 16 + 8], hi);
    }
    __syncthreads();
    mfma_tile(As, Bs, wm, wn, lane, acc0, acc1);
    __syncthreads();
  }
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int64_t nn = n0 + wn + 32 * h + (lane & 31);
#pragma unroll
    for (int i4 = 0; i4 < 4; ++i4)
#pragma unroll
      for (int jj = 0; jj < 4; ++jj) {
        const int m = m0 + wm + 8 * i4 + 4 * (lane >> 5) + jj;
        if (m < a.Co && nn < a.N) {
          float v = h ? acc1[4 * i4 + jj] : acc0[4 * i4 + jj];
          if (a.bias) v += a.bias[m];
          if (a.relu) v = fmaxf(v, 0.0f);
          a.y[(int64_t)m * a.N + nn] = v;
        }
      }
  }
}

// dx = sum over (co, tap) of W[co][c 9 + tap] dy[co][b][(y - dy)/s][(x - dx)/s] (terms whose
// source position is whole and inside): M = C, N = B H W, K = Co 9, k = 9 co + tap.
__global__ void __launch_bounds__(256) k_conv_bwd_data(ConvArgs a) {
  __shared__ __attribute__((aligned(16))) uint16_t As[TM][KP];
  __shared__ __attribute__((aligned(16))) uint16_t Bs[TN][KP];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int m0 = blockIdx.y * TM;
  const int64_t n0 = (int64_t)blockIdx.x * TN;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 64;
  f32x16 acc0 = {}, acc1 = {};
  const int nl = tid % TN, kh = tid / TN;
  const int64_t n = n0 + nl;
  const bool n_ok = n < a.N;
  int b = 0, yq = 0, xq = 0;
  if (n_ok) {
    xq = (int)(n % a.W);
    const int64_t t = n / a.W;
    yq = (int)(t % a.H);
    b = (int)(t / a.H);
  }
  const int64_t ostride = (int64_t)a.B * a.Ho * a.Wo;
  const uint16_t* db = a.dy16 + (int64_t)b * a.Ho * a.Wo;
  const int KC = a.C * 9;   // weight row length
  for (int k0 = 0; k0 < a.K; k0 += TK) {
    {
      // A[m = c][k = 9 co + tap] = w16[co][9 c + tap]
      const int m = tid >> 2, kq = (tid & 3) * 8;
      const int gm = m0 + m, gk = k0 + kq;
      uint16_t v[8];
      int co = gk / 9, tap = gk - 9 * co;
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        v[q] = (gm < a.C && gk + q < a.K) ? a.w16[(int64_t)co * KC + 9 * gm + tap] : (uint16_t)0;
        if (++tap == 9) {
          tap = 0;
          ++co;
        }
      }
      lds_store8(&As[m][kq], v);
    }
    {
      const int kb = k0 + kh * 16;
      int co = kb / 9, tap = kb - 9 * co;
      uint16_t v[16];
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        uint16_t val = 0;
        const int yy = yq - (tap / 3 - 1), xx = xq - (tap % 3 - 1);
        if (n_ok && kb + q < a.K && yy >= 0 && xx >= 0 && yy % a.s == 0 && xx % a.s == 0) {
          const int ii = yy / a.s, jj = xx / a.s;
          if (ii < a.Ho && jj < a.Wo) val = db[(int64_t)co * ostride + (int64_t)ii * a.Wo + jj];
        }
        v[q] = val;
        if (++tap == 9) {
          tap = 0;
          ++co;
        }
      }
      uint16_t lo[8], hi[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        lo[q] = v[q];
        hi[q] = v[q + 8];
      }
      lds_store8(&Bs[nl][kh * 16], lo);
      lds_store8(&Bs[nl][kh * 16 + 8], hi);
    }
    __syncthreads();
    mfma_tile(As, Bs, wm, wn, lane, acc0, acc1);
    __syncthreads();
  }
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int64_t nn = n0 + wn + 32 * h + (lane & 31);
#pragma unroll
    for (int i4 = 0; i4 < 4; ++i4)
#pragma unroll
      for (int jj = 0; jj < 4; ++jj) {
        const int m = m0 + wm + 8 * i4 + 4 * (lane >> 5) + jj;
        if (m < a.C && nn < a.N) a.y[(int64_t)m * a.N + nn] = h ? acc1[4 * i4 + jj] : acc0[4 * i4 + jj];
      }
  }
}

// Weight gradient, split along the pixels like msl_nn_gemm_bf16_splitk:
// part z accumulates dW[o][9c + t] over pixels [z kchunk, (z + 1) kchunk) into
// partials + z Co 9C.  M = Co, N = 9C, K = B Ho Wo.  Thread t loads dy row
// m0 + t/4, pixels 8 (t mod 4) .. +8, and the patch values of pixel t mod 32
// for the 16 (channel, tap) columns n0 + 16 (t / 32) .. +16.
__global__ void __launch_bounds__(256) k_conv_bwd_weight(ConvArgs a, int kchunk, float* __restrict__ partials) {
  __shared__ __attribute__((aligned(16))) uint16_t As[TM][KP];
  __shared__ __attribute__((aligned(16))) uint16_t Bs[TN][KP];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int m0 = blockIdx.y * TM, n0 = blockIdx.x * TN;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 64;
  f32x16 acc0 = {}, acc1 = {};
  const int64_t npix = (int64_t)a.B * a.Ho * a.Wo;
  const int64_t kbeg = (int64_t)blockIdx.z * kchunk;
  const int64_t kend = kbeg + kchunk < npix ? kbeg + kchunk : npix;
  const int NC = a.C * 9;
  const int64_t cstride = (int64_t)a.B * a.H * a.W;
  const bool dy_vec = (npix & 7) == 0 && (reinterpret_cast<uintptr_t>(a.dy16) & 15) == 0;
  const int kk = tid & 31, nq = (tid >> 5) * 16;
  for (int64_t k0 = kbeg; k0 < kend; k0 += TK) {
    {
      const int m = tid >> 2, kq = (tid & 3) * 8;
      const int gm = m0 + m;
      const int64_t gk = k0 + kq;
      uint16_t v[8];
      if (dy_vec && gm < a.Co && gk + 8 <= kend) {
        const uint4 u = *reinterpret_cast<const uint4*>(a.dy16 + (int64_t)gm * npix + gk);
        v[0] = (uint16_t)u.x; v[1] = (uint16_t)(u.x >> 16); v[2] = (uint16_t)u.y; v[3] = (uint16_t)(u.y >> 16);
        v[4] = (uint16_t)u.z; v[5] = (uint16_t)(u.z >> 16); v[6] = (uint16_t)u.w; v[7] = (uint16_t)(u.w >> 16);
      } else {
#pragma unroll
        for (int q = 0; q < 8; ++q) v[q] = (gm < a.Co && gk + q < kend) ? a.dy16[(int64_t)gm * npix + gk + q] : (uint16_t)0;
      }
      lds_store8(&As[m][kq], v);
    }
    {
      const int64_t p = k0 + kk;
      const bool p_ok = p < kend;
      int b = 0, i = 0, j = 0;
      if (p_ok) {
        j = (int)(p % a.Wo);
        const int64_t t = p / a.Wo;
        i = (int)(t % a.Ho);
        b = (int)(t / a.Ho);
      }
      const int y0 = a.s * i - 1, x0 = a.s * j - 1;
      const int64_t ib = (int64_t)b * a.H * a.W;
      const int nb = n0 + nq;
      int c = nb / 9, tap = nb - 9 * c;
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        uint16_t val = 0;
        const int yy = y0 + tap / 3, xx = x0 + tap % 3;
        if (p_ok && nb + q < NC && yy >= 0 && yy < a.H && xx >= 0 && xx < a.W) {
          const int64_t e = ib + (int64_t)c * cstride + (int64_t)yy * a.W + xx;
          val = a.x16 ? a.x16[e] : to_bf16(a.x[e]);
        }
        Bs[nq + q][kk] = val;
        if (++tap == 9) {
          tap = 0;
          ++c;
        }
      }
    }
    __syncthreads();
    mfma_tile(As, Bs, wm, wn, lane, acc0, acc1);
    __syncthreads();
  }
  float* const P = partials + (int64_t)blockIdx.z * a.Co * NC;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int n = n0 + wn + 32 * h + (lane & 31);
#pragma unroll
    for (int i4 = 0; i4 < 4; ++i4)
#pragma unroll
      for (int jj = 0; jj < 4; ++jj) {
        const int m = m0 + wm + 8 * i4 + 4 * (lane >> 5) + jj;
        if (m < a.Co && n < NC) P[(int64_t)m * NC + n] = h ? acc1[4 * i4 + jj] : acc0[4 * i4 + jj];
      }
  }
}

// ---------------------------------------------------------------------------
// 3x3 convolutions on halo tiles.  A workgroup owns MT output channels (rows)
// x NT = 8192 / MT pixels of one image, a TH x TW block of output positions.
// For every chunk of 16 input channels it stages once, in LDS and as
// bfloat16, the input block the 3x3 windows of its pixels cover (the halo:
// (TH - 1) s + 3 rows of (TW - 1) s + 3 positions, each position's 16
// channels contiguous) and the weights of its rows for those channels (all
// nine taps); the nine taps then read shifted views of the same staged block,
// so each input value crosses from memory once per chunk instead of once per
// tap.  k runs over (tap, channel), one 16-deep MFMA step per tap, as the
// gfx950 32x32x16 bfloat16 instruction: each of the four wavefronts
// accumulates a 32-row x 64-pixel part in two 32 x 32 float32 tiles.
//
// Staging: a thread reads four neighbouring positions of four channels (one
// 16-byte read per channel, 16-byte aligned groups along the row), swaps the
// 4 x 4 block in registers and writes each position's four channels as one
// 8-byte LDS store.  The weights are first packed by k_pack_weights into
// [row][tap][channel] order (channels padded to a multiple of 16), so a
// workgroup stages them with 16-byte reads.
//
// The same kernel computes the input gradient of a stride-1 convolution: a
// stride-1 convolution of the output gradient with the weights transposed
// (input and output channels swapped) and rotated by 180 degrees (flip).

constexpr int HCK = 16;         // input channels per chunk (one MFMA k step per tap)
constexpr int HCKP = HCK + 8;   // bfloat16 slots per staged position: 48-byte stride, conflict-free 16-byte reads

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

__host__ __device__ inline int pad16(int n) { return (n + 15) / 16 * 16; }

// wp[m][t][c] (c < pad16(Cin), zero beyond Cin) from w16 [Co][9 C]:
//   mode 0 (rows m = o, Cin = C, 9 taps): w16[m][9 c + t];
//   mode 1 (rows m = c, Cin = Co, 9 taps): w16[c][9 m + 8 - t] (stride-1 input gradient);
//   mode 2 (rows m = 4c + 2py + px, Cin = Co, 4 taps t = 2a + b): w16[c][9 c' + 3 k(py, a) + k(px, b)]
//   with c' the row's channel, zero where k has no tap (stride-2 input gradient, sub-pixel form).
__device__ __forceinline__ int sub_tap(int p, int a) { return p == 0 ? (a == 0 ? 1 : -1) : (a == 0 ? 2 : 0); }

__global__ void __launch_bounds__(256) k_pack_weights(int Co, int C, int mode, const uint16_t* __restrict__ w16,
                                                      uint16_t* __restrict__ wp) {
  const int M = mode == 0 ? Co : (mode == 1 ? C : 4 * C), Cin = mode == 0 ? C : Co, Cp = pad16(Cin);
  const int ntap = mode == 2 ? 4 : 9;
  const int64_t n = (int64_t)M * ntap * Cp;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    const int c = (int)(e % Cp);
    const int64_t mt = e / Cp;
    const int t = (int)(mt % ntap), m = (int)(mt / ntap);
    uint16_t v = 0;
    if (c < Cin) {
      if (mode == 0) {
        v = w16[(int64_t)m * 9 * C + 9 * c + t];
      } else if (mode == 1) {
        v = w16[(int64_t)c * 9 * C + 9 * m + 8 - t];
      } else {
        const int ch = m >> 2, py = (m >> 1) & 1, px = m & 1;
        const int ky = sub_tap(py, t >> 1), kx = sub_tap(px, t & 1);
        if (ky >= 0 && kx >= 0) v = w16[(int64_t)c * 9 * C + 9 * ch + 3 * ky + kx];
      }
    }
    wp[e] = v;
  }
}

struct HaloArgs {
  int M;                 // output channels (rows of the product)
  int C;                 // input channels
  int B, H, W, s, Ho, Wo, relu;
  int TW, TH, tiles_x, tiles_y;
  int Cp;                // row length of wp per tap: pad16(C)
  int vec;               // W a multiple of 4 and x aligned: whole 4-position groups read at once
  int accum;             // add the result to y instead of overwriting it (float32 y only)
  int ybf16;             // y holds bfloat16 bits (rounded to nearest even) instead of float32
  const uint16_t* wp;    // packed weights [M][9][Cp] (k_pack_weights)
  const void* x;         // [C][B][H][W], float32 or (xbf16) bfloat16 bits
  const float* bias;     // [M] or nullptr
  void* y;               // [M][B][Ho][Wo], float32 or (ybf16) bfloat16 bits
};

// Four consecutive values of one channel row as bfloat16 bits: positions x0 .. x0+3 of row `row`
// (zero outside [0, W)); a 16-byte (float) or 8-byte (bfloat16) read when all four are inside.
template <bool XBF16>
__device__ __forceinline__ void load4(const void* x, int64_t row, int x0, int W, bool vec, uint16_t (&o)[4]) {
  if constexpr (XBF16) {
    const uint16_t* p = static_cast<const uint16_t*>(x) + row;
    if (vec && x0 >= 0 && x0 + 3 < W) {
      const uint2 u = *reinterpret_cast<const uint2*>(p + x0);
      o[0] = (uint16_t)u.x; o[1] = (uint16_t)(u.x >> 16); o[2] = (uint16_t)u.y; o[3] = (uint16_t)(u.y >> 16);
    } else {
#pragma unroll
      for (int i = 0; i < 4; ++i) o[i] = (x0 + i >= 0 && x0 + i < W) ? p[x0 + i] : (uint16_t)0;
    }
  } else {
    const float* p = static_cast<const float*>(x) + row;
    if (vec && x0 >= 0 && x0 + 3 < W) {
      const float4 u = *reinterpret_cast<const float4*>(p + x0);
      o[0] = to_bf16(u.x); o[1] = to_bf16(u.y); o[2] = to_bf16(u.z); o[3] = to_bf16(u.w);
    } else {
#pragma unroll
      for (int i = 0; i < 4; ++i) o[i] = (x0 + i >= 0 && x0 + i < W) ? to_bf16(p[x0 + i]) : (uint16_t)0;
    }
  }
}

// Stages channels c0 .. c0+CH-1 (zero beyond C) of the HH x HW input block whose corner is (iy0,
// ix0) in image `img` (zero outside the image) into xs[(hy HW + hx) CHP + c] as bfloat16.  Item =
// (row, 4-position group from ix0 rounded down to a multiple of 4, channel quad); each thread reads
// the four positions of four channels (one 16- or 8-byte read per channel when vec and the group
// lies inside the row), swaps the 4 x 4 block and writes each position's four channels as one
// 8-byte LDS store.  All threads of the block call it.
template <int CH, int CHP, bool XBF16>
__device__ __forceinline__ void stage_block(uint16_t* xs, const void* x, int C, int c0, int64_t cstride, int64_t img,
                                            int H, int W, int iy0, int ix0, int HH, int HW, bool vec) {
  constexpr int NQ = CH / 4;
  const int xa = ix0 & ~3, ngx = (ix0 + HW - xa + 3) >> 2, nitems = HH * ngx * NQ;
  for (int it = threadIdx.x; it < nitems; it += blockDim.x) {
    const int cq = it % NQ, rg = it / NQ;
    const int hy = rg / ngx, g = rg - hy * ngx;
    const int yy = iy0 + hy, xg = xa + 4 * g;
    uint16_t v[4][4];   // [channel][position]
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int c = c0 + 4 * cq + k;
      if (yy >= 0 && yy < H && c < C) {
        load4<XBF16>(x, (int64_t)c * cstride + img + (int64_t)yy * W, xg, W, vec, v[k]);
      } else {
#pragma unroll
        for (int i = 0; i < 4; ++i) v[k][i] = 0;
      }
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int hx = xg + i - ix0;   // staged position in the row
      if (hx >= 0 && hx < HW) {
        uint2 u;
        u.x = (uint32_t)v[0][i] | ((uint32_t)v[1][i] << 16);
        u.y = (uint32_t)v[2][i] | ((uint32_t)v[3][i] << 16);
        *reinterpret_cast<uint2*>(&xs[(hy * HW + hx) * CHP + 4 * cq]) = u;
      }
    }
  }
}

// LDS bytes of a halo workgroup: the weights [MT][NTAP][16], then the staged positions [HH HW][HCKP].
int halo_lds_bytes(int MT, int TW, int TH, int s, bool sub) {
  const int HW = sub ? TW + 1 : (TW - 1) * s + 3, HH = sub ? TH + 1 : (TH - 1) * s + 3;
  return (MT * (sub ? 4 : 9) * HCK + HH * HW * HCKP) * (int)sizeof(uint16_t);
}

// SUB = false: the 3x3 convolution of stride a.s described above.  SUB = true: the input gradient
// of a stride-2 convolution split by output parity (sub-pixel form).  Input position (2u + py,
// 2v + px) receives dy[u + a][v + b] through the weight of tap (ky, kx) = (k(py, a), k(px, b)),
// a, b in {0, 1}, k(0, 0) = 1, k(1, 0) = 2, k(1, 1) = 0 (k(0, 1): no tap); so the gradient is a
// stride-1 2x2 convolution over dy (window corner at (u, v)) with 4 C rows, row 4c + 2py + px,
// whose packed weights are zero where there is no tap.  The four rows of a channel land in one
// lane's accumulator (elements 4i + j, j = 2py + px), which writes the 2 x 2 block of dx at
// (2u, 2v) as two 8-byte stores.  a.Ho, a.Wo are then the half-resolution grid (dy's size).
template <int MT, bool XBF16, bool SUB>
__global__ void __launch_bounds__(256) k_conv_halo(HaloArgs a) {
  constexpr int NTAP = SUB ? 4 : 9;
  extern __shared__ __attribute__((aligned(16))) uint16_t halo_smem[];
  uint16_t* const ws = halo_smem;                     // [MT][NTAP][HCK]
  uint16_t* const xs = halo_smem + MT * NTAP * HCK;   // [HH * HW][HCKP]
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int m0 = blockIdx.y * MT;
  int t = blockIdx.x;
  const int ox0 = (t % a.tiles_x) * a.TW;
  t /= a.tiles_x;
  const int oy0 = (t % a.tiles_y) * a.TH;
  const int b = t / a.tiles_y;
  const int s = SUB ? 1 : a.s;
  const int HW = SUB ? a.TW + 1 : (a.TW - 1) * s + 3, HH = SUB ? a.TH + 1 : (a.TH - 1) * s + 3;
  const int iy0 = SUB ? oy0 : oy0 * s - 1, ix0 = SUB ? ox0 : ox0 * s - 1;
  const bool vec = a.vec != 0;
  constexpr int MB = MT / 32;        // 32-row blocks per workgroup
  const int cb = wave % MB, pb = wave / MB;  // this wave's row block and 64-pixel block
  const int kq = 8 * (lane >> 5);
  // this lane's two pixels of the tile: n0 (first accumulator) and n0 + 32 (second)
  const int n0 = pb * 64 + (lane & 31), n1 = n0 + 32;
  const int ty0 = n0 / a.TW, tx0 = n0 - ty0 * a.TW, ty1 = n1 / a.TW, tx1 = n1 - ty1 * a.TW;
  const int hoff0 = (ty0 * HW + tx0) * s, hoff1 = (ty1 * HW + tx1) * s;
  const int64_t plane = (int64_t)a.H * a.W, cstride = (int64_t)a.B * plane;
  const int64_t img = (int64_t)b * plane;
  f32x16 acc0 = {}, acc1 = {};
  for (int c0 = 0; c0 < a.C; c0 += HCK) {
    stage_block<HCK, HCKP, XBF16>(xs, a.x, a.C, c0, cstride, img, a.H, a.W, iy0, ix0, HH, HW, vec);
    // weights: MT rows x NTAP taps x two 16-byte halves
    for (int e = tid; e < MT * NTAP * 2; e += 256) {
      const int half = e & 1, mt = e >> 1;
      const int gm = m0 + mt / NTAP;
      uint4 u = make_uint4(0u, 0u, 0u, 0u);
      if (gm < a.M) u = *reinterpret_cast<const uint4*>(a.wp + ((int64_t)m0 * NTAP + mt) * a.Cp + c0 + 8 * half);
      *reinterpret_cast<uint4*>(&ws[mt * HCK + 8 * half]) = u;
    }
    __syncthreads();
#pragma unroll
    for (int tap = 0; tap < NTAP; ++tap) {
      const int sh = SUB ? (tap >> 1) * HW + (tap & 1) : (tap / 3) * HW + tap % 3;
      const bf16x8 av =
          *reinterpret_cast<const bf16x8*>(&ws[((cb * 32 + (lane & 31)) * NTAP + tap) * HCK + kq]);
      const bf16x8 b0 = *reinterpret_cast<const bf16x8*>(&xs[(hoff0 + sh) * HCKP + kq]);
      const bf16x8 b1 = *reinterpret_cast<const bf16x8*>(&xs[(hoff1 + sh) * HCKP + kq]);
      acc0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, b0, acc0, 0, 0, 0);
      acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, b1, acc1, 0, 0, 0);
    }
    __syncthreads();
  }
  // accumulator element 4i + j of lane l: row 8i + 4 (l / 32) + j, pixel l mod 32 of the 32 x 32 tile
  auto store = [&](const f32x16& acc, int ty, int tx) {
    const int oy = oy0 + ty, ox = ox0 + tx;
    if (oy >= a.Ho || ox >= a.Wo) return;
    if constexpr (SUB) {
      // rows 4c + j: channel c = (row block + 8i + 4 (l / 32)) / 4, parity class j
      const int W2 = 2 * a.Wo;
      const int64_t npix2 = (int64_t)a.B * 4 * a.Ho * a.Wo;
      const int64_t o = ((int64_t)b * 2 * a.Ho + 2 * oy) * W2 + 2 * ox;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int c = (m0 + cb * 32 + 8 * i + 4 * (lane >> 5)) >> 2;
        if (4 * c < a.M) {
          float* const d = static_cast<float*>(a.y) + (int64_t)c * npix2 + o;
          float2 u0 = make_float2(acc[4 * i + 0], acc[4 * i + 1]), u1 = make_float2(acc[4 * i + 2], acc[4 * i + 3]);
          if (a.accum) {
            const float2 p0 = *reinterpret_cast<const float2*>(d), p1 = *reinterpret_cast<const float2*>(d + W2);
            u0 = make_float2(p0.x + u0.x, p0.y + u0.y);
            u1 = make_float2(p1.x + u1.x, p1.y + u1.y);
          }
          *reinterpret_cast<float2*>(d) = u0;
          *reinterpret_cast<float2*>(d + W2) = u1;
        }
      }
    } else {
      const int64_t npix = (int64_t)a.B * a.Ho * a.Wo;
      const int64_t o = ((int64_t)b * a.Ho + oy) * a.Wo + ox;
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int m = m0 + cb * 32 + 8 * i + 4 * (lane >> 5) + j;
          if (m < a.M) {
            float v = acc[4 * i + j];
            if (a.bias) v += a.bias[m];
            if (a.relu) v = fmaxf(v, 0.0f);
            const int64_t e = (int64_t)m * npix + o;
            if (a.ybf16) {
              static_cast<uint16_t*>(a.y)[e] = to_bf16(v);
            } else {
              float* const yf = static_cast<float*>(a.y);
              if (a.accum) v += yf[e];
              yf[e] = v;
            }
          }
        }
    }
  };
  store(acc0, ty0, tx0);
  store(acc1, ty1, tx1);
}

// Weight gradient on halo tiles: dw[o][9c + t] = sum over output pixels p of dy[o][p] times the
// input value of channel c under tap t of p (rounded to bfloat16 as in the forward).  A workgroup of
// three wavefronts owns 32 input channels x 32 output channels and a range of spatial tiles (its
// part of the pixel sum); wavefront r computes the three taps of kernel row r.  Per tile it stages
// the input block of its 32 channels (stage_block, positions channel-contiguous) and the output
// gradient of its 32 output channels at the tile's pixels ([o][pixel]); k runs over the pixels, 16
// per 32x32x16 MFMA: A = the channels' values under the tap at 16 pixels (8 per lane, gathered from
// the staged positions), B = dy at those pixels (8 consecutive per lane, one 16-byte LDS read).
constexpr int WCK = 32;        // input channels per workgroup
constexpr int WCKP = WCK + 4;  // staged position stride (bfloat16): 72 bytes
constexpr int WOC = 32;        // output channels per workgroup tile (a workgroup takes one or two)

struct WgradArgs {
  int Co, C, B, H, W, s, Ho, Wo;
  int TW, TH, KT, tiles_x, tiles_y, ntiles, per_part;
  int vec;
  const uint16_t* dy16;  // [Co][B][Ho][Wo]
  const void* x;         // [C][B][H][W], float32 or (XBF16) bfloat16 bits
  float* partials;       // [parts][Co][9C]
};

// bfloat16 slots of the staged input block, rounded up to 16 bytes (the dy tile after it is read
// with 16-byte accesses)
__host__ __device__ inline int wgrad_xs_slots(int TW, int TH, int s) {
  const int HW = (TW - 1) * s + 3, HH = (TH - 1) * s + 3;
  return (HH * HW * WCKP + 7) / 8 * 8;
}

int wgrad_lds_bytes(int TW, int TH, int s, int ot) {
  return (wgrad_xs_slots(TW, TH, s) + ot * WOC * (TW * TH + 8)) * (int)sizeof(uint16_t);
}

template <int OT, bool XBF16>
__global__ void __launch_bounds__(192) k_conv_wgrad_halo(WgradArgs a) {
  constexpr int NOC = 32 * OT;                      // output channels of this workgroup
  extern __shared__ __attribute__((aligned(16))) uint16_t wg_smem[];
  const int HW = (a.TW - 1) * a.s + 3, HH = (a.TH - 1) * a.s + 3;
  const int DKP = a.KT + 8;                         // row stride of the staged dy tile
  uint16_t* const xs = wg_smem;                     // [HH * HW][WCKP]
  uint16_t* const dys = wg_smem + wgrad_xs_slots(a.TW, a.TH, a.s);   // [NOC][DKP]
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int c0 = blockIdx.x * WCK, o0 = blockIdx.y * NOC, part = blockIdx.z;
  const int kq = 8 * (lane >> 5);
  const int64_t plane = (int64_t)a.H * a.W, cstride = (int64_t)a.B * plane;
  const int64_t npix = (int64_t)a.B * a.Ho * a.Wo;
  const bool vec = a.vec != 0;
  const bool dvec = (a.Wo & 7) == 0 && (reinterpret_cast<uintptr_t>(a.dy16) & 15) == 0;
  f32x16 acc[3][OT];                                // [tap column dx][output-channel tile]
#pragma unroll
  for (int dx = 0; dx < 3; ++dx)
#pragma unroll
    for (int ot = 0; ot < OT; ++ot) acc[dx][ot] = f32x16{};
  const int t0 = part * a.per_part, t1 = min(a.ntiles, t0 + a.per_part);
  for (int tile = t0; tile < t1; ++tile) {
    int t = tile;
    const int ox0 = (t % a.tiles_x) * a.TW;
    t /= a.tiles_x;
    const int oy0 = (t % a.tiles_y) * a.TH;
    const int b = t / a.tiles_y;
    const int iy0 = oy0 * a.s - 1, ix0 = ox0 * a.s - 1;
    stage_block<WCK, WCKP, XBF16>(xs, a.x, a.C, c0, cstride, (int64_t)b * plane, a.H, a.W, iy0, ix0, HH, HW, vec);
    // dy tile: item = (output channel, 8-pixel group of a tile row)
    const int ng = a.KT / 8;
    for (int it = tid; it < NOC * ng; it += blockDim.x) {
      const int oc = it / ng, g = it - oc * ng;
      const int n = 8 * g, ty = n / a.TW, tx = n - ty * a.TW;
      const int o = o0 + oc, oy = oy0 + ty, ox = ox0 + tx;
      uint4 u = make_uint4(0u, 0u, 0u, 0u);
      if (o < a.Co && oy < a.Ho) {
        const uint16_t* src = a.dy16 + (int64_t)o * npix + ((int64_t)b * a.Ho + oy) * a.Wo;
        if (dvec && ox + 7 < a.Wo) {
          u = *reinterpret_cast<const uint4*>(src + ox);
        } else {
          uint16_t v[8];
#pragma unroll
          for (int q = 0; q < 8; ++q) v[q] = ox + q < a.Wo ? src[ox + q] : (uint16_t)0;
          u.x = (uint32_t)v[0] | ((uint32_t)v[1] << 16);
          u.y = (uint32_t)v[2] | ((uint32_t)v[3] << 16);
          u.z = (uint32_t)v[4] | ((uint32_t)v[5] << 16);
          u.w = (uint32_t)v[6] | ((uint32_t)v[7] << 16);
        }
      }
      *reinterpret_cast<uint4*>(&dys[oc * DKP + n]) = u;
    }
    __syncthreads();
    for (int k0 = 0; k0 < a.KT; k0 += 16) {
      const int n = k0 + kq;                         // this lane's 8 pixels: n .. n+7, one tile row
      const int ty = n / a.TW, tx = n - ty * a.TW;
      bf16x8 bv[OT];
#pragma unroll
      for (int ot = 0; ot < OT; ++ot)
        bv[ot] = *reinterpret_cast<const bf16x8*>(&dys[(32 * ot + (lane & 31)) * DKP + n]);
      const int base = ((ty * a.s + wave) * HW + tx * a.s) * WCKP + (lane & 31);
      const int step = a.s * WCKP;
#pragma unroll
      for (int dx = 0; dx < 3; ++dx) {
        bf16x8 av;
        const uint16_t* src = xs + base + dx * WCKP;
#pragma unroll
        for (int i = 0; i < 8; ++i) av[i] = __builtin_bit_cast(__bf16, src[i * step]);
#pragma unroll
        for (int ot = 0; ot < OT; ++ot)
          acc[dx][ot] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, bv[ot], acc[dx][ot], 0, 0, 0);
      }
    }
    __syncthreads();
  }
  // accumulator element 4i + j of lane l: channel row 8i + 4 (l / 32) + j, output channel l mod 32
  const int NC = 9 * a.C;
#pragma unroll
  for (int ot = 0; ot < OT; ++ot) {
    const int o = o0 + 32 * ot + (lane & 31);
    if (o >= a.Co) continue;
    float* const P = a.partials + ((int64_t)part * a.Co + o) * NC;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int c = c0 + 8 * i + 4 * (lane >> 5) + j;
        if (c < a.C) {
          P[9 * c + 3 * wave + 0] = acc[0][ot][4 * i + j];
          P[9 * c + 3 * wave + 1] = acc[1][ot][4 * i + j];
          P[9 * c + 3 * wave + 2] = acc[2][ot][4 * i + j];
        }
      }
  }
}

// C[i] = sum over the parts s of P[s][i].  A workgroup takes 16 consecutive elements; its 16 thread
// slices each sum the parts s = slice, slice + 16, ... of every element (four independent loads in
// flight per thread), then slice sums are added in slice order, so the result does not depend on the
// launch and many parts over few elements still fill the GPU.
__global__ void __launch_bounds__(256) k_sum_parts(int64_t mn, int parts, const float* __restrict__ P, int M, int N,
                                                   int ldc, float* __restrict__ C) {
  __shared__ float part_sum[16][17];
  const int ei = threadIdx.x & 15, sl = threadIdx.x >> 4;
  const int64_t e = (int64_t)blockIdx.x * 16 + ei;
  float a0 = 0.0f, a1 = 0.0f, a2 = 0.0f, a3 = 0.0f;
  if (e < mn) {
    int s = sl;
    for (; s + 48 < parts; s += 64) {
      a0 += P[(int64_t)s * mn + e];
      a1 += P[(int64_t)(s + 16) * mn + e];
      a2 += P[(int64_t)(s + 32) * mn + e];
      a3 += P[(int64_t)(s + 48) * mn + e];
    }
    for (; s < parts; s += 16) a0 += P[(int64_t)s * mn + e];
  }
  part_sum[sl][ei] = (a0 + a1) + (a2 + a3);
  __syncthreads();
  if (sl == 0 && e < mn) {
    float acc = 0.0f;
    for (int q = 0; q < 16; ++q) acc += part_sum[q][ei];
    C[(e / N) * ldc + e % N] = acc;
  }
}

// grid: y = patch row r = c * 9 + tap, x over groups of output image rows (b, i).  A thread
// writes eight consecutive columns j of one output row (one 16-byte store when they are whole and
// aligned); cpr threads cover a row, 256 / cpr rows share a workgroup.
__global__ void __launch_bounds__(256) k_im2col(int C, int B, int H, int W, int s, int cpr, const float* __restrict__ x,
                                                uint16_t* __restrict__ col) {
  const int Ho = H / s, Wo = W / s;
  const int64_t ncol = (int64_t)B * Ho * Wo;
  const int r = blockIdx.y, c = r / 9, t = r % 9, dy = t / 3 - 1, dx = t % 3 - 1;
  const int rpb = 256 / cpr;
  const int rowid = blockIdx.x * rpb + (int)threadIdx.x / cpr;  // output image row b * Ho + i
  if (rowid >= B * Ho) return;
  const int b = rowid / Ho, i = rowid % Ho;
  const int y = s * i + dy;
  const bool row_ok = y >= 0 && y < H;
  const float* xr = x + ((int64_t)c * B + b) * H * W + (int64_t)(row_ok ? y : 0) * W;
  uint16_t* o = col + (int64_t)r * ncol + (int64_t)rowid * Wo;
  for (int j0 = 8 * ((int)threadIdx.x % cpr); j0 < Wo; j0 += 8 * cpr) {
    uint16_t v[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int jj = j0 + q, xx = s * jj + dx;
      v[q] = to_bf16(row_ok && jj < Wo && xx >= 0 && xx < W ? xr[xx] : 0.0f);
    }
    if (j0 + 8 <= Wo && (reinterpret_cast<uintptr_t>(o + j0) & 15) == 0) {
      uint4 w;
      w.x = (uint32_t)v[0] | ((uint32_t)v[1] << 16);
      w.y = (uint32_t)v[2] | ((uint32_t)v[3] << 16);
      w.z = (uint32_t)v[4] | ((uint32_t)v[5] << 16);
      w.w = (uint32_t)v[6] | ((uint32_t)v[7] << 16);
      *reinterpret_cast<uint4*>(o + j0) = w;
    } else {
      for (int q = 0; q < 8 && j0 + q < Wo; ++q) o[j0 + q] = v[q];
    }
  }
}

__global__ void __launch_bounds__(256) k_col2im(int C, int B, int H, int W, int s, const float* __restrict__ col,
                                                float* __restrict__ dx) {
  const int Ho = H / s, Wo = W / s;
  const int64_t ncol = (int64_t)B * Ho * Wo, total = (int64_t)C * B * H * W;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int xx = (int)(e % W), y = (int)((e / W) % H), b = (int)((e / ((int64_t)W * H)) % B);
    const int c = (int)(e / ((int64_t)W * H * B));
    float acc = 0.0f;
    for (int t = 0; t < 9; ++t) {
      const int dy = t / 3 - 1, dxx = t % 3 - 1;
      const int yi = y - dy, xj = xx - dxx;
      if (yi < 0 || xj < 0 || yi % s || xj % s) continue;
      const int i = yi / s, j = xj / s;
      if (i >= Ho || j >= Wo) continue;
      acc += col[((int64_t)c * 9 + t) * ncol + ((int64_t)b * Ho + i) * Wo + j];
    }
    dx[e] = acc;
  }
}

// Two equal neighbouring elements as one store (8 bytes for float32, 4 for bfloat16 bits).
__device__ __forceinline__ void store_pair(float* p, float v) { *reinterpret_cast<float2*>(p) = make_float2(v, v); }
__device__ __forceinline__ void store_pair(uint16_t* p, uint16_t v) {
  *reinterpret_cast<uint32_t*>(p) = (uint32_t)v | ((uint32_t)v << 16);
}

// Nearest 2x upsampling, one thread per input element x[r][w] (r over C B H rows): it writes the
// 2 x 2 block y[2r + d][2w .. 2w+1] (output row 2r + d of [C][B][2H][2W] is row r's copy d), as
// two pair stores when y is aligned for them.  IDX: the index type (32-bit when the sizes allow);
// T: float (float32) or uint16_t (bfloat16 bits, copied unchanged).
template <typename IDX, typename T>
__global__ void __launch_bounds__(256) k_upsample2(IDX total, int W, int vec, const T* __restrict__ x,
                                                   T* __restrict__ y) {
  for (IDX e = (IDX)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (IDX)gridDim.x * blockDim.x) {
    const IDX r = e / W, w = e - r * W;
    const T v = x[e];
    T* const o = y + 2 * r * (2 * (IDX)W) + 2 * w;
    if (vec) {
      store_pair(o, v);
      store_pair(o + 2 * W, v);
    } else {
      o[0] = v;
      o[1] = v;
      o[2 * W] = v;
      o[2 * W + 1] = v;
    }
  }
}

// Its adjoint: dx[r][w] = (dy[2r][2w] + dy[2r][2w+1]) + (dy[2r+1][2w] + dy[2r+1][2w+1]).
template <typename IDX>
__global__ void __launch_bounds__(256) k_upsample2_adj(IDX total, int W, int vec, const float* __restrict__ dy,
                                                       float* __restrict__ dx) {
  for (IDX e = (IDX)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (IDX)gridDim.x * blockDim.x) {
    const IDX r = e / W, w = e - r * W;
    const float* const p = dy + 2 * r * (2 * (IDX)W) + 2 * w;
    float2 a, b;
    if (vec) {
      a = *reinterpret_cast<const float2*>(p);
      b = *reinterpret_cast<const float2*>(p + 2 * W);
    } else {
      a = make_float2(p[0], p[1]);
      b = make_float2(p[2 * W], p[2 * W + 1]);
    }
    dx[e] = (a.x + a.y) + (b.x + b.y);
  }
}

// Per image row: the mean over all columns, the centre column, and the mean
// over the seven columns around the centre (fixed summation order), each
// shifted and scaled (when given), as bfloat16.
__global__ void __launch_bounds__(256) k_row_features(int B, int H, int W, const float* __restrict__ x,
                                                      const float* __restrict__ shift,
                                                      const float* __restrict__ scale, uint16_t* __restrict__ f) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)B * H) return;
  const int64_t b = e / H;
  const int r = (int)(e % H);
  const float* row = x + e * W;
  float all = 0.0f;
  for (int z = 0; z < W; ++z) all += row[z];
  const int c = W / 2;
  float mid = 0.0f;
  for (int z = c - 3; z <= c + 3; ++z) mid += row[z];
  const float v[3] = {all * (1.0f / (float)W), row[c], mid * (1.0f / 7.0f)};
  uint16_t* fb = f + b * 3 * H;
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    const int i = q * H + r;
    const float t = shift ? v[q] - shift[i] : v[q];
    fb[i] = to_bf16(scale ? t * scale[i] : t);
  }
}

// y[b][r][z] += p[r][b]
__global__ void __launch_bounds__(256) k_add_row_bias(int64_t total, int B, int R, int W, const float* __restrict__ p,
                                                      float* __restrict__ y) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int r = (int)((e / W) % R);
    const int b = (int)(e / ((int64_t)W * R));
    y[e] += p[(int64_t)r * B + b];
  }
}

// dp[r][b] = sum over z of dy[b][r][z] (z ascending)
__global__ void __launch_bounds__(256) k_row_bias_adjoint(int B, int R, int W, const float* __restrict__ dy,
                                                          float* __restrict__ dp) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)B * R) return;
  const int r = (int)(e / B), b = (int)(e % B);
  const float* row = dy + ((int64_t)b * R + r) * W;
  float acc = 0.0f;
  for (int z = 0; z < W; ++z) acc += row[z];
  dp[e] = acc;
}

__global__ void __launch_bounds__(256) k_rowpool(int64_t total, int H, int W, int f, const float* __restrict__ x,
                                                 float* __restrict__ y) {
  const int Hp = H / f;
  const float inv = 1.0f / (float)f;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int w = (int)(e % W), r = (int)((e / W) % Hp);
    const int64_t b = e / ((int64_t)W * Hp);
    float acc = 0.0f;
    for (int q = 0; q < f; ++q) acc += x[(b * H + (int64_t)f * r + q) * W + w];
    y[e] = acc * inv;
  }
}

__global__ void __launch_bounds__(256) k_rowpool_adj(int64_t total, int H, int W, int f, const float* __restrict__ dy,
                                                     float* __restrict__ dx) {
  const int Hp = H / f;
  const float inv = 1.0f / (float)f;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int w = (int)(e % W), Y = (int)((e / W) % H);
    const int64_t b = e / ((int64_t)W * H);
    dx[e] = dy[(b * Hp + Y / f) * W + w] * inv;
  }
}

__global__ void __launch_bounds__(256) k_relu_adj(int64_t n, const float* __restrict__ y, float* __restrict__ dy) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
    if (!(y[e] > 0.0f)) dy[e] = 0.0f;
}

__global__ void __launch_bounds__(256) k_add(int64_t n, const float* __restrict__ x, float* __restrict__ y) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
    y[e] += x[e];
}

__global__ void __launch_bounds__(256) k_to_bf16(int64_t n, const float* __restrict__ x, uint16_t* __restrict__ y) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
    y[e] = to_bf16(x[e]);
}

// row sums in two fixed-order stages: grid (parts, M) partial sums of column chunks, then one
// workgroup per row over the parts (deterministic)
constexpr int kRowParts = 64;

__global__ void __launch_bounds__(256) k_rowsum_parts(int N, const float* __restrict__ X, float* __restrict__ part) {
  __shared__ float red[256];
  const int chunk = (N + kRowParts - 1) / kRowParts;
  const int n0 = blockIdx.x * chunk, n1 = min(N, n0 + chunk);
  const float* row = X + (int64_t)blockIdx.y * N;
  float acc = 0.0f;
  for (int n = n0 + threadIdx.x; n < n1; n += 256) acc += row[n];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.y * kRowParts + blockIdx.x] = red[0];
}

__global__ void __launch_bounds__(64) k_rowsum_final(const float* __restrict__ part, float* __restrict__ out) {
  __shared__ float red[64];
  red[threadIdx.x] = part[blockIdx.x * kRowParts + threadIdx.x];
  __syncthreads();
  for (int w = 32; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[blockIdx.x] = red[0];
}

// Output-gradient preparation of one layer's backward, in one pass: g = dy masked by y > 0 (when y
// is given: the ReLU adjoint), written as bfloat16 to dy16, and the partial row sums of g (bias
// gradient; rows of N columns, kRowParts column chunks each, finished by k_rowsum_final).  dy is
// read only.  VEC: N a multiple of 4 and the arrays aligned, four columns per access.
template <bool VEC, bool YBF16>
__global__ void __launch_bounds__(256) k_grad_prep(int N, int chunk, const void* __restrict__ yv,
                                                   const float* __restrict__ dy, uint16_t* __restrict__ dy16,
                                                   float* __restrict__ part) {
  const float* const y = static_cast<const float*>(yv);
  const uint16_t* const y16 = static_cast<const uint16_t*>(yv);
  auto bf = [](uint32_t h) { return __uint_as_float(h << 16); };
  __shared__ float red[256];
  const int n0 = blockIdx.x * chunk, n1 = min(N, n0 + chunk);
  const int64_t row = (int64_t)blockIdx.y * N;
  float acc = 0.0f;
  if constexpr (VEC) {
    for (int n = n0 + 4 * (int)threadIdx.x; n < n1; n += 4 * 256) {
      float4 g = *reinterpret_cast<const float4*>(dy + row + n);
      if (yv) {
        float4 v;
        if constexpr (YBF16) {
          const uint2 h = *reinterpret_cast<const uint2*>(y16 + row + n);
          v = make_float4(bf(h.x & 0xffffu), bf(h.x >> 16), bf(h.y & 0xffffu), bf(h.y >> 16));
        } else {
          v = *reinterpret_cast<const float4*>(y + row + n);
        }
        if (!(v.x > 0.0f)) g.x = 0.0f;
        if (!(v.y > 0.0f)) g.y = 0.0f;
        if (!(v.z > 0.0f)) g.z = 0.0f;
        if (!(v.w > 0.0f)) g.w = 0.0f;
      }
      uint2 u;
      u.x = (uint32_t)to_bf16(g.x) | ((uint32_t)to_bf16(g.y) << 16);
      u.y = (uint32_t)to_bf16(g.z) | ((uint32_t)to_bf16(g.w) << 16);
      *reinterpret_cast<uint2*>(dy16 + row + n) = u;
      acc += (g.x + g.y) + (g.z + g.w);
    }
  } else {
    for (int n = n0 + (int)threadIdx.x; n < n1; n += 256) {
      float g = dy[row + n];
      if (yv && !((YBF16 ? bf(y16[row + n]) : y[row + n]) > 0.0f)) g = 0.0f;
      dy16[row + n] = to_bf16(g);
      acc += g;
    }
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.y * kRowParts + blockIdx.x] = red[0];
}

// Mean squared error in two fixed-order stages: kMseParts workgroups each sum the squared
// differences of one contiguous chunk in FP64 (and write the gradient), then one workgroup adds
// the partial sums in order.
constexpr int kMseParts = 256;

__global__ void __launch_bounds__(256) k_mse_parts(int64_t n, int64_t chunk, const float* __restrict__ p,
                                                   const float* __restrict__ t, float* __restrict__ grad,
                                                   double* __restrict__ part) {
  __shared__ double red[256];
  const double inv = 1.0 / (double)n;
  const int64_t e0 = (int64_t)blockIdx.x * chunk, e1 = min(n, e0 + chunk);
  double acc = 0.0;
  for (int64_t e = e0 + threadIdx.x; e < e1; e += 256) {
    const double d = (double)p[e] - (double)t[e];
    acc += d * d;
    if (grad) grad[e] = (float)(2.0 * d * inv);
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void __launch_bounds__(256) k_mse_final(int64_t n, const double* __restrict__ part,
                                                   double* __restrict__ loss) {
  __shared__ double red[256];
  red[threadIdx.x] = part[threadIdx.x];
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) loss[0] = red[0] / (double)n;
}

__global__ void __launch_bounds__(256) k_adam_flat(int64_t n, float* __restrict__ w, const float* __restrict__ g,
                                                   float* __restrict__ m, float* __restrict__ v,
                                                   uint16_t* __restrict__ w16, float lr, float b1, float b2,
                                                   float eps, float c1, float c2) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    const float gi = g[e];
    const float mi = __builtin_fmaf(b1, m[e], (1.0f - b1) * gi);
    const float vi = __builtin_fmaf(b2, v[e], (1.0f - b2) * (gi * gi));
    const float wi = w[e] - lr * (mi * c1) / (sqrtf(vi * c2) + eps);
    m[e] = mi;
    v[e] = vi;
    w[e] = wi;
    if (w16) w16[e] = to_bf16(wi);
  }
}

__global__ void __launch_bounds__(256) k_logmap(int64_t n, const float* __restrict__ x, float eps, float a, float b,
                                                float* __restrict__ out) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
    out[e] = __builtin_fmaf(a, logf(x[e] + eps), b);
}

// grid: x = row-column blocks of one slice, y = pool slice, z = sample
__global__ void __launch_bounds__(256) k_render(int ny, int nz, int sub_rows, float sub_d, float sub_b,
                                                const float* __restrict__ boxes, const int32_t* __restrict__ nf,
                                                const int32_t* __restrict__ cuts, const int32_t* __restrict__ np,
                                                const int64_t* __restrict__ off, float* __restrict__ pd,
                                                float* __restrict__ pb) {
  const int i = blockIdx.z, u = blockIdx.y;
  if (u >= np[i]) return;
  const int64_t m = (int64_t)ny * nz;
  const float x = (float)cuts[i * MSL_NN_MAX_CUTS + u];
  const float* bx = boxes + (int64_t)i * MSL_NN_MAX_BOXES * 8;
  const int nb = nf[i];
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m; e += (int64_t)gridDim.x * blockDim.x) {
    const float y = (float)(e / nz), z = (float)(e % nz);
    float d = y < (float)sub_rows ? sub_d : 0.0f, b = y < (float)sub_rows ? sub_b : 0.0f;
    for (int f = 0; f < nb; ++f) {
      const float* q = bx + 8 * f;
      if (x >= q[0] && x < q[1] && y >= q[2] && y < q[3] && z >= q[4] && z < q[5]) {
        d = q[6];
        b = q[7];
      }
    }
    const int64_t o = (off[i] + u) * m + e;
    pd[o] = d;
    pb[o] = b;
  }
}

__global__ void __launch_bounds__(256) k_pool_average(int ny, int nz, int y0, int rows, const float* __restrict__ w,
                                                      const int32_t* __restrict__ np, const int64_t* __restrict__ off,
                                                      const float* __restrict__ pool, float scale,
                                                      float* __restrict__ out) {
  const int i = blockIdx.y;
  const int64_t m = (int64_t)ny * nz, n = (int64_t)rows * nz;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t src = (int64_t)(y0 + e / nz) * nz + e % nz;
    float acc = 0.0f;
    for (int u = 0; u < np[i]; ++u) acc = __builtin_fmaf(w[i * MSL_NN_MAX_CUTS + u], pool[(off[i] + u) * m + src], acc);
    out[(int64_t)i * n + e] = scale * acc;
  }
}

unsigned blocks_for(int64_t n) {
  const int64_t b = (n + 255) / 256;
  return (unsigned)(b < 65536 ? b : 65536);
}

msl_status need(bool ok, const char* what) { return ok ? MSL_OK : fail(MSL_ERR_ARG, what); }

msl_status launched(const char* what) { return hip_check(hipGetLastError(), what); }

// Halo-tile shape of a convolution with M output rows and Ho x Wo outputs per image: rows per
// workgroup 32, 64 or 128 (one block up to 128 rows), pixels 8192 / MT as a TH x TW block, TW the
// largest power of two <= min(Wo, 64).  Packs the weights into wscratch first (k_pack_weights,
// mode 0 forward, 1 stride-1 input gradient, 2 stride-2 input gradient in sub-pixel form).
msl_status launch_conv_halo(HaloArgs a, int Co, int C, int mode, const uint16_t* w16, uint16_t* wscratch, bool xbf16,
                            hipStream_t st) {
  const bool sub = mode == 2;
  const int MT = a.M <= 32 ? 32 : (a.M <= 64 ? 64 : 128);
  const int NT = 8192 / MT;
  int TW = 1;
  while (2 * TW <= std::min(a.Wo, 64)) TW *= 2;
  a.TW = TW;
  a.TH = NT / TW;
  a.tiles_x = (a.Wo + a.TW - 1) / a.TW;
  a.tiles_y = (a.Ho + a.TH - 1) / a.TH;
  a.Cp = pad16(a.C);
  a.wp = wscratch;
  a.vec = (a.W % 4 == 0 && aligned(a.x, xbf16 ? 8 : 16)) ? 1 : 0;
  const int64_t nx = (int64_t)a.tiles_x * a.tiles_y * a.B;
  const int lds = halo_lds_bytes(MT, a.TW, a.TH, a.s, sub);
  MSL_TRY(need(nx < (1ll << 31) && (a.M + MT - 1) / MT <= 65535 && lds <= 64 * 1024, "conv: sizes too large"));
  const int64_t npack = (int64_t)a.M * (sub ? 4 : 9) * a.Cp;
  hipLaunchKernelGGL(k_pack_weights, dim3(blocks_for(npack)), dim3(256), 0, st, Co, C, mode, w16, wscratch);
  const dim3 grid((unsigned)nx, (unsigned)((a.M + MT - 1) / MT));
  switch (MT * 4 + (xbf16 ? 2 : 0) + (sub ? 1 : 0)) {
    case 128: hipLaunchKernelGGL((k_conv_halo<32, false, false>), grid, dim3(256), lds, st, a); break;
    case 130: hipLaunchKernelGGL((k_conv_halo<32, true, false>), grid, dim3(256), lds, st, a); break;
    case 131: hipLaunchKernelGGL((k_conv_halo<32, true, true>), grid, dim3(256), lds, st, a); break;
    case 256: hipLaunchKernelGGL((k_conv_halo<64, false, false>), grid, dim3(256), lds, st, a); break;
    case 258: hipLaunchKernelGGL((k_conv_halo<64, true, false>), grid, dim3(256), lds, st, a); break;
    case 259: hipLaunchKernelGGL((k_conv_halo<64, true, true>), grid, dim3(256), lds, st, a); break;
    case 512: hipLaunchKernelGGL((k_conv_halo<128, false, false>), grid, dim3(256), lds, st, a); break;
    case 514: hipLaunchKernelGGL((k_conv_halo<128, true, false>), grid, dim3(256), lds, st, a); break;
    case 515: hipLaunchKernelGGL((k_conv_halo<128, true, true>), grid, dim3(256), lds, st, a); break;
    default: return fail(MSL_ERR_ARG, "conv: no kernel for this shape");
  }
  return launched("conv kernel");
}

}  // namespace

extern "C" {

msl_status msl_nn_gemm_bf16(int32_t M, int32_t N, int32_t K, const uint16_t* A, int32_t lda, int32_t transA,
                            const uint16_t* B, int32_t ldb, int32_t transB, float* C, int32_t ldc, float beta,
                            const float* bias, int32_t relu, uint16_t* C16, void* hip_stream) {
  MSL_TRY(need(M >= 1 && N >= 1 && K >= 1, "gemm: M, N, K must be >= 1"));
  MSL_TRY(need(lda >= (transA ? M : K) && ldb >= (transB ? K : N) && ldc >= N, "gemm: leading dimension too small"));
  MSL_TRY(need(std::isfinite(beta), "gemm: beta must be finite"));
  MSL_TRY(check_ptr(A, 2, "A"));
  MSL_TRY(check_ptr(B, 2, "B"));
  MSL_TRY(check_ptr(C, 4, "C"));
  MSL_TRY(check_ptr(bias, 4, "bias", true));
  MSL_TRY(check_ptr(C16, 2, "C16", true));
  GemmArgs g{M, N, K, lda, transA ? 1 : 0, ldb, transB ? 1 : 0, ldc, relu ? 1 : 0, K, beta, A, B, C, bias, C16};
  const dim3 grid((N + TN - 1) / TN, (M + TM - 1) / TM);
  MSL_TRY(need(grid.y <= 65535, "gemm: M too large"));
  hipLaunchKernelGGL(k_gemm_bf16, grid, dim3(256), 0, static_cast<hipStream_t>(hip_stream), g);
  return launched("gemm kernel");
}

msl_status msl_nn_gemm_bf16_splitk(int32_t M, int32_t N, int32_t K, const uint16_t* A, int32_t lda, int32_t transA,
                                   const uint16_t* B, int32_t ldb, int32_t transB, float* C, int32_t ldc,
                                   int32_t splits, float* partials, void* hip_stream) {
  MSL_TRY(need(M >= 1 && N >= 1 && K >= 1, "gemm: M, N, K must be >= 1"));
  MSL_TRY(need(lda >= (transA ? M : K) && ldb >= (transB ? K : N) && ldc >= N, "gemm: leading dimension too small"));
  MSL_TRY(need(splits >= 1 && splits <= 4096, "gemm: splits must be in [1, 4096]"));
  MSL_TRY(check_ptr(A, 2, "A"));
  MSL_TRY(check_ptr(B, 2, "B"));
  MSL_TRY(check_ptr(C, 4, "C"));
  MSL_TRY(check_ptr(partials, 4, "partials"));
  // K range per part: a multiple of the K tile
  int kchunk = (K + splits - 1) / splits;
  kchunk = (kchunk + TK - 1) / TK * TK;
  const int parts = (K + kchunk - 1) / kchunk;
  GemmArgs g{M, N, K, lda, transA ? 1 : 0, ldb, transB ? 1 : 0, N, 0, kchunk, 0.0f, A, B, partials, nullptr, nullptr};
  const dim3 grid((N + TN - 1) / TN, (M + TM - 1) / TM, parts);
  MSL_TRY(need(grid.y <= 65535, "gemm: M too large"));
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  hipLaunchKernelGGL(k_gemm_bf16, grid, dim3(256), 0, st, g);
  const int64_t mn = (int64_t)M * N;
  hipLaunchKernelGGL(k_sum_parts, dim3((unsigned)((mn + 15) / 16)), dim3(256), 0, st, mn, parts, partials, M, N, ldc,
                     C);
  return launched("split gemm kernels");
}

int64_t msl_nn_conv3x3_scratch_elems(int32_t Co, int32_t C) {
  if (Co < 1 || C < 1) return 0;
  return (int64_t)16 * pad16(Co) * pad16(C);
}

msl_status msl_nn_conv3x3(int32_t Co, int32_t C, int32_t B, int32_t H, int32_t W, int32_t stride, const uint16_t* w16,
                          const void* x, int32_t x_bf16, const float* bias, int32_t relu, void* y, int32_t y_bf16,
                          uint16_t* wscratch, void* hip_stream) {
  MSL_TRY(need(Co >= 1 && C >= 1 && B >= 1 && H >= 1 && W >= 1 && (stride == 1 || stride == 2) && H % stride == 0 &&
                   W % stride == 0, "conv: need Co, C, B, H, W >= 1, stride 1 or 2 dividing H and W"));
  MSL_TRY(check_ptr(w16, 2, "w16"));
  MSL_TRY(check_ptr(x, x_bf16 ? 2 : 4, "x"));
  MSL_TRY(check_ptr(bias, 4, "bias", true));
  MSL_TRY(check_ptr(y, y_bf16 ? 2 : 4, "y"));
  MSL_TRY(check_ptr(wscratch, 16, "wscratch"));
  MSL_TRY(need((int64_t)C * 9 < (1 << 30) && (int64_t)B * H * W < (1ll << 40), "conv: sizes too large"));
  HaloArgs a{};
  a.M = Co; a.C = C; a.B = B; a.H = H; a.W = W; a.s = stride; a.Ho = H / stride; a.Wo = W / stride;
  a.relu = relu ? 1 : 0;
  a.ybf16 = y_bf16 ? 1 : 0;
  a.x = x; a.bias = bias; a.y = y;
  return launch_conv_halo(a, Co, C, 0, w16, wscratch, x_bf16 != 0, static_cast<hipStream_t>(hip_stream));
}

msl_status msl_nn_conv3x3_adjoint(int32_t Co, int32_t C, int32_t B, int32_t H, int32_t W, int32_t stride,
                                  const uint16_t* w16, const uint16_t* dy16, float* dx, int32_t accumulate,
                                  uint16_t* wscratch, void* hip_stream) {
  MSL_TRY(need(Co >= 1 && C >= 1 && B >= 1 && H >= 1 && W >= 1 && (stride == 1 || stride == 2) && H % stride == 0 &&
                   W % stride == 0, "conv adjoint: need Co, C, B, H, W >= 1, stride 1 or 2 dividing H and W"));
  MSL_TRY(check_ptr(w16, 2, "w16"));
  MSL_TRY(check_ptr(dy16, 2, "dy16"));
  MSL_TRY(check_ptr(dx, 4, "dx"));
  if (stride == 1 || aligned(dx, 8)) {
    // stride 1: a stride-1 convolution of dy with the weights transposed and rotated; stride 2: the
    // sub-pixel form, a 2x2 convolution over dy with 4 C rows (see k_conv_halo)
    MSL_TRY(check_ptr(wscratch, 16, "wscratch"));
    MSL_TRY(need((int64_t)C * 9 < (1 << 30) && (int64_t)B * H * W < (1ll << 40), "conv adjoint: sizes too large"));
    HaloArgs h{};
    h.M = stride == 1 ? C : 4 * C;
    h.C = Co; h.B = B; h.s = 1;
    h.H = H / stride; h.W = W / stride;   // the input of this product: dy
    h.Ho = H / stride; h.Wo = W / stride; // its output grid (half resolution for stride 2)
    h.relu = 0;
    h.accum = accumulate ? 1 : 0;
    h.x = dy16; h.bias = nullptr; h.y = dx;
    return launch_conv_halo(h, Co, C, stride == 1 ? 1 : 2, w16, wscratch, true, static_cast<hipStream_t>(hip_stream));
  }
  MSL_TRY(need(!accumulate, "conv adjoint: accumulate needs dx 8-byte aligned"));
  ConvArgs a{};
  a.Co = Co; a.C = C; a.B = B; a.H = H; a.W = W; a.s = stride; a.Ho = H / stride; a.Wo = W / stride;
  a.K = Co * 9;
  a.N = (int64_t)B * H * W;
  MSL_TRY(need((int64_t)Co * 9 < (1 << 30) && a.N < (1ll << 40), "conv adjoint: sizes too large"));
  a.w16 = w16; a.dy16 = dy16; a.y = dx;
  const dim3 grid((unsigned)((a.N + TN - 1) / TN), (unsigned)((C + TM - 1) / TM));
  MSL_TRY(need(grid.y <= 65535, "conv adjoint: too many input channels"));
  hipLaunchKernelGGL(k_conv_bwd_data, grid, dim3(256), 0, static_cast<hipStream_t>(hip_stream), a);
  return launched("conv adjoint kernel");
}

msl_status msl_nn_conv3x3_weight_grad(int32_t Co, int32_t C, int32_t B, int32_t H, int32_t W, int32_t stride,
                                     const uint16_t* dy16, const void* x, int32_t x_bf16, float* dw, int32_t splits,
                                     float* partials, void* hip_stream) {
  MSL_TRY(need(Co >= 1 && C >= 1 && B >= 1 && H >= 1 && W >= 1 && (stride == 1 || stride == 2) && H % stride == 0 &&
                   W % stride == 0, "conv weight gradient: need Co, C, B, H, W >= 1, stride 1 or 2 dividing H and W"));
  MSL_TRY(need(splits >= 1 && splits <= 4096, "conv weight gradient: splits must be in [1, 4096]"));
  MSL_TRY(check_ptr(dy16, 2, "dy16"));
  MSL_TRY(check_ptr(x, x_bf16 ? 2 : 4, "x"));
  MSL_TRY(check_ptr(dw, 4, "dw"));
  MSL_TRY(check_ptr(partials, 4, "partials"));
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  if ((W / stride) % 8 == 0) {
    // halo tiles (k_conv_wgrad_halo): 128 / s pixels per tile, as TH x TW, TW <= 64
    WgradArgs w{};
    w.Co = Co; w.C = C; w.B = B; w.H = H; w.W = W; w.s = stride; w.Ho = H / stride; w.Wo = W / stride;
    int TW = 8;
    while (2 * TW <= std::min(w.Wo, 64)) TW *= 2;
    w.TW = TW;
    w.KT = 128 / stride;   // smaller tiles: less LDS per workgroup, more of them per CU
    w.TH = w.KT / TW;
    w.tiles_x = (w.Wo + TW - 1) / TW;
    w.tiles_y = (w.Ho + w.TH - 1) / w.TH;
    const int64_t ntiles = (int64_t)w.tiles_x * w.tiles_y * B;
    MSL_TRY(need(ntiles < (1ll << 31) && (int64_t)C * 9 < (1 << 30), "conv weight gradient: sizes too large"));
    w.ntiles = (int)ntiles;
    // two output-channel tiles per workgroup when there are 64 or more output channels: each staged
    // input block then feeds twice the products
    const int ot = Co >= 2 * WOC ? 2 : 1;
    const int cb = (C + WCK - 1) / WCK, ob = (Co + ot * WOC - 1) / (ot * WOC);
    // parts: at most `splits`, enough workgroups to fill the GPU (about 2048), at least one tile each
    int parts = std::min<int64_t>(splits, ntiles);
    parts = std::max(1, std::min(parts, (2048 + cb * ob - 1) / (cb * ob)));
    w.per_part = (int)((ntiles + parts - 1) / parts);
    parts = (int)((ntiles + w.per_part - 1) / w.per_part);
    w.vec = (W % 4 == 0 && aligned(x, x_bf16 ? 8 : 16)) ? 1 : 0;
    w.dy16 = dy16; w.x = x; w.partials = partials;
    const int lds = wgrad_lds_bytes(w.TW, w.TH, stride, ot);
    MSL_TRY(need(lds <= 64 * 1024 && cb <= 65535 && ob <= 65535, "conv weight gradient: sizes too large"));
    const dim3 grid(cb, ob, parts);
    if (ot == 2 && x_bf16) hipLaunchKernelGGL((k_conv_wgrad_halo<2, true>), grid, dim3(192), lds, st, w);
    else if (ot == 2) hipLaunchKernelGGL((k_conv_wgrad_halo<2, false>), grid, dim3(192), lds, st, w);
    else if (x_bf16) hipLaunchKernelGGL((k_conv_wgrad_halo<1, true>), grid, dim3(192), lds, st, w);
    else hipLaunchKernelGGL((k_conv_wgrad_halo<1, false>), grid, dim3(192), lds, st, w);
    const int64_t mn = (int64_t)Co * 9 * C;
    hipLaunchKernelGGL(k_sum_parts, dim3((unsigned)((mn + 15) / 16)), dim3(256), 0, st, mn, parts, partials, Co,
                       9 * C, 9 * C, dw);
    return launched("conv weight gradient kernels");
  }
  ConvArgs a{};
  a.Co = Co; a.C = C; a.B = B; a.H = H; a.W = W; a.s = stride; a.Ho = H / stride; a.Wo = W / stride;
  a.dy16 = dy16;
  if (x_bf16) a.x16 = static_cast<const uint16_t*>(x);
  else a.x = static_cast<const float*>(x);
  const int64_t npix = (int64_t)B * a.Ho * a.Wo;
  MSL_TRY(need(npix < (1ll << 40) && (int64_t)C * 9 < (1 << 30), "conv weight gradient: sizes too large"));
  // pixel range per part: a multiple of the K tile (the split of msl_nn_gemm_bf16_splitk)
  int64_t kchunk = (npix + splits - 1) / splits;
  kchunk = (kchunk + TK - 1) / TK * TK;
  MSL_TRY(need(kchunk < (1ll << 31), "conv weight gradient: too few parts"));
  const int parts = (int)((npix + kchunk - 1) / kchunk);
  const int NC = C * 9;
  const dim3 grid((unsigned)((NC + TN - 1) / TN), (unsigned)((Co + TM - 1) / TM), (unsigned)parts);
  MSL_TRY(need(grid.y <= 65535 && grid.z <= 65535, "conv weight gradient: too many channels or parts"));
  hipLaunchKernelGGL(k_conv_bwd_weight, grid, dim3(256), 0, st, a, (int)kchunk, partials);
  const int64_t mn = (int64_t)Co * NC;
  hipLaunchKernelGGL(k_sum_parts, dim3((unsigned)((mn + 15) / 16)), dim3(256), 0, st, mn, parts, partials, Co, NC,
                     NC, dw);
  return launched("conv weight gradient kernels");
}

msl_status msl_nn_im2col3x3(int32_t C, int32_t B, int32_t H, int32_t W, int32_t stride, const float* x,
                            uint16_t* col, void* hip_stream) {
  MSL_TRY(need(C >= 1 && B >= 1 && H >= 1 && W >= 1 && (stride == 1 || stride == 2) && H % stride == 0 &&
                   W % stride == 0, "im2col: need C, B, H, W >= 1, stride 1 or 2 dividing H and W"));
  MSL_TRY(check_ptr(x, 4, "x"));
  MSL_TRY(check_ptr(col, 2, "col"));
  const int64_t ncol = (int64_t)B * (H / stride) * (W / stride);
  MSL_TRY(need(ncol < (1ll << 31) && C * 9 <= 65535, "im2col: too many columns or channels"));
  const int Wo = W / stride, rows = B * (H / stride);
  const int cpr = std::min(32, (Wo + 7) / 8);   // threads per output row (a power of two or fewer)
  int cp = 1;
  while (cp < cpr) cp *= 2;
  const int rpb = 256 / cp;
  const unsigned bx = (unsigned)((rows + rpb - 1) / rpb);
  hipLaunchKernelGGL(k_im2col, dim3(bx, C * 9), dim3(256), 0, static_cast<hipStream_t>(hip_stream), C, B, H, W, stride,
                     cp, x, col);
  return launched("im2col kernel");
}

msl_status msl_nn_col2im3x3(int32_t C, int32_t B, int32_t H, int32_t W, int32_t stride, const float* col, float* dx,
                            void* hip_stream) {
  MSL_TRY(need(C >= 1 && B >= 1 && H >= 1 && W >= 1 && (stride == 1 || stride == 2) && H % stride == 0 &&
                   W % stride == 0, "col2im: need C, B, H, W >= 1, stride 1 or 2 dividing H and W"));
  MSL_TRY(check_ptr(col, 4, "col"));
  MSL_TRY(check_ptr(dx, 4, "dx"));
  const int64_t total = (int64_t)C * B * H * W;
  hipLaunchKernelGGL(k_col2im, dim3(blocks_for(total)), dim3(256), 0, static_cast<hipStream_t>(hip_stream), C, B, H, W,
                     stride, col, dx);
  return launched("col2im kernel");
}

msl_status msl_nn_upsample2(int32_t C, int32_t B, int32_t H, int32_t W, const void* x, void* y, int32_t bf16,
                            void* hip_stream) {
  MSL_TRY(need(C >= 1 && B >= 1 && H >= 1 && W >= 1, "upsample: sizes must be >= 1"));
  const int es = bf16 ? 2 : 4;
  MSL_TRY(check_ptr(x, es, "x"));
  MSL_TRY(check_ptr(y, es, "y"));
  const int64_t total = (int64_t)C * B * H * W;   // input elements
  const int vec = aligned(y, 2 * es) ? 1 : 0;
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  const dim3 grid(blocks_for(total));
  const bool small = 4 * total < (1ll << 31);
  if (bf16) {
    const uint16_t* xb = static_cast<const uint16_t*>(x);
    uint16_t* yb = static_cast<uint16_t*>(y);
    if (small) hipLaunchKernelGGL((k_upsample2<int32_t, uint16_t>), grid, dim3(256), 0, st, (int32_t)total, W, vec, xb, yb);
    else hipLaunchKernelGGL((k_upsample2<int64_t, uint16_t>), grid, dim3(256), 0, st, total, W, vec, xb, yb);
  } else {
    const float* xf = static_cast<const float*>(x);
    float* yf = static_cast<float*>(y);
    if (small) hipLaunchKernelGGL((k_upsample2<int32_t, float>), grid, dim3(256), 0, st, (int32_t)total, W, vec, xf, yf);
    else hipLaunchKernelGGL((k_upsample2<int64_t, float>), grid, dim3(256), 0, st, total, W, vec, xf, yf);
  }
  return launched("upsample kernel");
}

msl_status msl_nn_upsample2_adjoint(int32_t C, int32_t B, int32_t H, int32_t W, const float* dy, float* dx,
                                    void* hip_stream) {
  MSL_TRY(need(C >= 1 && B >= 1 && H >= 1 && W >= 1, "upsample adjoint: sizes must be >= 1"));
  MSL_TRY(check_ptr(dy, 4, "dy"));
  MSL_TRY(check_ptr(dx, 4, "dx"));
  const int64_t total = (int64_t)C * B * H * W;
  const int vec = aligned(dy, 8) ? 1 : 0;
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  if (4 * total < (1ll << 31))
    hipLaunchKernelGGL(k_upsample2_adj<int32_t>, dim3(blocks_for(total)), dim3(256), 0, st, (int32_t)total, W, vec, dy,
                       dx);
  else
    hipLaunchKernelGGL(k_upsample2_adj<int64_t>, dim3(blocks_for(total)), dim3(256), 0, st, total, W, vec, dy, dx);
  return launched("upsample adjoint kernel");
}

msl_status msl_nn_row_features(int32_t B, int32_t H, int32_t W, const float* x, const float* shift, const float* scale,
                               uint16_t* f16, void* hip_stream) {
  MSL_TRY(need(B >= 1 && H >= 1 && W >= 8, "row features: need B, H >= 1 and W >= 8"));
  MSL_TRY(check_ptr(x, 4, "x"));
  MSL_TRY(check_ptr(shift, 4, "shift", true));
  MSL_TRY(check_ptr(scale, 4, "scale", true));
  MSL_TRY(check_ptr(f16, 2, "f16"));
  const int64_t n = (int64_t)B * H;
  MSL_TRY(need(n < (1ll << 31), "row features: too many rows"));
  hipLaunchKernelGGL(k_row_features, dim3((unsigned)((n + 255) / 256)), dim3(256), 0,
                     static_cast<hipStream_t>(hip_stream), B, H, W, x, shift, scale, f16);
  return launched("row features kernel");
}

msl_status msl_nn_add_row_bias(int32_t B, int32_t R, int32_t W, const float* p, float* y, void* hip_stream) {
  MSL_TRY(need(B >= 1 && R >= 1 && W >= 1, "add row bias: need B, R, W >= 1"));
  MSL_TRY(check_ptr(p, 4, "p"));
  MSL_TRY(check_ptr(y, 4, "y"));
  const int64_t total = (int64_t)B * R * W;
  hipLaunchKernelGGL(k_add_row_bias, dim3(blocks_for(total)), dim3(256), 0, static_cast<hipStream_t>(hip_stream),
                     total, B, R, W, p, y);
  return launched("add row bias kernel");
}

msl_status msl_nn_row_bias_adjoint(int32_t B, int32_t R, int32_t W, const float* dy, float* dp, void* hip_stream) {
  MSL_TRY(need(B >= 1 && R >= 1 && W >= 1, "row bias adjoint: need B, R, W >= 1"));
  MSL_TRY(check_ptr(dy, 4, "dy"));
  MSL_TRY(check_ptr(dp, 4, "dp"));
  const int64_t n = (int64_t)B * R;
  MSL_TRY(need(n < (1ll << 31), "row bias adjoint: too many rows"));
  hipLaunchKernelGGL(k_row_bias_adjoint, dim3((unsigned)((n + 255) / 256)), dim3(256), 0,
                     static_cast<hipStream_t>(hip_stream), B, R, W, dy, dp);
  return launched("row bias adjoint kernel");
}

msl_status msl_nn_rowpool(int32_t B, int32_t H, int32_t W, int32_t f, const float* x, float* y, void* hip_stream) {
  MSL_TRY(need(B >= 1 && H >= 1 && W >= 1 && f >= 1 && H % f == 0, "rowpool: need f dividing H"));
  MSL_TRY(check_ptr(x, 4, "x"));
  MSL_TRY(check_ptr(y, 4, "y"));
  const int64_t total = (int64_t)B * (H / f) * W;
  hipLaunchKernelGGL(k_rowpool, dim3(blocks_for(total)), dim3(256), 0, static_cast<hipStream_t>(hip_stream), total, H,
                     W, f, x, y);
  return launched("rowpool kernel");
}

msl_status msl_nn_rowpool_adjoint(int32_t B, int32_t H, int32_t W, int32_t f, const float* dy, float* dx,
                                  void* hip_stream) {
  MSL_TRY(need(B >= 1 && H >= 1 && W >= 1 && f >= 1 && H % f == 0, "rowpool adjoint: need f dividing H"));
  MSL_TRY(check_ptr(dy, 4, "dy"));
  MSL_TRY(check_ptr(dx, 4, "dx"));
  const int64_t total = (int64_t)B * H * W;
  hipLaunchKernelGGL(k_rowpool_adj, dim3(blocks_for(total)), dim3(256), 0, static_cast<hipStream_t>(hip_stream), total,
                     H, W, f, dy, dx);
  return launched("rowpool adjoint kernel");
}

msl_status msl_nn_relu_adjoint(int64_t n, const float* y, float* dy, void* hip_stream) {
  MSL_TRY(need(n >= 1, "relu adjoint: n must be >= 1"));
  MSL_TRY(check_ptr(y, 4, "y"));
  MSL_TRY(check_ptr(dy, 4, "dy"));
  hipLaunchKernelGGL(k_relu_adj, dim3(blocks_for(n)), dim3(256), 0, static_cast<hipStream_t>(hip_stream), n, y, dy);
  return launched("relu adjoint kernel");
}

msl_status msl_nn_add(int64_t n, const float* x, float* y, void* hip_stream) {
  MSL_TRY(need(n >= 1, "add: n must be >= 1"));
  MSL_TRY(check_ptr(x, 4, "x"));
  MSL_TRY(check_ptr(y, 4, "y"));
  hipLaunchKernelGGL(k_add, dim3(blocks_for(n)), dim3(256), 0, static_cast<hipStream_t>(hip_stream), n, x, y);
  return launched("add kernel");
}

msl_status msl_nn_to_bf16(int64_t n, const float* x, uint16_t* y16, void* hip_stream) {
  MSL_TRY(need(n >= 1, "to_bf16: n must be >= 1"));
  MSL_TRY(check_ptr(x, 4, "x"));
  MSL_TRY(check_ptr(y16, 2, "y16"));
  hipLaunchKernelGGL(k_to_bf16, dim3(blocks_for(n)), dim3(256), 0, static_cast<hipStream_t>(hip_stream), n, x, y16);
  return launched("bf16 conversion kernel");
}

msl_status msl_nn_rowsum(int32_t M, int32_t N, const float* X, float* out, float* parts, void* hip_stream) {
  MSL_TRY(need(M >= 1 && N >= 1, "rowsum: M, N must be >= 1"));
  MSL_TRY(check_ptr(X, 4, "X"));
  MSL_TRY(check_ptr(out, 4, "out"));
  MSL_TRY(need(M <= 65535, "rowsum: M too large"));
  MSL_TRY(check_ptr(parts, 4, "parts"));
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  hipLaunchKernelGGL(k_rowsum_parts, dim3(kRowParts, M), dim3(256), 0, st, N, X, parts);
  hipLaunchKernelGGL(k_rowsum_final, dim3(M), dim3(64), 0, st, parts, out);
  return launched("rowsum kernels");
}

msl_status msl_nn_grad_prep(int32_t M, int32_t N, const void* y, int32_t y_bf16, const float* dy, uint16_t* dy16,
                            float* bias_grad, float* parts, void* hip_stream) {
  MSL_TRY(need(M >= 1 && N >= 1 && M <= 65535, "grad prep: need 1 <= M <= 65535 and N >= 1"));
  MSL_TRY(check_ptr(y, y_bf16 ? 2 : 4, "y", true));
  MSL_TRY(check_ptr(dy, 4, "dy"));
  MSL_TRY(check_ptr(dy16, 2, "dy16"));
  MSL_TRY(check_ptr(bias_grad, 4, "bias_grad"));
  MSL_TRY(check_ptr(parts, 4, "parts"));
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  const bool vec = N % 4 == 0 && aligned(dy, 16) && aligned(dy16, 8) && (!y || aligned(y, y_bf16 ? 8 : 16));
  int chunk = (N + kRowParts - 1) / kRowParts;
  if (vec) chunk = (chunk + 3) / 4 * 4;
  const dim3 grid(kRowParts, M);
  if (vec && y_bf16) hipLaunchKernelGGL((k_grad_prep<true, true>), grid, dim3(256), 0, st, N, chunk, y, dy, dy16, parts);
  else if (vec) hipLaunchKernelGGL((k_grad_prep<true, false>), grid, dim3(256), 0, st, N, chunk, y, dy, dy16, parts);
  else if (y_bf16) hipLaunchKernelGGL((k_grad_prep<false, true>), grid, dim3(256), 0, st, N, chunk, y, dy, dy16, parts);
  else hipLaunchKernelGGL((k_grad_prep<false, false>), grid, dim3(256), 0, st, N, chunk, y, dy, dy16, parts);
  hipLaunchKernelGGL(k_rowsum_final, dim3(M), dim3(64), 0, st, parts, bias_grad);
  return launched("gradient preparation kernels");
}

msl_status msl_nn_mse(int64_t n, const float* pred, const float* target, float* grad, double* loss_out,
                      double* parts, void* hip_stream) {
  MSL_TRY(need(n >= 1, "mse: n must be >= 1"));
  MSL_TRY(check_ptr(pred, 4, "pred"));
  MSL_TRY(check_ptr(target, 4, "target"));
  MSL_TRY(check_ptr(grad, 4, "grad", true));
  MSL_TRY(check_ptr(loss_out, 8, "loss_out"));
  MSL_TRY(check_ptr(parts, 8, "parts"));
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  const int64_t chunk = (n + kMseParts - 1) / kMseParts;
  hipLaunchKernelGGL(k_mse_parts, dim3(kMseParts), dim3(256), 0, st, n, chunk, pred, target, grad, parts);
  hipLaunchKernelGGL(k_mse_final, dim3(1), dim3(256), 0, st, n, parts, loss_out);
  return launched("mse kernels");
}

msl_status msl_nn_adam(int64_t n, float* w, const float* g, float* m, float* v, uint16_t* w16, float lr, float beta1,
                       float beta2, float eps, int32_t t, void* hip_stream) {
  MSL_TRY(need(n >= 1 && t >= 1, "adam: need n >= 1 and t >= 1"));
  MSL_TRY(need(std::isfinite(lr) && lr >= 0 && beta1 >= 0 && beta1 < 1 && beta2 >= 0 && beta2 < 1 &&
                   std::isfinite(eps) && eps > 0,
               "adam: need lr >= 0, 0 <= beta1, beta2 < 1, eps > 0"));
  MSL_TRY(check_ptr(w, 4, "w"));
  MSL_TRY(check_ptr(g, 4, "g"));
  MSL_TRY(check_ptr(m, 4, "m"));
  MSL_TRY(check_ptr(v, 4, "v"));
  MSL_TRY(check_ptr(w16, 2, "w16", true));
  const float c1 = (float)(1.0 / (1.0 - std::pow((double)beta1, (double)t)));
  const float c2 = (float)(1.0 / (1.0 - std::pow((double)beta2, (double)t)));
  hipLaunchKernelGGL(k_adam_flat, dim3(blocks_for(n)), dim3(256), 0, static_cast<hipStream_t>(hip_stream), n, w, g, m,
                     v, w16, lr, beta1, beta2, eps, c1, c2);
  return launched("adam kernel");
}

msl_status msl_nn_logmap(int64_t n, const float* x, float eps, float a, float b, float* out, void* hip_stream) {
  MSL_TRY(need(n >= 1 && std::isfinite(eps) && eps > 0 && std::isfinite(a) && std::isfinite(b),
               "logmap: need n >= 1, eps > 0, finite a, b"));
  MSL_TRY(check_ptr(x, 4, "x"));
  MSL_TRY(check_ptr(out, 4, "out"));
  hipLaunchKernelGGL(k_logmap, dim3(blocks_for(n)), dim3(256), 0, static_cast<hipStream_t>(hip_stream), n, x, eps, a, b,
                     out);
  return launched("logmap kernel");
}

msl_status msl_nn_render_pools(int32_t n_samples, int32_t ny, int32_t nz, int32_t substrate_rows, float sub_delta,
                               float sub_beta, const float* boxes, const int32_t* nf, const int32_t* cuts,
                               const int32_t* np, const int64_t* pool_off, int32_t max_pool, float* pool_delta,
                               float* pool_beta, void* hip_stream) {
  MSL_TRY(need(n_samples >= 1 && n_samples <= 65535 && ny >= 1 && nz >= 1 && max_pool >= 1 &&
                   max_pool <= MSL_NN_MAX_CUTS - 1 && substrate_rows >= 0,
               "render: need 1 <= n_samples <= 65535, sizes >= 1, 1 <= max_pool < MSL_NN_MAX_CUTS"));
  MSL_TRY(check_ptr(boxes, 4, "boxes"));
  MSL_TRY(check_ptr(nf, 4, "nf"));
  MSL_TRY(check_ptr(cuts, 4, "cuts"));
  MSL_TRY(check_ptr(np, 4, "np"));
  MSL_TRY(check_ptr(pool_off, 8, "pool_off"));
  MSL_TRY(check_ptr(pool_delta, 4, "pool_delta"));
  MSL_TRY(check_ptr(pool_beta, 4, "pool_beta"));
  const int64_t m = (int64_t)ny * nz;
  const unsigned bx = (unsigned)std::min<int64_t>((m + 255) / 256, 256);
  hipLaunchKernelGGL(k_render, dim3(bx, max_pool, n_samples), dim3(256), 0, static_cast<hipStream_t>(hip_stream), ny,
                     nz, substrate_rows, sub_delta, sub_beta, boxes, nf, cuts, np, pool_off, pool_delta, pool_beta);
  return launched("render kernel");
}

msl_status msl_nn_pool_average(int32_t n_samples, int32_t ny, int32_t nz, int32_t y0, int32_t rows, const float* w,
                               const int32_t* np, const int64_t* pool_off, int32_t max_pool, const float* pool,
                               float scale, float* out, void* hip_stream) {
  MSL_TRY(need(n_samples >= 1 && n_samples <= 65535 && ny >= 1 && nz >= 1 && rows >= 1 && y0 >= 0 && y0 + rows <= ny &&
                   max_pool >= 1 && max_pool <= MSL_NN_MAX_CUTS - 1,
               "pool average: need 1 <= n_samples <= 65535, rows inside the grid"));
  MSL_TRY(check_ptr(w, 4, "w"));
  MSL_TRY(check_ptr(np, 4, "np"));
  MSL_TRY(check_ptr(pool_off, 8, "pool_off"));
  MSL_TRY(check_ptr(pool, 4, "pool"));
  MSL_TRY(check_ptr(out, 4, "out"));
  const int64_t n = (int64_t)rows * nz;
  const unsigned bx = (unsigned)std::min<int64_t>((n + 255) / 256, 256);
  hipLaunchKernelGGL(k_pool_average, dim3(bx, n_samples), dim3(256), 0, static_cast<hipStream_t>(hip_stream), ny, nz,
                     y0, rows, w, np, pool_off, pool, scale, out);
  return launched("pool average kernel");
}

}  // extern "C"

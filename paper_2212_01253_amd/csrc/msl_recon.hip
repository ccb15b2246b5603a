// libmsl reconstruction support [Sec. 4.1 of arXiv 2212.01253]: the delta
// values of a box of voxels are the unknowns (beta tied to delta by a fixed
// ratio); these kernels write a parameter vector into the slice stack and take
// one ADAM step (Kingma and Ba 2014) from the stack gradients of the loss.
// Both are elementwise over the box and bound by HBM bandwidth: the ADAM step
// reads two gradients and three parameter arrays and writes five arrays,
// 40 bytes per unknown.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <string>

#include "msl.h"
#include "msl_common.hpp"

using namespace msl_host;

namespace {

struct Box {
  int32_t s0, y0, z0, ny, nz;  // box origin and transverse extent
  int64_t n;                   // ns * ny * nz
  int32_t gny, gnz;            // stack grid
};

__device__ __forceinline__ int64_t box_to_stack(const Box& b, int64_t i) {
  const int64_t z = i % b.nz;
  const int64_t r = i / b.nz;
  const int64_t y = r % b.ny;
  const int64_t s = r / b.ny;
  return ((b.s0 + s) * b.gny + (b.y0 + y)) * b.gnz + (b.z0 + z);
}

__global__ void __launch_bounds__(256) k_region_scatter(Box b, float ratio, const float* __restrict__ theta,
                                                        float* __restrict__ delta, float* __restrict__ beta) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < b.n; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t e = box_to_stack(b, i);
    const float th = theta[i];
    delta[e] = th;
    beta[e] = ratio * th;
  }
}

// ---- object rotation: trilinear resampling of the sample volume into the lab stack

struct Rot {
  float m[9];              // sample offset = m * lab offset (row-major, axes a, y, z)
  float lp[3], sp[3];      // lab and sample pivots (nm)
  float ld[3], sd[3];      // lab and sample voxel pitch (nm)
  int ln[3], sn[3];        // lab and sample extents
};

__global__ void __launch_bounds__(256) k_rotate(Rot r, const float* __restrict__ ds, const float* __restrict__ bs,
                                                float* __restrict__ dl, float* __restrict__ bl) {
  const int64_t total = (int64_t)r.ln[0] * r.ln[1] * r.ln[2];
  const int64_t splane = (int64_t)r.sn[1] * r.sn[2];
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int l = (int)(e % r.ln[2]), j = (int)((e / r.ln[2]) % r.ln[1]), s = (int)(e / ((int64_t)r.ln[2] * r.ln[1]));
    const float u0 = s * r.ld[0] - r.lp[0], u1 = j * r.ld[1] - r.lp[1], u2 = l * r.ld[2] - r.lp[2];
    float q[3];
#pragma unroll
    for (int d = 0; d < 3; ++d)
      q[d] = (__builtin_fmaf(r.m[3 * d], u0, __builtin_fmaf(r.m[3 * d + 1], u1, r.m[3 * d + 2] * u2)) + r.sp[d]) / r.sd[d];
    int i0[3];
    float f[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const float fl = floorf(q[d]);
      i0[d] = (int)fl;
      f[d] = q[d] - fl;
    }
    float accd = 0.0f, accb = 0.0f;
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      const int ia = i0[0] + (c & 1), iy = i0[1] + ((c >> 1) & 1), iz = i0[2] + (c >> 2);
      if (ia < 0 || ia >= r.sn[0] || iy < 0 || iy >= r.sn[1] || iz < 0 || iz >= r.sn[2]) continue;
      const float w = ((c & 1) ? f[0] : 1.0f - f[0]) * (((c >> 1) & 1) ? f[1] : 1.0f - f[1]) * ((c >> 2) ? f[2] : 1.0f - f[2]);
      const int64_t o = ia * splane + (int64_t)iy * r.sn[2] + iz;
      accd = __builtin_fmaf(w, ds[o], accd);
      accb = __builtin_fmaf(w, bs[o], accb);
    }
    dl[e] = accd;
    bl[e] = accb;
  }
}

// ---- shrink-wrap: separable Gaussian blur of |theta|, global max, threshold mask

struct Blur {
  int n[3];          // box extents (a, y, z)
  int axis, radius;
  float w[64];       // normalised weights w[0 .. radius]
};

__global__ void __launch_bounds__(256) k_blur(Blur b, int take_abs, const float* __restrict__ in,
                                              float* __restrict__ out) {
  const int64_t total = (int64_t)b.n[0] * b.n[1] * b.n[2];
  const int64_t stride = b.axis == 0 ? (int64_t)b.n[1] * b.n[2] : (b.axis == 1 ? b.n[2] : 1);
  const int len = b.n[b.axis];
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int pos = (int)((e / stride) % len);
    float acc = 0.0f;
    for (int k = -b.radius; k <= b.radius; ++k) {
      const int q = pos + k;
      if (q < 0 || q >= len) continue;
      const float v = in[e + (int64_t)k * stride];
      acc = __builtin_fmaf(b.w[k < 0 ? -k : k], take_abs ? fabsf(v) : v, acc);
    }
    out[e] = acc;
  }
}

// per-block maxima, then one block over them (max is order-independent)
__global__ void __launch_bounds__(256) k_max_parts(int64_t n, const float* __restrict__ x, float* __restrict__ part) {
  __shared__ float red[256];
  float m = 0.0f;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
    m = fmaxf(m, x[e]);
  red[threadIdx.x] = m;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void __launch_bounds__(1024) k_max_final(int n, float* __restrict__ part) {
  __shared__ float red[1024];
  red[threadIdx.x] = (int)threadIdx.x < n ? part[threadIdx.x] : 0.0f;
  __syncthreads();
  for (int w = 512; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) part[1023] = red[0];   // the maximum, read by k_wrap
}

__global__ void __launch_bounds__(256) k_wrap(Box b, float ratio, float thr, const float* __restrict__ blurred,
                                              const float* __restrict__ part, float* __restrict__ theta,
                                              float* __restrict__ delta, float* __restrict__ beta) {
  const float cut = thr * part[1023];
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < b.n; i += (int64_t)gridDim.x * blockDim.x) {
    const float th = blurred[i] > cut ? theta[i] : 0.0f;
    const int64_t e = box_to_stack(b, i);
    theta[i] = th;
    delta[e] = th;
    beta[e] = ratio * th;
  }
}

struct Levels {
  float v[MSL_MAX_LEVELS];
  int n;
};

__global__ void __launch_bounds__(256) k_region_snap(Box b, float ratio, Levels lv, float* __restrict__ theta,
                                                     float* __restrict__ delta, float* __restrict__ beta) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < b.n; i += (int64_t)gridDim.x * blockDim.x) {
    const float th = theta[i];
    float best = lv.v[0], bd = fabsf(th - lv.v[0]);
    for (int l = 1; l < lv.n; ++l) {
      const float dl = fabsf(th - lv.v[l]);
      if (dl < bd) {
        bd = dl;
        best = lv.v[l];
      }
    }
    const int64_t e = box_to_stack(b, i);
    theta[i] = best;
    delta[e] = best;
    beta[e] = ratio * best;
  }
}

// c1 = 1 / (1 - beta1^t), c2 = 1 / (1 - beta2^t) (bias corrections, from the host)
__global__ void __launch_bounds__(256) k_region_adam(Box b, float ratio, msl_adam a, float c1, float c2, float gscale,
                                                     const float* __restrict__ gd, const float* __restrict__ gb,
                                                     float* __restrict__ theta, float* __restrict__ m,
                                                     float* __restrict__ v, float* __restrict__ delta,
                                                     float* __restrict__ beta) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < b.n; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t e = box_to_stack(b, i);
    const float g = gscale * __builtin_fmaf(ratio, gb[e], gd[e]);
    const float mi = __builtin_fmaf(a.beta1, m[i], (1.0f - a.beta1) * g);
    const float vi = __builtin_fmaf(a.beta2, v[i], (1.0f - a.beta2) * (g * g));
    const float step = a.lr * (mi * c1) / (sqrtf(vi * c2) + a.eps);
    const float th = fminf(fmaxf(theta[i] - step, a.lo), a.hi);
    m[i] = mi;
    v[i] = vi;
    theta[i] = th;
    delta[e] = th;
    beta[e] = ratio * th;
  }
}

msl_status check_region(const msl_geometry& g, const msl_region* r, Box& b) {
  if (!r) return fail(MSL_ERR_ARG, "region pointer is NULL");
  if (r->ns < 1 || r->ny < 1 || r->nz < 1) return fail(MSL_ERR_ARG, "region extents must be >= 1");
  if (r->s0 < 0 || r->y0 < 0 || r->z0 < 0 || (int64_t)r->s0 + r->ns > g.n_slices || (int64_t)r->y0 + r->ny > g.ny ||
      (int64_t)r->z0 + r->nz > g.nz)
    return fail(MSL_ERR_ARG, "region box outside the slice stack");
  if (!std::isfinite(r->beta_over_delta)) return fail(MSL_ERR_ARG, "beta_over_delta must be finite");
  b.s0 = r->s0;
  b.y0 = r->y0;
  b.z0 = r->z0;
  b.ny = r->ny;
  b.nz = r->nz;
  b.n = (int64_t)r->ns * r->ny * r->nz;
  b.gny = g.ny;
  b.gnz = g.nz;
  return MSL_OK;
}

unsigned elementwise_blocks(int64_t n) {
  const int64_t b = (n + 255) / 256;
  return (unsigned)(b < 65536 ? b : 65536);
}

}  // namespace

extern "C" {

msl_status msl_region_scatter(const msl_geometry* g, const msl_region* r, const float* theta, float* delta,
                              float* beta, void* hip_stream) {
  MSL_TRY(check_geometry(g));
  Box b;
  MSL_TRY(check_region(*g, r, b));
  MSL_TRY(check_ptr(theta, 4, "theta"));
  MSL_TRY(check_ptr(delta, 4, "delta"));
  MSL_TRY(check_ptr(beta, 4, "beta"));
  hipLaunchKernelGGL(k_region_scatter, dim3(elementwise_blocks(b.n)), dim3(256), 0,
                     static_cast<hipStream_t>(hip_stream), b, r->beta_over_delta, theta, delta, beta);
  return hip_check(hipGetLastError(), "scatter kernel");
}

msl_status msl_rotate_object(const msl_geometry* g, double lab_pivot_a_nm, double lab_pivot_y_nm,
                             double lab_pivot_z_nm, const msl_sample_grid* sg, double pitch_rad, double yaw_rad,
                             const float* delta_s, const float* beta_s, float* delta, float* beta,
                             void* hip_stream) {
  MSL_TRY(check_geometry(g));
  if (!sg) return fail(MSL_ERR_ARG, "sample grid pointer is NULL");
  if (sg->na < 1 || sg->ny < 1 || sg->nz < 1 || !finite_pos(sg->da_nm) || !finite_pos(sg->dy_nm) ||
      !finite_pos(sg->dz_nm))
    return fail(MSL_ERR_ARG, "sample grid: extents >= 1 and pitches > 0 required");
  if (!std::isfinite(pitch_rad) || !std::isfinite(yaw_rad) || !std::isfinite(lab_pivot_a_nm) ||
      !std::isfinite(lab_pivot_y_nm) || !std::isfinite(lab_pivot_z_nm) || !std::isfinite(sg->pivot_a_nm) ||
      !std::isfinite(sg->pivot_y_nm) || !std::isfinite(sg->pivot_z_nm))
    return fail(MSL_ERR_ARG, "angles and pivots must be finite");
  MSL_TRY(check_ptr(delta_s, 4, "delta_s"));
  MSL_TRY(check_ptr(beta_s, 4, "beta_s"));
  MSL_TRY(check_ptr(delta, 4, "delta"));
  MSL_TRY(check_ptr(beta, 4, "beta"));
  const double cp = std::cos(pitch_rad), sp = std::sin(pitch_rad), cw = std::cos(yaw_rad), sw = std::sin(yaw_rad);
  const double m[9] = {cp * cw, sp, -cp * sw, -sp * cw, cp, sp * sw, sw, 0.0, cw};
  Rot r{};
  for (int i = 0; i < 9; ++i) r.m[i] = (float)m[i];
  r.lp[0] = (float)lab_pivot_a_nm;
  r.lp[1] = (float)lab_pivot_y_nm;
  r.lp[2] = (float)lab_pivot_z_nm;
  r.sp[0] = (float)sg->pivot_a_nm;
  r.sp[1] = (float)sg->pivot_y_nm;
  r.sp[2] = (float)sg->pivot_z_nm;
  r.ld[0] = (float)g->dx_nm;
  r.ld[1] = (float)g->dy_nm;
  r.ld[2] = (float)g->dz_nm;
  r.sd[0] = (float)sg->da_nm;
  r.sd[1] = (float)sg->dy_nm;
  r.sd[2] = (float)sg->dz_nm;
  r.ln[0] = g->n_slices;
  r.ln[1] = g->ny;
  r.ln[2] = g->nz;
  r.sn[0] = sg->na;
  r.sn[1] = sg->ny;
  r.sn[2] = sg->nz;
  const int64_t total = (int64_t)g->n_slices * g->ny * g->nz;
  hipLaunchKernelGGL(k_rotate, dim3(elementwise_blocks(total)), dim3(256), 0, static_cast<hipStream_t>(hip_stream), r,
                     delta_s, beta_s, delta, beta);
  return hip_check(hipGetLastError(), "rotation kernel");
}

msl_status msl_region_shrinkwrap(const msl_geometry* g, const msl_region* r, float sigma_a, float sigma_y,
                                 float sigma_z, float threshold, float* theta, float* scratch, float* delta,
                                 float* beta, void* hip_stream) {
  MSL_TRY(check_geometry(g));
  Box bx;
  MSL_TRY(check_region(*g, r, bx));
  const float sig[3] = {sigma_a, sigma_y, sigma_z};
  for (int d = 0; d < 3; ++d)
    if (!(std::isfinite(sig[d]) && sig[d] >= 0.0f && sig[d] <= 20.0f))
      return fail(MSL_ERR_ARG, "shrink-wrap: sigmas must be in [0, 20] voxels");
  if (!(std::isfinite(threshold) && threshold >= 0.0f && threshold < 1.0f))
    return fail(MSL_ERR_ARG, "shrink-wrap: threshold must be in [0, 1)");
  MSL_TRY(check_ptr(theta, 4, "theta"));
  MSL_TRY(check_ptr(scratch, 4, "scratch"));
  MSL_TRY(check_ptr(delta, 4, "delta"));
  MSL_TRY(check_ptr(beta, 4, "beta"));
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  float* b0 = scratch;
  float* b1 = scratch + bx.n;
  float* part = scratch + 2 * bx.n;
  const unsigned blocks = elementwise_blocks(bx.n);
  const float* src = theta;
  float* dst = b0;
  for (int d = 0; d < 3; ++d) {
    Blur bl{};
    bl.n[0] = r->ns;
    bl.n[1] = r->ny;
    bl.n[2] = r->nz;
    bl.axis = d;
    bl.radius = (int)(3.0f * sig[d] + 0.5f);
    double wsum = 0.0, w[64];
    for (int k = 0; k <= bl.radius; ++k) {
      w[k] = sig[d] > 0.0f ? std::exp(-0.5 * (double)k * k / ((double)sig[d] * sig[d])) : (k == 0 ? 1.0 : 0.0);
      wsum += k == 0 ? w[k] : 2.0 * w[k];
    }
    for (int k = 0; k <= bl.radius; ++k) bl.w[k] = (float)(w[k] / wsum);
    hipLaunchKernelGGL(k_blur, dim3(blocks), dim3(256), 0, st, bl, d == 0 ? 1 : 0, src, dst);
    src = dst;
    dst = dst == b0 ? b1 : b0;
  }
  const unsigned mparts = blocks < 1023 ? blocks : 1023;
  hipLaunchKernelGGL(k_max_parts, dim3(mparts), dim3(256), 0, st, bx.n, src, part);
  hipLaunchKernelGGL(k_max_final, dim3(1), dim3(1024), 0, st, (int)mparts, part);
  hipLaunchKernelGGL(k_wrap, dim3(blocks), dim3(256), 0, st, bx, r->beta_over_delta, threshold, src, part, theta, delta,
                     beta);
  return hip_check(hipGetLastError(), "shrink-wrap kernels");
}

msl_status msl_region_snap(const msl_geometry* g, const msl_region* r, const float* levels, int32_t n_levels,
                           float* theta, float* delta, float* beta, void* hip_stream) {
  MSL_TRY(check_geometry(g));
  Box b;
  MSL_TRY(check_region(*g, r, b));
  if (!levels || n_levels < 1 || n_levels > MSL_MAX_LEVELS)
    return fail(MSL_ERR_ARG, "levels: need 1 <= n_levels <= " + std::to_string(MSL_MAX_LEVELS) + " values");
  Levels lv{};
  lv.n = n_levels;
  for (int l = 0; l < n_levels; ++l) {
    if (!std::isfinite(levels[l])) return fail(MSL_ERR_ARG, "levels must be finite");
    lv.v[l] = levels[l];
  }
  MSL_TRY(check_ptr(theta, 4, "theta"));
  MSL_TRY(check_ptr(delta, 4, "delta"));
  MSL_TRY(check_ptr(beta, 4, "beta"));
  hipLaunchKernelGGL(k_region_snap, dim3(elementwise_blocks(b.n)), dim3(256), 0, static_cast<hipStream_t>(hip_stream),
                     b, r->beta_over_delta, lv, theta, delta, beta);
  return hip_check(hipGetLastError(), "snap kernel");
}

msl_status msl_region_adam_step(const msl_geometry* g, const msl_region* r, const msl_adam* a, int32_t t,
                                float grad_scale, const float* grad_delta, const float* grad_beta, float* theta,
                                float* m, float* v, float* delta, float* beta, void* hip_stream) {
  MSL_TRY(check_geometry(g));
  Box b;
  MSL_TRY(check_region(*g, r, b));
  if (!a) return fail(MSL_ERR_ARG, "adam parameter pointer is NULL");
  if (!(std::isfinite(a->lr) && a->lr >= 0) || !(a->beta1 >= 0 && a->beta1 < 1) || !(a->beta2 >= 0 && a->beta2 < 1) ||
      !(std::isfinite(a->eps) && a->eps > 0) || std::isnan(a->lo) || std::isnan(a->hi) || !(a->lo <= a->hi))
    return fail(MSL_ERR_ARG, "adam parameters: need lr >= 0, 0 <= beta1, beta2 < 1, eps > 0, lo <= hi");
  if (t < 1) return fail(MSL_ERR_ARG, "adam step count t must be >= 1");
  if (!std::isfinite(grad_scale)) return fail(MSL_ERR_ARG, "grad_scale must be finite");
  MSL_TRY(check_ptr(grad_delta, 4, "grad_delta"));
  MSL_TRY(check_ptr(grad_beta, 4, "grad_beta"));
  MSL_TRY(check_ptr(theta, 4, "theta"));
  MSL_TRY(check_ptr(m, 4, "m"));
  MSL_TRY(check_ptr(v, 4, "v"));
  MSL_TRY(check_ptr(delta, 4, "delta"));
  MSL_TRY(check_ptr(beta, 4, "beta"));
  const float c1 = (float)(1.0 / (1.0 - std::pow((double)a->beta1, (double)t)));
  const float c2 = (float)(1.0 / (1.0 - std::pow((double)a->beta2, (double)t)));
  hipLaunchKernelGGL(k_region_adam, dim3(elementwise_blocks(b.n)), dim3(256), 0, static_cast<hipStream_t>(hip_stream),
                     b, r->beta_over_delta, *a, c1, c2, grad_scale, grad_delta, grad_beta, theta, m, v, delta, beta);
  return hip_check(hipGetLastError(), "adam kernel");
}

}  // extern "C"

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

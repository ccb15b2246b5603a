// Host-side helpers shared by the libmsl translation units: the thread-local
// error text behind msl_last_error, argument checks and the HIP status check.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <string>

#include "msl.h"

namespace msl_host {

inline thread_local std::string g_last_error;

inline msl_status fail(msl_status s, const std::string& msg) {
  g_last_error = msg;
  return s;
}

inline bool is_pow2_in(int n, int lo, int hi) { return n >= lo && n <= hi && (n & (n - 1)) == 0; }
inline bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }
inline bool aligned(const void* p, size_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }

inline msl_status check_geometry(const msl_geometry* g) {
  if (!g) return fail(MSL_ERR_ARG, "geometry pointer is NULL");
  if (!is_pow2_in(g->ny, 16, 1024) || !is_pow2_in(g->nz, 16, 1024))
    return fail(MSL_ERR_ARG, "ny and nz must be powers of two in [16, 1024], got " + std::to_string(g->ny) + " x " +
                                 std::to_string(g->nz));
  if (g->n_slices < 1) return fail(MSL_ERR_ARG, "n_slices must be >= 1");
  if (!finite_pos(g->dy_nm) || !finite_pos(g->dz_nm)) return fail(MSL_ERR_ARG, "dy_nm and dz_nm must be finite and > 0");
  if (!finite_pos(g->dx_nm)) return fail(MSL_ERR_ARG, "dx_nm must be finite and > 0");
  if (!finite_pos(g->wavelength_nm)) return fail(MSL_ERR_ARG, "wavelength_nm must be finite and > 0");
  if (!std::isfinite(g->alpha_i_rad) || std::fabs(g->alpha_i_rad) >= M_PI / 2)
    return fail(MSL_ERR_ARG, "alpha_i_rad must be finite with |alpha| < pi/2");
  if (g->propagator != MSL_PROP_PARAXIAL && g->propagator != MSL_PROP_EXACT)
    return fail(MSL_ERR_ARG, "propagator must be MSL_PROP_PARAXIAL (0) or MSL_PROP_EXACT (1)");
  return MSL_OK;
}

inline msl_status check_ptr(const void* p, size_t align, const char* name, bool allow_null = false) {
  if (!p) return allow_null ? MSL_OK : fail(MSL_ERR_ARG, std::string(name) + " is NULL");
  if (!aligned(p, align)) return fail(MSL_ERR_ARG, std::string(name) + " is not " + std::to_string(align) + "-byte aligned");
  return MSL_OK;
}

inline msl_status hip_check(hipError_t e, const char* what) {
  if (e != hipSuccess) return fail(MSL_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
  return MSL_OK;
}

}  // namespace msl_host

#define MSL_TRY(expr)            \
  do {                           \
    msl_status _s = (expr);      \
    if (_s != MSL_OK) return _s; \
  } while (0)

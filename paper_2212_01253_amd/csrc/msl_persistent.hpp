// Persistent schedule: one cooperative launch runs every pass of a phase,
// with a device-wide barrier between passes.
//
// Each pass is an all-to-all dependency (a column needs every row of the
// previous pass), so a barrier per pass is the minimum synchronisation.  A
// kernel launch per pass costs a launch, a drain and a ramp-up; a barrier
// inside one resident grid costs one round of agent-scope atomics.  Grid
// size is capped by what is co-resident (hipLaunchCooperativeKernel refuses
// anything larger), so every block that waits at a barrier is running.
//
// Barrier: a monotonic arrival counter in the workspace, zeroed by a small
// kernel before the launch.  Every wave releases its stores at agent scope
// (the XCDs' L2 caches are not coherent with each other), one thread per
// block adds its arrival and spins with s_sleep until all blocks of this
// pass have arrived, then every wave acquires.  The spin is bounded: after
// kSpinLimit polls it sets an error word and stops waiting, in this and
// every later barrier, so the grid always drains.
#pragma once

#include "msl_passes.hpp"

namespace msl {

constexpr unsigned kSpinLimit = 1u << 22;

__device__ __forceinline__ void grid_barrier(unsigned* bar, unsigned target) {
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) {
    __hip_atomic_fetch_add(bar, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    unsigned spins = 0;
    while (__hip_atomic_load(bar, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
      if (__hip_atomic_load(bar + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u) break;
      __builtin_amdgcn_s_sleep(1);
      if (++spins > kSpinLimit) {
        __hip_atomic_fetch_or(bar + 1, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        break;
      }
    }
  }
  __syncthreads();
  __threadfence();
}

// Lines of one pass handled by one block per round, and block size.
template <int N>
struct PersistShape {
  static constexpr int L = N / 8;
  static constexpr int T0 = N >= 1024 ? 256 : (N >= 512 ? 128 : 64);
  static constexpr int T = T0 < N * L ? T0 : N * L;  // at most N lines per block
  static constexpr int G = T / L;
  static constexpr int LDS = G * (N + N / 8);
};

template <int N>
__global__ void __launch_bounds__(256) k_persist(Ctx c, PhaseSpec ph, int np, unsigned* bar, int rounds) {
  using S = PersistShape<N>;
  __shared__ float2 lds[S::LDS];
  const int g = threadIdx.x / S::L, j = threadIdx.x % S::L;
  const int nb = gridDim.x;
  const int bid = xcd_group(blockIdx.x, nb);
  float2* sh = lds + g * (N + N / 8);
  unsigned target = 0;
  for (int p = 0; p < np; ++p) {
    const PassDesc pd = phase_pass(ph, p);
    for (int r = 0; r < rounds; ++r) {
      const int line = (r * nb + bid) * S::G + g;
      LineIn<N> in;
      if (pd.axis == ROW) {
        load_field<N, ROW>(c, pd, line, j, in);
        load_static<N, ROW>(c, pd, line, j, in);
        compute_line<N, ROW>(c, pd, line, j, sh, in);
      } else {
        load_field<N, COL>(c, pd, line, j, in);
        load_static<N, COL>(c, pd, line, j, in);
        compute_line<N, COL>(c, pd, line, j, sh, in);
      }
    }
    if (p + 1 < np) {
      target += (unsigned)nb;
      grid_barrier(bar, target);
    }
  }
}

__global__ void k_zero_words(unsigned* p, int n) {
  const int i = threadIdx.x;
  if (i < n) p[i] = 0u;
}

// The persistent schedule serves square grids (both pass axes have the same
// line length and line count); long phases profit most.
inline bool persistent_preferred(const Ctx& c, int np) { return false && c.ny == c.nz && np >= 8; }

struct PersistLaunch {
  int grid = 0, block = 0, rounds = 0;
};

template <int N>
hipError_t persist_shape(PersistLaunch& pl) {
  using S = PersistShape<N>;
  static int max_blocks = -1;  // co-resident blocks on this device (cached per process)
  if (max_blocks < 0) {
    int dev = 0, per_cu = 0;
    hipDeviceProp_t prop;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    e = hipGetDeviceProperties(&prop, dev);
    if (e != hipSuccess) return e;
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_persist<N>, S::T, 0);
    if (e != hipSuccess) return e;
    max_blocks = per_cu * prop.multiProcessorCount;
  }
  const int groups = N / S::G;  // line groups per pass (square grid: N lines)
  int grid = 1;
  while (grid * 2 <= groups && grid * 2 <= max_blocks) grid *= 2;
  if (grid < 1 || max_blocks < 1) return hipErrorCooperativeLaunchTooLarge;
  pl.grid = grid;
  pl.block = S::T;
  pl.rounds = groups / grid;
  return hipSuccess;
}

template <int N>
hipError_t launch_persistent_n(const Ctx& c, const PhaseSpec& ph, int np, unsigned* bar, hipStream_t st) {
  PersistLaunch pl;
  hipError_t e = persist_shape<N>(pl);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_zero_words, dim3(1), dim3(64), 0, st, bar, 64);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  Ctx cc = c;
  PhaseSpec pp = ph;
  int npp = np, rr = pl.rounds;
  void* args[] = {&cc, &pp, &npp, &bar, &rr};
  return hipLaunchCooperativeKernel(reinterpret_cast<const void*>(&k_persist<N>), dim3(pl.grid), dim3(pl.block),
                                    args, 0, st);
}

inline hipError_t launch_persistent(const Ctx& c, const PhaseSpec& ph, int np, unsigned* bar, hipStream_t st) {
  if (c.ny != c.nz) return hipErrorNotSupported;
  switch (c.ny) {
    case 16: return launch_persistent_n<16>(c, ph, np, bar, st);
    case 32: return launch_persistent_n<32>(c, ph, np, bar, st);
    case 64: return launch_persistent_n<64>(c, ph, np, bar, st);
    case 128: return launch_persistent_n<128>(c, ph, np, bar, st);
    case 256: return launch_persistent_n<256>(c, ph, np, bar, st);
    case 512: return launch_persistent_n<512>(c, ph, np, bar, st);
    case 1024: return launch_persistent_n<1024>(c, ph, np, bar, st);
    default: return hipErrorNotSupported;
  }
}

}  // namespace msl

// Persistent schedule: one cooperative launch runs every pass of a phase (or
// of two independent phases side by side), with a device-wide barrier
// between passes.
//
// Each pass is an all-to-all dependency (a column needs every row of the
// previous pass), so one barrier per pass is the minimum synchronisation.
// Grid size is capped by what is co-resident (hipLaunchCooperativeKernel
// refuses anything larger), so every block that waits at a barrier runs.
//
// Exchange and barrier.  The per-XCD L2 caches are not coherent with each
// other, and an agent-scope release fence writes back a whole L2, which
// costs more than the pass itself.  Instead, the field that passes hand to
// each other is written and read with device-coherent (agent-scope atomic)
// accesses, and the barrier only has to order them: every wave waits for
// its own stores to complete, then each block publishes the barrier epoch
// in its own flag word, and every block polls all flags.  No counter is
// shared, so arrivals do not serialise on one address.  Other outputs
// (checkpoints, segment fields, gradients) are read only by later kernels.
// The wait is bounded: after `spin_limit` polls a block raises an error word
// and stops waiting, in this and every later barrier, so the grid always
// drains.  After the launch a fold kernel turns a raised error word into the
// workspace's status word (which msl_workspace_status reports) and overwrites
// the phase's working fields with NaN, so a result computed across a barrier
// that gave up cannot pass for a valid one.
//
// Barrier area (unsigned words at the start of the workspace): [0] error word
// of the current launch, [1] status word of the current call, [8 ...] one flag
// per block.
#pragma once

#include "msl_passes.hpp"

namespace msl {

constexpr unsigned kDefaultSpinLimit = 1u << 22;
constexpr int kMaxFlags = 2040;  // flag words after the first eight words of the barrier area

__device__ __forceinline__ void grid_barrier(unsigned* bar, unsigned epoch, int nb, unsigned spin_limit) {
  unsigned* err = bar;
  unsigned* flags = bar + 8;
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __builtin_amdgcn_s_waitcnt(0);  // this wave's stores have completed
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __syncthreads();
  if (threadIdx.x == 0) __hip_atomic_store(flags + blockIdx.x, epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  unsigned spins = 0;
  for (;;) {
    int ok = 1;
    for (int t = threadIdx.x; t < nb; t += blockDim.x)
      ok &= __hip_atomic_load(flags + t, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= epoch;
    const int errd = threadIdx.x == 0 && __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u;
    if (__syncthreads_and(ok) || __syncthreads_or(errd)) break;
    if (++spins > spin_limit) {
      if (threadIdx.x == 0) __hip_atomic_store(err, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      break;
    }
    __builtin_amdgcn_s_sleep(2);
  }
}

// Block size and lines per block of one field (neighbouring lines, which
// share the tiles of the working field).
template <int N>
struct PersistShape {
  static constexpr int L = LinePts<N>::L;
  static constexpr int T0 = N >= 1024 ? 256 : 128;
  static constexpr int T = T0 < N * L ? T0 : N * L;  // at most N lines per block
  static constexpr int G = T / L;
  static constexpr int LDS = 2 * G * line_lds<N>();  // two exchange buffers per line
};

// Blocks [0, nbA) run phase A, blocks [nbA, gridDim.x) run phase B (if npB > 0).
template <int N>
__global__ void __launch_bounds__(256) k_persist(Ctx c, PhaseSpec A, PhaseSpec B, int npA, int npB, int nbA,
                                                 unsigned* bar, int rounds, unsigned spin_limit) {
  using S = PersistShape<N>;
  __shared__ float2 lds[S::LDS];
  const int g = threadIdx.x % S::G, j = threadIdx.x / S::G;
  const bool second = (int)blockIdx.x >= nbA;
  const PhaseSpec ph = second ? B : A;
  const int np_mine = second ? npB : npA;
  const int np_all = npA > npB ? npA : npB;
  const int nb = second ? (int)gridDim.x - nbA : nbA;
  const int bid = xcd_group(second ? (int)blockIdx.x - nbA : (int)blockIdx.x, nb);
  const LineLds sh{lds + g * line_lds<N>(), lds + (S::G + g) * line_lds<N>()};
  for (int p = 0; p < np_all; ++p) {
    if (p < np_mine) {
      const PassDesc pd = phase_pass(ph, p);
      for (int r = 0; r < rounds; ++r) run_line_any<N, true>(c, pd, (r * nb + bid) * S::G + g, j, sh);
    }
    if (p + 1 < np_all) grid_barrier(bar, (unsigned)(p + 1), (int)gridDim.x, spin_limit);
  }
}

// Clears the error word and the first n flags (not the status word).
__global__ void k_reset_barrier(unsigned* bar, int n) {
  if (threadIdx.x == 0) bar[0] = 0u;
  for (int i = threadIdx.x; i < n; i += blockDim.x) bar[8 + i] = 0u;
}

// Clears the status word (start of a call that may run persistent phases).
__global__ void k_clear_status(unsigned* bar) {
  if (threadIdx.x == 0 && blockIdx.x == 0) bar[1] = 0u;
}

// After a persistent launch: if a barrier gave up, raise the status word and
// fill the up to four working fields of m elements with NaN.
__global__ void k_fold_barrier_error(unsigned* bar, float2* f0, float2* f1, float2* f2, float2* f3, int64_t m) {
  if (__hip_atomic_load(bar, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0u) return;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0) bar[1] = 1u;
  if (i >= m) return;
  const float q = __builtin_nanf("");
  if (f0) f0[i] = make_float2(q, q);
  if (f1) f1[i] = make_float2(q, q);
  if (f2) f2[i] = make_float2(q, q);
  if (f3) f3[i] = make_float2(q, q);
}

// The persistent schedule serves square grids (both pass axes have the same
// line length and line count).
inline bool persistent_preferred(const Ctx& c, int np) { return false && c.ny == c.nz && np >= 8; }

struct PersistLaunch {
  int grid = 0, block = 0, rounds = 0;
};

// Blocks per field: the largest power of two <= line groups that fits
// `fields` times in the co-resident limit.
template <int N>
hipError_t persist_shape(PersistLaunch& pl, int fields) {
  using S = PersistShape<N>;
  static int max_blocks = -1;  // co-resident blocks on the current device (cached per process)
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
  const int groups = N / S::G;
  const int cap = max_blocks / fields;
  if (cap < 1) return hipErrorCooperativeLaunchTooLarge;
  int grid = 1;
  while (grid * 2 <= groups && grid * 2 <= cap && grid * 2 * fields <= kMaxFlags) grid *= 2;
  pl.grid = grid;
  pl.block = S::T;
  pl.rounds = groups / grid;
  return hipSuccess;
}

template <int N>
hipError_t launch_persistent_n(const Ctx& c, const PhaseSpec& a, int npa, const PhaseSpec* b, int npb,
                               unsigned* bar, unsigned spin_limit, hipStream_t st) {
  const int fields = (b && npb > 0) ? 2 : 1;
  PersistLaunch pl;
  hipError_t e = persist_shape<N>(pl, fields);
  if (e != hipSuccess) return e;
  const int total = pl.grid * fields;
  hipLaunchKernelGGL(k_reset_barrier, dim3(1), dim3(256), 0, st, bar, total);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  Ctx cc = c;
  PhaseSpec pa = a, pb = fields == 2 ? *b : a;
  int npa_ = npa, npb_ = fields == 2 ? npb : 0, nba = pl.grid, rr = pl.rounds;
  unsigned sl = spin_limit;
  void* args[] = {&cc, &pa, &pb, &npa_, &npb_, &nba, &bar, &rr, &sl};
  e = hipLaunchCooperativeKernel(reinterpret_cast<const void*>(&k_persist<N>), dim3(total), dim3(pl.block), args,
                                 0, st);
  if (e != hipSuccess) return e;
  const int64_t m = c.m;
  hipLaunchKernelGGL(k_fold_barrier_error, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, st, bar, pa.field,
                     pa.out_rm, fields == 2 ? pb.field : nullptr, fields == 2 ? pb.out_rm : nullptr, m);
  return hipGetLastError();
}

// Runs phase a (and phase b beside it, if given) as one cooperative launch.
inline hipError_t launch_persistent(const Ctx& c, const PhaseSpec& a, int npa, const PhaseSpec* b, int npb,
                                    unsigned* bar, unsigned spin_limit, hipStream_t st) {
  if (c.ny != c.nz) return hipErrorNotSupported;
  switch (c.ny) {
    case 16: return launch_persistent_n<16>(c, a, npa, b, npb, bar, spin_limit, st);
    case 32: return launch_persistent_n<32>(c, a, npa, b, npb, bar, spin_limit, st);
    case 64: return launch_persistent_n<64>(c, a, npa, b, npb, bar, spin_limit, st);
    case 128: return launch_persistent_n<128>(c, a, npa, b, npb, bar, spin_limit, st);
    case 256: return launch_persistent_n<256>(c, a, npa, b, npb, bar, spin_limit, st);
    case 512: return launch_persistent_n<512>(c, a, npa, b, npb, bar, spin_limit, st);
    case 1024: return launch_persistent_n<1024>(c, a, npa, b, npb, bar, spin_limit, st);
    default: return hipErrorNotSupported;
  }
}

}  // namespace msl

// Host-only check of the pass programs (msl_passes.hpp).
//
// Executes the PassDesc sequences that the library launches, with a plain
// FP64 line engine (naive DFTs, exact propagator factors and transmission),
// and compares the results with direct 2-D evaluations of the same
// quantities.  This tests the scheduling logic (pass order, axis alternation,
// checkpoint and segment slots, reverse indexing, the constants' cycle
// positions) without a GPU; the GPU kernels are checked separately against
// the oracle.
//
// Build: hipcc --offload-host-only -std=c++17 -I include -o schedule_check schedule_check.cpp
// Run:   ./schedule_check   (prints "OK" and exits 0 on success)
#include <complex>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "msl_passes.hpp"

using cd = std::complex<double>;
using Field = std::vector<cd>;

namespace {

struct Geo {
  int ny, nz, ns;
  double dy, dz, dx, lam;
  bool exact;
};

double kf(int m, int n, double d) {
  const int f = m < n / 2 ? m : m - n;
  return 2 * M_PI * f / (n * d);
}

cd hpar(int m, int n, double d, const Geo& g) {
  const double k = 2 * M_PI / g.lam, q = kf(m, n, d);
  return std::polar(1.0, g.dx * q * q / (2 * k));
}

// Stand-in for the cycle of single-float32 constants of the paraxial passes:
// the engine multiplies the one-axis propagator factor of a pass at cycle
// position t by a small phase that depends on t, the axis and the frequency,
// and the direct references apply the factor that the slice calls for (its
// pass along each axis advances one position every two slices).  A pass with
// another position than its slice's, or a recompute or reverse pass whose
// position differs from the forward's, then changes the results.
cd tabmod(int t, int axis, int i) { return std::polar(1.0, 1e-3 * (t + 1) * (axis + 2) * (1 + i % 3)); }

int slice_tab(int q) { return q / 2 % msl::DITHER; }

cd hexact(int my, int mz, const Geo& g) {
  const double k = 2 * M_PI / g.lam, ky = kf(my, g.ny, g.dy), kz = kf(mz, g.nz, g.dz);
  const double kp2 = ky * ky + kz * kz;
  return std::polar(1.0, g.dx * kp2 / (k + std::sqrt(k * k - kp2)));
}

// 1-D DFT of a line, sign -1 forward, +1 inverse (unnormalised)
std::vector<cd> dft(const std::vector<cd>& x, int sign) {
  const int n = (int)x.size();
  std::vector<cd> y(n);
  for (int u = 0; u < n; ++u) {
    cd s = 0;
    for (int j = 0; j < n; ++j) s += x[j] * std::polar(1.0, sign * 2 * M_PI * double(u) * j / n);
    y[u] = s;
  }
  return y;
}

struct Engine {
  Geo g;
  std::vector<float> delta, beta;      // [ns][ny][nz]
  std::vector<double> gdelta, gbeta;
  std::vector<float> gI;               // shifted
  std::vector<double> inten;           // shifted
  // device pointers are stand-ins: map float2* tags to host fields
  std::vector<Field*> bufs;
  std::vector<const float2*> tags;

  Field* buf(const float2* p) {
    for (size_t i = 0; i < tags.size(); ++i)
      if (tags[i] == p) return bufs[i];
    // pointer inside a registered array of fields (ckpt / seg)
    return nullptr;
  }
};

struct Arr {
  std::vector<Field> f;
  const float2* base;
  int64_t m;
  Field* at(const float2* p) {
    const int64_t off = p - base;
    if (off < 0 || off % m) return nullptr;
    const int64_t i = off / m;
    if (i >= (int64_t)f.size()) return nullptr;
    return &f[i];
  }
};

std::vector<Arr*> g_arrays;

Field* resolve(const float2* p) {
  for (Arr* a : g_arrays)
    if (Field* f = a->at(p)) return f;
  std::fprintf(stderr, "unresolved pointer\n");
  std::exit(3);
}

cd tfun(const Engine& E, int s, int64_t e) {
  const double k = 2 * M_PI / E.g.lam;
  const int64_t m = (int64_t)E.g.ny * E.g.nz;
  return std::exp(cd(0, 1) * k * E.g.dx * cd(E.delta[s * m + e], E.beta[s * m + e]));
}

int g_bad_layout = 0;

void run_pass(Engine& E, const msl::PassDesc& pd) {
  const Geo& g = E.g;
  const int64_t m = (int64_t)g.ny * g.nz;
  const bool row = pd.axis == msl::ROW;
  const int nl = row ? g.ny : g.nz, n = row ? g.nz : g.ny;
  Field* src = resolve(pd.src);
  Field* dst = pd.dst ? resolve(pd.dst) : nullptr;
  // a pass may rewrite its own lines in place, but never read one layout of a
  // buffer while writing the other (other lines would be overwritten)
  if (dst == src && pd.dst_lay != pd.src_lay) ++g_bad_layout;
  if ((pd.src_lay != msl::LAY_R && pd.src_lay != msl::LAY_T) || (pd.dst && pd.dst_lay != msl::LAY_R &&
                                                                 pd.dst_lay != msl::LAY_T))
    ++g_bad_layout;
  // fields in column tile order are only ever touched by column passes
  if ((pd.psi_store && pd.store_lay == msl::LAY_C && row) || (pd.psi_load && pd.load_lay == msl::LAY_C && row))
    ++g_bad_layout;
  const double k = 2 * M_PI / g.lam;
  for (int line = 0; line < nl; ++line) {
    auto addr = [&](int i) -> int64_t { return row ? (int64_t)line * g.nz + i : (int64_t)i * g.nz + line; };
    // row-major, or the 2x2-tiled layout of the library's working fields (the
    // same index map as msl::tile_addr, written out here on its own)
    auto laddr = [&](int lay, int i) -> int64_t {
      const int64_t y = row ? line : i, z = row ? i : line;
      if (lay == msl::LAY_T) return ((y / 2) * (g.nz / 2) + z / 2) * 4 + (y % 2) * 2 + z % 2;
      if (lay == msl::LAY_C) return ((z / 2) * (g.ny / 2) + y / 2) * 4 + (y % 2) * 2 + z % 2;
      return y * g.nz + z;
    };
    std::vector<cd> v(n);
    for (int i = 0; i < n; ++i) v[i] = (*src)[laddr(pd.src_lay, i)];
    auto prop = [&](bool conj) {
      v = dft(v, -1);
      for (int i = 0; i < n; ++i) {
        cd h = (row ? hpar(i, g.nz, g.dz, g) : hpar(i, g.ny, g.dy, g)) * tabmod(pd.tab, pd.axis, i);
        v[i] *= (conj ? std::conj(h) : h) / double(n);
      }
      v = dft(v, +1);
    };
    switch (pd.pre) {
      case msl::PRE_PROP: prop(pd.conj); break;
      case msl::PRE_FFT: v = dft(v, -1); break;
      case msl::PRE_IFFT_N: v = dft(v, +1); for (auto& x : v) x /= double(n); break;
      case msl::PRE_IFFT_U: v = dft(v, +1); break;
      default: break;
    }
    if (pd.psi_store) {
      Field* st = resolve(pd.psi_store);
      for (int i = 0; i < n; ++i) (*st)[laddr(pd.store_lay, i)] = v[i];
    }
    if (pd.mid == msl::MID_T_FWD) {
      for (int i = 0; i < n; ++i) v[i] *= tfun(E, pd.slice, addr(i));
    } else if (pd.mid == msl::MID_T_ADJ) {
      Field* ps = resolve(pd.psi_load);
      for (int i = 0; i < n; ++i) {
        const cd T = tfun(E, pd.slice, addr(i));
        const cd pt = T * (*ps)[laddr(pd.load_lay, i)];
        const cd c = std::conj(v[i]) * pt;
        E.gdelta[pd.slice * m + addr(i)] = -k * g.dx * c.imag();
        E.gbeta[pd.slice * m + addr(i)] = -k * g.dx * c.real();
        v[i] *= std::conj(T);
      }
    } else if (pd.mid == msl::MID_FF_OUT || pd.mid == msl::MID_FF_SEED) {
      for (int i = 0; i < n; ++i) {
        const int r = row ? line : i, c = row ? i : line;
        const int64_t sidx = (int64_t)((r + g.ny / 2) % g.ny) * g.nz + (c + g.nz / 2) % g.nz;
        if (pd.mid == msl::MID_FF_OUT) E.inten[sidx] = std::norm(v[i]) / double(m);
        else v[i] *= 2.0 * E.gI[sidx] / double(m);
      }
    }
    switch (pd.post) {
      case msl::POST_PROP: prop(pd.conj); break;
      case msl::POST_FFT: v = dft(v, -1); break;
      case msl::POST_PROP2D:
        v = dft(v, -1);
        for (int i = 0; i < n; ++i) {
          const cd h = hexact(i, line, g) / double(g.ny);
          v[i] *= pd.conj ? std::conj(h) : h;
        }
        v = dft(v, +1);
        break;
      default: break;
    }
    if (dst)
      for (int i = 0; i < n; ++i) (*dst)[laddr(pd.dst_lay, i)] = v[i];
  }
}

void run_phase(Engine& E, const msl::PhaseSpec& ph) {
  const int np = msl::phase_npasses(ph);
  for (int p = 0; p < np; ++p) run_pass(E, msl::phase_pass(ph, p));
}

// --- direct 2-D references
Field dft2(const Field& x, const Geo& g, int sign) {
  Field y = x;
  for (int r = 0; r < g.ny; ++r) {
    std::vector<cd> v(y.begin() + (int64_t)r * g.nz, y.begin() + (int64_t)(r + 1) * g.nz);
    v = dft(v, sign);
    std::copy(v.begin(), v.end(), y.begin() + (int64_t)r * g.nz);
  }
  for (int c = 0; c < g.nz; ++c) {
    std::vector<cd> v(g.ny);
    for (int r = 0; r < g.ny; ++r) v[r] = y[(int64_t)r * g.nz + c];
    v = dft(v, sign);
    for (int r = 0; r < g.ny; ++r) y[(int64_t)r * g.nz + c] = v[r];
  }
  return y;
}

cd H2(int my, int mz, const Geo& g) {
  return g.exact ? hexact(my, mz, g) : hpar(my, g.ny, g.dy, g) * hpar(mz, g.nz, g.dz, g);
}

Field prop2(const Field& x, const Geo& g, bool conj) {
  Field y = dft2(x, g, -1);
  const double m = double(g.ny) * g.nz;
  for (int r = 0; r < g.ny; ++r)
    for (int c = 0; c < g.nz; ++c) {
      cd h = H2(r, c, g);
      y[(int64_t)r * g.nz + c] *= (conj ? std::conj(h) : h) / m;
    }
  return dft2(y, g, +1);
}

// Paraxial propagation between the transmissions of slices s and s + 1 (s =
// ns - 1: after the last): the second half of the pass of slice s and the
// first half of the pass of slice s + 1, one along each axis, each with the
// cycle factor of its own pass.
Field prop_slice(const Field& x, const Geo& g, int s, bool conj) {
  if (g.exact) return prop2(x, g, conj);
  const int qr = (s % 2 == 0) ? s : s + 1, qc = (s % 2 == 1) ? s : s + 1;  // row pass: even slice
  Field y = dft2(x, g, -1);
  const double m = double(g.ny) * g.nz;
  for (int r = 0; r < g.ny; ++r)
    for (int c = 0; c < g.nz; ++c) {
      const cd h = H2(r, c, g) * tabmod(slice_tab(qr), msl::ROW, c) * tabmod(slice_tab(qc), msl::COL, r);
      y[(int64_t)r * g.nz + c] *= (conj ? std::conj(h) : h) / m;
    }
  return dft2(y, g, +1);
}

// Per axis, the forward phase's passes must take consecutive cycle positions
// (one step per pass of that axis, wrapping at DITHER) from 0.
int check_tab_sequence(const msl::PhaseSpec& ph) {
  int next[2] = {0, 0};
  for (int p = 0; p < msl::phase_npasses(ph); ++p) {
    const msl::PassDesc d = msl::phase_pass(ph, p);
    if (d.tab != next[d.axis]) {
      std::printf("pass %d (axis %d) at cycle position %d, expected %d\n", p, d.axis, d.tab, next[d.axis]);
      return 1;
    }
    next[d.axis] = (next[d.axis] + 1) % msl::DITHER;
  }
  return 0;
}

double rel(const Field& a, const Field& b) {
  double n = 0, d = 0;
  for (size_t i = 0; i < a.size(); ++i) { n += std::norm(a[i] - b[i]); d += std::norm(b[i]); }
  return std::sqrt(n / d);
}

double relv(const std::vector<double>& a, const std::vector<double>& b) {
  double n = 0, d = 0;
  for (size_t i = 0; i < a.size(); ++i) { n += (a[i] - b[i]) * (a[i] - b[i]); d += b[i] * b[i]; }
  return std::sqrt(n / d);
}

int check(const Geo& g, int kck) {
  const int64_t m = (int64_t)g.ny * g.nz;
  std::mt19937_64 rng(12345 + g.ny * 7 + g.nz + g.ns + kck + (g.exact ? 1000 : 0));
  std::uniform_real_distribution<double> U(0, 1);
  Engine E;
  E.g = g;
  E.delta.resize(g.ns * m);
  E.beta.resize(g.ns * m);
  for (auto& x : E.delta) x = float(U(rng) * 2e-3);
  for (auto& x : E.beta) x = float(U(rng) * 2e-4);
  E.gdelta.assign(g.ns * m, 0);
  E.gbeta.assign(g.ns * m, 0);
  E.gI.resize(m);
  for (auto& x : E.gI) x = float(U(rng) - 0.5);
  E.inten.assign(m, 0);
  Field probe(m);
  for (auto& x : probe) x = cd(U(rng) - 0.5, U(rng) - 0.5);

  // fake device addresses: distinct, well separated, multiples of m
  const int64_t SPAN = 1 << 20;
  auto fake = [&](int slot) { return reinterpret_cast<float2*>((uintptr_t)(SPAN * 64 * (slot + 1))); };
  const int nck = (g.ns + kck - 1) / kck;
  // row-major caller arrays: probe, exit wave, checkpoints, cotangent in, probe cotangent out;
  // working fields (tiled unless a phase is row-major): field, W, G, tmp; segments tiled
  Arr probeA{{probe}, fake(10), m}, out{{Field(m)}, fake(9), m}, gfield{{Field(m)}, fake(11), m},
      gprobe{{Field(m)}, fake(12), m};
  Arr field{{Field(m)}, fake(0), m}, ckpt{std::vector<Field>(nck, Field(m)), fake(1), m},
      seg{std::vector<Field>(kck > 1 ? 2 * (kck - 1) : 1, Field(m)), fake(2), m}, W{{Field(m)}, fake(3), m},
      G{{Field(m)}, fake(4), m}, tmp{{Field(m)}, fake(5), m};
  g_arrays = {&field, &ckpt, &seg, &W, &G, &tmp, &probeA, &out, &gfield, &gprobe};

  // forward with checkpoints: tiled working field between row-major probe and
  // exit wave, or (odd slice counts) row-major on the exit-wave array itself
  msl::PhaseSpec ph{};
  ph.kind = msl::PH_FWD_FULL; ph.exact = g.exact; ph.s0 = 0; ph.s1 = g.ns; ph.ns = g.ns; ph.m = m;
  if (g.ns % 2) {
    out.f[0] = probe;
    ph.field = fake(9);
    ph.rowmajor = 1;
  } else {
    ph.field = fake(0);
    ph.in_rm = fake(10);
    ph.out_rm = fake(9);
  }
  ph.ckpt = fake(1); ph.ckpt_every = kck;
  int bad = check_tab_sequence(ph);
  run_phase(E, ph);

  // direct reference
  std::vector<Field> kept;
  Field psi = probe;
  for (int s = 0; s < g.ns; ++s) {
    kept.push_back(psi);
    for (int64_t e = 0; e < m; ++e) psi[e] *= tfun(E, s, e);
    psi = prop_slice(psi, g, s, false);
  }
  const double ef = rel(out.f[0], psi);
  if (ef > 1e-10) { std::printf("forward mismatch %g\n", ef); ++bad; }
  for (int c = 0; c < nck; ++c) {
    const double e = rel(ckpt.f[c], kept[c * kck]);
    if (e > 1e-10) { std::printf("checkpoint %d mismatch %g\n", c, e); ++bad; }
  }

  // far field of the exit wave
  msl::PhaseSpec ff{};
  ff.kind = msl::PH_FF; ff.m = m; ff.in_rm = fake(9); ff.field = fake(5);
  run_phase(E, ff);
  Field A = dft2(psi, g, +1);
  std::vector<double> Iref(m);
  for (int r = 0; r < g.ny; ++r)
    for (int c = 0; c < g.nz; ++c)
      Iref[(int64_t)((r + g.ny / 2) % g.ny) * g.nz + (c + g.nz / 2) % g.nz] = std::norm(A[(int64_t)r * g.nz + c]) / m;
  if (relv(E.inten, Iref) > 1e-10) { std::printf("far field mismatch\n"); ++bad; }

  // far-field adjoint into the row-major cotangent array
  msl::PhaseSpec fa{};
  fa.kind = msl::PH_FFADJ; fa.m = m; fa.in_rm = fake(9); fa.field = fake(5); fa.out_rm = fake(11);
  run_phase(E, fa);
  Field seed(m);
  for (int r = 0; r < g.ny; ++r)
    for (int c = 0; c < g.nz; ++c) {
      const double gi = E.gI[(int64_t)((r + g.ny / 2) % g.ny) * g.nz + (c + g.nz / 2) % g.nz];
      seed[(int64_t)r * g.nz + c] = 2.0 * gi * A[(int64_t)r * g.nz + c] / double(m);
    }
  Field gref = dft2(seed, g, -1);
  if (rel(gfield.f[0], gref) > 1e-10) { std::printf("far-field adjoint mismatch %g\n", rel(gfield.f[0], gref)); ++bad; }

  // adjoint with recompute: the same order as the library (segment c-1 is
  // recomputed beside the reverse sweep over segment c, into the other of two
  // segment buffers); the first reverse phase reads the cotangent array, the
  // last writes the probe's cotangent
  auto recomp = [&](int c) {
    const int s0 = c * kck, s1 = std::min(s0 + kck, g.ns);
    if (s1 - s0 < 2) return;
    msl::PhaseSpec rc{};
    rc.kind = msl::PH_FWD_RECOMP; rc.exact = g.exact; rc.s0 = s0; rc.s1 = s1; rc.ns = g.ns; rc.m = m;
    rc.field = fake(3); rc.in_rm = fake(1) + (int64_t)c * m;
    rc.seg = fake(2) + (c & 1) * (int64_t)(kck > 1 ? kck - 1 : 0) * m;
    run_phase(E, rc);
  };
  if (kck == 1) {
    // the library's direct sweep: every entrance field is a checkpoint, read row-major
    msl::PhaseSpec rv{};
    rv.kind = msl::PH_REV; rv.exact = g.exact; rv.s0 = 0; rv.s1 = g.ns; rv.ns = g.ns; rv.m = m;
    rv.leading = 1; rv.field = fake(4); rv.in_rm = fake(11); rv.out_rm = fake(12);
    rv.seg = fake(1) + m; rv.ckpt_c = fake(1); rv.seg_row_major = 1;
    run_phase(E, rv);
  }
  if (kck > 1) recomp(nck - 1);
  for (int c = nck - 1; c >= 0 && kck > 1; --c) {
    const int s0 = c * kck, s1 = std::min(s0 + kck, g.ns);
    msl::PhaseSpec rv{};
    rv.kind = msl::PH_REV; rv.exact = g.exact; rv.s0 = s0; rv.s1 = s1; rv.ns = g.ns; rv.m = m;
    rv.leading = c == nck - 1; rv.field = fake(4);
    rv.in_rm = c == nck - 1 ? fake(11) : nullptr;
    rv.out_rm = c == 0 ? fake(12) : nullptr;
    rv.seg = fake(2) + (c & 1) * (int64_t)(kck > 1 ? kck - 1 : 0) * m;
    rv.ckpt_c = fake(1) + (int64_t)c * m;
    run_phase(E, rv);
    if (c >= 1) recomp(c - 1);
  }
  // direct reverse sweep
  Field gg = gref;
  std::vector<double> gd(g.ns * m), gb(g.ns * m);
  const double k = 2 * M_PI / g.lam;
  for (int s = g.ns - 1; s >= 0; --s) {
    Field gp = prop_slice(gg, g, s, true);
    for (int64_t e = 0; e < m; ++e) {
      const cd T = tfun(E, s, e);
      const cd cc = std::conj(gp[e]) * (T * kept[s][e]);
      gd[s * m + e] = -k * g.dx * cc.imag();
      gb[s * m + e] = -k * g.dx * cc.real();
      gp[e] *= std::conj(T);
    }
    gg = gp;
  }
  if (relv(E.gdelta, gd) > 1e-9) { std::printf("grad delta mismatch %g\n", relv(E.gdelta, gd)); ++bad; }
  if (relv(E.gbeta, gb) > 1e-9) { std::printf("grad beta mismatch %g\n", relv(E.gbeta, gb)); ++bad; }
  if (rel(gprobe.f[0], gg) > 1e-10) { std::printf("grad probe mismatch %g\n", rel(gprobe.f[0], gg)); ++bad; }
  if (g_bad_layout) { std::printf("layout hazard in %d passes\n", g_bad_layout); ++bad; g_bad_layout = 0; }
  std::printf("%s ny=%d nz=%d ns=%d k=%d: field %.1e -> %s\n", g.exact ? "exact" : "paraxial", g.ny, g.nz, g.ns,
              kck, ef, bad ? "FAIL" : "ok");
  return bad;
}

}  // namespace

int main() {
  int bad = 0;
  for (int exact = 0; exact < 2; ++exact) {
    const int cfg[][4] = {{8, 16, 1, 1}, {8, 16, 5, 2}, {16, 8, 7, 3}, {8, 8, 6, 6}, {16, 16, 9, 4}, {8, 32, 4, 10},
                          {16, 8, 11, 5}, {8, 8, 8, 3}, {16, 16, 2, 1}, {8, 8, 140, 16}};
    for (auto& c : cfg) {
      Geo g{c[0], c[1], c[2], 0.9, 1.3, 7.0, 0.15, exact == 1};
      bad += check(g, c[3]);
    }
  }
  std::printf(bad ? "FAILED\n" : "OK\n");
  return bad ? 1 : 0;
}

// Pass programs: which line passes make up each phase of the multislice
// forward sweep, the adjoint sweep and the far field.
//
// Paraxial propagator.  The Fresnel propagator of Eq. (1) (arXiv 2212.01253)
// factorises, exp(i dx (ky^2 + kz^2)/2k) = h_y(ky) h_z(kz), so one slice's
// 2-D propagation is the product of a propagation along rows (P_z) and one
// along columns (P_y), and the two commute.  Alternating the order from one
// slice to the next puts the two halves that touch the same axis side by
// side:  T_0, P_z | P_y, T_1, P_y | P_z, T_2, P_z | ...  so every slice is
// ONE pass over lines of one axis: propagate, transmit, propagate.  That is
// one field round trip and one global exchange per slice instead of two.
// Slice s is always transmitted in a pass of axis s mod 2 (rows for even
// slices, columns for odd ones), in every phase, so everything that belongs
// to one slice (its precomputed transmission, its stored entrance field, the
// odd slices' gradients) can be laid out for that axis: 2x2 tiles in row
// order for even slices, in column order for odd ones.
//
// Exact angular-spectrum propagator.  It does not factorise; each slice takes
// a row pass (z-IFFT, transmission, z-FFT) and a column pass (y-FFT, H, y-IFFT)
// with the field kept in (y, kz) order between them.
#pragma once

#include "msl_device.hpp"

namespace msl {

enum PhaseKind : int {
  PH_FWD_FULL = 0,    // slices [s0, s1) from psi_{s0}, ending with psi_{s1}
  PH_FWD_RECOMP = 1,  // slices [s0, s1): store psi_s, s0 < s < s1, into seg[s - s0 - 1]
  PH_REV = 2,         // reverse sweep over slices s1-1 .. s0 on the cotangent
  PH_FF = 3,          // far-field intensity of the field in in_rm
  PH_FFADJ = 4        // far-field adjoint: cotangent of the field in in_rm, into out_rm
};

// A phase works on one field, its working field, held 2x2-tiled (LAY_T: the
// 2x2 block of rows 2a, 2a+1 and columns 2b, 2b+1 in 32 consecutive bytes), so
// that row passes and column passes both read and write whole 32-byte
// segments when each workgroup takes neighbouring lines.  Every pass reads
// its lines from the working field and writes them back in place (a tile
// holds elements of two lines, never one element twice).  Caller arrays stay
// row-major: a phase's first pass may read its input from a row-major array
// (`in_rm`) and its last pass may write its result to one (`out_rm`).
// Checkpoints are row-major (caller arrays), segment fields tiled.  With
// `rowmajor` set the working field is itself row-major (used where no
// workspace holds a tiled buffer).
struct PhaseSpec {
  int kind;
  int exact;          // exact (non-separable) propagator
  int s0, s1, ns;
  int ckpt_every;
  int leading;        // PH_REV: first reverse phase (adds the leading half-propagation)
  int64_t m;
  float2* field;          // working field
  const float2* in_rm;    // row-major input of the first pass, or nullptr (the working field holds it)
  float2* out_rm;         // row-major output of the last pass, or nullptr (the working field)
  float2* ckpt;           // PH_FWD_FULL: checkpoint array or nullptr
  float2* seg;            // PH_FWD_RECOMP output / PH_REV input
  const float2* ckpt_c;   // PH_REV: psi_{s0} (row-major)
  int rowmajor;           // the working field is row-major instead of tiled
  int seg_row_major;      // PH_REV: `seg` holds row-major fields (the forward's checkpoints) instead of
                          // tiled segment fields (the recompute's)
};

__host__ __device__ inline int phase_npasses(const PhaseSpec& ph) {
  const int n = ph.s1 - ph.s0;
  switch (ph.kind) {
    case PH_FWD_FULL: return ph.exact ? 2 * n + 1 : n + 1;
    case PH_FWD_RECOMP: return n < 2 ? 0 : (ph.exact ? 2 * n - 1 : n);
    case PH_REV: return (ph.exact ? 2 * n : n) + (ph.leading ? 1 : 0);
    case PH_FF: return 2;
    case PH_FFADJ: return 3;
    default: return 0;
  }
}

__host__ __device__ inline int work_lay(const PhaseSpec& ph) { return ph.rowmajor ? LAY_R : LAY_T; }

// Cycle position of the constants (twiddles, sqrt(1/2), one-axis propagator)
// in the passes that belong to slice s (s = ns: the pass after the last
// slice).  Paraxial passes alternate axes with the slice parity, so each axis
// advances one position every two slices; the exact schedule runs a pass
// along each axis per slice.  Every phase (forward, recompute, reverse)
// derives it from the slice alone, so the recompute repeats the forward
// bit for bit and the reverse sweep applies the adjoint of the same constants.
__host__ __device__ inline int tab_of(const PhaseSpec& ph, int s) {
  return (ph.exact ? s : (s >> 1)) & (DITHER - 1);
}

// Layout of a segment field of slice s (its entrance field, stored by the
// recompute and read by the reverse sweep): in the paraxial schedule both
// passes run along the slice's own axis, so odd slices' fields are kept in
// column tile order, which column passes access contiguously.
__host__ __device__ inline int seg_lay(const PhaseSpec& ph, int s) {
  if (ph.rowmajor) return LAY_R;
  return (!ph.exact && (s & 1)) ? LAY_C : LAY_T;
}

// A pass along `axis`, the first and/or the last of its phase.
__host__ __device__ inline PassDesc make_pass(const PhaseSpec& ph, int axis, bool first, bool last) {
  PassDesc p;
  p.axis = axis;
  p.pre = PRE_NONE;
  p.mid = MID_NONE;
  p.post = POST_NONE;
  p.conj = 0;
  p.slice = 0;
  p.tab = 0;
  const int wl = work_lay(ph);
  if (first && ph.in_rm) {
    p.src = ph.in_rm;
    p.src_lay = LAY_R;
  } else {
    p.src = ph.field;
    p.src_lay = wl;
  }
  if (last && ph.out_rm) {
    p.dst = ph.out_rm;
    p.dst_lay = LAY_R;
  } else {
    p.dst = ph.field;
    p.dst_lay = wl;
  }
  p.psi_store = nullptr;
  p.psi_load = nullptr;
  p.store_lay = LAY_R;
  p.load_lay = LAY_R;
  return p;
}

__host__ __device__ inline float2* ckpt_slot(const PhaseSpec& ph, int s) {
  if (!ph.ckpt || ph.ckpt_every <= 0 || (s % ph.ckpt_every) != 0) return nullptr;
  return ph.ckpt + (int64_t)(s / ph.ckpt_every) * ph.m;
}

// Axis of the first pass of a phase.
__host__ __device__ inline int phase_first_axis(const PhaseSpec& ph) {
  if (ph.exact) return ROW;
  switch (ph.kind) {
    case PH_FWD_FULL:
    case PH_FWD_RECOMP: return (ph.s0 & 1) ? COL : ROW;
    case PH_REV: return ph.leading ? ((ph.ns & 1) ? COL : ROW) : (((ph.s1 - 1) & 1) ? COL : ROW);
    default: return ROW;
  }
}

__host__ __device__ inline PassDesc phase_pass(const PhaseSpec& ph, int p) {
  const int n = ph.s1 - ph.s0;
  const int np = phase_npasses(ph);
  const bool first = p == 0, last = p == np - 1;
  const int wl = work_lay(ph);
  switch (ph.kind) {
    case PH_FWD_FULL:
      if (!ph.exact) {
        const int axis = ((ph.s0 + p) & 1) ? COL : ROW;
        PassDesc d = make_pass(ph, axis, first, last);
        d.tab = tab_of(ph, ph.s0 + p);
        if (p < n) {
          d.pre = p == 0 ? PRE_NONE : PRE_PROP;
          d.mid = MID_T_FWD;
          d.slice = ph.s0 + p;
          d.psi_store = ckpt_slot(ph, ph.s0 + p);
          d.store_lay = LAY_R;
          d.post = POST_PROP;
        } else {
          d.pre = PRE_PROP;
        }
        return d;
      } else {
        if (p & 1) {
          PassDesc d = make_pass(ph, COL, first, last);
          d.tab = tab_of(ph, ph.s0 + p / 2);
          d.post = POST_PROP2D;
          return d;
        }
        const int q = p / 2;
        PassDesc d = make_pass(ph, ROW, first, last);
        d.tab = tab_of(ph, ph.s0 + q);
        d.pre = q == 0 ? PRE_NONE : PRE_IFFT_N;
        if (q < n) {
          d.mid = MID_T_FWD;
          d.slice = ph.s0 + q;
          d.psi_store = ckpt_slot(ph, ph.s0 + q);
          d.store_lay = LAY_R;
          d.post = POST_FFT;
        }
        return d;
      }
    case PH_FWD_RECOMP:
      if (!ph.exact) {
        const int axis = ((ph.s0 + p) & 1) ? COL : ROW;
        PassDesc d = make_pass(ph, axis, first, false);
        d.tab = tab_of(ph, ph.s0 + p);
        d.pre = p == 0 ? PRE_NONE : PRE_PROP;
        if (p > 0) {
          d.psi_store = ph.seg + (int64_t)(p - 1) * ph.m;
          d.store_lay = seg_lay(ph, ph.s0 + p);
        }
        if (p < n - 1) {
          d.mid = MID_T_FWD;
          d.slice = ph.s0 + p;
          d.post = POST_PROP;
        } else {
          d.dst = nullptr;
        }
        return d;
      } else {
        if (p & 1) {
          PassDesc d = make_pass(ph, COL, first, false);
          d.tab = tab_of(ph, ph.s0 + p / 2);
          d.post = POST_PROP2D;
          return d;
        }
        const int q = p / 2;
        PassDesc d = make_pass(ph, ROW, first, false);
        d.tab = tab_of(ph, ph.s0 + q);
        d.pre = q == 0 ? PRE_NONE : PRE_IFFT_N;
        if (q > 0) {
          d.psi_store = ph.seg + (int64_t)(q - 1) * ph.m;
          d.store_lay = wl;
        }
        if (q < n - 1) {
          d.mid = MID_T_FWD;
          d.slice = ph.s0 + q;
          d.post = POST_FFT;
        } else {
          d.dst = nullptr;
        }
        return d;
      }
    case PH_REV: {
      if (ph.leading && p == 0) {
        // precedes the pass of slice ns - 1, so it takes the other axis
        PassDesc d = make_pass(ph, phase_first_axis(ph), first, last);
        d.tab = tab_of(ph, ph.ns);
        if (ph.exact) d.post = POST_FFT;
        else { d.pre = PRE_PROP; d.conj = 1; }
        return d;
      }
      const int q = p - (ph.leading ? 1 : 0);
      if (!ph.exact) {
        const int s = ph.s1 - 1 - q;
        const int axis = (s & 1) ? COL : ROW;
        PassDesc d = make_pass(ph, axis, first, last);
        d.tab = tab_of(ph, s);
        d.pre = PRE_PROP;
        d.conj = 1;
        d.mid = MID_T_ADJ;
        d.slice = s;
        if (s == ph.s0) {
          d.psi_load = ph.ckpt_c;
          d.load_lay = LAY_R;
        } else {
          d.psi_load = ph.seg + (int64_t)(s - ph.s0 - 1) * ph.m;
          d.load_lay = ph.seg_row_major ? LAY_R : seg_lay(ph, s);
        }
        d.post = s == 0 ? POST_NONE : POST_PROP;
        return d;
      } else {
        const int s = ph.s1 - 1 - q / 2;
        if ((q & 1) == 0) {
          PassDesc d = make_pass(ph, COL, first, last);
          d.tab = tab_of(ph, s);
          d.post = POST_PROP2D;
          d.conj = 1;
          return d;
        }
        PassDesc d = make_pass(ph, ROW, first, last);
        d.tab = tab_of(ph, s);
        d.pre = PRE_IFFT_N;
        d.mid = MID_T_ADJ;
        d.slice = s;
        if (s == ph.s0) {
          d.psi_load = ph.ckpt_c;
          d.load_lay = LAY_R;
        } else {
          d.psi_load = ph.seg + (int64_t)(s - ph.s0 - 1) * ph.m;
          d.load_lay = ph.seg_row_major ? LAY_R : wl;
        }
        d.post = s == 0 ? POST_NONE : POST_FFT;
        return d;
      }
    }
    case PH_FF:
      if (p == 0) {
        PassDesc d = make_pass(ph, ROW, first, false);
        d.pre = PRE_IFFT_U;
        return d;
      } else {
        PassDesc d = make_pass(ph, COL, false, false);
        d.dst = nullptr;
        d.pre = PRE_IFFT_U;
        d.mid = MID_FF_OUT;
        return d;
      }
    case PH_FFADJ:
    default:
      if (p == 0) {
        PassDesc d = make_pass(ph, ROW, first, false);
        d.pre = PRE_IFFT_U;
        return d;
      } else if (p == 1) {
        PassDesc d = make_pass(ph, COL, false, false);
        d.pre = PRE_IFFT_U;
        d.mid = MID_FF_SEED;
        d.post = POST_FFT;
        return d;
      } else {
        PassDesc d = make_pass(ph, ROW, false, last);
        d.pre = PRE_FFT;
        return d;
      }
  }
}

}  // namespace msl

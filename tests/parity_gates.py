"""Element-wise parity gates of the complex64 GPU results against the FP64 oracle.

Every forward, batch and full-size parity test applies these on top of the
relative-L2 bars (exit field 2e-5, intensity 1e-4).  The bounds follow from
the float32 error model of the path, not from what the GPU happens to reach.

Quantities and their relative budgets tol:
* the exit field psi: FIELD_TOL = 2e-5;
* the far-field amplitude a = sqrt(I), the quantity the amplitude loss (Eq. 4)
  compares: AMP_TOL = 2.5e-5.  With A the unnormalised far-field sum and
  I = |A|^2 / M, | |A + dA| - |A| | <= |dA| pixel by pixel, and by Parseval
  ||dA|| / ||A|| = ||d psi|| / ||psi||, so the amplitude relative L2 is at most
  the field's plus the rounding of the far-field transform itself (float32
  rounding over log2 M radix-2 levels, about 2 x 20 x 6e-8 < 5e-6).

Error model.  The error of a result splits into
  (i) a part uncorrelated with the result: the random walk of data rounding,
      spread over the whole grid by the FFTs, of uniform variance; the
      relative-L2 budget bounds its RMS by tol * RMS(x_ref), on every pixel
      alike, bright or dark;
 (ii) a part proportional to the result: a slightly wrong amplitude or phase
      of what is there (coherent drift; near a dominant beam it also feeds the
      neighbouring, nearly resonant modes), at most tol * |x_ref| in its own
      element.
Two gates follow.
* Every element: |x_gpu - x_ref| <= tol * max|x_ref| + TAIL * tol * RMS(x_ref).
  Part (ii) at its largest is the whole budget of the dominant element; part
  (i) is a complex Gaussian of RMS at most sigma = tol * RMS(x_ref), and
  P(|e| > t sigma) = exp(-t^2): at t = TAIL = 6 that is 2.3e-16 per element,
  below 3e-10 over the largest grid (2^20 elements).
* Every brightness class (elements with |x_ref| / RMS(x_ref) in one decade,
  at least 16 of them; everything below 1e-6 RMS in the lowest class):
  RMS_class(x_gpu - x_ref) <= tol * RMS_class(x_ref) + 2 * tol * RMS(x_ref).
  Part (ii) contributes at most the first term, part (i) at most tol * RMS,
  doubled for the sampling spread of an RMS over a finite class (for 16 or
  more complex Gaussian samples the probability of twice the true RMS is
  below 1e-9).  Dark classes - the diffuse far field - are thereby held to
  the uniform floor in absolute terms: a wrong region of dim pixels fails
  here even when the relative-L2 norms, set by the bright peaks, do not move.
"""
import numpy as np

FIELD_TOL = 2e-5
INT_TOL = 1e-4
AMP_TOL = 2.5e-5
CLASS_SLACK = 2.0
TAIL = 6.0
MIN_CLASS = 16


def rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def element_gates(x, ref, tol):
    """Worst ratios (<= 1 passes) of the element gate and of the brightness-class gate, and
    a description of the worst class."""
    ref = np.asarray(ref)
    x = np.asarray(x)
    d = np.abs(x.astype(np.complex128) - ref.astype(np.complex128)).ravel()
    mag = np.abs(ref).ravel().astype(np.float64)
    rms = float(np.sqrt(np.mean(mag ** 2)))
    r_elem = float(d.max() / (tol * mag.max() + TAIL * tol * rms))
    k = np.floor(np.log10(np.maximum(mag / rms, 1e-6))).astype(int)
    worst, where = 0.0, ""
    for c in np.unique(k):
        m = k == c
        if m.sum() < MIN_CLASS:
            continue
        err = float(np.sqrt(np.mean(d[m] ** 2)))
        bound = tol * float(np.sqrt(np.mean(mag[m] ** 2))) + CLASS_SLACK * tol * rms
        if err / bound > worst:
            worst, where = err / bound, f"class [1e{c}, 1e{c + 1}) RMS, {int(m.sum())} elements, error RMS {err / rms:.2e}"
    return r_elem, worst, where


def check_field(f, rf, tol=FIELD_TOL, what="field"):
    rf = np.asarray(rf, dtype=np.complex128)
    e_rel = rel(np.asarray(f).astype(np.complex128), rf)
    r_elem, r_class, where = element_gates(f, rf, tol)
    assert e_rel <= tol, f"{what}: relative L2 {e_rel:.3e} > {tol:.1e}"
    assert r_elem <= 1.0, f"{what}: an element is off by {r_elem:.2f} x its bound"
    assert r_class <= 1.0, f"{what}: {r_class:.2f} x the class bound in {where}"
    return e_rel, max(r_elem, r_class)


def check_intensity(I, rI, tol_i=INT_TOL, tol_a=AMP_TOL, what="intensity"):
    I = np.asarray(I, dtype=np.float64)
    rI = np.asarray(rI, dtype=np.float64)
    a = np.sqrt(np.maximum(I, 0.0))
    ra = np.sqrt(np.maximum(rI, 0.0))
    e_i = rel(I, rI)
    e_a = rel(a, ra)
    r_elem, r_class, where = element_gates(a, ra, tol_a)
    assert e_i <= tol_i, f"{what}: relative L2 {e_i:.3e} > {tol_i:.1e}"
    assert e_a <= tol_a, f"{what}: amplitude relative L2 {e_a:.3e} > {tol_a:.1e}"
    assert r_elem <= 1.0, f"{what}: an amplitude is off by {r_elem:.2f} x its bound"
    assert r_class <= 1.0, f"{what}: amplitudes {r_class:.2f} x the class bound in {where}"
    return e_i, e_a, max(r_elem, r_class)


def check_forward(f, rf, I, rI, what=""):
    """Field and far-field gates together; returns the five figures for printing."""
    ef = check_field(f, rf, what=f"{what} field".strip())
    ei = check_intensity(I, rI, what=f"{what} intensity".strip())
    return ef + ei


def fmt(errs):
    names = ("field", "field gates", "I", "sqrt(I)", "sqrt(I) gates")
    return " ".join(f"{n} {e:.2e}" for n, e in zip(names, errs))

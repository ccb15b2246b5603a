"""FP64 CPU oracle for the reflection-geometry multislice model (arXiv 2212.01253).

TEST INFRASTRUCTURE ONLY.  This module is the plain, slow, obviously correct
definition that the HIP library is checked against.  Only the test-suite, the
package smoke check and the benchmark's ``cpu_baseline`` leg may import it;
the product path never does.  It shares no code with the HIP path: it builds
its own frequency grids, propagators, probe and transforms from NumPy/SciPy
primitives in complex128.

What it computes (paper section / equation followed):

* Multislice recurrence, Eq. (1) of Sec. 1: for every slice the field is
  multiplied by the slice transmission, Fourier transformed, multiplied by the
  Fresnel propagator and inverse transformed; the exit wave of one slice is the
  entrance wave of the next (Sec. 1 and the Fig. 1 caption).
* Far-field detector image (Sec. 1, Fig. 1 caption): the final exit wave is
  Fourier transformed and squared; the phase is lost.
* Amplitude loss, Eq. (4) of Sec. 4.1: squared difference of predicted and
  measured scattering amplitudes summed over the detector (the mean is the sum
  over the pixel count).
* Gradient of that loss with respect to the slice indices (Sec. 1 and 4: the
  paper obtains it by automatic differentiation; here it is the explicit
  adjoint of the same recurrence, see ``adjoint``).

Readings of the paper used here (each one is also listed in the design notes):

* Sign convention.  Eq. (1) is written for exp(+ikZ) waves with
  n = 1 - delta + i*beta.  This implementation uses the complex-conjugate
  convention throughout: transmission exp(i k dx (delta + i beta)), paraxial
  propagator exp(+i dx (ky^2 + kz^2) / 2k), incident tilt exp(+i k sin(a) y)
  and the far field as the unnormalised backward DFT.  Every field is the
  complex conjugate of the paper-convention field and every detector
  intensity is identical bin for bin (``forward_paper_convention`` shows it).
* First-order slice projection: the integral of (1 - n^2) over a slice is
  taken as 2*dx*(delta - i*beta) with slice-averaged delta and beta (the
  second-order term is dropped), which gives the transmission above.
* The global carrier exp(ik dx) of Eq. (1) is dropped: it is one phase factor
  per slice and cannot change any intensity.
* Incidence enters as a tilt of the probe in the sample frame instead of a
  rotation of the object (Eq. 2-3); the two are the same system rotated.
* Far field: A = sum_j psi_j exp(+2 pi i u j / N) over both axes,
  I = |A|^2 / (Ny*Nz), fftshifted so that row Ny/2 is the horizon (q_y = 0).
* Loss: L = sum (sqrt(I) - m)^2 with m the measured amplitude; where I = 0
  the derivative of sqrt is taken as 0.

Grid convention: the field is an [Ny][Nz] array; rows are y (surface normal,
row 0 is the deepest substrate row), columns are z; slices advance along x,
the beam axis, each dx thick.
"""
from __future__ import annotations

import math
import os

import numpy as np
import scipy.fft as sfft

PARAXIAL = 0
EXACT = 1

# FFT threads: the cores this process may run on
WORKERS = len(os.sched_getaffinity(0))


def _g(geom, name):
    return geom[name] if isinstance(geom, dict) else getattr(geom, name)


def wavenumber(geom) -> float:
    """k = 2 pi / lambda (nm^-1)."""
    return 2.0 * math.pi / float(_g(geom, "wavelength_nm"))


def spatial_frequencies(n: int, d: float) -> np.ndarray:
    """Angular spatial frequencies 2 pi * fftfreq(n, d) in DFT order (FP64)."""
    return 2.0 * math.pi * np.fft.fftfreq(n, d)


def propagator(geom, conj_convention: bool = False) -> np.ndarray:
    """Fourier-space propagator H(ky, kz) for one slice, [Ny][Nz] complex128.

    Paraxial (Eq. 1): exp(+i dx (ky^2 + kz^2) / 2k).
    Exact angular spectrum: exp(+i dx kp^2 / (k + sqrt(k^2 - kp^2))) for
    kp < k; for kp >= k the mode decays as exp(-dx sqrt(kp^2 - k^2)) with the
    carrier phase exp(+i k dx) (the carrier is dropped only for propagating
    modes, where it is a global phase).
    ``conj_convention`` returns the paper-convention propagator (conjugate).
    """
    ny, nz = int(_g(geom, "ny")), int(_g(geom, "nz"))
    dx = float(_g(geom, "dx_nm"))
    k = wavenumber(geom)
    ky = spatial_frequencies(ny, float(_g(geom, "dy_nm")))
    kz = spatial_frequencies(nz, float(_g(geom, "dz_nm")))
    kp2 = ky[:, None] ** 2 + kz[None, :] ** 2
    if int(_g(geom, "propagator")) == PARAXIAL:
        H = np.exp(1j * dx * kp2 / (2.0 * k))
    else:
        H = np.empty(kp2.shape, np.complex128)
        prop = kp2 < k * k
        H[prop] = np.exp(1j * dx * kp2[prop] / (k + np.sqrt(k * k - kp2[prop])))
        ev = ~prop
        H[ev] = np.exp(1j * k * dx) * np.exp(-dx * np.sqrt(kp2[ev] - k * k))
    return np.conj(H) if conj_convention else H


def tilted_probe(geom, conj_convention: bool = False) -> np.ndarray:
    """Plane wave tilted by the incidence angle toward the substrate (row 0).

    psi0[j, l] = exp(+i k sin(alpha_i) y_j), y_j = j * dy.
    """
    ny, nz = int(_g(geom, "ny")), int(_g(geom, "nz"))
    k = wavenumber(geom)
    y = np.arange(ny, dtype=np.float64) * float(_g(geom, "dy_nm"))
    ph = k * math.sin(float(_g(geom, "alpha_i_rad"))) * y
    col = np.exp(-1j * ph) if conj_convention else np.exp(1j * ph)
    return np.repeat(col[:, None], nz, axis=1)


def transmission(delta_s, beta_s, geom) -> np.ndarray:
    """Slice transmission T = exp(i k dx (delta + i beta)) (first-order projection)."""
    k = wavenumber(geom)
    dx = float(_g(geom, "dx_nm"))
    return np.exp(1j * k * dx * (np.asarray(delta_s, np.float64)
                                 + 1j * np.asarray(beta_s, np.float64)))


def transmission_exact_index(delta_s, beta_s, geom) -> np.ndarray:
    """Slice transmission with the full projection of (1 - n^2) instead of its first order.

    With n = 1 - delta + i beta, (1 - n^2) / 2 = (delta - i beta) - (delta - i beta)^2 / 2; in this
    convention (the conjugate of Eq. 1's) T = exp(i k dx [(delta + i beta) - (delta + i beta)^2 / 2]).
    A physics variant for comparisons, not what the library computes.
    """
    k = wavenumber(geom)
    dx = float(_g(geom, "dx_nm"))
    z = np.asarray(delta_s, np.float64) + 1j * np.asarray(beta_s, np.float64)
    return np.exp(1j * k * dx * (z - 0.5 * z * z))


def forward_exact_index(geom, delta, beta, probe=None):
    """``forward`` with ``transmission_exact_index``."""
    ns = int(_g(geom, "n_slices"))
    H = propagator(geom)
    psi = (tilted_probe(geom) if probe is None
           else np.asarray(probe, np.complex128).copy())
    for s in range(ns):
        psi = psi * transmission_exact_index(delta[s], beta[s], geom)
        psi = _ifft2(H * _fft2(psi))
    return psi


def rotation_matrix(pitch, yaw):
    """Sample-frame offset of a lab-frame offset, axes in library order (slice axis a = the paper's
    Z, row y = Y, column z = X): the paper's pitch and yaw rotations (Eq. 2-3) applied to the lab
    position, R_pitch(pitch) R_yaw(yaw) in (X, Y, Z), re-indexed to (Z, Y, X)."""
    cp, sp, cw, sw = math.cos(pitch), math.sin(pitch), math.cos(yaw), math.sin(yaw)
    return np.array([[cp * cw, sp, -cp * sw],
                     [-sp * cw, cp, sp * sw],
                     [sw, 0.0, cw]])


def rotate_object(geom, lab_pivot, sample, pitch, yaw, delta_s, beta_s):
    """Lab-frame slice stacks [Ns][ny][nz] of a sample-frame volume (Eq. 2-3 taken literally):
    lab voxel (s, j, l) at u = (s dx, j dy, l dz) - lab_pivot takes the trilinear interpolate of the
    sample volume at M u + sample pivot (sample voxel (i, j, k) at (i da, j dy, k dz), zero outside)."""
    from scipy.ndimage import map_coordinates
    ns, ny, nz = int(_g(geom, "n_slices")), int(_g(geom, "ny")), int(_g(geom, "nz"))
    d = [float(_g(geom, "dx_nm")), float(_g(geom, "dy_nm")), float(_g(geom, "dz_nm"))]
    S, J, L = np.meshgrid(np.arange(ns), np.arange(ny), np.arange(nz), indexing="ij")
    u = np.stack([S * d[0] - lab_pivot[0], J * d[1] - lab_pivot[1], L * d[2] - lab_pivot[2]])
    M = rotation_matrix(pitch, yaw)
    v = np.einsum("ij,j...->i...", M, u)
    piv = [sample["pivot_a_nm"], sample["pivot_y_nm"], sample["pivot_z_nm"]]
    pit = [sample["da_nm"], sample["dy_nm"], sample["dz_nm"]]
    idx = np.stack([(v[i] + piv[i]) / pit[i] for i in range(3)])
    out = []
    for vol in (delta_s, beta_s):
        out.append(map_coordinates(np.asarray(vol, np.float64), idx, order=1, mode="grid-constant", cval=0.0))
    return out[0], out[1]


def _fft2(x):
    return sfft.fft2(x, workers=WORKERS)


def _ifft2(x):
    return sfft.ifft2(x, workers=WORKERS)


def forward(geom, delta, beta, probe=None, keep=False):
    """Multislice exit wave psi_Ns (complex128 [Ny][Nz]).

    For s = 0 .. Ns-1:  psi <- T_s * psi ;  psi <- IFFT2( H * FFT2(psi) ).
    With ``keep`` it also returns the list of slice-entrance fields psi_s
    (psi_0 is the probe), which the adjoint and the checkpoint tests use.
    """
    ns = int(_g(geom, "n_slices"))
    H = propagator(geom)
    psi = (tilted_probe(geom) if probe is None
           else np.asarray(probe, np.complex128).copy())
    kept = []
    for s in range(ns):
        if keep:
            kept.append(psi.copy())
        psi = psi * transmission(delta[s], beta[s], geom)
        psi = _ifft2(H * _fft2(psi))
    return (psi, kept) if keep else psi


def forward_paper_convention(geom, delta, beta, probe_conj=None):
    """The same model in the paper's exp(+ikZ) convention (Eq. 1 literally).

    T = exp(-i k dx (delta - i beta)), H = exp(-i dx kp^2 / 2k), probe
    exp(-i k sin(alpha) y); returns (psi_Ns, I) with I from the forward DFT.
    """
    ns = int(_g(geom, "n_slices"))
    k = wavenumber(geom)
    dx = float(_g(geom, "dx_nm"))
    H = propagator(geom, conj_convention=True)
    psi = (tilted_probe(geom, conj_convention=True) if probe_conj is None
           else np.asarray(probe_conj, np.complex128).copy())
    for s in range(ns):
        d = np.asarray(delta[s], np.float64)
        b = np.asarray(beta[s], np.float64)
        psi = psi * np.exp(-1j * k * dx * (d - 1j * b))
        psi = _ifft2(H * _fft2(psi))
    m = psi.shape[0] * psi.shape[1]
    A = _fft2(psi)
    return psi, np.fft.fftshift(np.abs(A) ** 2 / m)


def far_field_amplitude(psi) -> np.ndarray:
    """Unshifted complex far field A = M * IFFT2(psi) (backward DFT, no 1/M)."""
    m = psi.shape[0] * psi.shape[1]
    return m * _ifft2(np.asarray(psi, np.complex128))


def far_field(geom, psi) -> np.ndarray:
    """Detector intensity I = fftshift(|A|^2 / M), float64 [Ny][Nz]."""
    m = psi.shape[0] * psi.shape[1]
    return np.fft.fftshift(np.abs(far_field_amplitude(psi)) ** 2 / m)


def amp_loss(intensity, measured_amp):
    """Eq. (4) with amplitudes: L = sum (sqrt(I) - m)^2 and dL/dI.

    Returns (L_sum, L_mean, dL/dI); dL/dI = 1 - m / sqrt(I), and 0 where I = 0.
    """
    I = np.asarray(intensity, np.float64)
    m = np.asarray(measured_amp, np.float64)
    a = np.sqrt(I)
    r = a - m
    L = float(np.sum(r * r))
    g = np.zeros_like(I)
    nz = a > 0
    g[nz] = 1.0 - m[nz] / a[nz]
    return L, L / I.size, g


def far_field_adjoint(geom, psi, grad_intensity):
    """Cotangent of psi from a cotangent of the (shifted) intensity.

    dI = (2/M) Re(conj(A) dA) and dA = M * IFFT2(dpsi), so the cotangent is
    FFT2(2 * gI * A / M) (unnormalised forward DFT), with gI unshifted first.
    Complex cotangents follow the convention dL = Re sum conj(g) * dz.
    """
    m = psi.shape[0] * psi.shape[1]
    A = far_field_amplitude(psi)
    gI = np.fft.ifftshift(np.asarray(grad_intensity, np.float64))
    return _fft2(2.0 * gI * A / m)


def adjoint(geom, delta, beta, grad_field, probe=None, kept=None):
    """Reverse-mode gradient of a real loss through the multislice recurrence.

    ``grad_field`` is the cotangent of psi_Ns.  Going back over the slices:
    g' = IFFT2(conj(H) * FFT2(g)) is the cotangent of the transmitted field
    psi'_s = T_s psi_s; then dL/d delta_s = -k dx Im(conj(g') psi'_s),
    dL/d beta_s = -k dx Re(conj(g') psi'_s) and g <- conj(T_s) g'.
    Returns (grad_delta, grad_beta, grad_probe), float64 / complex128.
    """
    ns = int(_g(geom, "n_slices"))
    k = wavenumber(geom)
    dx = float(_g(geom, "dx_nm"))
    if kept is None:
        _, kept = forward(geom, delta, beta, probe, keep=True)
    Hc = np.conj(propagator(geom))
    g = np.asarray(grad_field, np.complex128).copy()
    gd = np.zeros((ns,) + g.shape, np.float64)
    gb = np.zeros((ns,) + g.shape, np.float64)
    for s in range(ns - 1, -1, -1):
        T = transmission(delta[s], beta[s], geom)
        gp = _ifft2(Hc * _fft2(g))
        pt = T * kept[s]
        c = np.conj(gp) * pt
        gd[s] = -k * dx * c.imag
        gb[s] = -k * dx * c.real
        g = np.conj(T) * gp
    return gd, gb, g


def loss_and_gradient(geom, delta, beta, measured_amp, probe=None):
    """Full chain: forward, far field, amplitude loss and its gradient."""
    psi, kept = forward(geom, delta, beta, probe, keep=True)
    I = far_field(geom, psi)
    L, _, gI = amp_loss(I, measured_amp)
    gpsi = far_field_adjoint(geom, psi, gI)
    gd, gb, gp = adjoint(geom, delta, beta, gpsi, probe, kept)
    return L, gd, gb, gp, psi, I


# ---------------------------------------------------------------------------
# Brute-force variant: explicit DFT matrices instead of FFTs.

def dft_matrix(n: int, sign: int = -1) -> np.ndarray:
    """Dense DFT matrix W[u, j] = exp(sign * 2 pi i u j / n)."""
    u = np.arange(n)
    return np.exp(sign * 2j * math.pi * np.outer(u, u) / n)


def brute_forward(geom, delta, beta, probe=None, kron=False):
    """Multislice with dense DFTs, either separable or as one (Ny*Nz)^2 matrix."""
    ny, nz = int(_g(geom, "ny")), int(_g(geom, "nz"))
    ns = int(_g(geom, "n_slices"))
    Fy, Fz = dft_matrix(ny, -1), dft_matrix(nz, -1)
    By, Bz = dft_matrix(ny, +1) / ny, dft_matrix(nz, +1) / nz
    H = propagator(geom)
    psi = (tilted_probe(geom) if probe is None
           else np.asarray(probe, np.complex128).copy())
    if kron:
        F = np.kron(Fy, Fz)
        B = np.kron(By, Bz)
    for s in range(ns):
        psi = psi * transmission(delta[s], beta[s], geom)
        if kron:
            spec = (F @ psi.reshape(-1)).reshape(ny, nz)
            psi = (B @ (H * spec).reshape(-1)).reshape(ny, nz)
        else:
            spec = Fy @ psi @ Fz.T
            psi = By @ (H * spec) @ Bz.T
    return psi


def brute_far_field(psi) -> np.ndarray:
    """Far field by the explicit double sum over all pixels (tiny grids only)."""
    ny, nz = psi.shape
    out = np.zeros((ny, nz), np.float64)
    jj, ll = np.meshgrid(np.arange(ny), np.arange(nz), indexing="ij")
    for u in range(ny):
        for v in range(nz):
            ph = np.exp(2j * math.pi * (u * jj / ny + v * ll / nz))
            out[u, v] = abs(np.sum(psi * ph)) ** 2 / (ny * nz)
    return np.fft.fftshift(out)


# ---------------------------------------------------------------------------
# Closed forms used to pin the oracle.

def fresnel_reflectivity(alpha, delta, beta):
    """Grazing-incidence Fresnel reflectivity R = |r|^2 of a flat substrate.

    Small-angle form r = (a - sqrt(a^2 - 2 delta + 2 i beta)) /
    (a + sqrt(a^2 - 2 delta + 2 i beta)) with the principal square root; this
    is the continuum limit of the paraxial model above.
    """
    a = np.asarray(alpha, np.float64)
    kz2 = np.sqrt(a * a - 2.0 * delta + 2.0j * beta)
    r = (a - kz2) / (a + kz2)
    return np.abs(r) ** 2


def fresnel_reflectivity_exact(alpha, delta, beta):
    """Fresnel (s-polarised) reflectivity with the full Snell law, n = 1 - delta + i beta."""
    a = np.asarray(alpha, np.float64)
    n = 1.0 - delta + 1j * beta
    k1 = np.sin(a)
    k2 = np.sqrt(n * n - np.cos(a) ** 2)
    r = (k1 - k2) / (k1 + k2)
    return np.abs(r) ** 2

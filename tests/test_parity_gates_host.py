"""The element-wise parity gates themselves (host only): what they let through and what
they catch that the relative-L2 bars alone do not."""
import numpy as np
import pytest

from parity_gates import AMP_TOL, FIELD_TOL, check_field, check_intensity


def _field(seed, n=128):
    rng = np.random.default_rng(seed)
    y = np.arange(n)[:, None]
    # a tilted plane wave plus weak scattering: a far field with a bright direct beam
    # and a diffuse background many decades below it
    psi = np.exp(2j * np.pi * 5 * y / n) * np.ones((1, n))
    psi = psi + 1e-3 * (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)))
    return psi


def _far(psi):
    A = np.fft.ifft2(psi) * psi.size
    return np.fft.fftshift(np.abs(A) ** 2 / psi.size)


def test_multiplicative_and_uncorrelated_errors_within_the_budget_pass():
    rng = np.random.default_rng(1)
    psi = _field(0)
    noise = rng.standard_normal(psi.shape) + 1j * rng.standard_normal(psi.shape)
    # half the budget as a coherent amplitude/phase error, half as white noise
    err = 0.5 * FIELD_TOL * psi * np.exp(0.3j) + 0.5 * FIELD_TOL * noise / np.sqrt(2)
    check_field(psi + err, psi)
    check_intensity(_far(psi + err), _far(psi))


def test_wrong_dim_pixels_fail_although_the_l2_norms_pass():
    psi = _field(2)
    I = _far(psi)
    bad = I.copy()
    dim = I < 1e-6 * I.max()
    assert dim.mean() > 0.5
    # the diffuse background of a quarter of the detector 20 % too bright
    mask = dim & (np.arange(I.shape[0])[:, None] < I.shape[0] // 4)
    bad[mask] *= 1.2
    rel_I = np.linalg.norm(bad - I) / np.linalg.norm(I)
    assert rel_I < 1e-6           # invisible to the intensity bar (1e-4)
    with pytest.raises(AssertionError, match="amplitude"):
        check_intensity(bad, I)


def test_one_wrong_field_element_fails():
    psi = _field(3, 256)
    bad = psi.copy()
    bad[17, 100] += 4e-3          # relative L2 1.6e-5, under the 2e-5 bar
    assert np.linalg.norm(bad - psi) / np.linalg.norm(psi) < FIELD_TOL
    with pytest.raises(AssertionError, match="element"):
        check_field(bad, psi)


def test_amplitude_bound_is_the_field_bound_plus_transform_rounding():
    # | |A + dA| - |A| | <= |dA| and Parseval: the amplitude error of the far field of a
    # perturbed field is within the field's relative error, pixel by pixel in absolute terms
    rng = np.random.default_rng(4)
    psi = _field(4)
    d = 1e-5 * (rng.standard_normal(psi.shape) + 1j * rng.standard_normal(psi.shape))
    a, a0 = np.sqrt(_far(psi + d)), np.sqrt(_far(psi))
    A_err = np.abs(np.fft.fftshift(np.fft.ifft2(d) * psi.size)) / np.sqrt(psi.size)
    assert np.all(np.abs(a - a0) <= A_err + 1e-12)
    assert np.linalg.norm(a - a0) / np.linalg.norm(a0) <= np.linalg.norm(d) / np.linalg.norm(psi) * (1 + 1e-9)
    assert AMP_TOL >= FIELD_TOL

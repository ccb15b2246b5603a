"""Planted mistakes in the oracle must fail its pins (CPU only).

Each case edits the oracle's source text in memory (a flipped sign, a dropped
factor, a wrong axis, a swapped order), loads the edited copy as a separate
module, points the pin tests at it and checks that at least one pin fails.
The committed oracle is never modified.
"""
import importlib.util
import os
import types

import pytest

import tests.test_oracle_pins as pins

ORACLE_SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                          "oracle", "msl_oracle.py")

P = pins
CASES = {
    "propagator sign": (
        "H = np.exp(1j * dx * kp2 / (2.0 * k))", "H = np.exp(-1j * dx * kp2 / (2.0 * k))",
        [lambda: P.test_p3_plane_wave(0)]),
    "exact propagator form": (
        "H[prop] = np.exp(1j * dx * kp2[prop] / (k + np.sqrt(k * k - kp2[prop])))",
        "H[prop] = np.exp(1j * dx * kp2[prop] / (2 * np.sqrt(k * k - kp2[prop])))",
        [lambda: P.test_p3_plane_wave(1)]),
    "transmission sign": (
        "return np.exp(1j * k * dx * (np.asarray(delta_s, np.float64)",
        "return np.exp(-1j * k * dx * (np.asarray(delta_s, np.float64)",
        [P.test_p4_uniform_slab]),
    "absorption sign": (
        "+ 1j * np.asarray(beta_s, np.float64)))", "- 1j * np.asarray(beta_s, np.float64)))",
        [P.test_p4_uniform_slab]),
    "slice thickness dropped": (
        "return np.exp(1j * k * dx * (np.asarray(delta_s", "return np.exp(1j * k * (np.asarray(delta_s",
        [P.test_p4_uniform_slab, P.test_p8_born_limit]),
    "z frequencies on the y pitch": (
        'kz = spatial_frequencies(nz, float(_g(geom, "dz_nm")))',
        'kz = spatial_frequencies(nz, float(_g(geom, "dy_nm")))',
        [lambda: P.test_p3_plane_wave(0)]),
    "probe tilt sign": (
        "col = np.exp(-1j * ph) if conj_convention else np.exp(1j * ph)",
        "col = np.exp(1j * ph) if conj_convention else np.exp(-1j * ph)",
        [P.test_p3_tilted_probe_is_on_bin_plane_wave]),
    "far field by forward DFT": (
        "return m * _ifft2(np.asarray(psi, np.complex128))", "return _fft2(np.asarray(psi, np.complex128))",
        [lambda: P.test_p1_brute_force_dft(4, 8, 0)]),
    "far field not shifted": (
        "return np.fft.fftshift(np.abs(far_field_amplitude(psi)) ** 2 / m)",
        "return np.abs(far_field_amplitude(psi)) ** 2 / m",
        [lambda: P.test_p1_brute_force_dft(4, 8, 0)]),
    "propagate before transmit": (
        "        psi = psi * transmission(delta[s], beta[s], geom)\n        psi = _ifft2(H * _fft2(psi))\n    return (psi, kept)",
        "        psi = _ifft2(H * _fft2(psi))\n        psi = psi * transmission(delta[s], beta[s], geom)\n    return (psi, kept)",
        [lambda: P.test_p1_brute_force_dft(4, 8, 0)]),
    "adjoint without conj(H)": (
        "Hc = np.conj(propagator(geom))", "Hc = propagator(geom)",
        [lambda: P.test_p11_dot_product(0), P.test_p12_reversibility]),
    "delta gradient sign": (
        "gd[s] = -k * dx * c.imag", "gd[s] = k * dx * c.imag",
        [P.test_p11_linearised_delta_map]),
    "beta gradient uses Im": (
        "gb[s] = -k * dx * c.real", "gb[s] = -k * dx * c.imag",
        [P.test_p10_gradient_finite_differences]),
    "loss gradient doubled": (
        "g[nz] = 1.0 - m[nz] / a[nz]", "g[nz] = 2.0 * (1.0 - m[nz] / a[nz])",
        [P.test_amp_loss_closed_form]),
    "far-field adjoint factor 2 dropped": (
        "return _fft2(2.0 * gI * A / m)", "return _fft2(gI * A / m)",
        [P.test_far_field_adjoint_finite_differences]),
}


def _load_mutant(old, new):
    src = open(ORACLE_SRC).read()
    assert src.count(old) == 1, old
    mod = types.ModuleType("oracle_mutant")
    mod.__file__ = ORACLE_SRC
    exec(compile(src.replace(old, new), ORACLE_SRC, "exec"), mod.__dict__)
    return mod


@pytest.mark.parametrize("name", sorted(CASES))
def test_planted_mistake_is_caught(name, monkeypatch):
    old, new, checks = CASES[name]
    monkeypatch.setattr(pins, "O", _load_mutant(old, new))
    caught = 0
    for check in checks:
        try:
            check()
        except AssertionError:
            caught += 1
    assert caught > 0, f"no pin caught: {name}"


def test_unmutated_oracle_passes_the_same_checks():
    for _, _, checks in CASES.values():
        for check in checks:
            check()

"""Pins of the oracle's object rotation (Eq. 2-3 read literally) on the CPU."""
import math

import numpy as np
import pytest

from oracle import msl_oracle as O
from paper_2212_01253_amd import synth


def test_matrix_is_the_papers_pitch_times_yaw():
    # Eq. 3 as printed, in (X, Y, Z) order; the library orders axes (Z, Y, X)
    for p, w in [(0.0035, 0.0), (0.0, 0.3), (0.2, -0.7)]:
        Rp = np.array([[1, 0, 0], [0, math.cos(p), -math.sin(p)], [0, math.sin(p), math.cos(p)]])
        Ry = np.array([[math.cos(w), 0, math.sin(w)], [0, 1, 0], [-math.sin(w), 0, math.cos(w)]])
        R = Rp @ Ry
        perm = [2, 1, 0]
        assert np.allclose(O.rotation_matrix(p, w), R[np.ix_(perm, perm)], atol=1e-15)
    # pitch > 0: a point on the sample surface plane y' = 0 rises along the beam
    M = O.rotation_matrix(0.01, 0.0)
    # y' = -sin(p) a + cos(p) y = 0  ->  y = tan(p) a
    a = 1000.0
    assert (M @ np.array([a, math.tan(0.01) * a, 0.0]))[1] == pytest.approx(0.0, abs=1e-9)


def grid(ns, ny, nz, d=(2.0, 1.0, 1.0)):
    return synth.Geometry(ny, nz, ns, d[1], d[2], d[0], 0.1, 0.0, 0)


def test_no_rotation_is_the_identity():
    rng = np.random.default_rng(1)
    vol = rng.random((6, 8, 5))
    g = grid(6, 8, 5)
    s = {"da_nm": 2.0, "dy_nm": 1.0, "dz_nm": 1.0, "pivot_a_nm": 3.0, "pivot_y_nm": 2.0, "pivot_z_nm": 1.0}
    d, b = O.rotate_object(g, (3.0, 2.0, 1.0), s, 0.0, 0.0, vol, 2 * vol)
    assert np.allclose(d, vol, atol=1e-12) and np.allclose(b, 2 * vol, atol=1e-12)


def test_linear_fields_are_reproduced_exactly():
    # trilinear interpolation is exact for linear functions: the rotated field is the linear
    # function evaluated at the rotated positions (inside the sample)
    na, ny, nz = 30, 20, 24
    s = {"da_nm": 2.0, "dy_nm": 1.0, "dz_nm": 1.5, "pivot_a_nm": 30.0, "pivot_y_nm": 10.0, "pivot_z_nm": 18.0}
    A, Y, Z = np.meshgrid(np.arange(na) * 2.0, np.arange(ny) * 1.0, np.arange(nz) * 1.5, indexing="ij")
    c = np.array([0.3, -1.1, 0.7])
    vol = 5.0 + c[0] * A + c[1] * Y + c[2] * Z
    g = grid(10, 8, 8, d=(1.0, 1.0, 1.0))
    lab_pivot = (5.0, 4.0, 4.0)
    pitch, yaw = 0.05, 0.2
    d, _ = O.rotate_object(g, lab_pivot, s, pitch, yaw, vol, vol)
    M = O.rotation_matrix(pitch, yaw)
    S, J, L = np.meshgrid(np.arange(10) * 1.0, np.arange(8) * 1.0, np.arange(8) * 1.0, indexing="ij")
    u = np.stack([S - lab_pivot[0], J - lab_pivot[1], L - lab_pivot[2]])
    v = np.einsum("ij,j...->i...", M, u) + np.array([30.0, 10.0, 18.0])[:, None, None, None]
    ref = 5.0 + c[0] * v[0] + c[1] * v[1] + c[2] * v[2]
    assert np.allclose(d, ref, atol=1e-9)


def test_quarter_yaw_permutes_axes():
    # yaw 90 deg: lab column z samples sample position a' = -z, and lab slice a samples z' = a
    rng = np.random.default_rng(2)
    vol = rng.random((8, 3, 8))
    s = {"da_nm": 1.0, "dy_nm": 1.0, "dz_nm": 1.0, "pivot_a_nm": 7.0, "pivot_y_nm": 0.0, "pivot_z_nm": 0.0}
    g = grid(8, 3, 8, d=(1.0, 1.0, 1.0))
    d, _ = O.rotate_object(g, (0.0, 0.0, 0.0), s, 0.0, math.pi / 2, vol, vol)
    ref = np.transpose(vol, (2, 1, 0))[:, :, ::-1]      # d[a, y, z] = vol[7 - z, y, a]
    assert np.allclose(d, ref, atol=1e-9)

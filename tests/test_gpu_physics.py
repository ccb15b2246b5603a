"""Physics on the HIP path itself: total external reflection from a flat substrate.

The paraxial multislice model of a flat substrate reflects a grazing beam
with the Fresnel reflectivity (the continuum limit of its own equations):
r = (a - sqrt(a^2 - 2 delta + 2 i beta)) / (a + sqrt(...)).  A Gaussian beam
300 nm above a 7.6e-6 / 1.7e-7 substrate, propagated by the library until the
reflected beam has separated, must put the Fresnel fraction of its power
above the horizon of the detector (averaged over the beam's angular spread).
The substrate is z- and x-uniform, so it is one pool slice in the batched
entry point.
"""
import math

import numpy as np
import pytest

from oracle import msl_oracle as O
from paper_2212_01253_amd import synth

pytestmark = pytest.mark.gpu

SUB_D, SUB_B = 7.6e-6, 1.7e-7


class Repeat:
    """A slice stack whose every slice is the same 2-D map."""

    def __init__(self, arr):
        self.arr = arr

    def __getitem__(self, s):
        return self.arr


def fresnel(a, d, b):
    s = np.sqrt(a.astype(np.complex128) ** 2 - 2 * d + 2j * b)
    return np.abs((a - s) / (a + s)) ** 2


def fresnel_averaged(alpha, w0, k):
    sig = 2.0 / (k * w0)
    t = np.linspace(-4 * sig, 4 * sig, 801)
    wgt = np.exp(-2 * (t / sig) ** 2)
    return float(np.sum(fresnel(alpha + t, SUB_D, SUB_B) * wgt) / np.sum(wgt))


@pytest.fixture(scope="module")
def M():   # the binding module
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2212_01253_amd import msl
    msl.lib()
    return msl


@pytest.mark.parametrize("alpha_deg", [0.12, 0.18, 0.21, 0.24, 0.30])
def test_fresnel_reflectivity_on_the_gpu(M, alpha_deg):
    import torch
    ny, nz, dy, dx, lam, w0, h0 = 1024, 16, 2.0, 50.0, 0.1, 150.0, 300.0
    a = math.radians(alpha_deg)
    k = 2 * math.pi / lam
    ns = int(math.ceil((2 * h0 + 3 * w0) / math.tan(a) / dx))
    g = synth.Geometry(ny, nz, ns, dy, 1.0, dx, lam, a, 0)
    half = ny // 2
    d = np.zeros((1, ny, nz), np.float32)
    b = np.zeros((1, ny, nz), np.float32)
    d[0, :half] = SUB_D
    b[0, :half] = SUB_B
    sponge = 128   # absorbing layer at the bottom keeps the refracted beam from wrapping round
    b[0, :sponge] += (1e-4 * np.cos(0.5 * math.pi * np.arange(sponge) / sponge) ** 2)[:, None].astype(np.float32)
    probe = synth.gaussian_probe(g, w0, half * dy + h0)
    dev = lambda x: torch.from_numpy(np.ascontiguousarray(x)).cuda()
    item = {"geom": g, "pool_delta": dev(d), "pool_beta": dev(b), "slice_index": dev(np.zeros(ns, np.int32)),
            "probe": dev(probe), "field": torch.empty((ny, nz), dtype=torch.complex64, device="cuda"),
            "intensity": torch.empty((ny, nz), dtype=torch.float32, device="cuda")}
    M.forward_batch([item])
    torch.cuda.synchronize()
    I = item["intensity"].cpu().numpy().astype(np.float64)   # fftshifted: the z-uniform beam is in column nz/2
    R = float(I[half + 1:].sum() / np.sum(np.abs(probe.astype(np.complex128)) ** 2))
    RF = fresnel_averaged(a, w0, k)
    # the same run in the FP64 oracle (one column: the stack is z-uniform)
    g1 = synth.Geometry(ny, 1, ns, dy, 1.0, dx, lam, a, 0)
    psi_in = probe[:, :1].astype(np.complex128)
    psi = O.forward(g1, Repeat(d[0, :, :1].astype(np.float64)), Repeat(b[0, :, :1].astype(np.float64)), psi_in)
    I1 = O.far_field(g1, psi)[:, 0]
    R1 = float(I1[half + 1:].sum() / np.sum(np.abs(probe[:, 0].astype(np.complex128)) ** 2))
    print(f"alpha {alpha_deg} deg: {ns} slices, R {R:.4f}, oracle {R1:.4f}, Fresnel {RF:.4f}")
    assert abs(R - R1) < 1e-3
    # measured: |R - Fresnel| <= 0.0073 (at 0.24 deg, on the steep edge above the critical angle)
    assert abs(R - RF) < 0.02


def test_object_rotation_matches_the_oracle(M):
    import torch
    rng = np.random.default_rng(3)
    s = {"na": 40, "ny": 30, "nz": 20, "da_nm": 5.0, "dy_nm": 1.0, "dz_nm": 1.5,
         "pivot_a_nm": 100.0, "pivot_y_nm": 12.0, "pivot_z_nm": 15.0}
    d_s = rng.random((40, 30, 20)).astype(np.float32)
    b_s = rng.random((40, 30, 20)).astype(np.float32)
    g = synth.Geometry(32, 16, 48, 1.0, 1.0, 4.0, 0.1, 0.0, 0)
    lab_pivot = (96.0, 14.0, 8.0)
    for pitch, yaw in [(0.0, 0.0), (0.02, 0.0), (0.01, 0.3), (-0.05, -1.0)]:
        dev = lambda x: torch.from_numpy(np.ascontiguousarray(x)).cuda()
        dl, bl = M.rotate_object(g, lab_pivot, s, pitch, yaw, dev(d_s), dev(b_s))
        torch.cuda.synchronize()
        rd, rb = O.rotate_object(g, lab_pivot, s, pitch, yaw, d_s, b_s)
        # float32 positions and weights: agreement to ~1e-5 of the unit-range values
        assert np.max(np.abs(dl.cpu().numpy() - rd)) <= 2e-5, (pitch, yaw)
        assert np.max(np.abs(bl.cpu().numpy() - rb)) <= 2e-5, (pitch, yaw)
        assert np.any(rd > 0) and np.any(rd == 0)   # the sample covers part of the lab box


@pytest.mark.parametrize("alpha_deg", [0.12, 0.18, 0.24, 0.30])
def test_fresnel_reflectivity_with_the_object_tilted(M, alpha_deg):
    """Eq. 2-3 taken literally: a straight Gaussian beam and the flat substrate pitched by the
    incidence angle (msl_rotate_object) reflect the Fresnel fraction too, into the specular
    direction 2 alpha above the direct beam (the beam-tilt reading gives the same physics)."""
    import torch
    ny, nz, dy, dx, lam, w0, h0 = 1024, 16, 2.0, 50.0, 0.1, 75.0, 150.0
    a = math.radians(alpha_deg)
    k = 2 * math.pi / lam
    ns = int(math.ceil((2 * h0 + 3 * w0) / math.tan(a) / dx))
    g = synth.Geometry(ny, nz, ns, dy, 1.0, dx, lam, 0.0, 0)
    # the sample: a substrate below y' = 2000 nm, uniform along the beam and across (two voxels
    # a billion nm apart along those axes); lab row 300 nm is the surface at the first slice
    nys = 1600
    sd = np.zeros((2, nys, 2), np.float32)
    sb = np.zeros_like(sd)
    sd[:, :1000] = SUB_D
    sb[:, :1000] = SUB_B
    s = {"na": 2, "ny": nys, "nz": 2, "da_nm": 1e9, "dy_nm": dy, "dz_nm": 1e9,
         "pivot_a_nm": 0.0, "pivot_y_nm": 2000.0, "pivot_z_nm": 0.0}
    dev = lambda x: torch.from_numpy(np.ascontiguousarray(x)).cuda()
    D, B = M.rotate_object(g, (0.0, 300.0, 0.0), s, a, 0.0, dev(sd), dev(sb))
    sponge = 128   # lab-frame absorbing rows: the refracted beam must not wrap round
    ramp = (1e-4 * np.cos(0.5 * math.pi * np.arange(sponge) / sponge) ** 2).astype(np.float32)
    B[:, :sponge, :] += dev(ramp).view(1, sponge, 1)
    probe = synth.gaussian_probe(g, w0, 300.0 + h0)
    f, _ = M.forward(g, D, B, dev(probe))
    I = M.far_field(g, f).cpu().numpy().astype(np.float64)
    m = k * math.sin(a) * ny * dy / (2 * math.pi)     # rows between the direct and the tilt direction
    R = float(I[int(round(ny // 2 + m)) + 1:].sum() / np.sum(np.abs(probe.astype(np.complex128)) ** 2))
    RF = fresnel_averaged(a, w0, k)
    peak = int(np.argmax(I.sum(axis=1)))
    print(f"alpha {alpha_deg} deg: R {R:.4f}, Fresnel {RF:.4f}, brightest row {peak}, specular {ny // 2 + 2 * m:.1f}")
    # measured |R - Fresnel| <= 0.0065
    assert abs(R - RF) < 0.02
    if RF > 0.5:
        assert abs(peak - (ny // 2 + 2 * m)) <= 6

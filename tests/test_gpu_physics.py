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
def M():
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

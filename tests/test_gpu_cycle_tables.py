"""The paraxial passes' single-float32 constants, read back from the workspace after a forward
call and checked against their definition.  Every twiddle W_n^e = exp(-2 pi i e / n) and every
one-axis propagator factor exp(i dx q^2 / 2k) / n (q = 2 pi f / (n d), f the signed DFT bin) is
stored as a cycle of 64 rows; each entry must be one of the two float32 neighbours of the exact
value (the value itself when float32 holds it), and over the cycle every running sum of an
entry's rounding errors must stay within half an ulp (a first-order sigma-delta order of the two
neighbours), so that the errors cancel over 64 passes instead of adding up with the slice count.

The table regions are found from the workspace layout: the 8 KiB status and barrier area at
offset 0, then the [64][nz] twiddles of rows (W_nz), [64][ny] of columns, and the propagator
factors of rows and columns, each region 256-byte aligned.
"""
import math

import numpy as np
import pytest

from paper_2212_01253_amd import synth

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

CYCLE = 64


def up(n):
    return (n + 255) // 256 * 256


def neighbours(c):
    """Float32 values just below and just above each FP64 value (equal when float32 holds it)."""
    f = c.astype(np.float32)
    lo = np.where(f.astype(np.float64) <= c, f, np.nextafter(f, np.float32(-np.inf)))
    hi = np.where(f.astype(np.float64) >= c, f, np.nextafter(f, np.float32(np.inf)))
    return lo.astype(np.float64), hi.astype(np.float64)


def check_cycle(table, exact, what):
    """table float32 [CYCLE][n] (one component), exact float64 [n]."""
    t = table.astype(np.float64)
    # values within FP64 rounding of 0 or +-1 are those (cos(pi/2) evaluates to 6e-17 in FP64;
    # the library's tables take sin and cos of pi times the exact fraction)
    exact = np.where(np.abs(exact) <= 1e-15, 0.0, exact)
    exact = np.where(np.abs(np.abs(exact) - 1.0) <= 1e-15, np.sign(exact), exact)
    lo, hi = neighbours(exact)
    ok = (t == lo) | (t == hi)
    assert ok.all(), f"{what}: entries that are not float32 neighbours of the exact value: {np.argwhere(~ok)[:5]}"
    ulp = hi - lo
    run = np.cumsum(t - exact, axis=0)
    rep = ulp == 0
    assert np.all(run[:, rep] == 0), f"{what}: a representable value changes along the cycle"
    worst = np.max(np.abs(run[:, ~rep]) / ulp[~rep])
    assert worst <= 0.5 + 1e-9, f"{what}: running error sum reaches {worst:.3f} ulp"
    # hence the cycle's mean is within 1/128 ulp of the exact value (round to nearest: up to 1/2)
    assert np.all(np.abs(t.mean(axis=0) - exact)[~rep] <= ulp[~rep] / (2 * CYCLE) * (1 + 1e-9))
    return worst


@pytest.mark.parametrize("ny,nz", [(64, 128), (256, 32)])
def test_cycle_tables_hold_sigma_delta_orders_of_the_exact_constants(ny, nz):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2212_01253_amd import msl
    g = synth.Geometry(ny, nz, 6, dy_nm=1.0, dz_nm=1.3, dx_nm=7.0, wavelength_nm=0.11,
                       alpha_i_rad=math.radians(0.2))
    d = torch.zeros((6, ny, nz), dtype=torch.float32, device="cuda")
    b = torch.zeros_like(d)
    ws = msl.workspace(g, 0)
    msl.forward(g, d, b, ws=ws)
    torch.cuda.synchronize()
    raw = ws.cpu().numpy()
    off = up(8192)
    regions = {}
    for name, n in (("twz", nz), ("twy", ny), ("hz", nz), ("hy", ny)):
        size = CYCLE * n * 8
        regions[name] = raw[off:off + size].view(np.float32).reshape(CYCLE, n, 2)
        off += up(size)
    k = 2 * math.pi / g.wavelength_nm
    for name, n, pitch in (("twz", nz, None), ("twy", ny, None), ("hz", nz, g.dz_nm), ("hy", ny, g.dy_nm)):
        e = np.arange(n)
        if pitch is None:
            z = np.exp(-2j * np.pi * e / n)
        else:
            f = np.where(e < n // 2, e, e - n)
            q = 2 * np.pi * f / (n * pitch)
            z = np.exp(1j * g.dx_nm * q * q / (2 * k)) / n
        wr = check_cycle(regions[name][:, :, 0], z.real, name + " real")
        wi = check_cycle(regions[name][:, :, 1], z.imag, name + " imaginary")
        print(f"{name}: largest running error {max(wr, wi):.3f} ulp")

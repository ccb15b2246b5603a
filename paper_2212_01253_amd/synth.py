"""Seeded synthetic inputs for the multislice forward model.

This module only draws inputs: slice stacks of slice-averaged refractive
index decrements (delta) and absorption indices (beta), measured amplitudes
and geometry records.  It holds none of the multislice arithmetic, so the
FP64 oracle and the HIP path can both consume what it produces without
sharing any computation.

The paper's samples (Table 1 of arXiv 2212.01253) are elongated bars on a
substrate: much longer along the beam than wide, and only tens of nanometres
high.  Its experimental images are not public (Data availability), so these
generators stand in for them with the same structure: a substrate slab in the
low rows (row 0 is the deepest substrate row), and rectangular bars and lines
on top, each a box in (x = slice index, y = row, z = column).

All random draws use ``numpy.random.Generator(PCG64(seed))``; values are drawn
in float64 and handed out as float32, which is what both sides compute from.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, asdict, field

import numpy as np

# Optical constants used by the synthetic workloads (not printed by the paper;
# typical hard-X-ray values for a Si-like substrate and an Au-like pattern).
SUBSTRATE_DELTA = 7.6e-6
SUBSTRATE_BETA = 1.7e-7
BAR_DELTA = 1.5e-5
BAR_BETA = 1.0e-6


@dataclass
class Geometry:
    """Grid and beam parameters of one multislice run (lengths in nm, angles in rad)."""

    ny: int
    nz: int
    n_slices: int
    dy_nm: float = 1.0
    dz_nm: float = 1.0
    dx_nm: float = 10.0
    wavelength_nm: float = 0.1
    alpha_i_rad: float = 0.0
    propagator: int = 0  # 0 = paraxial (Fresnel), 1 = exact angular spectrum

    def as_dict(self):
        return asdict(self)


@dataclass
class Workload:
    geom: Geometry
    delta: np.ndarray  # float32 [Ns][Ny][Nz]
    beta: np.ndarray   # float32 [Ns][Ny][Nz]
    seed: int
    name: str
    meta: dict = field(default_factory=dict)


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def _fill_box(arr, x0, x1, y0, y1, z0, z1, value):
    arr[x0:x1, y0:y1, z0:z1] = value


def _draw_features(geom: Geometry, seed: int, *, substrate_rows: int,
                   n_bars=(3, 8), bar_height=(5, 20), bar_width=(2, 16),
                   bar_len_frac=(0.25, 1.0), n_lines=(0, 0),
                   line_height=(2, 40), line_width=(1, 4),
                   delta_range=None, beta_over_delta=None,
                   bar_delta=BAR_DELTA, bar_beta=BAR_BETA):
    """The seeded feature list: (kind, x0, length, y0, y1, z0, width, delta, beta) boxes in draw order."""
    ny, nz, ns = geom.ny, geom.nz, geom.n_slices
    rng = _rng(seed)
    y_base = substrate_rows
    feats = []

    def feature_values():
        if delta_range is None:
            return float(bar_delta), float(bar_beta)
        d = float(rng.uniform(delta_range[0], delta_range[1]))
        return d, d * float(beta_over_delta)

    nb = int(rng.integers(n_bars[0], n_bars[1] + 1))
    for _ in range(nb):
        h = int(rng.integers(bar_height[0], bar_height[1] + 1))
        w = int(rng.integers(bar_width[0], min(bar_width[1], nz) + 1))
        lo = max(1, int(math.ceil(bar_len_frac[0] * ns)))
        hi = max(lo, int(math.floor(bar_len_frac[1] * ns)))
        ln = int(rng.integers(lo, hi + 1))
        z0 = int(rng.integers(0, nz - w + 1))
        x0 = int(rng.integers(0, ns - ln + 1))
        y1 = min(ny, y_base + h)
        d, b = feature_values()
        feats.append(("bar", x0, ln, y_base, y1, z0, w, d, b))
    nl = int(rng.integers(n_lines[0], n_lines[1] + 1)) if n_lines[1] > 0 else 0
    for _ in range(nl):
        h = int(rng.integers(line_height[0], line_height[1] + 1))
        w = int(rng.integers(line_width[0], min(line_width[1], nz) + 1))
        z0 = int(rng.integers(0, nz - w + 1))
        y1 = min(ny, y_base + h)
        d, b = feature_values()
        feats.append(("line", 0, ns, y_base, y1, z0, w, d, b))
    return feats


def _render_slice(geom, substrate_rows, substrate, feats, x):
    """delta, beta of slice x (float32 [ny][nz]): substrate, then the features covering x in order."""
    d = np.zeros((geom.ny, geom.nz), np.float32)
    b = np.zeros((geom.ny, geom.nz), np.float32)
    d[:substrate_rows] = np.float32(substrate[0])
    b[:substrate_rows] = np.float32(substrate[1])
    for (_, x0, ln, y0, y1, z0, w, fd, fb) in feats:
        if x0 <= x < x0 + ln:
            d[y0:y1, z0:z0 + w] = np.float32(fd)
            b[y0:y1, z0:z0 + w] = np.float32(fb)
    return d, b


def bars_on_substrate(geom: Geometry, seed: int, *, substrate_rows: int,
                      substrate=(SUBSTRATE_DELTA, SUBSTRATE_BETA), **kw) -> Workload:
    """Substrate slab plus seeded rectangular bars (and optional full-length lines).

    Integer ranges are inclusive.  When ``delta_range`` is given every feature
    draws its own delta uniformly in that range and beta = delta * beta_over_delta;
    otherwise all features use (bar_delta, bar_beta).  Later features overwrite
    earlier ones where they overlap.  Bars start at the substrate surface row.
    """
    feats = _draw_features(geom, seed, substrate_rows=substrate_rows, **kw)
    ns, ny, nz = geom.n_slices, geom.ny, geom.nz
    delta = np.zeros((ns, ny, nz), np.float32)
    beta = np.zeros((ns, ny, nz), np.float32)
    delta[:, :substrate_rows, :] = np.float32(substrate[0])
    beta[:, :substrate_rows, :] = np.float32(substrate[1])
    for (_, x0, ln, y0, y1, z0, w, fd, fb) in feats:
        _fill_box(delta, x0, x0 + ln, y0, y1, z0, z0 + w, np.float32(fd))
        _fill_box(beta, x0, x0 + ln, y0, y1, z0, z0 + w, np.float32(fb))
    return Workload(geom, delta, beta, seed, "bars", {"features": feats})


@dataclass
class CompactStack:
    """A slice stack as a pool of distinct slices plus the pool index of every slice."""
    geom: Geometry
    pool_delta: np.ndarray   # float32 [n_unique][ny][nz]
    pool_beta: np.ndarray
    index: np.ndarray        # int32 [n_slices]
    seed: int
    name: str

    def dense(self):
        return self.pool_delta[self.index], self.pool_beta[self.index]


def compact_bars_on_substrate(geom: Geometry, seed: int, *, substrate_rows: int,
                              substrate=(SUBSTRATE_DELTA, SUBSTRATE_BETA), **kw) -> CompactStack:
    """The stack of ``bars_on_substrate`` (same draws) without materialising it: the features
    are boxes along the beam, so the slice content changes only where a box starts or ends."""
    feats = _draw_features(geom, seed, substrate_rows=substrate_rows, **kw)
    ns = geom.n_slices
    cuts = sorted({0, ns} | {x0 for f in feats for x0 in (f[1],)} | {f[1] + f[2] for f in feats})
    cuts = [c for c in cuts if 0 <= c <= ns]
    pd, pb = [], []
    index = np.zeros(ns, np.int32)
    for a, b in zip(cuts[:-1], cuts[1:]):
        d, bb = _render_slice(geom, substrate_rows, substrate, feats, a)
        index[a:b] = len(pd)
        pd.append(d)
        pb.append(bb)
    return CompactStack(geom, np.stack(pd), np.stack(pb), index, seed, "bars")


def parity_small(seed: int = 0) -> Workload:
    """64x64 grid, 128 slices of 10 nm, 0.1 nm wavelength, 0.2 deg incidence.

    Substrate in rows 0..23 (delta 7.6e-6, beta 1.7e-7); 3..8 bars of height
    5..20 px, width 2..16 px and length Ns/4..Ns slices (delta 1.5e-5, beta 1e-6).
    """
    g = Geometry(64, 64, 128, 1.0, 1.0, 10.0, 0.1, math.radians(0.2), 0)
    w = bars_on_substrate(g, seed, substrate_rows=24)
    w.name = "parity_64x64x128"
    return w


def throughput_512(seed: int = 2212, n_slices: int = 2048, n: int = 512) -> Workload:
    """512x512 grid, 2048 slices of 5 nm, 0.1 nm wavelength, incidence U[0.1, 0.4] deg.

    Substrate in the lower quarter of the rows; 8..32 bars (height 2..40,
    width 4..64, length Ns/8..Ns) and 2..8 full-length lines (height 2..40,
    width 1..4), each feature with delta U[5e-6, 3e-5] and beta = delta/20.
    ``n_slices`` and ``n`` exist so tests can draw the same kind of stack at
    reduced size; the throughput workload uses the defaults.
    """
    rng = _rng(seed)
    alpha = math.radians(float(rng.uniform(0.1, 0.4)))
    g = Geometry(n, n, n_slices, 1.0, 1.0, 5.0, 0.1, alpha, 0)
    w = bars_on_substrate(g, seed + 1, substrate_rows=n // 4, n_bars=(8, 32),
                          bar_height=(2, 40), bar_width=(4, 64),
                          bar_len_frac=(1.0 / 8.0, 1.0), n_lines=(2, 8),
                          line_height=(2, 40), line_width=(1, 4),
                          delta_range=(5e-6, 3e-5), beta_over_delta=1.0 / 20.0)
    w.name = f"bars_{n}x{n}x{n_slices}"
    w.seed = seed   # the workload's seed (incidence draw; the features use seed + 1)
    return w


def recon_256(seed: int = 4242, n_slices: int = 1024, n: int = 256) -> Workload:
    """256x256 grid, 1024 slices of 5 nm, 0.1 nm, 0.2 deg: the gradient workload.

    The pattern occupies the 64 rows above a substrate of Ny/4 rows; beta = delta/20.
    """
    g = Geometry(n, n, n_slices, 1.0, 1.0, 5.0, 0.1, math.radians(0.2), 0)
    w = bars_on_substrate(g, seed, substrate_rows=n // 4, n_bars=(8, 32),
                          bar_height=(2, 40), bar_width=(4, 64),
                          bar_len_frac=(1.0 / 8.0, 1.0), n_lines=(2, 8),
                          line_height=(2, 40), line_width=(1, 4),
                          delta_range=(5e-6, 3e-5), beta_over_delta=1.0 / 20.0)
    w.name = f"recon_{n}x{n}x{n_slices}"
    return w


def random_stack(ny, nz, ns, seed, delta_scale=1e-5, beta_scale=5e-7):
    """Dense random slice stack (uniform [0, scale)), float32."""
    rng = _rng(seed)
    d = (rng.random((ns, ny, nz)) * delta_scale).astype(np.float32)
    b = (rng.random((ns, ny, nz)) * beta_scale).astype(np.float32)
    return d, b


def random_field(ny, nz, seed, scale=1.0):
    """Random complex64 field with standard-normal real and imaginary parts."""
    rng = _rng(seed)
    return ((rng.standard_normal((ny, nz)) + 1j * rng.standard_normal((ny, nz)))
            * scale).astype(np.complex64)


def random_measured_amplitude(ny, nz, seed, scale=1.0):
    """Non-negative float32 amplitudes (a stand-in for sqrt of detector counts)."""
    rng = _rng(seed)
    return (np.abs(rng.standard_normal((ny, nz))) * scale).astype(np.float32)


# ---------------------------------------------------------------------------
# reconstruction workload inputs

def pattern_region(geom: Geometry, substrate_rows: int, height: int, beta_over_delta: float = 1.0 / 20.0) -> dict:
    """Box of unknown voxels: all slices and columns, `height` rows above the substrate."""
    return {"s0": 0, "ns": geom.n_slices, "y0": substrate_rows, "ny": height, "z0": 0, "nz": geom.nz,
            "beta_over_delta": beta_over_delta}


def known_stack(w: Workload, region: dict):
    """The workload's stacks with the unknown box zeroed (what the reconstruction knows)."""
    d, b = w.delta.copy(), w.beta.copy()
    ix = (slice(region["s0"], region["s0"] + region["ns"]), slice(region["y0"], region["y0"] + region["ny"]),
          slice(region["z0"], region["z0"] + region["nz"]))
    d[ix] = 0
    b[ix] = 0
    return d, b


def box_values(w: Workload, region: dict) -> np.ndarray:
    """Ground-truth delta on the box, float32 [ns][ny][nz]."""
    return np.ascontiguousarray(w.delta[region["s0"]:region["s0"] + region["ns"],
                                        region["y0"]:region["y0"] + region["ny"],
                                        region["z0"]:region["z0"] + region["nz"]])


def random_init(region: dict, seed: int, hi: float = 3e-5) -> np.ndarray:
    """Plain initial guess: delta ~ U[0, hi) on the box, float32."""
    return (_rng(seed).random((region["ns"], region["ny"], region["nz"])) * hi).astype(np.float32)


def poisson_counts(intensity: np.ndarray, total: float, seed: int):
    """Detector counts Poisson(s I) with s = total / sum(I); returns (counts float32, s)."""
    I = np.asarray(intensity, np.float64)
    s = float(total) / float(I.sum())
    return _rng(seed).poisson(s * I).astype(np.float32), s


def fd_voxels(region: dict, n: int, seed: int) -> np.ndarray:
    """n distinct random voxel indices (s, y, z) inside the box."""
    rng = _rng(seed)
    size = region["ns"] * region["ny"] * region["nz"]
    flat = rng.choice(size, size=n, replace=False)
    return np.stack(np.unravel_index(flat, (region["ns"], region["ny"], region["nz"])), axis=1)


# ---------------------------------------------------------------------------
# batched workload: many instances of the throughput generator

GRID_CHOICES = (128, 256, 512, 1024)


def batch_instance(seed: int, grids=GRID_CHOICES, ns_range=(256, 4096), alpha_deg=(0.05, 0.5),
                   wavelength_nm=(0.08, 0.15)) -> CompactStack:
    """One instance of the batched workload: grid N from `grids`, Ns ~ U{ns_range}, incidence and
    wavelength uniform in their ranges, 1 nm pixels, 5 nm slices, and the throughput workload's
    bars and lines with heights and widths scaled by N / 512 over a substrate of N/4 rows."""
    rng = _rng(seed)
    n = int(grids[int(rng.integers(0, len(grids)))])
    ns = int(rng.integers(ns_range[0], ns_range[1] + 1))
    alpha = math.radians(float(rng.uniform(*alpha_deg)))
    lam = float(rng.uniform(*wavelength_nm))
    g = Geometry(n, n, ns, 1.0, 1.0, 5.0, lam, alpha, 0)
    f = n / 512.0
    sc = lambda lo, hi: (max(1, int(round(lo * f))), max(1, int(round(hi * f))))
    cs = compact_bars_on_substrate(g, seed + 1, substrate_rows=n // 4, n_bars=(8, 32),
                                   bar_height=sc(2, 40), bar_width=sc(4, 64),
                                   bar_len_frac=(1.0 / 8.0, 1.0), n_lines=(2, 8),
                                   line_height=sc(2, 40), line_width=sc(1, 4),
                                   delta_range=(5e-6, 3e-5), beta_over_delta=1.0 / 20.0)
    cs.name = f"batch_{n}x{n}x{ns}"
    return cs


def batch_workload(n_instances: int = 96, base_seed: int = 1000, **kw):
    """The batched workload: instances seeded base_seed + i."""
    return [batch_instance(base_seed + i, **kw) for i in range(n_instances)]


def gaussian_probe(geom: Geometry, waist_nm: float, center_nm: float) -> np.ndarray:
    """Gaussian beam entering tilted by the incidence angle (the paper's Gaussian probe):
    exp(-((y - yc) / w)^2) exp(+i k sin(alpha) (y - yc)), uniform along z; complex64 [ny][nz]."""
    y = np.arange(geom.ny) * geom.dy_nm
    k = 2.0 * math.pi / geom.wavelength_nm
    p = np.exp(-((y - center_nm) / waist_nm) ** 2) * np.exp(1j * k * math.sin(geom.alpha_i_rad) * (y - center_nm))
    return np.repeat(p[:, None], geom.nz, axis=1).astype(np.complex64)


def bar_boxes(geom: Geometry, seed: int, *, substrate_rows: int, **kw):
    """The feature boxes of ``compact_bars_on_substrate`` (same draws) without rendering:
    (boxes float32 [nf][8] = x0, x1, y0, y1, z0, z1, delta, beta; cuts int32 [n_pool + 1],
    pool slice u covering slices [cuts[u], cuts[u + 1]))."""
    feats = _draw_features(geom, seed, substrate_rows=substrate_rows, **kw)
    ns = geom.n_slices
    cuts = sorted({0, ns} | {f[1] for f in feats} | {f[1] + f[2] for f in feats})
    cuts = [c for c in cuts if 0 <= c <= ns]
    boxes = np.array([[x0, x0 + ln, y0, y1, z0, z0 + w, d, b] for (_, x0, ln, y0, y1, z0, w, d, b) in feats],
                     np.float32).reshape(-1, 8)
    return boxes, np.array(cuts, np.int32)


def training_sample(seed: int, n: int = 256, n_slices: int = 1024, alpha_deg=(0.1, 0.4)):
    """One training sample of the learned initialiser: the reconstruction workload's generator
    (``recon_256``: bars and lines over an n/4-row substrate, 5 nm slices, 0.1 nm) on an n x n grid
    at a random incidence in alpha_deg; returns (geometry, boxes, cuts)."""
    rng = _rng(seed)
    alpha = math.radians(float(rng.uniform(*alpha_deg)))
    g = Geometry(n, n, n_slices, 1.0, 1.0, 5.0, 0.1, alpha, 0)
    boxes, cuts = bar_boxes(g, seed + 1, substrate_rows=n // 4, n_bars=(8, 32), bar_height=(2, 40),
                            bar_width=(4, 64), bar_len_frac=(1.0 / 8.0, 1.0), n_lines=(2, 8),
                            line_height=(2, 40), line_width=(1, 4), delta_range=(5e-6, 3e-5),
                            beta_over_delta=1.0 / 20.0)
    return g, boxes, cuts

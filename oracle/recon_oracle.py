"""FP64 CPU oracle for the reconstruction step (arXiv 2212.01253, Sec. 4.1).

TEST INFRASTRUCTURE ONLY, like ``msl_oracle``: only the test-suite, the
package smoke check and the benchmark's ``cpu_baseline`` leg may import it.
It shares no code with the HIP path.

What it computes:

* The unknowns of a reconstruction are the delta values of the voxels in one
  box of the slice stack; beta is tied to delta by a fixed ratio (the
  workloads use beta = delta / 20), and every voxel outside the box is known.
  ``region_loss_and_gradient`` evaluates the amplitude loss of Eq. (4) for a
  box parameter vector and its gradient by the chain rule through that tie:
  dL/dtheta = dL/ddelta + ratio * dL/dbeta on the box.
* The paper minimises that loss with the ADAM optimiser (Sec. 4.1, citing
  Kingma and Ba 2014).  ``adam_step`` is ADAM as published there (first and
  second moment estimates, bias correction, step lr * mhat / (sqrt(vhat) + eps)),
  followed by a clamp of the parameters to a box [lo, hi] (delta >= 0 is the
  physical range of an index decrement of these materials).
* ``snap``: the paper's nearest-refractive-index filter on the parameters.
* ``shrinkwrap``: the shrink-wrap support (Marchesini et al. 2003, cited in
  Sec. 4.1): blur |theta| with a Gaussian, keep what exceeds a fraction of
  the largest blurred value.
* ``poisson_loss_scale``: the detector model of the reconstruction workload
  compares sqrt(s * I) with sqrt(counts) for the fixed photon scale s; that
  loss is s times the amplitude loss of I against sqrt(counts / s).
"""
from __future__ import annotations

import numpy as np

from . import msl_oracle as O


def box_slices(region):
    """numpy index of the box inside a [n_slices][ny][nz] stack."""
    g = (lambda k: region[k]) if isinstance(region, dict) else (lambda k: getattr(region, k))
    s0, ns, y0, ny, z0, nz = (int(g(k)) for k in ("s0", "ns", "y0", "ny", "z0", "nz"))
    return (slice(s0, s0 + ns), slice(y0, y0 + ny), slice(z0, z0 + nz))


def ratio_of(region):
    return float(region["beta_over_delta"] if isinstance(region, dict) else region.beta_over_delta)


def scatter(known_delta, known_beta, region, theta):
    """Stacks with the box set to delta = theta, beta = ratio * theta (float64 copies)."""
    d = np.array(known_delta, np.float64)
    b = np.array(known_beta, np.float64)
    ix = box_slices(region)
    d[ix] = theta
    b[ix] = ratio_of(region) * np.asarray(theta, np.float64)
    return d, b


def region_loss_and_gradient(geom, known_delta, known_beta, region, theta, measured_amp, probe=None):
    """(L, dL/dtheta) for the amplitude loss with the box parameters theta."""
    d, b = scatter(known_delta, known_beta, region, theta)
    L, gd, gb, _, _, _ = O.loss_and_gradient(geom, d, b, measured_amp, probe)
    ix = box_slices(region)
    return L, gd[ix] + ratio_of(region) * gb[ix]


def adam_step(theta, grad, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8, lo=-np.inf, hi=np.inf):
    """One ADAM step (t >= 1 is the step count after this update); returns new (theta, m, v)."""
    g = np.asarray(grad, np.float64)
    m = beta1 * np.asarray(m, np.float64) + (1.0 - beta1) * g
    v = beta2 * np.asarray(v, np.float64) + (1.0 - beta2) * g * g
    mhat = m / (1.0 - beta1 ** t)
    vhat = v / (1.0 - beta2 ** t)
    theta = np.asarray(theta, np.float64) - lr * mhat / (np.sqrt(vhat) + eps)
    return np.clip(theta, lo, hi), m, v


def poisson_loss_scale(counts, scale):
    """Measured amplitudes for msl amplitude loss: sqrt(counts / s); the detector loss is s times it."""
    return np.sqrt(np.asarray(counts, np.float64) / scale)


def snap(theta, levels):
    """Nearest-value filter (Sec. 4.1): every parameter becomes the nearest of `levels`.

    Distances are taken in float32, the precision in which the library decides; on a tie the
    lower level index wins."""
    t = np.asarray(theta, np.float32)[..., None]
    lv = np.asarray(levels, np.float32)
    return lv[np.argmin(np.abs(t - lv), axis=-1)]


def shrinkwrap(theta, sigmas, threshold):
    """(theta with zeros outside the support, blurred |theta|) for the shrink-wrap support."""
    from scipy.ndimage import gaussian_filter1d
    b = np.abs(np.asarray(theta, np.float64))
    for axis, sg in enumerate(sigmas):
        if sg > 0:
            b = gaussian_filter1d(b, sg, axis=axis, mode="constant", cval=0.0, truncate=3.0)
    keep = b > threshold * b.max()
    return np.where(keep, theta, 0.0), b

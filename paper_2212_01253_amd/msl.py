"""ctypes binding of libmsl (C ABI in include/msl.h) plus autograd wrappers.

Argument marshalling only: every step of the multislice path runs in the HIP
library.  PyTorch provides device memory (tensors, the workspace) and the
stream (``torch.cuda.current_stream()``).  If ``libmsl.so`` is missing the
first call raises; there is no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import c_double, c_int32, c_size_t, c_void_p

import torch

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libmsl.so")

OK, ERR_ARG, ERR_UNSUPPORTED, ERR_WORKSPACE, ERR_HIP = 0, -1, -2, -3, -4
REUSE_SLICE_PACK = 1
PROP_PARAXIAL, PROP_EXACT = 0, 1
SCHED_AUTO, SCHED_PER_PASS, SCHED_PERSISTENT = 0, 1, 2

EXPORTS = ("msl_abi_version", "msl_workspace_bytes", "msl_checkpoint_count", "msl_pack_slices", "msl_forward",
           "msl_far_field", "msl_amp_loss", "msl_far_field_adjoint", "msl_adjoint",
           "msl_set_schedule", "msl_last_error", "msl_region_scatter", "msl_region_adam_step",
           "msl_batch_workspace_bytes", "msl_forward_batch", "msl_region_snap", "msl_rotate_object",
           "msl_region_shrinkwrap", "msl_set_tuning", "msl_get_tuning", "msl_autotune_forward",
           "msl_autotune_batch", "msl_forward_noalloc", "msl_workspace_status", "msl_set_barrier_spin_limit")

TUNE_SLOTS = 11  # MSL_TUNE_SLOTS


class CTuning(ctypes.Structure):
    """Mirror of msl_tuning."""

    _fields_ = [("lines_per_group", c_int32 * 11), ("points_per_lane", c_int32 * 11), ("batch_streams", c_int32)]


class CGeometry(ctypes.Structure):
    """Mirror of msl_geometry."""

    _fields_ = [("ny", c_int32), ("nz", c_int32), ("n_slices", c_int32),
                ("dy_nm", c_double), ("dz_nm", c_double), ("dx_nm", c_double),
                ("wavelength_nm", c_double), ("alpha_i_rad", c_double),
                ("propagator", c_int32)]


class CRegion(ctypes.Structure):
    """Mirror of msl_region: box of unknown voxels, beta = beta_over_delta * delta."""

    _fields_ = [("s0", c_int32), ("ns", c_int32), ("y0", c_int32), ("ny", c_int32),
                ("z0", c_int32), ("nz", c_int32), ("beta_over_delta", ctypes.c_float)]


class CAdam(ctypes.Structure):
    """Mirror of msl_adam."""

    _fields_ = [("lr", ctypes.c_float), ("beta1", ctypes.c_float), ("beta2", ctypes.c_float),
                ("eps", ctypes.c_float), ("lo", ctypes.c_float), ("hi", ctypes.c_float)]


class CSampleGrid(ctypes.Structure):
    """Mirror of msl_sample_grid."""

    _fields_ = [("na", c_int32), ("ny", c_int32), ("nz", c_int32), ("da_nm", c_double), ("dy_nm", c_double),
                ("dz_nm", c_double), ("pivot_a_nm", c_double), ("pivot_y_nm", c_double), ("pivot_z_nm", c_double)]


class CInstance(ctypes.Structure):
    """Mirror of msl_instance."""

    _fields_ = [("g", CGeometry), ("n_pool", c_int32), ("pool_delta", c_void_p), ("pool_beta", c_void_p),
                ("slice_index", c_void_p), ("probe", c_void_p), ("field_out", c_void_p),
                ("intensity_out", c_void_p)]


class MslError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"libmsl status {status}: {msg}")
        self.status = status


_lib = None


def lib():
    """Load libmsl.so (once); raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
    L = ctypes.CDLL(LIB_PATH)
    P = c_void_p
    G = ctypes.POINTER(CGeometry)
    L.msl_abi_version.restype = c_int32
    L.msl_abi_version.argtypes = []
    L.msl_workspace_bytes.restype = c_size_t
    L.msl_workspace_bytes.argtypes = [G, c_int32]
    L.msl_checkpoint_count.restype = c_int32
    L.msl_checkpoint_count.argtypes = [G, c_int32]
    L.msl_forward.restype = c_int32
    L.msl_pack_slices.restype = c_int32
    L.msl_pack_slices.argtypes = [G, P, P, P, c_size_t, P]
    L.msl_forward.argtypes = [G, P, P, P, P, P, c_int32, ctypes.c_uint32, P, c_size_t, P]
    L.msl_forward_noalloc.restype = c_int32
    L.msl_forward_noalloc.argtypes = [G, P, P, P, P, P, c_int32, P]
    L.msl_far_field.restype = c_int32
    L.msl_far_field.argtypes = [G, P, P, P, c_size_t, P]
    L.msl_amp_loss.restype = c_int32
    L.msl_amp_loss.argtypes = [G, P, P, P, P, P, c_size_t, P]
    L.msl_far_field_adjoint.restype = c_int32
    L.msl_far_field_adjoint.argtypes = [G, P, P, P, P, c_size_t, P]
    L.msl_adjoint.restype = c_int32
    L.msl_adjoint.argtypes = [G, P, P, P, P, c_int32, P, P, P, P, ctypes.c_uint32, P, c_size_t, P]
    L.msl_set_schedule.restype = c_int32
    L.msl_set_schedule.argtypes = [c_int32]
    L.msl_workspace_status.restype = c_int32
    L.msl_workspace_status.argtypes = [P, c_size_t, P]
    L.msl_set_barrier_spin_limit.restype = c_int32
    L.msl_set_barrier_spin_limit.argtypes = [c_int32]
    T = ctypes.POINTER(CTuning)
    L.msl_set_tuning.restype = c_int32
    L.msl_set_tuning.argtypes = [T]
    L.msl_get_tuning.restype = c_int32
    L.msl_get_tuning.argtypes = [T]
    L.msl_autotune_forward.restype = c_int32
    L.msl_autotune_forward.argtypes = [G, P, P, P, P, c_size_t, c_int32, P, T, ctypes.POINTER(ctypes.c_float)]
    L.msl_last_error.restype = ctypes.c_char_p
    L.msl_last_error.argtypes = []
    L.msl_rotate_object.restype = c_int32
    L.msl_rotate_object.argtypes = [G, c_double, c_double, c_double, ctypes.POINTER(CSampleGrid), c_double, c_double,
                                    P, P, P, P, P]
    Ip = ctypes.POINTER(CInstance)
    L.msl_batch_workspace_bytes.restype = c_size_t
    L.msl_batch_workspace_bytes.argtypes = [Ip, c_int32]
    L.msl_forward_batch.restype = c_int32
    L.msl_forward_batch.argtypes = [Ip, c_int32, P, c_size_t, P]
    L.msl_autotune_batch.restype = c_int32
    L.msl_autotune_batch.argtypes = [Ip, c_int32, P, c_size_t, c_int32, P, ctypes.POINTER(CTuning),
                                     ctypes.POINTER(ctypes.c_float)]
    R = ctypes.POINTER(CRegion)
    L.msl_region_scatter.restype = c_int32
    L.msl_region_scatter.argtypes = [G, R, P, P, P, P]
    L.msl_region_shrinkwrap.restype = c_int32
    L.msl_region_shrinkwrap.argtypes = [G, R, ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                                        P, P, P, P, P]
    L.msl_region_snap.restype = c_int32
    L.msl_region_snap.argtypes = [G, R, ctypes.POINTER(ctypes.c_float), c_int32, P, P, P, P]
    L.msl_region_adam_step.restype = c_int32
    L.msl_region_adam_step.argtypes = [G, R, ctypes.POINTER(CAdam), c_int32, ctypes.c_float,
                                       P, P, P, P, P, P, P, P]
    _lib = L
    return L


def geometry(g) -> CGeometry:
    """msl_geometry from a synth.Geometry, a dict or a CGeometry."""
    if isinstance(g, CGeometry):
        return g
    get = (lambda k: g[k]) if isinstance(g, dict) else (lambda k: getattr(g, k))
    return CGeometry(int(get("ny")), int(get("nz")), int(get("n_slices")),
                     float(get("dy_nm")), float(get("dz_nm")), float(get("dx_nm")),
                     float(get("wavelength_nm")), float(get("alpha_i_rad")),
                     int(get("propagator")))


def _check(status):
    if status != OK:
        raise MslError(status, lib().msl_last_error().decode())


def _ptr(t, dtype, shape, name, allow_none=False):
    if t is None:
        if allow_none:
            return None
        raise ValueError(f"{name} is required")
    if not t.is_cuda:
        raise ValueError(f"{name} must be a GPU tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t.data_ptr()


def _stream():
    return c_void_p(torch.cuda.current_stream().cuda_stream)


def abi_version():
    return lib().msl_abi_version()


def set_schedule(mode: int) -> int:
    r = lib().msl_set_schedule(int(mode))
    if r < 0:
        _check(r)
    return r


def workspace_status(ws):
    """msl_workspace_status: raises MslError if the last phase-running call on ``ws`` is invalid
    (a persistent-schedule barrier gave up); waits for the current stream."""
    _check(lib().msl_workspace_status(ws.data_ptr(), ws.numel(), _stream()))


def set_barrier_spin_limit(polls: int) -> int:
    """msl_set_barrier_spin_limit: returns the previous limit."""
    r = lib().msl_set_barrier_spin_limit(int(polls))
    if r < 0:
        _check(r)
    return r


def _tuning_dict(t):
    return {"lines_per_group": {1 << e: int(t.lines_per_group[e]) for e in range(4, TUNE_SLOTS)},
            "points_per_lane": {1 << e: int(t.points_per_lane[e]) for e in range(4, TUNE_SLOTS)},
            "batch_streams": int(t.batch_streams)}


def get_tuning() -> dict:
    """msl_get_tuning: {"lines_per_group": {line length: value (0 = default)},
    "points_per_lane": {line length: 4, 8 or 0 = default}, "batch_streams": n}."""
    t = CTuning()
    _check(lib().msl_get_tuning(ctypes.byref(t)))
    return _tuning_dict(t)


def _slot(n):
    n = int(n)
    e = n.bit_length() - 1
    if n < 1 or (1 << e) != n or e >= TUNE_SLOTS:
        raise ValueError(f"line length {n} is not a power of two below 2^{TUNE_SLOTS}")
    return e


def set_tuning(lines_per_group=None, batch_streams=0, points_per_lane=None):
    """msl_set_tuning; lines_per_group and points_per_lane map line lengths (16 .. 1024) to values."""
    t = CTuning()
    for n, v in (lines_per_group or {}).items():
        t.lines_per_group[_slot(n)] = int(v)
    for n, v in (points_per_lane or {}).items():
        t.points_per_lane[_slot(n)] = int(v)
    t.batch_streams = int(batch_streams)
    _check(lib().msl_set_tuning(ctypes.byref(t)))


def restore_tuning(t: dict):
    """Apply a dict get_tuning returned."""
    set_tuning(t["lines_per_group"], t["batch_streams"], t["points_per_lane"])


def autotune_forward(g, delta, beta, ws=None, reps=3, scratch=None):
    """msl_autotune_forward: returns (tuning dict now in effect, mean forward ms)."""
    cg = geometry(g)
    ny, nz, ns = cg.ny, cg.nz, cg.n_slices
    if ws is None:
        ws = workspace(cg, 0, delta.device)
    if scratch is None:
        scratch = torch.empty((ny, nz), dtype=torch.complex64, device=delta.device)
    t = CTuning()
    ms = ctypes.c_float()
    _check(lib().msl_autotune_forward(
        ctypes.byref(cg), _ptr(delta, torch.float32, (ns, ny, nz), "delta"),
        _ptr(beta, torch.float32, (ns, ny, nz), "beta"), _ptr(scratch, torch.complex64, (ny, nz), "scratch"),
        ws.data_ptr(), ws.numel(), int(reps), _stream(), ctypes.byref(t), ctypes.byref(ms)))
    return _tuning_dict(t), float(ms.value)


def workspace_bytes(g, ckpt_every=0) -> int:
    return int(lib().msl_workspace_bytes(ctypes.byref(geometry(g)), int(ckpt_every)))


def checkpoint_count(g, ckpt_every) -> int:
    return int(lib().msl_checkpoint_count(ctypes.byref(geometry(g)), int(ckpt_every)))


def workspace(g, ckpt_every=0, device="cuda"):
    """A workspace tensor large enough for every entry point at this geometry."""
    n = workspace_bytes(g, ckpt_every)
    if n == 0:
        raise ValueError("invalid geometry")
    ws = torch.empty(n, dtype=torch.uint8, device=device)
    if ws.data_ptr() % 256:
        ws = torch.empty(n + 256, dtype=torch.uint8, device=device)
        off = (-ws.data_ptr()) % 256
        ws = ws[off:off + n]
    return ws


def pack_slices(g, delta, beta, ws):
    """msl_pack_slices: writes every slice's transmission T - 1 (the slice pack) into ``ws``."""
    cg = geometry(g)
    ny, nz, ns = cg.ny, cg.nz, cg.n_slices
    _check(lib().msl_pack_slices(ctypes.byref(cg), _ptr(delta, torch.float32, (ns, ny, nz), "delta"),
                                 _ptr(beta, torch.float32, (ns, ny, nz), "beta"),
                                 ws.data_ptr(), ws.numel(), _stream()))


def forward(g, delta, beta, probe=None, ckpt_every=0, ws=None, out=None, ckpt=None, reuse_pack=False):
    """msl_forward: returns (psi_Ns complex64 [ny, nz], checkpoints or None).

    ``reuse_pack`` may be set only when ``ws`` already holds the slice pack of
    these delta, beta (``pack_slices`` or an earlier call on ``ws``).
    """
    cg = geometry(g)
    ny, nz, ns = cg.ny, cg.nz, cg.n_slices
    dev = delta.device
    if ws is None:
        ws = workspace(cg, ckpt_every, dev)
    if out is None:
        out = torch.empty((ny, nz), dtype=torch.complex64, device=dev)
    if ckpt_every and ckpt is None:
        ckpt = torch.empty((checkpoint_count(cg, ckpt_every), ny, nz), dtype=torch.complex64, device=dev)
    st = lib().msl_forward(
        ctypes.byref(cg), _ptr(delta, torch.float32, (ns, ny, nz), "delta"),
        _ptr(beta, torch.float32, (ns, ny, nz), "beta"),
        _ptr(probe, torch.complex64, (ny, nz), "probe", True),
        _ptr(out, torch.complex64, (ny, nz), "out"),
        _ptr(ckpt, torch.complex64, (checkpoint_count(cg, ckpt_every), ny, nz), "ckpt", True)
        if ckpt_every else None,
        int(ckpt_every), REUSE_SLICE_PACK if reuse_pack else 0, ws.data_ptr(), ws.numel(), _stream())
    _check(st)
    return out, (ckpt if ckpt_every else None)


def forward_noalloc(g, delta, beta, probe=None, ckpt_every=0, out=None, ckpt=None):
    """msl_forward_noalloc: as ``forward`` without a workspace (the library's fixed
    per-GPU scratch holds its tables); returns (psi_Ns, checkpoints or None)."""
    cg = geometry(g)
    ny, nz, ns = cg.ny, cg.nz, cg.n_slices
    dev = delta.device
    if out is None:
        out = torch.empty((ny, nz), dtype=torch.complex64, device=dev)
    if ckpt_every and ckpt is None:
        ckpt = torch.empty((checkpoint_count(cg, ckpt_every), ny, nz), dtype=torch.complex64, device=dev)
    _check(lib().msl_forward_noalloc(
        ctypes.byref(cg), _ptr(delta, torch.float32, (ns, ny, nz), "delta"),
        _ptr(beta, torch.float32, (ns, ny, nz), "beta"),
        _ptr(probe, torch.complex64, (ny, nz), "probe", True),
        _ptr(out, torch.complex64, (ny, nz), "out"),
        _ptr(ckpt, torch.complex64, (checkpoint_count(cg, ckpt_every), ny, nz), "ckpt", True)
        if ckpt_every else None,
        int(ckpt_every), _stream()))
    return out, (ckpt if ckpt_every else None)


def far_field(g, field, ws=None, out=None):
    cg = geometry(g)
    if ws is None:
        ws = workspace(cg, 0, field.device)
    if out is None:
        out = torch.empty((cg.ny, cg.nz), dtype=torch.float32, device=field.device)
    _check(lib().msl_far_field(ctypes.byref(cg), _ptr(field, torch.complex64, (cg.ny, cg.nz), "field"),
                               _ptr(out, torch.float32, (cg.ny, cg.nz), "intensity"),
                               ws.data_ptr(), ws.numel(), _stream()))
    return out


def amp_loss(g, intensity, meas_amp, ws=None, want_grad=True, loss=None, gI=None):
    """msl_amp_loss: returns (loss float64 scalar tensor on the device, dL/dI or None);
    ``loss`` and ``gI`` may be given as output buffers."""
    cg = geometry(g)
    dev = intensity.device
    if ws is None:
        ws = workspace(cg, 0, dev)
    if loss is None:
        loss = torch.empty((), dtype=torch.float64, device=dev)
    if want_grad and gI is None:
        gI = torch.empty((cg.ny, cg.nz), dtype=torch.float32, device=dev)
    if not want_grad:
        gI = None
    _check(lib().msl_amp_loss(ctypes.byref(cg), _ptr(intensity, torch.float32, (cg.ny, cg.nz), "intensity"),
                              _ptr(meas_amp, torch.float32, (cg.ny, cg.nz), "meas_amp"),
                              loss.data_ptr(), gI.data_ptr() if gI is not None else None,
                              ws.data_ptr(), ws.numel(), _stream()))
    return loss, gI


def far_field_adjoint(g, field, grad_intensity, ws=None, out=None):
    cg = geometry(g)
    if ws is None:
        ws = workspace(cg, 0, field.device)
    if out is None:
        out = torch.empty((cg.ny, cg.nz), dtype=torch.complex64, device=field.device)
    _check(lib().msl_far_field_adjoint(
        ctypes.byref(cg), _ptr(field, torch.complex64, (cg.ny, cg.nz), "field"),
        _ptr(grad_intensity, torch.float32, (cg.ny, cg.nz), "grad_intensity"),
        _ptr(out, torch.complex64, (cg.ny, cg.nz), "grad_field"), ws.data_ptr(), ws.numel(), _stream()))
    return out


def adjoint(g, delta, beta, ckpt, ckpt_every, grad_field, probe=None, ws=None,
            want_delta=True, want_beta=True, want_probe=True, gd=None, gb=None, reuse_pack=False):
    """msl_adjoint: returns (dL/d delta, dL/d beta, dL/d probe), None where not wanted.

    ``reuse_pack`` may be set only when ``ws`` is the workspace the matching
    ``forward`` call used and delta, beta have not changed since.
    """
    cg = geometry(g)
    ny, nz, ns = cg.ny, cg.nz, cg.n_slices
    dev = delta.device
    if ws is None:
        ws = workspace(cg, ckpt_every, dev)
    if want_delta and gd is None:
        gd = torch.empty((ns, ny, nz), dtype=torch.float32, device=dev)
    if want_beta and gb is None:
        gb = torch.empty((ns, ny, nz), dtype=torch.float32, device=dev)
    gp = torch.empty((ny, nz), dtype=torch.complex64, device=dev) if want_probe else None
    _check(lib().msl_adjoint(
        ctypes.byref(cg), _ptr(delta, torch.float32, (ns, ny, nz), "delta"),
        _ptr(beta, torch.float32, (ns, ny, nz), "beta"),
        _ptr(probe, torch.complex64, (ny, nz), "probe", True),
        _ptr(ckpt, torch.complex64, (checkpoint_count(cg, ckpt_every), ny, nz), "ckpt"),
        int(ckpt_every), _ptr(grad_field, torch.complex64, (ny, nz), "grad_field"),
        gd.data_ptr() if want_delta else None, gb.data_ptr() if want_beta else None,
        gp.data_ptr() if gp is not None else None, REUSE_SLICE_PACK if reuse_pack else 0,
        ws.data_ptr(), ws.numel(), _stream()))
    return (gd if want_delta else None), (gb if want_beta else None), gp


# ---------------------------------------------------------------------------
# autograd wrappers

class Multislice(torch.autograd.Function):
    """psi_Ns = Multislice.apply(delta, beta, geom, probe=None, ckpt_every=32)."""

    @staticmethod
    def forward(ctx, delta, beta, geom, probe=None, ckpt_every=32):
        cg = geometry(geom)
        k = max(1, min(int(ckpt_every), cg.n_slices))
        ws = workspace(cg, k, delta.device)
        out, ck = forward(cg, delta.contiguous(), beta.contiguous(), probe, ckpt_every=k, ws=ws)
        ctx.save_for_backward(delta, beta, ck)
        ctx.cg, ctx.k, ctx.has_probe, ctx.ws = cg, k, probe is not None, ws
        return out

    @staticmethod
    def backward(ctx, grad_out):
        delta, beta, ck = ctx.saved_tensors
        # saved tensors are version-checked by autograd, so the forward's pack is still valid
        gd, gb, gp = adjoint(ctx.cg, delta.contiguous(), beta.contiguous(), ck, ctx.k,
                             grad_out.contiguous(), ws=ctx.ws,
                             want_delta=ctx.needs_input_grad[0], want_beta=ctx.needs_input_grad[1],
                             want_probe=ctx.has_probe and ctx.needs_input_grad[3], reuse_pack=True)
        ctx.ws = None
        return gd, gb, None, gp, None


class FarField(torch.autograd.Function):
    """I = FarField.apply(field, geom): fftshifted detector intensity."""

    @staticmethod
    def forward(ctx, field, geom):
        cg = geometry(geom)
        ctx.cg = cg
        ctx.save_for_backward(field)
        return far_field(cg, field.contiguous())

    @staticmethod
    def backward(ctx, gI):
        (field,) = ctx.saved_tensors
        return far_field_adjoint(ctx.cg, field.contiguous(), gI.contiguous()), None


class AmpLoss(torch.autograd.Function):
    """L = AmpLoss.apply(I, meas_amp, geom) = sum (sqrt(I) - m)^2 (float64 scalar)."""

    @staticmethod
    def forward(ctx, intensity, meas_amp, geom):
        cg = geometry(geom)
        loss, gI = amp_loss(cg, intensity.contiguous(), meas_amp.contiguous())
        ctx.save_for_backward(gI)
        return loss

    @staticmethod
    def backward(ctx, gL):
        (gI,) = ctx.saved_tensors
        return gI * gL.to(torch.float32), None, None


# ---------------------------------------------------------------------------
# reconstruction support

def region(r) -> CRegion:
    """msl_region from a CRegion or a mapping with s0, ns, y0, ny, z0, nz, beta_over_delta."""
    if isinstance(r, CRegion):
        return r
    get = (lambda k: r[k]) if isinstance(r, dict) else (lambda k: getattr(r, k))
    return CRegion(int(get("s0")), int(get("ns")), int(get("y0")), int(get("ny")), int(get("z0")),
                   int(get("nz")), float(get("beta_over_delta")))


def region_scatter(g, r, theta, delta, beta):
    """delta[box] = theta, beta[box] = ratio * theta (in place on the stacks)."""
    cg, cr = geometry(g), region(r)
    stack = (cg.n_slices, cg.ny, cg.nz)
    _check(lib().msl_region_scatter(ctypes.byref(cg), ctypes.byref(cr),
                                    _ptr(theta, torch.float32, (cr.ns, cr.ny, cr.nz), "theta"),
                                    _ptr(delta, torch.float32, stack, "delta"),
                                    _ptr(beta, torch.float32, stack, "beta"), _stream()))


def region_snap(g, r, levels, theta, delta, beta):
    """theta <- nearest of `levels` (host floats), then the scatter into delta, beta."""
    cg, cr = geometry(g), region(r)
    stack = (cg.n_slices, cg.ny, cg.nz)
    lv = (ctypes.c_float * len(levels))(*[float(x) for x in levels])
    _check(lib().msl_region_snap(ctypes.byref(cg), ctypes.byref(cr), lv, len(levels),
                                 _ptr(theta, torch.float32, (cr.ns, cr.ny, cr.nz), "theta"),
                                 _ptr(delta, torch.float32, stack, "delta"),
                                 _ptr(beta, torch.float32, stack, "beta"), _stream()))


def region_shrinkwrap(g, r, sigmas, threshold, theta, delta, beta, scratch=None):
    """Shrink-wrap support on theta (in place) and the scatter; sigmas = (a, y, z) in voxels."""
    cg, cr = geometry(g), region(r)
    stack = (cg.n_slices, cg.ny, cg.nz)
    n = cr.ns * cr.ny * cr.nz
    if scratch is None:
        scratch = torch.empty(2 * n + 1024, dtype=torch.float32, device=theta.device)
    _check(lib().msl_region_shrinkwrap(ctypes.byref(cg), ctypes.byref(cr), float(sigmas[0]), float(sigmas[1]),
                                       float(sigmas[2]), float(threshold),
                                       _ptr(theta, torch.float32, (cr.ns, cr.ny, cr.nz), "theta"),
                                       _ptr(scratch, torch.float32, (2 * n + 1024,), "scratch"),
                                       _ptr(delta, torch.float32, stack, "delta"),
                                       _ptr(beta, torch.float32, stack, "beta"), _stream()))


def region_adam_step(g, r, adam, t, grad_delta, grad_beta, theta, m, v, delta, beta, grad_scale=1.0):
    """One ADAM step on theta (in place, with m, v) and the scatter of the new theta."""
    cg, cr = geometry(g), region(r)
    stack = (cg.n_slices, cg.ny, cg.nz)
    box = (cr.ns, cr.ny, cr.nz)
    a = adam if isinstance(adam, CAdam) else CAdam(*[float(x) for x in adam])
    _check(lib().msl_region_adam_step(
        ctypes.byref(cg), ctypes.byref(cr), ctypes.byref(a), int(t), float(grad_scale),
        _ptr(grad_delta, torch.float32, stack, "grad_delta"), _ptr(grad_beta, torch.float32, stack, "grad_beta"),
        _ptr(theta, torch.float32, box, "theta"), _ptr(m, torch.float32, box, "m"),
        _ptr(v, torch.float32, box, "v"), _ptr(delta, torch.float32, stack, "delta"),
        _ptr(beta, torch.float32, stack, "beta"), _stream()))


# ---------------------------------------------------------------------------
# batched forward

def _instances(items):
    arr = (CInstance * len(items))()
    for i, it in enumerate(items):
        cg = geometry(it["geom"])
        ny, nz, ns = cg.ny, cg.nz, cg.n_slices
        npool = int(it["pool_delta"].shape[0])
        arr[i] = CInstance(cg, npool,
                           _ptr(it["pool_delta"], torch.float32, (npool, ny, nz), "pool_delta"),
                           _ptr(it["pool_beta"], torch.float32, (npool, ny, nz), "pool_beta"),
                           _ptr(it["slice_index"], torch.int32, (ns,), "slice_index"),
                           _ptr(it.get("probe"), torch.complex64, (ny, nz), "probe", True),
                           _ptr(it["field"], torch.complex64, (ny, nz), "field"),
                           _ptr(it.get("intensity"), torch.float32, (ny, nz), "intensity", True))
    return arr


def batch_workspace(items, device=None):
    arr = _instances(items)
    n = int(lib().msl_batch_workspace_bytes(arr, len(items)))
    if n == 0:
        _check(ERR_ARG)
    dev = device or items[0]["field"].device
    ws = torch.empty(n + 256, dtype=torch.uint8, device=dev)
    off = (-ws.data_ptr()) % 256
    return ws[off:off + n]


def autotune_batch(items, ws=None, reps=1):
    """msl_autotune_batch: returns (tuning dict now in effect, mean batch ms); overwrites the
    items' outputs."""
    arr = _instances(items)
    if ws is None:
        ws = batch_workspace(items)
    t = CTuning()
    ms = ctypes.c_float()
    _check(lib().msl_autotune_batch(arr, len(items), ws.data_ptr(), ws.numel(), int(reps), _stream(),
                                    ctypes.byref(t), ctypes.byref(ms)))
    return _tuning_dict(t), float(ms.value)


def forward_batch(items, ws=None):
    """msl_forward_batch over a list of instances: dicts with geom, pool_delta, pool_beta,
    slice_index (device int32), field (output), optional probe and intensity (output)."""
    arr = _instances(items)
    if ws is None:
        ws = batch_workspace(items)
    _check(lib().msl_forward_batch(arr, len(items), ws.data_ptr(), ws.numel(), _stream()))
    return ws


def rotate_object(g, lab_pivot, sample_grid, pitch_rad, yaw_rad, delta_s, beta_s, delta=None, beta=None):
    """msl_rotate_object: lab-frame stacks [Ns][ny][nz] from a sample-frame volume; sample_grid is a
    CSampleGrid or a dict of its fields; lab_pivot = (a, y, z) in nm."""
    cg = geometry(g)
    sg = sample_grid if isinstance(sample_grid, CSampleGrid) else CSampleGrid(**sample_grid)
    dev = delta_s.device
    shape = (cg.n_slices, cg.ny, cg.nz)
    if delta is None:
        delta = torch.empty(shape, dtype=torch.float32, device=dev)
    if beta is None:
        beta = torch.empty(shape, dtype=torch.float32, device=dev)
    sshape = (sg.na, sg.ny, sg.nz)
    _check(lib().msl_rotate_object(ctypes.byref(cg), float(lab_pivot[0]), float(lab_pivot[1]), float(lab_pivot[2]),
                                   ctypes.byref(sg), float(pitch_rad), float(yaw_rad),
                                   _ptr(delta_s, torch.float32, sshape, "delta_s"),
                                   _ptr(beta_s, torch.float32, sshape, "beta_s"),
                                   _ptr(delta, torch.float32, shape, "delta"),
                                   _ptr(beta, torch.float32, shape, "beta"), _stream()))
    return delta, beta

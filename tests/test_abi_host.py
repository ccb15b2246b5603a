"""Host-side checks of the C ABI (CPU only: no call here reaches the GPU).

The library must load, export every function declared in include/msl.h, and
reject invalid arguments on the host with the documented status codes before
it touches HIP.  Only arguments that fail validation are passed, so no kernel
is ever enqueued.
"""
import ctypes
import os
import re

import pytest

from paper_2212_01253_amd import msl

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for h in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if h.endswith(".h"):
            src = open(os.path.join(ROOT, "include", h)).read()
            src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
            names |= set(re.findall(r"\b(msl_[a-z0-9_]+)\s*\(", src))
    return sorted(names)


@pytest.fixture(scope="module")
def L():
    return msl.lib()


def test_exports_every_declared_symbol(L):
    names = declared_functions()
    assert len(names) >= 9
    for n in names:
        assert hasattr(L, n), n
    from paper_2212_01253_amd import nn
    assert set(names) == set(msl.EXPORTS) | set(nn.EXPORTS)
    nn.lib()   # every binding signature resolves


def test_abi_version(L):
    assert msl.abi_version() == 6


def G(**kw):
    base = dict(ny=64, nz=64, n_slices=8, dy_nm=1.0, dz_nm=1.0, dx_nm=10.0,
                wavelength_nm=0.1, alpha_i_rad=0.003, propagator=0)
    base.update(kw)
    return msl.CGeometry(**base)


FAKE = 0x7F0000000000  # never dereferenced: validation fails first


def fwd(L, g, delta=FAKE, beta=FAKE, probe=None, out=FAKE, ckpt=None, k=0, ws=FAKE, wsb=1 << 40, flags=0):
    return L.msl_forward(ctypes.byref(g), delta, beta, probe, out, ckpt, k, flags, ws, wsb, None)


@pytest.mark.parametrize("kw", [dict(ny=15), dict(nz=2048), dict(ny=8), dict(nz=48), dict(n_slices=0),
                                dict(dy_nm=0.0), dict(dz_nm=-1.0), dict(dx_nm=float("nan")),
                                dict(wavelength_nm=0.0), dict(alpha_i_rad=1.6), dict(propagator=2)])
def test_invalid_geometry(L, kw):
    assert fwd(L, G(**kw)) == msl.ERR_ARG
    assert L.msl_last_error().decode()
    assert L.msl_workspace_bytes(ctypes.byref(G(**kw)), 0) == 0


def test_null_and_misaligned_pointers(L):
    g = G()
    assert fwd(L, g, delta=None) == msl.ERR_ARG
    assert "delta" in L.msl_last_error().decode()
    assert fwd(L, g, beta=FAKE + 2) == msl.ERR_ARG
    assert fwd(L, g, out=FAKE + 4) == msl.ERR_ARG
    assert fwd(L, g, probe=FAKE + 4) == msl.ERR_ARG


def test_checkpoint_argument_rules(L):
    g = G()
    assert fwd(L, g, flags=2) == msl.ERR_ARG
    assert "flags" in L.msl_last_error().decode()
    assert fwd(L, g, ckpt=FAKE, k=0) == msl.ERR_ARG
    assert fwd(L, g, ckpt=None, k=4) == msl.ERR_ARG
    # the adjoint requires checkpoints
    st = L.msl_adjoint(ctypes.byref(g), FAKE, FAKE, None, None, 4, FAKE, FAKE, FAKE, None, 0, FAKE, 1 << 40, None)
    assert st == msl.ERR_ARG
    st = L.msl_adjoint(ctypes.byref(g), FAKE, FAKE, None, FAKE, 0, FAKE, FAKE, FAKE, None, 0, FAKE, 1 << 40, None)
    assert st == msl.ERR_ARG
    st = L.msl_adjoint(ctypes.byref(g), FAKE, FAKE, None, FAKE, 4, FAKE, FAKE, FAKE, None, 6, FAKE, 1 << 40, None)
    assert "flags" in L.msl_last_error().decode()
    assert st == msl.ERR_ARG


def test_workspace_rules(L):
    g = G()
    need = L.msl_workspace_bytes(ctypes.byref(g), 0)
    assert need > 0
    assert fwd(L, g, ws=None) == msl.ERR_WORKSPACE
    assert fwd(L, g, ws=FAKE + 128) == msl.ERR_WORKSPACE
    assert fwd(L, g, wsb=need - 1) == msl.ERR_WORKSPACE
    assert "need" in L.msl_last_error().decode()
    # adjoint workspace grows with the checkpoint interval (segment buffer)
    assert L.msl_workspace_bytes(ctypes.byref(g), 8) > L.msl_workspace_bytes(ctypes.byref(g), 2) > need
    st = L.msl_adjoint(ctypes.byref(g), FAKE, FAKE, None, FAKE, 8, FAKE, FAKE, FAKE, None, 0, FAKE,
                       L.msl_workspace_bytes(ctypes.byref(g), 2), None)
    assert st == msl.ERR_WORKSPACE


def test_checkpoint_count(L):
    assert L.msl_checkpoint_count(ctypes.byref(G(n_slices=100)), 32) == 4
    assert L.msl_checkpoint_count(ctypes.byref(G(n_slices=96)), 32) == 3
    assert L.msl_checkpoint_count(ctypes.byref(G(n_slices=5)), 1) == 5
    assert L.msl_checkpoint_count(ctypes.byref(G()), 0) == 0


def test_other_entry_points_validate(L):
    g = G()
    assert L.msl_pack_slices(ctypes.byref(g), None, FAKE, FAKE, 1 << 40, None) == msl.ERR_ARG
    assert L.msl_pack_slices(ctypes.byref(G(nz=48)), FAKE, FAKE, FAKE, 1 << 40, None) == msl.ERR_ARG
    assert L.msl_pack_slices(ctypes.byref(g), FAKE, FAKE, FAKE, 16, None) == msl.ERR_WORKSPACE
    assert L.msl_far_field(ctypes.byref(g), None, FAKE, FAKE, 1 << 40, None) == msl.ERR_ARG
    assert L.msl_far_field(ctypes.byref(G(ny=3)), FAKE, FAKE, FAKE, 1 << 40, None) == msl.ERR_ARG
    assert L.msl_amp_loss(ctypes.byref(g), FAKE, FAKE, FAKE + 4, None, FAKE, 1 << 40, None) == msl.ERR_ARG
    assert L.msl_far_field_adjoint(ctypes.byref(g), FAKE, None, FAKE, FAKE, 1 << 40, None) == msl.ERR_ARG


def test_schedule_setter(L):
    prev = msl.set_schedule(msl.SCHED_PER_PASS)
    assert msl.set_schedule(prev) == msl.SCHED_PER_PASS
    with pytest.raises(msl.MslError):
        msl.set_schedule(7)


def test_region_entry_points_validate(L):
    g = G(n_slices=8)
    R = ctypes.byref
    ok = msl.CRegion(0, 8, 2, 4, 0, 64, 0.05)
    adam = msl.CAdam(1e-6, 0.9, 0.999, 1e-12, 0.0, 1e-3)
    for bad in (msl.CRegion(0, 9, 2, 4, 0, 64, 0.05), msl.CRegion(-1, 2, 2, 4, 0, 64, 0.05),
                msl.CRegion(0, 8, 62, 4, 0, 64, 0.05), msl.CRegion(0, 8, 2, 0, 0, 64, 0.05),
                msl.CRegion(0, 8, 2, 4, 1, 64, 0.05), msl.CRegion(0, 8, 2, 4, 0, 64, float("inf"))):
        assert L.msl_region_scatter(R(g), R(bad), FAKE, FAKE, FAKE, None) == msl.ERR_ARG
        assert "region" in L.msl_last_error().decode() or "beta_over_delta" in L.msl_last_error().decode()
    assert L.msl_region_scatter(R(g), None, FAKE, FAKE, FAKE, None) == msl.ERR_ARG
    assert L.msl_region_scatter(R(g), R(ok), FAKE + 2, FAKE, FAKE, None) == msl.ERR_ARG

    def step(a=adam, t=1, scale=1.0, gd=FAKE):
        return L.msl_region_adam_step(R(g), R(ok), R(a) if a is not None else None, t, scale, gd, FAKE, FAKE,
                                      FAKE, FAKE, FAKE, FAKE, None)
    assert step(t=0) == msl.ERR_ARG
    assert step(a=None) == msl.ERR_ARG
    assert step(a=msl.CAdam(1e-6, 1.0, 0.999, 1e-12, 0.0, 1e-3)) == msl.ERR_ARG
    assert step(a=msl.CAdam(1e-6, 0.9, 0.999, 0.0, 0.0, 1e-3)) == msl.ERR_ARG
    assert step(a=msl.CAdam(1e-6, 0.9, 0.999, 1e-12, 1.0, 0.0)) == msl.ERR_ARG
    assert step(a=msl.CAdam(-1.0, 0.9, 0.999, 1e-12, 0.0, 1.0)) == msl.ERR_ARG
    assert step(scale=float("nan")) == msl.ERR_ARG
    assert step(gd=None) == msl.ERR_ARG


def test_batch_entry_points_validate(L):
    def inst(**kw):
        base = dict(g=G(n_slices=8), n_pool=3, pool_delta=FAKE, pool_beta=FAKE, slice_index=FAKE, probe=None,
                    field_out=FAKE, intensity_out=None)
        base.update(kw)
        return msl.CInstance(**base)
    arr = (msl.CInstance * 2)(inst(), inst(g=G(ny=32, nz=128, n_slices=3)))
    need = L.msl_batch_workspace_bytes(arr, 2)
    assert need > 0
    assert L.msl_batch_workspace_bytes(arr, 0) == 0
    assert L.msl_forward_batch(arr, 0, FAKE, need, None) == msl.ERR_ARG
    assert L.msl_forward_batch(None, 1, FAKE, need, None) == msl.ERR_ARG
    assert L.msl_forward_batch(arr, 2, FAKE, need - 1, None) == msl.ERR_WORKSPACE
    assert L.msl_forward_batch(arr, 2, None, need, None) == msl.ERR_WORKSPACE
    for bad, code in ((inst(g=G(propagator=1)), msl.ERR_UNSUPPORTED), (inst(n_pool=0), msl.ERR_ARG),
                      (inst(slice_index=None), msl.ERR_ARG), (inst(field_out=FAKE + 4), msl.ERR_ARG),
                      (inst(g=G(ny=48)), msl.ERR_ARG), (inst(intensity_out=FAKE + 2), msl.ERR_ARG)):
        arr = (msl.CInstance * 2)(inst(), bad)
        assert L.msl_forward_batch(arr, 2, FAKE, 1 << 40, None) == code
        assert L.msl_last_error().decode().startswith("instance 1")
        assert L.msl_batch_workspace_bytes(arr, 2) == 0


def test_snap_validates(L):
    g = G(n_slices=8)
    ok = msl.CRegion(0, 8, 2, 4, 0, 64, 0.05)
    lv = (ctypes.c_float * 17)(*range(17))
    R = ctypes.byref
    assert L.msl_region_snap(R(g), R(ok), lv, 0, FAKE, FAKE, FAKE, None) == msl.ERR_ARG
    assert L.msl_region_snap(R(g), R(ok), lv, 17, FAKE, FAKE, FAKE, None) == msl.ERR_ARG
    assert L.msl_region_snap(R(g), R(ok), None, 2, FAKE, FAKE, FAKE, None) == msl.ERR_ARG
    nan = (ctypes.c_float * 2)(0.0, float("nan"))
    assert L.msl_region_snap(R(g), R(ok), nan, 2, FAKE, FAKE, FAKE, None) == msl.ERR_ARG
    assert L.msl_region_snap(R(g), R(ok), lv, 2, FAKE + 2, FAKE, FAKE, None) == msl.ERR_ARG


def test_nn_entry_points_validate(L):
    from paper_2212_01253_amd import nn
    N = nn.lib()
    assert N.msl_nn_gemm_bf16(0, 4, 4, FAKE, 4, 0, FAKE, 4, 0, FAKE, 4, 0.0, None, 0, None, None) == msl.ERR_ARG
    assert N.msl_nn_gemm_bf16(4, 4, 4, FAKE, 3, 0, FAKE, 4, 0, FAKE, 4, 0.0, None, 0, None, None) == msl.ERR_ARG
    assert N.msl_nn_gemm_bf16(4, 4, 4, FAKE + 1, 4, 0, FAKE, 4, 0, FAKE, 4, 0.0, None, 0, None, None) == msl.ERR_ARG
    assert N.msl_nn_im2col3x3(2, 1, 5, 4, 2, FAKE, FAKE, None) == msl.ERR_ARG
    assert N.msl_nn_im2col3x3(2, 1, 4, 4, 3, FAKE, FAKE, None) == msl.ERR_ARG
    assert N.msl_nn_rowpool(1, 10, 4, 4, FAKE, FAKE, None) == msl.ERR_ARG
    assert N.msl_nn_adam(8, FAKE, FAKE, FAKE, FAKE, None, 1e-3, 1.0, 0.999, 1e-8, 1, None) == msl.ERR_ARG
    assert N.msl_nn_adam(8, FAKE, FAKE, FAKE, FAKE, None, 1e-3, 0.9, 0.999, 1e-8, 0, None) == msl.ERR_ARG
    assert N.msl_nn_mse(0, FAKE, FAKE, None, FAKE, FAKE, None) == msl.ERR_ARG
    assert N.msl_nn_mse(8, FAKE, FAKE, None, FAKE, None, None) == msl.ERR_ARG     # no scratch
    assert N.msl_nn_row_features(2, 4, 6, FAKE, None, None, FAKE, None) == msl.ERR_ARG       # W < 8
    assert N.msl_nn_row_features(2, 4, 8, FAKE, None, None, FAKE + 1, None) == msl.ERR_ARG  # misaligned
    assert N.msl_nn_row_features(2, 4, 8, FAKE, FAKE + 2, None, FAKE, None) == msl.ERR_ARG  # misaligned
    assert N.msl_nn_add_row_bias(0, 4, 8, FAKE, FAKE, None) == msl.ERR_ARG
    assert N.msl_nn_row_bias_adjoint(2, 0, 8, FAKE, FAKE, None) == msl.ERR_ARG
    assert N.msl_nn_row_bias_adjoint(2, 4, 8, None, FAKE, None) == msl.ERR_ARG
    # conv3x3(Co, C, B, H, W, stride, w16, x, x_bf16, bias, relu, y, y_bf16, wscratch, stream)
    assert N.msl_nn_conv3x3(4, 3, 2, 8, 8, 3, FAKE, FAKE, 0, None, 0, FAKE, 0, FAKE, None) == msl.ERR_ARG      # stride 3
    assert N.msl_nn_conv3x3(4, 3, 2, 9, 8, 2, FAKE, FAKE, 0, None, 0, FAKE, 0, FAKE, None) == msl.ERR_ARG      # odd H
    assert N.msl_nn_conv3x3(4, 3, 2, 8, 8, 1, FAKE + 1, FAKE, 0, None, 0, FAKE, 0, FAKE, None) == msl.ERR_ARG  # misaligned
    assert N.msl_nn_conv3x3(0, 3, 2, 8, 8, 1, FAKE, FAKE, 0, None, 0, FAKE, 0, FAKE, None) == msl.ERR_ARG
    assert N.msl_nn_conv3x3(4, 3, 2, 8, 8, 1, FAKE, FAKE, 0, None, 0, FAKE, 0, None, None) == msl.ERR_ARG      # no scratch
    assert N.msl_nn_conv3x3(4, 3, 2, 8, 8, 1, FAKE, FAKE, 0, None, 0, FAKE, 0, FAKE + 8, None) == msl.ERR_ARG  # misaligned
    # float32 x or y must be 4-byte aligned (bfloat16 bits 2-byte)
    assert N.msl_nn_conv3x3(4, 3, 2, 8, 8, 1, FAKE, FAKE + 2, 0, None, 0, FAKE, 0, FAKE, None) == msl.ERR_ARG
    assert N.msl_nn_conv3x3(4, 3, 2, 8, 8, 1, FAKE, FAKE, 0, None, 0, FAKE + 2, 0, FAKE, None) == msl.ERR_ARG
    assert N.msl_nn_conv3x3(4, 3, 2, 8, 8, 1, FAKE, FAKE + 1, 1, None, 0, FAKE, 0, FAKE, None) == msl.ERR_ARG
    assert N.msl_nn_conv3x3_adjoint(4, 3, 2, 8, 8, 1, FAKE, None, FAKE, 0, FAKE, None) == msl.ERR_ARG
    assert N.msl_nn_conv3x3_adjoint(4, 0, 2, 8, 8, 1, FAKE, FAKE, FAKE, 0, FAKE, None) == msl.ERR_ARG
    assert N.msl_nn_conv3x3_adjoint(4, 3, 2, 8, 8, 1, FAKE, FAKE, FAKE, 0, None, None) == msl.ERR_ARG   # no scratch
    assert N.msl_nn_conv3x3_adjoint(4, 3, 2, 8, 8, 2, FAKE, FAKE, FAKE + 4, 1, FAKE, None) == msl.ERR_ARG  # accumulate, dx misaligned
    assert N.msl_nn_conv3x3_scratch_elems(20, 3) == 16 * 32 * 16 and N.msl_nn_conv3x3_scratch_elems(0, 3) == 0
    # weight_grad(Co, C, B, H, W, stride, dy16, x, x_bf16, dw, splits, partials, stream)
    assert N.msl_nn_conv3x3_weight_grad(4, 3, 2, 8, 8, 1, FAKE, FAKE, 0, FAKE, 0, FAKE, None) == msl.ERR_ARG   # splits
    assert N.msl_nn_conv3x3_weight_grad(4, 3, 2, 8, 8, 1, FAKE, FAKE, 0, FAKE, 2, None, None) == msl.ERR_ARG
    assert N.msl_nn_conv3x3_weight_grad(4, 3, 2, 8, 8, 1, FAKE, FAKE + 2, 0, FAKE, 2, FAKE, None) == msl.ERR_ARG
    assert N.msl_nn_conv3x3_weight_grad(4, 3, 2, 8, 8, 1, FAKE, FAKE + 1, 1, FAKE, 2, FAKE, None) == msl.ERR_ARG
    # grad_prep(M, N, y, y_bf16, dy, dy16, bias_grad, parts, stream); upsample2(C, B, H, W, x, y, bf16, stream)
    assert N.msl_nn_grad_prep(4, 8, FAKE + 2, 0, FAKE, FAKE, FAKE, FAKE, None) == msl.ERR_ARG
    assert N.msl_nn_grad_prep(4, 8, FAKE + 1, 1, FAKE, FAKE, FAKE, FAKE, None) == msl.ERR_ARG
    assert N.msl_nn_upsample2(2, 1, 4, 4, FAKE + 2, FAKE, 0, None) == msl.ERR_ARG
    assert N.msl_nn_upsample2(2, 1, 4, 4, FAKE, FAKE + 1, 1, None) == msl.ERR_ARG


def test_rotation_validates(L):
    g = G()
    R = ctypes.byref
    ok = msl.CSampleGrid(4, 4, 4, 1.0, 1.0, 1.0, 0.0, 0.0, 0.0)
    assert L.msl_rotate_object(R(g), 0.0, 0.0, 0.0, None, 0.0, 0.0, FAKE, FAKE, FAKE, FAKE, None) == msl.ERR_ARG
    bad = msl.CSampleGrid(0, 4, 4, 1.0, 1.0, 1.0, 0.0, 0.0, 0.0)
    assert L.msl_rotate_object(R(g), 0.0, 0.0, 0.0, R(bad), 0.0, 0.0, FAKE, FAKE, FAKE, FAKE, None) == msl.ERR_ARG
    bad = msl.CSampleGrid(4, 4, 4, 1.0, -1.0, 1.0, 0.0, 0.0, 0.0)
    assert L.msl_rotate_object(R(g), 0.0, 0.0, 0.0, R(bad), 0.0, 0.0, FAKE, FAKE, FAKE, FAKE, None) == msl.ERR_ARG
    assert L.msl_rotate_object(R(g), 0.0, 0.0, 0.0, R(ok), float("nan"), 0.0, FAKE, FAKE, FAKE, FAKE, None) == msl.ERR_ARG
    assert L.msl_rotate_object(R(g), 0.0, 0.0, 0.0, R(ok), 0.0, 0.0, FAKE + 1, FAKE, FAKE, FAKE, None) == msl.ERR_ARG


def test_shrinkwrap_validates(L):
    g = G(n_slices=8)
    ok = msl.CRegion(0, 8, 2, 4, 0, 64, 0.05)
    R = ctypes.byref
    assert L.msl_region_shrinkwrap(R(g), R(ok), -1.0, 1.0, 1.0, 0.2, FAKE, FAKE, FAKE, FAKE, None) == msl.ERR_ARG
    assert L.msl_region_shrinkwrap(R(g), R(ok), 1.0, 21.0, 1.0, 0.2, FAKE, FAKE, FAKE, FAKE, None) == msl.ERR_ARG
    assert L.msl_region_shrinkwrap(R(g), R(ok), 1.0, 1.0, 1.0, 1.0, FAKE, FAKE, FAKE, FAKE, None) == msl.ERR_ARG
    assert L.msl_region_shrinkwrap(R(g), R(ok), 1.0, 1.0, 1.0, 0.2, FAKE, None, FAKE, FAKE, None) == msl.ERR_ARG


def test_tuning_validates_and_round_trips(L):
    before = msl.get_tuning()
    try:
        msl.set_tuning({512: 2, 256: 4, 128: 1, 16: 64}, batch_streams=2, points_per_lane={512: 4, 64: 8})
        t = msl.get_tuning()
        assert t["lines_per_group"][512] == 2 and t["lines_per_group"][256] == 4
        assert t["lines_per_group"][128] == 1 and t["lines_per_group"][16] == 64
        assert t["lines_per_group"][1024] == 0 and t["batch_streams"] == 2
        assert t["points_per_lane"][512] == 4 and t["points_per_lane"][64] == 8 and t["points_per_lane"][256] == 0
        # group limits at 8 points per lane: 64: 32, 128: 16, 256: 8, 512: 4, 1024: 2;
        # at 4: 16: 64, 32: 32, 64: 16, 128: 8, 256: 4, 512: 2, 1024: 1
        msl.set_tuning({512: 4, 1024: 2, 64: 32, 128: 16, 256: 8}, points_per_lane={64: 8, 128: 8, 256: 8})
        msl.set_tuning({512: 2, 1024: 1, 16: 64, 32: 32, 64: 16, 128: 8, 256: 4},
                       points_per_lane={512: 4, 1024: 4, 16: 4, 32: 4, 64: 4, 128: 4, 256: 4})
        msl.restore_tuning(t)
        bad = [({512: 3}, 0, {}), ({512: 8}, 0, {}), ({1024: 4}, 0, {}), ({256: -1}, 0, {}), ({8: 1}, 0, {}),
               ({}, 5, {}), ({}, -1, {}),
               ({}, 0, {512: 2}), ({}, 0, {512: 16}), ({}, 0, {32: 8}), ({}, 0, {16: 8}), ({}, 0, {8: 4}),
               ({}, 0, {256: -4}), ({512: 4}, 0, {512: 4}), ({1024: 2}, 0, {1024: 4}), ({64: 64}, 0, {64: 8}),
               ({64: 32}, 0, {64: 4}), ({256: 8}, 0, {}), ({256: 16}, 0, {256: 8})]
        for lpg, bs, ppl in bad:
            with pytest.raises(msl.MslError):
                msl.set_tuning(lpg, batch_streams=bs, points_per_lane=ppl)
            assert msl.get_tuning() == t      # nothing changes on an error
    finally:
        msl.restore_tuning(before)
    assert msl.get_tuning() == before


def test_autotune_validates(L):
    g = G()
    f = ctypes.c_float()
    st = L.msl_autotune_forward(ctypes.byref(g), FAKE, FAKE, None, FAKE, 1 << 40, 3, None, None, ctypes.byref(f))
    assert st == msl.ERR_ARG                              # no scratch field
    st = L.msl_autotune_forward(ctypes.byref(g), FAKE, FAKE, FAKE, FAKE, 1 << 40, 0, None, None, ctypes.byref(f))
    assert st == msl.ERR_ARG                              # reps < 1
    st = L.msl_autotune_forward(ctypes.byref(G(ny=48)), FAKE, FAKE, FAKE, FAKE, 1 << 40, 3, None, None, None)
    assert st == msl.ERR_ARG                              # not a power of two
    assert L.msl_autotune_batch(None, 1, FAKE, 1 << 40, 1, None, None, None) == msl.ERR_ARG   # no instances


def test_forward_noalloc_validates(L):
    def nf(g, delta=FAKE, beta=FAKE, probe=None, out=FAKE, ckpt=None, k=0):
        return L.msl_forward_noalloc(ctypes.byref(g), delta, beta, probe, out, ckpt, k, None)

    assert nf(G(ny=15)) == msl.ERR_ARG
    assert nf(G(), delta=None) == msl.ERR_ARG
    assert nf(G(), out=FAKE + 4) == msl.ERR_ARG
    assert nf(G(), probe=FAKE + 4) == msl.ERR_ARG
    assert nf(G(), ckpt=FAKE, k=0) == msl.ERR_ARG
    assert nf(G(), ckpt=None, k=3) == msl.ERR_ARG
    # beyond the fixed scratch: the exact propagator's 2-D table of grids above 512 x 512
    for ny, nz in ((1024, 1024), (512, 1024)):
        assert nf(G(ny=ny, nz=nz, propagator=1)) == msl.ERR_UNSUPPORTED
        assert "scratch" in L.msl_last_error().decode()


def test_status_query_and_spin_limit_validate(L):
    assert L.msl_workspace_status(None, 1 << 20, None) == msl.ERR_WORKSPACE
    assert L.msl_workspace_status(FAKE + 128, 1 << 20, None) == msl.ERR_WORKSPACE
    assert L.msl_workspace_status(FAKE, 4096, None) == msl.ERR_WORKSPACE
    assert L.msl_set_barrier_spin_limit(-1) == msl.ERR_ARG
    prev = L.msl_set_barrier_spin_limit(7)
    assert prev == 1 << 22
    assert L.msl_set_barrier_spin_limit(prev) == 7

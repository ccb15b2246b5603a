"""msl_forward_noalloc (the forward entry point that allocates nothing: its tables live in
the library's fixed per-GPU scratch array) against msl_forward, through the C ABI, on two
calls in a row, the second with a smaller input; and the size limit of its scratch."""
import math

import numpy as np
import pytest

from paper_2212_01253_amd import synth
from parity_gates import check_field

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def M():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2212_01253_amd import msl
    msl.lib()
    return msl


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


CASES = [
    # (geometry, checkpoint interval, probe seed or None): the larger call first
    (synth.Geometry(256, 512, 37, 1.0, 0.8, 5.0, 0.1, math.radians(0.3), 0), 8, None),
    (synth.Geometry(64, 32, 19, 0.9, 1.1, 7.0, 0.12, math.radians(0.2), 1), 5, 3),
]


def test_noalloc_forward_equals_forward_on_two_calls(M):
    for i, (g, k, pseed) in enumerate(CASES):
        d, b = synth.random_stack(g.ny, g.nz, g.n_slices, 500 + i, 3e-5, 2e-6)
        D, B = dev(d), dev(b)
        P = None if pseed is None else dev(synth.random_field(g.ny, g.nz, pseed).astype(np.complex64))
        ref, rck = M.forward(g, D, B, P, k)
        out, ck = M.forward_noalloc(g, D, B, P, k)
        torch.cuda.synchronize()
        f, rf = out.cpu().numpy(), ref.cpu().numpy()
        bitwise = np.array_equal(f, rf) and np.array_equal(ck.cpu().numpy(), rck.cpu().numpy())
        print(f"call {i}: {g.ny}x{g.nz}x{g.n_slices} propagator {g.propagator}: bitwise equal {bitwise}")
        check_field(f, rf.astype(np.complex128), what=f"call {i} field")
        for c in range(rck.shape[0]):
            check_field(ck[c].cpu().numpy(), rck[c].cpu().numpy().astype(np.complex128), what=f"call {i} ckpt {c}")


def test_noalloc_rejects_what_its_scratch_cannot_hold(M):
    g = synth.Geometry(1024, 1024, 1, 1.0, 1.0, 5.0, 0.1, 0.0, 1)
    z = torch.zeros((1, 1024, 1024), dtype=torch.float32, device="cuda")
    with pytest.raises(M.MslError) as e:
        M.forward_noalloc(g, z, z)
    assert e.value.status == M.ERR_UNSUPPORTED and "scratch" in str(e.value)

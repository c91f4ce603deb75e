"""fio_apply_batch_noalloc (the apply whose row-stage output and grids live
in the library's fixed scratch array) against fio_apply_batch, called
through the C ABI: two calls in a row, the second with a smaller input,
must equal the plan-workspace apply bit for bit; a plan whose one
right-hand side does not fit the array is refused before any launch."""
import ctypes

import numpy as np
import pytest

import fio_inputs as fi

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _setup():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")


def _call(lib, plan, fd, out):
    torch.cuda.synchronize()
    st = lib.fio_apply_batch_noalloc(plan.handle, fd.shape[0], ctypes.c_void_p(fd.data_ptr()),
                                     ctypes.c_void_p(out.data_ptr()), None)
    return st


def test_noalloc_apply_equals_workspace_apply_twice():
    from paper_math_0610051_amd import Plan, fio
    lib = fio.load_library()
    cases = [(128, 3, "c1c2", (1.0,)), (96, 1, "radial", (0.05, 0.5))]   # the second call is smaller
    for N, B, kind, params in cases:
        print("noalloc: N=%d B=%d %s" % (N, B, kind), flush=True)
        p = Plan(N, kind, 1e-4, params=params, max_batch=4)
        rng = np.random.default_rng(N)
        fd = torch.from_numpy(fi.fhat_from_f(fi.complex_gaussian(N, rng, B=B)).astype(np.complex64)).cuda()
        ref = torch.empty_like(fd)
        st = lib.fio_apply_batch(p.handle, B, ctypes.c_void_p(fd.data_ptr()), ctypes.c_void_p(ref.data_ptr()), None)
        assert st == 0
        out = torch.full_like(fd, float("nan"))
        assert _call(lib, p, fd, out) == 0
        torch.cuda.synchronize()
        assert torch.equal(out, ref), (N, B)
        p.close()


def test_noalloc_refuses_a_plan_beyond_the_array():
    from paper_math_0610051_amd import Plan, fio
    lib = fio.load_library()
    p = Plan(512, "c1c2", 1e-4, params=(1.0,), max_batch=1)
    fd = torch.zeros((1, 512, 512), dtype=torch.complex64, device="cuda")
    out = torch.zeros_like(fd)
    st = _call(lib, p, fd, out)
    assert st == fio.FIO_EINVAL
    assert b"scratch" in lib.fio_last_error()
    p.close()

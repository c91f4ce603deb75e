"""Host-side checks of the C ABI library (no GPU needed).

The library must load on a machine without a GPU, export every function the
header declares, reject bad arguments before touching a device, and its
host linear algebra (the plan's Hermitian eigen-solver) must be right.
"""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_math_0610051_amd import fio

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    return fio.load_library()


def _declared_functions():
    txt = open(os.path.join(ROOT, "include", "fio.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    names = set(re.findall(r"\b(fio_[a-z_0-9]+)\s*\(", txt))
    return sorted(names)


def test_header_declares_the_boundary():
    names = _declared_functions()
    for required in ("fio_plan", "fio_plan_ex", "fio_apply", "fio_apply_batch", "fio_apply_multi",
                     "fio_destroy", "fio_last_error", "fio_plan_info"):
        assert required in names


def test_library_exports_every_declared_symbol(lib):
    missing = [n for n in _declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_default_options(lib):
    o = fio.default_options()
    assert o.precision == 0 and o.partition == 0 and o.max_batch == 8
    assert abs(o.sep_tol_frac - 0.25) < 1e-15 and abs(o.nufft_tol_frac - 0.1) < 1e-15
    assert o.sigma == 2.0 and o.r0 == 32 and o.verify_samples == 200


@pytest.mark.parametrize("n", [1, 2, 3, 5, 16, 33, 128, 256])
def test_host_eigh_matches_lapack(n):
    rng = np.random.default_rng(n)
    A = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    A = A + A.conj().T
    w, V = fio.host_eigh(A)
    ref = np.linalg.eigvalsh(A)[::-1]
    np.testing.assert_allclose(w, ref, atol=1e-12 * max(1, np.abs(ref).max()))
    assert np.max(np.abs(A @ V - V * w)) < 1e-11 * max(1, np.abs(ref).max())
    assert np.max(np.abs(V.conj().T @ V - np.eye(n))) < 1e-12


def test_host_eigh_on_gram_of_unimodular_columns():
    """The plan's use: Gram matrices of exp(i phase) columns, spectrum spanning 1e-14."""
    rng = np.random.default_rng(5)
    m, r = 2000, 24
    t = rng.random(m)
    k = np.linspace(0, 3, r)
    A = np.exp(2j * np.pi * np.outer(t, k) * 0.3)
    G = A.conj().T @ A
    w, V = fio.host_eigh(G)
    s = np.linalg.svd(A, compute_uv=False)
    big = s ** 2 > 1e-12 * s[0] ** 2
    # normwise backward stable: eigenvalue errors of order eps * |G|
    np.testing.assert_allclose(w[big], (s ** 2)[big], rtol=1e-6, atol=1e-14 * s[0] ** 2)


def test_host_column_id_reproduces_a_low_rank_matrix():
    """An exactly rank-6 32 x 32 matrix: the decomposition keeps 6 columns,
    the kept columns are independent, and A[:, rest] = A[:, kept] T to
    rounding; a full-rank matrix keeps every column."""
    rng = np.random.default_rng(9)
    m, n, r = 32, 32, 6
    A = (rng.standard_normal((m, r)) + 1j * rng.standard_normal((m, r))) @ \
        (rng.standard_normal((r, n)) + 1j * rng.standard_normal((r, n)))
    k, perm, T = fio.host_column_id(A, 1e-10)
    assert k == r
    assert sorted(perm) == list(range(n))
    kept, rest = A[:, perm[:k]], A[:, perm[k:]]
    assert np.linalg.matrix_rank(kept) == r
    assert np.linalg.norm(rest - kept @ T) < 1e-11 * np.linalg.norm(A)
    B = rng.standard_normal((m, n)) + 1j * rng.standard_normal((m, n))
    kb, _, _ = fio.host_column_id(B, 1e-10)
    assert kb == n
    # the first pivot is the column of largest norm
    assert np.argmax(np.linalg.norm(B, axis=0)) == fio.host_column_id(B, 1e-10)[1][0]


def _plan_status(N=64, kind=2, tol=1e-4, amp_kind=0, **opts):
    lib = fio.load_library()
    ph = fio.make_phase(kind, (1.0,))
    amp = fio.fio_amplitude()
    amp.kind = amp_kind
    o = fio.default_options()
    for k, v in opts.items():
        setattr(o, k, v)
    h = ctypes.c_void_p()
    st = lib.fio_plan_ex(N, ctypes.byref(ph), ctypes.byref(amp), tol, ctypes.byref(o), ctypes.byref(h))
    return st, h


@pytest.mark.parametrize("kw,status", [
    (dict(N=63), fio.FIO_EINVAL),
    (dict(N=6), fio.FIO_EINVAL),
    (dict(N=8192), fio.FIO_EINVAL),
    (dict(kind=9), fio.FIO_EINVAL),
    (dict(tol=0.0), fio.FIO_EINVAL),
    (dict(tol=1.5), fio.FIO_EINVAL),
    (dict(amp_kind=2), fio.FIO_ENOTSUP),
    (dict(amp_kind=1, kind=0), fio.FIO_EINVAL),   # the Bessel amplitude needs h >= 0
    (dict(tol=1e-8), fio.FIO_ENOTSUP),
    (dict(tol=3e-7, precision=1), fio.FIO_ENOTSUP),
    (dict(precision=7), fio.FIO_EINVAL),
    (dict(partition=3), fio.FIO_EINVAL),
    (dict(max_batch=0), fio.FIO_EINVAL),
    (dict(kernel_width=40), fio.FIO_EINVAL),
    (dict(sigma=1.1), fio.FIO_EINVAL),
    (dict(sep_tol_frac=0.0), fio.FIO_EINVAL),
    (dict(factor_mode=3), fio.FIO_EINVAL),        # learned without a network
    (dict(factor_mode=5), fio.FIO_EINVAL),        # past FIO_FACTORS_TAYLOR
    (dict(factor_mode=2, amp_kind=1), fio.FIO_ENOTSUP),  # FP32 regeneration takes a = 1 only
    (dict(factor_mode=-1), fio.FIO_EINVAL),
])
def test_invalid_plans_are_rejected_before_device_use(kw, status):
    st, h = _plan_status(**kw)
    assert st == status
    assert not h.value
    assert fio.load_library().fio_last_error()


def test_null_handles(lib):
    assert lib.fio_apply(None, None, None, None) == fio.FIO_EINVAL
    assert lib.fio_apply_batch(None, 1, None, None, None) == fio.FIO_EINVAL
    assert lib.fio_destroy(None) == fio.FIO_OK
    assert lib.fio_plan_info(None, None) == fio.FIO_EINVAL
    assert lib.fio_apply_multi(0, None, None, None, None, None) == fio.FIO_EINVAL
    # the copy helper rejects null, misaligned and ragged requests before any launch
    assert lib.fio_copy(None, None, 16, None) == fio.FIO_EINVAL
    assert lib.fio_copy(ctypes.c_void_p(4096), ctypes.c_void_p(8192), 17, None) == fio.FIO_EINVAL
    assert lib.fio_copy(ctypes.c_void_p(4104), ctypes.c_void_p(8192), 32, None) == fio.FIO_EINVAL


def test_python_binding_raises_without_device_tensor():
    with pytest.raises(fio.FioError) as e:
        fio.Plan(63, "c1c2", 1e-4, params=(1.0,))
    assert e.value.status == fio.FIO_EINVAL


def test_plan_files_are_checked_before_device_use(lib, tmp_path):
    """fio_plan_save / fio_plan_load reject null arguments, missing files and
    files that are not (whole) plan files before any device call."""
    h = ctypes.c_void_p()
    assert lib.fio_plan_save(None, b"/tmp/x") == fio.FIO_EINVAL
    assert lib.fio_plan_load(None, ctypes.byref(h)) == fio.FIO_EINVAL
    assert lib.fio_plan_load(str(tmp_path / "none.plan").encode(), ctypes.byref(h)) == fio.FIO_EINVAL
    assert not h.value
    junk = tmp_path / "junk.plan"
    junk.write_bytes(b"not a plan at all, just bytes" * 4)
    assert lib.fio_plan_load(str(junk).encode(), ctypes.byref(h)) == fio.FIO_EINVAL
    assert b"not a plan file" in lib.fio_last_error()
    # the right magic and version, then a header cut short
    cut = tmp_path / "cut.plan"
    cut.write_bytes(b"FIOPLAN1" + (2).to_bytes(4, "little") + (128).to_bytes(4, "little"))
    assert lib.fio_plan_load(str(cut).encode(), ctypes.byref(h)) == fio.FIO_EINVAL
    assert not h.value
    # a file of the first format (no amplitude field) is refused by its version
    old = tmp_path / "old.plan"
    old.write_bytes(b"FIOPLAN1" + (1).to_bytes(4, "little") + bytes(64))
    assert lib.fio_plan_load(str(old).encode(), ctypes.byref(h)) == fio.FIO_EINVAL
    assert b"version" in lib.fio_last_error()


def test_host_eigh_degenerate_and_structured_spectra():
    """Repeated eigenvalues, a zero block, and a matrix already diagonal or
    tridiagonal (reflectors of zero columns are skipped)."""
    rng = np.random.default_rng(7)
    n = 40
    Qm, _ = np.linalg.qr(rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)))
    lam = np.concatenate([np.full(10, 3.0), np.zeros(10), np.linspace(-2, 1, 20)])
    for A in (Qm @ np.diag(lam) @ Qm.conj().T, np.diag(lam).astype(complex),
              np.diag(lam).astype(complex) + np.diag(np.full(n - 1, 0.5j), 1) + np.diag(np.full(n - 1, -0.5j), -1)):
        A = 0.5 * (A + A.conj().T)
        w, V = fio.host_eigh(A)
        ref = np.linalg.eigvalsh(A)[::-1]
        np.testing.assert_allclose(w, ref, atol=1e-12 * max(1, np.abs(ref).max()))
        assert np.max(np.abs(A @ V - V * w)) < 1e-11 * max(1, np.abs(ref).max())
        assert np.max(np.abs(V.conj().T @ V - np.eye(n))) < 1e-12

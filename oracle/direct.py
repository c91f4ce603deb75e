"""ctypes wrapper of the C direct-sum oracle (oracle/direct.c).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).  `build()` compiles
direct.c with gcc/OpenMP into oracle/_build/liboracle_direct.so.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "direct.c")
_OUT_DIR = os.path.join(_HERE, "_build")
_LIB_PATH = os.path.join(_OUT_DIR, "liboracle_direct.so")

PHASE_KINDS = {"linear": 0, "wave": 1, "c1c2": 2, "radial": 3, "paper_ellipse": 4, "paper_circle": 5}

_libs = {}


def build(force: bool = True, plant: int | None = None, out: str | None = None) -> str:
    """Compile the oracle with gcc -O2 -fopenmp; returns the library path.

    `plant` (tests only) builds a variant with a known planted mistake into
    `out`; the default build plants nothing.
    """
    path = out or _LIB_PATH
    os.makedirs(os.path.dirname(path), exist_ok=True)
    if force or not os.path.exists(path):
        tmp = path + ".tmp"
        cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"]
        if plant is not None:
            cmd.insert(1, "-DORACLE_PLANT=%d" % int(plant))
        subprocess.check_call(cmd)
        os.replace(tmp, path)
    return path


def _load(path: str | None = None):
    path = path or _LIB_PATH
    if path not in _libs:
        if not os.path.exists(path):
            build(force=False)
        lib = ctypes.CDLL(path)
        lib.oracle_direct.restype = ctypes.c_int
        lib.oracle_direct.argtypes = [
            ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_int,
            ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_int]
        lib.oracle_direct_amp.restype = ctypes.c_int
        lib.oracle_direct_amp.argtypes = [
            ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_int,
            ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_int]
        lib.oracle_direct_adjoint_amp.restype = ctypes.c_int
        lib.oracle_direct_adjoint_amp.argtypes = [
            ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_int,
            ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int]
        lib.oracle_amp_batch.restype = None
        lib.oracle_amp_batch.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_int, ctypes.c_int] + \
            [ctypes.c_void_p] * 5
        lib.oracle_direct_adjoint.restype = ctypes.c_int
        lib.oracle_direct_adjoint.argtypes = [
            ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_int,
            ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int]
        lib.oracle_h_batch.restype = None
        lib.oracle_h_batch.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_int] + [ctypes.c_void_p] * 5
        lib.oracle_max_threads.restype = ctypes.c_int
        _libs[path] = lib
    return _libs[path]


def _params(p) -> np.ndarray:
    a = np.zeros(8, dtype=np.float64)
    p = np.asarray(p, dtype=np.float64).ravel()
    a[: p.size] = p
    return a


def max_threads() -> int:
    return int(_load().oracle_max_threads())


def amp_values(kind: int, params, amp: int, x1, x2, k1, k2) -> np.ndarray:
    """a(x, xi) from the C oracle at paired points (complex)."""
    x1, x2, k1, k2 = (np.ascontiguousarray(np.asarray(a, dtype=np.float64).ravel()) for a in (x1, x2, k1, k2))
    out = np.empty(2 * x1.size)
    p = _params(params)
    _load().oracle_amp_batch(int(kind), p.ctypes.data, int(amp), x1.size, x1.ctypes.data, x2.ctypes.data,
                             k1.ctypes.data, k2.ctypes.data, out.ctypes.data)
    return out[0::2] + 1j * out[1::2]


def h_values(kind: int, params, x1, x2, k1, k2) -> np.ndarray:
    """h(x, xi) from the C oracle at paired points (for cross-checking families)."""
    x1, x2, k1, k2 = (np.ascontiguousarray(np.asarray(a, dtype=np.float64).ravel()) for a in (x1, x2, k1, k2))
    out = np.empty_like(x1)
    p = _params(params)
    _load().oracle_h_batch(int(kind), p.ctypes.data, x1.size, x1.ctypes.data, x2.ctypes.data,
                           k1.ctypes.data, k2.ctypes.data, out.ctypes.data)
    return out


def direct(N: int, kind: int, params, fhat, xidx, member=None, only: int = 0, threads: int = 0,
           lib_path: str | None = None, amp: int = 0) -> np.ndarray:
    """(Lf)(x) at flat sample indices `xidx` by FP64 direct summation (eq. dfio).

    fhat: (N, N) or (B, N, N) complex, centred layout.  Returns (ns,) or
    (B, ns) complex128.  `member`/`only` restrict the sum to one wedge;
    amp = 1 selects the Bessel amplitude of Section 4 (a = 1 otherwise).
    """
    fh = np.asarray(fhat)
    single = fh.ndim == 2
    fh = np.ascontiguousarray(fh.reshape(-1, N, N).astype(np.complex128))
    B = fh.shape[0]
    xs = np.ascontiguousarray(np.asarray(xidx, dtype=np.int64).ravel())
    out = np.empty((xs.size, B), dtype=np.complex128)
    mem = None
    if member is not None:
        mem = np.ascontiguousarray(np.asarray(member, dtype=np.int32).reshape(N * N))
    p = _params(params)
    lib = _load(lib_path)
    for b0 in range(0, B, 64):
        nb = min(64, B - b0)
        part = np.empty((xs.size, nb), dtype=np.complex128)
        chunk = np.ascontiguousarray(fh[b0:b0 + nb])
        rc = lib.oracle_direct_amp(int(N), int(kind), p.ctypes.data, int(amp), xs.size, xs.ctypes.data, nb,
                                   chunk.ctypes.data, None if mem is None else mem.ctypes.data, int(only),
                                   part.ctypes.data, int(threads))
        if rc != 0:
            raise ValueError("oracle_direct rejected its arguments")
        out[:, b0:b0 + nb] = part
    out = out.T
    return out[0] if single else out


def direct_adjoint(N: int, kind: int, params, g, xiidx, threads: int = 0, lib_path: str | None = None,
                   amp: int = 0) -> np.ndarray:
    """Fourier coefficients of L*g at flat centred frequency indices `xiidx`
    by FP64 direct summation (Section 3.5):
    hhat(xi) = (1/N) sum_y exp(-2 pi i Phi(y, xi)) g(y).

    g: (N, N) or (B, N, N) complex, row-major spatial layout.  Returns (ns,)
    or (B, ns) complex128.
    """
    ga = np.asarray(g)
    single = ga.ndim == 2
    ga = np.ascontiguousarray(ga.reshape(-1, N, N).astype(np.complex128))
    B = ga.shape[0]
    ks = np.ascontiguousarray(np.asarray(xiidx, dtype=np.int64).ravel())
    out = np.empty((ks.size, B), dtype=np.complex128)
    p = _params(params)
    lib = _load(lib_path)
    for b0 in range(0, B, 64):
        nb = min(64, B - b0)
        part = np.empty((ks.size, nb), dtype=np.complex128)
        chunk = np.ascontiguousarray(ga[b0:b0 + nb])
        rc = lib.oracle_direct_adjoint_amp(int(N), int(kind), p.ctypes.data, int(amp), ks.size, ks.ctypes.data,
                                           nb, chunk.ctypes.data, part.ctypes.data, int(threads))
        if rc != 0:
            raise ValueError("oracle_direct_adjoint rejected its arguments")
        out[:, b0:b0 + nb] = part
    out = out.T
    return out[0] if single else out

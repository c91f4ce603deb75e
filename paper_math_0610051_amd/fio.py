"""Thin ctypes binding of the gfx950 FIO library (include/fio.h).

Argument marshalling only: every step of the apply runs in the library's HIP
kernels.  PyTorch supplies device memory and streams (tensors are passed by
data pointer, the stream as torch.cuda.current_stream().cuda_stream).  If
the compiled library is missing, loading raises: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_char_p, c_double, c_int, c_longlong, c_ulonglong, c_void_p

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_lib", "libfio.so")

FIO_OK, FIO_EINVAL, FIO_ENOMEM, FIO_EDEVICE, FIO_EACCURACY, FIO_ENOTSUP = 0, -1, -2, -3, -4, -5
STATUS_NAMES = {0: "FIO_OK", -1: "FIO_EINVAL", -2: "FIO_ENOMEM", -3: "FIO_EDEVICE", -4: "FIO_EACCURACY",
                -5: "FIO_ENOTSUP"}

PHASE_KINDS = {"linear": 0, "wave": 1, "c1c2": 2, "radial": 3, "paper_ellipse": 4, "paper_circle": 5}
PRECISIONS = {"f32": 0, "f64": 1}
PARTITIONS = {"equiangular": 0, "coronae": 1}
FACTOR_MODES = {"auto": 0, "stored": 1, "regen": 2, "learned": 3, "taylor": 4}


class FioError(RuntimeError):
    def __init__(self, status, message):
        super().__init__("%s: %s" % (STATUS_NAMES.get(status, status), message))
        self.status = status


class fio_phase(ctypes.Structure):
    _fields_ = [("kind", c_int), ("p", c_double * 8)]


class fio_amplitude(ctypes.Structure):
    _fields_ = [("kind", c_int), ("p", c_double * 4)]


class fio_options(ctypes.Structure):
    _fields_ = [("precision", c_int), ("partition", c_int), ("n_wedges", c_int), ("factor_mode", c_int),
                ("seed", c_ulonglong), ("max_batch", c_int), ("sep_tol_frac", c_double),
                ("nufft_tol_frac", c_double), ("sigma", c_double), ("kernel_width", c_int), ("r0", c_int),
                ("verify_samples", c_int), ("learned", c_void_p), ("learned_scale", c_double)]


class fio_plan_info_t(ctypes.Structure):
    _fields_ = [("N", c_int), ("L", c_int), ("precision", c_int), ("factor_mode", c_int),
                ("kernel_width", c_int), ("max_rank", c_int), ("min_rank", c_int), ("fallback", c_int),
                ("sigma", c_double), ("tol", c_double), ("plan_ms", c_double), ("max_sep_error", c_double),
                ("fine_cells", c_longlong), ("box_cells", c_longlong), ("factor_bytes", c_longlong),
                ("workspace_bytes", c_longlong), ("compressed_bytes", c_longlong),
                ("learned_sep_error", c_double), ("learned_ms", c_double)]


class fio_tune_result_t(ctypes.Structure):
    _fields_ = [("n_wedges", c_int), ("sigma", c_double), ("kernel_width", c_int), ("sep_tol_frac", c_double),
                ("nufft_tol_frac", c_double), ("ms_per_rhs", c_double), ("error", c_double)]


class fio_wedge_info_t(ctypes.Structure):
    _fields_ = [("theta", c_double), ("members", c_int), ("rank", c_int), ("samples", c_int),
                ("M", c_int * 4), ("xi_c", c_int * 2), ("box", c_int * 2), ("lo", c_int * 2),
                ("fine", c_int * 2), ("sep_error", c_double)]


_lib = None


def load_library():
    """Load libfio.so (built in-tree); raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libfio.so is not built (%s); run __graft_entry__.build()" % LIB_PATH)
    lib = ctypes.CDLL(LIB_PATH)
    P = c_void_p
    sig = {
        "fio_default_options": (None, [POINTER(fio_options)]),
        "fio_plan": (c_int, [c_int, POINTER(fio_phase), POINTER(fio_amplitude), c_double, POINTER(P)]),
        "fio_plan_ex": (c_int, [c_int, POINTER(fio_phase), POINTER(fio_amplitude), c_double,
                                POINTER(fio_options), POINTER(P)]),
        "fio_apply": (c_int, [P, P, P, P]),
        "fio_apply_batch": (c_int, [P, c_int, P, P, P]),
        "fio_apply_multi": (c_int, [c_int, POINTER(P), POINTER(P), POINTER(P), POINTER(c_int), P]),
        "fio_apply_wedges": (c_int, [P, c_int, c_int, c_int, P, P, P]),
        "fio_apply_batch_noalloc": (c_int, [P, c_int, P, P, P]),
        "fio_apply_adjoint": (c_int, [P, P, P, P]),
        "fio_apply_adjoint_batch": (c_int, [P, c_int, P, P, P]),
        "fio_plan_info": (c_int, [P, POINTER(fio_plan_info_t)]),
        "fio_wedge_info": (c_int, [P, c_int, POINTER(fio_wedge_info_t)]),
        "fio_wedge_map": (c_int, [P, P]),
        "fio_wedge_factors": (c_int, [P, c_int, c_int, P, P, c_int, P, P]),
        "fio_wedge_warp": (c_int, [P, c_int, c_int, P, P]),
        "fio_destroy": (c_int, [P]),
        "fio_plan_save": (c_int, [P, c_char_p]),
        "fio_plan_load": (c_int, [c_char_p, POINTER(P)]),
        "fio_profile": (c_int, [P, c_int]),
        "fio_profile_read": (c_int, [P, P, P]),
        "fio_learned_create": (c_int, [c_int, POINTER(fio_phase), c_int, c_ulonglong, POINTER(P)]),
        "fio_learned_generate": (c_int, [P, c_int, P, c_int, c_int]),
        "fio_learned_train": (c_int, [P, c_int, c_int, c_double, c_double, P]),
        "fio_learned_eval": (c_int, [P, P]),
        "fio_learned_params": (c_int, [P, c_int, P, c_int]),
        "fio_learned_param_count": (c_int, []),
        "fio_learned_forward": (c_int, [P, c_int, P, P]),
        "fio_learned_grads": (c_int, [P, c_int, P, P, P, P]),
        "fio_learned_basis": (c_int, [P, c_int, c_int, P, P, P, P]),
        "fio_learned_targets": (c_int, [P, c_int, c_double, c_int, P, P]),
        "fio_learned_adam_step": (c_int, [P, P, c_double]),
        "fio_learned_save": (c_int, [P, c_char_p]),
        "fio_learned_load": (c_int, [c_char_p, POINTER(P)]),
        "fio_learned_destroy": (c_int, [P]),
        "fio_probe_error": (c_int, [P, P, P, c_int, c_ulonglong, P, P]),
        "fio_copy": (c_int, [P, P, ctypes.c_size_t, P]),
        "fio_autotune": (c_int, [c_int, POINTER(fio_phase), POINTER(fio_amplitude), c_double, POINTER(fio_options),
                                 c_int, P, c_int, P, POINTER(fio_tune_result_t)]),
        "fio_last_error": (c_char_p, []),
        "fio_host_eigh": (c_int, [c_int, P, P, P]),
        "fio_host_column_id": (c_int, [c_int, c_int, P, c_double, POINTER(c_int), P, P]),
        "fio_version": (c_char_p, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(status):
    if status != FIO_OK:
        msg = load_library().fio_last_error()
        raise FioError(status, msg.decode() if msg else "")


def make_phase(kind, params=()):
    """fio_phase from a family name or number and its parameters p0, p1, ..."""
    ph = fio_phase()
    ph.kind = PHASE_KINDS[kind] if isinstance(kind, str) else int(kind)
    for i, v in enumerate(params):
        ph.p[i] = float(v)
    return ph


def host_eigh(A: np.ndarray):
    """The library's host Hermitian eigen-solver (for CPU tests of the plan's linear algebra)."""
    A = np.ascontiguousarray(A, dtype=np.complex128)
    n = A.shape[0]
    w = np.empty(n)
    V = np.empty((n, n), dtype=np.complex128)
    _check(load_library().fio_host_eigh(n, A.ctypes.data, w.ctypes.data, V.ctypes.data))
    return w, V


def host_column_id(A: np.ndarray, tol: float):
    """The library's host column interpolative decomposition: (k, perm, T) with
    A[:, perm[k:]] ~ A[:, perm[:k]] @ T (for CPU tests)."""
    A = np.ascontiguousarray(A, dtype=np.complex128)
    m, n = A.shape
    k = c_int(0)
    perm = np.empty(n, dtype=np.int32)
    T = np.zeros(n * n, dtype=np.complex128)
    _check(load_library().fio_host_column_id(m, n, A.ctypes.data, float(tol), ctypes.byref(k), perm.ctypes.data,
                                             T.ctypes.data))
    k = k.value
    return k, perm, T[:k * (n - k)].reshape(k, n - k)


def default_options() -> fio_options:
    o = fio_options()
    load_library().fio_default_options(ctypes.byref(o))
    return o


def _torch():
    import torch
    return torch


AMPLITUDES = {"one": 0, "bessel": 1}


class Plan:
    """A built operator: fio_plan_ex(N, phase, amplitude, tol, options); amplitude
    "one" (a = 1) or "bessel" (the Section 4 amplitude)."""

    def __init__(self, N, phase, tol, *, params=(), precision="f32", partition="equiangular", n_wedges=0,
                 seed=None, max_batch=8, sep_tol_frac=None, nufft_tol_frac=None, sigma=None, kernel_width=0,
                 r0=0, verify_samples=0, factor_mode="auto", learned=None, learned_scale=1.0, amplitude="one"):
        lib = load_library()
        self._lib = lib
        self.N = int(N)
        self.precision = precision
        ph = phase if isinstance(phase, fio_phase) else make_phase(phase, params)
        amp = fio_amplitude()
        amp.kind = AMPLITUDES[amplitude]
        o = default_options()
        o.precision = PRECISIONS[precision]
        o.partition = PARTITIONS[partition]
        o.n_wedges = int(n_wedges)
        o.factor_mode = FACTOR_MODES[factor_mode]
        if seed is not None:
            o.seed = int(seed)
        o.max_batch = int(max_batch)
        if sep_tol_frac is not None:
            o.sep_tol_frac = float(sep_tol_frac)
        if nufft_tol_frac is not None:
            o.nufft_tol_frac = float(nufft_tol_frac)
        if sigma is not None:
            o.sigma = float(sigma)
        o.kernel_width = int(kernel_width)
        if r0:
            o.r0 = int(r0)
        if verify_samples:
            o.verify_samples = int(verify_samples)
        self._learned = learned  # keep the network alive while the plan exists
        if learned is not None:
            o.learned = learned.handle
            o.learned_scale = float(learned_scale)
        h = c_void_p()
        _check(lib.fio_plan_ex(self.N, ctypes.byref(ph), ctypes.byref(amp), float(tol), ctypes.byref(o),
                               ctypes.byref(h)))
        self.handle = h
        self.phase = ph

    # -- plan files
    def save(self, path):
        """Write the plan (build inputs and compressed factors) to `path`: fio_plan_save."""
        _check(self._lib.fio_plan_save(self.handle, str(path).encode()))

    @classmethod
    def load(cls, path):
        """A plan written by save(), rebuilt on the current device: fio_plan_load."""
        lib = load_library()
        h = c_void_p()
        _check(lib.fio_plan_load(str(path).encode(), ctypes.byref(h)))
        self = cls.__new__(cls)
        self._lib = lib
        self.handle = h
        self._learned = None
        self.phase = None
        info = self.info()
        self.N = int(info["N"])
        self.precision = "f64" if info["precision"] == PRECISIONS["f64"] else "f32"
        return self

    # -- lifetime
    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            self._lib.fio_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -- apply
    @property
    def dtype(self):
        torch = _torch()
        return torch.complex128 if self.precision == "f64" else torch.complex64

    def _io(self, fhat, out):
        torch = _torch()
        if not isinstance(fhat, torch.Tensor) or not fhat.is_cuda:
            raise TypeError("fhat must be a device tensor")
        if fhat.dtype != self.dtype:
            raise TypeError("fhat must be %s for a %s plan" % (self.dtype, self.precision))
        if fhat.shape[-2:] != (self.N, self.N) or fhat.dim() not in (2, 3):
            raise ValueError("fhat must have shape (N, N) or (B, N, N)")
        fhat = fhat.contiguous()
        if out is None:
            out = torch.empty_like(fhat)
        elif out.shape != fhat.shape or out.dtype != fhat.dtype or not out.is_contiguous():
            raise ValueError("out must be a contiguous tensor like fhat")
        B = 1 if fhat.dim() == 2 else fhat.shape[0]
        stream = torch.cuda.current_stream(fhat.device).cuda_stream
        return fhat, out, B, stream

    def apply(self, fhat, out=None):
        """u = L fhat for (N, N) or (B, N, N) centred fhat; returns u (row-major grid)."""
        fhat, out, B, stream = self._io(fhat, out)
        _check(self._lib.fio_apply_batch(self.handle, B, c_void_p(fhat.data_ptr()), c_void_p(out.data_ptr()),
                                         c_void_p(stream)))
        return out

    def apply_adjoint(self, g, out=None):
        """Fourier coefficients of L*g (centred) for (N, N) or (B, N, N) row-major g."""
        g, out, B, stream = self._io(g, out)
        _check(self._lib.fio_apply_adjoint_batch(self.handle, B, c_void_p(g.data_ptr()), c_void_p(out.data_ptr()),
                                                 c_void_p(stream)))
        return out

    def apply_noalloc(self, fhat, out):
        """fio_apply_batch_noalloc: u = L fhat into the caller's `out`, with the
        library's fixed scratch array in place of the plan's workspace."""
        if out is None:
            raise ValueError("apply_noalloc writes into a caller-provided out")
        fhat, out, B, stream = self._io(fhat, out)
        _check(self._lib.fio_apply_batch_noalloc(self.handle, B, c_void_p(fhat.data_ptr()),
                                                 c_void_p(out.data_ptr()), c_void_p(stream)))
        return out

    def apply_wedges(self, l0, l1, fhat, out=None):
        """Partial operator sum_{l0 <= ell < l1} L_ell fhat."""
        fhat, out, B, stream = self._io(fhat, out)
        _check(self._lib.fio_apply_wedges(self.handle, int(l0), int(l1), B, c_void_p(fhat.data_ptr()),
                                          c_void_p(out.data_ptr()), c_void_p(stream)))
        return out

    # -- introspection
    def info(self) -> dict:
        o = fio_plan_info_t()
        _check(self._lib.fio_plan_info(self.handle, ctypes.byref(o)))
        return {k: getattr(o, k) for k, _ in o._fields_}

    @property
    def L(self):
        return self.info()["L"]

    def wedge_info(self, ell) -> dict:
        o = fio_wedge_info_t()
        _check(self._lib.fio_wedge_info(self.handle, int(ell), ctypes.byref(o)))
        d = {}
        for k, _ in o._fields_:
            v = getattr(o, k)
            d[k] = list(v) if isinstance(v, ctypes.Array) else v
        return d

    def wedge_map(self) -> np.ndarray:
        ids = np.empty(self.N * self.N, dtype=np.int32)
        _check(self._lib.fio_wedge_map(self.handle, ids.ctypes.data))
        return ids.reshape(self.N, self.N)

    def wedge_factors(self, ell, xidx=(), xiidx=()):
        """Stored gamma^x at flat grid indices and gamma^xi at centred frequency indices (FP64 copies)."""
        q = self.wedge_info(ell)["rank"]
        xs = np.ascontiguousarray(np.asarray(xidx, dtype=np.int64).ravel())
        ks = np.ascontiguousarray(np.asarray(xiidx, dtype=np.int64).ravel())
        gx = np.zeros((xs.size, q), dtype=np.complex128)
        gxi = np.zeros((ks.size, q), dtype=np.complex128)
        _check(self._lib.fio_wedge_factors(self.handle, int(ell), xs.size, xs.ctypes.data if xs.size else None,
                                           gx.ctypes.data if xs.size else None, ks.size,
                                           ks.ctypes.data if ks.size else None, gxi.ctypes.data if ks.size else None))
        return gx, gxi

    def profile(self, on=True):
        """Start (and clear) or stop per-stage HIP-event timing of the apply stages."""
        _check(self._lib.fio_profile(self.handle, 1 if on else 0))

    def profile_read(self):
        """(ms per stage summed, launches per stage) for stages window+row FFT, column FFT, interpolation."""
        ms = np.zeros(3)
        n = np.zeros(3, dtype=np.int64)
        _check(self._lib.fio_profile_read(self.handle, ms.ctypes.data, n.ctypes.data))
        return ms, n

    def probe_error(self, fhat, u, nsamples=128, seed=1):
        """Relative l2 error of u against an on-device FP64 direct sum at sampled points."""
        torch = _torch()
        err = ctypes.c_double()
        stream = torch.cuda.current_stream(fhat.device).cuda_stream
        _check(self._lib.fio_probe_error(self.handle, c_void_p(fhat.data_ptr()), c_void_p(u.data_ptr()),
                                         int(nsamples), int(seed), ctypes.byref(err), c_void_p(stream)))
        return err.value

    def wedge_warp(self, ell, xidx):
        xs = np.ascontiguousarray(np.asarray(xidx, dtype=np.int64).ravel())
        y = np.zeros((xs.size, 2))
        _check(self._lib.fio_wedge_warp(self.handle, int(ell), xs.size, xs.ctypes.data, y.ctypes.data))
        return y


def apply_multi(plans, fhats, outs=None):
    """One fio_apply_multi call over instances of possibly different N."""
    torch = _torch()
    lib = load_library()
    n = len(plans)
    if outs is None:
        outs = [torch.empty_like(f) for f in fhats]
    hs = (c_void_p * n)(*[p.handle.value for p in plans])
    fs = (c_void_p * n)(*[f.data_ptr() for f in fhats])
    us = (c_void_p * n)(*[u.data_ptr() for u in outs])
    Bs = (c_int * n)(*[1 if f.dim() == 2 else f.shape[0] for f in fhats])
    for p, f, u in zip(plans, fhats, outs):
        if f.dtype != p.dtype or f.shape[-2:] != (p.N, p.N) or not f.is_contiguous() or u.shape != f.shape:
            raise ValueError("instance tensors must match their plans")
    stream = torch.cuda.current_stream(fhats[0].device).cuda_stream
    _check(lib.fio_apply_multi(n, hs, fs, us, Bs, c_void_p(stream)))
    return outs


class Learned:
    """The spatial-factor network (fio_learned_*): training data from the
    method's separation, BF16 matrix-core training and inference on the device."""

    def __init__(self, N, family, params=(), n_wedges=0, seed=1234, _handle=None):
        lib = load_library()
        self._lib = lib
        if _handle is not None:
            self.handle = _handle
            return
        ph = family if isinstance(family, fio_phase) else make_phase(family, params)
        h = c_void_p()
        _check(lib.fio_learned_create(int(N), ctypes.byref(ph), int(n_wedges), int(seed), ctypes.byref(h)))
        self.handle = h

    @staticmethod
    def param_count():
        return int(load_library().fio_learned_param_count())

    @classmethod
    def load(cls, path):
        lib = load_library()
        h = c_void_p()
        _check(lib.fio_learned_load(str(path).encode(), ctypes.byref(h)))
        return cls(0, None, _handle=h)

    def save(self, path):
        _check(self._lib.fio_learned_save(self.handle, str(path).encode()))

    def generate(self, scales, x_samples=4096, r_cols=48):
        sc = np.ascontiguousarray(np.asarray(scales, dtype=np.float64))
        _check(self._lib.fio_learned_generate(self.handle, sc.size, sc.ctypes.data, int(x_samples), int(r_cols)))

    def train(self, steps, batch=4096, lr=2e-3, lr_final=2e-5):
        loss = ctypes.c_double()
        _check(self._lib.fio_learned_train(self.handle, int(steps), int(batch), float(lr), float(lr_final),
                                           ctypes.byref(loss)))
        return loss.value

    def eval(self):
        loss = ctypes.c_double()
        _check(self._lib.fio_learned_eval(self.handle, ctypes.byref(loss)))
        return loss.value

    def params(self, values=None):
        n = self.param_count()
        if values is None:
            out = np.empty(n, dtype=np.float32)
            _check(self._lib.fio_learned_params(self.handle, 1, out.ctypes.data, n))
            return out
        v = np.ascontiguousarray(np.asarray(values, dtype=np.float32))
        _check(self._lib.fio_learned_params(self.handle, 0, v.ctypes.data, n))

    def forward(self, feat):
        f = np.ascontiguousarray(np.asarray(feat, dtype=np.float32))
        out = np.empty((f.shape[0], 32), dtype=np.float32)
        _check(self._lib.fio_learned_forward(self.handle, f.shape[0], f.ctypes.data, out.ctypes.data))
        return out

    def grads(self, feat, target):
        f = np.ascontiguousarray(np.asarray(feat, dtype=np.float32))
        t = np.ascontiguousarray(np.asarray(target, dtype=np.float32))
        g = np.empty(self.param_count(), dtype=np.float32)
        loss = ctypes.c_double()
        _check(self._lib.fio_learned_grads(self.handle, f.shape[0], f.ctypes.data, t.ctypes.data, g.ctypes.data,
                                           ctypes.byref(loss)))
        return g, loss.value

    def basis(self, ell):
        """(cols (r, 2) centred frequencies, V (r, 16) complex, s1) of wedge ell's targets."""
        cap = 256
        cols = np.empty(2 * cap)
        V = np.empty(32 * cap)
        r = ctypes.c_int()
        s1 = ctypes.c_double()
        _check(self._lib.fio_learned_basis(self.handle, int(ell), cap, ctypes.byref(r), cols.ctypes.data,
                                           V.ctypes.data, ctypes.byref(s1)))
        n = r.value
        Vc = V[:32 * n].reshape(n, 16, 2)
        return cols[:2 * n].reshape(n, 2).astype(np.int64), Vc[..., 0] + 1j * Vc[..., 1], s1.value

    def targets(self, ell, scale, xidx):
        """Training targets of wedge ell at phase scale `scale` at flat grid indices, (n, 32) float32."""
        x = np.ascontiguousarray(np.asarray(xidx, dtype=np.int64))
        out = np.empty((x.size, 32), dtype=np.float32)
        _check(self._lib.fio_learned_targets(self.handle, int(ell), float(scale), x.size, x.ctypes.data,
                                             out.ctypes.data))
        return out

    def adam_step(self, grads, lr):
        g = np.ascontiguousarray(np.asarray(grads, dtype=np.float32))
        if g.size != self.param_count():
            raise ValueError("gradient vector of the wrong size")
        _check(self._lib.fio_learned_adam_step(self.handle, g.ctypes.data, float(lr)))

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            self._lib.fio_learned_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def copy(src, dst):
    """fio_copy of src into dst (device tensors of equal byte size) on the current stream."""
    torch = _torch()
    nb = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != nb or not (src.is_cuda and dst.is_cuda):
        raise ValueError("copy needs two device tensors of the same byte size")
    stream = torch.cuda.current_stream(src.device).cuda_stream
    _check(load_library().fio_copy(c_void_p(src.data_ptr()), c_void_p(dst.data_ptr()), nb, c_void_p(stream)))
    return dst


def autotune(N, phase, tol, params=(), B=1, precision="f32", max_tried=256):
    """fio_autotune: returns (best, tried) as dicts; best's fields map onto Plan keywords."""
    lib = load_library()
    ph = phase if isinstance(phase, fio_phase) else make_phase(phase, params)
    amp = fio_amplitude()
    o = default_options()
    o.precision = PRECISIONS[precision]
    tried = (fio_tune_result_t * max_tried)()
    n = c_int()
    best = fio_tune_result_t()
    _check(lib.fio_autotune(int(N), ctypes.byref(ph), ctypes.byref(amp), float(tol), ctypes.byref(o), int(B),
                            tried, max_tried, ctypes.byref(n), ctypes.byref(best)))
    conv = lambda r: {k: getattr(r, k) for k, _ in r._fields_}
    return conv(best), [conv(tried[i]) for i in range(n.value)]

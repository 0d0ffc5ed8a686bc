"""ctypes binding of ``libchebdm.so``: argument marshalling only.

Every step of the computation runs in the library's HIP kernels; this module
turns torch tensors into device pointers and leading dimensions, picks up
torch's current HIP stream, and converts status codes into exceptions.
There is no fallback: if the library is missing the import of the first
entry point raises.
"""
from __future__ import annotations

import ctypes
import math
import os
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libchebdm.so")

FP64, FP32, BF16X3, BF16X6 = 0, 1, 2, 3
COMPOSITION, POWER = 0, 1
OK, WARN_NOCONV = 0, 1
ERR_ARG, ERR_HIP, ERR_OOM, ERR_NONFINITE, ERR_BRACKET, ERR_UNSUPPORTED = -1, -2, -3, -4, -5, -6

_PREC_NAMES = {"fp64": FP64, "f64": FP64, "fp32": FP32, "f32": FP32, "bf16x3": BF16X3, "bf16x6": BF16X6}
_BABY_NAMES = {"auto": 0, "stages": 1, "sequential": 2, "odd_chains": 3}
_FORM_NAMES = {"composition": COMPOSITION, "clenshaw": COMPOSITION, "power": POWER, "horner": POWER,
               "one_chain": 2, "two_chains": 3, "four_chains": 4}


class Opts(ctypes.Structure):
    _fields_ = [("prec", ctypes.c_int32), ("giant_form", ctypes.c_int32), ("k_override", ctypes.c_int32),
                ("n_quad", ctypes.c_int32), ("max_iter", ctypes.c_int32), ("baby_steps", ctypes.c_int32),
                ("search", ctypes.c_int32), ("damping", ctypes.c_int32), ("tol", ctypes.c_double),
                ("bounds", ctypes.c_int32), ("lanczos_steps", ctypes.c_int32), ("bounds_margin", ctypes.c_double)]


class Info(ctypes.Structure):
    _fields_ = [("k", ctypes.c_int32), ("m", ctypes.c_int32), ("n_gemm", ctypes.c_int32),
                ("n_quad", ctypes.c_int32), ("iters", ctypes.c_int32), ("status", ctypes.c_int32),
                ("emin", ctypes.c_double), ("emax", ctypes.c_double), ("mu", ctypes.c_double),
                ("trace", ctypes.c_double), ("trace_err", ctypes.c_double)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class Profile(ctypes.Structure):
    _fields_ = [("gemm_launches", ctypes.c_int64), ("gemm_products", ctypes.c_int64), ("gemm_ms", ctypes.c_double),
                ("gemm_flop", ctypes.c_double), ("combine_calls", ctypes.c_int64), ("combine_ms", ctypes.c_double),
                ("combine_bytes", ctypes.c_double), ("gram_calls", ctypes.c_int64), ("gram_ms", ctypes.c_double),
                ("gram_bytes", ctypes.c_double), ("search_calls", ctypes.c_int64), ("search_ms", ctypes.c_double)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class ChebdmError(RuntimeError):
    def __init__(self, code: int, message: str):
        super().__init__(f"chebdm error {code}: {message}")
        self.code = code


_lib = None

_SIGNATURES = {
    "chebdm_default_opts": (None, [ctypes.POINTER(Opts)]),
    "chebdm_abi_version": (ctypes.c_int, []),
    "chebdm_last_error": (ctypes.c_char_p, []),
    "chebdm_create": (ctypes.c_int, [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int, ctypes.c_void_p]),
    "chebdm_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "chebdm_set_stream": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "chebdm_bounds": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64,
                                     ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]),
    "chebdm_bounds_noalloc": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64,
                                             ctypes.c_void_p]),
    "chebdm_bounds_lanczos": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64,
                                             ctypes.c_int32, ctypes.c_double, ctypes.c_uint64,
                                             ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                                             ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                                             ctypes.POINTER(ctypes.c_int32)]),
    "chebdm_commutator_norm": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                                              ctypes.c_int64, ctypes.c_int64, ctypes.POINTER(ctypes.c_double)]),
    "chebdm_coeffs": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                     ctypes.c_double, ctypes.c_int32, ctypes.c_int32,
                                     ctypes.POINTER(ctypes.c_double)]),
    "chebdm_density": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64,
                                      ctypes.c_double, ctypes.c_double, ctypes.c_int32, ctypes.POINTER(Opts),
                                      ctypes.c_double, ctypes.c_double, ctypes.c_void_p, ctypes.c_int64,
                                      ctypes.POINTER(Info)]),
    "chebdm_mu_search": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64,
                                        ctypes.c_double, ctypes.c_double, ctypes.c_int32, ctypes.POINTER(Opts),
                                        ctypes.c_double, ctypes.c_double, ctypes.POINTER(ctypes.c_double),
                                        ctypes.c_void_p, ctypes.c_int64, ctypes.POINTER(Info)]),
    "chebdm_moments": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64,
                                      ctypes.c_int32, ctypes.POINTER(Opts), ctypes.c_double, ctypes.c_double,
                                      ctypes.POINTER(ctypes.c_double)]),
    "chebdm_block_coeffs": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.c_int32,
                                           ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32),
                                           ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_double)]),
    "chebdm_batch_create": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_int64),
                                           ctypes.c_int32, ctypes.POINTER(Opts), ctypes.c_int64,
                                           ctypes.POINTER(ctypes.c_void_p)]),
    "chebdm_batch_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "chebdm_batch_tune": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_char_p, ctypes.c_char_p, ctypes.c_int32]),
    "chebdm_batch_mu_search": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p),
                                              ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_double),
                                              ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_void_p),
                                              ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_double),
                                              ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                                              ctypes.POINTER(ctypes.c_double)]),
    "chebdm_batch_info": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int32),
                                         ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                                         ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_double)]),
    "chebdm_batch_set_search": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_double]),
    "chebdm_batch_stats": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int32),
                                          ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_double),
                                          ctypes.POINTER(ctypes.c_double)]),
    "chebdm_batch_features": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "chebdm_mlp_num_params": (ctypes.c_int, []),
    "chebdm_mlp_forward": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                                          ctypes.c_void_p]),
    "chebdm_mlp_backward": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                           ctypes.c_int32, ctypes.c_void_p, ctypes.POINTER(ctypes.c_float)]),
    "chebdm_mlp_adam": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                       ctypes.c_void_p, ctypes.c_int32, ctypes.c_float, ctypes.c_float,
                                       ctypes.c_float, ctypes.c_float]),
    "chebdm_workspace_size": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.POINTER(Opts),
                                             ctypes.POINTER(ctypes.c_size_t)]),
    "chebdm_profile_enable": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int]),
    "chebdm_profile_read": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Profile)]),
}

EXPORTED = tuple(_SIGNATURES)


def load_library(path: str = LIB_PATH):
    """Load ``libchebdm.so`` once; raise if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    # torch first: the library then binds to the HIP runtime torch has loaded; loaded the other
    # way round, the process holds two runtimes and the second finds no device
    import torch  # noqa: F401

    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_2306_12616_amd.build` "
                           "(there is no CPU fallback)")
    lib = ctypes.CDLL(path)
    for name, (res, args) in _SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(rc: int, allow_warn: bool = False) -> int:
    if rc < 0 or (rc > 0 and not allow_warn):
        msg = load_library().chebdm_last_error().decode(errors="replace")
        raise ChebdmError(rc, msg)
    return rc


_SEARCH_NAMES = {"bisection": 0, "newton": 1}
_DAMPING_NAMES = {"none": 0, "jackson": 1}
_BOUNDS_NAMES = {"gershgorin": 0, "lanczos": 1}


def make_opts(prec="fp64", giant="composition", k_override: int = 0, n_quad: int = 0,
              max_iter: int = 0, tol: float = 0.0, baby="auto", search="bisection", damping="none",
              bounds="gershgorin", lanczos_steps: int = 0, bounds_margin: float = 0.0) -> Opts:
    o = Opts()
    load_library().chebdm_default_opts(ctypes.byref(o))
    o.prec = _PREC_NAMES[prec] if isinstance(prec, str) else int(prec)
    o.giant_form = _FORM_NAMES[giant] if isinstance(giant, str) else int(giant)
    o.k_override = int(k_override)
    o.n_quad = int(n_quad)
    o.baby_steps = _BABY_NAMES[baby] if isinstance(baby, str) else int(baby)
    o.search = _SEARCH_NAMES[search] if isinstance(search, str) else int(search)
    o.damping = _DAMPING_NAMES[damping] if isinstance(damping, str) else int(damping)
    o.bounds = _BOUNDS_NAMES[bounds] if isinstance(bounds, str) else int(bounds)
    o.lanczos_steps = int(lanczos_steps)
    o.bounds_margin = float(bounds_margin)
    if max_iter:
        o.max_iter = int(max_iter)
    if tol:
        o.tol = float(tol)
    return o


def _current_stream_ptr(device: int) -> int:
    import torch

    return int(torch.cuda.current_stream(device).cuda_stream)


def _matrix_args(t, name: str):
    import torch

    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a torch tensor on a HIP device")
    if t.dtype != torch.float64 or t.dim() != 2 or t.shape[0] != t.shape[1]:
        raise TypeError(f"{name} must be a square float64 matrix")
    if t.stride(1) != 1 or t.stride(0) < t.shape[0]:
        raise TypeError(f"{name} must be row-major with leading dimension >= n")
    return ctypes.c_void_p(t.data_ptr()), int(t.shape[0]), int(t.stride(0))


class Handle:
    """Owns a ``chebdm_handle`` bound to one device; follows torch's current stream."""

    def __init__(self, device: int = 0):
        lib = load_library()
        self.device = int(device)
        self._stream = _current_stream_ptr(self.device)
        h = ctypes.c_void_p()
        _check(lib.chebdm_create(ctypes.byref(h), self.device, ctypes.c_void_p(self._stream)))
        self._h = h

    @property
    def ptr(self):
        s = _current_stream_ptr(self.device)
        if s != self._stream:
            _check(load_library().chebdm_set_stream(self._h, ctypes.c_void_p(s)))
            self._stream = s
        return self._h

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            load_library().chebdm_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def chebdm_bounds(h: Handle, H):
    p, n, ld = _matrix_args(H, "H")
    lo, hi = ctypes.c_double(), ctypes.c_double()
    _check(load_library().chebdm_bounds(h.ptr, p, n, ld, ctypes.byref(lo), ctypes.byref(hi)))
    return lo.value, hi.value


def chebdm_bounds_noalloc(h: Handle, H, out):
    """Gershgorin bounds into `out` (a float64 device tensor of at least 2 elements), stream-ordered,
    no device allocation and no synchronisation (NaN, NaN when H holds NaN or Inf)."""
    import torch

    p, n, ld = _matrix_args(H, "H")
    if not isinstance(out, torch.Tensor) or not out.is_cuda or out.dtype != torch.float64 or \
            not out.is_contiguous() or out.numel() < 2:
        raise TypeError("out must be a contiguous float64 device tensor of at least 2 elements")
    _check(load_library().chebdm_bounds_noalloc(h.ptr, p, n, ld, ctypes.c_void_p(out.data_ptr())))
    return out


def chebdm_bounds_lanczos(h: Handle, H, steps: int = 40, margin: float = 0.01, seed: int = 0):
    """(emin, emax, alpha, beta): Lanczos bounds and the tridiagonal (alpha, beta of the steps done)."""
    p, n, ld = _matrix_args(H, "H")
    lo, hi = ctypes.c_double(), ctypes.c_double()
    a = np.zeros(steps, dtype=np.float64)
    b = np.zeros(steps, dtype=np.float64)
    done = ctypes.c_int32()
    dp = ctypes.POINTER(ctypes.c_double)
    _check(load_library().chebdm_bounds_lanczos(h.ptr, p, n, ld, int(steps), float(margin), int(seed),
                                                ctypes.byref(lo), ctypes.byref(hi), a.ctypes.data_as(dp),
                                                b.ctypes.data_as(dp), ctypes.byref(done)))
    k = done.value
    return lo.value, hi.value, a[:k], b[:k]


def chebdm_commutator_norm(h: Handle, H, D) -> float:
    """max |H D - D H| of two symmetric device matrices (float64)."""
    p, n, ld = _matrix_args(H, "H")
    pd, nd, ldd = _matrix_args(D, "D")
    if nd != n:
        raise ValueError("D must match H's size")
    out = ctypes.c_double()
    _check(load_library().chebdm_commutator_norm(h.ptr, p, ld, pd, ldd, n, ctypes.byref(out)))
    return out.value


def chebdm_coeffs(h: Handle, beta: float, mu: float, emin: float, emax: float, order: int, n_quad: int = 0):
    out = np.empty(order + 1, dtype=np.float64)
    _check(load_library().chebdm_coeffs(h.ptr, beta, mu, emin, emax, order, n_quad,
                                        out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
    return out


def chebdm_block_coeffs(h: Handle, c, order: int, giant="composition", k_override: int = 0):
    c = np.ascontiguousarray(c, dtype=np.float64)
    if c.size < order + 1:
        raise ValueError("need order + 1 coefficients")
    form = _FORM_NAMES[giant] if isinstance(giant, str) else int(giant)
    k, m = ctypes.c_int32(), ctypes.c_int32()
    lib = load_library()
    _check(lib.chebdm_block_coeffs(h.ptr, None, order, form, k_override, ctypes.byref(k), ctypes.byref(m), None))
    out = np.empty(k.value * m.value, dtype=np.float64)
    _check(lib.chebdm_block_coeffs(h.ptr, c.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), order, form,
                                   k_override, ctypes.byref(k), ctypes.byref(m),
                                   out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
    return k.value, m.value, out.reshape(m.value, k.value)


def chebdm_density(h: Handle, H, beta: float, mu: float, order: int, opts: Optional[Opts] = None,
                   emin: float = math.nan, emax: float = math.nan, D=None, want_info: bool = True):
    import torch

    p, n, ld = _matrix_args(H, "H")
    if D is None:
        D = torch.empty((n, n), dtype=torch.float64, device=H.device)
    pd, nd, ldd = _matrix_args(D, "D")
    if nd != n:
        raise ValueError("D must match H's size")
    info = Info()
    _check(load_library().chebdm_density(h.ptr, p, n, ld, beta, mu, order,
                                         ctypes.byref(opts) if opts is not None else None, emin, emax, pd, ldd,
                                         ctypes.byref(info) if want_info else None))
    return D, (info.as_dict() if want_info else None)


def chebdm_mu_search(h: Handle, H, beta: float, n_elec: float, order: int, opts: Optional[Opts] = None,
                     emin: float = math.nan, emax: float = math.nan, want_density: bool = True, D=None,
                     allow_noconv: bool = True):
    import torch

    p, n, ld = _matrix_args(H, "H")
    pd, ldd = None, n
    if want_density:
        if D is None:
            D = torch.empty((n, n), dtype=torch.float64, device=H.device)
        pd, nd, ldd = _matrix_args(D, "D")
        if nd != n:
            raise ValueError("D must match H's size")
    else:
        D = None
    mu = ctypes.c_double()
    info = Info()
    rc = load_library().chebdm_mu_search(h.ptr, p, n, ld, beta, n_elec, order,
                                         ctypes.byref(opts) if opts is not None else None, emin, emax,
                                         ctypes.byref(mu), pd, ldd, ctypes.byref(info))
    _check(rc, allow_warn=allow_noconv)
    return mu.value, D, info.as_dict()


def chebdm_moments(h: Handle, H, order: int, opts: Optional[Opts] = None, emin: float = math.nan,
                   emax: float = math.nan):
    p, n, ld = _matrix_args(H, "H")
    out = np.empty(order + 1, dtype=np.float64)
    _check(load_library().chebdm_moments(h.ptr, p, n, ld, order, ctypes.byref(opts) if opts is not None else None,
                                         emin, emax, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
    return out


def chebdm_profile_enable(h: Handle, enable: bool = True):
    _check(load_library().chebdm_profile_enable(h.ptr, 1 if enable else 0))


def chebdm_workspace_size(n: int, order: int, opts: Optional[Opts] = None) -> int:
    """Device bytes a handle holds for calls of this size (no device needed)."""
    out = ctypes.c_size_t()
    _check(load_library().chebdm_workspace_size(None, int(n), int(order),
                                                ctypes.byref(opts) if opts is not None else None, ctypes.byref(out)))
    return int(out.value)


def chebdm_profile_read(h: Handle):
    p = Profile()
    _check(load_library().chebdm_profile_read(h.ptr, ctypes.byref(p)))
    return p.as_dict()


def _arr(ctype, values):
    a = (ctype * len(values))()
    for i, v in enumerate(values):
        a[i] = v
    return a


class Batch:
    """A batched plan (``chebdm_batch``): many Hamiltonians of different n, one order, one graph."""

    def __init__(self, handle: Handle, sizes, order: int, opts: Optional[Opts] = None, max_quad: int = 0):
        self.handle = handle
        self.sizes = [int(v) for v in sizes]
        self.order = int(order)
        b = ctypes.c_void_p()
        _check(load_library().chebdm_batch_create(handle.ptr, len(self.sizes), _arr(ctypes.c_int64, self.sizes),
                                                  self.order, ctypes.byref(opts) if opts is not None else None,
                                                  int(max_quad), ctypes.byref(b)))
        self._b = b
        self.search_mode = int(opts.search) if opts is not None else 0
        self._weights = None

    def tune(self, cache_path: Optional[str] = None) -> str:
        buf = ctypes.create_string_buffer(1024)
        _check(load_library().chebdm_batch_tune(self._b, cache_path.encode() if cache_path else None, buf, 1024))
        return buf.value.decode()

    def info(self):
        k, m, pp = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        tiles, flop = ctypes.c_int64(), ctypes.c_double()
        _check(load_library().chebdm_batch_info(self._b, ctypes.byref(k), ctypes.byref(m), ctypes.byref(pp),
                                                ctypes.byref(tiles), ctypes.byref(flop)))
        return {"k": k.value, "m": m.value, "products_per_problem": pp.value, "tiles_per_step": tiles.value,
                "flop_per_run": flop.value}

    SEARCH_MODES = {"bisection": 0, "newton": 1, "learned": 2}

    def set_search(self, mode="bisection", weights=None, delta: float = 0.02):
        """Search mode for later runs; ``weights`` (device float32, kept alive here) for "learned"."""
        m = self.SEARCH_MODES[mode] if isinstance(mode, str) else int(mode)
        ptr = None
        if weights is not None:
            if weights.dtype != _torch().float32 or not weights.is_contiguous() or \
                    weights.numel() != chebdm_mlp_num_params():
                raise ValueError("weights must be a contiguous float32 vector of chebdm_mlp_num_params() entries")
            ptr = weights.data_ptr()
        _check(load_library().chebdm_batch_set_search(self._b, m, ptr, float(delta)))
        self._weights = weights
        self.search_mode = m

    def stats(self):
        """Per problem: evaluations of t, learned bracket taken, mu~ and beta' of the last run."""
        count = len(self.sizes)
        ev, le = (ctypes.c_int32 * count)(), (ctypes.c_int32 * count)()
        mus, bs = (ctypes.c_double * count)(), (ctypes.c_double * count)()
        _check(load_library().chebdm_batch_stats(self._b, ev, le, mus, bs))
        return (np.array(ev[:], dtype=np.int32), np.array(le[:], dtype=np.int32), np.array(mus[:]),
                np.array(bs[:]))

    def features(self):
        """Network inputs of the last run (count x 64, float32 on the plan's device)."""
        torch = _torch()
        out = torch.empty((len(self.sizes), 64), dtype=torch.float32, device=f"cuda:{self.handle.device}")
        _check(load_library().chebdm_batch_features(self._b, ctypes.c_void_p(out.data_ptr())))
        return out

    def mu_only(self, Hs, betas, n_elecs, allow_errors: bool = False):
        """Moments and mu search only (no density); returns (mu, status, iters, t(mu))."""
        return self._run(Hs, betas, n_elecs, None, allow_errors, with_density=False)

    def mu_search(self, Hs, betas, n_elecs, Ds=None, allow_errors: bool = False):
        mu, Ds, status, iters, trace = self._run(Hs, betas, n_elecs, Ds, allow_errors, with_density=True)
        return mu, Ds, status, iters, trace

    def _run(self, Hs, betas, n_elecs, Ds, allow_errors, with_density):
        import torch

        count = len(self.sizes)
        if len(Hs) != count or len(betas) != count or len(n_elecs) != count:
            raise ValueError("one H, beta and n_elec per problem")
        hp, hl = [], []
        for H, n in zip(Hs, self.sizes):
            p, nn, ld = _matrix_args(H, "H")
            if nn != n:
                raise ValueError("H size does not match the plan")
            hp.append(p.value)
            hl.append(ld)
        dp, dl = [], []
        if with_density:
            if Ds is None:
                Ds = [torch.empty((n, n), dtype=torch.float64, device=H.device) for H, n in zip(Hs, self.sizes)]
            for D, n in zip(Ds, self.sizes):
                p, nn, ld = _matrix_args(D, "D")
                if nn != n:
                    raise ValueError("D size does not match the plan")
                dp.append(p.value)
                dl.append(ld)
        mu = (ctypes.c_double * count)()
        status = (ctypes.c_int32 * count)()
        iters = (ctypes.c_int32 * count)()
        trace = (ctypes.c_double * count)()
        self.handle.ptr   # follow torch's current stream
        rc = load_library().chebdm_batch_mu_search(self._b, _arr(ctypes.c_void_p, hp), _arr(ctypes.c_int64, hl),
                                                   _arr(ctypes.c_double, [float(v) for v in betas]),
                                                   _arr(ctypes.c_double, [float(v) for v in n_elecs]),
                                                   _arr(ctypes.c_void_p, dp) if with_density else None,
                                                   _arr(ctypes.c_int64, dl) if with_density else None, mu, status,
                                                   iters, trace)
        if rc < 0 and not allow_errors:
            _check(rc)
        out = (np.array(mu[:]), np.array(status[:], dtype=np.int32), np.array(iters[:], dtype=np.int32),
               np.array(trace[:]))
        return (out[0], Ds) + out[1:] if with_density else out

    def close(self):
        if getattr(self, "_b", None) is not None and self._b.value:
            load_library().chebdm_batch_destroy(self._b)
            self._b = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def chebdm_batch_create(h: Handle, sizes, order: int, opts: Optional[Opts] = None, max_quad: int = 0) -> Batch:
    return Batch(h, sizes, order, opts, max_quad)


# ---- the learned chemical-potential network --------------------------------------------------

def _torch():
    import torch

    return torch


def _f32_dev(t, name, numel=None):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or t.dtype != torch.float32 or not t.is_cuda or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous float32 CUDA tensor")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name} must hold {numel} entries")
    return ctypes.c_void_p(t.data_ptr())


def chebdm_mlp_num_params() -> int:
    return int(load_library().chebdm_mlp_num_params())


def chebdm_mlp_forward(h: Handle, W, X):
    """y = net(X) for X (batch x 64); returns a new float32 tensor of batch entries."""
    torch = _torch()
    if X.dim() != 2 or X.shape[1] != 64:
        raise ValueError("X must be batch x 64")
    Y = torch.empty(X.shape[0], dtype=torch.float32, device=X.device)
    _check(load_library().chebdm_mlp_forward(h.ptr, _f32_dev(W, "W", chebdm_mlp_num_params()), _f32_dev(X, "X"),
                                             int(X.shape[0]), _f32_dev(Y, "Y")))
    return Y


def chebdm_mlp_backward(h: Handle, W, X, T, grad=None, want_loss: bool = True):
    """(gradient of the mean squared error, loss or None); ``grad`` is reused when given."""
    torch = _torch()
    if X.dim() != 2 or X.shape[1] != 64 or T.numel() != X.shape[0]:
        raise ValueError("X must be batch x 64 and T hold batch entries")
    if grad is None:
        grad = torch.empty_like(W)
    loss = ctypes.c_float()
    _check(load_library().chebdm_mlp_backward(h.ptr, _f32_dev(W, "W", chebdm_mlp_num_params()), _f32_dev(X, "X"),
                                              _f32_dev(T, "T"), int(X.shape[0]),
                                              _f32_dev(grad, "grad", chebdm_mlp_num_params()),
                                              ctypes.byref(loss) if want_loss else None))
    return grad, (loss.value if want_loss else None)


def chebdm_mlp_adam(h: Handle, W, G, M, V, step: int, lr: float = 1e-3, beta1: float = 0.9, beta2: float = 0.999,
                    eps: float = 1e-8) -> None:
    n = chebdm_mlp_num_params()
    _check(load_library().chebdm_mlp_adam(h.ptr, _f32_dev(W, "W", n), _f32_dev(G, "G", n), _f32_dev(M, "M", n),
                                          _f32_dev(V, "V", n), int(step), float(lr), float(beta1), float(beta2),
                                          float(eps)))

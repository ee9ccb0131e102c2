"""Python binding of the ffbie C ABI (include/ffbie.h).

Argument marshalling only: every step of the computation runs in the HIP
library ``libffbie.so`` built from ``csrc/``.  torch provides device memory and
the stream.  There is no fallback: if the library is missing or no GPU is
present, the calls raise.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libffbie.so")

FFBIE_OK = 0
PAIR_SINGULAR, PAIR_ROOT_FALLBACK, PAIR_REFINED, PAIR_UNRESOLVED, PAIR_FAR = 1, 2, 4, 8, 16
KAPPA_SWAP, KAPPA_PAPER_CONV = 0, 1

EXPORTS = ("ffbie_create", "ffbie_destroy", "ffbie_last_error", "ffbie_set_problem",
           "ffbie_kernel_coeffs", "ffbie_singular_factor", "ffbie_enable_timing", "ffbie_get_timing")
P_SHIFT = 8


class FfbieError(RuntimeError):
    pass


class _Geometry(ctypes.Structure):
    _fields_ = [("lmax", ctypes.c_int), ("mmax", ctypes.c_int), ("a", ctypes.POINTER(ctypes.c_double))]


class _Disc(ctypes.Structure):
    _fields_ = [("n_panels", ctypes.c_int), ("M", ctypes.c_int), ("M0", ctypes.c_int),
                ("eps0", ctypes.c_double), ("kappa_variant", ctypes.c_int)]


_lib = None


def load_library(path=LIB_PATH):
    """Load libffbie.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise FfbieError(f"{path} not found: build it with paper_2608_16208_amd.build.build()")
    lib = ctypes.CDLL(path)
    vp, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int
    lib.ffbie_create.argtypes = [ctypes.POINTER(vp), i32, vp]
    lib.ffbie_destroy.argtypes = [vp]
    lib.ffbie_last_error.argtypes = [vp]
    lib.ffbie_last_error.restype = ctypes.c_char_p
    lib.ffbie_set_problem.argtypes = [vp, ctypes.POINTER(_Geometry), ctypes.POINTER(_Disc), ctypes.c_double]
    lib.ffbie_kernel_coeffs.argtypes = [vp, i64, vp, vp, vp, vp, vp, vp, vp]
    lib.ffbie_singular_factor.argtypes = [vp, i64, vp, i32, vp]
    lib.ffbie_enable_timing.argtypes = [vp, i32]
    dp = ctypes.POINTER(ctypes.c_double)
    lib.ffbie_get_timing.argtypes = [vp, dp, dp, dp]
    for name in EXPORTS:
        f = getattr(lib, name)
        if name != "ffbie_last_error":
            f.restype = ctypes.c_int
    _lib = lib
    return lib


def _ptr(x):
    return None if x is None else ctypes.c_void_p(x.data_ptr())


class Context:
    """One library context on a device, enqueuing on torch's current stream."""

    def __init__(self, device=0, stream=None):
        import torch
        self._torch = torch
        self.lib = load_library()
        if not torch.cuda.is_available():
            raise FfbieError("no GPU visible to torch")
        self.device = torch.device("cuda", device)
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        self.stream = stream
        h = ctypes.c_void_p()
        self._check(self.lib.ffbie_create(ctypes.byref(h), device, ctypes.c_void_p(stream.cuda_stream)),
                    None)
        self.h = h
        self.M = None

    def _check(self, rc, h):
        if rc < 0:
            msg = self.lib.ffbie_last_error(h).decode() if h is not None else "ffbie_create failed"
            raise FfbieError(f"{msg} (status {rc})")
        return rc

    def close(self):
        if getattr(self, "h", None):
            self.lib.ffbie_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_problem(self, amp, n_panels, M, k, M0=None, eps0=0.0, variant=KAPPA_SWAP):
        a = np.ascontiguousarray(np.zeros((0, 1)) if amp is None else amp, dtype=np.float64)
        self._amp = a
        geo = _Geometry(a.shape[0], a.shape[1] - 1, a.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
        disc = _Disc(int(n_panels), int(M), int(M if M0 is None else M0), float(eps0), int(variant))
        self._check(self.lib.ffbie_set_problem(self.h, ctypes.byref(geo), ctypes.byref(disc), float(k)), self.h)
        self.M, self.M0 = int(M), int(M if M0 is None else M0)

    def kernel_coeffs(self, t, az, ts, rhoinv=False, root=False, status=True, kappa=None):
        """kappa [n, 2M] complex128 (n = -M+1..M); optional <rho^-1> [n, M+M0+1],
        root [n, 2] (a - theta_j, b) and per-pair status [n] int32."""
        torch = self._torch
        dev = self.device
        t = t.to(dev, torch.float64).contiguous()
        ts = ts.to(dev, torch.float64).contiguous()
        az = az.to(dev, torch.int32).contiguous()
        n = t.numel()
        if az.numel() != n or ts.numel() != n:
            raise FfbieError("t, az and ts must have the same length")
        out = {}
        out["kappa"] = kappa if kappa is not None else torch.empty((n, 2 * self.M), dtype=torch.complex128, device=dev)
        out["rhoinv"] = torch.empty((n, self.M + self.M0 + 1), dtype=torch.complex128, device=dev) if rhoinv else None
        out["root"] = torch.empty((n, 2), dtype=torch.float64, device=dev) if root else None
        out["status"] = torch.empty((n,), dtype=torch.int32, device=dev) if status else None
        rc = self.lib.ffbie_kernel_coeffs(self.h, n, _ptr(t), _ptr(az), _ptr(ts), _ptr(out["kappa"]),
                                          _ptr(out["rhoinv"]), _ptr(out["root"]), _ptr(out["status"]))
        self._check(rc, self.h)
        return out

    def enable_timing(self, on=True):
        self._check(self.lib.ffbie_enable_timing(self.h, int(bool(on))), self.h)

    def timing(self):
        """(ms_root, ms_main, ms_refine) of the last kernel_coeffs call (HIP events)."""
        v = [ctypes.c_double() for _ in range(3)]
        self._check(self.lib.ffbie_get_timing(self.h, *(ctypes.byref(x) for x in v)), self.h)
        return tuple(x.value for x in v)

    def singular_factor(self, b, m_max):
        torch = self._torch
        b = b.to(self.device, torch.float64).contiguous()
        A = torch.empty((b.numel(), m_max + 1), dtype=torch.float64, device=self.device)
        self._check(self.lib.ffbie_singular_factor(self.h, b.numel(), _ptr(b), int(m_max), _ptr(A)), self.h)
        return A

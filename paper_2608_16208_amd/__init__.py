"""Python binding of the ffbie C ABI (include/ffbie.h).

Argument marshalling only: every step of the computation runs in the HIP
library ``libffbie.so`` built from ``csrc/``.  torch provides device memory and
the stream.  There is no fallback: if the library is missing or no GPU is
present, the calls raise.
"""
import ctypes
import weakref
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libffbie.so")

FFBIE_OK = 0
PAIR_SINGULAR, PAIR_ROOT_FALLBACK, PAIR_REFINED, PAIR_UNRESOLVED, PAIR_FAR = 1, 2, 4, 8, 16
PAIR_NOT_PD = 32
KAPPA_SWAP, KAPPA_PAPER_CONV = 0, 1

EXPORTS = ("ffbie_create", "ffbie_destroy", "ffbie_last_error", "ffbie_set_problem",
           "ffbie_kernel_coeffs", "ffbie_singular_factor", "ffbie_enable_timing", "ffbie_get_timing",
           "ffbie_builtin_near_rule", "ffbie_set_near_rule", "ffbie_query", "ffbie_near_pairs",
           "ffbie_collocation", "ffbie_rhs", "ffbie_assemble", "ffbie_eval_field", "ffbie_solve",
           "ffbie_residual", "ffbie_kernel_coeffs_batched", "ffbie_lu_factor", "ffbie_lu_solve",
           "ffbie_mlp_param_count", "ffbie_mlp_init", "ffbie_mlp_set_params", "ffbie_mlp_get_params",
           "ffbie_mlp_forward", "ffbie_mlp_train_step", "ffbie_mode_features", "ffbie_mode_targets",
           "ffbie_mlp_precondition", "ffbie_blockjacobi_setup", "ffbie_blockjacobi_apply",
           "ffbie_kernel_coeffs_mixed", "ffbie_set_tuning", "ffbie_get_tuning",
           "ffbie_batch_plan_create", "ffbie_batch_plan_execute", "ffbie_batch_plan_get_tuning",
           "ffbie_batch_plan_destroy", "ffbie_batch_plan_classes", "ffbie_gemm_sub",
           "ffbie_assembly_report", "ffbie_mlp_train", "ffbie_mlp_save", "ffbie_mlp_load",
           "ffbie_kernel_coeffs_noalloc", "ffbie_kernel_coeffs_dl", "ffbie_assemble_op",
           "ffbie_eval_field_op", "ffbie_set_tuning_cache", "ffbie_rhoinv_banded")
SOLVE_LU64, SOLVE_LU32_IR64, SOLVE_GMRES, SOLVE_FGMRES_MLP, SOLVE_GMRES_BLOCKJACOBI = 0, 1, 2, 3, 4
SOLVE_GMRES_LU32, SOLVE_FGMRES_BJ_MLP = 5, 6
MLP_IN, MLP_HIDDEN, MLP_OUT = 514, 256, 512
WNOTCONV, WUNRESOLVED = 2, 3
RHS_POINT_SOURCE, RHS_PLANE_WAVE, RHS_PLANE_WAVE_DN, RHS_POINT_SOURCE_DN = 0, 1, 2, 3
OP_S, OP_K, OP_KP = 0, 1, 2
UNKNOWN_SCALED, UNKNOWN_DENSITY = 0, 1
P_SHIFT = 8


class FfbieError(RuntimeError):
    pass


class _Geometry(ctypes.Structure):
    _fields_ = [("lmax", ctypes.c_int), ("mmax", ctypes.c_int), ("a", ctypes.POINTER(ctypes.c_double)),
                ("axes", ctypes.POINTER(ctypes.c_double))]


def _axes_ptr(axes, owner):
    """Pointer to three float64 axes (kept alive on owner), or NULL."""
    if axes is None:
        owner._axes = None
        return None
    owner._axes = np.ascontiguousarray(axes, dtype=np.float64).reshape(3)
    return owner._axes.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


class _Disc(ctypes.Structure):
    _fields_ = [("n_panels", ctypes.c_int), ("M", ctypes.c_int), ("M0", ctypes.c_int),
                ("eps0", ctypes.c_double), ("kappa_variant", ctypes.c_int)]


class _BatchItem(ctypes.Structure):
    _fields_ = [("g", _Geometry), ("d", _Disc), ("k", ctypes.c_double), ("n_pairs", ctypes.c_int64),
                ("d_t", ctypes.c_void_p), ("d_az", ctypes.c_void_p), ("d_ts", ctypes.c_void_p),
                ("d_kappa", ctypes.c_void_p), ("d_pair_status", ctypes.c_void_p)]


class _Tuning(ctypes.Structure):
    _fields_ = [("fft_radix", ctypes.c_int), ("pairs_per_item", ctypes.c_int),
                ("waves_per_block", ctypes.c_int), ("persistent", ctypes.c_int)]


class _SolveInfo(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int), ("converged", ctypes.c_int), ("rel_residual", ctypes.c_double),
                ("fell_back", ctypes.c_int)]


class _TrainCfg(ctypes.Structure):
    _fields_ = [("n_samples", ctypes.c_int64), ("d_x", ctypes.c_void_p), ("d_t", ctypes.c_void_p),
                ("steps", ctypes.c_int), ("batch", ctypes.c_int), ("lr", ctypes.c_float),
                ("seed", ctypes.c_uint64)]


class _TrainInfo(ctypes.Structure):
    _fields_ = [("loss_first", ctypes.c_double), ("loss_last", ctypes.c_double),
                ("loss_full", ctypes.c_double), ("steps", ctypes.c_int)]


class _NearRule(ctypes.Structure):
    _fields_ = [(name, (ctypes.c_double * 16) * 16) for name in ("self_x", "self_w", "right_x", "right_w")]


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
    lib.ffbie_kernel_coeffs_mixed.argtypes = [vp, i64, vp, vp, vp, vp, vp, vp, vp]
    lib.ffbie_kernel_coeffs_noalloc.argtypes = [vp, i64, vp, vp, vp, vp, vp, vp, vp]
    lib.ffbie_kernel_coeffs_dl.argtypes = [vp, i64, vp, vp, vp, i32, vp, vp, vp]
    lib.ffbie_rhoinv_banded.argtypes = [vp, i64, vp, vp, vp, i32, vp, vp, ctypes.POINTER(i32)]
    lib.ffbie_singular_factor.argtypes = [vp, i64, vp, i32, vp]
    lib.ffbie_enable_timing.argtypes = [vp, i32]
    dp = ctypes.POINTER(ctypes.c_double)
    lib.ffbie_get_timing.argtypes = [vp, dp, dp, dp]
    lib.ffbie_builtin_near_rule.argtypes = [ctypes.POINTER(_NearRule)]
    lib.ffbie_set_near_rule.argtypes = [vp, ctypes.POINTER(_NearRule)]
    pi64 = ctypes.POINTER(ctypes.c_int64)
    lib.ffbie_query.argtypes = [vp, pi64, pi64, pi64]
    lib.ffbie_assembly_report.argtypes = [vp, pi64, pi64, pi64]
    lib.ffbie_mlp_train.argtypes = [vp, ctypes.POINTER(_TrainCfg), ctypes.POINTER(_TrainInfo)]
    lib.ffbie_mlp_save.argtypes = [vp, ctypes.c_char_p]
    lib.ffbie_mlp_load.argtypes = [vp, ctypes.c_char_p]
    lib.ffbie_near_pairs.argtypes = [vp, vp, vp, vp]
    lib.ffbie_collocation.argtypes = [vp, vp, vp, vp]
    lib.ffbie_rhs.argtypes = [vp, i32, dp, vp]
    lib.ffbie_assemble.argtypes = [vp, vp, i64]
    lib.ffbie_eval_field.argtypes = [vp, i64, vp, vp, vp]
    lib.ffbie_set_tuning_cache.argtypes = [vp, ctypes.c_char_p]
    lib.ffbie_assemble_op.argtypes = [vp, i32, ctypes.c_double, i32, vp, i64]
    lib.ffbie_eval_field_op.argtypes = [vp, i32, i32, i64, vp, vp, vp]
    lib.ffbie_solve.argtypes = [vp, i32, vp, i64, vp, vp, ctypes.c_double, i32, ctypes.POINTER(_SolveInfo)]
    lib.ffbie_residual.argtypes = [vp, vp, i64, vp, vp, vp]
    lib.ffbie_kernel_coeffs_batched.argtypes = [vp, i32, ctypes.POINTER(_BatchItem)]
    lib.ffbie_set_tuning.argtypes = [vp, ctypes.POINTER(_Tuning)]
    lib.ffbie_get_tuning.argtypes = [vp, ctypes.POINTER(_Tuning)]
    lib.ffbie_batch_plan_create.argtypes = [vp, i32, ctypes.POINTER(_BatchItem), i32,
                                            ctypes.POINTER(_Tuning), ctypes.POINTER(vp)]
    lib.ffbie_batch_plan_execute.argtypes = [vp, vp]
    lib.ffbie_batch_plan_get_tuning.argtypes = [vp, i32, ctypes.POINTER(_Tuning), dp,
                                                ctypes.POINTER(ctypes.c_int)]
    lib.ffbie_batch_plan_classes.argtypes = [vp]
    lib.ffbie_batch_plan_destroy.argtypes = [vp]
    lib.ffbie_lu_factor.argtypes = [vp, vp, i64]
    lib.ffbie_lu_solve.argtypes = [vp, vp, i64, vp]
    lib.ffbie_mlp_param_count.argtypes = []
    lib.ffbie_mlp_param_count.restype = i64
    lib.ffbie_mlp_init.argtypes = [vp, ctypes.c_uint64]
    fp = ctypes.POINTER(ctypes.c_float)
    lib.ffbie_mlp_set_params.argtypes = [vp, fp]
    lib.ffbie_mlp_get_params.argtypes = [vp, fp]
    lib.ffbie_mlp_forward.argtypes = [vp, i64, vp, vp]
    lib.ffbie_mlp_train_step.argtypes = [vp, i64, vp, vp, ctypes.c_float, i32, vp, dp]
    lib.ffbie_mode_features.argtypes = [vp, vp, vp, vp]
    lib.ffbie_mode_targets.argtypes = [vp, vp, vp, vp]
    lib.ffbie_mlp_precondition.argtypes = [vp, vp, vp]
    lib.ffbie_blockjacobi_setup.argtypes = [vp, vp, i64]
    lib.ffbie_blockjacobi_apply.argtypes = [vp, vp, vp]
    lib.ffbie_gemm_sub.argtypes = [vp, i32, i64, i64, i64, vp, vp, vp, i64]
    for name in EXPORTS:
        f = getattr(lib, name)
        if name not in ("ffbie_last_error", "ffbie_mlp_param_count", "ffbie_batch_plan_classes"):
            f.restype = ctypes.c_int
    _lib = lib
    return lib


def _ptr(x):
    return None if x is None else ctypes.c_void_p(x.data_ptr())


def builtin_near_rule():
    """The library's built-in 16-node near-panel rules (host call, no GPU):
    dict of float64 arrays self_x, self_w, right_x, right_w, each [16][16]."""
    lib = load_library()
    r = _NearRule()
    rc = lib.ffbie_builtin_near_rule(ctypes.byref(r))
    if rc != FFBIE_OK:
        raise FfbieError(f"ffbie_builtin_near_rule failed ({rc})")
    return {name: np.ctypeslib.as_array(getattr(r, name)).copy() for name, _ in _NearRule._fields_}


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
        for plan in list(getattr(self, "_plans", ())):
            plan.close()
        if getattr(self, "h", None):
            self.lib.ffbie_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_problem(self, amp, n_panels, M, k, M0=None, eps0=0.0, variant=KAPPA_SWAP, axes=None):
        """Surface (amplitude table, optional axes of the stretch D), panels,
        M, wavenumber k, M0, truncation threshold eps0, kappa variant."""
        a = np.ascontiguousarray(np.zeros((0, 1)) if amp is None else amp, dtype=np.float64)
        self._amp = a
        geo = _Geometry(a.shape[0], a.shape[1] - 1, a.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                        _axes_ptr(axes, self))
        disc = _Disc(int(n_panels), int(M), int(M if M0 is None else M0), float(eps0), int(variant))
        self._check(self.lib.ffbie_set_problem(self.h, ctypes.byref(geo), ctypes.byref(disc), float(k)), self.h)
        self.M, self.M0 = int(M), int(M if M0 is None else M0)

    def kernel_coeffs(self, t, az, ts, rhoinv=False, root=False, status=True, kappa=None,
                      mixed=False, rhoinv_out=None, noalloc=False):
        """kappa [n, 2M] complex128 (n = -M+1..M); optional <rho^-1> [n, M+M0+1],
        root [n, 2] (a - theta_j, b) and per-pair status [n] int32.  With
        mixed=True the FP32 spectral-stage path runs and kappa / <rho^-1> are
        complex64.  noalloc=True calls ffbie_kernel_coeffs_noalloc (the library
        allocates nothing; outputs passed in are used as they are)."""
        torch = self._torch
        dev = self.device
        cdt = torch.complex64 if mixed else torch.complex128
        t = t.to(dev, torch.float64).contiguous()
        ts = ts.to(dev, torch.float64).contiguous()
        az = az.to(dev, torch.int32).contiguous()
        n = t.numel()
        if az.numel() != n or ts.numel() != n:
            raise FfbieError("t, az and ts must have the same length")
        out = {}
        if kappa is not None and (kappa.dtype != cdt or kappa.shape != (n, 2 * self.M)
                                  or not kappa.is_contiguous()):
            raise FfbieError("kappa must be a contiguous [n, 2M] %s tensor" % cdt)
        out["kappa"] = kappa if kappa is not None else torch.empty((n, 2 * self.M), dtype=cdt, device=dev)
        if rhoinv_out is not None:
            if rhoinv_out.dtype != cdt or tuple(rhoinv_out.shape) != (n, self.M + self.M0 + 1) \
                    or not rhoinv_out.is_contiguous():
                raise FfbieError("rhoinv_out must be a contiguous [n, M+M0+1] %s tensor" % cdt)
            out["rhoinv"] = rhoinv_out
        else:
            out["rhoinv"] = torch.empty((n, self.M + self.M0 + 1), dtype=cdt, device=dev) if rhoinv else None
        out["root"] = torch.empty((n, 2), dtype=torch.float64, device=dev) if root else None
        out["status"] = torch.empty((n,), dtype=torch.int32, device=dev) if status else None
        if noalloc and mixed:
            raise FfbieError("the no-allocation entry point has no mixed-precision form")
        fn = (self.lib.ffbie_kernel_coeffs_mixed if mixed else
              self.lib.ffbie_kernel_coeffs_noalloc if noalloc else self.lib.ffbie_kernel_coeffs)
        rc = fn(self.h, n, _ptr(t), _ptr(az), _ptr(ts), _ptr(out["kappa"]), _ptr(out["rhoinv"]),
                _ptr(out["root"]), _ptr(out["status"]))
        self._check(rc, self.h)
        return out

    def kernel_coeffs_dl(self, t, az, ts, adjoint=False, root=False, status=True, kappa=None):
        """Double-layer coefficients <tau_0 (ik rho - 1) e^{ik rho} / rho^3>_n,
        n = -M+1..M, as kappa [n, 2M] complex128: K (adjoint=False, normal at
        the source) or K' (adjoint=True, normal at the target); optional root
        [n, 2] and per-pair status [n] int32."""
        torch = self._torch
        dev = self.device
        t = t.to(dev, torch.float64).contiguous()
        ts = ts.to(dev, torch.float64).contiguous()
        az = az.to(dev, torch.int32).contiguous()
        n = t.numel()
        if az.numel() != n or ts.numel() != n:
            raise FfbieError("t, az and ts must have the same length")
        if kappa is not None and (kappa.dtype != torch.complex128 or tuple(kappa.shape) != (n, 2 * self.M)
                                  or not kappa.is_contiguous()):
            raise FfbieError("kappa must be a contiguous [n, 2M] complex128 tensor")
        out = {"kappa": kappa if kappa is not None else
               torch.empty((n, 2 * self.M), dtype=torch.complex128, device=dev)}
        out["root"] = torch.empty((n, 2), dtype=torch.float64, device=dev) if root else None
        out["status"] = torch.empty((n,), dtype=torch.int32, device=dev) if status else None
        rc = self.lib.ffbie_kernel_coeffs_dl(self.h, n, _ptr(t), _ptr(az), _ptr(ts), int(adjoint),
                                             _ptr(out["kappa"]), _ptr(out["root"]), _ptr(out["status"]))
        self._check(rc, self.h)
        return out

    def rhoinv_banded(self, t, az, ts, m0=0, status=True, rhoinv=None):
        """<rho^-1>_l, l = 0..M+M0, by the banded route of Sec. 3.2.1, as
        rhoinv [n, M+M0+1] complex128; m0 = 0 applies the rule of eq. (3.13).
        Returns dict(rhoinv, status, m0)."""
        torch = self._torch
        dev = self.device
        t = t.to(dev, torch.float64).contiguous()
        ts = ts.to(dev, torch.float64).contiguous()
        az = az.to(dev, torch.int32).contiguous()
        n = t.numel()
        if az.numel() != n or ts.numel() != n:
            raise FfbieError("t, az and ts must have the same length")
        shape = (n, self.M + self.M0 + 1)
        if rhoinv is not None and (rhoinv.dtype != torch.complex128 or tuple(rhoinv.shape) != shape
                                   or not rhoinv.is_contiguous()):
            raise FfbieError("rhoinv must be a contiguous [n, M+M0+1] complex128 tensor")
        out = {"rhoinv": rhoinv if rhoinv is not None else
               torch.empty(shape, dtype=torch.complex128, device=dev)}
        out["status"] = torch.empty((n,), dtype=torch.int32, device=dev) if status else None
        used = ctypes.c_int(-1)
        rc = self.lib.ffbie_rhoinv_banded(self.h, n, _ptr(t), _ptr(az), _ptr(ts), int(m0),
                                          _ptr(out["rhoinv"]), _ptr(out["status"]), ctypes.byref(used))
        self._check(rc, self.h)
        out["m0"] = used.value
        return out

    def _batch_items(self, problems, mixed=False):
        torch = self._torch
        dev = self.device
        cdt = torch.complex64 if mixed else torch.complex128
        keep, outs = [], []
        arr = (_BatchItem * max(1, len(problems)))()
        for i, pr in enumerate(problems):
            a = np.ascontiguousarray(np.zeros((0, 1)) if pr.get("amp") is None else pr["amp"], dtype=np.float64)
            M = int(pr["M"])
            t = pr["t"].to(dev, torch.float64).contiguous()
            ts = pr["ts"].to(dev, torch.float64).contiguous()
            az = pr["az"].to(dev, torch.int32).contiguous()
            n = t.numel()
            if az.numel() != n or ts.numel() != n:
                raise FfbieError("t, az and ts must have the same length")
            kap = pr.get("kappa")
            if kap is None:
                kap = torch.empty((n, 2 * M), dtype=cdt, device=dev)
            elif kap.dtype != cdt or tuple(kap.shape) != (n, 2 * M) or not kap.is_contiguous():
                raise FfbieError("kappa of item %d must be a contiguous [n, 2M] %s tensor" % (i, cdt))
            st = pr.get("status")
            if st is None:
                st = torch.empty((n,), dtype=torch.int32, device=dev)
            keep += [a, t, ts, az, kap, st]
            it = arr[i]
            ax = None if pr.get("axes") is None else np.ascontiguousarray(pr["axes"], dtype=np.float64)
            if ax is not None:
                keep.append(ax)
            it.g = _Geometry(a.shape[0], a.shape[1] - 1, a.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                             None if ax is None else ax.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
            it.d = _Disc(1, M, int(pr.get("M0", M)), float(pr.get("eps0", 0.0)), KAPPA_SWAP)
            it.k = float(pr["k"])
            it.n_pairs = n
            it.d_t, it.d_az, it.d_ts = t.data_ptr(), az.data_ptr(), ts.data_ptr()
            it.d_kappa, it.d_pair_status = kap.data_ptr(), st.data_ptr()
            outs.append({"kappa": kap, "status": st})
        return arr, keep, outs

    def kernel_coeffs_batched(self, problems):
        """Coefficient path for several problems in one launch per phase.
        problems: list of dicts with amp, M, k, t, az, ts (and optional M0, eps0,
        kappa [n, 2M] and status [n] output tensors).  Returns a list of dicts
        with kappa and status."""
        arr, keep, outs = self._batch_items(problems)
        rc = self.lib.ffbie_kernel_coeffs_batched(self.h, len(problems), arr)
        self._check(rc, self.h)
        self._batch_keep = keep        # inputs stay alive until the stream has used them
        return outs

    def batch_plan(self, problems, graph=False, autotune=False, mixed=False, tuning=None):
        """A reusable batch plan (see BatchPlan) over `problems` (as for
        kernel_coeffs_batched; with mixed=True the kappa outputs are complex64)."""
        return BatchPlan(self, problems, graph, autotune, mixed, tuning)

    def set_tuning(self, fft_radix=0, pairs_per_item=16, waves_per_block=4, persistent=0):
        t = _Tuning(fft_radix, pairs_per_item, waves_per_block, persistent)
        self._check(self.lib.ffbie_set_tuning(self.h, ctypes.byref(t)), self.h)

    def get_tuning(self):
        t = _Tuning()
        self._check(self.lib.ffbie_get_tuning(self.h, ctypes.byref(t)), self.h)
        return {"fft_radix": t.fft_radix, "pairs_per_item": t.pairs_per_item,
                "waves_per_block": t.waves_per_block, "persistent": t.persistent}

    def set_tuning_cache(self, path):
        """File of the batch autotuner's choices (None clears it); autotuned
        plans read their M classes from it and add what they tune."""
        self._check(self.lib.ffbie_set_tuning_cache(self.h, None if path is None else str(path).encode()),
                    self.h)

    def enable_timing(self, on=True):
        self._check(self.lib.ffbie_enable_timing(self.h, int(bool(on))), self.h)

    def timing(self):
        """(ms_root, ms_main, ms_refine) of the last kernel_coeffs call (HIP events)."""
        v = [ctypes.c_double() for _ in range(3)]
        self._check(self.lib.ffbie_get_timing(self.h, *(ctypes.byref(x) for x in v)), self.h)
        return tuple(x.value for x in v)

    # ---- discrete single-layer system -------------------------------------
    def set_near_rule(self, rule=None):
        """Near-panel rules: dict as returned by builtin_near_rule(), or None
        for the built-in rules."""
        if rule is None:
            self._check(self.lib.ffbie_set_near_rule(self.h, None), self.h)
            return
        r = _NearRule()
        for name, _ in _NearRule._fields_:
            np.ctypeslib.as_array(getattr(r, name))[:] = np.asarray(rule[name], dtype=np.float64)
        self._check(self.lib.ffbie_set_near_rule(self.h, ctypes.byref(r)), self.h)

    def query(self):
        """(N unknowns, number of near pairs)."""
        n, p = ctypes.c_int64(), ctypes.c_int64()
        self._check(self.lib.ffbie_query(self.h, ctypes.byref(n), ctypes.byref(p), None), self.h)
        return n.value, p.value

    def workspace_bytes(self):
        """Upper bound of the device workspace of assembly + the largest solve."""
        w = ctypes.c_int64()
        self._check(self.lib.ffbie_query(self.h, None, None, ctypes.byref(w)), self.h)
        return w.value

    def assembly_report(self):
        """Near pairs of the last assembly: {pairs, unresolved, root_fallback}."""
        v = [ctypes.c_int64() for _ in range(3)]
        self._check(self.lib.ffbie_assembly_report(self.h, *(ctypes.byref(x) for x in v)), self.h)
        return {"pairs": v[0].value, "unresolved": v[1].value, "root_fallback": v[2].value}

    def near_pairs(self):
        torch = self._torch
        _, n = self.query()
        t = torch.empty(n, dtype=torch.float64, device=self.device)
        az = torch.empty(n, dtype=torch.int32, device=self.device)
        ts = torch.empty(n, dtype=torch.float64, device=self.device)
        self._check(self.lib.ffbie_near_pairs(self.h, _ptr(t), _ptr(az), _ptr(ts)), self.h)
        return t, az, ts

    def collocation(self):
        """(xyz [N, 3], J [N], wq [N]) on the device."""
        torch = self._torch
        N, _ = self.query()
        xyz = torch.empty((N, 3), dtype=torch.float64, device=self.device)
        jac = torch.empty(N, dtype=torch.float64, device=self.device)
        wq = torch.empty(N, dtype=torch.float64, device=self.device)
        self._check(self.lib.ffbie_collocation(self.h, _ptr(xyz), _ptr(jac), _ptr(wq)), self.h)
        return xyz, jac, wq

    def rhs(self, kind, params):
        torch = self._torch
        N, _ = self.query()
        g = torch.empty(N, dtype=torch.complex128, device=self.device)
        p = (ctypes.c_double * 3)(*[float(v) for v in params])
        self._check(self.lib.ffbie_rhs(self.h, int(kind), p, _ptr(g)), self.h)
        return g

    def assemble(self, S=None, op=OP_S, shift=0.0, unknowns=UNKNOWN_SCALED):
        """Row-major N x N complex128 matrix of op + shift I (allocated if S is
        None): op = OP_S the single layer, OP_K the double layer, OP_KP its
        adjoint; shift = +1 with OP_K is the exterior Dirichlet equation
        (K + I) psi = g, shift = -1 with OP_KP the exterior Neumann one.
        unknowns: UNKNOWN_SCALED (density x Jacobian) or UNKNOWN_DENSITY."""
        torch = self._torch
        N, _ = self.query()
        if S is None:
            S = torch.empty((N, N), dtype=torch.complex128, device=self.device)
        if S.dim() != 2 or S.shape[0] != N or S.stride(1) != 1 or S.stride(0) < N or S.dtype != torch.complex128:
            raise FfbieError("S must be a row-major complex128 [N, >=N] device tensor")
        if op == OP_S and shift == 0.0 and unknowns == UNKNOWN_SCALED:
            rc = self.lib.ffbie_assemble(self.h, _ptr(S), S.stride(0))
        else:
            rc = self.lib.ffbie_assemble_op(self.h, int(op), float(shift), int(unknowns), _ptr(S),
                                            S.stride(0))
        self._check(rc, self.h)
        self.last_assembly = dict(self.assembly_report(), status=rc)
        return S

    def eval_field(self, pts, phi, op=OP_S, unknowns=UNKNOWN_SCALED):
        """Field of the single-layer (op = OP_S) or double-layer (OP_K)
        representation with density phi (given as the system's unknowns) at
        points pts [n, 3]."""
        torch = self._torch
        pts = pts.to(self.device, torch.float64).contiguous()
        phi = phi.to(self.device, torch.complex128).contiguous()
        u = torch.empty(pts.shape[0], dtype=torch.complex128, device=self.device)
        if op == OP_S and unknowns == UNKNOWN_SCALED:
            rc = self.lib.ffbie_eval_field(self.h, pts.shape[0], _ptr(pts), _ptr(phi), _ptr(u))
        else:
            rc = self.lib.ffbie_eval_field_op(self.h, int(op), int(unknowns), pts.shape[0], _ptr(pts),
                                              _ptr(phi), _ptr(u))
        self._check(rc, self.h)
        return u

    def solve(self, S, g, method=SOLVE_LU64, tol=1e-12, max_iter=50, phi=None):
        """phi with S phi = g.  LU64 overwrites S with its factors.  Returns
        (phi, info dict)."""
        torch = self._torch
        g = g.to(self.device, torch.complex128).contiguous()
        if phi is None:
            phi = torch.empty_like(g)
        info = _SolveInfo()
        rc = self.lib.ffbie_solve(self.h, int(method), _ptr(S), S.stride(0), _ptr(g), _ptr(phi),
                                  float(tol), int(max_iter), ctypes.byref(info))
        self._check(rc, self.h)
        return phi, dict(iterations=info.iterations, converged=bool(info.converged),
                         rel_residual=info.rel_residual, fell_back=bool(info.fell_back), status=rc)

    def lu_factor(self, S):
        """Overwrite S with its LU64 factors (kept for lu_solve)."""
        self._check(self.lib.ffbie_lu_factor(self.h, _ptr(S), S.stride(0)), self.h)

    def lu_solve(self, S, b):
        torch = self._torch
        x = b.to(self.device, torch.complex128).clone()
        self._check(self.lib.ffbie_lu_solve(self.h, _ptr(S), S.stride(0), _ptr(x)), self.h)
        return x

    # ---- learned preconditioner --------------------------------------------
    def mlp_param_count(self):
        return int(self.lib.ffbie_mlp_param_count())

    def mlp_init(self, seed):
        self._check(self.lib.ffbie_mlp_init(self.h, ctypes.c_uint64(int(seed))), self.h)

    def mlp_set_params(self, params):
        p = np.ascontiguousarray(params, dtype=np.float32)
        if p.size != self.mlp_param_count():
            raise FfbieError("wrong parameter count")
        self._check(self.lib.ffbie_mlp_set_params(self.h, p.ctypes.data_as(ctypes.POINTER(ctypes.c_float))),
                    self.h)

    def mlp_get_params(self):
        p = np.empty(self.mlp_param_count(), dtype=np.float32)
        self._check(self.lib.ffbie_mlp_get_params(self.h, p.ctypes.data_as(ctypes.POINTER(ctypes.c_float))),
                    self.h)
        return p

    def mlp_forward(self, x):
        torch = self._torch
        x = x.to(self.device, torch.float32).contiguous()
        y = torch.empty((x.shape[0], MLP_OUT), dtype=torch.float32, device=self.device)
        self._check(self.lib.ffbie_mlp_forward(self.h, x.shape[0], _ptr(x), _ptr(y)), self.h)
        return y

    def mlp_train_step(self, x, t, lr=1e-3, update=True, grads=False):
        """(loss before the step, gradient tensor or None)."""
        torch = self._torch
        g = torch.empty(self.mlp_param_count(), dtype=torch.float32, device=self.device) if grads else None
        loss = ctypes.c_double()
        self._check(self.lib.ffbie_mlp_train_step(self.h, x.shape[0], _ptr(x), _ptr(t), float(lr),
                                                  int(bool(update)), _ptr(g), ctypes.byref(loss)), self.h)
        return loss.value, g

    def mlp_train(self, x, t, steps, batch=2048, lr=1e-3, seed=0):
        """Train on (x [n, 514], t [n, 512]) float32 device tensors with the
        library's loop (ffbie_mlp_train); returns the loss record."""
        torch = self._torch
        x = x.to(self.device, torch.float32).contiguous()
        t = t.to(self.device, torch.float32).contiguous()
        cfg = _TrainCfg(x.shape[0], x.data_ptr(), t.data_ptr(), int(steps), int(batch), float(lr), int(seed))
        info = _TrainInfo()
        self._check(self.lib.ffbie_mlp_train(self.h, ctypes.byref(cfg), ctypes.byref(info)), self.h)
        return {"loss_first": info.loss_first, "loss_last": info.loss_last, "loss_full": info.loss_full,
                "steps": info.steps}

    def mlp_save(self, path):
        self._check(self.lib.ffbie_mlp_save(self.h, os.fsencode(path)), self.h)

    def mlp_load(self, path):
        self._check(self.lib.ffbie_mlp_load(self.h, os.fsencode(path)), self.h)

    def mode_features(self, r):
        torch = self._torch
        nm = 2 * self.M
        x = torch.empty((nm, MLP_IN), dtype=torch.float32, device=self.device)
        sc = torch.empty(nm, dtype=torch.float64, device=self.device)
        self._check(self.lib.ffbie_mode_features(self.h, _ptr(r), _ptr(x), _ptr(sc)), self.h)
        return x, sc

    def mode_targets(self, e, scale):
        torch = self._torch
        t = torch.empty((2 * self.M, MLP_OUT), dtype=torch.float32, device=self.device)
        self._check(self.lib.ffbie_mode_targets(self.h, _ptr(e), _ptr(scale), _ptr(t)), self.h)
        return t

    def blockjacobi_setup(self, S):
        self._check(self.lib.ffbie_blockjacobi_setup(self.h, _ptr(S), S.stride(0)), self.h)

    def blockjacobi_apply(self, v):
        z = self._torch.empty_like(v)
        self._check(self.lib.ffbie_blockjacobi_apply(self.h, _ptr(v), _ptr(z)), self.h)
        return z

    def mlp_precondition(self, v):
        z = self._torch.empty_like(v)
        self._check(self.lib.ffbie_mlp_precondition(self.h, _ptr(v), _ptr(z)), self.h)
        return z

    def residual(self, S, phi, g):
        torch = self._torch
        r = torch.empty_like(g)
        self._check(self.lib.ffbie_residual(self.h, _ptr(S), S.stride(0), _ptr(phi), _ptr(g), _ptr(r)),
                    self.h)
        return r

    def gemm_sub(self, C, A, B, m, n, k, ld):
        """C -= A B on complex column-major blocks with leading dimension ld:
        A, B and C are device tensors (complex128 or complex64, all the same)
        whose storage starts at the blocks' first elements."""
        torch = self._torch
        dt = C.dtype
        if dt not in (torch.complex128, torch.complex64) or A.dtype != dt or B.dtype != dt:
            raise FfbieError("gemm_sub needs complex128 or complex64 tensors of one dtype")
        rc = self.lib.ffbie_gemm_sub(self.h, int(dt == torch.complex64), int(m), int(n), int(k),
                                     _ptr(A), _ptr(B), _ptr(C), int(ld))
        self._check(rc, self.h)

    def singular_factor(self, b, m_max):
        torch = self._torch
        b = b.to(self.device, torch.float64).contiguous()
        A = torch.empty((b.numel(), m_max + 1), dtype=torch.float64, device=self.device)
        self._check(self.lib.ffbie_singular_factor(self.h, b.numel(), _ptr(b), int(m_max), _ptr(A)), self.h)
        return A


class BatchPlan:
    """A batch of coefficient problems prepared once (descriptors, workspace,
    optionally an autotuned launch shape and a captured HIP graph) and executed
    any number of times; outputs are in .outs (list of {kappa, status})."""

    PLAN_GRAPH, PLAN_AUTOTUNE, PLAN_MIXED = 1, 2, 4

    def __init__(self, ctx, problems, graph=False, autotune=False, mixed=False, tuning=None):
        self.ctx = ctx
        self.arr, self._keep, self.outs = ctx._batch_items(problems, mixed)
        flags = (self.PLAN_GRAPH if graph else 0) | (self.PLAN_AUTOTUNE if autotune else 0) | \
                (self.PLAN_MIXED if mixed else 0)
        t = None
        if tuning is not None:
            # one dict for every M class, or {M: dict} (classes not named keep
            # the context's tuning)
            base = ctx.get_tuning()
            t = (_Tuning * 4)()
            for q, M in enumerate((16, 32, 64, 128)):
                d = tuning.get(M, base) if all(isinstance(k, int) for k in tuning) else tuning
                t[q] = _Tuning(d["fft_radix"], d["pairs_per_item"], d["waves_per_block"],
                               d.get("persistent", 0))
        h = ctypes.c_void_p()
        rc = ctx.lib.ffbie_batch_plan_create(ctx.h, len(problems), self.arr, flags, t, ctypes.byref(h))
        ctx._check(rc, ctx.h)
        self.h = h
        if not hasattr(ctx, "_plans"):
            ctx._plans = weakref.WeakSet()
        ctx._plans.add(self)

    def execute(self):
        self.ctx._check(self.ctx.lib.ffbie_batch_plan_execute(self.ctx.h, self.h), self.ctx.h)
        return self.outs

    def tuning(self):
        """Per M class: {M, fft_radix, pairs_per_item, waves_per_block, persistent,
        tuned_ms}."""
        out = []
        for k in range(self.ctx.lib.ffbie_batch_plan_classes(self.h)):
            t, ms, M = _Tuning(), ctypes.c_double(), ctypes.c_int()
            rc = self.ctx.lib.ffbie_batch_plan_get_tuning(self.h, k, ctypes.byref(t), ctypes.byref(ms),
                                                          ctypes.byref(M))
            self.ctx._check(rc, self.ctx.h)
            out.append({"M": M.value, "fft_radix": t.fft_radix, "pairs_per_item": t.pairs_per_item,
                        "waves_per_block": t.waves_per_block, "persistent": t.persistent,
                        "tuned_ms": ms.value})
        return out

    def close(self):
        if getattr(self, "h", None) and getattr(self.ctx, "h", None):
            self.ctx.lib.ffbie_batch_plan_destroy(self.h)
        self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

"""Python binding of the MI355X spheroidal boundary-integral library (libsbie.so).

Argument marshalling only: every step of the operator apply runs in the HIP
kernels behind the C ABI declared in include/sbie.h.  PyTorch provides device
memory and streams.  There is no CPU fallback: importing the binding without a
built library raises.
"""
from __future__ import annotations

import atexit
import ctypes
import os
import weakref

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsbie.so")

SBIE_OP_S, SBIE_OP_D, SBIE_OP_STOKES_S, SBIE_OP_SP, SBIE_OP_DP, SBIE_OP_STOKES_SP, SBIE_OP_STOKES_D = range(7)
SBIE_FP64, SBIE_MIXED = 0, 1
SBIE_DEVICE_PTRS = 0x1
SBIE_TIMING = 0x2
SBIE_PARTS_SELF, SBIE_PARTS_NEAR, SBIE_PARTS_FAR, SBIE_PARTS_ALL = 0x10, 0x20, 0x40, 0x70
SBIE_FAR_TREE = 0x100
SBIE_INPUT_COEFFS = 0x200

STATUS = {0: "SBIE_OK", -1: "SBIE_E_INVALID", -2: "SBIE_E_DEGENERATE", -3: "SBIE_E_OVERLAP", -4: "SBIE_E_NOMEM",
          -5: "SBIE_E_BUDGET", -6: "SBIE_E_DEVICE", -7: "SBIE_E_TIMEOUT", -8: "SBIE_E_NUMERIC", -9: "SBIE_E_STATE"}

# symbols declared in include/sbie.h
EXPORTS = [
    "sbie_ctx_create", "sbie_ctx_destroy", "sbie_geom_create", "sbie_geom_destroy", "sbie_geom_num_nodes",
    "sbie_geom_num_near_pairs", "sbie_geom_footprint_bytes", "sbie_geom_nodes", "sbie_geom_near_pairs",
    "sbie_apply", "sbie_geom_sync", "sbie_transform", "sbie_geom_spectra", "sbie_geom_timing",
    "sbie_session_bytes", "sbie_server_create", "sbie_server_destroy", "sbie_session_open", "sbie_session_apply",
    "sbie_session_close", "sbie_wait", "sbie_server_get_info", "sbie_status_str", "sbie_last_error",
    "sbie_completion_eta", "sbie_apply_completed", "sbie_solve_completed", "sbie_solve_neumann",
    "sbie_eval_targets", "sbie_geom_far_tree", "sbie_geom_far_tree_info", "sbie_far_tree_plan",
    "sbie_eval_targets_noalloc", "sbie_geom_set_depth_cap",
]
SBIE_TARGETS_SCRATCH_BYTES = 64 << 20
SBIE_COMPLETE_POINT, SBIE_COMPLETE_SINGLE = 0, 1
SBIE_SERVER_GRAPHS = 0x100
SBIE_SERVER_BATCH = 0x200
SBIE_SERVER_TREE = 0x400
SBIE_MAX_PASS = 8


class SbieError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status


class TreeInfo(ctypes.Structure):
    _fields_ = [("clusters", ctypes.c_int32), ("proxy_clusters", ctypes.c_int32), ("proxy_pairs", ctypes.c_int64),
                ("direct_pairs", ctypes.c_int64), ("proxy_evals", ctypes.c_int64), ("direct_evals", ctypes.c_int64),
                ("charge_evals", ctypes.c_int64), ("device_bytes", ctypes.c_uint64)]


class Timing(ctypes.Structure):
    _fields_ = [("prep_ms", ctypes.c_double), ("transform_ms", ctypes.c_double), ("near_ms", ctypes.c_double),
                ("far_kernel_ms", ctypes.c_double), ("assemble_ms", ctypes.c_double), ("total_ms", ctypes.c_double),
                ("far_pairs", ctypes.c_int64), ("near_evals", ctypes.c_int64), ("count", ctypes.c_int64),
                ("far_launches", ctypes.c_int64)]


class ApplyStats(ctypes.Structure):
    _fields_ = [("open_us", ctypes.c_double), ("admit_us", ctypes.c_double), ("ready_us", ctypes.c_double),
                ("submit_us", ctypes.c_double), ("start_us", ctypes.c_double), ("end_us", ctypes.c_double),
                ("session", ctypes.c_int64), ("lane", ctypes.c_int32), ("status", ctypes.c_int32)]


class ServerInfo(ctypes.Structure):
    _fields_ = [("budget_bytes", ctypes.c_uint64), ("in_use_bytes", ctypes.c_uint64), ("peak_bytes", ctypes.c_uint64),
                ("pending", ctypes.c_int64), ("active", ctypes.c_int64), ("admitted", ctypes.c_int64),
                ("passed", ctypes.c_int64), ("waited", ctypes.c_int64), ("applies", ctypes.c_int64),
                ("lanes", ctypes.c_int32), ("graphs", ctypes.c_int32), ("batched", ctypes.c_int64),
                ("tree_sessions", ctypes.c_int64)]


_lib = None
_live = []


def _close_all():
    for ref in reversed(_live):
        obj = ref()
        if obj is not None:
            try:
                obj.close()
            except Exception:
                pass
    _live.clear()


atexit.register(_close_all)


def lib() -> ctypes.CDLL:
    """Load libsbie.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_2506_20809_amd.build.build()")
        L = ctypes.CDLL(LIB_PATH)
        vp, dp = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double)
        L.sbie_ctx_create.argtypes = [ctypes.c_int, ctypes.POINTER(vp)]
        L.sbie_ctx_destroy.argtypes = [vp]
        L.sbie_ctx_destroy.restype = None
        L.sbie_geom_create.argtypes = [vp, dp, dp, dp, dp, ctypes.c_int32, ctypes.c_int32, ctypes.c_double,
                                       ctypes.POINTER(vp)]
        L.sbie_geom_destroy.argtypes = [vp]
        L.sbie_geom_destroy.restype = None
        L.sbie_geom_num_nodes.argtypes = [vp]
        L.sbie_geom_num_nodes.restype = ctypes.c_int64
        L.sbie_geom_num_near_pairs.argtypes = [vp]
        L.sbie_geom_num_near_pairs.restype = ctypes.c_int64
        L.sbie_geom_footprint_bytes.argtypes = [vp]
        L.sbie_geom_footprint_bytes.restype = ctypes.c_uint64
        L.sbie_geom_nodes.argtypes = [vp, dp, dp, dp]
        ip = ctypes.POINTER(ctypes.c_int32)
        L.sbie_geom_near_pairs.argtypes = [vp, ip, ip, ctypes.c_int64, ctypes.POINTER(ctypes.c_int64)]
        L.sbie_apply.argtypes = [vp, ctypes.c_int, ctypes.c_int, ctypes.c_int32, vp, vp, vp, ctypes.c_uint32]
        L.sbie_geom_sync.argtypes = [vp, vp]
        L.sbie_geom_set_depth_cap.argtypes = [vp, ctypes.c_int32]
        L.sbie_transform.argtypes = [vp, ctypes.c_int, ctypes.c_int32, vp, vp, vp, ctypes.c_uint32]
        L.sbie_geom_spectra.argtypes = [vp, dp]
        L.sbie_geom_timing.argtypes = [vp, ctypes.POINTER(Timing)]
        L.sbie_session_bytes.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int]
        L.sbie_session_bytes.restype = ctypes.c_uint64
        L.sbie_server_create.argtypes = [vp, ctypes.c_int32, ctypes.c_uint64, ctypes.c_uint32, ctypes.POINTER(vp)]
        L.sbie_server_destroy.argtypes = [vp]
        L.sbie_server_destroy.restype = None
        L.sbie_session_open.argtypes = [vp, dp, dp, dp, dp, ctypes.c_int32, ctypes.c_int32, ctypes.c_double,
                                        ctypes.c_int, ctypes.c_int, ctypes.POINTER(vp)]
        L.sbie_session_apply.argtypes = [vp, vp, vp, ctypes.c_uint32, ctypes.POINTER(ctypes.c_uint64)]
        L.sbie_session_close.argtypes = [vp]
        L.sbie_wait.argtypes = [vp, ctypes.c_uint64, ctypes.c_int64, ctypes.POINTER(ApplyStats)]
        L.sbie_server_get_info.argtypes = [vp, ctypes.POINTER(ServerInfo)]
        L.sbie_completion_eta.argtypes = [vp, ctypes.c_int, dp]
        L.sbie_apply_completed.argtypes = [vp, ctypes.c_int, ctypes.c_int, dp, vp, vp, vp, ctypes.c_uint32]
        L.sbie_solve_completed.argtypes = [vp, ctypes.c_int, ctypes.c_int, dp, vp, vp, ctypes.c_double,
                                           ctypes.c_int32, ctypes.POINTER(ctypes.c_int32),
                                           ctypes.POINTER(ctypes.c_double), vp, ctypes.c_uint32]
        L.sbie_solve_neumann.argtypes = [vp, ctypes.c_int, vp, vp, ctypes.c_double, ctypes.c_int32,
                                         ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_double), vp,
                                         ctypes.c_uint32]
        L.sbie_eval_targets.argtypes = [vp, ctypes.c_int, ctypes.c_int, vp, ctypes.c_int64, vp, vp, vp, vp,
                                        ctypes.c_uint32]
        L.sbie_eval_targets_noalloc.argtypes = [vp, ctypes.c_int, ctypes.c_int, vp, ctypes.c_int64, vp, vp, vp,
                                                vp, ctypes.c_uint32]
        L.sbie_geom_far_tree.argtypes = [vp, ctypes.c_double, ctypes.c_int32, ctypes.c_int32]
        L.sbie_geom_far_tree_info.argtypes = [vp, ctypes.POINTER(TreeInfo)]
        i64p = ctypes.POINTER(ctypes.c_int64)
        L.sbie_far_tree_plan.argtypes = [ctypes.c_int32, ctypes.c_int32, dp, dp, vp, ctypes.c_int32, ctypes.c_double,
                                         ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32), i64p, i64p,
                                         dp, ip, ip, ip, i64p, ip, i64p, ip]
        L.sbie_status_str.argtypes = [ctypes.c_int]
        L.sbie_status_str.restype = ctypes.c_char_p
        L.sbie_last_error.argtypes = []
        L.sbie_last_error.restype = ctypes.c_char_p
        _lib = L
    return _lib


def _check(rc: int):
    if rc != 0:
        raise SbieError(rc, lib().sbie_last_error().decode())


def _dp(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


class Context:
    """sbie_ctx: one HIP device and its stream."""

    def __init__(self, device: int = 0):
        self._h = ctypes.c_void_p()
        _check(lib().sbie_ctx_create(int(device), ctypes.byref(self._h)))
        _live.append(weakref.ref(self))

    @property
    def handle(self):
        return self._h

    def close(self):
        if self._h:
            lib().sbie_ctx_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Geometry:
    """sbie_geom: a suspension at order p with its near/far split (eta)."""

    def __init__(self, ctx: Context, geom: dict, p: int, eta: float = 1.0):
        self.ctx = ctx
        c = np.ascontiguousarray(geom["centers"], dtype=np.float64)
        q = np.ascontiguousarray(geom["quats"], dtype=np.float64)
        A = np.ascontiguousarray(geom["A"], dtype=np.float64)
        C = np.ascontiguousarray(geom["C"], dtype=np.float64)
        self.M = int(len(A))
        self.p = int(p)
        self._h = ctypes.c_void_p()
        _check(lib().sbie_geom_create(ctx.handle, _dp(c), _dp(q), _dp(A), _dp(C), self.M, self.p, float(eta),
                                      ctypes.byref(self._h)))
        self.N = int(lib().sbie_geom_num_nodes(self._h))
        _live.append(weakref.ref(self))

    @property
    def handle(self):
        return self._h

    @property
    def num_near_pairs(self) -> int:
        return int(lib().sbie_geom_num_near_pairs(self._h))

    @property
    def footprint_bytes(self) -> int:
        return int(lib().sbie_geom_footprint_bytes(self._h))

    def nodes(self):
        xyz = np.zeros((self.N, 3))
        nrm = np.zeros((self.N, 3))
        w = np.zeros(self.N)
        _check(lib().sbie_geom_nodes(self._h, _dp(xyz), _dp(nrm), _dp(w)))
        return xyz, nrm, w

    def near_pairs(self):
        cnt = ctypes.c_int64()
        _check(lib().sbie_geom_near_pairs(self._h, None, None, 0, ctypes.byref(cnt)))
        src = np.zeros(cnt.value, dtype=np.int32)
        dst = np.zeros(cnt.value, dtype=np.int32)
        ip = ctypes.POINTER(ctypes.c_int32)
        _check(lib().sbie_geom_near_pairs(self._h, src.ctypes.data_as(ip), dst.ctypes.data_as(ip), cnt.value,
                                          ctypes.byref(cnt)))
        return src, dst

    def apply(self, op: int, density, precision: int = SBIE_FP64, parts: int = SBIE_PARTS_ALL, out=None,
              stream=None, timing: bool = False, tree: bool = False, coeffs: bool = False):
        """Apply S, D, S', D' or the Stokes single layer.  density: torch CUDA float64
        tensor [nrhs, N] or [N] (device pointers, on the current stream), or a numpy
        array (host pointers, synchronous).  SBIE_OP_STOKES_SP returns [4, N]
        (velocity, then pressure).  tree: the far field of S or D through the
        geometry's tree (far_tree).  coeffs: S or D of given transform
        coefficients, density [nrhs, M, (p+1)^2] or [M, (p+1)^2] as transform()
        returns them (SBIE_INPUT_COEFFS); the result is [nrhs, N] or [N]."""
        flags = (int(parts) | (SBIE_TIMING if timing else 0) | (SBIE_FAR_TREE if tree else 0)
                 | (SBIE_INPUT_COEFFS if coeffs else 0))
        nin = self.M * (self.p + 1) ** 2 if coeffs else self.N
        if isinstance(density, np.ndarray):
            d = np.ascontiguousarray(density, dtype=np.float64)
            nrhs = d.size // nin if coeffs else (1 if d.ndim == 1 else d.shape[0])
            if d.size != nrhs * nin or nrhs < 1:
                raise ValueError(f"density has {d.size} entries, expected nrhs x {nin}")
            if op == SBIE_OP_STOKES_SP:
                o = np.zeros((4, self.N))
            else:
                o = np.zeros((nrhs, self.N) if (d.ndim > (2 if coeffs else 1)) else (self.N,))
            _check(lib().sbie_apply(self._h, int(op), int(precision), nrhs, d.ctypes.data, o.ctypes.data, None,
                                    flags))
            return o
        import torch

        if not (density.is_cuda and density.dtype == torch.float64 and density.is_contiguous()):
            raise ValueError("density must be a contiguous float64 CUDA tensor")
        nrhs = density.numel() // nin if coeffs else (1 if density.dim() == 1 else density.shape[0])
        if density.numel() != nrhs * nin or nrhs < 1:
            raise ValueError(f"density has {density.numel()} entries, expected {nrhs} x {nin}")
        if out is None:
            if op == SBIE_OP_STOKES_SP:
                out = torch.empty((4, self.N), dtype=torch.float64, device=density.device)
            elif coeffs:
                shape = (nrhs, self.N) if density.dim() > 2 else (self.N,)
                out = torch.empty(shape, dtype=torch.float64, device=density.device)
            else:
                out = torch.empty_like(density)
        if stream is None:
            stream = torch.cuda.current_stream(density.device)
        if stream.cuda_stream == 0:
            # a NULL stream selects the context's own stream, which does not
            # wait for work queued on the default stream: finish that first
            stream.synchronize()
        _check(lib().sbie_apply(self._h, int(op), int(precision), nrhs, density.data_ptr(), out.data_ptr(),
                                ctypes.c_void_p(stream.cuda_stream), flags | SBIE_DEVICE_PTRS))
        return out

    def far_tree(self, theta: float = 0.6, order: int = 10, leaf: int = 2):
        """Build the geometry's tree far field (sbie_geom_far_tree); returns far_tree_info()."""
        _check(lib().sbie_geom_far_tree(self._h, float(theta), int(order), int(leaf)))
        return self.far_tree_info()

    def far_tree_info(self) -> dict:
        info = TreeInfo()
        _check(lib().sbie_geom_far_tree_info(self._h, ctypes.byref(info)))
        return {name: getattr(info, name) for name, _ in TreeInfo._fields_}

    def completion_eta(self, completion: int) -> np.ndarray:
        """The eta table's scaling of each particle for the completion."""
        out = np.zeros(self.M)
        _check(lib().sbie_completion_eta(self._h, int(completion), _dp(out)))
        return out

    def _vectors(self, x, name):
        import torch

        if not (x.is_cuda and x.dtype == torch.float64 and x.is_contiguous() and x.numel() == self.N):
            raise ValueError(f"{name} must be a contiguous float64 CUDA tensor of {self.N} entries")
        stream = torch.cuda.current_stream(x.device)
        # the calls run on the context's stream and return after completion
        stream.synchronize()

    def apply_completed(self, completion: int, sigma, eta=None, precision: int = SBIE_FP64):
        """K[sigma] = sigma/2 + D[sigma] + C[sigma] (numpy: host pointers; torch CUDA
        float64: device pointers)."""
        e = None if eta is None else np.ascontiguousarray(eta, dtype=np.float64)
        ep = None if e is None else _dp(e)
        if isinstance(sigma, np.ndarray):
            d = np.ascontiguousarray(sigma, dtype=np.float64)
            if d.size != self.N:
                raise ValueError(f"sigma has {d.size} entries, expected {self.N}")
            o = np.zeros_like(d)
            _check(lib().sbie_apply_completed(self._h, int(precision), int(completion), ep, d.ctypes.data,
                                              o.ctypes.data, None, 0))
            return o
        import torch

        self._vectors(sigma, "sigma")
        o = torch.empty_like(sigma)
        _check(lib().sbie_apply_completed(self._h, int(precision), int(completion), ep, sigma.data_ptr(),
                                          o.data_ptr(), None, SBIE_DEVICE_PTRS))
        return o

    def solve_completed(self, completion: int, f, eta=None, tol: float = 1e-10, maxit: int = 500,
                        precision: int = SBIE_FP64):
        """GMRES for K[sigma] = f; returns (sigma, iterations, relative residual)."""
        e = None if eta is None else np.ascontiguousarray(eta, dtype=np.float64)
        ep = None if e is None else _dp(e)
        it = ctypes.c_int32(0)
        res = ctypes.c_double(0.0)
        if isinstance(f, np.ndarray):
            d = np.ascontiguousarray(f, dtype=np.float64)
            if d.size != self.N:
                raise ValueError(f"f has {d.size} entries, expected {self.N}")
            sig = np.zeros_like(d)
            _check(lib().sbie_solve_completed(self._h, int(precision), int(completion), ep, d.ctypes.data,
                                              sig.ctypes.data, float(tol), int(maxit), ctypes.byref(it),
                                              ctypes.byref(res), None, 0))
            return sig, it.value, res.value
        import torch

        self._vectors(f, "f")
        sig = torch.empty_like(f)
        _check(lib().sbie_solve_completed(self._h, int(precision), int(completion), ep, f.data_ptr(),
                                          sig.data_ptr(), float(tol), int(maxit), ctypes.byref(it),
                                          ctypes.byref(res), None, SBIE_DEVICE_PTRS))
        return sig, it.value, res.value

    def eval_targets(self, op: int, density, pts, precision: int = SBIE_FP64, gradient: bool = True):
        """S or D of the nodal density at points outside every particle: returns
        (value [n], gradient [n, 3] or None).  numpy inputs use host pointers;
        torch CUDA float64 tensors device pointers."""
        if isinstance(density, np.ndarray):
            d = np.ascontiguousarray(density, dtype=np.float64)
            x = np.ascontiguousarray(pts, dtype=np.float64).reshape(-1, 3)
            if d.size != self.N:
                raise ValueError(f"density has {d.size} entries, expected {self.N}")
            val = np.zeros(len(x))
            grad = np.zeros((len(x), 3)) if gradient else None
            _check(lib().sbie_eval_targets(self._h, int(op), int(precision), d.ctypes.data, len(x), x.ctypes.data,
                                           val.ctypes.data, grad.ctypes.data if gradient else None, None, 0))
            return val, grad
        import torch

        self._vectors(density, "density")
        if not (pts.is_cuda and pts.dtype == torch.float64 and pts.is_contiguous() and pts.dim() == 2
                and pts.shape[1] == 3):
            raise ValueError("pts must be a contiguous float64 CUDA tensor [n, 3]")
        n = pts.shape[0]
        val = torch.empty(n, dtype=torch.float64, device=pts.device)
        grad = torch.empty((n, 3), dtype=torch.float64, device=pts.device) if gradient else None
        _check(lib().sbie_eval_targets(self._h, int(op), int(precision), density.data_ptr(), n, pts.data_ptr(),
                                       val.data_ptr(), grad.data_ptr() if gradient else None, None,
                                       SBIE_DEVICE_PTRS))
        return val, grad

    def eval_targets_noalloc(self, op: int, density, pts, val, grad=None, precision: int = SBIE_FP64, stream=None):
        """sbie_eval_targets_noalloc: as eval_targets on torch CUDA float64 tensors, into
        the caller's val [n] and grad [n, 3] (or None), with the library's static
        work space instead of allocations."""
        import torch

        for name, t in (("density", density), ("pts", pts), ("val", val)) + ((("grad", grad),) if grad is not None
                                                                          else ()):
            if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
                raise ValueError(f"{name} must be a contiguous float64 CUDA tensor")
        n = pts.shape[0]
        if density.numel() != self.N or pts.dim() != 2 or pts.shape[1] != 3 or val.numel() != n or (
                grad is not None and grad.numel() != 3 * n):
            raise ValueError("density [N], pts [n, 3], val [n] and grad [n, 3] expected")
        if stream is None:
            torch.cuda.current_stream(pts.device).synchronize()
        _check(lib().sbie_eval_targets_noalloc(self._h, int(op), int(precision), density.data_ptr(), n,
                                               pts.data_ptr(), val.data_ptr(),
                                               grad.data_ptr() if grad is not None else None,
                                               ctypes.c_void_p(stream.cuda_stream) if stream is not None else None,
                                               SBIE_DEVICE_PTRS))
        return val, grad

    def solve_neumann(self, data, tol: float = 1e-10, maxit: int = 500, precision: int = SBIE_FP64):
        """GMRES for -rho/2 + S'[rho] = data (single-layer Neumann problem);
        returns (rho, iterations, relative residual)."""
        it = ctypes.c_int32(0)
        res = ctypes.c_double(0.0)
        if isinstance(data, np.ndarray):
            d = np.ascontiguousarray(data, dtype=np.float64)
            if d.size != self.N:
                raise ValueError(f"data has {d.size} entries, expected {self.N}")
            rho = np.zeros_like(d)
            _check(lib().sbie_solve_neumann(self._h, int(precision), d.ctypes.data, rho.ctypes.data, float(tol),
                                            int(maxit), ctypes.byref(it), ctypes.byref(res), None, 0))
            return rho, it.value, res.value
        import torch

        self._vectors(data, "data")
        rho = torch.empty_like(data)
        _check(lib().sbie_solve_neumann(self._h, int(precision), data.data_ptr(), rho.data_ptr(), float(tol),
                                        int(maxit), ctypes.byref(it), ctypes.byref(res), None, SBIE_DEVICE_PTRS))
        return rho, it.value, res.value

    def transform(self, op: int, density: np.ndarray) -> np.ndarray:
        """Forward transform (host arrays): coefficients [nrhs][M][(p+1)^2]."""
        d = np.ascontiguousarray(density, dtype=np.float64)
        nrhs = 1 if d.ndim == 1 else d.shape[0]
        out = np.zeros((nrhs, self.M, (self.p + 1) ** 2))
        _check(lib().sbie_transform(self._h, int(op), nrhs, d.ctypes.data, out.ctypes.data, None, 0))
        return out

    def spectra(self) -> np.ndarray:
        """Per-particle spectra [M][(p+1)(p+2)/2][4]."""
        out = np.zeros((self.M, (self.p + 1) * (self.p + 2) // 2, 4))
        _check(lib().sbie_geom_spectra(self._h, _dp(out)))
        return out

    def set_depth_cap(self, steps: int = 100000):
        """Cap the near-field recurrence at `steps` steps past degree p+1 (a test
        control: an evaluation needing more is reported as SBIE_E_NUMERIC)."""
        _check(lib().sbie_geom_set_depth_cap(self._h, int(steps)))

    def sync(self, stream=None):
        """Wait for the stream (torch stream or None for the current one) and raise on a
        numerical failure recorded by the kernels since the last check."""
        import torch

        if stream is None:
            stream = torch.cuda.current_stream()
        _check(lib().sbie_geom_sync(self._h, ctypes.c_void_p(stream.cuda_stream)))

    def timing(self) -> Timing:
        """Per-part device times averaged over the timed applies since the last call."""
        t = Timing()
        _check(lib().sbie_geom_timing(self._h, ctypes.byref(t)))
        return t

    def close(self):
        if self._h:
            lib().sbie_geom_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def session_bytes(M: int, p: int, op: int) -> int:
    """Device bytes a served session holds while admitted."""
    return int(lib().sbie_session_bytes(int(M), int(p), int(op)))


class Server:
    """sbie_server: served mode (lanes of a host thread and a stream each, one HBM arena)."""

    def __init__(self, ctx: Context, max_sessions: int = 8, budget_bytes: int = 1 << 30, graphs: bool = True,
                 batch: bool = False, tree: bool = False):
        self.ctx = ctx
        self._h = ctypes.c_void_p()
        flags = ((SBIE_SERVER_GRAPHS if graphs else 0) | (SBIE_SERVER_BATCH if batch else 0)
                 | (SBIE_SERVER_TREE if tree else 0))
        _check(lib().sbie_server_create(ctx.handle, int(max_sessions), int(budget_bytes), flags,
                                        ctypes.byref(self._h)))
        _live.append(weakref.ref(self))

    def open(self, geom: dict, p: int, op: int, precision: int = SBIE_FP64, eta: float = 1.0) -> "Session":
        return Session(self, geom, p, op, precision, eta)

    def wait(self, ticket: int, timeout_us: int = -1) -> ApplyStats:
        """Wait for an apply; raises SbieError on its failure (SBIE_E_TIMEOUT keeps the ticket)."""
        st = ApplyStats()
        _check(lib().sbie_wait(self._h, ctypes.c_uint64(ticket), int(timeout_us), ctypes.byref(st)))
        return st

    def info(self) -> ServerInfo:
        out = ServerInfo()
        _check(lib().sbie_server_get_info(self._h, ctypes.byref(out)))
        return out

    def close(self):
        if self._h:
            lib().sbie_server_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Session:
    """sbie_session: one suspension, operator and precision on a Server."""

    def __init__(self, server: Server, geom: dict, p: int, op: int, precision: int, eta: float):
        self.server = server
        c = np.ascontiguousarray(geom["centers"], dtype=np.float64)
        q = np.ascontiguousarray(geom["quats"], dtype=np.float64)
        A = np.ascontiguousarray(geom["A"], dtype=np.float64)
        C = np.ascontiguousarray(geom["C"], dtype=np.float64)
        self.M, self.p, self.op = int(len(A)), int(p), int(op)
        self.nrhs = 3 if op == SBIE_OP_STOKES_S else 1
        self.N = self.M * (self.p + 1) * (2 * self.p + 2)
        self._h = ctypes.c_void_p()
        _check(lib().sbie_session_open(server._h, _dp(c), _dp(q), _dp(A), _dp(C), self.M, self.p, float(eta),
                                       int(op), int(precision), ctypes.byref(self._h)))
        self._keep = {}

    def submit(self, density, out) -> int:
        """Queue an apply.  density/out: contiguous float64 CUDA tensors or numpy arrays of
        nrhs*N entries; they must stay alive until the ticket is waited for."""
        if isinstance(density, np.ndarray):
            if not (isinstance(out, np.ndarray) and density.flags.c_contiguous and out.flags.c_contiguous
                    and density.dtype == np.float64 and out.dtype == np.float64):
                raise ValueError("density and out must be contiguous float64 arrays")
            n, no = density.size, out.size
            dptr, optr, flags = density.ctypes.data, out.ctypes.data, 0
        else:
            import torch

            for t_ in (density, out):
                if not (t_.is_cuda and t_.dtype == torch.float64 and t_.is_contiguous()):
                    raise ValueError("density and out must be contiguous float64 CUDA tensors")
            n, no = density.numel(), out.numel()
            dptr, optr, flags = density.data_ptr(), out.data_ptr(), SBIE_DEVICE_PTRS
            # the lanes run on their own streams: the density must be complete
            torch.cuda.current_stream(density.device).synchronize()
        if n != self.nrhs * self.N or no != n:
            raise ValueError(f"density/out hold {n}/{no} values, expected {self.nrhs} x {self.N}")
        t = ctypes.c_uint64()
        _check(lib().sbie_session_apply(self._h, ctypes.c_void_p(dptr), ctypes.c_void_p(optr), flags,
                                        ctypes.byref(t)))
        self._keep[t.value] = (density, out)
        return t.value

    def apply(self, density, out=None):
        """Submit and wait (closed loop); returns (out, stats)."""
        if out is None:
            out = np.zeros_like(density) if isinstance(density, np.ndarray) else density.new_empty(density.shape)
        t = self.submit(density, out)
        try:
            st = self.server.wait(t)
        finally:
            self._keep.pop(t, None)
        return out, st

    def close(self):
        if self._h:
            _check(lib().sbie_session_close(self._h))
            self._h = ctypes.c_void_p()


def far_tree_plan(centers, radii, excl, T: int, theta: float = 0.5, order: int = 8, leaf: int = 2) -> dict:
    """The tree far field's plan on the host (sbie_far_tree_plan; no device).
    excl: bool [M, M], excl[t, s] true iff source particle s is excluded for
    target particle t."""
    c = np.ascontiguousarray(centers, dtype=np.float64)
    r = np.ascontiguousarray(radii, dtype=np.float64)
    e = np.asarray(excl, dtype=bool)
    M = len(r)
    words = (M + 31) // 32
    ex = np.zeros((M, words), dtype=np.uint32)
    t, s = np.nonzero(e)
    np.bitwise_or.at(ex, (t, s >> 5), np.left_shift(np.uint32(1), (s & 31).astype(np.uint32)))
    nc, npx, ndr = ctypes.c_int32(), ctypes.c_int64(), ctypes.c_int64()
    args = [M, int(T), _dp(c), _dp(r), ex.ctypes.data, words, float(theta), int(order), int(leaf)]
    counts = [ctypes.byref(nc), ctypes.byref(npx), ctypes.byref(ndr)]
    _check(lib().sbie_far_tree_plan(*args, *counts, *([None] * 8)))
    out = {"box": np.zeros((nc.value, 6)), "first": np.zeros(nc.value, np.int32), "count": np.zeros(nc.value, np.int32),
           "perm": np.zeros(M, np.int32), "proxy_ptr": np.zeros(M + 1, np.int64),
           "proxy_idx": np.zeros(max(npx.value, 1), np.int32), "direct_ptr": np.zeros(M + 1, np.int64),
           "direct_idx": np.zeros(max(ndr.value, 1), np.int32)}
    P = ctypes.POINTER
    ptrs = [out["box"].ctypes.data_as(P(ctypes.c_double))] + [
        out[k].ctypes.data_as(P(ctypes.c_int32 if out[k].dtype == np.int32 else ctypes.c_int64))
        for k in ("first", "count", "perm", "proxy_ptr", "proxy_idx", "direct_ptr", "direct_idx")]
    _check(lib().sbie_far_tree_plan(*args, *counts, *ptrs))
    out["proxy_idx"] = out["proxy_idx"][:npx.value]
    out["direct_idx"] = out["direct_idx"][:ndr.value]
    return out

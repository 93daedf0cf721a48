"""Python binding of ``libhbmc.so`` (the C ABI declared in include/hbmc.h).

Argument marshalling only: every step of the method runs in the library.
PyTorch provides device memory (tensors whose pointers are handed to the
library) and the current HIP stream.  The binding fails loudly when the
library is missing; there is no fallback implementation.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libhbmc.so")

HBMC_OK, HBMC_EINVAL, HBMC_ENOTSYM, HBMC_EDIAG, HBMC_EBREAKDOWN = 0, -1, -2, -3, -4
HBMC_EHIP, HBMC_ENOMEM, HBMC_ENOTREADY, HBMC_ENOCONV = -5, -6, -7, 1
HBMC_F64, HBMC_F32 = 0, 1
HBMC_KERNEL_AUTO, HBMC_KERNEL_SWEEP, HBMC_KERNEL_ROWS = 0, 1, 2
HBMC_SYNC_AUTO, HBMC_SYNC_LAUNCH = 0, 1
HBMC_SMOOTH_SYMMETRIC, HBMC_SMOOTH_FORWARD = 0, 1

# every symbol include/hbmc.h declares
SYMBOLS = (
    "hbmc_last_error", "hbmc_order", "hbmc_order_rcm", "hbmc_rcm", "hbmc_order_batch", "hbmc_order_info",
    "hbmc_order_perm",
    "hbmc_order_destroy", "ic0_factor", "hbmc_factor_export", "hbmc_factor_device_bytes",
    "hbmc_factor_upload", "hbmc_factor_destroy", "hbmc_factor_set_kernel", "hbmc_factor_set_rhs_tile",
    "hbmc_factor_set_sync", "hbmc_factor_set_wait_limit", "ic0_apply", "ic0_apply_ws_bytes", "ic0_apply_ws", "hbmc_matrix_create",
    "hbmc_matrix_device_bytes", "hbmc_matrix_upload", "hbmc_matrix_destroy", "hbmc_spmv",
    "hbmc_to_hbmc", "hbmc_from_hbmc", "iccg_workspace_bytes", "iccg_solve", "iccg_solve_noalloc",
    "iccg_history",
    "ssor_factor", "hbmc_smooth_workspace_bytes", "hbmc_smooth",
    "hbmc_factor_image", "hbmc_matrix_image", "hbmc_set_num_threads",
    "hbmc_revalue_create", "hbmc_revalue_device_bytes", "hbmc_revalue_upload", "hbmc_revalue_destroy",
    "ic0_refactor", "ssor_refactor", "hbmc_matrix_revalue",
    "hbmc_device_build_bytes", "hbmc_device_build", "hbmc_device_build_create", "hbmc_device_build_fill",
    "hbmc_device_build_destroy",
)


class HbmcError(RuntimeError):
    def __init__(self, call: str, code: int, msg: str):
        super().__init__(f"{call} -> {code}: {msg}")
        self.code = code


class OrderInfo(C.Structure):
    _fields_ = [("n", C.c_int64), ("n_pad", C.c_int64), ("n_blocks", C.c_int64),
                ("n_colors", C.c_int32), ("bs", C.c_int32), ("w", C.c_int32),
                ("n_systems", C.c_int32)]


class SolveOpts(C.Structure):
    _fields_ = [("x0_zero", C.c_int32), ("check_every", C.c_int32),
                ("use_graph", C.c_int32), ("record_history", C.c_int32), ("x0_scale", C.c_int32)]


class SolveStats(C.Structure):
    _fields_ = [("iters", C.c_int32), ("status", C.c_int32), ("rel_res", C.c_double),
                ("true_rel_res", C.c_double), ("x0_scale", C.c_double)]


_lib = None


def lib():
    """Loads libhbmc.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_1908_00741_amd.build`")
        L = C.CDLL(LIB_PATH)
        P, i32, i64, f64, sz = C.c_void_p, C.c_int32, C.c_int64, C.c_double, C.c_size_t
        L.hbmc_last_error.restype = C.c_char_p
        L.hbmc_order.argtypes = [i32, P, P, i32, i32, P]
        L.hbmc_order_rcm.argtypes = [i32, P, P, i32, i32, P]
        L.hbmc_rcm.argtypes = [i32, P, P, P]
        L.hbmc_order_batch.argtypes = [i32, P, i32, P, P, i32, i32, P]
        L.hbmc_order_info.argtypes = [P, P]
        L.hbmc_order_perm.argtypes = [P, P, P]
        L.hbmc_order_destroy.argtypes = [P]
        L.hbmc_order_destroy.restype = None
        L.ic0_factor.argtypes = [P, P, P, P, i32, f64, P]
        L.hbmc_factor_export.argtypes = [P, P, P, P, P, P]
        L.hbmc_factor_device_bytes.argtypes = [P, P]
        L.hbmc_factor_upload.argtypes = [P, P, sz, P]
        L.hbmc_factor_set_kernel.argtypes = [P, i32]
        L.hbmc_factor_set_rhs_tile.argtypes = [P, i32]
        L.hbmc_factor_destroy.argtypes = [P]
        L.hbmc_factor_destroy.restype = None
        L.ic0_apply.argtypes = [P, P, P, i32, P]
        L.hbmc_factor_set_sync.argtypes = [P, i32]
        L.hbmc_factor_set_wait_limit.argtypes = [P, i64]
        L.ic0_apply_ws_bytes.argtypes = [P, P]
        L.ic0_apply_ws.argtypes = [P, P, P, i32, P, sz, P]
        L.hbmc_matrix_create.argtypes = [P, P, P, P, P]
        L.hbmc_matrix_device_bytes.argtypes = [P, P]
        L.hbmc_matrix_upload.argtypes = [P, P, sz, P]
        L.hbmc_matrix_destroy.argtypes = [P]
        L.hbmc_matrix_destroy.restype = None
        L.hbmc_spmv.argtypes = [P, P, P, i32, P]
        L.hbmc_to_hbmc.argtypes = [P, P, P, i32, P]
        L.hbmc_from_hbmc.argtypes = [P, P, P, i32, P]
        L.iccg_workspace_bytes.argtypes = [P, i32, P]
        L.iccg_solve.argtypes = [P, P, P, P, i32, f64, i32, P, P, P, sz, P]
        L.iccg_solve_noalloc.argtypes = [P, P, P, P, i32, f64, i32, P, P, P]
        L.iccg_history.argtypes = [P, sz, P, P, i32, P]
        L.ssor_factor.argtypes = [P, P, P, P, i32, f64, P]
        L.hbmc_smooth_workspace_bytes.argtypes = [P, i32, P]
        L.hbmc_smooth.argtypes = [P, P, P, P, i32, i32, i32, P, sz, P]
        L.hbmc_factor_image.argtypes = [P, P, sz]
        L.hbmc_matrix_image.argtypes = [P, P, sz]
        L.hbmc_set_num_threads.argtypes = [i32]
        L.hbmc_revalue_create.argtypes = [P, P, P, P]
        L.hbmc_revalue_device_bytes.argtypes = [P, P]
        L.hbmc_revalue_upload.argtypes = [P, P, sz, P]
        L.hbmc_revalue_destroy.argtypes = [P]
        L.hbmc_revalue_destroy.restype = None
        L.ic0_refactor.argtypes = [P, P, P, f64, P]
        L.ssor_refactor.argtypes = [P, P, P, f64, P]
        L.hbmc_matrix_revalue.argtypes = [P, P, P, P]
        L.hbmc_device_build_bytes.argtypes = [P, i64, P]
        L.hbmc_device_build.argtypes = [P, P, P, P, i64, i32, f64, P, sz, P, P]
        L.hbmc_device_build_create.argtypes = [P, P, P]
        L.hbmc_device_build_fill.argtypes = [P, P, P, P, sz, P, sz, P, P]
        L.hbmc_device_build_destroy.argtypes = [P]
        L.hbmc_device_build_destroy.restype = None
        _lib = L
    return _lib


def _check(call: str, code: int, ok=(HBMC_OK,)):
    if code not in ok:
        raise HbmcError(call, code, lib().hbmc_last_error().decode())
    return code


def _ptr(a: np.ndarray):
    assert a.flags.c_contiguous
    return a.ctypes.data_as(C.c_void_p)


def _csr_arrays(A):
    return (np.ascontiguousarray(A.rowptr, np.int64), np.ascontiguousarray(A.col, np.int32),
            np.ascontiguousarray(A.val, np.float64))


def _stream(stream=None):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return C.c_void_p(s.cuda_stream)


def _dptr(t):
    return C.c_void_p(t.data_ptr())


class Order:
    """Handle of hbmc_order: BMC blocking + coloring + HBMC reordering."""

    def __init__(self, handle, A):
        self._h = handle
        info = OrderInfo()
        _check("hbmc_order_info", lib().hbmc_order_info(self._h, C.byref(info)))
        self.n, self.n_pad, self.n_blocks = info.n, info.n_pad, info.n_blocks
        self.n_colors, self.bs, self.w = info.n_colors, info.bs, info.w
        self.n_systems = info.n_systems

    @property
    def handle(self):
        return self._h

    def perm(self):
        perm = np.empty(self.n, np.int32)
        cs = np.empty(self.n_colors + 1, np.int64)
        _check("hbmc_order_perm", lib().hbmc_order_perm(self._h, _ptr(perm), _ptr(cs)))
        return perm, cs

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.hbmc_order_destroy(self._h)
            self._h = None


def hbmc_order(A, bs: int, w: int, rcm: bool = False) -> Order:
    """HBMC ordering of A's pattern; with rcm, of the pattern renumbered by
    reverse Cuthill-McKee first (hbmc_order_rcm), in A's numbering."""
    rp, ci, _ = _csr_arrays(A)
    h = C.c_void_p()
    name = "hbmc_order_rcm" if rcm else "hbmc_order"
    _check(name, getattr(lib(), name)(A.n, _ptr(rp), _ptr(ci), bs, w, C.byref(h)))
    return Order(h, A)


def hbmc_rcm(A) -> np.ndarray:
    """Reverse Cuthill-McKee numbering: entry k is the unknown numbered k."""
    rp, ci, _ = _csr_arrays(A)
    out = np.empty(A.n, np.int32)
    _check("hbmc_rcm", lib().hbmc_rcm(A.n, _ptr(rp), _ptr(ci), _ptr(out)))
    return out


def hbmc_order_batch(A, sys_ptr, bs: int, w: int) -> Order:
    """Batch of independent systems: A is block diagonal and system s owns rows
    sys_ptr[s] .. sys_ptr[s + 1] - 1."""
    rp, ci, _ = _csr_arrays(A)
    sp = np.ascontiguousarray(sys_ptr, np.int64)
    h = C.c_void_p()
    _check("hbmc_order_batch", lib().hbmc_order_batch(len(sp) - 1, _ptr(sp), A.n, _ptr(rp), _ptr(ci),
                                                      bs, w, C.byref(h)))
    return Order(h, A)


class Factor:
    """Handle of ic0_factor; ``upload()`` places it in device memory."""

    def __init__(self, handle, order: Order, precision: int):
        self._h = handle
        self.n, self.n_pad, self.bs, self.w = order.n, order.n_pad, order.bs, order.w
        self.n_colors, self.n_systems = order.n_colors, order.n_systems
        self.precision = precision
        self.dev = None

    @property
    def handle(self):
        return self._h

    def image(self) -> np.ndarray:
        """Host copy of the device image (bytes)."""
        out = np.empty(self.device_bytes(), np.uint8)
        _check("hbmc_factor_image", lib().hbmc_factor_image(self._h, _ptr(out), out.size))
        return out

    def export(self):
        """(d, lower_rowptr, lower_col, lower_val) of the FP64 factor."""
        nnz = C.c_int64(0)
        _check("hbmc_factor_export", lib().hbmc_factor_export(self._h, None, None, None, None,
                                                              C.byref(nnz)))
        d = np.empty(self.n_pad)
        rp = np.empty(self.n_pad + 1, np.int64)
        ci = np.empty(nnz.value, np.int32)
        v = np.empty(nnz.value)
        _check("hbmc_factor_export", lib().hbmc_factor_export(self._h, _ptr(d), _ptr(rp), _ptr(ci),
                                                              _ptr(v), C.byref(nnz)))
        return d, rp, ci, v

    def device_bytes(self) -> int:
        b = C.c_size_t(0)
        _check("hbmc_factor_device_bytes", lib().hbmc_factor_device_bytes(self._h, C.byref(b)))
        return b.value

    def set_kernel(self, kernel: int):
        _check("hbmc_factor_set_kernel", lib().hbmc_factor_set_kernel(self._h, int(kernel)))
        return self

    def set_sync(self, sync: int):
        _check("hbmc_factor_set_sync", lib().hbmc_factor_set_sync(self._h, int(sync)))
        return self

    def set_wait_limit(self, us: int):
        _check("hbmc_factor_set_wait_limit", lib().hbmc_factor_set_wait_limit(self._h, int(us)))
        return self

    def apply_ws_bytes(self) -> int:
        b = C.c_size_t(0)
        _check("ic0_apply_ws_bytes", lib().ic0_apply_ws_bytes(self._h, C.byref(b)))
        return b.value

    def set_rhs_tile(self, nr: int):
        _check("hbmc_factor_set_rhs_tile", lib().hbmc_factor_set_rhs_tile(self._h, int(nr)))
        return self

    def upload(self, device="cuda", stream=None):
        import torch
        nbytes = self.device_bytes()
        self.dev = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=device)
        _check("hbmc_factor_upload", lib().hbmc_factor_upload(self._h, _dptr(self.dev), nbytes,
                                                              _stream(stream)))
        return self

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.hbmc_factor_destroy(self._h)
            self._h = None


def ic0_factor(order: Order, A, precision: int = HBMC_F64, shift: float = 0.0) -> Factor:
    rp, ci, v = _csr_arrays(A)
    h = C.c_void_p()
    _check("ic0_factor", lib().ic0_factor(order.handle, _ptr(rp), _ptr(ci), _ptr(v), precision,
                                          float(shift), C.byref(h)))
    return Factor(h, order, precision)


class Revalue:
    """Handle of hbmc_revalue_create: the pattern data with which
    ic0_refactor and hbmc_matrix_revalue take new values of the same
    matrix on the device."""

    def __init__(self, order: Order, A):
        rp, ci, _ = _csr_arrays(A)
        h = C.c_void_p()
        _check("hbmc_revalue_create", lib().hbmc_revalue_create(order.handle, _ptr(rp), _ptr(ci), C.byref(h)))
        self._h = h
        self.nnz = int(rp[-1])
        self.dev = None

    @property
    def handle(self):
        return self._h

    def upload(self, device="cuda", stream=None):
        import torch
        b = C.c_size_t(0)
        _check("hbmc_revalue_device_bytes", lib().hbmc_revalue_device_bytes(self._h, C.byref(b)))
        self.dev = torch.empty(max(b.value, 256), dtype=torch.uint8, device=device)
        _check("hbmc_revalue_upload", lib().hbmc_revalue_upload(self._h, _dptr(self.dev), b.value,
                                                                _stream(stream)))
        return self

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.hbmc_revalue_destroy(self._h)
            self._h = None


def _val_check(rv: Revalue, val):
    import torch
    if not (val.is_cuda and val.dtype == torch.float64 and val.is_contiguous() and val.numel() == rv.nnz):
        raise ValueError(f"val must be a contiguous float64 device tensor of {rv.nnz} entries")


def ic0_refactor(f: Factor, rv: Revalue, val, shift: float = 0.0, stream=None) -> Factor:
    """IC(0) of new values (the caller's CSR order, same pattern) computed on
    the device, written into f's device image."""
    _val_check(rv, val)
    _check("ic0_refactor", lib().ic0_refactor(f.handle, rv.handle, _dptr(val), float(shift), _stream(stream)))
    return f


def ssor_refactor(f: Factor, rv: Revalue, val, omega: float = 1.0, stream=None) -> Factor:
    """The SSOR splitting of new values (same pattern), on the device."""
    _val_check(rv, val)
    _check("ssor_refactor", lib().ssor_refactor(f.handle, rv.handle, _dptr(val), float(omega), _stream(stream)))
    return f


def hbmc_matrix_revalue(m: Matrix, rv: Revalue, val, stream=None) -> Matrix:
    _val_check(rv, val)
    _check("hbmc_matrix_revalue", lib().hbmc_matrix_revalue(m.handle, rv.handle, _dptr(val), _stream(stream)))
    return m


def set_num_threads(threads: int = 0) -> None:
    """Host threads of the setup (0 = all hardware threads)."""
    _check("hbmc_set_num_threads", lib().hbmc_set_num_threads(int(threads)))


def ssor_factor(order: Order, A, precision: int = HBMC_F64, omega: float = 1.0) -> Factor:
    """SSOR splitting of Abar (d = a_ii / omega, L = strict lower part of
    Abar) in the factor's layout: a preconditioner for iccg_solve and the
    operator of hbmc_smooth."""
    rp, ci, v = _csr_arrays(A)
    h = C.c_void_p()
    _check("ssor_factor", lib().ssor_factor(order.handle, _ptr(rp), _ptr(ci), _ptr(v), precision,
                                            float(omega), C.byref(h)))
    return Factor(h, order, precision)


class Matrix:
    """Handle of hbmc_matrix_create: Abar in sliced ELL."""

    def __init__(self, handle, order: Order):
        self._h = handle
        self.n, self.n_pad = order.n, order.n_pad
        self.dev = None

    @property
    def handle(self):
        return self._h

    def device_bytes(self) -> int:
        b = C.c_size_t(0)
        _check("hbmc_matrix_device_bytes", lib().hbmc_matrix_device_bytes(self._h, C.byref(b)))
        return b.value

    def image(self) -> np.ndarray:
        """Host copy of the device image (bytes)."""
        out = np.empty(self.device_bytes(), np.uint8)
        _check("hbmc_matrix_image", lib().hbmc_matrix_image(self._h, _ptr(out), out.size))
        return out

    def upload(self, device="cuda", stream=None):
        import torch
        nbytes = self.device_bytes()
        self.dev = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=device)
        _check("hbmc_matrix_upload", lib().hbmc_matrix_upload(self._h, _dptr(self.dev), nbytes,
                                                              _stream(stream)))
        return self

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.hbmc_matrix_destroy(self._h)
            self._h = None


def hbmc_matrix_create(order: Order, A) -> Matrix:
    rp, ci, v = _csr_arrays(A)
    h = C.c_void_p()
    _check("hbmc_matrix_create", lib().hbmc_matrix_create(order.handle, _ptr(rp), _ptr(ci), _ptr(v),
                                                          C.byref(h)))
    return Matrix(h, order)


@dataclass
class DeviceBuild:
    """Factor and matrix built by hbmc_device_build from a CSR in device
    memory (the device images are those of the host build, byte for byte);
    work holds d and L for Factor.export."""
    factor: Factor
    matrix: Matrix
    work: object
    seconds: dict


def device_build(order: Order, A=None, precision: int = HBMC_F64, shift: float = 0.0, device="cuda",
                 csr_dev=None, stream=None) -> DeviceBuild:
    """IC(0) factor and matrix of A under order, set up on the device.  A is
    a host CSR (copied to the device first, timed apart) or csr_dev =
    (rowptr, col, val) device tensors (int64, int32, float64)."""
    import time
    import torch
    t0 = time.perf_counter()
    if csr_dev is None:
        rp, ci, v = _csr_arrays(A)
        csr_dev = (torch.from_numpy(rp).to(device), torch.from_numpy(ci).to(device), torch.from_numpy(v).to(device))
        torch.cuda.synchronize()
    t1 = time.perf_counter()
    rp_d, ci_d, v_d = csr_dev
    nnz = int(ci_d.numel())
    b = C.c_size_t(0)
    _check("hbmc_device_build_bytes", lib().hbmc_device_build_bytes(order.handle, nnz, C.byref(b)))
    work = torch.empty(max(b.value, 256), dtype=torch.uint8, device=device)
    h = C.c_void_p()
    _check("hbmc_device_build", lib().hbmc_device_build(order.handle, _dptr(rp_d), _dptr(ci_d), _dptr(v_d), nnz,
                                                        int(precision), float(shift), _dptr(work), work.numel(),
                                                        _stream(stream), C.byref(h)))
    try:
        fh, mh = C.c_void_p(), C.c_void_p()
        _check("hbmc_device_build_create", lib().hbmc_device_build_create(h, C.byref(fh), C.byref(mh)))
        f, m = Factor(fh, order, precision), Matrix(mh, order)
        fdev = torch.empty(max(f.device_bytes(), 256), dtype=torch.uint8, device=device)
        mdev = torch.empty(max(m.device_bytes(), 256), dtype=torch.uint8, device=device)
        _check("hbmc_device_build_fill", lib().hbmc_device_build_fill(h, fh, mh, _dptr(fdev), fdev.numel(),
                                                                      _dptr(mdev), mdev.numel(), _dptr(work),
                                                                      _stream(stream)))
        f.dev, m.dev = fdev, mdev
    finally:
        lib().hbmc_device_build_destroy(h)
    t2 = time.perf_counter()
    return DeviceBuild(f, m, work, {"csr_upload": t1 - t0, "build": t2 - t1})


def _vec_check(t, n, nrhs, name):
    import torch
    if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
        raise ValueError(f"{name} must be a contiguous float64 device tensor")
    if t.numel() != n * nrhs:
        raise ValueError(f"{name} has {t.numel()} elements, expected {n * nrhs}")


def ic0_apply(f: Factor, r, z=None, nrhs: int = 1, stream=None):
    """z = M^-1 r on device vectors in HBMC order ([n_pad][nrhs])."""
    import torch
    _vec_check(r, f.n_pad, nrhs, "r")
    if z is None:
        z = torch.empty_like(r)
    _vec_check(z, f.n_pad, nrhs, "z")
    _check("ic0_apply", lib().ic0_apply(f.handle, _dptr(r), _dptr(z), nrhs, _stream(stream)))
    return z


def apply_workspace(f: Factor, device="cuda"):
    """A device workspace for ic0_apply_ws (ic0_apply_ws_bytes bytes)."""
    import torch
    return torch.zeros(f.apply_ws_bytes(), dtype=torch.uint8, device=device)


def ic0_apply_ws(f: Factor, r, z=None, ws=None, nrhs: int = 1, stream=None):
    """ic0_apply with a workspace (the one-launch form of the row kernel
    where it applies); ws from apply_workspace, allocated if None."""
    import torch
    _vec_check(r, f.n_pad, nrhs, "r")
    if z is None:
        z = torch.empty_like(r)
    _vec_check(z, f.n_pad, nrhs, "z")
    if ws is None:
        ws = apply_workspace(f, r.device)
    if ws.dtype != torch.uint8 or not ws.is_contiguous():
        raise ValueError("ws must be a contiguous uint8 tensor")
    _check("ic0_apply_ws", lib().ic0_apply_ws(f.handle, _dptr(r), _dptr(z), nrhs, _dptr(ws), ws.numel(),
                                              _stream(stream)))
    return z


def apply_ws_error(ws) -> int:
    """The error word of an ic0_apply_ws workspace (nonzero: a wait timed
    out and z holds NaN); synchronizes with the device."""
    import torch
    return int(ws[:4].view(torch.int32).item())


def smooth_workspace(f: Factor, nrhs: int = 1, device="cuda"):
    import torch
    b = C.c_size_t(0)
    _check("hbmc_smooth_workspace_bytes", lib().hbmc_smooth_workspace_bytes(f.handle, nrhs, C.byref(b)))
    return torch.empty(max(b.value, 256), dtype=torch.uint8, device=device)


def hbmc_smooth(f: Factor, m: Matrix, b, x, sweeps: int = 1, mode: int = HBMC_SMOOTH_SYMMETRIC,
                nrhs: int = 1, work=None, stream=None):
    """sweeps steps x <- x + c M^-1 (b - Abar x) in place on device vectors in
    HBMC order ([n_pad][nrhs]); returns x."""
    _vec_check(b, f.n_pad, nrhs, "b")
    _vec_check(x, f.n_pad, nrhs, "x")
    if work is None:
        work = smooth_workspace(f, nrhs, x.device)
    _check("hbmc_smooth", lib().hbmc_smooth(f.handle, m.handle, _dptr(b), _dptr(x), nrhs, int(sweeps),
                                            int(mode), _dptr(work), work.numel(), _stream(stream)))
    return x


def hbmc_spmv(m: Matrix, x, y=None, nrhs: int = 1, stream=None):
    import torch
    _vec_check(x, m.n_pad, nrhs, "x")
    if y is None:
        y = torch.empty_like(x)
    _check("hbmc_spmv", lib().hbmc_spmv(m.handle, _dptr(x), _dptr(y), nrhs, _stream(stream)))
    return y


def hbmc_to_hbmc(f: Factor, v, nrhs: int = 1, stream=None):
    import torch
    _vec_check(v, f.n, nrhs, "v")
    vb = torch.empty(f.n_pad * nrhs, dtype=torch.float64, device=v.device)
    _check("hbmc_to_hbmc", lib().hbmc_to_hbmc(f.handle, _dptr(v), _dptr(vb), nrhs, _stream(stream)))
    return vb


def hbmc_from_hbmc(f: Factor, vb, nrhs: int = 1, stream=None):
    import torch
    _vec_check(vb, f.n_pad, nrhs, "vb")
    v = torch.empty(f.n * nrhs, dtype=torch.float64, device=vb.device)
    _check("hbmc_from_hbmc", lib().hbmc_from_hbmc(f.handle, _dptr(vb), _dptr(v), nrhs, _stream(stream)))
    return v


@dataclass
class Stats:
    iters: int
    status: int
    rel_res: float
    true_rel_res: float
    x0_scale: float = 1.0


def workspace(f: Factor, nrhs: int = 1, device="cuda"):
    import torch
    b = C.c_size_t(0)
    _check("iccg_workspace_bytes", lib().iccg_workspace_bytes(f.handle, nrhs, C.byref(b)))
    return torch.empty(max(b.value, 256), dtype=torch.uint8, device=device)


def iccg_solve(f: Factor, m: Matrix, b, x=None, tol: float = 1e-7, maxit: int = 10000,
               nrhs: int = 1, x0_zero: bool | None = None, check_every: int = 0,
               use_graph: bool = True, history: bool = False, work=None, stream=None,
               x0_scale: bool = False):
    """Solves A x = b (original numbering, device FP64).  Returns (x, stats),
    or (x, stats, hist) with history=True; stats is a list (system-major,
    then right-hand side) unless there is one system and one right-hand side.
    x0_scale: start from c x with the A-norm-optimal c (0 falls back to x = 0)."""
    import torch
    _vec_check(b, f.n, nrhs, "b")
    if x is None:
        x = torch.zeros_like(b)
        if x0_zero is None:
            x0_zero = True
    _vec_check(x, f.n, nrhs, "x")
    if work is None:
        work = workspace(f, nrhs, b.device)
    opts = SolveOpts(1 if x0_zero else 0, int(check_every), 1 if use_graph else 0,
                     1 if history else 0, 1 if x0_scale else 0)
    nst = f.n_systems * nrhs
    stats = (SolveStats * nst)()
    code = lib().iccg_solve(f.handle, m.handle, _dptr(b), _dptr(x), nrhs, float(tol), int(maxit),
                            C.byref(opts), stats, _dptr(work), work.numel(), _stream(stream))
    _check("iccg_solve", code, ok=(HBMC_OK, HBMC_ENOCONV))
    out = [Stats(s.iters, s.status, s.rel_res, s.true_rel_res, s.x0_scale) for s in stats]
    if history:
        h = np.empty(out[0].iters + 1)
        _check("iccg_history", lib().iccg_history(_dptr(work), work.numel(), f.handle, _ptr(h),
                                                  len(h), _stream(stream)))
        return x, (out[0] if nst == 1 else out), h
    return x, (out[0] if nst == 1 else out)


# bytes of the library's static workspace used by iccg_solve_noalloc (per device)
NOALLOC_SCRATCH_BYTES = 64 << 20


def iccg_solve_noalloc(f: Factor, m: Matrix, b, x, tol: float = 1e-7, maxit: int = 10000,
                       nrhs: int = 1, x0_zero: bool = False, check_every: int = 0, stream=None):
    """iccg_solve with the library's static device workspace: the call itself
    allocates nothing, so x must be given (device FP64, original numbering;
    overwritten with the solution).  Returns stats as iccg_solve does."""
    _vec_check(b, f.n, nrhs, "b")
    _vec_check(x, f.n, nrhs, "x")
    opts = SolveOpts(1 if x0_zero else 0, int(check_every), 0, 0, 0)
    nst = f.n_systems * nrhs
    stats = (SolveStats * nst)()
    code = lib().iccg_solve_noalloc(f.handle, m.handle, _dptr(b), _dptr(x), nrhs, float(tol), int(maxit),
                                    C.byref(opts), stats, _stream(stream))
    _check("iccg_solve_noalloc", code, ok=(HBMC_OK, HBMC_ENOCONV))
    out = [Stats(s.iters, s.status, s.rel_res, s.true_rel_res, s.x0_scale) for s in stats]
    return out[0] if nst == 1 else out


@dataclass
class Solver:
    """Ordering, factor and matrix of one system (or of a batch of independent
    systems, with sys_ptr), uploaded to the device."""
    order: Order
    factor: Factor
    matrix: Matrix

    @staticmethod
    def setup(A, bs: int, w: int, precision: int = HBMC_F64, shift: float = 0.0,
              device="cuda", kernel: int = HBMC_KERNEL_AUTO, sys_ptr=None,
              omega: float | None = None, rcm: bool = False) -> "Solver":
        """IC(0) factor, or the SSOR splitting with relaxation omega when
        omega is given; with rcm, the ordering of the pattern renumbered by
        reverse Cuthill-McKee (one system)."""
        if sys_ptr is not None and rcm:
            raise ValueError("the renumbered ordering takes one system")
        o = hbmc_order(A, bs, w, rcm=rcm) if sys_ptr is None else hbmc_order_batch(A, sys_ptr, bs, w)
        f = ic0_factor(o, A, precision, shift) if omega is None else ssor_factor(o, A, precision, omega)
        f = f.set_kernel(kernel).upload(device)
        m = hbmc_matrix_create(o, A).upload(device)
        return Solver(o, f, m)

    def solve(self, b, x=None, **kw):
        return iccg_solve(self.factor, self.matrix, b, x, **kw)

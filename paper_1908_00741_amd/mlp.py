"""The warm-start network x0 = s * MLP(theta), 12 -> 256 -> 256 -> n, on the
kernels of include/hbmc_mlp.h.

Argument marshalling only: products, activations, loss, reductions and Adam
run in the library; PyTorch provides the device buffers and the stream.
Weights are kept as FP32 master copies with Adam moments, and as compute
copies in the compute type (BF16, or FP32 for checking).
"""
from __future__ import annotations

import ctypes as C
import math
from dataclasses import dataclass

import numpy as np

from . import hbmc

MLP_BF16, MLP_F32 = 0, 1
MLP_NN, MLP_TN, MLP_NT = 0, 1, 2

SYMBOLS = ("mlp_gemm", "mlp_linear_fwd", "mlp_linear_fwd_mse", "mlp_mse_parts", "mlp_sum_rows",
           "mlp_relu_bwd", "mlp_adam", "mlp_cast", "mlp_cast_f64", "mlp_to_f64", "mlp_gaussian_rhs",
           "mlp_combine", "mlp_workspace_bytes", "mlp_forward", "mlp_backward", "mlp_adam_step",
           "mlp_train_step")

_ready = False


def lib():
    global _ready
    L = hbmc.lib()
    if not _ready:
        P, i32, i64, f32, f64 = C.c_void_p, C.c_int32, C.c_int64, C.c_float, C.c_double
        L.mlp_gemm.argtypes = [i32, i32, i32, i32, i32, P, i64, P, i64, P, i64, i32, P]
        L.mlp_linear_fwd.argtypes = [i32, i32, i32, i32, P, P, P, i32, P, P, P]
        L.mlp_linear_fwd_mse.argtypes = [i32, i32, i32, i32, P, P, P, P, f32, P, P, P, P]
        L.mlp_mse_parts.argtypes = [i32, i32, P, P]
        L.mlp_sum_rows.argtypes = [i64, i64, P, i64, P, P]
        L.mlp_relu_bwd.argtypes = [i32, i64, P, P, P, P, P]
        L.mlp_adam.argtypes = [i32, i64, P, P, P, P, P, f32, f32, f32, f32, i32, P]
        L.mlp_cast.argtypes = [i32, i64, P, P, P]
        L.mlp_cast_f64.argtypes = [i32, i64, P, f64, P, P]
        L.mlp_to_f64.argtypes = [i64, P, f64, P, P]
        L.mlp_gaussian_rhs.argtypes = [i32, P, P, P]
        L.mlp_combine.argtypes = [i32, i32, i64, P, i64, P, P, f32, P, P]
        L.mlp_workspace_bytes.argtypes = [i32, i32, i32, i32, i32, P]
        L.mlp_forward.argtypes = [i32, i32, i32, i32, i32, P, P, P, P, P, P, C.c_size_t, P]
        L.mlp_backward.argtypes = [i32, i32, i32, i32, i32, P, P, P, P, P, P, P, C.c_size_t, P]
        L.mlp_adam_step.argtypes = [i32, i32, P, P, P, P, P, P, f32, f32, f32, f32, i32, P]
        L.mlp_train_step.argtypes = [i32, i32, i32, i32, i32, P, P, P, P, P, P, P, f32, f32, f32, f32, i32, P, P,
                                     C.c_size_t, P]
        _ready = True
    return L


def _p(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _s(stream=None):
    return hbmc._stream(stream)


def _ck(name, code):
    return hbmc._check(name, code)


def _torch_dtype(dtype):
    import torch
    return torch.int16 if dtype == MLP_BF16 else torch.float32   # BF16 held as 16-bit patterns


def gemm(dtype, layout, M, N, K, A, lda, B, ldb, Cout, ldc, nsplit=1, stream=None):
    _ck("mlp_gemm", lib().mlp_gemm(dtype, layout, M, N, K, _p(A), lda, _p(B), ldb, _p(Cout), ldc, nsplit,
                                   _s(stream)))


def sum_rows(R, N, src, ld, out, stream=None):
    _ck("mlp_sum_rows", lib().mlp_sum_rows(R, N, _p(src), ld, _p(out), _s(stream)))


def cast(dtype, src, dst, stream=None):
    _ck("mlp_cast", lib().mlp_cast(dtype, src.numel(), _p(src), _p(dst), _s(stream)))


def cast_f64(dtype, src, scale, dst, stream=None):
    _ck("mlp_cast_f64", lib().mlp_cast_f64(dtype, src.numel(), _p(src), float(scale), _p(dst), _s(stream)))


def to_f64(src, scale, dst, stream=None):
    _ck("mlp_to_f64", lib().mlp_to_f64(src.numel(), _p(src), float(scale), _p(dst), _s(stream)))


def gaussian_rhs(N, theta, b, stream=None):
    th = np.ascontiguousarray(theta, np.float64)
    assert th.size == 12
    _ck("mlp_gaussian_rhs", lib().mlp_gaussian_rhs(N, th.ctypes.data_as(C.c_void_p), _p(b), _s(stream)))


def combine(dtype, G, idx, amp, scale, out, stream=None):
    """out[m] = scale * sum_q amp[m, q] * G[idx[m, q]] for host arrays idx
    (int [M][4], values checked against G's rows here) and amp ([M][4]); G
    and out are device tensors [rows][n] and [>= M][n] in the compute type."""
    import torch
    idx = np.ascontiguousarray(idx, np.int32)
    amp = np.ascontiguousarray(amp, np.float32)
    M = idx.shape[0]
    if idx.shape != (M, 4) or amp.shape != (M, 4) or out.shape[0] < M:
        raise ValueError("idx and amp must be [M][4] and out must hold M rows")
    if idx.min() < 0 or idx.max() >= G.shape[0]:
        raise ValueError("idx out of range")
    di = torch.from_numpy(idx).to(G.device)
    da = torch.from_numpy(amp).to(G.device)
    _ck("mlp_combine", lib().mlp_combine(dtype, M, G.shape[1], _p(G), G.shape[0], _p(di), _p(da), float(scale),
                                         _p(out), _s(stream)))


@dataclass
class Adam:
    lr: float = 1e-3
    beta1: float = 0.9
    beta2: float = 0.999
    eps: float = 1e-8


class MLP:
    """Weights W1 [12][256], W2 [256][256], W3 [256][n] and biases, FP32
    master copies initialised uniform(-1/sqrt(fan_in), 1/sqrt(fan_in)) from
    seed; compute copies in dtype."""

    def __init__(self, n_out, n_in=12, hidden=256, dtype=MLP_BF16, seed=0, device="cuda"):
        import torch
        self.dims = [n_in, hidden, hidden, n_out]
        self.dtype = dtype
        self.device = torch.device(device)
        rng = np.random.default_rng(seed)
        self.master, self.comp, self.m, self.v, self.grad = [], [], [], [], []
        for k in range(3):
            fi, fo = self.dims[k], self.dims[k + 1]
            bound = 1.0 / math.sqrt(fi)
            for shape in ((fi, fo), (fo,)):
                w = torch.from_numpy(rng.uniform(-bound, bound, shape).astype(np.float32)).to(self.device)
                self.master.append(w)
                self.comp.append(torch.empty(shape, dtype=_torch_dtype(dtype), device=self.device))
                self.m.append(torch.zeros_like(w))
                self.v.append(torch.zeros_like(w))
                self.grad.append(torch.zeros_like(w))
        self.step_no = 0
        self.sync_copies()
        self._bufs = {}

    # parameters: [W1, b1, W2, b2, W3, b3]
    def set_weights(self, arrays):
        """Master weights from host arrays [W1, b1, W2, b2, W3, b3] (FP32)."""
        import torch
        for dst, a in zip(self.master, arrays):
            dst.copy_(torch.from_numpy(np.ascontiguousarray(a, np.float32)).to(dst.device))
        self.sync_copies()

    def sync_copies(self, stream=None):
        for w, c in zip(self.master, self.comp):
            cast(self.dtype, w, c, stream)

    def _buffers(self, M):
        import torch
        if M not in self._bufs:
            n_in, h, _, n = self.dims
            nb = C.c_size_t(0)
            _ck("mlp_workspace_bytes", lib().mlp_workspace_bytes(self.dtype, M, n_in, h, n, C.byref(nb)))
            self._bufs[M] = dict(
                x=torch.empty((M, n_in), dtype=_torch_dtype(self.dtype), device=self.device),
                work=torch.empty(max(nb.value, 256), dtype=torch.uint8, device=self.device),
                loss=torch.empty(1, dtype=torch.float32, device=self.device))
        return self._bufs[M]

    def _ptrs(self):
        W = (C.c_void_p * 3)(*[t.data_ptr() for t in self.comp[0::2]])
        b = (C.c_void_p * 3)(*[t.data_ptr() for t in self.master[1::2]])
        return W, b

    def load_input(self, theta, stream=None):
        """theta: FP32 device tensor [M][12] -> the compute-type input."""
        B = self._buffers(theta.shape[0])
        cast(self.dtype, theta.contiguous(), B["x"], stream)
        return B

    def forward(self, theta, stream=None):
        """FP32 output [M][n] of the network for FP32 inputs theta [M][12]."""
        import torch
        M = theta.shape[0]
        B = self.load_input(theta, stream)
        n_in, h, _, n = self.dims
        if "yf" not in B:
            B["yf"] = torch.empty((M, n), dtype=torch.float32, device=self.device)
        W, b = self._ptrs()
        _ck("mlp_forward", lib().mlp_forward(self.dtype, M, n_in, h, n, _p(B["x"]), W, b, None, _p(B["yf"]),
                                             _p(B["work"]), B["work"].numel(), _s(stream)))
        return B["yf"]

    def loss_and_grads(self, theta, target, stream=None):
        """Mean squared error against target (compute type [M][n]) and the
        gradients of every parameter into self.grad.  Returns a device
        tensor holding M n times the loss."""
        M = theta.shape[0]
        B = self.load_input(theta, stream)
        n_in, h, _, n = self.dims
        W, b = self._ptrs()
        g = (C.c_void_p * 6)(*[t.data_ptr() for t in self.grad])
        _ck("mlp_backward", lib().mlp_backward(self.dtype, M, n_in, h, n, _p(B["x"]), _p(target), W, b, g,
                                               _p(B["loss"]), _p(B["work"]), B["work"].numel(), _s(stream)))
        return B["loss"]

    def adam_step(self, opt: Adam, stream=None):
        step = self.step_no + 1   # counted once the call is accepted
        k = len(self.master)
        arr = lambda ts: (C.c_void_p * k)(*[t.data_ptr() for t in ts])
        sizes = (C.c_int64 * k)(*[t.numel() for t in self.master])
        _ck("mlp_adam_step", lib().mlp_adam_step(self.dtype, k, sizes, arr(self.master), arr(self.m), arr(self.v),
                                                 arr(self.grad), arr(self.comp), opt.lr, opt.beta1, opt.beta2,
                                                 opt.eps, step, _s(stream)))
        self.step_no = step

    def train_step(self, theta, target, opt: Adam, stream=None):
        """loss_and_grads then adam_step in one call, with the output layer's
        update applied in its weight-gradient product (self.grad[4] is not
        written).  Returns the loss tensor of loss_and_grads."""
        M = theta.shape[0]
        B = self.load_input(theta, stream)
        n_in, h, _, n = self.dims
        step = self.step_no + 1   # counted once the call is accepted
        arr = lambda ts: (C.c_void_p * 6)(*[t.data_ptr() for t in ts])
        _ck("mlp_train_step", lib().mlp_train_step(self.dtype, M, n_in, h, n, _p(B["x"]), _p(target),
                                                   arr(self.master), arr(self.m), arr(self.v), arr(self.grad),
                                                   arr(self.comp), opt.lr, opt.beta1, opt.beta2, opt.eps,
                                                   step, _p(B["loss"]), _p(B["work"]), B["work"].numel(),
                                                   _s(stream)))
        self.step_no = step
        return B["loss"]

    def state(self):
        """Host copies of the master weights, moments and step (checkpoint)."""
        return {"master": [w.cpu() for w in self.master], "m": [t.cpu() for t in self.m],
                "v": [t.cpu() for t in self.v], "step": self.step_no, "dims": self.dims, "dtype": self.dtype}

    def load_state(self, st):
        for dst, src in zip(self.master + self.m + self.v, st["master"] + st["m"] + st["v"]):
            dst.copy_(src.to(dst.device))
        self.step_no = int(st["step"])
        self.sync_copies()

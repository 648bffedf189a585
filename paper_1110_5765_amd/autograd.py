"""Differentiable linear layer through the throughput-distortion GEMM.

TDLinearFn computes Y = X W (+ b) forward and, backward, dX = dY W^T and
dW = X^T dY, each product through tdgemm_plan + the fused tdgemm_gemm of the
library (transposed operands are passed as views, so the library reads them
in place). Rounding is treated as straight-through: the backward products are
the packed products of the incoming gradient, not derivatives of the rounding.
This is how the paper accelerates the back-propagation products of its
metadata-learning perceptron (Sec. 8.B). With prec "i8" or "e4m3" the three
products run in the block-scaled form instead (Remark 1: the same rounded
integer operands on the INT8 / FP8 matrix cores, per-block scales).

Only argument marshalling happens here; every arithmetic step of the method
runs in the library's HIP kernels. The bias gradient is a plain column sum.
"""
from __future__ import annotations

import dataclasses

import torch

from . import tdgemm as td


@dataclasses.dataclass
class TDConfig:
    """Settings of every product of a layer (see make_desc). prec "i8" / "e4m3": the
    block-scaled form with separable block scales of range sep_q (L = 128; the
    other control settings do not apply)."""
    L: int = 64
    form: str = "sym"
    prec: str = "f32"
    ctrl: str = "snr"
    snr_db: float = 30.0
    w_allowed: tuple = (1, 2)
    fixed_w: int = 2
    fixed_rmax: float = float(2 ** 20)
    sep_q: float = 127.0
    min_dim: int = 128          # products with a smaller M, N or K stay plain (torch)
    k_split: int | None = None  # groups of the l-sum per product; None: auto_k_split


class TDContext:
    """Calibration table and cached workspaces shared by the products of a model."""

    def __init__(self, cfg: TDConfig, calib: td.DeviceCalib | None):
        self.cfg = cfg
        self.calib = calib
        self._ws: dict = {}
        self._prep: dict = {}
        self._views: dict = {}
        self.calls = 0
        self.plain_calls = 0
        self.last_plan = None

    def workspace(self, need: int, device) -> torch.Tensor:
        """The shared device workspace, grown on demand to `need` bytes."""
        ws = self._ws.get(device)
        if ws is None or ws.numel() < need:
            ws = torch.empty(need, dtype=torch.uint8, device=device)
            self._ws[device] = ws
        return ws

    def prepared(self, A: torch.Tensor, B: torch.Tensor):
        """(descriptor, workspace bytes, byte-operand shapes or None) of a product,
        built once per operand shape, strides and dtype (a training loop repeats
        the same few products every step)."""
        key = (tuple(A.shape), A.stride(), tuple(B.shape), B.stride(), A.dtype, B.dtype)
        p = self._prep.get(key)
        if p is None:
            c = self.cfg
            M, K = A.shape
            N = B.shape[1]
            shapes = None
            if c.prec in ("i8", "e4m3"):
                desc = td.make_desc(A, B, L=128, prec=c.prec, ctrl="separable", fixed_w=1, sep_q=c.sep_q)
                nI, nL, nJ = -(-M // 128), -(-K // 128), -(-N // 128)
                shapes = {"qA": (nI * 128, nL * 128), "qB": (nJ * 128, nL * 128)}
            else:
                ks = td.auto_k_split(M, N, K, c.L, c.prec) if c.k_split is None else c.k_split
                desc = td.make_desc(A, B, L=c.L, form=c.form, prec=c.prec, ctrl=c.ctrl, snr_db=c.snr_db,
                                    w_allowed=c.w_allowed, fixed_w=c.fixed_w, fixed_rmax=c.fixed_rmax,
                                    sep_q=c.sep_q, k_split=ks)
            p = (desc, max(td.tdgemm_workspace_size(desc), 256), shapes)
            self._prep[key] = p
        return p

    def byte_operands(self, shapes: dict, device) -> tuple[torch.Tensor, torch.Tensor]:
        """Cached byte operand buffers of the block-scaled forms (grown on demand),
        and their views per operand shape (a training step asks for the same few)."""
        vk = (device, shapes["qA"], shapes["qB"])
        v = self._views.get(vk)
        if v is not None:
            return v
        key = ("bytes", device)
        need = shapes["qA"][0] * shapes["qA"][1] + shapes["qB"][0] * shapes["qB"][1]
        buf = self._ws.get(key)
        if buf is None or buf.numel() < need:
            buf = torch.empty(need, dtype=torch.uint8, device=device)
            self._ws[key] = buf
            self._views = {}                      # views of the former buffer
        na = shapes["qA"][0] * shapes["qA"][1]
        v = (buf[:na].view(shapes["qA"]), buf[na:need].view(shapes["qB"]))
        self._views[vk] = v
        return v

    def matmul(self, A: torch.Tensor, B: torch.Tensor) -> torch.Tensor:
        """A B through the library (A, B row-major or transposed views)."""
        c = self.cfg
        M, K = A.shape
        N = B.shape[1]
        if min(M, N, K) < c.min_dim:
            self.plain_calls += 1
            return A @ B
        desc, need, shapes = self.prepared(A, B)
        ws = self.workspace(need, A.device)
        st = torch.cuda.current_stream(A.device)
        if shapes is not None:
            # block-scaled form (Remark 1): separable block scales, byte operands,
            # INT8 / FP8 matrix cores, float32 C
            plan = td.tdgemm_plan(desc, A, B, None, ws, stream=st)
            qA, qB = self.byte_operands(shapes, A.device)
            out = torch.empty((M, N), dtype=torch.float32, device=A.device)
            td.tdgemm_compand(plan, A, B, qA, qB, stream=st)
            td.tdgemm_gemm(plan, qA, qB, out, fused=1, stream=st)
            self.calls += 1
            self.last_plan = plan
            return out
        plan = td.tdgemm_plan(desc, A, B, self.calib if c.ctrl in ("snr", "accel", "target") else None, ws,
                              stream=st)
        out = torch.empty((M, N), dtype=td.torch_dtype(desc.prec), device=A.device)
        td.tdgemm_gemm(plan, A, B, out, fused=1, stream=st)
        self.calls += 1
        self.last_plan = plan
        return out


class TDLinearFn(torch.autograd.Function):
    """Y = X W + b with packed products forward and backward (straight-through)."""

    @staticmethod
    def forward(ctx, X, W, b, tdc: TDContext):
        ctx.tdc = tdc
        ctx.has_bias = b is not None
        ctx.save_for_backward(X, W)
        Y = tdc.matmul(X, W)
        if b is not None:
            Y = Y + b
        return Y

    @staticmethod
    def backward(ctx, dY):
        X, W = ctx.saved_tensors
        tdc = ctx.tdc
        dY = dY.contiguous()
        dX = tdc.matmul(dY, W.t()) if ctx.needs_input_grad[0] else None
        dW = tdc.matmul(X.t(), dY) if ctx.needs_input_grad[1] else None
        db = dY.sum(0) if ctx.has_bias and ctx.needs_input_grad[2] else None
        return dX, dW, db, None


class TDLinear(torch.nn.Module):
    """Linear layer y = x W + b (W stored in_features x out_features)."""

    def __init__(self, W: torch.Tensor, b: torch.Tensor | None, tdc: TDContext):
        super().__init__()
        self.weight = torch.nn.Parameter(W)
        self.bias = torch.nn.Parameter(b) if b is not None else None
        self.tdc = tdc

    def forward(self, x):
        return TDLinearFn.apply(x, self.weight, self.bias, self.tdc)


def calibrate(L: int, form: str, prec: str, ws=(2,), device="cuda") -> td.DeviceCalib:
    """s(R, W) measured on the GPU path (Sec. 4.B) for the given W values."""
    from .calib import device_table
    return device_table(L, form, prec, ws, device)[0]

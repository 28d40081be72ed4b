"""The learned energy sampler's network on the GPU: binding of the kernels declared in
``include/knit_mlp.h`` and the layer loop that sequences them.

Every arithmetic operation (GEMMs, activations, softmax cross-entropy, bias
gradients, AdamW) runs in the HIP kernels of ``libknit.so``; this module holds
the parameter buffers and issues the calls in order:

    forward:   X0 = bf16(x);  Z_l = X_{l-1} W_l^T + b_l;  X_l = bf16(gelu(Z_l));  logits = Z_n
    loss:      mean cross-entropy of softmax(logits) against target densities q
    backward:  dZ_n = bf16((p - q) / B);  dW_l = dZ_l^T X_{l-1};  db_l = sum_b dZ_l;
               dX_{l-1} = dZ_l W_l;  dZ_{l-1} = bf16(dX_{l-1} gelu'(Z_{l-1}))
    update:    AdamW on FP32 master weights, BF16 copies for the next forward
"""

from __future__ import annotations

import ctypes
from dataclasses import dataclass, field

import numpy as np
import torch

from . import knit as K

_lib = K._lib
c_i32, c_i64, c_f32, c_vp = ctypes.c_int32, ctypes.c_int64, ctypes.c_float, ctypes.c_void_p

_lib.knit_mlp_gemm.restype = c_i32
_lib.knit_mlp_gemm.argtypes = [c_i32, c_i32, c_i32, c_vp, c_i64, c_i64, c_vp, c_i64, c_i64, c_vp, c_f32, c_vp,
                               c_i64, c_vp]
_lib.knit_mlp_act_fwd.restype = c_i32
_lib.knit_mlp_act_fwd.argtypes = [c_i64, c_vp, c_vp, c_i32, c_vp]
_lib.knit_mlp_gelu_bwd.restype = c_i32
_lib.knit_mlp_gelu_bwd.argtypes = [c_i64, c_vp, c_vp, c_vp, c_vp]
_lib.knit_mlp_softmax_xent.restype = c_i32
_lib.knit_mlp_softmax_xent.argtypes = [c_i32, c_i32, c_vp, c_vp, c_f32, c_vp, c_vp, c_vp, c_vp]
_lib.knit_mlp_colsum.restype = c_i32
_lib.knit_mlp_colsum.argtypes = [c_i32, c_i32, c_vp, c_vp, c_vp]
_lib.knit_mlp_adamw.restype = c_i32
_lib.knit_mlp_adamw.argtypes = [c_i64, c_vp, c_vp, c_vp, c_vp, c_vp, c_f32, c_f32, c_f32, c_f32, c_f32, c_i32,
                                c_vp]

EXPORTED = ["knit_mlp_gemm", "knit_mlp_act_fwd", "knit_mlp_gelu_bwd", "knit_mlp_softmax_xent", "knit_mlp_colsum",
            "knit_mlp_adamw"]


def _p(t):
    return K._ptr(t)


def _s(stream):
    return K._stream(stream)


def knit_mlp_gemm(M, N, K_, A, sam, sak, B, sbn, sbk, C, ldc, bias=None, beta=0.0, stream=None):
    K._check(_lib.knit_mlp_gemm(int(M), int(N), int(K_), _p(A), int(sam), int(sak), _p(B), int(sbn), int(sbk),
                                _p(bias), float(beta), _p(C), int(ldc), _s(stream)), "knit_mlp_gemm")


def knit_mlp_act_fwd(Z, Y, gelu=True, stream=None):
    assert Z.dtype == torch.float32 and Y.dtype == torch.bfloat16 and Z.numel() == Y.numel()
    K._check(_lib.knit_mlp_act_fwd(Z.numel(), _p(Z), _p(Y), int(bool(gelu)), _s(stream)), "knit_mlp_act_fwd")


def knit_mlp_gelu_bwd(dY, Z, dZ, stream=None):
    assert dY.dtype == torch.float32 and Z.dtype == torch.float32 and dZ.dtype == torch.bfloat16
    K._check(_lib.knit_mlp_gelu_bwd(dY.numel(), _p(dY), _p(Z), _p(dZ), _s(stream)), "knit_mlp_gelu_bwd")


def knit_mlp_softmax_xent(logits, q=None, scale=1.0, loss=None, probs=None, dlogits=None, stream=None):
    B, C = logits.shape
    K._check(_lib.knit_mlp_softmax_xent(B, C, _p(logits), _p(q), float(scale), _p(loss), _p(probs), _p(dlogits),
                                        _s(stream)), "knit_mlp_softmax_xent")


def knit_mlp_colsum(X, out, stream=None):
    R, N = X.shape
    K._check(_lib.knit_mlp_colsum(R, N, _p(X), _p(out), _s(stream)), "knit_mlp_colsum")


def knit_mlp_adamw(w, w16, g, m, v, lr, b1, b2, eps, wd, t, stream=None):
    K._check(_lib.knit_mlp_adamw(w.numel(), _p(w), _p(w16), _p(g), _p(m), _p(v), float(lr), float(b1), float(b2),
                                 float(eps), float(wd), int(t), _s(stream)), "knit_mlp_adamw")


@dataclass
class Network:
    """Linear layers sizes[0] -> sizes[1] -> ... -> sizes[-1], GELU between, softmax output."""
    sizes: list
    device: str = "cuda"
    seed: int = 0
    W: list = field(default_factory=list)      # FP32 master weights [out, in]
    b: list = field(default_factory=list)      # FP32 biases [out]
    W16: list = field(default_factory=list)    # BF16 copies used by the kernels
    mW: list = field(default_factory=list)
    vW: list = field(default_factory=list)
    mb: list = field(default_factory=list)
    vb: list = field(default_factory=list)
    step: int = 0

    def __post_init__(self):
        rng = np.random.Generator(np.random.PCG64(self.seed))
        for fi, fo in zip(self.sizes[:-1], self.sizes[1:]):
            w = rng.normal(0.0, 1.0 / np.sqrt(fi), size=(fo, fi)).astype(np.float32)
            self.W.append(torch.from_numpy(w).to(self.device))
            self.b.append(torch.zeros(fo, dtype=torch.float32, device=self.device))
            self.W16.append(torch.empty((fo, fi), dtype=torch.bfloat16, device=self.device))
            self.mW.append(torch.zeros_like(self.W[-1]))
            self.vW.append(torch.zeros_like(self.W[-1]))
            self.mb.append(torch.zeros_like(self.b[-1]))
            self.vb.append(torch.zeros_like(self.b[-1]))
        self.sync_bf16()

    def params_numpy(self):
        return [(W.cpu().numpy(), b.cpu().numpy()) for W, b in zip(self.W, self.b)]

    def load_numpy(self, params):
        for li, (w, bb) in enumerate(params):
            self.W[li].copy_(torch.from_numpy(np.asarray(w, np.float32)))
            self.b[li].copy_(torch.from_numpy(np.asarray(bb, np.float32)))
        self.sync_bf16()

    def sync_bf16(self):
        """BF16 copies from the master weights (the kernels' rounding cast)."""
        for li in range(len(self.W)):
            knit_mlp_act_fwd(self.W[li], self.W16[li], gelu=False)

    def forward(self, x: torch.Tensor, stream=None):
        """x: FP32 [B, sizes[0]] on the device.  Returns (logits FP32, cache)."""
        B = x.shape[0]
        X0 = torch.empty(x.shape, dtype=torch.bfloat16, device=self.device)
        knit_mlp_act_fwd(x.contiguous(), X0, gelu=False, stream=stream)
        Xs, Zs = [X0], []
        n = len(self.W)
        for li in range(n):
            fo, fi = self.W[li].shape
            Z = torch.empty((B, fo), dtype=torch.float32, device=self.device)
            knit_mlp_gemm(B, fo, fi, Xs[-1], fi, 1, self.W16[li], fi, 1, Z, fo, bias=self.b[li], stream=stream)
            Zs.append(Z)
            if li < n - 1:
                Y = torch.empty((B, fo), dtype=torch.bfloat16, device=self.device)
                knit_mlp_act_fwd(Z, Y, gelu=True, stream=stream)
                Xs.append(Y)
        return Zs[-1], {"X": Xs, "Z": Zs}

    def loss_and_grads(self, x, q, stream=None):
        """Mean cross-entropy against q [B, C] and the gradients [(dW, db)] (FP32)."""
        logits, cache = self.forward(x, stream)
        B, C = logits.shape
        loss = torch.empty(B, dtype=torch.float32, device=self.device)
        dZ = torch.empty((B, C), dtype=torch.bfloat16, device=self.device)
        knit_mlp_softmax_xent(logits, q.contiguous(), 1.0 / B, loss=loss, dlogits=dZ, stream=stream)
        grads = [None] * len(self.W)
        for li in range(len(self.W) - 1, -1, -1):
            fo, fi = self.W[li].shape
            Xin = cache["X"][li]
            dW = torch.empty((fo, fi), dtype=torch.float32, device=self.device)
            # dW[o, i] = sum_b dZ[b, o] X[b, i]
            knit_mlp_gemm(fo, fi, B, dZ, 1, fo, Xin, 1, fi, dW, fi, stream=stream)
            db = torch.empty(fo, dtype=torch.float32, device=self.device)
            knit_mlp_colsum(dZ, db, stream=stream)
            grads[li] = (dW, db)
            if li > 0:
                # dX[b, i] = sum_o dZ[b, o] W[o, i]
                dX = torch.empty((B, fi), dtype=torch.float32, device=self.device)
                knit_mlp_gemm(B, fi, fo, dZ, fo, 1, self.W16[li], 1, fi, dX, fi, stream=stream)
                dZn = torch.empty((B, fi), dtype=torch.bfloat16, device=self.device)
                knit_mlp_gelu_bwd(dX, cache["Z"][li - 1], dZn, stream=stream)
                dZ = dZn
        return loss, grads

    def adamw_step(self, grads, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8, wd=1e-4, stream=None):
        self.step += 1
        for li, (dW, db) in enumerate(grads):
            knit_mlp_adamw(self.W[li], self.W16[li], dW, self.mW[li], self.vW[li], lr, b1, b2, eps, wd, self.step,
                           stream)
            knit_mlp_adamw(self.b[li], None, db, self.mb[li], self.vb[li], lr, b1, b2, eps, 0.0, self.step, stream)

    def probs(self, x, stream=None):
        logits, _ = self.forward(x, stream)
        p = torch.empty_like(logits)
        knit_mlp_softmax_xent(logits, None, 1.0, probs=p, stream=stream)
        return p

"""The predictor's network on the GPU: every product, activation, loss and
update runs in the HIP kernels of include/hdc_mlp.h; torch supplies the
device buffers only.

Network (a classifier, section 6.3): d_in -> [128 relu] x 3 -> K logits,
softmax cross-entropy, Adam.
"""
from __future__ import annotations

import ctypes
from typing import List, Optional, Sequence

import numpy as np

_F = ctypes.c_void_p
_I = ctypes.c_int64

SIGNATURES = {
    "hdc_mlp_linear_forward": [_F, _F, _F, _F, _I, _I, _I, ctypes.c_int, _F],
    "hdc_mlp_linear_backward": [_F, _F, _F, _F, _F, _F, _I, _I, _I, _F],
    "hdc_mlp_relu_backward": [_F, _F, _I, _F],
    "hdc_mlp_softmax_xent": [_F, _F, _F, _F, _F, _I, _I, _F],
    "hdc_mlp_softmax_xent_soft": [_F, _F, _F, _F, _F, _I, _I, _F],
    "hdc_mlp_adam": [_F, _F, _F, _F, _I, ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_float, _I, _F],
}


def bind(L):
    for name, args in SIGNATURES.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int


def _p(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def he_init(sizes: Sequence[int], seed: int = 0):
    """He-normal weights and zero biases (float64 host arrays), drawn from a seeded PCG64."""
    r = np.random.Generator(np.random.PCG64(np.random.SeedSequence([230610016, 77, int(seed)])))
    out = []
    for i in range(len(sizes) - 1):
        out.append((r.normal(0.0, np.sqrt(2.0 / sizes[i]), (sizes[i + 1], sizes[i])), np.zeros(sizes[i + 1])))
    return out


class MLP:
    def __init__(self, sizes: Sequence[int], params=None, seed: int = 0, device: str = "cuda"):
        import torch
        from ._lib import lib, check
        self._lib = lib()
        self._check = check
        self.sizes = list(sizes)
        self.device = device
        params = params if params is not None else he_init(sizes, seed)
        f32 = dict(dtype=torch.float32, device=device)
        self.W = [torch.tensor(np.asarray(W), **f32).contiguous() for W, _ in params]
        self.b = [torch.tensor(np.asarray(b), **f32).contiguous() for _, b in params]
        self.mW = [torch.zeros_like(w) for w in self.W]
        self.vW = [torch.zeros_like(w) for w in self.W]
        self.mb = [torch.zeros_like(b) for b in self.b]
        self.vb = [torch.zeros_like(b) for b in self.b]
        self.t = 0

    def _stream(self):
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)

    def forward(self, X):
        """Logits and the list of layer inputs [X, a_1, ..., a_{L-1}]."""
        import torch
        acts = [X]
        a = X
        s = self._stream()
        B = X.shape[0]
        for li, (W, b) in enumerate(zip(self.W, self.b)):
            out = torch.empty((B, W.shape[0]), dtype=torch.float32, device=self.device)
            relu = 1 if li < len(self.W) - 1 else 0
            self._check(self._lib.hdc_mlp_linear_forward(_p(a), _p(W), _p(b), _p(out), B, W.shape[1], W.shape[0],
                                                         relu, s))
            if relu:
                acts.append(out)
            a = out
        return a, acts

    def probs(self, X):
        import torch
        Z, _ = self.forward(X)
        P = torch.empty_like(Z)
        self._check(self._lib.hdc_mlp_softmax_xent(_p(Z), None, _p(P), None, None, Z.shape[0], Z.shape[1],
                                                   self._stream()))
        return P

    def gradients(self, X, y=None, T=None):
        """(loss tensor[1], [(dW, db)]) of the mean cross-entropy against labels y (int32)
        or target distributions T (float32, B x K), all on the device."""
        import torch
        Z, acts = self.forward(X)
        B, K = Z.shape
        s = self._stream()
        P = torch.empty_like(Z)
        dZ = torch.empty_like(Z)
        loss = torch.empty(1, dtype=torch.float32, device=self.device)
        if T is not None:
            self._check(self._lib.hdc_mlp_softmax_xent_soft(_p(Z), _p(T), _p(P), _p(dZ), _p(loss), B, K, s))
        else:
            self._check(self._lib.hdc_mlp_softmax_xent(_p(Z), _p(y), _p(P), _p(dZ), _p(loss), B, K, s))
        grads: List = [None] * len(self.W)
        d = dZ
        for li in range(len(self.W) - 1, -1, -1):
            W = self.W[li]
            dW = torch.empty_like(W)
            db = torch.empty_like(self.b[li])
            dX = torch.empty((B, W.shape[1]), dtype=torch.float32, device=self.device) if li > 0 else None
            self._check(self._lib.hdc_mlp_linear_backward(_p(acts[li]), _p(W), _p(d), _p(dX), _p(dW), _p(db),
                                                          B, W.shape[1], W.shape[0], s))
            grads[li] = (dW, db)
            if li > 0:
                self._check(self._lib.hdc_mlp_relu_backward(_p(dX), _p(acts[li]), dX.numel(), s))
                d = dX
        return loss, grads

    def adam(self, grads, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        self.t += 1
        s = self._stream()
        for li, (dW, db) in enumerate(grads):
            for P, G, M, V in ((self.W[li], dW, self.mW[li], self.vW[li]), (self.b[li], db, self.mb[li], self.vb[li])):
                self._check(self._lib.hdc_mlp_adam(_p(P), _p(G), _p(M), _p(V), P.numel(), lr, b1, b2, eps, self.t, s))

    def train(self, X, y, epochs: int = 200, batch: int = 256, lr: float = 1e-3, seed: int = 0,
              log_every: int = 0, soft: bool = False) -> List[float]:
        """Mini-batch Adam over host arrays X (n x d) and integer labels y (n,), or target
        distributions y (n x K) when soft; every batch is shuffled on the host and
        uploaded.  Returns the mean loss of each epoch."""
        import torch
        X = np.ascontiguousarray(X, np.float32)
        y = np.ascontiguousarray(y, np.float32 if soft else np.int32)
        n = X.shape[0]
        r = np.random.Generator(np.random.PCG64(seed))
        hist = []
        for ep in range(epochs):
            order = r.permutation(n)
            losses = []
            for i in range(0, n, batch):
                idx = order[i:i + batch]
                xb = torch.from_numpy(X[idx]).to(self.device)
                yb = torch.from_numpy(y[idx]).to(self.device)
                loss, g = self.gradients(xb, T=yb) if soft else self.gradients(xb, yb)
                self.adam(g, lr=lr)
                losses.append(loss)
            hist.append(float(np.mean([float(v) for v in losses])))
            if log_every and ep % log_every == 0:
                print(f"[mlp] epoch {ep} loss {hist[-1]:.4f}", flush=True)
        return hist

    def predict_proba(self, X) -> np.ndarray:
        import torch
        xt = torch.from_numpy(np.ascontiguousarray(X, np.float32)).to(self.device)
        return self.probs(xt).cpu().numpy()

    def host_params(self):
        return [(W.cpu().numpy().astype(np.float64), b.cpu().numpy().astype(np.float64)) for W, b in zip(self.W, self.b)]

"""Adam through the library's pinn_adam_step: one launch updates every
parameter tensor of a network in place (the optimizer of the paper's training
runs).  Marshalling only; the arithmetic is the HIP kernel's."""
from __future__ import annotations

import ctypes
from typing import Sequence, Tuple

import torch

from ._lib import Adam as _AdamHP, check, lib, ptr_array


def _stream() -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


class AdamState:
    """Moments for a list of (W, b) device tensors; step(grads) applies one
    Adam step to the parameters in place, on the current stream."""

    def __init__(self, params: Sequence[Tuple[torch.Tensor, torch.Tensor]], lr: float = 1e-3,
                 betas: Tuple[float, float] = (0.9, 0.999), eps: float = 1e-8):
        self.params = list(params)
        self.hp = _AdamHP(float(lr), float(betas[0]), float(betas[1]), float(eps))
        self.m = [(torch.zeros_like(W), torch.zeros_like(b)) for W, b in self.params]
        self.v = [(torch.zeros_like(W), torch.zeros_like(b)) for W, b in self.params]
        self.t = 0
        dims = [int(self.params[0][0].shape[1])] + [int(W.shape[0]) for W, _ in self.params]
        self._dims = (ctypes.c_int32 * len(dims))(*dims)
        self._W = ptr_array([W.data_ptr() for W, _ in self.params])
        self._b = ptr_array([b.data_ptr() for _, b in self.params])
        self._mW = ptr_array([m.data_ptr() for m, _ in self.m])
        self._mb = ptr_array([m.data_ptr() for _, m in self.m])
        self._vW = ptr_array([v.data_ptr() for v, _ in self.v])
        self._vb = ptr_array([v.data_ptr() for _, v in self.v])

    def step(self, grads: Sequence[Tuple[torch.Tensor, torch.Tensor]]) -> None:
        self.t += 1
        key = tuple((g.data_ptr(), h.data_ptr()) for g, h in grads)
        if getattr(self, "_gkey", None) != key:  # pointer arrays of the gradient tensors, reused while unchanged
            self._gkey = key
            self._dW = ptr_array([g for g, _ in key])
            self._db = ptr_array([h for _, h in key])
        check(lib.pinn_adam_step(len(self.params), ctypes.cast(self._dims, ctypes.POINTER(ctypes.c_int32)),
                                 self._W[0], self._b[0], self._dW[0], self._db[0], self._mW[0], self._vW[0],
                                 self._mb[0], self._vb[0], self.t, ctypes.byref(self.hp), _stream()))

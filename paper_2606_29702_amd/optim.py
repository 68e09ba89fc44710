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


def chain_runs(shapes):
    """Splits a list of weight shapes (out, in) into runs of consecutive layers
    that form a chain (each layer's input width is the previous layer's output
    width): pinn_adam_step takes the sizes of a chain as one dims array.  A
    plain MLP is one run; the modified MLP (two encoders, then the chain from
    the embedding) is three."""
    runs, start = [], 0
    for l in range(1, len(shapes)):
        if shapes[l][1] != shapes[l - 1][0]:
            runs.append((start, l))
            start = l
    runs.append((start, len(shapes)))
    return runs


class AdamState:
    """Moments for a list of (W, b) device tensors; step(grads) applies one
    Adam step to the parameters in place, on the current stream (one launch
    per chain of layers, see chain_runs)."""

    def __init__(self, params: Sequence[Tuple[torch.Tensor, torch.Tensor]], lr: float = 1e-3,
                 betas: Tuple[float, float] = (0.9, 0.999), eps: float = 1e-8):
        self.params = list(params)
        for l, (W, b) in enumerate(self.params):
            if W.dim() != 2 or tuple(b.shape) != (W.shape[0],):
                raise ValueError(f"layer {l}: W {tuple(W.shape)} and b {tuple(b.shape)} do not form a layer")
        self.hp = _AdamHP(float(lr), float(betas[0]), float(betas[1]), float(eps))
        self.m = [(torch.zeros_like(W), torch.zeros_like(b)) for W, b in self.params]
        self.v = [(torch.zeros_like(W), torch.zeros_like(b)) for W, b in self.params]
        self.t = 0
        self.shapes = [tuple(int(v) for v in W.shape) for W, _ in self.params]
        self.runs = []
        for a, e in chain_runs(self.shapes):
            dims = [self.shapes[a][1]] + [self.shapes[l][0] for l in range(a, e)]
            run = {"a": a, "e": e, "dims": (ctypes.c_int32 * len(dims))(*dims)}
            for key, seq in (("W", [W for W, _ in self.params]), ("b", [b for _, b in self.params]),
                             ("mW", [m for m, _ in self.m]), ("mb", [m for _, m in self.m]),
                             ("vW", [v for v, _ in self.v]), ("vb", [v for _, v in self.v])):
                run[key] = ptr_array([t.data_ptr() for t in seq[a:e]])
            self.runs.append(run)

    def step(self, grads: Sequence[Tuple[torch.Tensor, torch.Tensor]]) -> None:
        if len(grads) != len(self.params):
            raise ValueError(f"{len(grads)} gradient pairs for {len(self.params)} layers")
        for l, ((g, h), (W, b)) in enumerate(zip(grads, self.params)):
            if g.shape != W.shape or h.shape != b.shape:
                raise ValueError(f"layer {l}: gradient shapes differ from the parameters'")
        self.t += 1
        key = tuple((g.data_ptr(), h.data_ptr()) for g, h in grads)
        if getattr(self, "_gkey", None) != key:  # pointer arrays of the gradient tensors, reused while unchanged
            self._gkey = key
            for run in self.runs:
                run["dW"] = ptr_array([g for g, _ in key[run["a"]:run["e"]]])
                run["db"] = ptr_array([h for _, h in key[run["a"]:run["e"]]])
        for run in self.runs:
            check(lib.pinn_adam_step(run["e"] - run["a"], ctypes.cast(run["dims"], ctypes.POINTER(ctypes.c_int32)),
                                     run["W"][0], run["b"][0], run["dW"][0], run["db"][0], run["mW"][0],
                                     run["vW"][0], run["mb"][0], run["vb"][0], self.t, ctypes.byref(self.hp),
                                     _stream()))

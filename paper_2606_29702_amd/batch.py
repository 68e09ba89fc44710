"""Ensembles of independent partial-jet PINNs stepped together (C ABI
pinn_batch_*): one plan per network; every phase of the step is one grouped
launch over all networks at that phase (each on its own grid), networks of
one width share a stream, and the whole step (optionally with the Adam
update) is captured once into a HIP graph and replayed.

Gradient and loss buffers are owned by the batch object and reused across
steps, so that repeated steps with the same parameter and point tensors
replay the captured graph.
"""
from __future__ import annotations

import ctypes
from typing import List, Optional, Sequence, Tuple

import torch

from . import _lib
from ._lib import Adam as _AdamHP, KINDS, PRECISIONS, Net, Pde, Tuning, check, lib, ptr_array
from .jet import DEFAULT_COEF, _check_tensor, _stream


class PinnBatch:
    def __init__(self, dims: Sequence[Sequence[int]], pde: str, coefs: Sequence[Sequence[float]],
                 max_points: Sequence[int], precision: str = "bf16", device: str = "cuda"):
        self.n = len(dims)
        assert len(coefs) == self.n and len(max_points) == self.n
        self.dims = [list(d) for d in dims]
        self.pde = pde
        self.coefs = [tuple(c) for c in coefs]
        self.device = device
        keep = []
        nets = (Net * self.n)()
        for i, d in enumerate(self.dims):
            da = (ctypes.c_int32 * len(d))(*d)
            Wp, wa = ptr_array([1] * (len(d) - 1))
            bp, ba = ptr_array([1] * (len(d) - 1))
            keep += [da, wa, ba]
            nets[i] = Net(len(d) - 1, ctypes.cast(da, ctypes.POINTER(ctypes.c_int32)), Wp, bp)
        self._pdes = self._make_pdes()
        mp = (ctypes.c_int64 * self.n)(*[int(m) for m in max_points])
        h = ctypes.c_void_p()
        check(lib.pinn_batch_create(self.n, nets, self._pdes, mp, PRECISIONS[precision], 0, ctypes.byref(h)))
        self.handle = h
        self.loss = torch.zeros(self.n, device=device, dtype=torch.float32)
        self.grads: Optional[List[List[Tuple[torch.Tensor, torch.Tensor]]]] = None
        self._args = None
        self._args_key = None

    def _make_pdes(self):
        pdes = (Pde * self.n)()
        for i, c in enumerate(self.coefs):
            pdes[i].kind = KINDS[self.pde]
            for q, v in enumerate(c):
                pdes[i].coef[q] = float(v)
        return pdes

    def close(self) -> None:
        if getattr(self, "handle", None):
            check(lib.pinn_batch_destroy(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def configure(self, n_streams: int, use_graph: bool = True, per_network: bool = False,
                  width_lanes: bool = False) -> None:
        """Streams (lanes) and flags of the schedule; width_lanes (with
        per_network) keeps each lane to networks of one width."""
        flags = (_lib.PINN_BATCH_GRAPH if use_graph else 0) | (_lib.PINN_BATCH_PER_NETWORK if per_network else 0) | \
            (_lib.PINN_BATCH_WIDTH_LANES if width_lanes else 0)
        check(lib.pinn_batch_configure(self.handle, int(n_streams), flags))

    def config(self) -> dict:
        """{'streams', 'graph', 'per_network', 'width_lanes'} of the current schedule."""
        ns, fl = ctypes.c_int32(), ctypes.c_int32()
        check(lib.pinn_batch_get_config(self.handle, ctypes.byref(ns), ctypes.byref(fl)))
        return {"streams": ns.value, "graph": bool(fl.value & _lib.PINN_BATCH_GRAPH),
                "per_network": bool(fl.value & _lib.PINN_BATCH_PER_NETWORK),
                "width_lanes": bool(fl.value & _lib.PINN_BATCH_WIDTH_LANES)}

    def _marshal(self, params_list, xs):
        key = tuple(t.data_ptr() for ps in params_list for pair in ps for t in pair) + \
            tuple(x.data_ptr() for x in xs) + tuple(x.shape[0] for x in xs)
        if self._args_key == key:
            return self._args
        if self.grads is None:
            self.grads = [[(torch.empty_like(W), torch.empty_like(b)) for W, b in ps] for ps in params_list]
        keep = []
        nets = (Net * self.n)()
        dWs = (ctypes.c_void_p * self.n)()
        dbs = (ctypes.c_void_p * self.n)()
        for i, (ps, x) in enumerate(zip(params_list, xs)):
            _check_tensor(x, f"x[{i}]")
            for l, (W, b) in enumerate(ps):
                _check_tensor(W, f"W[{i}][{l}]")
                _check_tensor(b, f"b[{i}][{l}]")
            d = [int(ps[0][0].shape[1])] + [int(W.shape[0]) for W, _ in ps]
            da = (ctypes.c_int32 * len(d))(*d)
            Wp, wa = ptr_array([W.data_ptr() for W, _ in ps])
            bp, ba = ptr_array([b.data_ptr() for _, b in ps])
            gWp, gwa = ptr_array([g[0].data_ptr() for g in self.grads[i]])
            gbp, gba = ptr_array([g[1].data_ptr() for g in self.grads[i]])
            keep += [da, wa, ba, gwa, gba]
            nets[i] = Net(len(d) - 1, ctypes.cast(da, ctypes.POINTER(ctypes.c_int32)), Wp, bp)
            dWs[i] = ctypes.cast(gWp, ctypes.c_void_p)
            dbs[i] = ctypes.cast(gbp, ctypes.c_void_p)
        xp = (ctypes.c_void_p * self.n)(*[x.data_ptr() for x in xs])
        Ns = (ctypes.c_int64 * self.n)(*[int(x.shape[0]) for x in xs])
        self._args = (nets, xp, Ns, dWs, dbs, keep)
        self._args_key = key
        return self._args

    def step(self, params_list, xs) -> Tuple[torch.Tensor, List[List[Tuple[torch.Tensor, torch.Tensor]]]]:
        """One residual + gradient step of every network; returns (loss (n,), grads)."""
        nets, xp, Ns, dWs, dbs, _ = self._marshal(params_list, xs)
        pp = ctypes.POINTER(ctypes.c_void_p)
        check(lib.pinn_batch_step(self.handle, nets, self._pdes, ctypes.cast(xp, pp), Ns,
                                  ctypes.c_void_p(self.loss.data_ptr()), ctypes.cast(dWs, pp),
                                  ctypes.cast(dbs, pp), _stream()))
        return self.loss, self.grads

    def autotune(self, params_list, xs, reps: int = 3) -> Tuple[int, float]:
        nets, xp, Ns, dWs, dbs, _ = self._marshal(params_list, xs)
        pp = ctypes.POINTER(ctypes.c_void_p)
        bs, ms = ctypes.c_int32(), ctypes.c_double()
        check(lib.pinn_batch_autotune(self.handle, nets, self._pdes, ctypes.cast(xp, pp), Ns,
                                      ctypes.c_void_p(self.loss.data_ptr()), ctypes.cast(dWs, pp),
                                      ctypes.cast(dbs, pp), int(reps), ctypes.byref(bs), ctypes.byref(ms),
                                      _stream()))
        return bs.value, ms.value

    def profile(self, kernel_class: str) -> None:
        """Start timing grouped launches of one kernel class ('off' to stop); steps run eagerly meanwhile."""
        from ._lib import KERNEL_CLASSES
        cls = 0 if kernel_class == "off" else KERNEL_CLASSES[kernel_class]
        check(lib.pinn_batch_profile(self.handle, cls))

    def profile_read(self):
        """(summed kernel milliseconds, launches) since profile(); waits for the events."""
        ms, n = ctypes.c_double(), ctypes.c_int64()
        check(lib.pinn_batch_profile_read(self.handle, ctypes.byref(ms), ctypes.byref(n)))
        return ms.value, n.value

    def tuning(self, i: int) -> dict:
        """The tuning of network i (split count, forward point tile, fused weight
        gradient, wide backward point tile)."""
        t = Tuning()
        check(lib.pinn_batch_get_tuning(self.handle, int(i), ctypes.byref(t)))
        return {"dw_splits": t.dw_splits, "fwd_points": t.fwd_points, "bwd_fused": t.bwd_fused,
                "bwd_points": t.bwd_points}

    def set_tuning(self, i: int, dw_splits: int, fwd_points: int = 0, bwd_fused: int = 1,
                   bwd_points: int = 0) -> None:
        """Replace network i's tuning (PinnPlan.set_tuning); the next step rebuilds the schedule."""
        t = Tuning(int(dw_splits), int(fwd_points), int(bwd_fused), int(bwd_points))
        check(lib.pinn_batch_set_tuning(self.handle, int(i), ctypes.byref(t)))

    def schedule_classes(self) -> List[str]:
        """The kernel class of every grouped launch of the current schedule, in
        launch order lane by lane (see pinn_batch_schedule_classes)."""
        n = ctypes.c_int64()
        check(lib.pinn_batch_schedule_classes(self.handle, None, 0, ctypes.byref(n)))
        arr = (ctypes.c_int32 * max(n.value, 1))()
        check(lib.pinn_batch_schedule_classes(self.handle, arr, n.value, ctypes.byref(n)))
        names = {v: k for k, v in _lib.KERNEL_CLASSES.items()}
        return [names.get(arr[i], "other") for i in range(n.value)]

    def launches(self) -> int:
        """Grouped launches per step of the current schedule."""
        n = ctypes.c_int64()
        check(lib.pinn_batch_launches(self.handle, ctypes.byref(n)))
        return n.value

    def train_step(self, params_list, xs, adam: "BatchAdam"):
        """One residual + gradient + Adam step of every network (parameters
        updated in place; the step count advances on the device)."""
        nets, xp, Ns, dWs, dbs, _ = self._marshal(params_list, xs)
        pp = ctypes.POINTER(ctypes.c_void_p)
        check(lib.pinn_batch_train_step(self.handle, nets, self._pdes, ctypes.cast(xp, pp), Ns,
                                        ctypes.c_void_p(self.loss.data_ptr()), ctypes.cast(dWs, pp),
                                        ctypes.cast(dbs, pp), ctypes.cast(adam._mW, pp), ctypes.cast(adam._vW, pp),
                                        ctypes.cast(adam._mb, pp), ctypes.cast(adam._vb, pp), ctypes.byref(adam.hp),
                                        ctypes.c_void_p(adam.step.data_ptr()), _stream()))
        return self.loss, self.grads


class BatchAdam:
    """Adam moments (zero) for the parameters of every network of a batch, and
    the device step counter of the batch's training step."""

    def __init__(self, params_list, lr: float = 1e-3, betas: Tuple[float, float] = (0.9, 0.999),
                 eps: float = 1e-8):
        self.hp = _AdamHP(float(lr), float(betas[0]), float(betas[1]), float(eps))
        self.m = [[(torch.zeros_like(W), torch.zeros_like(b)) for W, b in ps] for ps in params_list]
        self.v = [[(torch.zeros_like(W), torch.zeros_like(b)) for W, b in ps] for ps in params_list]
        dev = params_list[0][0][0].device
        self.step = torch.zeros((), device=dev, dtype=torch.int64)
        self._keep = []

        def table(pairs, k):
            arrs = []
            for ps in pairs:
                p, keep = ptr_array([t[k].data_ptr() for t in ps])
                self._keep.append(keep)
                arrs.append(ctypes.cast(p, ctypes.c_void_p))
            return (ctypes.c_void_p * len(arrs))(*arrs)

        self._mW, self._mb = table(self.m, 0), table(self.m, 1)
        self._vW, self._vb = table(self.v, 0), table(self.v, 1)

"""Python binding of the partial-jet C ABI: a plan object and the
torch.autograd.Function whose backward is the library's hand-written adjoint.

Tensors are torch device tensors (float32, contiguous); torch supplies device
memory and the current stream, the library does all the arithmetic.
"""
from __future__ import annotations

import ctypes
from typing import List, Optional, Sequence, Tuple

import torch

from . import _lib
from ._lib import (KINDS, PRECISIONS, SEG_DATA, SEG_TYPES, Modified, Net, Pde, PinnError, Segment, Tuning, check, lib,
                   ptr_array)
from .closure import channels, resolve_kind

CHANNELS = {k: lib.pinn_pde_channels(v) for k, v in KINDS.items()}
RESIDUALS = {k: lib.pinn_pde_residuals(v) for k, v in KINDS.items()}

DEFAULT_COEF = {"burgers": (0.01 / 3.141592653589793,), "ns": (100.0,), "ks": (1.0, 1.0, 1.0),
                "heat": (0.1,), "aniso": (0.5,), "burgers_bc": ()}


def _stream() -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _check_tensor(t: torch.Tensor, name: str) -> None:
    if not (t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()):
        raise ValueError(f"{name} must be a contiguous float32 device tensor")


class _NetView:
    """Holds the ctypes pinn_net and the arrays it points to."""

    def __init__(self, params: Sequence[Tuple[torch.Tensor, torch.Tensor]]):
        dims = [int(params[0][0].shape[1])] + [int(W.shape[0]) for W, _ in params]
        for l, (W, b) in enumerate(params):
            _check_tensor(W, f"W[{l}]")
            _check_tensor(b, f"b[{l}]")
        self.dims = (ctypes.c_int32 * len(dims))(*dims)
        self.Wp, self._wa = ptr_array([W.data_ptr() for W, _ in params])
        self.bp, self._ba = ptr_array([b.data_ptr() for _, b in params])
        self.net = Net(len(params), ctypes.cast(self.dims, ctypes.POINTER(ctypes.c_int32)), self.Wp, self.bp)


def _pde(kind: str, coef: Sequence[float]) -> Pde:
    p = Pde()
    p.kind = KINDS[kind]
    for i, c in enumerate(coef):
        p.coef[i] = float(c)
    return p


class PinnPlan:
    """One network shape + PDE kind + maximum point count on the current device."""

    def __init__(self, dims: Sequence[int], pde: str, max_points: int, precision: str = "fp32",
                 verify_f64: bool = False, save_cap_bytes: int = 0,
                 coef: Optional[Sequence[float]] = None):
        self.dims = list(dims)
        self.pde = pde
        self.coef = tuple(coef) if coef is not None else DEFAULT_COEF[pde]
        self.precision = precision
        self.verify_f64 = verify_f64
        self.C = CHANNELS[pde]
        self.n_res = RESIDUALS[pde]
        self.max_points = int(max_points)
        # Shape-only net for plan creation: non-null placeholders are never read.
        ptrs = [1] * (len(dims) - 1)
        d = (ctypes.c_int32 * len(dims))(*dims)
        Wp, wa = ptr_array(ptrs)
        bp, ba = ptr_array(ptrs)
        net = Net(len(dims) - 1, ctypes.cast(d, ctypes.POINTER(ctypes.c_int32)), Wp, bp)
        handle = ctypes.c_void_p()
        flags = _lib.PINN_VERIFY_F64 if verify_f64 else 0
        check(lib.pinn_plan_create(ctypes.byref(net), ctypes.byref(_pde(pde, self.coef)), self.max_points,
                                   PRECISIONS[precision], flags, int(save_cap_bytes), ctypes.byref(handle)))
        self.handle = handle

    @classmethod
    def for_derivatives(cls, dims: Sequence[int], derivatives, max_points: int, pde: Optional[str] = None,
                        **kwargs) -> "PinnPlan":
        """A plan for a residual given by the coordinate derivatives it uses
        (tuples of input directions, () the value): the channel closure of
        Sec. 2.2 picks the compiled kind (or checks that `pde` carries it).
        Raises PinnError PINN_ERR_UNSUPPORTED when no compiled kind does."""
        derivatives = [tuple(d) for d in derivatives]
        kind = resolve_kind(derivatives, pde)
        if kind is None:
            raise PinnError(_lib.PINN_ERR_UNSUPPORTED,
                            f"no compiled kind carries the channel closure {channels(derivatives)}"
                            + (f" (kind {pde!r})" if pde else ""))
        return cls(dims, kind, max_points, **kwargs)

    def close(self) -> None:
        if getattr(self, "handle", None):
            check(lib.pinn_plan_destroy(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def memory(self) -> Tuple[int, int]:
        s, w = ctypes.c_size_t(), ctypes.c_size_t()
        check(lib.pinn_plan_memory(self.handle, ctypes.byref(s), ctypes.byref(w)))
        return s.value, w.value

    def tuning(self) -> dict:
        t = Tuning()
        check(lib.pinn_plan_get_tuning(self.handle, ctypes.byref(t)))
        return {"dw_splits": t.dw_splits, "fwd_points": t.fwd_points, "bwd_fused": t.bwd_fused,
                "bwd_points": t.bwd_points}

    def set_tuning(self, dw_splits: int, fwd_points: int = 0, bwd_fused: int = 1, bwd_points: int = 0) -> None:
        t = Tuning(int(dw_splits), int(fwd_points), int(bwd_fused), int(bwd_points))
        check(lib.pinn_plan_set_tuning(self.handle, ctypes.byref(t)))

    def autotune(self, params, x: torch.Tensor, reps: int = 3) -> Tuple[dict, float]:
        """Times the candidate tunings on (params, x), keeps the fastest; returns it and ms/step."""
        _check_tensor(x, "x")
        nv = _NetView(params)
        t, ms = Tuning(), ctypes.c_double()
        check(lib.pinn_plan_autotune(self.handle, ctypes.byref(nv.net), ctypes.byref(_pde(self.pde, self.coef)),
                                     ctypes.c_void_p(x.data_ptr()), x.shape[0], int(reps), ctypes.byref(t),
                                     ctypes.byref(ms), _stream()))
        return {"dw_splits": t.dw_splits, "fwd_points": t.fwd_points, "bwd_fused": t.bwd_fused,
                "bwd_points": t.bwd_points}, ms.value

    def profile(self, kernel_class: str) -> None:
        """Start timing launches of one kernel class ('off' to stop)."""
        cls = 0 if kernel_class == "off" else _lib.KERNEL_CLASSES[kernel_class]
        check(lib.pinn_plan_profile(self.handle, cls))

    def profile_read(self) -> Tuple[float, int]:
        """(summed kernel milliseconds, launches) since profile(); waits for the events."""
        ms, n = ctypes.c_double(), ctypes.c_int64()
        check(lib.pinn_plan_profile_read(self.handle, ctypes.byref(ms), ctypes.byref(n)))
        return ms.value, n.value

    # ---------------------------------------------------------------- calls
    def forward(self, params, x: torch.Tensor) -> torch.Tensor:
        """Jets (d_out, C, N) at the points x (N, d_in)."""
        _check_tensor(x, "x")
        nv = _NetView(params)
        N = x.shape[0]
        jets = torch.empty((self.dims[-1], self.C, N), device=x.device, dtype=torch.float32)
        check(lib.pinn_jet_forward(self.handle, ctypes.byref(nv.net), ctypes.c_void_p(x.data_ptr()), N,
                                   ctypes.c_void_p(jets.data_ptr()), _stream()))
        return jets

    def residual(self, params, x: torch.Tensor, want_jets: bool = False):
        """Returns (r (n_res, N), loss (1,), loss_f64 (1,) or None, jets or None)."""
        _check_tensor(x, "x")
        nv = _NetView(params)
        N = x.shape[0]
        dev = x.device
        r = torch.empty((self.n_res, N), device=dev, dtype=torch.float32)
        loss = torch.empty((), device=dev, dtype=torch.float32)
        loss64 = torch.empty((), device=dev, dtype=torch.float64) if self.verify_f64 else None
        jets = torch.empty((self.dims[-1], self.C, N), device=dev, dtype=torch.float32) if want_jets else None
        check(lib.pinn_jet_residual(
            self.handle, ctypes.byref(nv.net), ctypes.byref(_pde(self.pde, self.coef)),
            ctypes.c_void_p(x.data_ptr()), N, ctypes.c_void_p(r.data_ptr()), ctypes.c_void_p(loss.data_ptr()),
            ctypes.c_void_p(loss64.data_ptr()) if loss64 is not None else None,
            ctypes.c_void_p(jets.data_ptr()) if jets is not None else None, _stream()))
        return r, loss, loss64, jets

    def backward(self, params, x: torch.Tensor, r_bar: Optional[torch.Tensor] = None,
                 want_f64: bool = False, out=None, loss_bar: Optional[torch.Tensor] = None):
        """Gradient [(dW, db), ...] of <r_bar, r> + loss_bar * loss; r_bar and
        loss_bar (a device scalar) both None means the loss gradient.  With
        want_f64 also the FP64 reductions.  `out`, a list of (dW, db) tensors
        shaped like params, receives the gradient instead of new ones."""
        nv = _NetView(params)
        N = x.shape[0]
        dev = x.device
        if r_bar is not None:
            _check_tensor(r_bar, "r_bar")
            if tuple(r_bar.shape) != (self.n_res, N):
                raise ValueError("r_bar must be (n_res, N)")
        grads = out if out is not None else [(torch.empty_like(W), torch.empty_like(b)) for W, b in params]
        dWp, k1 = ptr_array([g[0].data_ptr() for g in grads])
        dbp, k2 = ptr_array([g[1].data_ptr() for g in grads])
        g64 = None
        dW64p = db64p = None
        if want_f64:
            g64 = [(torch.empty(W.shape, device=dev, dtype=torch.float64),
                    torch.empty(b.shape, device=dev, dtype=torch.float64)) for W, b in params]
            dW64p, k3 = ptr_array([g[0].data_ptr() for g in g64])
            db64p, k4 = ptr_array([g[1].data_ptr() for g in g64])
        if loss_bar is not None and not (loss_bar.is_cuda and loss_bar.dtype == torch.float32
                                         and loss_bar.numel() == 1):
            raise ValueError("loss_bar must be a one-element float32 device tensor")
        check(lib.pinn_jet_backward_cot(
            self.handle, ctypes.byref(nv.net), ctypes.byref(_pde(self.pde, self.coef)),
            ctypes.c_void_p(x.data_ptr()), N,
            ctypes.c_void_p(r_bar.data_ptr()) if r_bar is not None else None,
            ctypes.c_void_p(loss_bar.data_ptr()) if loss_bar is not None else None,
            dWp, dbp, dW64p, db64p, _stream()))
        return (grads, g64) if want_f64 else grads


    # ------------------------------------------------------------ composite loss
    @staticmethod
    def _segments(segments):
        arr = (Segment * len(segments))()
        for i, sg in enumerate(segments):
            arr[i].type = SEG_TYPES[sg["type"]]
            arr[i].data = SEG_DATA[sg.get("data", "zero")]
            arr[i].begin = int(sg["begin"])
            arr[i].count = int(sg["count"])
            arr[i].weight = float(sg.get("weight", 1.0))
            arr[i].mask = int(sg.get("mask", 0))
            for q, v in enumerate(sg.get("param", ())):
                arr[i].param[q] = float(v)
            if sg.get("data") == "values":
                vals = sg["values"]
                _check_tensor(vals, "values")
                arr[i].values = vals.data_ptr()
        return arr

    def loss(self, params, x: torch.Tensor, segments):
        """Composite loss over point segments (all points evaluated together,
        then split; see pinn_jet_loss).  segments: list of dicts with type
        ('pde', 'dirichlet', 'periodic'), begin, count, weight, mask, data
        ('zero', 'const', 'sin', 'values') and param; 'values' takes a device
        tensor of count x d_out float32 targets.  Returns (loss (), seg_loss (n,))."""
        _check_tensor(x, "x")
        nv = _NetView(params)
        segs = self._segments(segments)
        loss = torch.empty((), device=x.device, dtype=torch.float32)
        seg_loss = torch.empty(len(segments), device=x.device, dtype=torch.float32)
        check(lib.pinn_jet_loss(self.handle, ctypes.byref(nv.net), ctypes.byref(_pde(self.pde, self.coef)), segs,
                                len(segments), ctypes.c_void_p(x.data_ptr()), x.shape[0],
                                ctypes.c_void_p(loss.data_ptr()), ctypes.c_void_p(seg_loss.data_ptr()), _stream()))
        return loss, seg_loss

    def loss_backward(self, params, x: torch.Tensor, segments, out=None):
        """d loss / d theta of the composite loss of the preceding loss() call."""
        nv = _NetView(params)
        segs = self._segments(segments)
        grads = out if out is not None else [(torch.empty_like(W), torch.empty_like(b)) for W, b in params]
        dWp, k1 = ptr_array([g[0].data_ptr() for g in grads])
        dbp, k2 = ptr_array([g[1].data_ptr() for g in grads])
        check(lib.pinn_jet_loss_backward(self.handle, ctypes.byref(nv.net), ctypes.byref(_pde(self.pde, self.coef)),
                                         segs, len(segments), ctypes.c_void_p(x.data_ptr()), x.shape[0], dWp, dbp,
                                         _stream()))
        return grads

    def capture_step(self, params, x: torch.Tensor, adam=None) -> "PinnGraph":
        """The residual + loss-gradient step on (params, x) as a replayable
        HIP graph (pinn_graph_capture); outputs live on the returned object.
        With `adam` (an AdamState on the same params) the graph also applies
        the Adam update (pinn_graph_capture_train), counting steps on the
        device."""
        return PinnGraph(self, params, x, adam)


class ModifiedPlan(PinnPlan):
    """A plan for the modified MLP with periodic input embedding (the KS
    network of Sec. 3.1.1; pinn_plan_create_modified), FP32 operands.
    Parameters are [(W_U, b_U), (W_V, b_V), (W_1, b_1), .., (W_H, b_H),
    (W_o, b_o)]; forward, residual, backward, loss and loss_backward as for
    PinnPlan."""

    def __init__(self, hidden: int, width: int, harmonics: int, period: float, pde: str, max_points: int,
                 coef: Optional[Sequence[float]] = None):
        self.pde = pde
        self.coef = tuple(coef) if coef is not None else DEFAULT_COEF[pde]
        self.precision = "fp32"
        self.verify_f64 = False
        self.C = CHANNELS[pde]
        self.n_res = RESIDUALS[pde]
        self.max_points = int(max_points)
        self.hidden, self.width, self.harmonics, self.period = int(hidden), int(width), int(harmonics), float(period)
        self.dims = [2] + [self.width] * self.hidden + [1]  # inputs (x, t), output u (KS, Burgers)
        arch = Modified(self.hidden, self.width, self.harmonics, self.period)
        handle = ctypes.c_void_p()
        check(lib.pinn_plan_create_modified(ctypes.byref(arch), ctypes.byref(_pde(pde, self.coef)), self.max_points,
                                            PRECISIONS["fp32"], 0, ctypes.byref(handle)))
        self.handle = handle


class PinnGraph:
    """One captured step of a plan.  launch() replays it on the current
    stream, reading the current contents of the parameter and point tensors
    given at capture; r, loss and grads are overwritten by every launch."""

    def __init__(self, plan: PinnPlan, params, x: torch.Tensor, adam=None):
        _check_tensor(x, "x")
        self.plan = plan
        self.params = params  # kept alive: the graph holds their pointers
        self.x = x
        nv = _NetView(params)
        N = x.shape[0]
        dev = x.device
        self.r = torch.empty((plan.n_res, N), device=dev, dtype=torch.float32)
        self.loss = torch.empty((), device=dev, dtype=torch.float32)
        self.grads = [(torch.empty_like(W), torch.empty_like(b)) for W, b in params]
        dWp, self._k1 = ptr_array([g[0].data_ptr() for g in self.grads])
        dbp, self._k2 = ptr_array([g[1].data_ptr() for g in self.grads])
        handle = ctypes.c_void_p()
        self._nv = nv
        self.adam = adam
        if adam is None:
            check(lib.pinn_graph_capture(plan.handle, ctypes.byref(nv.net), ctypes.byref(_pde(plan.pde, plan.coef)),
                                         ctypes.c_void_p(x.data_ptr()), N, ctypes.c_void_p(self.r.data_ptr()),
                                         ctypes.c_void_p(self.loss.data_ptr()), dWp, dbp, ctypes.byref(handle)))
        else:
            if [p.data_ptr() for pair in adam.params for p in pair] != [p.data_ptr() for pair in params for p in pair]:
                raise ValueError("the AdamState must hold the same parameter tensors")
            if len(adam.runs) != 1:
                raise ValueError("a captured training step takes the parameters of a plain MLP (one chain)")
            run = adam.runs[0]
            self.step = torch.zeros((), device=dev, dtype=torch.int64)  # updates done so far
            check(lib.pinn_graph_capture_train(
                plan.handle, ctypes.byref(nv.net), ctypes.byref(_pde(plan.pde, plan.coef)),
                ctypes.c_void_p(x.data_ptr()), N, ctypes.c_void_p(self.r.data_ptr()),
                ctypes.c_void_p(self.loss.data_ptr()), dWp, dbp, run["mW"][0], run["vW"][0], run["mb"][0],
                run["vb"][0], ctypes.byref(adam.hp), ctypes.c_void_p(self.step.data_ptr()), ctypes.byref(handle)))
        self.handle = handle

    def launch(self) -> None:
        check(lib.pinn_graph_launch(self.handle, _stream()))

    def close(self) -> None:
        if getattr(self, "handle", None):
            check(lib.pinn_graph_destroy(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class JetResidual(torch.autograd.Function):
    """(r, loss) = JetResidual.apply(plan, x, W1, b1, ..., WL, bL).

    Backward hands both cotangents to the library (pinn_jet_backward_cot),
    which forms r_bar = g_r + g_loss * 2 r / N on the device and runs its
    adjoint; x receives no gradient."""

    @staticmethod
    def forward(ctx, plan: PinnPlan, x: torch.Tensor, *flat):
        params = [(flat[2 * i], flat[2 * i + 1]) for i in range(len(flat) // 2)]
        r, loss, _, _ = plan.residual(params, x)
        ctx.plan = plan
        ctx.params = params
        # an output that receives no gradient stays None in backward (not a
        # zero tensor), so that loss-only training hands the library the loss
        # cotangent alone and keeps its cotangent scaling
        ctx.set_materialize_grads(False)
        ctx.save_for_backward(x, r)
        return r, loss

    @staticmethod
    def backward(ctx, g_r, g_loss):
        x, r = ctx.saved_tensors
        r_bar = g_r.contiguous().float() if g_r is not None else None
        loss_bar = g_loss.reshape(1).contiguous().float() if g_loss is not None else None
        if r_bar is None and loss_bar is None:
            loss_bar = torch.zeros(1, device=x.device, dtype=torch.float32)
        grads = ctx.plan.backward(ctx.params, x, r_bar, loss_bar=loss_bar)
        out = [None, None]
        for dW, db in grads:
            out += [dW, db]
        return tuple(out)


def jet_residual(plan: PinnPlan, params, x: torch.Tensor):
    flat: List[torch.Tensor] = [t for pair in params for t in pair]
    return JetResidual.apply(plan, x, *flat)


def jet_step_noalloc(params, x: torch.Tensor, pde: str, coef: Optional[Sequence[float]] = None,
                     precision: str = "fp32", r: Optional[torch.Tensor] = None,
                     loss: Optional[torch.Tensor] = None, grads=None):
    """One residual + loss + loss-gradient step through pinn_jet_step_noalloc
    (no device allocation in the library; its workspace is a static device
    array).  r (n_res, N), loss () and grads [(dW, db), ...] are created here
    unless given; returns (r, loss, grads)."""
    _check_tensor(x, "x")
    nv = _NetView(params)
    N = x.shape[0]
    dev = x.device
    coef = tuple(coef) if coef is not None else DEFAULT_COEF[pde]
    if r is None:
        r = torch.empty((RESIDUALS[pde], N), device=dev, dtype=torch.float32)
    if loss is None:
        loss = torch.empty((), device=dev, dtype=torch.float32)
    if grads is None:
        grads = [(torch.empty_like(W), torch.empty_like(b)) for W, b in params]
    dWp, k1 = ptr_array([g[0].data_ptr() for g in grads])
    dbp, k2 = ptr_array([g[1].data_ptr() for g in grads])
    check(lib.pinn_jet_step_noalloc(ctypes.byref(nv.net), ctypes.byref(_pde(pde, coef)), PRECISIONS[precision],
                                    ctypes.c_void_p(x.data_ptr()), N, ctypes.c_void_p(r.data_ptr()),
                                    ctypes.c_void_p(loss.data_ptr()), dWp, dbp, _stream()))
    return r, loss, grads


def tuning_cache_clear() -> None:
    """Drops every entry of the process's autotuning cache."""
    check(lib.pinn_tuning_cache_clear())


def tuning_cache_size() -> int:
    n = ctypes.c_int64()
    check(lib.pinn_tuning_cache_size(ctypes.byref(n)))
    return n.value


def tuning_cache_save(path: str) -> None:
    check(lib.pinn_tuning_cache_save(path.encode()))


def tuning_cache_load(path: str) -> None:
    check(lib.pinn_tuning_cache_load(path.encode()))

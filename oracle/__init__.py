"""FP64 CPU oracle for residual-specific partial-jet propagation (Sec. 2.2, Eq. 1-3).

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check and by the
benchmark's CPU-baseline leg, never by the GPU library or its Python binding.
It shares no code with the GPU path.  Its arithmetic lives in pinn_oracle.cpp;
this module only marshals numpy arrays through ctypes.

Parameters are given as a list of (W, b) pairs, W shaped (out, in), and are
widened to float64.  A channel set is a list of (direction, order) pairs whose
first entry is the value (order 0).
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liborc.so")

ACT = {"tanh": 0, "identity": 1, "square": 2, "cube": 3, "sin": 4}
PDE = {"none": 0, "burgers": 1, "ns": 2, "ks": 3, "heat": 4, "aniso": 5, "burgers_bc": 6}
MIXED2 = -2  # channel order code of a mixed second derivative

_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import build as _b
            _b.build()
        lib = ctypes.CDLL(_LIB_PATH)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        lib.orc_n_res.argtypes = [ctypes.c_int]
        lib.orc_n_res.restype = ctypes.c_int
        lib.orc_eval.argtypes = [ctypes.c_int, ip, dp, ctypes.c_int, ctypes.c_int, dp,
                                 ctypes.c_int, ip, ip, ctypes.c_int64, dp,
                                 dp, dp, dp, dp, dp, ctypes.c_int]
        lib.orc_eval.restype = ctypes.c_int
        lib.orc_eval_cs.argtypes = [ctypes.c_int, ip, dp, dp, ctypes.c_double, ctypes.c_int,
                                    ctypes.c_int, dp, ctypes.c_int, ip, ip, ctypes.c_int64, dp,
                                    dp, dp, dp, ctypes.c_int]
        lib.orc_eval_cs.restype = ctypes.c_int
        i64p = ctypes.POINTER(ctypes.c_int64)
        seg_args = [ctypes.c_int, ip, i64p, i64p, dp, ip, ip, dp]
        lib.orc_eval_segments.argtypes = ([ctypes.c_int, ip, dp, ctypes.c_int, ctypes.c_int, dp, ctypes.c_int, ip,
                                           ip, ctypes.c_int64, dp] + seg_args + [dp, dp, dp, ctypes.c_int])
        lib.orc_eval_segments.restype = ctypes.c_int
        lib.orc_eval_segments_cs.argtypes = ([ctypes.c_int, ip, dp, dp, ctypes.c_double, ctypes.c_int, ctypes.c_int,
                                              dp, ctypes.c_int, ip, ip, ctypes.c_int64, dp] + seg_args +
                                             [dp, ctypes.c_int])
        lib.orc_eval_segments_cs.restype = ctypes.c_int
        mod_head = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_int]
        lib.orc_mod_n_theta.argtypes = mod_head + [i64p]
        lib.orc_mod_n_theta.restype = ctypes.c_int
        lib.orc_eval_mod.argtypes = (mod_head + [dp, ctypes.c_int, ctypes.c_int, dp, ctypes.c_int, ip, ip,
                                                 ctypes.c_int64, dp, dp] + seg_args + [dp, dp, dp, dp,
                                                                                      ctypes.c_int])
        lib.orc_eval_mod.restype = ctypes.c_int
        lib.orc_eval_mod_cs.argtypes = (mod_head + [dp, dp, ctypes.c_double, ctypes.c_int, ctypes.c_int, dp,
                                                    ctypes.c_int, ip, ip, ctypes.c_int64, dp, dp] + seg_args +
                                        [dp, dp, ctypes.c_int])
        lib.orc_eval_mod_cs.restype = ctypes.c_int
        lib.orc_adam.argtypes = [ctypes.c_int64, dp, dp, dp, dp, ctypes.c_int64, ctypes.c_double, ctypes.c_double,
                                 ctypes.c_double, ctypes.c_double]
        lib.orc_adam.restype = ctypes.c_int
        _lib = lib
    return _lib


def _dp(a: Optional[np.ndarray]):
    if a is None:
        return ctypes.POINTER(ctypes.c_double)()
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _ip(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))


def dims_of(params) -> list:
    dims = [int(params[0][0].shape[1])]
    for W, _ in params:
        dims.append(int(W.shape[0]))
    return dims


def pack_theta(params) -> np.ndarray:
    """Flatten [(W1, b1), ..., (WL, bL)] into one float64 vector (W then b per layer)."""
    parts = []
    for W, b in params:
        parts.append(np.asarray(W, dtype=np.float64).reshape(-1))
        parts.append(np.asarray(b, dtype=np.float64).reshape(-1))
    return np.ascontiguousarray(np.concatenate(parts))


def unpack_theta(theta: np.ndarray, dims: Sequence[int]) -> list:
    out, off = [], 0
    for l in range(len(dims) - 1):
        n_out, n_in = dims[l + 1], dims[l]
        W = theta[off:off + n_out * n_in].reshape(n_out, n_in)
        off += n_out * n_in
        b = theta[off:off + n_out]
        off += n_out
        out.append((W, b))
    return out


def n_res(pde: str) -> int:
    return int(_load().orc_n_res(PDE[pde]))


@dataclass
class OracleResult:
    jets: Optional[np.ndarray]   # (d_out, C, N)
    r: Optional[np.ndarray]      # (n_res, N)
    loss: Optional[float]
    grad: Optional[np.ndarray]   # packed like pack_theta


def _common(params, channels, coef):
    dims = np.ascontiguousarray(dims_of(params), dtype=np.int32)
    ch = list(channels)
    # a channel is (direction, order); a mixed second derivative is ((i, j), 2)
    ch_dir = np.ascontiguousarray([8 * c[0][0] + c[0][1] if isinstance(c[0], tuple)
                                   else (max(c[0], 0) if c[1] > 0 else 0) for c in ch], dtype=np.int32)
    ch_ord = np.ascontiguousarray([MIXED2 if isinstance(c[0], tuple) else c[1] for c in ch], dtype=np.int32)
    cf = np.zeros(4, dtype=np.float64)
    cf[:len(coef)] = np.asarray(coef, dtype=np.float64)
    return dims, ch_dir, ch_ord, cf


def evaluate(params, x, channels, pde: str = "none", coef: Sequence[float] = (), act: str = "tanh",
             want_jets: bool = True, want_residual: bool = True, want_grad: bool = True,
             r_bar: Optional[np.ndarray] = None, threads: int = 0) -> OracleResult:
    """Jets, residuals, loss and parameter gradient at the points x (N x d), in FP64."""
    lib = _load()
    dims, ch_dir, ch_ord, cf = _common(params, channels, coef)
    theta = pack_theta(params)
    xx = np.ascontiguousarray(x, dtype=np.float64)
    N = xx.shape[0]
    C = len(ch_dir)
    nr = n_res(pde)
    jets = np.zeros((dims[-1], C, N)) if want_jets else None
    has_res = want_residual and nr > 0
    r = np.zeros((nr, N)) if has_res else None
    loss = np.zeros(1) if has_res else None
    grad = np.zeros(theta.size) if (want_grad and nr > 0) else None
    rb = None if r_bar is None else np.ascontiguousarray(r_bar, dtype=np.float64).reshape(nr, N)
    st = lib.orc_eval(len(dims) - 1, _ip(dims), _dp(theta), ACT[act], PDE[pde], _dp(cf),
                      C, _ip(ch_dir), _ip(ch_ord), N, _dp(xx),
                      _dp(jets), _dp(r), _dp(loss), _dp(rb), _dp(grad), int(threads))
    if st != 0:
        raise ValueError(f"orc_eval failed with status {st}")
    return OracleResult(jets, r, None if loss is None else float(loss[0]), grad)


def complex_step(params, delta: np.ndarray, x, channels, pde: str = "none",
                 coef: Sequence[float] = (), act: str = "tanh", h: float = 1e-30,
                 threads: int = 0):
    """Directional derivatives along delta (packed like theta) of (jets, r, loss)."""
    lib = _load()
    dims, ch_dir, ch_ord, cf = _common(params, channels, coef)
    theta = pack_theta(params)
    dl = np.ascontiguousarray(delta, dtype=np.float64)
    assert dl.size == theta.size
    xx = np.ascontiguousarray(x, dtype=np.float64)
    N = xx.shape[0]
    C = len(ch_dir)
    nr = n_res(pde)
    djets = np.zeros((dims[-1], C, N))
    dr = np.zeros((nr, N)) if nr > 0 else None
    dloss = np.zeros(1) if nr > 0 else None
    st = lib.orc_eval_cs(len(dims) - 1, _ip(dims), _dp(theta), _dp(dl), float(h), ACT[act],
                         PDE[pde], _dp(cf), C, _ip(ch_dir), _ip(ch_ord), N, _dp(xx),
                         _dp(djets), _dp(dr), _dp(dloss), int(threads))
    if st != 0:
        raise ValueError(f"orc_eval_cs failed with status {st}")
    return djets, dr, None if dloss is None else float(dloss[0])


SEG = {"pde": 0, "dirichlet": 1, "periodic": 2}
DATA = {"zero": 0, "const": 1, "sin": 2, "values": 3}


def _segments(segments):
    """[{'type', 'begin', 'count', 'weight', 'mask', 'data', 'param'}, ...] -> ctypes arrays."""
    n = len(segments)
    typ = np.ascontiguousarray([SEG[s["type"]] for s in segments], dtype=np.int32)
    beg = np.ascontiguousarray([s["begin"] for s in segments], dtype=np.int64)
    cnt = np.ascontiguousarray([s["count"] for s in segments], dtype=np.int64)
    wt = np.ascontiguousarray([s.get("weight", 1.0) for s in segments], dtype=np.float64)
    mask = np.ascontiguousarray([s.get("mask", 0) for s in segments], dtype=np.int32)
    data = np.ascontiguousarray([DATA[s.get("data", "zero")] for s in segments], dtype=np.int32)
    par = np.zeros((n, 4))
    for i, s in enumerate(segments):
        p = s.get("param", ())
        par[i, :len(p)] = p
    par = np.ascontiguousarray(par)
    i64p = ctypes.POINTER(ctypes.c_int64)
    arrays = (typ, beg, cnt, wt, mask, data, par)
    args = [n, _ip(typ), beg.ctypes.data_as(i64p), cnt.ctypes.data_as(i64p), _dp(wt), _ip(mask), _ip(data), _dp(par)]
    return args, arrays


def evaluate_segments(params, x, channels, pde: str, coef: Sequence[float], segments, act: str = "tanh",
                      want_grad: bool = True, threads: int = 0):
    """Composite loss over point segments (all points evaluated together, then
    split): returns (seg_loss (n_seg,), loss, grad packed like theta or None)."""
    lib = _load()
    dims, ch_dir, ch_ord, cf = _common(params, channels, coef)
    theta = pack_theta(params)
    xx = np.ascontiguousarray(x, dtype=np.float64)
    sargs, keep = _segments(segments)
    seg_loss = np.zeros(len(segments))
    loss = np.zeros(1)
    grad = np.zeros(theta.size) if want_grad else None
    st = lib.orc_eval_segments(len(dims) - 1, _ip(dims), _dp(theta), ACT[act], PDE[pde], _dp(cf), len(ch_dir),
                               _ip(ch_dir), _ip(ch_ord), xx.shape[0], _dp(xx), *sargs, _dp(seg_loss), _dp(loss),
                               _dp(grad), int(threads))
    if st != 0:
        raise ValueError(f"orc_eval_segments failed with status {st}")
    return seg_loss, float(loss[0]), grad


def complex_step_segments(params, delta, x, channels, pde: str, coef: Sequence[float], segments,
                          act: str = "tanh", h: float = 1e-30, threads: int = 0) -> float:
    """Directional derivative of the composite loss along delta (complex step)."""
    lib = _load()
    dims, ch_dir, ch_ord, cf = _common(params, channels, coef)
    theta = pack_theta(params)
    dl = np.ascontiguousarray(delta, dtype=np.float64)
    xx = np.ascontiguousarray(x, dtype=np.float64)
    sargs, keep = _segments(segments)
    out = np.zeros(1)
    st = lib.orc_eval_segments_cs(len(dims) - 1, _ip(dims), _dp(theta), _dp(dl), float(h), ACT[act], PDE[pde],
                                  _dp(cf), len(ch_dir), _ip(ch_dir), _ip(ch_ord), xx.shape[0], _dp(xx), *sargs,
                                  _dp(out), int(threads))
    if st != 0:
        raise ValueError(f"orc_eval_segments_cs failed with status {st}")
    return float(out[0])


def _mod_shape(params, d: int):
    """(H, w, d, M, dout) of a modified-MLP parameter list [(W_U, b_U), (W_V, b_V),
    (W_1, b_1), .., (W_H, b_H), (W_o, b_o)]."""
    w, de = (int(v) for v in np.asarray(params[0][0]).shape)
    M = (de - d + 1) // 2
    if de != d - 1 + 2 * M or M < 1:
        raise ValueError(f"embedding width {de} does not fit d = {d}")
    return len(params) - 3, w, d, M, int(np.asarray(params[-1][0]).shape[0])


def _no_segments():
    i64p = ctypes.POINTER(ctypes.c_int64)
    return [0, ctypes.POINTER(ctypes.c_int)(), i64p(), i64p(), _dp(None), ctypes.POINTER(ctypes.c_int)(),
            ctypes.POINTER(ctypes.c_int)(), _dp(None)]


def evaluate_mod(params, x, channels, pde: str, coef: Sequence[float], period: float, d: int = 2,
                 segments=None, targets=None, want_grad: bool = True, act: str = "tanh", threads: int = 0):
    """The modified MLP with periodic embedding (see pinn_oracle.h): jets
    (d_out, C, N) and, with segments, (seg_loss, loss, grad packed like theta)."""
    lib = _load()
    H, w, d, M, dout = _mod_shape(params, d)
    _, ch_dir, ch_ord, cf = _common(params, channels, coef)
    theta = pack_theta(params)
    xx = np.ascontiguousarray(x, dtype=np.float64)
    N = xx.shape[0]
    jets = np.zeros((dout, len(channels), N))
    if segments:
        sargs, keep = _segments(segments)
        tg = np.ascontiguousarray(targets, dtype=np.float64) if targets is not None else None
        seg_loss, loss = np.zeros(len(segments)), np.zeros(1)
        grad = np.zeros(theta.size) if want_grad else None
        st = lib.orc_eval_mod(H, w, d, M, float(period), dout, _dp(theta), ACT[act], PDE[pde], _dp(cf),
                              len(channels), _ip(ch_dir), _ip(ch_ord), N, _dp(xx), _dp(jets), *sargs, _dp(tg),
                              _dp(seg_loss), _dp(loss), _dp(grad), int(threads))
        if st != 0:
            raise ValueError(f"orc_eval_mod failed with status {st}")
        return jets, seg_loss, float(loss[0]), grad
    st = lib.orc_eval_mod(H, w, d, M, float(period), dout, _dp(theta), ACT[act], PDE[pde], _dp(cf), len(channels),
                          _ip(ch_dir), _ip(ch_ord), N, _dp(xx), _dp(jets), *_no_segments(), _dp(None), _dp(None),
                          _dp(None), _dp(None), int(threads))
    if st != 0:
        raise ValueError(f"orc_eval_mod failed with status {st}")
    return jets


def complex_step_mod(params, delta, x, channels, pde: str, coef: Sequence[float], period: float, d: int = 2,
                     segments=None, targets=None, act: str = "tanh", h: float = 1e-30, threads: int = 0):
    """Directional derivatives along delta (complex step): (djets, dloss or None)."""
    lib = _load()
    H, w, d, M, dout = _mod_shape(params, d)
    _, ch_dir, ch_ord, cf = _common(params, channels, coef)
    theta = pack_theta(params)
    dl = np.ascontiguousarray(delta, dtype=np.float64)
    xx = np.ascontiguousarray(x, dtype=np.float64)
    N = xx.shape[0]
    djets = np.zeros((dout, len(channels), N))
    out = np.zeros(1)
    if segments:
        sargs, keep = _segments(segments)
        tg = np.ascontiguousarray(targets, dtype=np.float64) if targets is not None else None
    else:
        sargs, tg = _no_segments(), None
    st = lib.orc_eval_mod_cs(H, w, d, M, float(period), dout, _dp(theta), _dp(dl), float(h), ACT[act], PDE[pde],
                             _dp(cf), len(channels), _ip(ch_dir), _ip(ch_ord), N, _dp(xx), _dp(djets), *sargs,
                             _dp(tg), _dp(out) if segments else _dp(None), int(threads))
    if st != 0:
        raise ValueError(f"orc_eval_mod_cs failed with status {st}")
    return djets, (float(out[0]) if segments else None)


def adam_step(theta: np.ndarray, g: np.ndarray, m: np.ndarray, v: np.ndarray, step: int,
              lr: float = 1e-3, b1: float = 0.9, b2: float = 0.999, eps: float = 1e-8) -> None:
    """One Adam step in FP64, in place on theta, m and v (flat float64 arrays)."""
    for a in (theta, g, m, v):
        assert a.dtype == np.float64 and a.flags.c_contiguous and a.shape == theta.shape
    st = _load().orc_adam(theta.size, _dp(theta), _dp(g), _dp(m), _dp(v), int(step), float(lr), float(b1),
                          float(b2), float(eps))
    if st != 0:
        raise ValueError(f"orc_adam status {st}")

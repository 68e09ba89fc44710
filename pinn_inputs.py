"""Seeded synthetic inputs for the partial-jet PINN workloads.

This module only draws random numbers: network parameters, collocation points
and ensemble members.  It contains none of the method's arithmetic, and both
the GPU library's tests and the FP64 oracle take their inputs from here.

Recipe (all float64 draws from numpy PCG64, rounded once to float32):
  * weights: Xavier-normal, std = sqrt(2 / (fan_in + fan_out)), W shaped
    (out, in), drawn layer by layer; biases zero unless bias_std > 0 (tests use
    nonzero biases so the bias path is exercised);
  * points: N x d, each coordinate uniform on its interval, drawn after the
    weights from the same generator;
  * ensemble: a master SeedSequence spawns one child per network; each child
    draws width, depth, viscosity and point count, then weights, then points.

The workload shapes follow the library's five benchmark problems (viscous
Burgers, steady Navier-Stokes at Re = 100, Kuramoto-Sivashinsky, 3-D heat and
a 64-network Burgers ensemble).  Channel orders are the library's ABI orders.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

import numpy as np

# Channel sets in ABI order: (direction, order); direction indexes the input
# coordinates of the workload, order 0 is the value.
CHANNELS = {
    # inputs (x, t): u, u_t, u_x, u_xx
    "burgers": [(0, 0), (1, 1), (0, 1), (0, 2)],
    # inputs (x, y): value, d/dx, d/dy, d2/dx2, d2/dy2
    "ns": [(0, 0), (0, 1), (1, 1), (0, 2), (1, 2)],
    # inputs (x, t): u, u_t, u_x, u_xx, u_xxx, u_xxxx
    "ks": [(0, 0), (1, 1), (0, 1), (0, 2), (0, 3), (0, 4)],
    # inputs (x, y, z, t): u, u_t, u_x, u_y, u_z, u_xx, u_yy, u_zz
    "heat": [(0, 0), (3, 1), (0, 1), (1, 1), (2, 1), (0, 2), (1, 2), (2, 2)],
    # inputs (x, y): u, u_x, u_y, u_xx, u_yy, u_xy (a mixed second derivative)
    "aniso": [(0, 0), (0, 1), (1, 1), (0, 2), (1, 2), ((0, 1), 2)],
    # inputs (x, t): u only (initial and boundary data of Burgers)
    "burgers_bc": [(0, 0)],
}

N_RES = {"burgers": 1, "ns": 3, "ks": 1, "heat": 1, "aniso": 1, "burgers_bc": 1}


@dataclass
class Workload:
    name: str
    pde: str
    dims: List[int]
    coef: Tuple[float, ...]
    domain: List[Tuple[float, float]]
    N: int
    note: str = ""

    @property
    def width(self) -> int:
        return self.dims[1]

    @property
    def hidden(self) -> int:
        return len(self.dims) - 2


def _mlp(d_in: int, width: int, hidden: int, d_out: int) -> List[int]:
    return [d_in] + [width] * hidden + [d_out]


WORKLOADS = {
    "burgers": Workload("burgers", "burgers", _mlp(2, 32, 3, 1), (0.01 / math.pi,),
                        [(-1.0, 1.0), (0.0, 1.0)], 1024,
                        "viscous Burgers u_t + u u_x - (0.01/pi) u_xx, 2-32x3-1 tanh"),
    "ns": Workload("ns", "ns", _mlp(2, 128, 6, 3), (100.0,), [(0.0, 1.0), (0.0, 1.0)], 65536,
                   "steady incompressible Navier-Stokes, Re = 100, 2-128x6-3 tanh"),
    "ks": Workload("ks", "ks", _mlp(2, 256, 8, 1), (1.0, 1.0, 1.0),
                   [(0.0, 32.0 * math.pi), (0.0, 1.0)], 131072,
                   "Kuramoto-Sivashinsky u_t + u u_x + u_xx + u_xxxx, 2-256x8-1 tanh"),
    "heat": Workload("heat", "heat", _mlp(4, 512, 8, 1), (0.1,), [(0.0, 1.0)] * 4, 262144,
                     "3-D heat u_t - 0.1 Lap u - f, 4-512x8-1 tanh"),
    # a test operator with a mixed derivative (Eq. 3 with i != j); not one of
    # the paper's problems, shaped like the NS network
    "aniso": Workload("aniso", "aniso", _mlp(2, 128, 6, 1), (0.5,), [(0.0, 1.0), (0.0, 1.0)], 65536,
                      "anisotropic operator u_xx + 2c u_xy + u_yy, c = 0.5, 2-128x6-1 tanh"),
    # the data term of the Burgers problem: points on the initial segment
    # t = 0 (half) and on the walls x = +-1 (half); the network of "burgers"
    "burgers_bc": Workload("burgers_bc", "burgers_bc", _mlp(2, 32, 3, 1), (), [(-1.0, 1.0), (0.0, 1.0)], 256,
                           "Burgers initial/boundary data u + sin(pi x) = 0 on t = 0 and x = +-1"),
}


def boundary_points(N: int, rng: np.random.Generator):
    """Burgers initial/boundary points: half on t = 0 with x uniform on [-1, 1],
    half on the walls x = -1, +1 (alternating) with t uniform on [0, 1]."""
    k = N // 2
    ic = np.stack([rng.uniform(-1.0, 1.0, k), np.zeros(k)], 1)
    wall = np.stack([np.where(np.arange(N - k) % 2 == 0, -1.0, 1.0), rng.uniform(0.0, 1.0, N - k)], 1)
    return np.concatenate([ic, wall]).astype(np.float32)


def xavier_params(dims: Sequence[int], rng: np.random.Generator, bias_std: float = 0.0):
    params = []
    for l in range(len(dims) - 1):
        fan_in, fan_out = dims[l], dims[l + 1]
        std = math.sqrt(2.0 / (fan_in + fan_out))
        W = rng.normal(0.0, std, size=(fan_out, fan_in)).astype(np.float32)
        if bias_std > 0.0:
            b = rng.normal(0.0, bias_std, size=(fan_out,)).astype(np.float32)
        else:
            b = np.zeros((fan_out,), dtype=np.float32)
        params.append((W, b))
    return params


def uniform_points(N: int, domain: Sequence[Tuple[float, float]], rng: np.random.Generator):
    d = len(domain)
    u = rng.random((N, d))
    lo = np.array([a for a, _ in domain])
    hi = np.array([b for _, b in domain])
    return (lo + (hi - lo) * u).astype(np.float32)


@dataclass
class Problem:
    workload: Workload
    params: list                    # [(W float32 (out, in), b float32 (out,)), ...]
    x: np.ndarray                   # (N, d) float32
    coef: Tuple[float, ...]
    channels: list = field(default_factory=list)


def make_problem(name: str, N: Optional[int] = None, seed: int = 0, bias_std: float = 0.0,
                 dims: Optional[Sequence[int]] = None) -> Problem:
    """Workload `name` with its default shape; N and dims may be overridden for tests."""
    wl = WORKLOADS[name]
    if dims is not None or N is not None:
        wl = Workload(wl.name, wl.pde, list(dims) if dims is not None else list(wl.dims), wl.coef,
                      wl.domain, int(N) if N is not None else wl.N, wl.note)
    rng = np.random.Generator(np.random.PCG64(seed))
    params = xavier_params(wl.dims, rng, bias_std)
    x = boundary_points(wl.N, rng) if wl.pde == "burgers_bc" else uniform_points(wl.N, wl.domain, rng)
    return Problem(wl, params, x, wl.coef, CHANNELS[wl.pde])


@dataclass
class EnsembleMember:
    width: int
    hidden: int
    nu: float
    N: int
    params: list
    x: np.ndarray

    @property
    def dims(self) -> List[int]:
        return _mlp(2, self.width, self.hidden, 1)


def make_ensemble(n_nets: int = 64, seed: int = 0, widths=(32, 64, 128, 256), depth=(3, 8),
                  nu_range=(1e-3, 1e-1), n_range=(2048, 65536), bias_std: float = 0.0,
                  with_points: bool = True) -> List[EnsembleMember]:
    """Burgers ensemble: width categorical, hidden depth uniform integer, nu log-uniform,
    N uniform integer (inclusive bounds), on x in [-1, 1], t in [0, 1]."""
    children = np.random.SeedSequence(seed).spawn(n_nets)
    out = []
    dom = WORKLOADS["burgers"].domain
    for ss in children:
        rng = np.random.Generator(np.random.PCG64(ss))
        w = int(rng.choice(np.asarray(widths)))
        H = int(rng.integers(depth[0], depth[1] + 1))
        nu = float(math.exp(rng.uniform(math.log(nu_range[0]), math.log(nu_range[1]))))
        N = int(rng.integers(n_range[0], n_range[1] + 1))
        params = xavier_params(_mlp(2, w, H, 1), rng, bias_std)
        x = uniform_points(N, dom, rng) if with_points else None
        out.append(EnsembleMember(w, H, nu, N, params, x))
    return out


# ---------------------------------------------------------------- training sets
# The paper's complete training runs (Sec. 3.1.1) use an all-points layout: the
# initial-condition, boundary and PDE points are concatenated, evaluated once
# and split afterwards.  A training set is the concatenated points plus the
# list of loss segments over them (the library's segment records: type, begin,
# count, weight, mask, data, param).  Counts default to the paper's; tests pass
# smaller ones.  The paper does not print the Burgers initial profile or the
# term weights; the defaults here are the readings stated with each function.

@dataclass
class TrainingSet:
    name: str
    dims: List[int]
    coef: Tuple[float, ...]
    x: np.ndarray          # (N, d) float32, segments in order
    segments: list
    params: list


def burgers_segments(n_pde: int, n_ic: int, n_pairs: int, w_ic: float = 10.0, w_pde: float = 1.0,
                     w_per: float = 1.0):
    """PDE points, initial points (u(x, 0) = -sin(2 pi x)), then periodic pairs
    (x = 0 and x = 1 at one t) comparing u (channel 0) and u_x (channel 2 of
    the Burgers channel set)."""
    return [dict(type="pde", begin=0, count=n_pde, weight=w_pde),
            dict(type="dirichlet", begin=n_pde, count=n_ic, weight=w_ic, mask=1, data="sin", param=(-1.0, 2.0)),
            dict(type="periodic", begin=n_pde + n_ic, count=2 * n_pairs, weight=w_per, mask=(1 << 0) | (1 << 2))]


def cavity_segments(n_pde: int, n_wall: int, n_lid: int, C: int = 5, w_wall: float = 1.0, w_lid: float = 1.0,
                    w_pde: float = 1.0):
    """PDE points, no-slip wall points (u = v = 0), lid points (u = 1, v = 0)."""
    uv = (1 << 0) | (1 << C)
    return [dict(type="pde", begin=0, count=n_pde, weight=w_pde),
            dict(type="dirichlet", begin=n_pde, count=n_wall, weight=w_wall, mask=uv, data="zero"),
            dict(type="dirichlet", begin=n_pde + n_wall, count=n_lid, weight=w_lid, mask=uv, data="const",
                 param=(1.0, 0.0))]


def burgers_training_set(seed: int = 0, n_pde: int = 10000, n_ic: int = 101, n_pairs: int = 1000,
                         width: int = 64, hidden: int = 6, bias_std: float = 0.0, **weights) -> TrainingSet:
    """Viscous Burgers on (x, t) in [0, 1]^2, nu = 0.01: PDE points uniform,
    initial points on t = 0 at evenly spaced x, periodic time samples uniform
    on [0, 1] with each sample giving the pair (0, t), (1, t)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    dims = _mlp(2, width, hidden, 1)
    params = xavier_params(dims, rng, bias_std)
    pde = rng.random((n_pde, 2))
    ic = np.stack([np.linspace(0.0, 1.0, n_ic), np.zeros(n_ic)], 1)
    t = rng.random(n_pairs)
    pairs = np.stack([np.tile([0.0, 1.0], n_pairs), np.repeat(t, 2)], 1)
    x = np.concatenate([pde, ic, pairs]).astype(np.float32)
    return TrainingSet("burgers", dims, (0.01,), x, burgers_segments(n_pde, n_ic, n_pairs, **weights), params)


def cavity_training_set(seed: int = 0, n_pde: int = 10000, n_wall: int = 1499, n_lid: int = 499,
                        width: int = 64, hidden: int = 6, bias_std: float = 0.0, **weights) -> TrainingSet:
    """Lid-driven cavity on the unit square at Re = 100: PDE points uniform,
    wall points spread over the left, right and bottom sides by arc length,
    lid points uniform on y = 1."""
    rng = np.random.Generator(np.random.PCG64(seed))
    dims = _mlp(2, width, hidden, 3)
    params = xavier_params(dims, rng, bias_std)
    pde = rng.random((n_pde, 2))
    s = 3.0 * rng.random(n_wall)  # arc length along left (0..1), bottom (1..2), right (2..3)
    wall = np.where((s < 1.0)[:, None], np.stack([np.zeros(n_wall), s], 1),
                    np.where((s < 2.0)[:, None], np.stack([s - 1.0, np.zeros(n_wall)], 1),
                             np.stack([np.ones(n_wall), s - 2.0], 1)))
    lid = np.stack([rng.random(n_lid), np.ones(n_lid)], 1)
    x = np.concatenate([pde, wall, lid]).astype(np.float32)
    return TrainingSet("ns", dims, (100.0,), x, cavity_segments(n_pde, n_wall, n_lid, **weights), params)


def modified_params(hidden: int, width: int, harmonics: int, rng: np.random.Generator, d_in: int = 2, d_out: int = 1,
                    bias_std: float = 0.0):
    """Xavier-normal parameters of the modified MLP with periodic embedding, in
    the order (W_U, b_U), (W_V, b_V), (W_1, b_1), .., (W_H, b_H), (W_o, b_o);
    embedding width de = d_in - 1 + 2 harmonics."""
    de = d_in - 1 + 2 * harmonics
    shapes = [(width, de), (width, de), (width, de)] + [(width, width)] * (hidden - 1) + [(d_out, width)]
    out = []
    for fo, fi in shapes:
        W = rng.normal(0.0, math.sqrt(2.0 / (fi + fo)), size=(fo, fi)).astype(np.float32)
        b = (rng.normal(0.0, bias_std, size=(fo,)) if bias_std > 0 else np.zeros(fo)).astype(np.float32)
        out.append((W, b))
    return out


@dataclass
class ModifiedSet:
    hidden: int
    width: int
    harmonics: int
    period: float
    coef: Tuple[float, ...]
    x: np.ndarray           # (N, 2) float32: PDE points, then initial points
    targets: np.ndarray     # (N, 1) float32: initial data at the initial points (0 elsewhere)
    segments: list
    params: list


def ks_training_set(seed: int = 0, n_pde: int = 4096, n_ic: int = 512, width: int = 64, hidden: int = 6,
                    harmonics: int = 1, t_end: float = 1.0, w_ic: float = 1.0, bias_std: float = 0.0) -> ModifiedSet:
    """Kuramoto-Sivashinsky training set of the paper's size (4096 PDE and 512
    initial points), r = u_t + 5 u u_x + 0.5 u_xx + 0.005 u_xxxx, on x in
    [0, 2 pi) (periodic, imposed by the embedding) and t in [0, t_end]; the
    initial data u(x, 0) = cos x (1 + sin x) stands in for the paper's
    reference solution.  Modified MLP with `harmonics` embedding frequencies."""
    rng = np.random.Generator(np.random.PCG64(seed))
    params = modified_params(hidden, width, harmonics, rng, bias_std=bias_std)
    period = 2.0 * math.pi
    pde = np.stack([period * rng.random(n_pde), t_end * rng.random(n_pde)], 1)
    xi = np.arange(n_ic) * (period / n_ic)
    ic = np.stack([xi, np.zeros(n_ic)], 1)
    x = np.concatenate([pde, ic]).astype(np.float32)
    targets = np.zeros((x.shape[0], 1), dtype=np.float32)
    x0 = x[n_pde:, 0].astype(np.float64)
    targets[n_pde:, 0] = (np.cos(x0) * (1.0 + np.sin(x0))).astype(np.float32)
    segs = [dict(type="pde", begin=0, count=n_pde, weight=1.0),
            dict(type="dirichlet", begin=n_pde, count=n_ic, weight=w_ic, mask=1, data="values")]
    return ModifiedSet(hidden, width, harmonics, period, (5.0, 0.5, 0.005), x, targets, segs, params)

"""Channel closure of a residual (the on-demand closure of Sec. 2.2): which
derivative channels every layer has to carry so that the residual's
derivatives can be formed by the jet recursion of Eq. 2-3.

A derivative is written as a tuple of input directions: () is the value,
(i,) the first derivative along x_i, (i, i) the second along x_i, (i, j) with
i != j a mixed second derivative, and so on.  The recursion for a pure
derivative of order k along x_i uses the pure derivatives of orders 1..k-1
along x_i; a mixed second derivative along (x_i, x_j) uses the first
derivatives along x_i and x_j.  Host-side helper: the GPU kernels carry
compile-time channel sets, one per PDE kind (KIND_CHANNELS), `kind_for` names
the kind whose set is exactly a given closure and `resolve_kind` picks the
compiled kind for a residual's derivative list (PinnPlan.for_derivatives).
"""
from __future__ import annotations

from typing import Iterable, List, Optional, Sequence, Tuple

Deriv = Tuple[int, ...]

# The channel sets the compiled kernels carry, in the library's ABI order
# (channel c of output o is jets[o][c]): (direction, order), order 0 the value.
KIND_CHANNELS = {
    "burgers": [(0, 0), (1, 1), (0, 1), (0, 2)],                             # inputs (x, t)
    "ns": [(0, 0), (0, 1), (1, 1), (0, 2), (1, 2)],                          # inputs (x, y)
    "ks": [(0, 0), (1, 1), (0, 1), (0, 2), (0, 3), (0, 4)],                  # inputs (x, t)
    "heat": [(0, 0), (3, 1), (0, 1), (1, 1), (2, 1), (0, 2), (1, 2), (2, 2)],  # inputs (x, y, z, t)
    "aniso": [(0, 0), (0, 1), (1, 1), (0, 2), (1, 2), ((0, 1), 2)],          # inputs (x, y)
    "burgers_bc": [(0, 0)],                                                  # inputs (x, t)
}


def _as_channel(dv: Deriv):
    """Derivative tuple -> the (direction, order) form of the channel lists."""
    if len(dv) == 0:
        return (0, 0)
    if len(set(dv)) == 1:
        return (dv[0], len(dv))
    if len(dv) == 2:
        return ((min(dv), max(dv)), 2)
    raise ValueError(f"mixed derivatives above second order are not supported: {dv}")


def closure(required: Iterable[Deriv]) -> List[Deriv]:
    """The smallest set of derivatives that contains `required` and the value
    and is closed under the recursion; canonical order: the value, then pure
    derivatives by order and direction, then mixed ones."""
    need = {()}
    for dv in required:
        dv = tuple(sorted(dv))
        if len(dv) == 0:
            continue
        if len(set(dv)) == 1:  # pure: all lower orders along that direction
            for k in range(1, len(dv) + 1):
                need.add((dv[0],) * k)
        elif len(dv) == 2:  # mixed second derivative: both first derivatives
            need.update({dv, (dv[0],), (dv[1],)})
        else:
            raise ValueError(f"mixed derivatives above second order are not supported: {dv}")
    pure = sorted((d for d in need if len(set(d)) <= 1 and d), key=lambda d: (len(d), d[0]))
    mixed = sorted(d for d in need if len(set(d)) > 1)
    return [()] + pure + mixed


def channels(required: Iterable[Deriv]) -> list:
    """closure() in the (direction, order) channel form of the oracle and the
    workload definitions."""
    return [_as_channel(dv) for dv in closure(required)]


def kind_for(channel_list: Sequence, kind_channels: dict) -> Optional[str]:
    """The PDE kind whose channel set equals `channel_list` (as sets), or None."""
    want = set(channel_list)
    for kind, chans in kind_channels.items():
        if set(chans) == want:
            return kind
    return None


def resolve_kind(required: Iterable[Deriv], pde: Optional[str] = None) -> Optional[str]:
    """The compiled kind that serves a residual using the derivatives
    `required`: with `pde` given, that kind if its channel set contains the
    closure (else None); without, the one kind whose set equals the closure
    (None if no kind or several do)."""
    want = set(channels(required))
    if pde is not None:
        have = KIND_CHANNELS.get(pde)
        return pde if have is not None and want <= set(have) else None
    hits = [k for k, chans in KIND_CHANNELS.items() if set(chans) == want]
    return hits[0] if len(hits) == 1 else None

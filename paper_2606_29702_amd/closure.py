"""Channel closure of a residual (the on-demand closure of Sec. 2.2): which
derivative channels every layer has to carry so that the residual's
derivatives can be formed by the jet recursion of Eq. 2-3.

A derivative is written as a tuple of input directions: () is the value,
(i,) the first derivative along x_i, (i, i) the second along x_i, (i, j) with
i != j a mixed second derivative, and so on.  The recursion for a pure
derivative of order k along x_i uses the pure derivatives of orders 1..k-1
along x_i; a mixed second derivative along (x_i, x_j) uses the first
derivatives along x_i and x_j.  Host-side helper: the GPU kernels carry
compile-time channel sets, one per PDE kind, and `kind_for` names the kind
whose set is exactly a given closure.
"""
from __future__ import annotations

from typing import Iterable, List, Optional, Sequence, Tuple

Deriv = Tuple[int, ...]


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

"""Pins of the oracle's modified MLP with periodic input embedding (the
Kuramoto-Sivashinsky network of Sec. 3.1.1; the form is stated in the
oracle's header).  Each pin checks it against something other than itself:
nested torch.autograd through the same network written with plain torch
operations, complex-step directional derivatives, the Taylor remainder, exact
periodicity, and the structural zeros of the gated layers when U = V."""
import math

import numpy as np
import pytest
import torch

import oracle
import pinn_inputs as pi
from tests import autograd_ref

KS_CH = pi.CHANNELS["ks"]
KS_COEF = (5.0, 0.5, 0.005)  # the paper's KS coefficients
PERIOD = 2.0 * math.pi


def rel(a, b):
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def mod_params(w=8, H=3, M=2, d=2, dout=1, seed=0, scale=0.6):
    rng = np.random.default_rng(seed)
    de = d - 1 + 2 * M
    shapes = [(w, de), (w, de), (w, de)] + [(w, w)] * (H - 1) + [(dout, w)]
    return [(rng.normal(0, scale, s), rng.normal(0, 0.3, s[0])) for s in shapes]


def ks_points(n, seed=1):
    rng = np.random.default_rng(seed)
    return np.stack([rng.uniform(0, PERIOD, n), rng.uniform(0, 1, n)], 1)


def ks_segments(n_pde, n_ic, w_ic=7.0, w_pde=0.9):
    return [dict(type="pde", begin=0, count=n_pde, weight=w_pde),
            dict(type="dirichlet", begin=n_pde, count=n_ic, weight=w_ic, mask=1, data="values")]


def net(period):
    return lambda p64, X: autograd_ref.modified_mlp(p64, X, period)


@pytest.mark.parametrize("H,M", [(1, 1), (3, 2), (4, 3)])
def test_jets_against_nested_autograd(H, M):
    """All six KS channels (u, u_t, u_x .. u_xxxx) at every point."""
    params = mod_params(H=H, M=M, seed=H)
    x = ks_points(17, seed=M)
    J = oracle.evaluate_mod(params, x, KS_CH, "ks", KS_COEF, PERIOD)
    jets, _ = autograd_ref.nested_jets(autograd_ref.torch_params(params), x, KS_CH, net=net(PERIOD))
    ref = np.stack([np.stack([jets[(0, c)].detach().numpy() for c in range(len(KS_CH))])])
    for c in range(len(KS_CH)):
        assert rel(J[0, c], ref[0, c]) < 1e-12, c


def test_composite_loss_and_gradient_against_nested_autograd():
    """PDE segment at the paper's KS coefficients plus an initial-condition
    segment with per-point target values; segment losses, loss, gradient."""
    params = mod_params(H=3, M=2, seed=5)
    n_pde, n_ic = 23, 9
    x = np.concatenate([ks_points(n_pde, 3), np.stack([np.linspace(0, PERIOD, n_ic), np.zeros(n_ic)], 1)])
    tg = np.cos(x[:, :1]) * (1.0 + np.sin(x[:, :1]))
    segs = ks_segments(n_pde, n_ic)
    _, sl, L, g = oracle.evaluate_mod(params, x, KS_CH, "ks", KS_COEF, PERIOD, segments=segs, targets=tg)
    sl_ref, L_ref, g_ref, _ = autograd_ref.evaluate_segments(params, x, KS_CH, "ks", KS_COEF, segs,
                                                             net=net(PERIOD), targets=tg)
    assert np.allclose(sl, sl_ref, rtol=1e-12, atol=0)
    assert abs(L - L_ref) <= 1e-12 * abs(L_ref)
    assert rel(g, g_ref) < 1e-11


def test_complex_step_and_taylor():
    params = mod_params(H=3, M=2, seed=7)
    n_pde, n_ic = 19, 7
    x = np.concatenate([ks_points(n_pde, 4), np.stack([np.linspace(0, PERIOD, n_ic), np.zeros(n_ic)], 1)])
    tg = np.sin(x[:, :1])
    segs = ks_segments(n_pde, n_ic)
    _, _, L0, g = oracle.evaluate_mod(params, x, KS_CH, "ks", KS_COEF, PERIOD, segments=segs, targets=tg)
    rng = np.random.default_rng(9)
    theta = oracle.pack_theta(params)
    delta = rng.normal(size=theta.size)
    _, dl = oracle.complex_step_mod(params, delta, x, KS_CH, "ks", KS_COEF, PERIOD, segments=segs, targets=tg)
    assert abs(dl - g @ delta) <= 1e-10 * abs(dl)
    # Taylor remainder |L(theta + h delta) - L - h <g, delta>| = O(h^2)

    def unpack(th):
        out, off = [], 0
        for W, b in params:
            W = np.asarray(W)
            nw = W.size
            out.append((th[off:off + nw].reshape(W.shape), th[off + nw:off + nw + W.shape[0]]))
            off += nw + W.shape[0]
        return out

    rem = []
    hs = [1e-2 / 2 ** k for k in range(4)]
    for h in hs:
        _, _, Lh, _ = oracle.evaluate_mod(unpack(theta + h * delta), x, KS_CH, "ks", KS_COEF, PERIOD,
                                          segments=segs, targets=tg, want_grad=False)
        rem.append(abs(Lh - L0 - h * (g @ delta)))
    slopes = [math.log(rem[k] / rem[k + 1]) / math.log(2.0) for k in range(len(hs) - 1)]
    assert all(1.8 < s < 2.2 for s in slopes), slopes


def test_jet_tangents_by_complex_step():
    """Directional derivatives of every jet channel in parameter space: the
    complex-step tangent of the oracle against central differences of nested
    autograd jets (a second, independent route)."""
    params = mod_params(H=2, M=2, seed=11)
    x = ks_points(9, 5)
    rng = np.random.default_rng(2)
    theta = oracle.pack_theta(params)
    delta = rng.normal(size=theta.size)
    dJ, _ = oracle.complex_step_mod(params, delta, x, KS_CH, "ks", KS_COEF, PERIOD)

    def jets_at(th):
        p = []
        off = 0
        for W, b in params:
            W = np.asarray(W)
            p.append((th[off:off + W.size].reshape(W.shape), th[off + W.size:off + W.size + W.shape[0]]))
            off += W.size + W.shape[0]
        js, _ = autograd_ref.nested_jets(autograd_ref.torch_params(p, requires_grad=False), x, KS_CH,
                                         net=net(PERIOD))
        return np.stack([js[(0, c)].detach().numpy() for c in range(len(KS_CH))])

    h = 1e-5
    fd = (jets_at(theta + h * delta) - jets_at(theta - h * delta)) / (2 * h)
    assert rel(dJ[0], fd) < 1e-7


def test_periodic_in_x():
    """The embedding makes every jet channel exactly periodic in x with the
    stated period (up to FP64 rounding of the shifted argument)."""
    params = mod_params(H=3, M=3, seed=13)
    x = ks_points(11, 6)
    J0 = oracle.evaluate_mod(params, x, KS_CH, "ks", KS_COEF, PERIOD)
    x2 = x.copy()
    x2[:, 0] += PERIOD
    J1 = oracle.evaluate_mod(params, x2, KS_CH, "ks", KS_COEF, PERIOD)
    assert rel(J1, J0) < 1e-12
    x3 = x.copy()
    x3[:, 0] += 0.5 * PERIOD  # half a period is not a symmetry
    assert rel(oracle.evaluate_mod(params, x3, KS_CH, "ks", KS_COEF, PERIOD), J0) > 1e-2


def test_equal_encoders_make_the_gated_layers_inert():
    """With U = V every gated layer outputs U whatever Z is: the network is
    W_o U + b_o, the gradient of every hidden layer (W_1 .. W_H) is exactly
    zero, and the jets equal those of the one-layer network on the embedding."""
    params = mod_params(H=3, M=2, seed=17)
    params[1] = (params[0][0].copy(), params[0][1].copy())
    n_pde, n_ic = 15, 5
    x = np.concatenate([ks_points(n_pde, 8), np.stack([np.linspace(0, PERIOD, n_ic), np.zeros(n_ic)], 1)])
    tg = np.cos(x[:, :1])
    J, _, _, g = oracle.evaluate_mod(params, x, KS_CH, "ks", KS_COEF, PERIOD, segments=ks_segments(n_pde, n_ic),
                                     targets=tg)
    sizes = [np.asarray(W).size + np.asarray(W).shape[0] for W, _ in params]
    off = np.cumsum([0] + sizes)
    assert np.all(g[off[2]:off[-2]] == 0.0)  # W_1, b_1 .. W_H, b_H
    assert np.linalg.norm(g[off[0]:off[2]]) > 0 and np.linalg.norm(g[off[-2]:]) > 0
    # one-layer network: params (W_U, b_U) then the output layer
    one = [params[0], params[-1]]
    jets, _ = autograd_ref.nested_jets(
        autograd_ref.torch_params(one, requires_grad=False), x, KS_CH,
        net=lambda p64, X: torch.tanh(_embed(X, PERIOD, 2) @ p64[0][0].T + p64[0][1]) @ p64[1][0].T + p64[1][1])
    ref = np.stack([jets[(0, c)].detach().numpy() for c in range(len(KS_CH))])
    assert rel(J[0], ref) < 1e-12


def _embed(X, period, M):
    om = 2.0 * math.pi / period
    feats = [X[:, 1:2]]
    for m in range(1, M + 1):
        feats += [torch.cos(m * om * X[:, 0:1]), torch.sin(m * om * X[:, 0:1])]
    return torch.cat(feats, dim=1)

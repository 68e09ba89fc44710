"""Nested torch.autograd reference, the paper's AD baseline (Sec. 3.1.1): the
network is evaluated as a plain tanh MLP and every coordinate derivative the
residual needs is obtained by repeated autograd.grad calls.  FP64 on the CPU.
Used only to pin the oracle; it is a library route independent of both the
oracle's jet recursion and the GPU kernels."""
import math

import numpy as np
import torch


def mlp(params64, X, act=torch.tanh):
    h = X
    L = len(params64)
    for l, (W, b) in enumerate(params64):
        h = h @ W.T + b
        if l < L - 1:
            h = act(h)
    return h


def torch_params(params, requires_grad=True):
    out = []
    for W, b in params:
        Wt = torch.tensor(np.asarray(W, dtype=np.float64), requires_grad=requires_grad)
        bt = torch.tensor(np.asarray(b, dtype=np.float64), requires_grad=requires_grad)
        out.append((Wt, bt))
    return out


def modified_mlp(params64, X, period, act=torch.tanh):
    """The modified MLP with periodic embedding in x_0 (the form documented in
    the oracle's header), written with plain torch operations."""
    (WU, bU), (WV, bV) = params64[0], params64[1]
    de = WU.shape[1]
    d = X.shape[1]
    M = (de - d + 1) // 2
    om = 2.0 * math.pi / period
    feats = [X[:, j:j + 1] for j in range(1, d)]
    for m in range(1, M + 1):
        feats += [torch.cos(m * om * X[:, 0:1]), torch.sin(m * om * X[:, 0:1])]
    E = torch.cat(feats, dim=1)
    U = act(E @ WU.T + bU)
    V = act(E @ WV.T + bV)
    W1, b1 = params64[2]
    h = act(E @ W1.T + b1)
    for W, b in params64[3:-1]:
        Z = act(h @ W.T + b)
        h = (1.0 - Z) * U + Z * V
    Wo, bo = params64[-1]
    return h @ Wo.T + bo


def nested_jets(params64, x, channels, act=torch.tanh, net=None):
    """Returns (jets dict {(o, c): tensor (N,)}, X) with a graph kept for backward.
    net(params64, X) evaluates the network (default: the plain MLP)."""
    X = torch.tensor(np.asarray(x, dtype=np.float64), requires_grad=True)
    U = mlp(params64, X, act) if net is None else net(params64, X)
    jets = {}
    for o in range(U.shape[1]):
        u = U[:, o]
        for c, (dr, k) in enumerate(channels):
            if k == 0:
                jets[(o, c)] = u
                continue
            g = u
            dirs = list(dr) if isinstance(dr, tuple) else [dr] * k  # mixed: ((i, j), 2)
            for d_ in dirs:
                g = torch.autograd.grad(g.sum(), X, create_graph=True)[0][:, d_]
            jets[(o, c)] = g
    return jets, X


def residuals(pde, jets, channels, X, coef):
    idx = {ch: c for c, ch in enumerate(channels)}

    def J(o, dr, k):
        return jets[(o, idx[(0, 0)] if k == 0 else idx[(dr, k)])]

    if pde == "burgers":  # inputs (x, t)
        nu = coef[0]
        return [J(0, 1, 1) + J(0, 0, 0) * J(0, 0, 1) - nu * J(0, 0, 2)]
    if pde == "ns":  # Eq. 16, inputs (x, y), outputs (u, v, p)
        Re = coef[0]
        u, v = J(0, 0, 0), J(1, 0, 0)
        rc = J(0, 0, 1) + J(1, 1, 1)
        ru = u * J(0, 0, 1) + v * J(0, 1, 1) + J(2, 0, 1) - (J(0, 0, 2) + J(0, 1, 2)) / Re
        rv = u * J(1, 0, 1) + v * J(1, 1, 1) + J(2, 1, 1) - (J(1, 0, 2) + J(1, 1, 2)) / Re
        return [rc, ru, rv]
    if pde == "ks":  # inputs (x, t)
        a, b, g = coef
        return [J(0, 1, 1) + a * J(0, 0, 0) * J(0, 0, 1) + b * J(0, 0, 2) + g * J(0, 0, 4)]
    if pde == "burgers_bc":  # inputs (x, t): u + sin(pi x) on the initial and boundary segments
        return [J(0, 0, 0) + torch.sin(math.pi * X.detach()[:, 0])]
    if pde == "aniso":  # inputs (x, y): u_xx + 2 c u_xy + u_yy
        c = coef[0]
        return [J(0, 0, 2) + 2.0 * c * jets[(0, idx[((0, 1), 2)])] + J(0, 1, 2)]
    if pde == "heat":  # inputs (x, y, z, t)
        ka = coef[0]
        Xd = X.detach()
        f = (torch.sin(math.pi * Xd[:, 0]) * torch.sin(math.pi * Xd[:, 1]) *
             torch.sin(math.pi * Xd[:, 2]) * torch.exp(-Xd[:, 3]))
        return [J(0, 3, 1) - ka * (J(0, 0, 2) + J(0, 1, 2) + J(0, 2, 2)) - f]
    raise ValueError(pde)


def evaluate(params, x, channels, pde, coef, act=torch.tanh):
    """(jets (d_out, C, N), r (n_res, N), loss, grad packed W,b per layer) in FP64."""
    p64 = torch_params(params)
    jets, X = nested_jets(p64, x, channels, act)
    rs = residuals(pde, jets, channels, X, coef)
    N = X.shape[0]
    loss = sum((r * r).sum() / N for r in rs)
    leaves = [t for pair in p64 for t in pair]
    grads = torch.autograd.grad(loss, leaves, allow_unused=True)
    grads = [torch.zeros_like(t) if g is None else g for g, t in zip(grads, leaves)]
    d_out = params[-1][0].shape[0]
    C = len(channels)
    J = np.stack([np.stack([jets[(o, c)].detach().numpy() for c in range(C)]) for o in range(d_out)])
    R = np.stack([r.detach().numpy() for r in rs])
    G = np.concatenate([g.detach().numpy().reshape(-1) for g in grads])
    return J, R, float(loss.detach()), G


def evaluate_segments(params, x, channels, pde, coef, segments, act=torch.tanh, net=None, targets=None):
    """The composite loss of Sec. 3.1.1 written with nested autograd in FP64:
    all points through the network at once, outputs split by segment; each
    segment's mean of squared terms times its weight.  Returns (seg_losses,
    loss, grad packed W, b per layer)."""
    p64 = torch_params(params)
    jets, X = nested_jets(p64, x, channels, act, net)
    idx = {ch: c for c, ch in enumerate(channels)}
    d_out = params[-1][0].shape[0]
    C = len(channels)
    terms = []
    for s in segments:
        b, n = s["begin"], s["count"]
        sl = slice(b, b + n)
        if s["type"] == "pde":
            rs = residuals(pde, {k: v[sl] for k, v in jets.items()}, channels, X[sl], coef)
            t = sum((r * r).sum() for r in rs) / n
        elif s["type"] == "dirichlet":
            par = list(s.get("param", ())) + [0.0] * 4
            xs = X.detach()[sl, 0]
            t = 0.0
            for o in range(d_out):
                if not (s["mask"] >> (o * C)) & 1:
                    continue
                if s.get("data", "zero") == "const":
                    g = torch.full_like(xs, par[o])
                elif s.get("data", "zero") == "sin":
                    g = par[0] * torch.sin(par[1] * math.pi * xs)
                elif s.get("data", "zero") == "values":
                    g = torch.tensor(np.asarray(targets, dtype=np.float64)[b:b + n, o])
                else:
                    g = torch.zeros_like(xs)
                r = jets[(o, idx[(0, 0)])][sl] - g
                t = t + (r * r).sum()
            t = t / n
        else:  # periodic pairs: first minus second of each consecutive pair
            t = 0.0
            for o in range(d_out):
                for c in range(C):
                    if not (s["mask"] >> (o * C + c)) & 1:
                        continue
                    v = jets[(o, c)][sl]
                    r = v[0::2] - v[1::2]
                    t = t + (r * r).sum()
            t = t / (n // 2)
        terms.append(t)
    loss = sum(s.get("weight", 1.0) * t for s, t in zip(segments, terms))
    leaves = [t for pair in p64 for t in pair]
    grads = torch.autograd.grad(loss, leaves, allow_unused=True)
    grads = [torch.zeros_like(t) if g is None else g for g, t in zip(grads, leaves)]
    G = np.concatenate([g.detach().numpy().reshape(-1) for g in grads])
    J = np.stack([np.stack([jets[(o, c)].detach().numpy() for c in range(C)]) for o in range(d_out)])
    return np.array([float(t.detach()) for t in terms]), float(loss.detach()), G, J

#!/usr/bin/env python3
"""Throughput of the partial-jet PINN step on one MI355X.

A step is the whole hot path on one batch of collocation points: forward
partial-jet pass through every layer, residual, mean-squared loss and the
hand-written adjoint down to dL/dtheta.  Inputs (network parameters and points)
are resident in device memory before the timed region starts.

Default workload (the headline): the 64-network viscous Burgers ensemble of
seed 0.  Widths are drawn from {32, 64, 128, 256}, depths from 3 to 8, nu
log-uniform on [1e-3, 1e-1], N uniform on [2048, 65536] per network (2,091,275
points in all).  It is stepped with BF16 GEMM operands by the grouped batch
(pinn_batch_step: one launch per phase for all networks, captured in one HIP
graph), against 64 sequential calls of the plain FP32 jet path on the same
GPU.  Beside it: the FP64 CPU oracle on the host cores (all of them, and one),
the BF16 error against that oracle per member, and legs for the steady
Navier-Stokes and 3-D heat workloads.

Prints one JSON line.
"""
import argparse
import json
import math
import os
import platform
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "collocation pts/s, residual+dθ step: BF16/batched vs plain FP32 jet, same GPU"
PEAK = {"bf16": 2500.0, "fp16": 2500.0, "fp32": 157.3}  # dense MFMA TFLOP/s
HBM_PEAK = 8000.0  # GB/s
GEMM_CLASSES = ("layer_fwd", "layer_bwd", "dw_hidden", "bwd_dw", "out_bwd")
ALL_CLASSES = ("layer_fwd", "layer_bwd", "dw_hidden", "bwd_dw", "out_fwd", "out_bwd", "seed_fwd", "other")


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def source_hash():
    """Hash of the HIP library sources, to tie counter figures to the kernels they measured."""
    import hashlib
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2606_29702_amd", "csrc")
    for f in sorted(os.listdir(d)):
        if f.endswith((".hip", ".hpp", ".cpp")):
            h.update(f.encode())
            with open(os.path.join(d, f), "rb") as fh:
                h.update(fh.read())
    return h.hexdigest()[:16]


def profiled_traffic(workload, prec, kernel_class):
    """HBM bytes per launch of a kernel class from the committed rocprofv3
    counter summary (FETCH_SIZE + WRITE_SIZE, copy-calibrated), or None when
    there is none for this workload or the kernels changed since it was taken."""
    path = os.path.join(ROOT, "profiles", f"{workload}_{prec}_hbm_bytes.md")
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as fh:
        for line in fh:
            if " = " in line:
                k, v = line.strip().split(" = ", 1)
                vals[k.strip()] = v.strip()
    if vals.get("source_sha256") != source_hash() or kernel_class not in vals:
        return None
    return float(vals[kernel_class])


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def copy_probe(mib):
    """A plain device copy of known size (calibration of the HBM byte counters)."""
    import torch
    n = mib * (1 << 20) // 4
    src = torch.ones(n, device="cuda", dtype=torch.float32)
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    log(f"copy probe: {mib} MiB read + {mib} MiB written per copy, 3 copies")


# --------------------------------------------------------------------------- algorithmic work
def gemm_unit(w, C, N):
    """G = 2 w^2 C N: one stacked-channel w x w GEMM over N points."""
    return 2.0 * w * w * C * N


def class_flops(w, H, C, N, fused):
    """Algorithmic hidden-layer GEMM flops per step by kernel class (the z
    recompute of the backward kernels is a design cost and not counted):
      forward           (H - 1) G            [layer_fwd]
      fused backward    top layer dW: G       [out_bwd]
                        layers H-1..2: 2 G    [bwd_dw]   (adjoint GEMM + dW)
                        layer 1 adjoint: G    [layer_bwd]
      separate backward dW per layer: G       [dw_hidden] x (H - 1)
                        adjoint per layer: G  [layer_bwd] x (H - 1)
    Both add up to 3 (H - 1) G."""
    G = gemm_unit(w, C, N)
    f = dict.fromkeys(ALL_CLASSES, 0.0)
    f["layer_fwd"] = (H - 1) * G
    if H < 2:
        return f
    if fused:
        f["out_bwd"] = G
        f["bwd_dw"] = 2 * (H - 2) * G
        f["layer_bwd"] = G
    else:
        f["dw_hidden"] = (H - 1) * G
        f["layer_bwd"] = (H - 1) * G
    return f


def class_stack_bytes(w, H, C, N_pad, fused, osz):
    """The design's stack traffic per step by kernel class (bytes): the layer
    stacks ([N_pad][C][w], osz bytes per element) each class reads or writes
    once.  It is a design cost (the algorithmic minimum is x, r and dtheta);
    it bounds the MFMA fraction a class can reach when its stacks come from
    HBM:
      forward (store-all)  writes A_1 .. A_H                     H stacks
      separate backward    adjoint, layers H .. 3: reads Zbar_l and A_{l-2}
                           (z recompute), writes Zbar_{l-1};  layer 2 reads
                           Zbar_2 (first-layer gradient from x)  3 (H - 2) + 1
                           dW per layer: Zbar_l and A_{l-1}      2 (H - 1)
                           top layer: A_{H-1} in, Zbar_H out     2
      fused backward       layers H-1 .. 2: Zbar_l, A_{l-1}, A_{l-2} in,
                           Zbar_{l-1} out                        4 (H - 2)
                           top layer with its dW                 2
                           layer 1 adjoint                       1"""
    S = float(C) * w * osz * N_pad
    b = dict.fromkeys(ALL_CLASSES, 0.0)
    b["layer_fwd"] = H * S
    if H < 2:
        return b
    b["out_bwd"] = 2 * S
    if fused:
        b["bwd_dw"] = 4 * (H - 2) * S
        b["layer_bwd"] = S
    else:
        b["layer_bwd"] = (3 * (H - 2) + 1) * S
        b["dw_hidden"] = 2 * (H - 1) * S
    return b


def roofline_from(cls, flops_per_step, cls_ms, launches, prec, workload, steps_timed, stack_bytes_per_step=None):
    """Dominant kernel class roofline: algorithmic flops per launch over the
    average launch time measured with HIP events.  With the class's design
    stack traffic, also the HBM fraction that traffic takes and the MFMA
    fraction it would allow at the HBM peak (the bound that applies when the
    stacks stream from HBM)."""
    avg_ms = cls_ms / max(launches, 1)
    per_launch = flops_per_step * steps_timed / max(launches, 1)
    achieved = per_launch / (avg_ms * 1e-3) / 1e12
    traffic = profiled_traffic(workload, prec, cls)
    out = dict(bound="mfma", achieved=round(achieved, 3), peak=PEAK[prec], unit="TFLOP/s",
               frac=round(achieved / PEAK[prec], 5), traffic=None if traffic is None else round(traffic),
               traffic_unit="bytes per launch (HBM, rocprofv3 FETCH_SIZE + WRITE_SIZE)",
               kernel_class=cls, avg_launch_us=round(avg_ms * 1e3, 2), launches=launches,
               flops_per_launch=per_launch,
               hbm_frac=None if traffic is None else round(traffic / (avg_ms * 1e-3) / 1e9 / HBM_PEAK, 4))
    if stack_bytes_per_step:
        sb = stack_bytes_per_step * steps_timed / max(launches, 1)
        out["stack_bytes_per_launch"] = round(sb)
        out["stack_hbm_frac"] = round(sb / (avg_ms * 1e-3) / 1e9 / HBM_PEAK, 4)
        out["stack_bound_mfma_frac"] = round(min(1.0, (per_launch / sb) / (PEAK[prec] * 1e12 / (HBM_PEAK * 1e9))), 4)
    return out


# --------------------------------------------------------------------------- the ensemble
def ensemble_inputs(seed=0):
    import torch
    import pinn_inputs as pi
    ens = pi.make_ensemble(seed=seed)
    params = [[(torch.tensor(W, device="cuda"), torch.tensor(b, device="cuda")) for W, b in m.params] for m in ens]
    xs = [torch.tensor(m.x, device="cuda") for m in ens]
    return ens, params, xs


def time_batch(batch, params, xs, steps, warmup):
    import torch
    for _ in range(max(warmup, 1)):
        batch.step(params, xs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        batch.step(params, xs)
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1e3 / steps


def ensemble_headline(ens, params, xs, prec, steps, warmup, runs, replays, counter_window=0):
    """The grouped BF16 ensemble step: autotuned, then exactly `steps` timed graph
    replays; the kernel class with the most time is then timed with events
    over `steps` eager steps of the same schedule."""
    import torch
    from paper_2606_29702_amd import PinnBatch
    batch = PinnBatch([m.dims for m in ens], "burgers", [(m.nu,) for m in ens], [m.N for m in ens], precision=prec)
    t0 = time.perf_counter()
    lanes, _ = batch.autotune(params, xs, reps=3)
    tune_s = time.perf_counter() - t0
    ms = time_batch(batch, params, xs, steps, warmup)
    # timing protocol: independent runs of many replays, median per run
    per_run = [time_batch(batch, params, xs, replays, 3) for _ in range(runs)]
    # kernel classes: one eager step each, then the dominant class over `steps`
    # steps.  Timed with the lanes on one stream, so that no two launches
    # overlap and each class's events bracket only its own kernels.
    cfg = batch.config()
    batch.configure(1, use_graph=cfg["graph"], per_network=False)
    class_ms = {}
    for cls in ALL_CLASSES:
        batch.profile(cls)
        batch.step(params, xs)
        class_ms[cls] = batch.profile_read()
    batch.profile("off")
    dom = max(GEMM_CLASSES, key=lambda c: class_ms[c][0])
    batch.profile(dom)
    for _ in range(steps):
        batch.step(params, xs)
    dom_ms, dom_n = batch.profile_read()
    batch.profile("off")
    batch.configure(cfg["streams"], use_graph=cfg["graph"], per_network=cfg["per_network"],
                    width_lanes=cfg["width_lanes"])
    batch.step(params, xs)
    tunings = [batch.tuning(i) for i in range(len(ens))]
    launches = batch.launches()
    lanes = batch.config()
    if counter_window:
        # the last GPU work of the run: `counter_window` eager steps on one
        # stream, whose dispatches a profiler run maps to kernel classes
        batch.configure(1, use_graph=False, per_network=False)
        batch.step(params, xs)
        torch.cuda.synchronize()
        classes = batch.schedule_classes()
        for _ in range(counter_window):
            batch.step(params, xs)
        torch.cuda.synchronize()
        log("counter window: " + json.dumps({"steps": counter_window, "classes": classes}))
    batch.close()
    flops = dict.fromkeys(ALL_CLASSES, 0.0)
    stack_bytes = dict.fromkeys(ALL_CLASSES, 0.0)
    osz = 4 if prec == "fp32" else 2
    for m, t in zip(ens, tunings):
        fused = bool(t["bwd_fused"]) and m.width <= 128
        for k, v in class_flops(m.width, m.hidden, 4, m.N, fused).items():
            flops[k] += v
        for k, v in class_stack_bytes(m.width, m.hidden, 4, -(-m.N // 128) * 128, fused, osz).items():
            stack_bytes[k] += v
    total_flops = sum(flops.values())
    return dict(ms=ms, per_run_ms=per_run, lanes=lanes, tune_s=tune_s, class_ms=class_ms, dominant=dom,
                dom_ms=dom_ms, dom_n=dom_n, flops=flops, total_flops=total_flops, launches=launches,
                tunings=tunings, stack_bytes=stack_bytes)


def tunings_by_width(ens, tunings):
    """How many members of each width the autotuner gave each tiling."""
    out = {}
    for m, t in zip(ens, tunings):
        key = f"fwd{t['fwd_points']}/{'fused' if t['bwd_fused'] and m.width <= 128 else 'split'}" + (
            f"/bwd{t['bwd_points']}" if m.width >= 256 else "")
        d = out.setdefault(str(m.width), {})
        d[key] = d.get(key, 0) + 1
    return out


def ensemble_fp32_sequential(ens, params, xs, steps):
    """The plain FP32 jet path, one network after another on one stream."""
    import torch
    from paper_2606_29702_amd import PinnPlan
    plans = [PinnPlan(m.dims, "burgers", m.N, precision="fp32", coef=(m.nu,)) for m in ens]
    for pl, p, x in zip(plans, params, xs):
        pl.autotune(p, x, reps=3)

    def seq():
        for pl, p, x in zip(plans, params, xs):
            pl.residual(p, x)
            pl.backward(p, x)

    seq()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        seq()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    for pl in plans:
        pl.close()
    return ms


def ensemble_cpu_baseline(ens, target_s, threads):
    """The FP64 oracle on the same mix of networks: the first ceil(f N_i)
    points of every member, f chosen for about target_s seconds.  The sample
    is cut into pieces of at most 256 points of one member, and `threads`
    host threads take the pieces (each oracle call single-threaded), so every
    thread works whatever the sample size."""
    from concurrent.futures import ThreadPoolExecutor
    import oracle
    import pinn_inputs as pi
    ch = pi.CHANNELS["burgers"]

    def piece(task):
        m, a, b = task
        oracle.evaluate(m.params, m.x[a:b], ch, "burgers", (m.nu,), want_jets=False, threads=1)
        return b - a

    def run(f):
        tasks = []
        for m in sorted(ens, key=lambda m: -m.width * m.width * m.hidden * m.N):
            n = max(1, int(math.ceil(f * m.N)))
            tasks += [(m, a, min(n, a + 256)) for a in range(0, n, 256)]
        t0 = time.perf_counter()
        if threads > 1:
            with ThreadPoolExecutor(threads) as ex:
                n_tot = sum(ex.map(piece, tasks))
        else:
            n_tot = sum(map(piece, tasks))
        return n_tot, time.perf_counter() - t0

    f = 1e-4
    n, dt = run(f)
    while dt < 0.5 and f < 1.0:
        f *= 4
        n, dt = run(f)
    for _ in range(2):  # fixed per-piece costs make the first scaling short of the target
        f = min(1.0, f * target_s / dt)
        n, dt = run(f)
        if dt >= 0.6 * target_s or f >= 1.0:
            break
    return dict(value=round(n / dt, 1), unit="pts/s", cores=threads, kind="oracle",
                sample=f"first {f:.2%} of the points of each of the {len(ens)} networks ({n} points), "
                       f"residual + loss + dtheta in FP64 ({dt:.1f} s)")


def ensemble_accuracy(ens, prec, n_pts=256):
    """Each member on its first n_pts points: the GPU path against the oracle."""
    import numpy as np
    import torch
    import oracle
    import pinn_inputs as pi
    from paper_2606_29702_amd import PinnPlan
    worst_r = worst_g = 0.0
    min_cos = 1.0
    for m in ens:
        x_np = m.x[:n_pts]
        plan = PinnPlan(m.dims, "burgers", n_pts, precision=prec, coef=(m.nu,))
        params = [(torch.tensor(W, device="cuda"), torch.tensor(b, device="cuda")) for W, b in m.params]
        x = torch.tensor(x_np, device="cuda")
        r, _, _, _ = plan.residual(params, x)
        grads = plan.backward(params, x)
        torch.cuda.synchronize()
        g = np.concatenate([np.concatenate([dW.double().cpu().numpy().ravel(), db.double().cpu().numpy().ravel()])
                            for dW, db in grads])
        ref = oracle.evaluate(m.params, x_np, pi.CHANNELS["burgers"], "burgers", (m.nu,), want_jets=False)
        plan.close()
        worst_r = max(worst_r, float(np.linalg.norm(r.double().cpu().numpy() - ref.r) / np.linalg.norm(ref.r)))
        worst_g = max(worst_g, float(np.linalg.norm(g - ref.grad) / np.linalg.norm(ref.grad)))
        min_cos = min(min_cos, float(g @ ref.grad / (np.linalg.norm(g) * np.linalg.norm(ref.grad))))
    return dict(points_per_member=n_pts, members=len(ens), worst_r_rel_l2=worst_r, worst_grad_rel_l2=worst_g,
                min_grad_cosine=min_cos)


# --------------------------------------------------------------------------- single-network legs
def time_plan(prob, prec, steps, warmup, save_cap=0, tuning=None):
    """A single-network step: autotuned (or given tuning), `steps` timed eager
    steps with the dominant kernel class bracketed by events."""
    import torch
    from paper_2606_29702_amd import PinnPlan
    wl = prob.workload
    N = prob.x.shape[0]
    plan = PinnPlan(wl.dims, wl.pde, N, precision=prec, coef=prob.coef, save_cap_bytes=save_cap)
    params = [(torch.tensor(W, device="cuda"), torch.tensor(b, device="cuda")) for W, b in prob.params]
    x = torch.tensor(prob.x, device="cuda")

    def step():
        plan.residual(params, x)
        plan.backward(params, x)

    if tuning is None:
        tuning, _ = plan.autotune(params, x, reps=3)
    else:
        plan.set_tuning(*tuning)
        tuning = plan.tuning()
    for _ in range(max(warmup, 1)):
        step()
    torch.cuda.synchronize()
    class_ms = {}
    for cls in ALL_CLASSES:
        plan.profile(cls)
        step()
        class_ms[cls] = plan.profile_read()
    plan.profile("off")
    dom = max(GEMM_CLASSES, key=lambda c: class_ms[c][0])
    plan.profile(dom)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    dom_ms, dom_n = plan.profile_read()
    plan.profile("off")
    plan.close()
    return dict(ms=ms, class_ms=class_ms, dominant=dom, dom_ms=dom_ms, dom_n=dom_n, tuning=tuning)


def nested_autograd_fp32(prob, steps):
    """The paper's AD baseline (Sec. 3.1.1): coordinate derivatives by nested
    torch.autograd through a plain tanh MLP, then reverse mode for dtheta.
    FP32 on the GPU; context only (NS residual, Eq. 16)."""
    import torch
    assert prob.workload.pde == "ns"
    Re = prob.coef[0]
    params = [(torch.tensor(W, device="cuda", requires_grad=True), torch.tensor(b, device="cuda", requires_grad=True))
              for W, b in prob.params]
    X0 = torch.tensor(prob.x, device="cuda")

    def step():
        X = X0.clone().requires_grad_(True)
        h = X
        for l, (W, b) in enumerate(params):
            h = h @ W.T + b
            if l < len(params) - 1:
                h = torch.tanh(h)
        d = {}
        for o in range(3):
            g = torch.autograd.grad(h[:, o].sum(), X, create_graph=True)[0]
            d[o, "x"], d[o, "y"] = g[:, 0], g[:, 1]
            d[o, "xx"] = torch.autograd.grad(d[o, "x"].sum(), X, create_graph=True)[0][:, 0]
            d[o, "yy"] = torch.autograd.grad(d[o, "y"].sum(), X, create_graph=True)[0][:, 1]
        u, v = h[:, 0], h[:, 1]
        rc = d[0, "x"] + d[1, "y"]
        ru = u * d[0, "x"] + v * d[0, "y"] + d[2, "x"] - (d[0, "xx"] + d[0, "yy"]) / Re
        rv = u * d[1, "x"] + v * d[1, "y"] + d[2, "y"] - (d[1, "xx"] + d[1, "yy"]) / Re
        N = X.shape[0]
        loss = ((rc * rc).sum() + (ru * ru).sum() + (rv * rv).sum()) / N
        return torch.autograd.grad(loss, [t for p in params for t in p])

    step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1e3 / steps


def nested_autograd_training(ts, steps, lr=1e-3):
    """The paper's AD baseline for a complete training step (Sec. 3.1.1): the
    composite loss (all points through the network at once, outputs split by
    segment) with coordinate derivatives by nested torch.autograd, reverse
    mode for dtheta and torch.optim.Adam.  FP32 on the GPU; returns ms per step."""
    import torch
    params = [t for W, b in ts.params for t in (torch.tensor(W, device="cuda", requires_grad=True),
                                                 torch.tensor(b, device="cuda", requires_grad=True))]
    opt = torch.optim.Adam(params, lr=lr)
    X0 = torch.tensor(ts.x, device="cuda")
    L = len(params) // 2

    def d(f, X, i):
        return torch.autograd.grad(f.sum(), X, create_graph=True)[0][:, i]

    def step():
        X = X0.clone().requires_grad_(True)
        h = X
        for l in range(L):
            h = h @ params[2 * l].T + params[2 * l + 1]
            if l < L - 1:
                h = torch.tanh(h)
        loss = 0.0
        if ts.name == "burgers":
            u = h[:, 0]
            u_x, u_t = d(u, X, 0), d(u, X, 1)
            u_xx = d(u_x, X, 0)
            for sg in ts.segments:
                a, n, w = sg["begin"], sg["count"], sg["weight"]
                if sg["type"] == "pde":
                    r = u_t[a:a + n] + u[a:a + n] * u_x[a:a + n] - ts.coef[0] * u_xx[a:a + n]
                    loss = loss + w * (r * r).mean()
                elif sg["type"] == "dirichlet":
                    amp, k = sg["param"][0], sg["param"][1]
                    r = u[a:a + n] - amp * torch.sin(k * math.pi * X0[a:a + n, 0])
                    loss = loss + w * (r * r).mean()
                else:
                    uu, ux = u[a:a + n], u_x[a:a + n]
                    loss = loss + w * (((uu[0::2] - uu[1::2]) ** 2 + (ux[0::2] - ux[1::2]) ** 2).mean())
        else:
            Re = ts.coef[0]
            g = {}
            for o in range(3):
                g[o, "x"], g[o, "y"] = d(h[:, o], X, 0), d(h[:, o], X, 1)
                if o < 2:
                    g[o, "xx"], g[o, "yy"] = d(g[o, "x"], X, 0), d(g[o, "y"], X, 1)
            u, v = h[:, 0], h[:, 1]
            for sg in ts.segments:
                a, n, w = sg["begin"], sg["count"], sg["weight"]
                sl = slice(a, a + n)
                if sg["type"] == "pde":
                    rc = g[0, "x"][sl] + g[1, "y"][sl]
                    ru = (u[sl] * g[0, "x"][sl] + v[sl] * g[0, "y"][sl] + g[2, "x"][sl]
                          - (g[0, "xx"][sl] + g[0, "yy"][sl]) / Re)
                    rv = (u[sl] * g[1, "x"][sl] + v[sl] * g[1, "y"][sl] + g[2, "y"][sl]
                          - (g[1, "xx"][sl] + g[1, "yy"][sl]) / Re)
                    loss = loss + w * (rc * rc + ru * ru + rv * rv).mean()
                else:
                    par = list(sg.get("param", ())) + [0.0, 0.0]
                    u0 = par[0] if sg.get("data") == "const" else 0.0
                    v0 = par[1] if sg.get("data") == "const" else 0.0
                    loss = loss + w * ((u[sl] - u0) ** 2 + (v[sl] - v0) ** 2).mean()
        opt.zero_grad(set_to_none=False)
        grads = torch.autograd.grad(loss, params)
        for p_, g_ in zip(params, grads):
            p_.grad = g_
        opt.step()

    for _ in range(3):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1e3 / steps


def ks_training_leg(steps):
    """The paper's KS training run (Sec. 3.1.1) on the modified MLP with
    periodic embedding: `steps` Adam steps on the composite loss (4096 PDE
    points + 512 initial points), FP32, eager calls."""
    import torch
    import pinn_inputs as pi
    from paper_2606_29702_amd import AdamState, ModifiedPlan
    ts = pi.ks_training_set(seed=0)
    N = ts.x.shape[0]
    plan = ModifiedPlan(ts.hidden, ts.width, ts.harmonics, ts.period, "ks", N, coef=ts.coef)
    params = [(torch.tensor(W, device="cuda"), torch.tensor(b, device="cuda")) for W, b in ts.params]
    x = torch.tensor(ts.x, device="cuda")
    segs = [dict(sg) for sg in ts.segments]
    ic = segs[1]
    ic["values"] = torch.tensor(ts.targets[ic["begin"]:ic["begin"] + ic["count"]], device="cuda").contiguous()
    opt = AdamState(params, lr=1e-3)
    grads = [(torch.empty_like(W), torch.empty_like(b)) for W, b in params]

    def step():
        plan.loss(params, x, segs)
        plan.loss_backward(params, x, segs, out=grads)
        opt.step(grads)

    for _ in range(5):
        step()
    torch.cuda.synchronize()
    l0 = float(plan.loss(params, x, segs)[0])
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    l1 = float(plan.loss(params, x, segs)[0])
    plan.close()
    return dict(workload="ks training set, modified MLP with periodic embedding", hidden=ts.hidden, width=ts.width,
                harmonics=ts.harmonics, points=N, precision="fp32", steps=steps, ms_per_step=round(ms, 4),
                run_s=round(ms * steps * 1e-3, 4), value=round(N / (ms * 1e-3), 1), unit="pts/s",
                loss_first=l0, loss_last=l1)


def nested_autograd_ks(steps, lr=1e-3):
    """The AD baseline for the KS run: the same modified MLP and loss with
    u_t, u_x .. u_xxxx by nested torch.autograd, torch.optim.Adam, FP32."""
    import torch
    import pinn_inputs as pi
    ts = pi.ks_training_set(seed=0)
    params = [t for W, b in ts.params for t in (torch.tensor(W, device="cuda", requires_grad=True),
                                                 torch.tensor(b, device="cuda", requires_grad=True))]
    opt = torch.optim.Adam(params, lr=lr)
    X0 = torch.tensor(ts.x, device="cuda")
    tg = torch.tensor(ts.targets, device="cuda")[:, 0]
    a, bb, g = ts.coef
    n_pde = ts.segments[0]["count"]
    w_ic = ts.segments[1]["weight"]
    om = 2.0 * math.pi / ts.period

    def net(X):
        feats = [X[:, 1:2]]
        for m in range(1, ts.harmonics + 1):
            feats += [torch.cos(m * om * X[:, 0:1]), torch.sin(m * om * X[:, 0:1])]
        E = torch.cat(feats, 1)
        U = torch.tanh(E @ params[0].T + params[1])
        V = torch.tanh(E @ params[2].T + params[3])
        h = torch.tanh(E @ params[4].T + params[5])
        for l in range(3, len(params) // 2 - 1):
            Z = torch.tanh(h @ params[2 * l].T + params[2 * l + 1])
            h = (1.0 - Z) * U + Z * V
        return (h @ params[-2].T + params[-1])[:, 0]

    def d(f, X, i):
        return torch.autograd.grad(f.sum(), X, create_graph=True)[0][:, i]

    def step():
        X = X0.clone().requires_grad_(True)
        u = net(X)
        ut, ux = d(u, X, 1), d(u, X, 0)
        uxx = d(ux, X, 0)
        uxxxx = d(d(uxx, X, 0), X, 0)
        r = (ut + a * u * ux + bb * uxx + g * uxxxx)[:n_pde]
        loss = (r * r).mean() + w_ic * ((u[n_pde:] - tg[n_pde:]) ** 2).mean()
        grads = torch.autograd.grad(loss, params)
        for p_, g_ in zip(params, grads):
            p_.grad = g_
        opt.step()

    for _ in range(3):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1e3 / steps


def pi_training_set(name):
    import pinn_inputs as pi
    return pi.burgers_training_set(seed=0) if name == "burgers" else pi.cavity_training_set(seed=0)


def training_leg(name, prec, steps):
    """A complete training run as the paper times it (Sec. 3.1.1): `steps`
    full-batch Adam steps on the composite loss of the paper's training set
    (all points evaluated together), eager calls of pinn_jet_loss,
    pinn_jet_loss_backward and pinn_adam_step."""
    import torch
    from paper_2606_29702_amd import AdamState, PinnPlan
    ts = pi_training_set(name)
    N = ts.x.shape[0]
    plan = PinnPlan(ts.dims, ts.name, N, precision=prec, coef=ts.coef)
    params = [(torch.tensor(W, device="cuda"), torch.tensor(b, device="cuda")) for W, b in ts.params]
    x = torch.tensor(ts.x, device="cuda")
    opt = AdamState(params, lr=1e-3)
    grads = [(torch.empty_like(W), torch.empty_like(b)) for W, b in params]

    def step():
        plan.loss(params, x, ts.segments)
        plan.loss_backward(params, x, ts.segments, out=grads)
        opt.step(grads)

    for _ in range(5):
        step()
    torch.cuda.synchronize()
    l0 = float(plan.loss(params, x, ts.segments)[0])
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    l1 = float(plan.loss(params, x, ts.segments)[0])
    plan.close()
    return dict(workload=f"{name} training set", dims=ts.dims, points=N, precision=prec, steps=steps,
                ms_per_step=round(ms, 4), run_s=round(ms * steps * 1e-3, 4),
                value=round(N / (ms * 1e-3), 1), unit="pts/s", loss_first=l0, loss_last=l1)


def plan_leg(name, prec, steps, warmup, save_cap=0, fp32_context=True):
    import pinn_inputs as pi
    prob = pi.make_problem(name)
    wl = prob.workload
    N = prob.x.shape[0]
    C = len(prob.channels)
    w, H = wl.width, wl.hidden
    run = time_plan(prob, prec, steps, warmup, save_cap=save_cap)
    tun = run["tuning"]
    fused = bool(tun["bwd_fused"]) and w <= 128
    fl = class_flops(w, H, C, N, fused)
    sb = class_stack_bytes(w, H, C, -(-N // 128) * 128, fused, 4 if prec == "fp32" else 2)
    dom = run["dominant"]
    roof = roofline_from(dom, fl[dom], run["dom_ms"], run["dom_n"], prec, name, steps, sb[dom])
    out = dict(workload=name, dims=wl.dims, N=N, channels=C, precision=prec, save_cap_bytes=save_cap,
               ms_per_step=round(run["ms"], 4), value=round(N / (run["ms"] * 1e-3), 1), unit="pts/s",
               step_mfma_frac=round(sum(fl.values()) / (run["ms"] * 1e-3) / 1e12 / PEAK[prec], 4),
               roofline=roof, tuning=tun,
               kernel_ms_per_step={k: round(v[0], 4) for k, v in run["class_ms"].items()})
    if fp32_context:
        f32 = time_plan(prob, "fp32", max(3, steps // 4), 2)
        out["fp32_jet"] = {"ms_per_step": round(f32["ms"], 4), "value": round(N / (f32["ms"] * 1e-3), 1),
                           "speedup": round(f32["ms"] / run["ms"], 3)}
    return out


def training_runs(names, prec, steps):
    """The paper's complete training runs (1000 full-batch Adam steps on the
    composite loss): the jet path in FP32 (and `prec` for the plain MLPs)
    beside the nested-autograd FP32 baseline on the same GPU."""
    runs = {}
    for name in [t for t in names.split(",") if t]:
        if name == "ks":
            r = {"fp32": ks_training_leg(steps)}
            ad_fn = lambda: nested_autograd_ks(50)  # noqa: E731
        else:
            r = {p: training_leg(name, p, steps) for p in ("fp32", prec)}
            ad_fn = lambda: nested_autograd_training(pi_training_set(name), 50)  # noqa: E731
        try:
            ad = ad_fn()
            r["nested_autograd_fp32"] = {"ms_per_step": round(ad, 4),
                                         "speedup_fp32_jet": round(ad / r["fp32"]["ms_per_step"], 3)}
        except RuntimeError as e:  # out of memory is reported, not fatal
            r["nested_autograd_fp32"] = {"error": str(e)[:200]}
        runs[name] = r
        log(f"training {name}: " + ", ".join(f"{k} {v.get('ms_per_step')} ms/step" for k, v in r.items()))
    return runs


# --------------------------------------------------------------------------- main
def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--precision", default="bf16", choices=["bf16", "fp16", "fp32"])
    ap.add_argument("--runs", type=int, default=3, help="independent timing runs of the protocol")
    ap.add_argument("--replays", type=int, default=100, help="graph replays per protocol run")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-context", action="store_true",
                    help="skip the FP32 comparison, the accuracy leg and the single-network legs")
    ap.add_argument("--legs", default="ns,heat", help="single-network legs (ns, ks, heat, burgers, aniso) or ''")
    ap.add_argument("--workload", default="ensemble",
                    help="'ensemble' (the headline) or one single-network workload, timed alone")
    ap.add_argument("--save-cap-gib", type=float, default=0.0, help="saved-state cap of a single-network workload")
    ap.add_argument("--tuning", default=None, help="dw_splits,fwd_points,bwd_fused for a single-network workload")
    ap.add_argument("--copy-probe-mib", type=int, default=0, help="only run a plain device copy of this size")
    ap.add_argument("--counter-window", type=int, default=0,
                    help="end the ensemble measurement with this many eager one-stream steps (counter profiles)")
    ap.add_argument("--training", default="burgers,ns,ks",
                    help="paper training runs (1000 Adam steps on the composite loss): burgers, ns, ks or ''")
    ap.add_argument("--training-steps", type=int, default=1000)
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the step runs on a single MI355X (data parallelism over points or "
              "networks across GPUs is a design note, not built). Use --gpus 1.", file=sys.stderr)
        sys.exit(2)
    if args.copy_probe_mib:
        copy_probe(args.copy_probe_mib)
        return

    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    prec = args.precision

    if args.workload == "training":  # only the paper's training runs
        print(json.dumps({"training_runs": training_runs(args.training, prec, args.training_steps)}), flush=True)
        return

    if args.workload != "ensemble":  # one single-network workload (profiling runs)
        import pinn_inputs as pi
        prob = pi.make_problem(args.workload)
        tuning = tuple(int(v) for v in args.tuning.split(",")) if args.tuning else None
        cap = int(args.save_cap_gib * (1 << 30))
        run = time_plan(prob, prec, args.steps, args.warmup, save_cap=cap, tuning=tuning)
        wl = prob.workload
        N = prob.x.shape[0]
        fused = bool(run["tuning"]["bwd_fused"]) and wl.width <= 128
        fl = class_flops(wl.width, wl.hidden, len(prob.channels), N, fused)
        sb = class_stack_bytes(wl.width, wl.hidden, len(prob.channels), -(-N // 128) * 128, fused,
                               4 if prec == "fp32" else 2)
        dom = run["dominant"]
        out = {"metric": METRIC, "value": round(N / (run["ms"] * 1e-3), 1), "unit": "pts/s", "n_gpus": 1,
               "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(run["ms"], 4),
               "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": prec,
               "data": "synthetic", "config": {"workload": args.workload, "dims": wl.dims, "N": N,
                                               "save_cap_bytes": cap},
               "roofline": roofline_from(dom, fl[dom], run["dom_ms"], run["dom_n"], prec, args.workload, args.steps,
                                         sb[dom]),
               "tuning": run["tuning"]}
        print(json.dumps(out), flush=True)
        return

    ens, params, xs = ensemble_inputs()
    total_N = sum(m.N for m in ens)
    log(f"ensemble: {len(ens)} networks, {total_N} points, precision {prec}")
    head = ensemble_headline(ens, params, xs, prec, args.steps, args.warmup, args.runs, args.replays,
                             args.counter_window)
    ms = head["ms"]
    value = total_N / (ms * 1e-3)
    dom = head["dominant"]
    roof = roofline_from(dom, head["flops"][dom], head["dom_ms"], head["dom_n"], prec, "ensemble", args.steps,
                         head["stack_bytes"][dom])
    log(f"{prec} grouped ensemble: {ms:.3f} ms/step, {value/1e6:.2f} Mpts/s, {head['launches']} launches, "
        f"dominant {dom} {roof['avg_launch_us']} us/launch, {roof['frac']:.4f} of peak")
    out = {
        "metric": METRIC, "value": round(value, 1), "unit": "pts/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": prec, "data": "synthetic",
        "config": {"workload": "burgers ensemble, 64 networks, seed 0", "networks": len(ens), "points": total_N,
                   "widths": sorted({m.width for m in ens}), "depths": [min(m.hidden for m in ens),
                                                                         max(m.hidden for m in ens)],
                   "step": "forward jets + residual + MSE loss + dtheta, every network",
                   "execution": "grouped launches (one per phase for all networks), one HIP graph"},
        "roofline": roof,
        "step_mfma_frac": round(head["total_flops"] / (ms * 1e-3) / 1e12 / PEAK[prec], 4),
        "hidden_gemm_tflop_per_step": round(head["total_flops"] / 1e12, 4),
        "grouped_launches_per_step": head["launches"],
        "tunings_by_width": tunings_by_width(ens, head["tunings"]),
        "lanes": head["lanes"],
        "autotune_s": round(head["tune_s"], 2),
        "timing_protocol": {"runs": args.runs, "replays_per_run": args.replays,
                            "ms_per_step_each_run": [round(v, 4) for v in head["per_run_ms"]],
                            "median_ms_per_step": round(statistics.median(head["per_run_ms"]), 4)},
        "kernel_ms_per_step_one_stream": {k: round(v[0], 4) for k, v in head["class_ms"].items()},
    }

    if not args.no_context:
        f32_ms = ensemble_fp32_sequential(ens, params, xs, max(3, args.steps // 4))
        out["fp32_sequential"] = {"ms_per_step": round(f32_ms, 4), "value": round(total_N / (f32_ms * 1e-3), 1),
                                  "unit": "pts/s", "note": "64 plain FP32 jet steps, one network after another"}
        out["speedup_vs_fp32_sequential"] = round(f32_ms / ms, 3)
        log(f"fp32 sequential: {f32_ms:.3f} ms/step (batched {prec} is {f32_ms / ms:.2f}x)")
        out["accuracy_vs_oracle"] = ensemble_accuracy(ens, prec)
        log(f"accuracy: {out['accuracy_vs_oracle']}")

    if not args.no_cpu_baseline:
        threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or (os.cpu_count() or 1)
        cb = ensemble_cpu_baseline(ens, 12.0, threads)
        cb["cpu_model"] = cpu_model()
        one = ensemble_cpu_baseline(ens, 8.0, 1)
        cb["one_core"] = {"value": one["value"], "unit": "pts/s", "sample": one["sample"]}
        out["cpu_baseline"] = cb
        log(f"cpu oracle: {cb['value']:.1f} pts/s on {threads} threads ({cb['cpu_model']}), "
            f"{one['value']:.1f} on one")

    if not args.no_context and args.legs:
        legs = {}
        for name in [s for s in args.legs.split(",") if s]:
            cap = (8 << 30) if name == "heat" else 0  # heat: saved state capped at 8 GiB
            legs[name] = plan_leg(name, prec, max(5, args.steps // 2), 2, save_cap=cap, fp32_context=name != "heat")
            log(f"leg {name}: {legs[name]['ms_per_step']} ms/step, roofline {legs[name]['roofline']['frac']}")
        if "ns" in legs:
            import pinn_inputs as pi
            try:
                ad_ms = nested_autograd_fp32(pi.make_problem("ns"), 3)
                legs["ns"]["nested_autograd_fp32"] = {"ms_per_step": round(ad_ms, 3),
                                                      "value": round(65536 / (ad_ms * 1e-3), 1)}
            except RuntimeError as e:  # out of memory is reported, not fatal
                legs["ns"]["nested_autograd_fp32"] = {"error": str(e)[:200]}
        out["legs"] = legs

    if not args.no_context and args.training:
        out["training_runs"] = training_runs(args.training, prec, args.training_steps)

    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

#!/usr/bin/env python3
"""Throughput of one partial-jet PINN step on one MI355X.

A step is the whole hot path on one batch of collocation points: forward
partial-jet pass through every layer, residual, mean-squared loss and the
hand-written adjoint down to dL/dtheta (pinn_jet_residual + pinn_jet_backward).
Inputs (network parameters and points) are resident in device memory before
the timed region starts.

Default workload: steady Navier-Stokes at Re = 100, MLP 2-128x6-3 tanh, 65536
points uniform in [0, 1]^2, channels (value, d/dx, d/dy, d2/dx2, d2/dy2).  The
headline value is the BF16-operand path (FP32 accumulation, FP32 jets,
residual and loss); the plain FP32 path on the same GPU, nested torch.autograd
(FP32) and the FP64 CPU oracle are reported beside it.

Prints one JSON line.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "collocation pts/s, residual+dθ step: BF16/batched vs plain FP32 jet, same GPU"
PEAK = {"bf16": 2500.0, "fp16": 2500.0, "fp32": 157.3}  # dense MFMA TFLOP/s
HBM_PEAK = 8000.0  # GB/s
GEMM_CLASSES = ("layer_fwd", "layer_bwd", "dw_hidden", "bwd_dw")


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


def make_inputs(workload, N=None, seed=0):
    import pinn_inputs as pi
    return pi.make_problem(workload, N=N, seed=seed)


def gpu_params(prob):
    import torch
    return [(torch.tensor(W, device="cuda"), torch.tensor(b, device="cuda")) for W, b in prob.params]


def time_path(prob, prec, steps, warmup, profile_dominant=True, tuning=None, save_cap=0):
    """Times `steps` residual+backward steps; returns ms/step and per-class kernel times."""
    import torch
    from paper_2606_29702_amd import PinnPlan
    wl = prob.workload
    N = prob.x.shape[0]
    plan = PinnPlan(wl.dims, wl.pde, N, precision=prec, coef=prob.coef, save_cap_bytes=save_cap)
    params = gpu_params(prob)
    x = torch.tensor(prob.x, device="cuda")

    def step():
        plan.residual(params, x)
        plan.backward(params, x)

    # the library's autotuner picks split-K, forward tiling and backward variant,
    # unless a tuning is given
    if tuning is None:
        tuning, _ = plan.autotune(params, x, reps=10)
    else:
        plan.set_tuning(*tuning)
        tuning = plan.tuning()
    # warmup; one profiled step per kernel class to find the dominant class
    class_ms = {}
    for i in range(max(warmup, 1)):
        step()
    torch.cuda.synchronize()
    for cls in ("layer_fwd", "layer_bwd", "dw_hidden", "bwd_dw", "out_fwd", "out_bwd", "seed_fwd", "other"):
        plan.profile(cls)
        step()
        ms, n = plan.profile_read()
        class_ms[cls] = (ms, n)
    plan.profile("off")
    dominant = max(class_ms, key=lambda c: class_ms[c][0])
    torch.cuda.synchronize()

    # timed region; launches of the dominant class are bracketed by events
    if profile_dominant:
        plan.profile(dominant)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    dom_ms, dom_n = plan.profile_read() if profile_dominant else (float("nan"), 0)
    plan.profile("off")
    # a training step: the same step plus the fused Adam update (lr 1e-3, as in
    # the paper's runs), on a copy of the parameters (context)
    from paper_2606_29702_amd import AdamState
    tparams = [(W.clone(), b.clone()) for W, b in params]
    tgrads = [(torch.empty_like(W), torch.empty_like(b)) for W, b in tparams]
    opt = AdamState(tparams, lr=1e-3)
    # a long warm-up: early in a long eager loop, with the host far ahead of the
    # GPU, a host call occasionally blocks for tens of milliseconds (seen with
    # and without the Adam step); later steps run at full rate
    for _ in range(max(warmup, 100)):
        plan.residual(tparams, x)
        opt.step(plan.backward(tparams, x, out=tgrads))
    torch.cuda.synchronize()
    a0 = time.perf_counter()
    for _ in range(steps):
        plan.residual(tparams, x)
        opt.step(plan.backward(tparams, x, out=tgrads))
    torch.cuda.synchronize()
    train_ms = (time.perf_counter() - a0) * 1e3 / steps
    # the training step captured as one graph (pinn_graph_capture_train)
    tgraph = plan.capture_step(tparams, x, adam=opt)
    for _ in range(5):
        tgraph.launch()
    torch.cuda.synchronize()
    a0 = time.perf_counter()
    for _ in range(steps):
        tgraph.launch()
    torch.cuda.synchronize()
    train_graph_ms = (time.perf_counter() - a0) * 1e3 / steps
    tgraph.close()
    # the same step captured once as a HIP graph and replayed (context)
    graph = plan.capture_step(params, x)
    graph.launch()
    torch.cuda.synchronize()
    g0 = time.perf_counter()
    for _ in range(steps):
        graph.launch()
    torch.cuda.synchronize()
    graph_ms = (time.perf_counter() - g0) * 1e3 / steps
    graph.close()
    plan.close()
    return dict(ms_per_step=(t1 - t0) * 1e3 / steps, class_ms=class_ms, dominant=dominant,
                dominant_avg_ms=dom_ms / max(dom_n, 1), dominant_launches=dom_n, tuning=tuning,
                graph_ms_per_step=graph_ms, train_ms_per_step=train_ms, train_graph_ms_per_step=train_graph_ms)


def nested_autograd_fp32(prob, steps):
    """The paper's AD baseline (Sec. 3.1.1): coordinate derivatives by nested
    torch.autograd, then reverse mode for dtheta.  FP32 on the GPU; context only."""
    import torch
    from tests import autograd_ref  # noqa: F401  (same formulas; FP32 tensors here)
    wl = prob.workload
    params = [(torch.tensor(W, device="cuda", requires_grad=True), torch.tensor(b, device="cuda", requires_grad=True))
              for W, b in prob.params]
    X0 = torch.tensor(prob.x, device="cuda")
    channels = prob.channels

    def step():
        X = X0.clone().requires_grad_(True)
        h = X
        for l, (W, b) in enumerate(params):
            h = h @ W.T + b
            if l < len(params) - 1:
                h = torch.tanh(h)
        jets = {}
        for o in range(h.shape[1]):
            u = h[:, o]
            for c, (d, k) in enumerate(channels):
                g = u
                for _ in range(k):
                    g = torch.autograd.grad(g.sum(), X, create_graph=True)[0][:, d]
                jets[(o, c)] = g
        rs = autograd_ref.residuals(wl.pde, jets, channels, X, prob.coef)
        N = X.shape[0]
        loss = sum((r * r).sum() / N for r in rs)
        grads = torch.autograd.grad(loss, [t for p in params for t in p], allow_unused=True)
        return grads

    step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1e3 / steps


def ensemble(steps, seed=0):
    """The 64-network Burgers ensemble: one BF16 step of all networks (side
    streams, HIP graph replay, autotuned stream count) against 64 sequential
    plain-FP32 calls on one stream, same GPU."""
    import torch
    import pinn_inputs as pi
    from paper_2606_29702_amd import PinnBatch, PinnPlan
    ens = pi.make_ensemble(seed=seed)
    total = sum(m.N for m in ens)
    params = [[(torch.tensor(W, device="cuda"), torch.tensor(b, device="cuda")) for W, b in m.params] for m in ens]
    xs = [torch.tensor(m.x, device="cuda") for m in ens]
    batch = PinnBatch([m.dims for m in ens], "burgers", [(m.nu,) for m in ens], [m.N for m in ens],
                      precision="bf16")
    n_streams, _ = batch.autotune(params, xs, reps=2)
    for _ in range(2):
        batch.step(params, xs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        batch.step(params, xs)
    torch.cuda.synchronize()
    t_b = (time.perf_counter() - t0) / steps
    batch.close()
    plans = [PinnPlan(m.dims, "burgers", m.N, precision="fp32", coef=(m.nu,)) for m in ens]

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
    t_s = (time.perf_counter() - t0) / steps
    for pl in plans:
        pl.close()
    return {"nets": len(ens), "points": total, "value": round(total / t_b, 1), "unit": "pts/s",
            "ms_per_step": round(t_b * 1e3, 3), "side_streams": n_streams,
            "fp32_sequential": {"value": round(total / t_s, 1), "ms_per_step": round(t_s * 1e3, 3)},
            "speedup_vs_fp32_sequential": round(t_s / t_b, 3)}


def cpu_baseline(prob, target_s=15.0):
    """The FP64 oracle on the host cores over a bounded sample of the same points."""
    import numpy as np
    import oracle
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or (os.cpu_count() or 1)
    # calibrate on growing samples until one takes a second, then scale to target_s
    n, dt = 128, 0.0
    while True:
        t0 = time.perf_counter()
        oracle.evaluate(prob.params, prob.x[:n], prob.channels, prob.workload.pde, prob.coef, threads=threads)
        dt = time.perf_counter() - t0
        if dt >= 1.0 or n >= prob.x.shape[0]:
            break
        n *= 2
    full = prob.x.shape[0]
    # the whole workload fits in the budget: repeat it to about target_s
    passes = max(1, int(round(target_s / dt))) if n >= full else 1
    n = int(min(full, max(n, n * target_s / dt)))
    n = max(64, n // 64 * 64)
    t0 = time.perf_counter()
    for _ in range(passes):
        res = oracle.evaluate(prob.params, prob.x[:n], prob.channels, prob.workload.pde, prob.coef,
                              threads=threads)
    dt = time.perf_counter() - t0
    what = f"first {n} of the {full} points" if passes == 1 else f"all {n} points, {passes} passes"
    return dict(value=passes * n / dt, unit="pts/s", cores=threads, kind="oracle",
                sample=f"{what}, residual + loss + dtheta in FP64 ({dt:.1f} s)"), n, res


def accuracy(prob, n, ref, prec):
    """GPU path on the oracle's sample against the oracle (rel. L2)."""
    import numpy as np
    import torch
    from paper_2606_29702_amd import PinnPlan
    wl = prob.workload
    plan = PinnPlan(wl.dims, wl.pde, n, precision=prec, coef=prob.coef)
    params = gpu_params(prob)
    x = torch.tensor(prob.x[:n], device="cuda")
    r, loss, _, _ = plan.residual(params, x)
    grads = plan.backward(params, x)
    torch.cuda.synchronize()
    g = np.concatenate([np.concatenate([dW.double().cpu().numpy().ravel(), db.double().cpu().numpy().ravel()])
                        for dW, db in grads])
    rr = r.double().cpu().numpy()
    plan.close()

    def rel(a, b):
        return float(np.linalg.norm(a.ravel() - b.ravel()) / np.linalg.norm(b.ravel()))

    return dict(r_rel_l2=rel(rr, ref.r), grad_rel_l2=rel(g, ref.grad),
                grad_cosine=float(g @ ref.grad / (np.linalg.norm(g) * np.linalg.norm(ref.grad))),
                points=n)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="ns", choices=["burgers", "ns", "ks", "heat", "aniso"])
    ap.add_argument("--precision", default="bf16", choices=["bf16", "fp16", "fp32"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-context", action="store_true", help="skip the FP32, nested-autograd and ensemble context runs")
    ap.add_argument("--copy-probe-mib", type=int, default=0, help="only run a plain device copy of this size")
    ap.add_argument("--save-cap-gib", type=float, default=0.0,
                    help="bound on the saved layer state (checkpointed backward); 0 = store every layer")
    ap.add_argument("--tuning", default=None,
                    help="dw_splits,fwd_points,bwd_fused instead of running the autotuner (e.g. for profiling)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the partial-jet step is run on a single MI355X "
              "(multi-GPU data parallelism over points is a design note, not built). Use --gpus 1.",
              file=sys.stderr)
        sys.exit(2)

    if args.copy_probe_mib:
        copy_probe(args.copy_probe_mib)
        return

    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    prob = make_inputs(args.workload)
    wl = prob.workload
    N = prob.x.shape[0]
    C = len(prob.channels)
    w, H = wl.width, wl.hidden

    log(f"workload {args.workload}: dims {wl.dims}, N {N}, C {C}, precision {args.precision}")
    tuning = tuple(int(v) for v in args.tuning.split(",")) if args.tuning else None
    save_cap = int(args.save_cap_gib * (1 << 30))
    main_run = time_path(prob, args.precision, args.steps, args.warmup, tuning=tuning, save_cap=save_cap)
    ms = main_run["ms_per_step"]
    value = N / (ms * 1e-3)
    log(f"{args.precision}: {ms:.3f} ms/step, {value/1e6:.2f} Mpts/s, dominant {main_run['dominant']} "
        f"{main_run['dominant_avg_ms']*1e3:.1f} us/launch")

    dom = main_run["dominant"]
    if dom in GEMM_CLASSES:
        # algorithmic flops per launch: G = 2 w^2 C N is one stacked-channel
        # w x w GEMM over the N points.  The whole-network forward kernel does
        # the H - 1 hidden-layer GEMMs of a step; a backward layer kernel one
        # (abar); the fused backward kernel two (abar and dW); a dW kernel one.
        # The z recompute in the backward kernels is a design cost, not counted.
        G = 2.0 * w * w * C * N
        n_dom = max(main_run["class_ms"][dom][1], 1)  # launches in one step
        per_step = {"layer_fwd": (H - 1) * G, "layer_bwd": n_dom * G, "dw_hidden": n_dom * G,
                    "bwd_dw": 2 * n_dom * G}[dom]
        flops = per_step / n_dom
        achieved = flops / (main_run["dominant_avg_ms"] * 1e-3) / 1e12
        traffic = profiled_traffic(args.workload, args.precision, dom)
        roof = dict(bound="mfma", achieved=round(achieved, 3), peak=PEAK[args.precision], unit="TFLOP/s",
                    frac=round(achieved / PEAK[args.precision], 5),
                    traffic=None if traffic is None else round(traffic),
                    traffic_unit="bytes per launch (HBM, rocprofv3 FETCH_SIZE + WRITE_SIZE)",
                    achieved_hbm_GBps=None if traffic is None else
                    round(traffic / (main_run["dominant_avg_ms"] * 1e-3) / 1e9, 1), kernel=dom,
                    avg_launch_us=round(main_run["dominant_avg_ms"] * 1e3, 2),
                    launches=main_run["dominant_launches"], flops_per_launch=flops,
                    hbm_frac=None if traffic is None else
                    round(traffic / (main_run["dominant_avg_ms"] * 1e-3) / 1e9 / HBM_PEAK, 4))
    else:
        roof = dict(bound="hbm", achieved=None, peak=HBM_PEAK, unit="GB/s", frac=None, traffic=None,
                    kernel=dom, avg_launch_us=round(main_run["dominant_avg_ms"] * 1e3, 2))

    out = {
        "metric": METRIC, "value": round(value, 1), "unit": "pts/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": args.precision, "data": "synthetic",
        "config": {"workload": args.workload, "dims": wl.dims, "N": N, "channels": C,
                   "coef": list(prob.coef), "step": "forward jets + residual + MSE loss + dtheta",
                   "save_cap_bytes": save_cap},
        "roofline": roof,
        "kernel_ms_per_step": {k: round(v[0], 4) for k, v in main_run["class_ms"].items()},
        "train_step_adam": {"ms_per_step": round(main_run["train_ms_per_step"], 4),
                            "value": round(N / (main_run["train_ms_per_step"] * 1e-3), 1), "unit": "pts/s",
                            "note": "residual + dtheta + fused Adam update (pinn_adam_step)",
                            "graph_ms_per_step": round(main_run["train_graph_ms_per_step"], 4)},
        "graph_replay": {"ms_per_step": round(main_run["graph_ms_per_step"], 4),
                         "value": round(N / (main_run["graph_ms_per_step"] * 1e-3), 1), "unit": "pts/s"},
        "tuning": main_run["tuning"],
    }

    if not args.no_context:
        fp32 = time_path(prob, "fp32", max(5, args.steps // 5), 3, profile_dominant=False)
        out["fp32_jet"] = {"value": round(N / (fp32["ms_per_step"] * 1e-3), 1), "unit": "pts/s",
                           "ms_per_step": round(fp32["ms_per_step"], 4)}
        out["speedup_vs_fp32_jet"] = round(fp32["ms_per_step"] / ms, 3)
        log(f"fp32 jet: {fp32['ms_per_step']:.3f} ms/step")
        try:
            ad_ms = nested_autograd_fp32(prob, 3)
            out["nested_autograd_fp32"] = {"value": round(N / (ad_ms * 1e-3), 1), "unit": "pts/s",
                                           "ms_per_step": round(ad_ms, 3)}
            log(f"nested autograd fp32: {ad_ms:.3f} ms/step")
        except RuntimeError as e:  # out of memory at large N is reported, not fatal
            out["nested_autograd_fp32"] = {"error": str(e)[:200]}
            torch.cuda.empty_cache()

    if not args.no_context:
        out["ensemble_burgers_64"] = ensemble(steps=5)
        log(f"ensemble: {out['ensemble_burgers_64']}")

    if not args.no_cpu_baseline:
        cb, n_s, ref = cpu_baseline(prob)
        out["cpu_baseline"] = cb
        log(f"cpu oracle: {cb['value']:.1f} pts/s on {cb['cores']} threads")
        out["accuracy_vs_oracle"] = accuracy(prob, n_s, ref, args.precision)
        log(f"accuracy: {out['accuracy_vs_oracle']}")

    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

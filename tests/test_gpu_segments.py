"""GPU parity of the composite training loss (Sec. 3.1.1): initial, boundary
and PDE points concatenated and evaluated once, the outputs split into the
weighted loss terms; pinn_jet_loss and pinn_jet_loss_backward against the FP64
oracle's composite loss on the same seeded training sets.

Bars: FP32 operands 1e-5 relative (each segment loss, the loss, the gradient);
16-bit operands the per-precision ceilings of the plain residual loss
(gradient 1e-2 BF16, 5e-3 FP16; losses 3e-2 BF16, 6e-3 FP16, the jets' bar,
since the data and periodic terms are differences of output values and
derivative channels).
"""
import ctypes

import numpy as np
import pytest
import torch

import oracle
import pinn_inputs as pi

pytestmark = pytest.mark.gpu

TOL = {"fp32": {"loss": 1e-5, "grad": 1e-5},
       "bf16": {"loss": 3e-2, "grad": 1e-2},
       "fp16": {"loss": 6e-3, "grad": 5e-3}}


def rel(a, b):
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.fixture(scope="module")
def lib():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2606_29702_amd as pj
    return pj


def dev(params):
    return [(torch.tensor(W, device="cuda"), torch.tensor(b, device="cuda")) for W, b in params]


def flat(grads):
    return np.concatenate([np.concatenate([W.detach().double().cpu().numpy().ravel(),
                                           b.detach().double().cpu().numpy().ravel()]) for W, b in grads])


def small_set(kind, seed=3, scale=1):
    """The paper's training layouts at a size the oracle finishes in seconds:
    several 128-point tiles, ragged segment boundaries and a ragged tail."""
    if kind == "burgers":
        return pi.burgers_training_set(seed=seed, n_pde=1203 * scale, n_ic=101, n_pairs=157 * scale, width=64,
                                       hidden=6, bias_std=0.2, w_ic=10.0, w_per=1.3, w_pde=0.7)
    return pi.cavity_training_set(seed=seed, n_pde=1111 * scale, n_wall=299, n_lid=99, width=64, hidden=6,
                                  bias_std=0.2, w_wall=2.0, w_lid=3.0, w_pde=0.6)


def run_gpu(lib, ts, prec, segments=None):
    segs = ts.segments if segments is None else segments
    N = ts.x.shape[0]
    plan = lib.PinnPlan(ts.dims, ts.name, N, precision=prec, coef=ts.coef)
    params = dev(ts.params)
    x = torch.tensor(ts.x, device="cuda")
    loss, seg_loss = plan.loss(params, x, segs)
    grads = plan.loss_backward(params, x, segs)
    torch.cuda.synchronize()
    out = float(loss), seg_loss.double().cpu().numpy(), flat(grads)
    plan.close()
    return out


@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp16"])
@pytest.mark.parametrize("kind", ["burgers", "ns"])
def test_composite_loss_matches_oracle(lib, kind, prec):
    ts = small_set(kind)
    loss, seg_loss, g = run_gpu(lib, ts, prec)
    sl_ref, L_ref, g_ref = oracle.evaluate_segments(ts.params, ts.x, pi.CHANNELS[kind], kind, ts.coef, ts.segments)
    tol = TOL[prec]
    for s in range(len(ts.segments)):
        assert abs(seg_loss[s] - sl_ref[s]) <= tol["loss"] * abs(sl_ref[s]), (s, seg_loss[s], sl_ref[s])
    assert abs(loss - L_ref) <= tol["loss"] * abs(L_ref), (loss, L_ref)
    assert rel(g, g_ref) <= tol["grad"], rel(g, g_ref)


@pytest.mark.parametrize("kind", ["burgers", "ns"])
def test_composite_loss_paper_size_fp32(lib, kind):
    """The paper's point counts (10000 PDE points plus 101 initial points and
    1000 periodic pairs, or 1499 wall and 499 lid points), 2-64x6 tanh MLP."""
    ts = pi.burgers_training_set(seed=5) if kind == "burgers" else pi.cavity_training_set(seed=5)
    loss, seg_loss, g = run_gpu(lib, ts, "fp32")
    sl_ref, L_ref, g_ref = oracle.evaluate_segments(ts.params, ts.x, pi.CHANNELS[kind], kind, ts.coef, ts.segments)
    assert np.all(np.abs(seg_loss - sl_ref) <= 1e-5 * np.abs(sl_ref))
    assert abs(loss - L_ref) <= 1e-5 * abs(L_ref)
    assert rel(g, g_ref) <= 1e-5


@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp16"])
def test_single_pde_segment_equals_residual_loss(lib, prec):
    """One PDE segment over all points with weight 1 is the plain residual
    loss: the same output cotangent and the same backward kernels, so the
    gradient equals pinn_jet_backward's bit for bit."""
    prob = pi.make_problem("ns", N=1000, seed=4, bias_std=0.2, dims=[2, 64, 64, 64, 3])
    N = prob.x.shape[0]
    plan = lib.PinnPlan(prob.workload.dims, "ns", N, precision=prec, coef=prob.coef)
    params = dev(prob.params)
    x = torch.tensor(prob.x, device="cuda")
    _, l_ref, _, _ = plan.residual(params, x)
    g_ref = flat(plan.backward(params, x))
    seg = [dict(type="pde", begin=0, count=N, weight=1.0)]
    loss, seg_loss = plan.loss(params, x, seg)
    g = flat(plan.loss_backward(params, x, seg))
    torch.cuda.synchronize()
    assert np.array_equal(g, g_ref)
    assert abs(float(loss) - float(l_ref)) <= 1e-6 * abs(float(l_ref))
    assert float(seg_loss[0]) == float(loss)
    plan.close()


def test_points_outside_segments_do_not_count(lib):
    """Points that no segment covers are evaluated but enter neither the loss
    nor the gradient: against the oracle on the covered points alone."""
    ts = small_set("burgers")
    segs = [dict(s) for s in ts.segments]
    segs[0]["begin"], segs[0]["count"] = 200, 700  # PDE points 0..199 and 900..1202 uncovered
    _, seg_loss, g = run_gpu(lib, ts, "fp32", segs)
    keep = np.r_[200:900, 1203:ts.x.shape[0]]
    sub = [dict(s) for s in segs]
    sub[0]["begin"] = 0
    for s in sub[1:]:
        s["begin"] -= 503
    sl_ref, _, g_ref = oracle.evaluate_segments(ts.params, ts.x[keep], pi.CHANNELS["burgers"], "burgers", ts.coef,
                                                sub)
    assert np.all(np.abs(seg_loss - sl_ref) <= 1e-5 * np.abs(sl_ref))
    assert rel(g, g_ref) <= 1e-5


def test_eight_segments_and_zero_weight(lib):
    """The largest segment count, segments in any order, and a zero weight
    (its loss is reported, its gradient contribution is zero)."""
    ts = small_set("ns")
    n = ts.x.shape[0]
    cuts = np.linspace(0, 1111, 6).astype(int)
    segs = [dict(type="pde", begin=int(a), count=int(b - a), weight=0.5 + 0.25 * k)
            for k, (a, b) in enumerate(zip(cuts[:-1], cuts[1:]))]
    segs[2]["weight"] = 0.0
    segs += [dict(s) for s in ts.segments[1:]]
    segs.append(dict(type="periodic", begin=1111 + 299 + 1, count=98, weight=0.8,
                     mask=(1 << 1) | (1 << 5 + 2) | (1 << 10 + 3)))
    segs[-2]["count"] = 1  # the lid keeps one point; the pairs take the rest
    segs = segs[::-1]
    assert len(segs) == 8 and sum(s["count"] for s in segs) == n
    _, seg_loss, g = run_gpu(lib, ts, "fp32", segs)
    sl_ref, _, g_ref = oracle.evaluate_segments(ts.params, ts.x, pi.CHANNELS["ns"], "ns", ts.coef, segs)
    assert np.all(np.abs(seg_loss - sl_ref) <= 1e-5 * np.abs(sl_ref))
    assert rel(g, g_ref) <= 1e-5


def test_segment_errors(lib):
    ts = small_set("burgers")
    N = ts.x.shape[0]
    plan = lib.PinnPlan(ts.dims, "burgers", N, precision="fp32", coef=ts.coef)
    params = dev(ts.params)
    x = torch.tensor(ts.x, device="cuda")
    bad = [
        [dict(type="pde", begin=0, count=10), dict(type="pde", begin=5, count=10)],          # overlap
        [dict(type="pde", begin=N - 5, count=10)],                                            # past N
        [dict(type="periodic", begin=0, count=9, mask=1)],                                    # odd pair count
        [dict(type="dirichlet", begin=0, count=9, mask=2)],                                   # derivative channel
        [dict(type="dirichlet", begin=0, count=9, mask=0)],                                   # empty mask
        [dict(type="pde", begin=0, count=10, weight=-1.0)],                                   # negative weight
        [dict(type="pde", begin=10 * k, count=10) for k in range(9)],                         # too many
    ]
    for segs in bad:
        with pytest.raises(lib.PinnError) as ei:
            plan.loss(params, x, segs)
        assert ei.value.status == -1, segs
    with pytest.raises(lib.PinnError):
        plan.loss(params, x, [])
    # backward must follow a loss call with the same segments
    plan.residual(params, x)
    with pytest.raises(lib.PinnError) as ei:
        plan.loss_backward(params, x, ts.segments)
    assert ei.value.status == -5
    plan.loss(params, x, ts.segments)
    other = [dict(s) for s in ts.segments]
    other[1]["weight"] = 2.0
    with pytest.raises(lib.PinnError) as ei:
        plan.loss_backward(params, x, other)
    assert ei.value.status == -5
    plan.loss_backward(params, x, ts.segments)
    plan.close()


def test_adam_trajectory_fp32_against_fp64(lib):
    """1000 full-batch Adam steps on the composite Burgers loss (the paper's
    training protocol, at a small size), the GPU in FP32.
    * At every 50th iterate of the GPU run, the oracle's FP64 loss and
      gradient at the GPU's own parameters match the GPU's to the FP32 bar
      (the gradient's error measured against the first gradient's norm).
    * Against the oracle's own FP64 Adam run from the same start, the loss
      curves agree to 1e-4 over the first 100 steps.  Later the FP32 run drifts
      away, as the paper reports for its FP32 Burgers and NS runs (Adam's
      normalisation amplifies rounding where gradient components are small,
      most visibly around loss spikes); both runs still train to within 10 %
      of each other's final loss."""
    ts = pi.burgers_training_set(seed=11, n_pde=300, n_ic=41, n_pairs=40, width=32, hidden=3, bias_std=0.1)
    steps, lr, every = 1000, 1e-3, 50
    N = ts.x.shape[0]
    plan = lib.PinnPlan(ts.dims, "burgers", N, precision="fp32", coef=ts.coef)
    params = dev(ts.params)
    x = torch.tensor(ts.x, device="cuda")
    opt = lib.AdamState(params, lr=lr)
    grads = [(torch.empty_like(W), torch.empty_like(b)) for W, b in params]
    gpu_loss = np.zeros(steps)
    samples = []
    for k in range(steps):
        loss, _ = plan.loss(params, x, ts.segments)
        plan.loss_backward(params, x, ts.segments, out=grads)
        if k % every == 0:
            torch.cuda.synchronize()
            samples.append((k, [(W.cpu().numpy().copy(), b.cpu().numpy().copy()) for W, b in params],
                            float(loss), flat(grads)))
        opt.step(grads)
        gpu_loss[k] = float(loss)
    torch.cuda.synchronize()
    g0 = None
    for k, ps, L, g in samples:
        _, L_ref, g_ref = oracle.evaluate_segments(ps, ts.x, pi.CHANNELS["burgers"], "burgers", ts.coef,
                                                   ts.segments)
        g0 = np.linalg.norm(g_ref) if g0 is None else g0
        print(f"iterate {k}: loss rel {abs(L - L_ref) / abs(L_ref):.1e}, grad rel {rel(g, g_ref):.1e}, "
              f"|g| / |g_0| {np.linalg.norm(g_ref) / g0:.2f}")
        assert abs(L - L_ref) <= 1e-5 * abs(L_ref), (k, L, L_ref)
        # the gradient is a sum of per-point terms that cancel more and more
        # as the loss falls; FP32 rounding in those terms stays at the scale of
        # the first gradient, so the bar is 1e-5 of |g_0|
        assert np.linalg.norm(g - g_ref) <= 1e-5 * g0, (k, rel(g, g_ref))
    theta = oracle.pack_theta(ts.params).astype(np.float64)
    m = np.zeros_like(theta)
    v = np.zeros_like(theta)
    ref_loss = np.zeros(steps)
    for k in range(steps):
        ps = oracle.unpack_theta(theta, ts.dims)
        _, L, g = oracle.evaluate_segments(ps, ts.x, pi.CHANNELS["burgers"], "burgers", ts.coef, ts.segments)
        ref_loss[k] = L
        oracle.adam_step(theta, g, m, v, k + 1, lr=lr)
    drift = np.abs(gpu_loss - ref_loss) / np.abs(ref_loss)
    print("FP32 GPU vs FP64 oracle Adam run, max relative loss difference per 100 steps:",
          " ".join(f"{drift[i:i + 100].max():.1e}" for i in range(0, steps, 100)))
    assert drift[:100].max() <= 1e-4, drift[:100].max()
    assert ref_loss[-1] < 0.2 * ref_loss[0] and gpu_loss[-1] < 0.2 * gpu_loss[0]  # both runs train
    assert abs(gpu_loss[-1] - ref_loss[-1]) <= 0.1 * ref_loss[-1]
    plan.close()

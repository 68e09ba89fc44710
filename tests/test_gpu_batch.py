"""GPU tests of the ensemble step (many networks, side streams, HIP graph
replay) and of the autotuners."""
import numpy as np
import pytest
import torch

import oracle
import pinn_inputs as pi

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2606_29702_amd as pj
    return pj


def flat(grads):
    return np.concatenate([np.concatenate([dW.detach().double().cpu().numpy().ravel(),
                                           db.detach().double().cpu().numpy().ravel()]) for dW, db in grads])


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / np.linalg.norm(np.ravel(b)))


def small_ensemble(n=7, seed=3):
    # the ensemble recipe (widths, depths, nu) with point counts small enough for the oracle
    return pi.make_ensemble(n_nets=n, seed=seed, n_range=(100, 700), bias_std=0.2)


def to_dev(members):
    params = [[(torch.tensor(W, device="cuda"), torch.tensor(b, device="cuda")) for W, b in m.params]
              for m in members]
    xs = [torch.tensor(m.x, device="cuda") for m in members]
    return params, xs


@pytest.mark.parametrize("prec", ["bf16", "fp32"])
def test_batch_graph_replays_match_eager_and_single_plans(lib, prec):
    ens = small_ensemble()
    params, xs = to_dev(ens)
    dims = [m.dims for m in ens]
    coefs = [(m.nu,) for m in ens]
    Ns = [m.N for m in ens]
    # reference: one plan per network, eager
    ref_loss, ref_g = [], []
    for m, p, x in zip(ens, params, xs):
        plan = lib.PinnPlan(m.dims, "burgers", m.N, precision=prec, coef=(m.nu,))
        _, loss, _, _ = plan.residual(p, x)
        g = plan.backward(p, x)
        torch.cuda.synchronize()
        ref_loss.append(float(loss))
        ref_g.append(flat(g))
        plan.close()
    batch = lib.PinnBatch(dims, "burgers", coefs, Ns, precision=prec)
    batch.configure(4, use_graph=False)
    loss, grads = batch.step(params, xs)
    torch.cuda.synchronize()
    eager = (loss.cpu().numpy().copy(), [flat(g) for g in grads])
    batch.configure(4, use_graph=True)
    for rep in range(4):  # capture, then replays with eager work and syncs in between
        loss, grads = batch.step(params, xs)
        torch.cuda.synchronize()
        _ = (xs[0] * 2.0).sum().item()
        assert np.array_equal(loss.cpu().numpy(), eager[0]), rep
        for i in range(len(ens)):
            assert np.array_equal(flat(grads[i]), eager[1][i]), (rep, i)
    # networks dealt to per-network lanes, and to lanes kept to one width:
    # the same results
    for ns, wl in ((3, False), (5, True), (2, True)):
        batch.configure(ns, use_graph=True, per_network=True, width_lanes=wl)
        assert batch.config() == {"streams": ns, "graph": True, "per_network": True, "width_lanes": wl}
        for rep in range(2):
            loss, grads = batch.step(params, xs)
            torch.cuda.synchronize()
            assert np.array_equal(loss.cpu().numpy(), eager[0]), (ns, wl, rep)
            for i in range(len(ens)):
                assert np.array_equal(flat(grads[i]), eager[1][i]), (ns, wl, rep, i)
    with pytest.raises(lib.PinnError):  # width lanes are per-network lanes
        batch.configure(4, use_graph=True, per_network=False, width_lanes=True)
    for i in range(len(ens)):
        assert eager[0][i] == np.float32(ref_loss[i])
        assert np.array_equal(eager[1][i], ref_g[i]), i
    # against the oracle: FP32 at the FP32 bar; BF16 at its measured ceiling
    # (rel. L2 up to 3.1e-3, margin 3)
    for i, m in enumerate(ens):
        ref = oracle.evaluate(m.params, m.x, pi.CHANNELS["burgers"], "burgers", (m.nu,))
        e = rel(eager[1][i], ref.grad)
        cos = float(eager[1][i] @ ref.grad / (np.linalg.norm(eager[1][i]) * np.linalg.norm(ref.grad)))
        print(prec, f"member {i} w={m.width} H={m.hidden} N={m.N} nu={m.nu:.3g}: grad rel {e:.2e} cos {cos:.6f}")
        if prec == "fp32":
            assert e <= 1e-5, (i, e)
        else:
            assert e <= 1e-2 and cos >= 0.9999, (i, e, cos)
    batch.close()


def test_batch_recaptures_on_new_inputs_and_autotunes(lib):
    ens = small_ensemble(n=5, seed=4)
    params, xs = to_dev(ens)
    batch = lib.PinnBatch([m.dims for m in ens], "burgers", [(m.nu,) for m in ens], [m.N for m in ens])
    loss1, _ = batch.step(params, xs)
    l1 = loss1.cpu().numpy().copy()
    xs2 = [x.flip(0).contiguous() for x in xs]  # same points, new buffers and order
    loss2, grads2 = batch.step(params, xs2)
    torch.cuda.synchronize()
    g2 = [flat(g) for g in grads2]
    np.testing.assert_allclose(loss2.cpu().numpy(), l1, rtol=1e-4)
    ns, ms = batch.autotune(params, xs2, reps=2)
    assert ns in (1, 2, 4, 8, 12, 16) and ms > 0
    cfg = batch.config()
    assert cfg["streams"] == ns and cfg["graph"] and (cfg["per_network"] == (ns >= 8))
    assert not cfg["width_lanes"] or cfg["per_network"]
    # the autotuner may pick other tilings and split counts per member, which
    # reorders sums: close to the earlier step, and steps with the tuned
    # schedule repeat bit for bit
    loss3, grads3 = batch.step(params, xs2)
    torch.cuda.synchronize()
    l3, g3 = loss3.cpu().numpy().copy(), [flat(g) for g in grads3]
    np.testing.assert_allclose(l3, loss2.cpu().numpy(), rtol=1e-3)
    for a, g in zip(g2, g3):
        assert rel(g, a) <= 1e-2
    loss4, grads4 = batch.step(params, xs2)
    torch.cuda.synchronize()
    assert np.array_equal(loss4.cpu().numpy(), l3)
    for a, g in zip(g3, grads4):
        assert np.array_equal(a, flat(g))
    # each member's tuned tiling and split count give the same bits on a plan
    # of its own
    for i, m in enumerate(ens):
        t = batch.tuning(i)
        plan = lib.PinnPlan(m.dims, "burgers", m.N, precision="bf16", coef=(m.nu,))
        plan.set_tuning(**t)
        _, l1, _, _ = plan.residual(params[i], xs2[i])
        g1 = plan.backward(params[i], xs2[i])
        torch.cuda.synchronize()
        assert float(l1) == float(l3[i]), (i, t)
        assert np.array_equal(flat(g1), g3[i]), (i, t)
        plan.close()
    batch.close()


def test_plan_autotune_and_tuning_validation(lib):
    from paper_2606_29702_amd import PinnError
    prob = pi.make_problem("ns", N=3000, seed=5, bias_std=0.2, dims=[2, 128, 128, 128, 3])
    plan = lib.PinnPlan(prob.workload.dims, "ns", 3000, precision="bf16", coef=prob.coef)
    params = [(torch.tensor(W, device="cuda"), torch.tensor(b, device="cuda")) for W, b in prob.params]
    x = torch.tensor(prob.x, device="cuda")
    t0 = plan.tuning()
    best, ms = plan.autotune(params, x, reps=2)
    assert ms > 0 and plan.tuning() == best
    plan.residual(params, x)
    g = flat(plan.backward(params, x))
    ref = oracle.evaluate(prob.params, prob.x, prob.channels, "ns", prob.coef)
    assert rel(g, ref.grad) <= 1e-2
    with pytest.raises(PinnError):
        plan.set_tuning(0, 0)
    with pytest.raises(PinnError):
        plan.set_tuning(t0["dw_splits"], 24)
    plan.set_tuning(t0["dw_splits"], 16)
    plan.close()


@pytest.mark.parametrize("prec", ["bf16", "fp32"])
def test_plan_graph_replays_match_eager(lib, prec):
    """A captured step replayed several times, with eager steps and in-place
    weight updates in between, equals the eager step on the same values bit
    for bit, every replay."""
    prob = pi.make_problem("ns", N=3000, seed=17, bias_std=0.3, dims=[2, 64, 64, 64, 3])
    params = [(torch.tensor(W, device="cuda"), torch.tensor(b, device="cuda")) for W, b in prob.params]
    x = torch.tensor(prob.x, device="cuda")
    plan = lib.PinnPlan([2, 64, 64, 64, 3], "ns", 3000, precision=prec,
                        coef=prob.coef)
    eager = lib.PinnPlan([2, 64, 64, 64, 3], "ns", 3000, precision=prec, coef=prob.coef)
    graph = plan.capture_step(params, x)
    for rep in range(3):
        graph.launch()
        r_e, loss_e, _, _ = eager.residual(params, x)
        g_e = eager.backward(params, x)
        torch.cuda.synchronize()
        assert torch.equal(graph.r, r_e), rep
        assert torch.equal(graph.loss, loss_e), rep
        for (a, b), (c, d) in zip(graph.grads, g_e):
            assert torch.equal(a, c) and torch.equal(b, d), rep
        # an optimizer-like in-place update between replays
        with torch.no_grad():
            for W, b in params:
                W.mul_(0.99)
                b.add_(0.01)
    graph.close()
    plan.close()
    eager.close()


def test_adam_step_matches_oracle(lib):
    """Three fused Adam steps on a network's parameters against the FP64
    oracle's Adam from the same FP32 starting values and gradients."""
    dims = [2, 64, 64, 3]
    rng = np.random.default_rng(23)
    params = [(torch.tensor(rng.standard_normal((dims[l + 1], dims[l])), dtype=torch.float32, device="cuda"),
               torch.tensor(rng.standard_normal(dims[l + 1]), dtype=torch.float32, device="cuda"))
              for l in range(len(dims) - 1)]
    flat0 = np.concatenate([np.concatenate([W.double().cpu().numpy().ravel(), b.double().cpu().numpy().ravel()])
                            for W, b in params])
    th, m, v = flat0.copy(), np.zeros_like(flat0), np.zeros_like(flat0)
    opt = lib.AdamState(params, lr=1e-3)
    for t in range(1, 4):
        grads = [(torch.tensor(rng.standard_normal(W.shape) * t, dtype=torch.float32, device="cuda"),
                  torch.tensor(rng.standard_normal(b.shape) * t, dtype=torch.float32, device="cuda"))
                 for W, b in params]
        g = np.concatenate([np.concatenate([dW.double().cpu().numpy().ravel(), db.double().cpu().numpy().ravel()])
                            for dW, db in grads])
        opt.step(grads)
        oracle.adam_step(th, g, m, v, t)
        torch.cuda.synchronize()
        got = np.concatenate([np.concatenate([W.double().cpu().numpy().ravel(), b.double().cpu().numpy().ravel()])
                              for W, b in params])
        err = np.max(np.abs(got - th) / np.maximum(np.abs(th), 1.0))
        print(f"step {t}: max err {err:.2e}")
        assert err <= 1e-6, t


def test_training_graph_matches_eager_training(lib):
    """A captured training step (residual, gradient, Adam) replayed four times
    equals four eager training steps bit for bit: parameters, loss and the
    device step counter."""
    dims = [2, 64, 64, 64, 3]
    prob = pi.make_problem("ns", N=4000, seed=29, bias_std=0.3, dims=dims)
    x = torch.tensor(prob.x, device="cuda")
    pg = [(torch.tensor(W, device="cuda"), torch.tensor(b, device="cuda")) for W, b in prob.params]
    pe = [(W.clone(), b.clone()) for W, b in pg]
    plan_g = lib.PinnPlan(dims, "ns", 4000, precision="bf16", coef=prob.coef)
    plan_e = lib.PinnPlan(dims, "ns", 4000, precision="bf16", coef=prob.coef)
    opt_g = lib.AdamState(pg, lr=1e-3)
    opt_e = lib.AdamState(pe, lr=1e-3)
    graph = plan_g.capture_step(pg, x, adam=opt_g)
    grads_e = [(torch.empty_like(W), torch.empty_like(b)) for W, b in pe]
    for k in range(4):
        graph.launch()
        _, loss_e, _, _ = plan_e.residual(pe, x)
        plan_e.backward(pe, x, out=grads_e)
        opt_e.step(grads_e)
        torch.cuda.synchronize()
        assert torch.equal(graph.loss, loss_e), k
        for (a, b), (c, d) in zip(pg, pe):
            assert torch.equal(a, c) and torch.equal(b, d), k
        assert int(graph.step) == k + 1
    graph.close()
    plan_g.close()
    plan_e.close()


@pytest.mark.parametrize("prec", ["bf16", "fp32"])
def test_batch_train_step_matches_eager_training(lib, prec):
    """Three batched training steps (grouped launches with the Adam update in
    one graph) equal three eager single-plan steps with AdamState per network,
    bit for bit: parameters, losses and the device step counter."""
    ens = small_ensemble(n=6, seed=7)
    pb, xs = to_dev(ens)
    pe = [[(W.clone(), b.clone()) for W, b in ps] for ps in pb]
    batch = lib.PinnBatch([m.dims for m in ens], "burgers", [(m.nu,) for m in ens], [m.N for m in ens],
                          precision=prec)
    adam = lib.BatchAdam(pb, lr=1e-3)
    plans = [lib.PinnPlan(m.dims, "burgers", m.N, precision=prec, coef=(m.nu,)) for m in ens]
    opts = [lib.AdamState(ps, lr=1e-3) for ps in pe]
    grads = [[(torch.empty_like(W), torch.empty_like(b)) for W, b in ps] for ps in pe]
    for k in range(3):
        loss_b, _ = batch.train_step(pb, xs, adam)
        losses = []
        for pl, ps, x, opt, g in zip(plans, pe, xs, opts, grads):
            _, l, _, _ = pl.residual(ps, x)
            pl.backward(ps, x, out=g)
            opt.step(g)
            losses.append(l)
        torch.cuda.synchronize()
        assert int(adam.step) == k + 1
        for i in range(len(ens)):
            assert float(loss_b[i]) == float(losses[i]), (k, i)
            for (a, b), (c, d) in zip(pb[i], pe[i]):
                assert torch.equal(a, c) and torch.equal(b, d), (k, i)
    assert batch.launches() > 0
    batch.close()
    for pl in plans:
        pl.close()


def test_batch_profile_times_a_kernel_class(lib):
    """Timing one kernel class runs the grouped launches eagerly with events
    on their lanes; the results equal those of the graph replay."""
    ens = small_ensemble(n=5, seed=8)
    params, xs = to_dev(ens)
    batch = lib.PinnBatch([m.dims for m in ens], "burgers", [(m.nu,) for m in ens], [m.N for m in ens])
    loss, grads = batch.step(params, xs)
    torch.cuda.synchronize()
    ref = (loss.cpu().numpy().copy(), [flat(g) for g in grads])
    batch.profile("layer_fwd")
    loss, grads = batch.step(params, xs)
    ms, n = batch.profile_read()
    batch.profile("off")
    torch.cuda.synchronize()
    assert n >= 1 and ms > 0
    assert np.array_equal(loss.cpu().numpy(), ref[0])
    for a, g in zip(ref[1], grads):
        assert np.array_equal(a, flat(g))
    batch.close()


def test_autotune_cache_hit(lib, tmp_path):
    """A second plan with the same key (width, depth, kind, operand type,
    point-count bucket) takes the cached tuning without timing; the cache
    survives a save and a load."""
    lib.tuning_cache_clear()
    prob = pi.make_problem("ns", N=3000, seed=5, bias_std=0.2, dims=[2, 64, 64, 64, 3])
    params = [(torch.tensor(W, device="cuda"), torch.tensor(b, device="cuda")) for W, b in prob.params]
    x = torch.tensor(prob.x, device="cuda")
    p1 = lib.PinnPlan(prob.workload.dims, "ns", 3000, precision="bf16", coef=prob.coef)
    t1, ms1 = p1.autotune(params, x, reps=2)
    assert lib.tuning_cache_size() == 1
    p2 = lib.PinnPlan(prob.workload.dims, "ns", 3000, precision="bf16", coef=prob.coef)
    t2, ms2 = p2.autotune(params, x, reps=2)
    assert t2 == t1 and ms2 == ms1
    path = str(tmp_path / "cache.txt")
    lib.tuning_cache_save(path)
    lib.tuning_cache_clear()
    lib.tuning_cache_load(path)
    assert lib.tuning_cache_size() == 1
    p1.close()
    p2.close()

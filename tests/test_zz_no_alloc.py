"""The no-allocation entry point pinn_jet_step_noalloc (workspace in a static
device array) against the plan-based entry points pinn_jet_residual +
pinn_jet_backward on a plan of the same shape with the default tuning: the
results must be bit for bit equal.  Two calls in a row, the second with a
smaller input, so that the second call runs on an array that still holds the
first call's contents."""
import numpy as np
import pytest
import torch

import pinn_inputs as pi
from tests.parity import flat

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2606_29702_amd as pj
    return pj


CASES = [("burgers", [2, 32, 32, 32, 1], "fp32", (3000, 1000)),
         ("burgers", [2, 32, 32, 32, 1], "bf16", (3000, 777)),
         ("ns", [2, 128, 128, 128, 128, 3], "bf16", (4000, 1500)),
         ("ks", [2, 64, 64, 64, 1], "fp16", (2500, 300))]


@pytest.mark.parametrize("pde,dims,prec,sizes", CASES)
def test_noalloc_equals_plan_entry_points(lib, pde, dims, prec, sizes):
    for N in sizes:
        prob = pi.make_problem(pde, N=N, seed=N, bias_std=0.3, dims=dims)
        params = [(torch.tensor(W, device="cuda"), torch.tensor(b, device="cuda")) for W, b in prob.params]
        x = torch.tensor(prob.x, device="cuda")
        plan = lib.PinnPlan(dims, pde, N, precision=prec, coef=prob.coef)
        r1, l1, _, _ = plan.residual(params, x)
        g1 = plan.backward(params, x)
        r2, l2, g2 = lib.jet_step_noalloc(params, x, pde, prob.coef, precision=prec)
        torch.cuda.synchronize()
        print(pde, prec, N, f"loss {float(l1):.6e} / {float(l2):.6e}")
        assert torch.equal(r1, r2), (N, "r")
        assert torch.equal(l1, l2), (N, "loss")
        assert np.array_equal(flat(g1), flat(g2)), (N, "grad")
        plan.close()


def test_noalloc_rejects_a_workspace_beyond_the_array(lib):
    from paper_2606_29702_amd import PinnError
    prob = pi.make_problem("ns", N=65536)
    params = [(torch.tensor(W, device="cuda"), torch.tensor(b, device="cuda")) for W, b in prob.params]
    x = torch.tensor(prob.x, device="cuda")
    with pytest.raises(PinnError) as e:
        lib.jet_step_noalloc(params, x, "ns", prob.coef, precision="bf16")
    assert e.value.status == -6 and "static scratch" in str(e.value)

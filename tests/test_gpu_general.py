"""Networks over variables of general dimension L (Sec. 2.1) through the
binary expansion of qbe_model_create_dims, contracted on the device in both
forms with slicing, against the oracle's direct complex128 sum.  Tolerance
as in test_gpu_parity (relative 1e-5), floored at 1e-5 of the sum of the
absolute products' scale for sums that cancel."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    assert torch.cuda.is_available()
    import paper_2004_10892_amd as qbe
    return qbe, qbe.Context(0)


@pytest.mark.parametrize("form", ["fused", "per_step"])
def test_general_dimension_networks_vs_direct_sum(env, form):
    qbe, ctx = env
    from circuitgen import random_general_network
    from oracle import general as Gn
    for seed in range(8):
        dims, tensors = random_general_network(seed, n_vars=9, n_tensors=9, max_rank=3, max_dim=5)
        want = Gn.contract_general(dims, tensors)
        scale = Gn.contract_general(dims, [(vs, np.abs(d)) for vs, d in tensors]).real
        qm = qbe.Model.from_dims(dims, tensors)
        order = qbe.qbe_order_min_fill(qm)
        m = min(3, qm.n_vars)
        mu, pi, _ = qbe.qbe_slice(qm, order, m)
        plan = qbe.Plan(qm, pi, mu, ctx=ctx, exec=form)
        print(f"case general seed={seed} dims={dims} {form} m={m}", flush=True)
        got = qbe.qbe_contract(ctx, plan, plan.workspace())
        assert abs(got - want) <= 1e-5 * max(abs(want), 1e-5 * scale), (seed, got, want)

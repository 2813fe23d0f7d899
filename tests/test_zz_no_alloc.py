"""qbe_contract_static (the allocation-free entry: the library's fixed
per-device workspace instead of a caller's) against qbe_contract_async on
the same plans, called through the C ABI: two calls in a row, the second on
a smaller input, plus the rejection of a plan whose workspace exceeds the
fixed size.  Bar: relative 1e-5 (both run the same kernels; the slice-group
size may differ with the workspace, the FP64 slice sum order does not)."""
import json
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(__file__), "golden", "amplitudes.json")


def _plan(qbe, ctx, name, form):
    from circuitgen import WORKLOADS, circuit_model, random_grid_circuit
    with open(GOLD) as f:
        seed = json.load(f)[name]["seed"]
    r, c, d, m = WORKLOADS[name]
    qm = qbe.Model.from_circuitgen(circuit_model(random_grid_circuit(r, c, d, seed)))
    _, mu, pi, _ = qbe.plan_circuit(qm, m=m)
    return qm, qbe.Plan(qm, pi, mu, ctx=ctx, exec=form)


def test_static_entry_matches_workspace_entry():
    import torch
    import paper_2004_10892_amd as qbe
    assert torch.cuda.is_available()
    ctx = qbe.Context(0)
    assert qbe.qbe_static_scratch_bytes() == 64 << 20
    # larger input first (per-step, 64 slices in slice groups), then smaller
    # ones: the second and third calls reuse the scratch the first one left
    cases = [("grid5x5_d16_m6", "per_step"), ("grid4x4_d10_m0", "fused"), ("grid4x4_d10_m0", "per_step"),
             ("grid5x5_d16_m6", "fused")]
    for name, form in cases:
        qm, plan = _plan(qbe, ctx, name, form)
        print(f"case static {name} {form} ws_min {plan.stats()['ws_bytes_min']}", flush=True)
        ref = torch.zeros(2, dtype=torch.float64, device="cuda")
        qbe.qbe_contract_async(ctx, plan, plan.workspace(), ref)
        got = torch.full((2,), float("nan"), dtype=torch.float64, device="cuda")
        qbe.qbe_contract_static(ctx, plan, got)
        torch.cuda.synchronize()
        a = complex(*got.cpu().numpy())
        b = complex(*ref.cpu().numpy())
        assert abs(a - b) <= 1e-5 * abs(b), (name, form, a, b)
        with open(GOLD) as f:
            want = complex(*json.load(f)[name]["oracle"])
        assert abs(a - want) <= 1e-5 * abs(want), (name, form, a, want)


def test_static_entry_rejects_plans_beyond_the_scratch():
    import torch
    import paper_2004_10892_amd as qbe
    from circuitgen import star_network
    ctx = qbe.Context(0)
    # hub-first star of 24 leaves: a rank-24 intermediate, 128 MiB a slice
    qm = qbe.Model.from_circuitgen(star_network(24, seed=1))
    plan = qbe.Plan(qm, list(range(25)), [], ctx=ctx, exec="per_step")
    assert plan.stats()["ws_bytes_min"] > qbe.qbe_static_scratch_bytes()
    out = torch.zeros(2, dtype=torch.float64, device="cuda")
    with pytest.raises(qbe.QbeError, match="MEM_CAP"):
        qbe.qbe_contract_static(ctx, plan, out)
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy(), np.zeros(2))

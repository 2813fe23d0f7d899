"""Plans made with Alg. 2's optional order recomputation (every k-th removal
the reduced order becomes Alg. 5's order of the anytime heuristic's tree
decomposition of the reduced graph) contracted on the device.  Slicing and
the order change the schedule, never the sum (Eqs. 2-4): the amplitude must
match the stored oracle amplitude of the workload at relative 1e-5, and the
host plan must equal the oracle's recomputed plan exactly."""
import json
import os

import pytest

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(__file__), "golden", "amplitudes.json")


@pytest.mark.parametrize("form", ["fused", "per_step"])
@pytest.mark.parametrize("every", [1, 2])
def test_recomputed_plan_contracts_to_the_oracle_amplitude(form, every):
    import torch
    import paper_2004_10892_amd as qbe
    from circuitgen import circuit_model, random_grid_circuit
    from oracle import planner as P
    assert torch.cuda.is_available()
    with open(GOLD) as f:
        g = json.load(f)["grid5x5_d16_m6"]
    want = complex(*g["oracle"])
    mod = circuit_model(random_grid_circuit(5, 5, 16, g["seed"]))
    qm = qbe.Model.from_circuitgen(mod)
    order = qbe.qbe_order_min_fill(qm)
    mu, pi, tau = qbe.qbe_slice(qm, order, 6, recompute_every=every, tries=4, seed=11)
    adj = P.simple_graph(mod.n_vars, [v for v, _ in mod.tensors])
    o_mu, _, o_pi, o_tau = P.greedy_treewidth_deletion_recompute(adj, P.min_fill_order(adj), 6, every, 4, 11)
    assert (mu, pi, tau) == (o_mu, o_pi, o_tau)
    plain_pi = [v for v in order if v not in mu]
    print(f"case 5x5 d16 recompute every {every} {form}: tau {tau}, order changed {pi != plain_pi}", flush=True)
    ctx = qbe.Context(0)
    plan = qbe.Plan(qm, pi, mu, ctx=ctx, exec=form)
    got = qbe.qbe_contract(ctx, plan, plan.workspace())
    assert abs(got - want) <= 1e-5 * abs(want), (got, want)

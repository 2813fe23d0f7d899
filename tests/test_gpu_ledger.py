"""The slice ledger over a real contraction (Sec. 2.4, Eq. 4): the 7x7
depth-24 circuit with the benchmark's sliced set (min-fill order,
tree-trimming with recomputation after every second removal, 16 tries, seed
5; 1024 slices) and its plan form (fused prefix and segments, merged
launches of at most two summed variables), in ranges of 96 slices (the last
one 64).  The job stops after four ranges, is saved, one recorded range is
dropped as lost, and the loaded ledger runs the rest: its sum must match the
oracle's amplitude at relative 1e-5 and the one-call contraction to FP64
rounding of the slice sum (bounded by 1e-12 of the sum of the slices'
magnitudes)."""
import json
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(__file__), "golden", "amplitudes.json")


@pytest.fixture(scope="module")
def case():
    import torch
    assert torch.cuda.is_available()
    import paper_2004_10892_amd as qbe
    from circuitgen import circuit_model, random_grid_circuit
    g = json.load(open(GOLD))["grid7x7_d24_m10"]
    qm = qbe.Model.from_circuitgen(circuit_model(random_grid_circuit(7, 7, 24, g["seed"])))
    mu, pi, _ = qbe.qbe_slice(qm, qbe.qbe_order_min_fill(qm), 10, recompute_every=2, tries=16, seed=5)
    ctx = qbe.Context(0)
    plan = qbe.Plan(qm, pi, mu, ctx=ctx, exec="per_step", fused_prefix=True, fused_segments=True, max_sums=2)
    return qbe, ctx, plan, complex(*g["oracle"])


def test_interrupted_job_resumes_after_a_lost_range(case, tmp_path):
    qbe, ctx, plan, want = case
    ws = plan.workspace()
    print("case ledger 7x7 d24: 1024 slices in ranges of 96", flush=True)
    led = qbe.Ledger(1024, 96, tag=2024)
    assert led.run(ctx, plan, ws, max_ranges=4) == 4
    assert led.next()[0] == 4
    path = str(tmp_path / "job.ledger")
    led.save(path)
    led.close()
    res = qbe.Ledger.load(path)
    res.drop(2)
    assert res.info()["n_done"] == 3
    assert res.run(ctx, plan, ws) == 11 - 3
    assert res.next() is None
    got = res.sum()
    assert abs(got - want) <= 1e-5 * abs(want)
    full, per = qbe.qbe_contract_slices(ctx, plan, 0, 1024, ws)
    assert abs(got - full) <= 1e-12 * np.abs(per).sum()
    # each recorded range is that range's own contraction
    done, part = res.get(10)
    one, _ = qbe.qbe_contract_slices(ctx, plan, 960, 1024, ws)
    assert done and part == one


def test_run_rejects_a_plan_of_another_slice_count(case):
    qbe, ctx, plan, _ = case
    led = qbe.Ledger(512, 64)
    with pytest.raises(qbe.QbeError, match="slice count"):
        led.run(ctx, plan, plan.workspace())
    assert led.info()["n_done"] == 0

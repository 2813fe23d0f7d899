"""The asynchronous entry points under HIP graph capture: every replay, with
eager work and synchronisations in between, must reproduce the eager result
bit for bit (the library records kernels only -- no memset or copy nodes)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _capture(torch, ctx, fn):
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        ctx.set_stream(s)
        fn()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    with torch.cuda.graph(g):
        ctx.set_stream(torch.cuda.current_stream())
        fn()
    ctx.set_stream(torch.cuda.current_stream())
    return g


@pytest.mark.parametrize("form", ["fused", "per_step", "per_step_tuned", "per_step_prefix", "per_step_segments"])
def test_plan_graph_replays_match_eager(form):
    import torch
    import paper_2004_10892_amd as qbe
    from circuitgen import circuit_model, random_grid_circuit
    print(f"case graph replay {form}", flush=True)
    ctx = qbe.Context(0)
    qm = qbe.Model.from_circuitgen(circuit_model(random_grid_circuit(5, 5, 16, 1)))
    _, mu, pi, _ = qbe.plan_circuit(qm, m=6)
    plan = qbe.Plan(qm, pi, mu, ctx=ctx, exec="fused" if form == "fused" else "per_step",
                    fused_prefix=form.endswith(("_prefix", "_segments")), fused_segments=form.endswith("_segments"))
    ws = plan.workspace()
    if form.endswith("_tuned"):
        plan.autotune(ws, min_elems=1 << 10)  # tuned launch shapes, as the benchmark captures them
    eager = qbe.qbe_contract(ctx, plan, ws)
    out = torch.zeros(2, dtype=torch.float64, device="cuda")
    g = _capture(torch, ctx, lambda: qbe.qbe_contract_async(ctx, plan, ws, out))
    for rep in range(4):
        out.fill_(float("nan"))
        junk = torch.randn(1 << 16, device="cuda") * 3.0  # eager work between replays
        g.replay()
        torch.cuda.synchronize()
        got = complex(*out.cpu().numpy())
        assert got == eager, (rep, got, eager)
        assert qbe.qbe_contract(ctx, plan, ws) == eager
        del junk


def test_batch_graph_replays_match_eager():
    import torch
    import paper_2004_10892_amd as qbe
    from circuitgen import batch_instances, circuit_model, random_grid_circuit
    print("case graph replay batch", flush=True)
    ctx = qbe.Context(0)
    plans = []
    for (r, c, d, m, seed) in batch_instances(40):
        qm = qbe.Model.from_circuitgen(circuit_model(random_grid_circuit(r, c, d, seed)))
        _, mu, pi, _ = qbe.plan_circuit(qm, m=m)
        plans.append(qbe.Plan(qm, pi, mu, ctx=ctx))
    batch = qbe.Batch(ctx, plans)
    ws = batch.workspace()
    amps = torch.zeros(2 * len(plans), dtype=torch.float64, device="cuda")
    batch.contract_async(ws, amps)
    torch.cuda.synchronize()
    eager = amps.cpu().numpy().copy()
    g = _capture(torch, ctx, lambda: batch.contract_async(ws, amps))
    for rep in range(4):
        amps.fill_(float("nan"))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(amps.cpu().numpy(), eager), rep

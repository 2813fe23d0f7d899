"""Many amplitudes of one circuit: plans cloned per output bitstring (same
schedule and programs, other entries), contracted one by one and as one
batch, against the complex128 oracle.  Tolerance as in test_gpu_parity:
relative 1e-5, floored at 1e-2 of a typical amplitude 2^(-n/2) for
amplitudes that cancel to near zero."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

TOL = 1e-5


@pytest.fixture(scope="module")
def qbe():
    import torch
    assert torch.cuda.is_available()
    import paper_2004_10892_amd as q
    return q


@pytest.fixture(scope="module")
def ctx(qbe):
    return qbe.Context(0)


def _oracle(mod, pi, mu):
    from oracle import contract as C
    sched = C.bucket_schedule(mod.n_vars, [v for v, _ in mod.tensors], list(pi), list(mu))
    return C.contract(mod.tensors, sched)[0]


@pytest.mark.parametrize("form", ["fused", "per_step"])
def test_clones_per_bitstring_match_oracle(qbe, ctx, form):
    import torch
    from circuitgen import circuit_model, random_grid_circuit
    circ = random_grid_circuit(4, 4, 10, 3)
    xs = [circ.bitstring, 0, (1 << 16) - 1, 0x5A5A, 0x1234, 0xBEEF]
    mods = [circuit_model(circ, x) for x in xs]
    qms = [qbe.Model.from_circuitgen(m) for m in mods]
    _, mu, pi, _ = qbe.plan_circuit(qms[0], m=2)
    base = qbe.Plan(qms[0], pi, mu, ctx=ctx, exec=form)
    clones = [base.clone(q) for q in qms[1:]]
    plans = [base] + clones
    print(f"case clones {form}: {len(plans)} bitstrings", flush=True)
    scale = 2.0 ** (-16 / 2) * 1e-2
    wants = [_oracle(m, pi, mu) for m in mods]
    for p, w, q in zip(plans, wants, qms):
        got = qbe.qbe_contract(ctx, p, p.workspace())
        assert abs(got - w) <= TOL * max(abs(w), scale)
        # a plan created from scratch runs the same program on the same data
        fresh = qbe.Plan(q, pi, mu, ctx=ctx, exec=form)
        assert qbe.qbe_contract(ctx, fresh, fresh.workspace()) == got
        fresh.close()
    # one batched launch over every bitstring
    batch = qbe.Batch(ctx, plans)
    amps = torch.zeros(2 * len(plans), dtype=torch.float64, device="cuda")
    batch.contract_async(batch.workspace(), amps)
    torch.cuda.synchronize()
    got = amps.cpu().numpy().view(np.complex128)
    for g, w in zip(got, wants):
        assert abs(g - w) <= TOL * max(abs(w), scale)
    batch.close()
    # the clones own their device memory: they outlive the plan they came from
    base.close()
    g1 = qbe.qbe_contract(ctx, clones[0], clones[0].workspace())
    assert abs(g1 - wants[1]) <= TOL * max(abs(wants[1]), scale)


def test_clone_rejects_other_structure(qbe, ctx):
    from circuitgen import circuit_model, random_grid_circuit
    a = qbe.Model.from_circuitgen(circuit_model(random_grid_circuit(3, 3, 6, 1)))
    b = qbe.Model.from_circuitgen(circuit_model(random_grid_circuit(3, 3, 7, 1)))
    _, mu, pi, _ = qbe.plan_circuit(a, m=1)
    p = qbe.Plan(a, pi, mu, ctx=ctx)
    with pytest.raises(qbe.QbeError):
        p.clone(b)

"""The largest intermediate the interface allows: a hub variable joined to
30 leaves, eliminated hub first, makes a rank-30 result (2^30 complex64
entries, 8 GiB a slice); the next bucket sums a leaf out of it, whose u = 1
entries sit 2^32 bytes above the u = 0 ones.  Sum over all assignments
factorises (Sec. 2.1, Eq. 2 with the hub last):
    sigma = sum_h prod_i (sum_{v_i} T_i[h, v_i]),
a closed form that the test evaluates directly in complex128."""
import numpy as np
import pytest

N_LEAVES = 30


def closed_form(model):
    total = 0j
    for h in (0, 1):
        prod = 1 + 0j
        for _, d in model.tensors:
            prod *= d[h, 0] + d[h, 1]
        total += prod
    return total


def star_plan_inputs(qbe, model):
    qm = qbe.Model.from_circuitgen(model)
    order = list(range(model.n_vars))  # hub, then the leaves
    return qm, order


def test_star_closed_form_equals_oracle_small():
    """The closed form agrees with the oracle's bucket elimination on a star
    small enough for the oracle (12 leaves, hub first and hub last)."""
    from circuitgen import star_network
    from oracle import contract as C
    m = star_network(12, seed=3)
    tv = [v for v, _ in m.tensors]
    for order in (list(range(13)), list(range(1, 13)) + [0]):
        got, _ = C.contract(m.tensors, C.bucket_schedule(m.n_vars, tv, order, []))
        assert abs(got - closed_form(m)) <= 1e-12 * abs(closed_form(m))


def test_rank30_plan_passes_host_check():
    import paper_2004_10892_amd as qbe
    from circuitgen import star_network
    qm, order = star_plan_inputs(qbe, star_network(N_LEAVES, seed=5))
    plan = qbe.Plan(qm, order, [], exec="per_step")
    st = plan.stats()
    assert st["width"] == N_LEAVES
    plan.check()


@pytest.mark.gpu
def test_rank30_intermediate_on_device():
    import torch
    import paper_2004_10892_amd as qbe
    from circuitgen import star_network
    assert torch.cuda.is_available()
    model = star_network(N_LEAVES, seed=5)
    want = closed_form(model)
    ctx = qbe.Context(0)
    qm, order = star_plan_inputs(qbe, model)
    plan = qbe.Plan(qm, order, [], ctx=ctx, exec="per_step")
    st = plan.stats()
    print(f"case star{N_LEAVES} rank-30 per-step ws {st['ws_bytes_min'] / 2**30:.1f} GiB", flush=True)
    ws = torch.empty(int(st["ws_bytes_min"]), dtype=torch.uint8, device="cuda")
    got = qbe.qbe_contract(ctx, plan, ws)
    del ws
    torch.cuda.empty_cache()
    # products of 30 factors of positive-real-part entries: no cancellation,
    # FP32 rounding along 30 products and 30 pairwise levels of sums
    assert abs(got - want) <= 1e-5 * abs(want), (got, want)

"""Fused-prefix plans on the host (no device): which buckets the prefix
takes, the plan check over its program and exports, the per-launch view,
and the option's validation."""
import pytest


@pytest.fixture(scope="module")
def c3():
    import paper_2004_10892_amd as qbe
    from circuitgen import circuit_model, random_grid_circuit
    qm = qbe.Model.from_circuitgen(circuit_model(random_grid_circuit(7, 7, 24, 1)))
    _, mu, pi, _ = qbe.plan_circuit(qm, m=10)
    return qbe, qm, mu, pi


def test_prefix_takes_small_buckets_and_keeps_the_byte_count(c3):
    qbe, qm, mu, pi = c3
    plain = qbe.Plan(qm, pi, mu, exec="per_step")
    pre = qbe.Plan(qm, pi, mu, exec="per_step", fused_prefix=True)
    pre.check()
    sp, sq = plain.stats(), pre.stats()
    assert sp["prefix_buckets"] == 0 and sq["prefix_buckets"] >= 2
    assert sq["n_steps"] == sp["n_steps"]
    # fewer launches; the prefix keeps its intermediates in LDS, so the
    # per-slice bytes the plan moves through device memory do not grow
    assert sq["n_launches"] < sp["n_launches"]
    assert sq["step_bytes_per_slice"] <= sp["step_bytes_per_slice"]
    la = pre.launches()
    assert la[0]["kind"] == "prefix" and la[0]["n_buckets"] == sq["prefix_buckets"]
    assert 4 <= la[0]["out_rank"] <= 14
    assert [l["kind"] for l in la[-2:]] == ["finalize", "reduce"]
    assert "prefix" not in [l["kind"] for l in la[1:]]
    assert len(la) == sq["n_launches"] + 2
    # the plan's step bytes are the sum over its contraction launches
    assert sum(l["bytes_per_slice"] for l in la[:-2]) == sq["step_bytes_per_slice"]
    assert sum(l["bytes_per_slice"] for l in plain.launches()[:-2]) == sp["step_bytes_per_slice"]


def test_prefix_needs_merging_and_is_ignored_by_fused_plans(c3):
    qbe, qm, mu, pi = c3
    assert qbe.Plan(qm, pi, mu, exec="per_step", merge=False, fused_prefix=True).stats()["prefix_buckets"] == 0
    from circuitgen import circuit_model, random_grid_circuit
    small = qbe.Model.from_circuitgen(circuit_model(random_grid_circuit(5, 5, 16, 1)))
    _, mu5, pi5, _ = qbe.plan_circuit(small, m=6)
    fused = qbe.Plan(small, pi5, mu5, exec="fused", fused_prefix=True)
    assert fused.stats()["exec"] == qbe.EXEC["fused"] and fused.stats()["prefix_buckets"] == 0
    auto = qbe.Plan(small, pi5, mu5, fused_prefix=True)
    if auto.stats()["exec"] == qbe.EXEC["fused"]:
        assert auto.stats()["prefix_buckets"] == 0
    per = qbe.Plan(small, pi5, mu5, exec="per_step", fused_prefix=True)
    per.check()
    assert per.stats()["prefix_buckets"] >= 2


def test_prefix_option_validation(c3):
    import ctypes as C
    import paper_2004_10892_amd as qbe
    _, qm, mu, pi = c3
    o = qbe.PlanOpts()
    o.exec = qbe.EXEC["per_step"]
    o.fused_prefix = 15
    h = C.c_void_p()
    import numpy as np
    po = np.asarray(pi, dtype=np.int32)
    pm = np.asarray(mu, dtype=np.int32)
    rc = qbe._lib.qbe_plan_create(None, qm.handle, po.ctypes.data_as(C.POINTER(C.c_int32)), len(po),
                                  pm.ctypes.data_as(C.POINTER(C.c_int32)), len(pm), C.byref(o), C.byref(h))
    assert qbe.ERRORS[rc] == "INVALID_ARG"
    assert "fused_prefix" in qbe._lib.qbe_last_error().decode()


def test_explicit_rank_bounds(c3):
    """fused_prefix = R takes the buckets of at most R + 1 variables whose
    producers all are such: a larger bound takes a superset."""
    qbe, qm, mu, pi = c3
    prev = 0
    for R in (4, 6, 8, 10):
        p = qbe.Plan(qm, pi, mu, exec="per_step", fused_prefix=R)
        p.check()
        la = p.launches()
        assert la[0]["kind"] == "prefix" and la[0]["out_rank"] == R
        assert la[0]["levels"] > 0 and 0 < la[0]["lds_bytes"] <= 160 * 1024
        assert all(l["levels"] == 0 and l["lds_bytes"] == 0 for l in la[1:])
        n = p.stats()["prefix_buckets"]
        assert n >= prev
        prev = n
    # the automatic bound: the largest whose prefix lets two workgroups
    # share a compute unit's 160 KB of LDS
    pair = 160 * 1024 // 2 - 16
    auto = qbe.Plan(qm, pi, mu, exec="per_step", fused_prefix=True).launches()[0]
    R = auto["out_rank"]
    assert auto["kind"] == "prefix" and auto["lds_bytes"] <= pair
    for bigger in range(R + 1, 15):
        la = qbe.Plan(qm, pi, mu, exec="per_step", fused_prefix=bigger).launches()[0]
        assert la["kind"] != "prefix" or la["lds_bytes"] > pair

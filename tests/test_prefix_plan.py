"""Fused-prefix and fused-segment plans on the host (no device): which
buckets they take, the plan check over their programs and rows, the
per-launch view, and the options' validation."""
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


def test_later_segments_take_runs_of_small_buckets(c3):
    """fused_segments: runs of at least three small buckets after the prefix
    become one launch each, importing what they read; the byte count of
    the plan is still the sum over its launches, and no bucket is lost."""
    qbe, qm, mu, pi = c3
    pre = qbe.Plan(qm, pi, mu, exec="per_step", fused_prefix=11)
    seg = qbe.Plan(qm, pi, mu, exec="per_step", fused_prefix=11, fused_segments=True)
    seg.check()
    sp, sq = pre.stats(), seg.stats()
    assert sp["n_fused_segments"] == 1 and sq["n_fused_segments"] >= 2
    assert sq["prefix_buckets"] == sp["prefix_buckets"]
    assert sq["fused_buckets"] > sp["fused_buckets"]
    assert sq["n_launches"] < sp["n_launches"]
    la = seg.launches()
    kinds = [l["kind"] for l in la]
    assert kinds[0] == "prefix" and kinds.count("prefix") == 1
    segs = [l for l in la if l["kind"] == "segment"]
    assert len(segs) == sq["n_fused_segments"] - 1
    assert sum(l["n_buckets"] for l in la if l["kind"] in ("prefix", "segment")) == sq["fused_buckets"]
    for l in segs:
        assert l["n_buckets"] >= 3 and l["n_ops"] >= 1 and l["levels"] > 0 and 0 < l["lds_bytes"] <= 160 * 1024
    assert sum(l["bytes_per_slice"] for l in la[:-2]) == sq["step_bytes_per_slice"]
    assert [l["kind"] for l in la[-2:]] == ["finalize", "reduce"]


def test_automatic_bound_with_segments_keeps_every_fused_launch_in_half_the_lds(c3):
    """With fused segments the automatic bound is the largest R whose prefix
    and every later run of small buckets fit in half a compute unit's LDS
    (two workgroups per unit), when some R allows that: its launches all
    do, and the explicit bound R gives the same launches."""
    qbe, qm, mu, pi = c3
    pair = 160 * 1024 // 2 - 16
    fused = lambda p: [l for l in p.launches() if l["kind"] in ("prefix", "segment")]
    auto = qbe.Plan(qm, pi, mu, exec="per_step", fused_prefix=True, fused_segments=True)
    auto.check()
    la = fused(auto)
    R = la[0]["out_rank"]
    assert la[0]["kind"] == "prefix" and all(l["lds_bytes"] <= pair for l in la)
    assert auto.stats()["fused_buckets"] == sum(l["n_buckets"] for l in la)
    same = qbe.Plan(qm, pi, mu, exec="per_step", fused_prefix=R, fused_segments=True)
    assert [l["lds_bytes"] for l in fused(same)] == [l["lds_bytes"] for l in la]


def test_segment_option_validation(c3):
    import ctypes as C
    import numpy as np
    import paper_2004_10892_amd as qbe
    _, qm, mu, pi = c3
    po = np.asarray(pi, dtype=np.int32)
    pm = np.asarray(mu, dtype=np.int32)
    for prefix, segments, what in ((0, 1, "fused_segments needs"), (1, 2, "fused_segments must")):
        o = qbe.PlanOpts()
        o.exec = qbe.EXEC["per_step"]
        o.fused_prefix = prefix
        o.fused_segments = segments
        h = C.c_void_p()
        rc = qbe._lib.qbe_plan_create(None, qm.handle, po.ctypes.data_as(C.POINTER(C.c_int32)), len(po),
                                      pm.ctypes.data_as(C.POINTER(C.c_int32)), len(pm), C.byref(o), C.byref(h))
        assert qbe.ERRORS[rc] == "INVALID_ARG"
        assert what in qbe._lib.qbe_last_error().decode()


@pytest.mark.parametrize("seed", range(4))
def test_segment_plans_of_random_circuits_pass_the_plan_check(seed):
    """Segments over other schedules (orders from the anytime heuristic,
    several slicing sizes): every plan passes the host check of every
    index its kernels and rows can form."""
    import paper_2004_10892_amd as qbe
    from circuitgen import circuit_model, random_grid_circuit
    qm = qbe.Model.from_circuitgen(circuit_model(random_grid_circuit(5 + seed % 2, 6, 12 + 4 * seed, 50 + seed)))
    for m in (0, 2, 5):
        _, mu, pi, _ = qbe.plan_circuit(qm, m=m)
        for R in (True, 4, 7):
            p = qbe.Plan(qm, pi, mu, exec="per_step", fused_prefix=R, fused_segments=True)
            p.check()
            st = p.stats()
            assert st["fused_buckets"] <= st["n_steps"]

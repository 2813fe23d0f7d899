"""Input folding on the host (no device): a plan multiplies the input tensors
of a bucket into one tensor once (Eq. 2's product of the bucket's tensors,
regrouped), so its launches carry fewer factors, while its schedule dump and
cost model stay those of the caller's model.  The folded data itself is
checked entry by entry in the sanitizer build (tests/native), and the
amplitudes of folded plans against the oracle in the GPU tests, which use
folding by default."""
import ctypes as C

import numpy as np
import pytest


@pytest.fixture(scope="module")
def c3():
    import paper_2004_10892_amd as qbe
    from circuitgen import circuit_model, random_grid_circuit
    qm = qbe.Model.from_circuitgen(circuit_model(random_grid_circuit(7, 7, 24, 1)))
    _, mu, pi, _ = qbe.plan_circuit(qm, m=10)
    return qbe, qm, mu, pi


def test_folding_keeps_the_schedule_and_cost_model(c3):
    qbe, qm, mu, pi = c3
    a = qbe.Plan(qm, pi, mu, exec="per_step", fold_inputs=False)
    b = qbe.Plan(qm, pi, mu, exec="per_step", fold_inputs=True)
    b.check()
    assert a.dump() == b.dump()
    sa, sb = a.stats(), b.stats()
    for k in ("n_vars", "n_tensors", "m", "width", "n_steps", "flops_per_slice", "bytes_per_slice",
              "peak_bytes_per_slice"):
        assert sa[k] == sb[k], k


def test_folding_leaves_fewer_factors_per_bucket(c3):
    """One launch per bucket (small ones grouped by level): the folded
    plan's launches multiply fewer factors in all, and none more than the
    most the unfolded plan has."""
    qbe, qm, mu, pi = c3
    la = qbe.Plan(qm, pi, mu, exec="per_step", merge=False, fold_inputs=False).launches()
    lb = qbe.Plan(qm, pi, mu, exec="per_step", merge=False, fold_inputs=True).launches()
    ka = [l["n_ops"] for l in la if l["kind"] == "bucket"]
    kb = [l["n_ops"] for l in lb if l["kind"] == "bucket"]
    assert max(kb) <= max(ka)
    assert sum(kb) < sum(ka)
    # the folded plans of the other forms pass the host check too
    for kw in (dict(exec="per_step"), dict(exec="per_step", fused_prefix=True, fused_segments=True)):
        qbe.Plan(qm, pi, mu, fold_inputs=True, **kw).check()


def test_clones_of_a_folded_plan_take_the_callers_structure(c3):
    qbe, qm, mu, pi = c3
    from circuitgen import circuit_model, random_grid_circuit
    plan = qbe.Plan(qm, pi, mu, exec="per_step", fused_prefix=True)
    other = qbe.Model.from_circuitgen(circuit_model(random_grid_circuit(7, 7, 24, 1), 5))
    twin = plan.clone(other)
    twin.check()
    assert twin.dump() == plan.dump()
    twin.update_data(qm)
    different = qbe.Model.from_circuitgen(circuit_model(random_grid_circuit(7, 7, 24, 2)))
    with pytest.raises(qbe.QbeError):
        plan.clone(different)


def test_no_fold_option_validation(c3):
    qbe, qm, mu, pi = c3
    o = qbe.PlanOpts()
    o.exec = qbe.EXEC["per_step"]
    o.no_fold = 2
    h = C.c_void_p()
    po = np.asarray(pi, dtype=np.int32)
    pm = np.asarray(mu, dtype=np.int32)
    rc = qbe._lib.qbe_plan_create(None, qm.handle, po.ctypes.data_as(C.POINTER(C.c_int32)), len(po),
                                  pm.ctypes.data_as(C.POINTER(C.c_int32)), len(pm), C.byref(o), C.byref(h))
    assert qbe.ERRORS[rc] == "INVALID_ARG"
    assert "no_fold" in qbe._lib.qbe_last_error().decode()


def test_max_sums_caps_the_summed_variables_of_merged_launches(c3):
    """qbe_plan_opts.max_sums: no per-step launch sums more variables than
    the cap (1: one launch per bucket); the schedule and cost model stay."""
    qbe, qm, mu, pi = c3
    base = qbe.Plan(qm, pi, mu, exec="per_step")
    assert max(l["n_sum"] for l in base.launches()) > 2
    for cap in (1, 2, 3):
        p = qbe.Plan(qm, pi, mu, exec="per_step", max_sums=cap)
        p.check()
        assert max(l["n_sum"] for l in p.launches()) <= cap
        assert p.dump() == base.dump()
        assert p.stats()["flops_per_slice"] == base.stats()["flops_per_slice"]
    o = qbe.PlanOpts()
    o.exec = qbe.EXEC["per_step"]
    o.max_sums = 5
    h = C.c_void_p()
    po = np.asarray(pi, dtype=np.int32)
    pm = np.asarray(mu, dtype=np.int32)
    rc = qbe._lib.qbe_plan_create(None, qm.handle, po.ctypes.data_as(C.POINTER(C.c_int32)), len(po),
                                  pm.ctypes.data_as(C.POINTER(C.c_int32)), len(pm), C.byref(o), C.byref(h))
    assert qbe.ERRORS[rc] == "INVALID_ARG"
    assert "max_sums" in qbe._lib.qbe_last_error().decode()

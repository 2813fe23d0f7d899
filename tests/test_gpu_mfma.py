"""Outer-product buckets on MFMA (FP32 and split-BF16) against the oracle.

Split-BF16 error bound used below: a float x is split into hi = bf16(x) and
lo = bf16(x - hi); hi + lo differs from x by at most 2^-17 |x|, and dropping
lo*lo costs at most 2^-18 |a b|, so one product carries a relative error of
at most 2.5 * 2^-17 (1.9e-5); the bound for a whole result is that per-product
figure times the number of split products along its longest chain, with the
same floor at the r.m.s. value as the FP32 tests.  The three-part split
(bf16x6: x = h + m + l, residual at most 2^-26 |x|, dropped products m*l,
l*m, l*l at most 2^-25 |a b| together) is held to the FP32 tolerance.
"""
import json
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(__file__), "golden")
SPLIT_EPS = 2.5 * 2.0 ** -17


@pytest.fixture(scope="module")
def env():
    import torch
    assert torch.cuda.is_available()
    import paper_2004_10892_amd as qbe
    return qbe, qbe.Context(0)


def outer_product_network(seed, n_c=2, n_a=5, n_b=4, u_ops=2):
    """A(u, c.., a..) B(u, c.., b..) plus rank-1 tensors on u: eliminating u
    first is one outer-product bucket with 2^n_c batches of 2^n_a x 2^n_b."""
    rng = np.random.default_rng(seed)
    u = 0
    c = list(range(1, 1 + n_c))
    av = list(range(1 + n_c, 1 + n_c + n_a))
    bv = list(range(1 + n_c + n_a, 1 + n_c + n_a + n_b))
    n = 1 + n_c + n_a + n_b

    def t(vs):
        shape = (2,) * len(vs)
        return (tuple(vs), rng.standard_normal(shape) + 1j * rng.standard_normal(shape))
    tensors = [t([u] + c + av), t(c + [u] + bv)]
    tensors += [t([u]) for _ in range(u_ops)]
    # close the remaining variables so the network sums to a scalar
    tensors += [t([v]) for v in c + av + bv]
    return n, tensors


@pytest.mark.parametrize("prec", ["fp32", "bf16x3", "bf16x6"])
@pytest.mark.parametrize("seed,m", [(0, 0), (1, 1), (2, 2), (3, 0)])
def test_outer_product_bucket_vs_brute_force(env, prec, seed, m):
    qbe, ctx = env
    from oracle import contract as C
    n, tensors = outer_product_network(seed, n_b=6, u_ops=seed % 3)
    order = list(range(n))
    # slice the last m variables (they are A- or B-private)
    mu = order[n - m:] if m else []
    pi = order[:n - m]
    qm = qbe.Model(n, tensors)
    # one launch per bucket, so that the outer-product bucket is not merged
    # into its consumer
    plan = qbe.Plan(qm, pi, mu, ctx=ctx, exec="per_step", precision=prec, merge=False)
    assert plan.stats()["n_mfma_steps"] >= 1
    print(f"case outer product seed={seed} m={m} {prec}", flush=True)
    got, per = qbe.qbe_contract_slices(ctx, plan, 0, plan.n_slices, plan.workspace())
    want = C.brute_force_sum(n, tensors)
    _, vals = C.contract(tensors, C.bucket_schedule(n, [v for v, _ in tensors], pi, mu))
    tol = 4 * SPLIT_EPS if prec == "bf16x3" else 1e-5
    assert abs(got - want) <= tol * abs(want)
    rms = float(np.sqrt(np.mean(np.abs(vals) ** 2)))
    assert np.all(np.abs(per - np.asarray(vals)) <= tol * np.maximum(np.abs(vals), rms))


def test_precision_forms_on_7x7_d24_slices(env):
    """FP32 and both split-BF16 forms on slices 0..15 of the 7x7 depth-24
    workload against the complex128 oracle; the errors are printed per
    result."""
    qbe, ctx = env
    from circuitgen import circuit_model, random_grid_circuit
    gold = json.load(open(os.path.join(GOLD, "amplitudes.json")))["grid7x7_d24_m10"]
    want = np.array([complex(*v) for v in gold["slices"][:16]])
    rms = float(np.sqrt(np.mean(np.abs(want) ** 2)))
    qm = qbe.Model.from_circuitgen(circuit_model(random_grid_circuit(7, 7, 24, gold["seed"])))
    _, mu, pi, _ = qbe.plan_circuit(qm, m=10)
    errs = {}
    for prec in ("fp32", "bf16x3", "bf16x6"):
        # one launch per bucket: all seven outer-product buckets on MFMA
        plan = qbe.Plan(qm, pi, mu, ctx=ctx, exec="per_step", precision=prec, merge=False)
        n_mm = plan.stats()["n_mfma_steps"]
        assert n_mm >= 1
        print(f"case 7x7 slices 0-15 {prec}", flush=True)
        part, per = qbe.qbe_contract_slices(ctx, plan, 0, 16, plan.workspace(all_slices=False))
        e = np.abs(per - want) / np.maximum(np.abs(want), rms)
        errs[prec] = (float(np.max(e)), abs(part - want.sum()) / abs(want.sum()))
        print(f"  {prec}: {n_mm} MFMA buckets, max per-slice rel err {errs[prec][0]:.3e}, "
              f"16-slice sum rel err {errs[prec][1]:.3e}", flush=True)
    assert errs["fp32"][0] <= 1e-5
    assert errs["bf16x3"][0] <= 7 * 4 * SPLIT_EPS
    assert errs["bf16x6"][0] <= 1e-5


def test_merged_mfma_precision_forms_on_7x7_d24_slices(env):
    """With merged chains the two-group products run on MFMA in every
    precision (K = 2^(j+1) per tile); slices 0..15 of the 7x7 depth-24
    workload against the complex128 oracle, bounds as above."""
    qbe, ctx = env
    from circuitgen import circuit_model, random_grid_circuit
    gold = json.load(open(os.path.join(GOLD, "amplitudes.json")))["grid7x7_d24_m10"]
    want = np.array([complex(*v) for v in gold["slices"][:16]])
    rms = float(np.sqrt(np.mean(np.abs(want) ** 2)))
    qm = qbe.Model.from_circuitgen(circuit_model(random_grid_circuit(7, 7, 24, gold["seed"])))
    _, mu, pi, _ = qbe.plan_circuit(qm, m=10)
    errs = {}
    for prec in ("fp32", "bf16x3", "bf16x6"):
        plan = qbe.Plan(qm, pi, mu, ctx=ctx, exec="per_step", precision=prec)
        st = plan.stats()
        assert st["n_merged_steps"] >= 1 and st["n_mfma_steps"] >= 6
        print(f"case merged 7x7 slices 0-15 {prec}", flush=True)
        _, per = qbe.qbe_contract_slices(ctx, plan, 0, 16, plan.workspace(all_slices=False))
        errs[prec] = float(np.max(np.abs(per - want) / np.maximum(np.abs(want), rms)))
        print(f"  {prec}: {st['n_mfma_steps']} MFMA launches, max per-slice rel err {errs[prec]:.3e}", flush=True)
    assert errs["fp32"] <= 1e-5
    assert errs["bf16x3"] <= 7 * 4 * SPLIT_EPS
    assert errs["bf16x6"] <= 1e-5

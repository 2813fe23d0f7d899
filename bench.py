"""Benchmark: amplitudes per second of sliced bucket-elimination contraction
on one MI355X.

Headline workload: a 7x7 grid circuit of depth 24 (49 qubits, seed 0,
bitstring from the seed), 10 variables sliced (1024 slices), one amplitude
per step with the plan cached -- the largest of the benchmark configurations
and the one whose bucket contractions stream through HBM.  Timed forms:

* chosen: the sliced set picked by the learned proposal or by tree-trimming
  (whichever has fewer exact FLOPs; the heuristic is the fallback), merged
  bucket chains, grouped small launches, autotuned tiles, all 1024 slices at
  once, products in FP32 or split-BF16 -- the fastest form whose amplitude is
  within 1e-5 of the complex128 oracle, issued directly or replayed from a
  HIP graph;
* plain FP32: tree-trimming's sliced set, one launch per bucket, FP32.

The line carries MFMA utilisation and memory traffic from hardware counters
(valid only for the sources and plan they were taken on), a live per-launch
timing of the chosen plan with the roofline of its dominant kernel, and the
CPU oracle timed on a bounded sample of the same amplitude's slices.  Extra
lines: the 5x5 depth-16 circuit (64 slices, LDS-resident fused kernel), a
batch of 512 uneven instances, 256 bitstrings of one circuit, the stand-alone
permute, and the learned proposal's evaluation on 8x8 depth-32 circuits.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-extra] [--no-cpu]
Prints one JSON line.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "amplitudes/sec + MFMA util, chosen vs plain FP32 form at rel err ≤1e-5"
HBM_PEAK_GBS = 8000.0
FP32_PEAK_TFLOPS = 157.3
SEEDS = {"grid4x4_d10_m0": 0, "grid5x5_d16_m6": 1, "grid7x7_d24_m10": 0}
# Memory traffic of one 5x5 depth-16 fused_kernel launch from the FETCH_SIZE
# and WRITE_SIZE counter runs in profiles/fused_kernel_grid5x5_d16_m6.md
# (621.44 KiB x 2.000 + 6.06 KiB x 1.000, the factors from a 256 MiB device copy),
# valid while the fused kernel's sources have the digest they were measured on.
FUSED_TRAFFIC = {"bytes": int(round((621.4375 * 2.000 + 6.0625 * 1.000) * 1024)),
                 "sources_sha256": "93236d854b90c0a5a94f0e7924ad3222847e38a09f3d72bc964ef4ee06cfbc90"}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


FUSED_SOURCES = ("fused.hip", "fused_format.hpp", "device_common.hpp")


def source_digest(names):
    """SHA-256 over the given sources under the package's csrc/."""
    import hashlib
    h = hashlib.sha256()
    for name in names:
        with open(os.path.join(ROOT, "paper_2004_10892_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def fused_source_digest():
    """SHA-256 over the sources the fused kernel is compiled from."""
    return source_digest(FUSED_SOURCES)


# permute_kernel on the 2^28-entry tensor: FETCH_SIZE and WRITE_SIZE per
# dispatch (KiB, median of five) scaled by the device copy's calibration
PERMUTE_SOURCES = ("permute.hip", "device_common.hpp")
PERMUTE_TRAFFIC = {"bytes": int(round((1048617.125 * 2.000 + 2097234.0 * 1.000) * 1024)),
                   "sources_sha256": "bc3e876746629b38794d4c483059e78eaf0fba2d97ef9a1f5deedcc9600cd450"}


def fused_traffic():
    """Counter-measured bytes per fused_kernel launch, or None once the fused
    kernel's sources differ from those the counters were taken on."""
    return FUSED_TRAFFIC["bytes"] if fused_source_digest() == FUSED_TRAFFIC["sources_sha256"] else None


def golden(name):
    with open(os.path.join(ROOT, "tests", "golden", "amplitudes.json")) as f:
        g = json.load(f)[name]
    return complex(*g["oracle"])


def build_plan(qbe, ctx, name, form, precision="fp32", merge=True):
    from circuitgen import WORKLOADS, circuit_model, random_grid_circuit
    r, c, d, m = WORKLOADS[name]
    mod = circuit_model(random_grid_circuit(r, c, d, SEEDS[name]))
    qm = qbe.Model.from_circuitgen(mod)
    t0 = time.perf_counter()
    order, mu, pi, tau = qbe.plan_circuit(qm, m=m)   # min-fill order + tree-trimming (Alg. 2)
    qbe.Plan(qm, pi, mu, exec=form, precision=precision, merge=merge).close()  # schedule + programs, host only
    t1 = time.perf_counter()
    plan = qbe.Plan(qm, pi, mu, ctx=ctx, exec=form, precision=precision, merge=merge)  # plus upload and prep
    t2 = time.perf_counter()
    return plan, (t1 - t0) * 1e3, {"rows": r, "cols": c, "depth": d, "m": m, "seed": SEEDS[name],
                                  "width": tau, "n_vars": mod.n_vars, "n_tensors": len(mod.tensors),
                                  "device_setup_ms": (t2 - t1) * 1e3}


def timed(torch, fn, steps, warmup):
    """Runs fn warmup + steps times; returns (wall ms per step, event ms per step)."""
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record()
    for _ in range(steps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    return (t1 - t0) * 1e3 / steps, e0.elapsed_time(e1) / steps


def graph_of(torch, qbe, ctx, fn):
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


_CPU_STATE = {}


def _cpu_setup(name):
    """Worker set-up (and mode (i)): the oracle's model and schedule of a
    workload, planned by the oracle's own min-fill and Alg. 2."""
    from circuitgen import WORKLOADS, circuit_model, random_grid_circuit
    from oracle import contract as C
    from oracle import planner as P
    r, c, d, m = WORKLOADS[name]
    mod = circuit_model(random_grid_circuit(r, c, d, SEEDS[name]))
    tv = [v for v, _ in mod.tensors]
    adj = P.simple_graph(mod.n_vars, tv)
    order = P.min_fill_order(adj)
    mu, _, pi, _ = P.greedy_treewidth_deletion(adj, order, m)
    _CPU_STATE["tensors"] = mod.tensors
    _CPU_STATE["sched"] = C.bucket_schedule(mod.n_vars, tv, pi, mu)
    return m


def _cpu_slice(s):
    from oracle import contract as C
    return C.contract_slice(_CPU_STATE["tensors"], _CPU_STATE["sched"], s)


def cpu_baseline(name, budget_s=12.0, max_workers=16):
    """The oracle as it stands, on the host, in the two modes of the CPU
    plan: (i) one process contracting whole amplitudes; (ii) the slices of
    each amplitude split across worker processes (spawned children that
    never touch the GPU).  Reports the better mode, with the cores it used."""
    from oracle import contract as C
    m = _cpu_setup(name)
    n = 0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < budget_s:
        C.contract(_CPU_STATE["tensors"], _CPU_STATE["sched"])
        n += 1
    single = n / (time.perf_counter() - t0)
    try:
        affinity = len(os.sched_getaffinity(0))
    except AttributeError:
        affinity = os.cpu_count() or 1
    workers = max(1, min(max_workers, affinity))
    modes = {"one_process": {"value": single, "cores": 1, "amplitudes": n}}
    if workers > 1:
        import multiprocessing as mp
        with mp.get_context("spawn").Pool(workers, initializer=_cpu_setup, initargs=(name,)) as pool:
            pool.map(_cpu_slice, range(1 << m))  # warm every worker
            k = 0
            t0 = time.perf_counter()
            while time.perf_counter() - t0 < budget_s:
                C.exact_sum(pool.map(_cpu_slice, range(1 << m), chunksize=max(1, (1 << m) // workers)))
                k += 1
            modes["slices_across_processes"] = {"value": k / (time.perf_counter() - t0), "cores": workers,
                                                "amplitudes": k}
    best = max(modes, key=lambda q: modes[q]["value"])
    return {"value": modes[best]["value"], "unit": "amplitudes/s", "cores": modes[best]["cores"],
            "kind": "oracle", "mode": best, "modes": modes,
            "sample": f"whole amplitudes of {name} (all {1 << m} slices each) for about {budget_s:.0f} s per "
                      f"mode, numpy complex128 einsum; host: {cpu_model()}, {os.cpu_count()} logical CPUs, "
                      f"{affinity} usable by this process"}


_COPY_GBS = []


def copy_peak_gbs(torch):
    """Measured HBM peak: a 2 GiB device-to-device copy (read + write bytes
    per second), timed once per process."""
    if not _COPY_GBS:
        src = torch.empty(1 << 28, dtype=torch.float64, device="cuda")
        src.fill_(1.0)
        dst = torch.empty_like(src)
        _, ev = timed(torch, lambda: dst.copy_(src), 10, 2)
        _COPY_GBS.append(2 * src.numel() * 8 / (ev * 1e-3) / 1e9)
        del src, dst
    return _COPY_GBS[0]


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"



# ------------------------------------------------------------ headline (C3) --

C3 = "grid7x7_d24_m10"
# Sources that decide the per-step form's kernels and launches: counters
# taken on other sources describe other code and are not reported.
STEP_SOURCES = ("device.hip", "device_common.hpp", "qbe_internal.hpp", "program.cpp", "planner.cpp", "fused.hip",
                "fused_format.hpp", "api.cpp")
# Hardware counters of one contraction of the headline plan
# (profiles/fused_and_step_kernels_grid7x7_d24_m10.md): per precision, summed over the
# contraction's dispatches.  mfma_busy: SQ_VALU_MFMA_BUSY_CYCLES; capacity:
# GRBM_GUI_ACTIVE / 8 XCDs x 256 CUs x 4 SIMDs; fetch/write: FETCH_SIZE x
# 2.000 and WRITE_SIZE x 1.000 bytes (the 256 MiB device-copy calibration);
# dominant: the same for the dominant kernel's launch.  Keyed by the
# sources' digest and the plan's sliced set.
C3_COUNTERS = {
    "sources_sha256": "63b1d349e053d6e9c26ee8c457492ad0801ed582060a62bd57813c3a7660407b",
    "plan": "min_fill+tt_rec2_t16_s5+segments+sums2",
    "mu": [
        119,
        353,
        183,
        220,
        335,
        66,
        486,
        359,
        490,
        169
    ],
    "fp32": {
        "mfma_util": 0.0,
        "mfma_busy_cycles": 0.0,
        "gui_active": 6689689.0,
        "amplitude": {
            "bytes": 472980128,
            "fetch_kib": 118763.3125,
            "write_kib": 224368.03125
        },
        "dominant": {
            "launch": 0,
            "kernel": "qbe::fused_kernel",
            "bytes": 39785984,
            "fetch_kib": 5570.75,
            "write_kib": 27712.0
        }
    },
    "bf16x6": {
        "mfma_util": 0.0011520879907202912,
        "mfma_busy_cycles": 1048576.0,
        "gui_active": 7110568.0
    },
    "plain_fp32": {
        "mfma_util": 0.0
    }
}


def step_source_digest():
    return source_digest(STEP_SOURCES)


def c3_counters(precision, mu, plan=None):
    """The committed counters of the headline plan, or (None, reason)."""
    if C3_COUNTERS.get("sources_sha256") != step_source_digest():
        return None, "per-step sources differ from those the counters were taken on"
    if C3_COUNTERS.get("mu") != list(mu) or (plan is not None and C3_COUNTERS.get("plan") != plan):
        return None, "the plan differs from the one the counters were taken on"
    rec = C3_COUNTERS.get(precision)
    if not rec:
        return None, f"no counters taken for {precision}"
    return rec, None


def c3_model(qbe):
    from circuitgen import circuit_model, random_grid_circuit
    r, c, d, m = 7, 7, 24, 10
    return qbe.Model.from_circuitgen(circuit_model(random_grid_circuit(r, c, d, SEEDS[C3]))), m


def train_net(qbe, ctx, labels=20000, epochs=20, elim_states=2):
    """The learned proposal's network trained on the device: ~20k exact-cost
    labels from seeded 6x6..8x8 circuits of depth 16..32, for both heads
    (slicing states along tree-trimming's trajectory, elimination states of
    the min-fill order)."""
    from circuitgen import SplitMix64, circuit_model, random_grid_circuit
    from paper_2004_10892_amd import learned as L
    rng = SplitMix64(2020)
    t0 = time.perf_counter()
    samples, n_labels, i = [], 0, 0
    while n_labels < labels and i < 400:
        r, c, d = 6 + rng.next() % 3, 6 + rng.next() % 3, 16 + rng.next() % 17
        qm = qbe.Model.from_circuitgen(circuit_model(random_grid_circuit(r, c, d, 2000 + i)))
        ss, n = L.make_dataset([qm], seed=i, elim_states=elim_states)
        samples += ss
        n_labels += n
        i += 1
    t1 = time.perf_counter()
    net = qbe.Gnn(ctx, seed=7)
    hist = L.train(net, samples, epochs=epochs, batch=8, lr=2e-3)
    t2 = time.perf_counter()
    return net, {"labels": n_labels, "train_circuits": i, "label_s": t1 - t0, "train_s": t2 - t1,
                 "samples": {h: sum(x.head == h for x in samples) for h in ("slicing", "elimination")},
                 "loss_first_epoch": hist[0], "loss_last_epoch": hist[-1]}


def plan_candidates(qbe, qm, m, net):
    """Candidate plans of one circuit: elimination orders (greedy min-fill;
    the anytime heuristic standing in for the paper's tree-decomposition
    solver; with a network, min-fill with learned tie-breaking) times sliced
    sets of m variables (tree-trimming; tree-trimming with Alg. 2's order
    recomputation after every k-th removal, k = 1..3, with 4 tries of the
    anytime heuristic and seeds 1-2 or 16 tries and seeds 1-8; with a
    network, the learned score with and without it).  Returns {name: (mu,
    reduced_order, planning_ms)}, duplicates dropped."""
    orders = {}
    t0 = time.perf_counter()
    orders["min_fill"] = (qbe.qbe_order_min_fill(qm), (time.perf_counter() - t0) * 1e3)
    t0 = time.perf_counter()
    orders["anytime8"] = (qbe.qbe_order_anytime(qm, [], 8, 1)[0], (time.perf_counter() - t0) * 1e3)
    if net is not None:
        t0 = time.perf_counter()
        orders["learned_order"] = (qbe.qbe_order_learned(qm, net, 16)[0], (time.perf_counter() - t0) * 1e3)
    slicings = {"tt": dict()}
    for k in (1, 2, 3):
        for tries, seeds in ((4, (1, 2)), (16, range(1, 9))):
            for seed in seeds:
                slicings[f"tt_rec{k}_t{tries}_s{seed}"] = dict(recompute_every=k, tries=tries, seed=seed)
    if net is not None:
        slicings["learned"] = dict(score="learned", net=net)
        for k in (1, 2):
            slicings[f"learned_rec{k}_t16_s2"] = dict(score="learned", net=net, recompute_every=k, tries=16, seed=2)
    cands, seen = {}, set()
    for on, (order, oms) in orders.items():
        for sn, kw in slicings.items():
            t0 = time.perf_counter()
            mu, pi, _ = qbe.qbe_slice(qm, order, m, **kw)
            ms = oms + (time.perf_counter() - t0) * 1e3
            key = (tuple(mu), tuple(pi))
            if key not in seen:
                seen.add(key)
                cands[f"{on}+{sn}"] = (mu, pi, ms)
    return cands


def time_plan(torch, qbe, ctx, plan, steps, warmup):
    """One amplitude per step, issued directly and replayed from a HIP
    graph (both must give the same bits)."""
    ws = plan.workspace()
    out = torch.zeros(2, dtype=torch.float64, device="cuda")
    fn = lambda: qbe.qbe_contract_async(ctx, plan, ws, out)  # noqa: E731
    wall_d, ev_d = timed(torch, fn, steps, warmup)
    got = complex(*out.cpu().numpy())
    g = graph_of(torch, qbe, ctx, fn)
    out.fill_(float("nan"))
    wall_g, ev_g = timed(torch, g.replay, steps, warmup)
    got_g = complex(*out.cpu().numpy())
    if got_g != got:
        raise SystemExit(f"graph replay {got_g} differs from direct launch {got}")
    forms = {"direct": {"ms_per_amplitude": ev_d, "wall_ms_per_amplitude": wall_d},
             "graph": {"ms_per_amplitude": ev_g, "wall_ms_per_amplitude": wall_g}}
    return forms, got, ws


def launch_profile(plan, ws, reps):
    """Per-launch HIP-event timing of whole contractions (qbe_plan_profile),
    averaged over reps; with each launch's algorithmic bytes and FLOPs."""
    import numpy as np
    info = plan.launches()
    ms = np.mean([plan.profile(ws) for _ in range(reps)], axis=0)
    n = plan.n_slices
    rows = []
    for i, (li, t) in enumerate(zip(info, ms)):
        rows.append(dict(li, index=i, ms=float(t), bytes=li["bytes_per_slice"] * n, flops=li["flops_per_slice"] * n))
    return rows


FUSED_FORMS = {"": (False, False), "+prefix": (True, False), "+segments": (True, True)}


def split_plan_name(name):
    """A timed plan's name: a candidate's, with "+prefix" appended when the
    plan runs its first small buckets in a fused prefix, "+segments" when
    later runs of small buckets are fused launches too, then "+sums<N>" when
    its merged per-step launches sum at most N variables.  Returns
    (candidate, fused_prefix, fused_segments, max_sums)."""
    sums = 0
    head, _, tail = name.rpartition("+sums")
    if head and tail.isdigit():
        name, sums = head, int(tail)
    for suffix, (pre, seg) in FUSED_FORMS.items():
        if suffix and name.endswith(suffix):
            return name[:-len(suffix)], pre, seg, sums
    return name, False, False, sums


def time_precisions(torch, qbe, ctx, qm, mu, pi, precisions, steps, warmup, want, keep=True, prefix=False,
                    segments=False, max_sums=0):
    """The plan (mu, pi) in each precision: autotuned, then timed issued
    directly and from a HIP graph; error against the oracle amplitude."""
    forms = {}
    for prec in precisions:
        plan = qbe.Plan(qm, pi, mu, ctx=ctx, exec="per_step", precision=prec, fused_prefix=prefix,
                        fused_segments=segments, max_sums=max_sums)
        ws0 = plan.workspace()
        t0 = time.perf_counter()
        plan.autotune(ws0)
        tune_ms = (time.perf_counter() - t0) * 1e3
        del ws0
        fr, got, ws = time_plan(torch, qbe, ctx, plan, steps, warmup)
        ev = min(f["ms_per_amplitude"] for f in fr.values())
        err = abs(got - want) / abs(want)
        forms[prec] = {"ms_per_amplitude": ev, "amplitudes_per_s": 1e3 / ev, "rel_err": err, "issue": fr,
                       "autotune_ms": tune_ms, "within_1e-5": err <= 1e-5}
        if keep:
            forms[prec].update(_plan=plan, _ws=ws)
        log(f"[bench] {prec}: {ev:.3f} ms/amplitude, rel err {err:.2e}")
    return forms


def bench_headline(torch, qbe, ctx, steps, warmup, net, n_timed=12, n_forms=3):
    from paper_2004_10892_amd import learned as L
    qm, m = c3_model(qbe)
    want = golden(C3)
    t_search = time.perf_counter()
    cands = plan_candidates(qbe, qm, m, net)
    # every candidate's schedule on the host; the most promising by a rough
    # estimate (bytes at 2.5 TB/s plus 6 us a launch) are built on the
    # device with fused segments, autotuned and timed in FP32, the fastest
    # few also without segments and without the prefix, and the fastest of
    # all is kept: the cost model's FLOPs do not rank plans for this
    # executor
    plans_info = {}
    for k, (mu_k, pi_k, ms_k) in cands.items():
        st_k = qbe.Plan(qm, pi_k, mu_k, exec="per_step").stats()
        c = qbe.qbe_schedule_cost(qm, pi_k, mu_k)
        plans_info[k] = {"width": c["width"], "log2_total_flops": L.total_log2_flops(c),
                         "step_MB_per_slice": st_k["step_bytes_per_slice"] / 1e6, "launches": st_k["n_launches"],
                         "peak_bytes_per_slice": c["peak_bytes_per_slice"], "planning_ms": ms_k,
                         "estimate_ms": st_k["step_bytes_per_slice"] * (1 << m) / 2.5e9 + 0.006 * st_k["n_launches"]}
    ranked = sorted(plans_info, key=lambda k: plans_info[k]["estimate_ms"])
    to_time = ranked[:n_timed]
    for extra in ("min_fill+tt", next((k for k in ranked if "learned" in k), None),
                  next((k for k in ranked if k.startswith("anytime8")), None)):
        if extra and extra not in to_time:
            to_time.append(extra)
    # each with fused segments (first small buckets in one LDS-resident
    # launch, later runs of small buckets too); the fastest n_forms also in
    # the plain per-step form and with the fused prefix only
    timed_ms = {}

    def time_forms(k, forms, max_sums=0):
        """Times plan k in the given fused forms (merged launches of at most
        max_sums summed variables when > 0); the forms that exist."""
        mu_k, pi_k, _ = cands[k]
        done = []
        for suffix in forms:
            pre, seg = FUSED_FORMS[suffix]
            plan_k = qbe.Plan(qm, pi_k, mu_k, ctx=ctx, exec="per_step", fused_prefix=pre, fused_segments=seg,
                              max_sums=max_sums)
            st_k = plan_k.stats()
            if (pre and st_k["prefix_buckets"] == 0) or (seg and st_k["n_fused_segments"] < 2):
                continue
            ws_k = plan_k.workspace()
            plan_k.autotune(ws_k)
            out_k = torch.zeros(2, dtype=torch.float64, device="cuda")
            _, ev_k = timed(torch, lambda: qbe.qbe_contract_async(ctx, plan_k, ws_k, out_k), max(3, steps // 2), 1)
            err_k = abs(complex(*out_k.cpu().numpy()) - want) / abs(want)
            name = suffix + (f"+sums{max_sums}" if max_sums else "")
            tag = name.replace("+", "_").strip("_") + "_" if name else ""
            plans_info[k][f"fp32_{tag}ms_per_amplitude"] = ev_k
            plans_info[k][f"rel_err_fp32_{tag}".rstrip("_")] = err_k
            plans_info[k][f"{tag}launches"] = st_k["n_launches"]
            if err_k <= 1e-5:
                timed_ms[k + name] = ev_k
            done.append(suffix)
            del ws_k, plan_k
        return done

    others = [f for f in FUSED_FORMS if f != "+segments"]
    for k in to_time:
        if not time_forms(k, ["+segments"]):
            time_forms(k, others)  # no segments in this plan: its other forms
    best = sorted((b for b in to_time if b + "+segments" in timed_ms), key=lambda b: timed_ms[b + "+segments"])
    for k in best[:n_forms]:
        time_forms(k, others)
        # merged launches of fewer summed variables: more launches and
        # round trips, fewer terms an entry -- which wins depends on the plan
        for cap in (2, 3):
            time_forms(k, ["+segments"], max_sums=cap)
    src = min(timed_ms, key=timed_ms.get)
    base, use_prefix, use_segments, use_sums = split_plan_name(src)
    mu, pi, _ = cands[base]
    search_s = time.perf_counter() - t_search
    log(f"[bench] {C3}: plan {src}; " + ", ".join(f"{k} {v:.3f} ms" for k, v in sorted(timed_ms.items())))
    forms = time_precisions(torch, qbe, ctx, qm, mu, pi, ("fp32", "bf16x6", "bf16x3"), steps, warmup, want,
                            prefix=use_prefix, segments=use_segments, max_sums=use_sums)
    ok = [p for p in forms if forms[p]["within_1e-5"]]
    if not ok:
        raise SystemExit("no form of the headline workload met the 1e-5 bound")
    chosen = min(ok, key=lambda p: forms[p]["ms_per_amplitude"])
    plan, ws = forms[chosen]["_plan"], forms[chosen]["_ws"]
    st = plan.stats()
    prof = launch_profile(plan, ws, max(3, steps // 4))
    # plain FP32 form: tree-trimming's sliced set, one launch per bucket,
    # every input tensor a factor of its own
    mu_t, pi_t, _ = cands["min_fill+tt"]
    plan_p = qbe.Plan(qm, pi_t, mu_t, ctx=ctx, exec="per_step", merge=False, fold_inputs=False)
    ws_p = plan_p.workspace()
    out_p = torch.zeros(2, dtype=torch.float64, device="cuda")
    wall_p, ev_p = timed(torch, lambda: qbe.qbe_contract_async(ctx, plan_p, ws_p, out_p), max(2, steps // 4), 1)
    err_p = abs(complex(*out_p.cpu().numpy()) - want) / abs(want)
    log(f"[bench] plain FP32 (one launch per bucket): {ev_p:.3f} ms/amplitude, rel err {err_p:.2e}")
    plain = {"form": "per_step, one launch per bucket; min-fill order, tree-trimming sliced set", "precision": "fp32",
             "ms_per_amplitude": ev_p, "amplitudes_per_s": 1e3 / ev_p, "rel_err": err_p,
             "launches_per_amplitude": plan_p.stats()["n_launches"] + 2}
    del ws_p, plan_p
    # the same for the chosen plan's schedule: what the executor alone gains
    plan_q = qbe.Plan(qm, pi, mu, ctx=ctx, exec="per_step", merge=False, fold_inputs=False)
    ws_q = plan_q.workspace()
    out_q = torch.zeros(2, dtype=torch.float64, device="cuda")
    _, ev_q = timed(torch, lambda: qbe.qbe_contract_async(ctx, plan_q, ws_q, out_q), max(2, steps // 4), 1)
    plain["same_plan"] = {"plan": base, "ms_per_amplitude": ev_q, "amplitudes_per_s": 1e3 / ev_q,
                          "rel_err": abs(complex(*out_q.cpu().numpy()) - want) / abs(want),
                          "launches_per_amplitude": plan_q.stats()["n_launches"] + 2}
    del ws_q, plan_q
    # the combined form with the learned proposal in the plan: the fastest
    # timed candidate that uses the network, in split-BF16 and FP32
    combined = None
    lk = [k for k in timed_ms if "learned" in k]
    if lk:
        kb = min(lk, key=timed_ms.get)
        kb_base, kb_prefix, kb_segments, kb_sums = split_plan_name(kb)
        mu_c, pi_c, _ = cands[kb_base]
        fc = forms if kb == src else time_precisions(torch, qbe, ctx, qm, mu_c, pi_c, ("bf16x3", "bf16x6", "fp32"),
                                                     max(3, steps // 2), 1, want, keep=False, prefix=kb_prefix,
                                                     segments=kb_segments, max_sums=kb_sums)
        combined = {"plan": kb, "forms": {p: {k: v for k, v in f.items() if not k.startswith("_")}
                                          for p, f in fc.items()},
                    "speedup_vs_plain": {p: ev_p / f["ms_per_amplitude"] for p, f in fc.items()},
                    "note": "learned proposal in the plan (order and/or sliced set), split-BF16 or FP32 products on "
                            "MFMA, all 1024 slices batched per launch; speedup over the plain FP32 form"}
    # roofline: the dominant kernel's launch (longest in the live per-launch
    # timing) and the whole amplitude
    dom = max(prof, key=lambda r: r["ms"])
    gbs = dom["bytes"] / (dom["ms"] * 1e-3) / 1e9
    total_ms = sum(r["ms"] for r in prof)
    amp_bytes = st["step_bytes_per_slice"] * plan.n_slices
    launch_flops = sum(r["flops"] for r in prof)
    cnt, why = c3_counters(chosen, mu, src)
    dom_cnt = cnt.get("dominant") if cnt else None
    if dom_cnt and dom_cnt["launch"] != dom["index"]:
        dom_cnt, why = None, f"the counters' dominant launch ({dom_cnt['launch']}) is not this run's"
    roof = {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS,
            "traffic": dom_cnt["bytes"] if dom_cnt else None,
            "traffic_kernel": dom_cnt["kernel"] if dom_cnt else None,
            "kernel": (f"launch {dom['index']}: fused {dom['kind']} (fused_kernel), {dom['n_buckets']} buckets "
                       f"of at most {dom['out_rank'] + 1} variables, {dom['levels']} levels, {dom['lds_bytes']} B LDS "
                       f"a workgroup, {dom['n_ops']} imported results"
                       if dom["kind"] in ("prefix", "segment") else
                       f"launch {dom['index']}: {dom['kind']}, {dom['n_ops']} operands, result rank "
                       f"{dom['out_rank']}, {dom['n_sum']} summed, {'MFMA' if dom['mfma'] else 'VALU'}"),
            "launch_ms": dom["ms"], "algorithmic_bytes_per_launch": dom["bytes"],
            "bytes_per_slice": dom["bytes_per_slice"], "slices_per_launch": plan.n_slices,
            "launch_share_of_amplitude": dom["ms"] / total_ms,
            "copy_peak": copy_peak_gbs(torch), "frac_vs_copy": gbs / copy_peak_gbs(torch),
            # the same launch against the vector ALU: its algorithmic flops
            # (the cost model's: 6 per complex product of factors, 2 per
            # complex addition of the sum) per second, against the FP32
            # vector peak (157.3 TFLOP/s counts packed FP32 pairs; these
            # kernels issue one FP32 operation a lane, whose peak is half
            # that)
            "alu_view": {"achieved_tflops": dom["flops"] / (dom["ms"] * 1e-3) / 1e12, "peak": FP32_PEAK_TFLOPS,
                         "frac": dom["flops"] / (dom["ms"] * 1e-3) / 1e12 / FP32_PEAK_TFLOPS,
                         "frac_of_unpacked_peak": dom["flops"] / (dom["ms"] * 1e-3) / 1e12 / (FP32_PEAK_TFLOPS / 2),
                         "flops_per_launch": dom["flops"]},
            "amplitude": {"algorithmic_bytes": amp_bytes, "cost_model_bytes": st["bytes_per_slice"] * plan.n_slices,
                          "ms": forms[chosen]["ms_per_amplitude"],
                          "achieved_GB_per_s": amp_bytes / (forms[chosen]["ms_per_amplitude"] * 1e-3) / 1e9,
                          "frac": amp_bytes / (forms[chosen]["ms_per_amplitude"] * 1e-3) / 1e9 / HBM_PEAK_GBS,
                          "traffic": cnt["amplitude"]["bytes"] if cnt and "amplitude" in cnt else None,
                          "launch_flops": launch_flops, "cost_model_flops": st["flops_per_slice"] * plan.n_slices},
            "note": "achieved = the dominant launch's algorithmic bytes (each operand read once, its result "
                    "written once, per slice x slices) / its average duration from HIP events around each launch "
                    "of whole contractions (qbe_plan_profile); amplitude: the same count over all launches "
                    "(merged chains keep their intermediates on chip) / the step time; cost_model_bytes: one "
                    "launch per bucket; traffic: FETCH_SIZE and WRITE_SIZE counters with the copy calibration"
                    + ("" if dom_cnt else f" (null: {why})")}
    mfma = {"value": cnt["mfma_util"] if cnt else None,
            "plain_fp32": C3_COUNTERS.get("plain_fp32", {}).get("mfma_util") if cnt else None,
            "ceiling": "bucket contractions of complex64 operands carry 1.6-4 flop/B (cost model); at 8 TB/s "
                       "that is at most ~30 TFLOP/s, 19% of the FP32 MFMA peak even if every flop ran on MFMA",
            "source": "SQ_VALU_MFMA_BUSY_CYCLES / (GRBM_GUI_ACTIVE / 8 x 256 CUs x 4 SIMDs) over all dispatches of "
                      "one contraction" + ("" if cnt else f" (null: {why})")}
    top = sorted(prof, key=lambda r: -r["ms"])[:8]
    result = {
        "chosen": chosen, "ev": forms[chosen]["ms_per_amplitude"], "rel_err": forms[chosen]["rel_err"],
        "forms": {p: {k: v for k, v in f.items() if not k.startswith("_")} for p, f in forms.items()},
        "plain": plain, "combined": combined, "roofline": roof, "mfma": mfma, "mu_source": src, "mu": mu,
        "plans": plans_info,
        "planning_ms": plans_info[base]["planning_ms"], "plan_search_s": search_s,
        "config": {"workload": C3, "rows": 7, "cols": 7, "depth": 24, "m": m, "seed": SEEDS[C3],
                   "slices": plan.n_slices, "width": st["width"], "n_vars": st["n_vars"], "n_tensors": st["n_tensors"],
                   "buckets": st["n_steps"], "launches": st["n_launches"], "merged_launches": st["n_merged_steps"],
                   "mfma_launches": st["n_mfma_steps"], "mu_source": src},
        "launches_top": [{k: r[k] for k in ("index", "kind", "n_ops", "out_rank", "n_sum", "mfma", "ms", "bytes")}
                         for r in top],
    }
    for f in forms.values():
        f.pop("_plan", None)
        f.pop("_ws", None)
    return result


def _cpu_slices_worker(s):
    return _cpu_slice(s)


def cpu_baseline_slices(name, budget_s=10.0, max_workers=16):
    """The oracle as it stands on the host, on a bounded sample of one
    amplitude's slices (slices 0, 1, 2, ... until the budget is spent),
    scaled to whole amplitudes: (i) one process; (ii) the slices spread over
    worker processes (spawned children that never touch the GPU)."""
    m = _cpu_setup(name)
    n_all = 1 << m
    k = 0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < budget_s and k < n_all:
        _cpu_slice(k)
        k += 1
    dt = time.perf_counter() - t0
    modes = {"one_process": {"value": k / dt / n_all, "cores": 1, "slices": k}}
    try:
        affinity = len(os.sched_getaffinity(0))
    except AttributeError:
        affinity = os.cpu_count() or 1
    workers = max(1, min(max_workers, affinity))
    if workers > 1:
        import multiprocessing as mp
        with mp.get_context("spawn").Pool(workers, initializer=_cpu_setup, initargs=(name,)) as pool:
            pool.map(_cpu_slices_worker, range(workers))  # warm every worker
            done = 0
            t0 = time.perf_counter()
            while time.perf_counter() - t0 < budget_s and done < n_all:
                chunk = list(range(done, min(n_all, done + 4 * workers)))
                pool.map(_cpu_slices_worker, chunk, chunksize=1)
                done += len(chunk)
            dt = time.perf_counter() - t0
            modes["slices_across_processes"] = {"value": done / dt / n_all, "cores": workers, "slices": done}
    best = max(modes, key=lambda q: modes[q]["value"])
    return {"value": modes[best]["value"], "unit": "amplitudes/s", "cores": modes[best]["cores"],
            "kind": "oracle", "mode": best, "modes": modes,
            "sample": f"slices 0..{modes[best]['slices'] - 1} of one {name} amplitude ({n_all} slices per "
                      f"amplitude; about {budget_s:.0f} s per mode), numpy complex128 einsum per bucket, scaled to "
                      f"whole amplitudes; host: {cpu_model()}, {os.cpu_count()} logical CPUs, {affinity} usable"}



def bench_batch(torch, qbe, ctx, steps):
    """512 uneven instances: one batched call vs one launch per bucket."""
    import numpy as np
    from circuitgen import batch_instances, circuit_model, random_grid_circuit
    t0 = time.perf_counter()
    plans_b, plans_p, scale = [], [], []
    for (r, c, d, m, seed) in batch_instances(512):
        scale.append(2.0 ** (-(r * c) / 2))  # typical |amplitude| of an n-qubit random circuit
        qm = qbe.Model.from_circuitgen(circuit_model(random_grid_circuit(r, c, d, seed)))
        _, mu, pi, _ = qbe.plan_circuit(qm, m=m)
        plans_b.append(qbe.Plan(qm, pi, mu, ctx=ctx))
        plans_p.append(qbe.Plan(qm, pi, mu, ctx=ctx, exec="per_step", merge=False, fold_inputs=False))
    plan_ms = (time.perf_counter() - t0) * 1e3
    batch = qbe.Batch(ctx, plans_b)
    ws = batch.workspace()
    amps = torch.zeros(2 * len(plans_b), dtype=torch.float64, device="cuda")
    # issued directly (host enqueues every launch and event of the call),
    # then replayed from a HIP graph of the same call
    wall_d, ev_d = timed(torch, lambda: batch.contract_async(ws, amps), steps, 2)
    res_d = amps.cpu().numpy().copy()
    g = graph_of(torch, qbe, ctx, lambda: batch.contract_async(ws, amps))
    wall_b, ev_b = timed(torch, g.replay, steps, 2)
    res_b = amps.cpu().numpy().copy()
    wsp = torch.empty(max(int(p.stats()["ws_bytes_all_slices"]) for p in plans_p), dtype=torch.uint8, device="cuda")
    outp = torch.zeros(2 * len(plans_p), dtype=torch.float64, device="cuda")

    def plain():
        for i, p in enumerate(plans_p):
            qbe.qbe_contract_async(ctx, p, wsp, outp[2 * i:])
    wall_p, ev_p = timed(torch, plain, max(1, steps // 4), 1)
    res_p = outp.cpu().numpy()
    a, b = res_b.view(np.complex128), res_p.view(np.complex128)
    n_fused = sum(p.stats()["exec"] == 2 for p in plans_b)
    return {"workload": "batch512_grid4-6_d10-20_m0-6", "instances": len(plans_b), "fused_instances": n_fused,
            "batched_ms": ev_b, "batched_amplitudes_per_s": len(plans_b) / (ev_b * 1e-3),
            "issue": {"graph": {"ms": ev_b, "wall_ms": wall_b}, "direct": {"ms": ev_d, "wall_ms": wall_d},
                      "same_bits": bool(np.array_equal(res_d, res_b))},
            "plain_ms": ev_p, "plain_amplitudes_per_s": len(plans_p) / (ev_p * 1e-3),
            "speedup": ev_p / ev_b, "planning_ms_total": plan_ms,
            "max_diff_batched_vs_plain": float(np.max(np.abs(a - b) / np.maximum(np.abs(b), np.asarray(scale)))),
            "note_diff": "|batched - plain| / max(|plain|, 2^(-n/2)): exact-zero amplitudes of shallow "
                         "circuits are compared on the scale of a typical amplitude"}


def bench_many(torch, qbe, ctx, steps, n_bits=256):
    """Many amplitudes of the headline circuit: one plan, cloned for each of
    n_bits seeded bitstrings (same schedule and programs, other output
    tensors), contracted in one batched fused launch."""
    import numpy as np
    from circuitgen import SplitMix64, WORKLOADS, circuit_model, random_grid_circuit
    name = "grid5x5_d16_m6"
    r, c, d, m = WORKLOADS[name]
    circ = random_grid_circuit(r, c, d, SEEDS[name])
    rng = SplitMix64(4242)
    xs = [circ.bitstring] + [rng.next() & ((1 << (r * c)) - 1) for _ in range(n_bits - 1)]
    t0 = time.perf_counter()
    qms = [qbe.Model.from_circuitgen(circuit_model(circ, x)) for x in xs]
    _, mu, pi, _ = qbe.plan_circuit(qms[0], m=m)
    base = qbe.Plan(qms[0], pi, mu, ctx=ctx, exec="fused")
    plans = [base] + [base.clone(q) for q in qms[1:]]
    setup_ms = (time.perf_counter() - t0) * 1e3
    batch = qbe.Batch(ctx, plans)
    ws = batch.workspace()
    amps = torch.zeros(2 * n_bits, dtype=torch.float64, device="cuda")
    fn = lambda: batch.contract_async(ws, amps)  # noqa: E731
    wall, ev = timed(torch, fn, steps, 2)
    got = amps.cpu().numpy().view(np.complex128).copy()
    # the same amplitudes one launch each, for the first few bitstrings
    single = []
    for p in plans[:8]:
        single.append(qbe.qbe_contract(ctx, p, p.workspace()))
    scale = 2.0 ** (-(r * c) / 2)
    diff = max(abs(g - s) / max(abs(s), scale) for g, s in zip(got[:8], single))
    want = golden(name)
    return {"workload": f"{name}_x{n_bits}_bitstrings", "bitstrings": n_bits, "slices_each": base.n_slices,
            "ms_per_batch": ev, "amplitudes_per_s": n_bits / (ev * 1e-3),
            "rel_err_first_vs_oracle": abs(got[0] - want) / abs(want),
            "max_diff_batched_vs_single": float(diff), "setup_ms": setup_ms,
            "note": "one plan (order, slicing, schedule, programs) cloned per bitstring; "
                    "all bitstrings x slices in one persistent fused launch"}


def bench_permute(torch, qbe, ctx, steps, r=28):
    """Stand-alone bit permutation of one 2^r-entry complex64 tensor (2 GiB
    at r = 28, the per-slice size cap of the planner's memory budget) by a
    seeded random permutation, against a device copy of the same bytes."""
    import numpy as np
    rng = np.random.default_rng(2828)
    perm = [int(p) for p in rng.permutation(r)]
    n = 1 << r
    # every entry a distinct bit pattern (compared as 64-bit integers)
    d_in = torch.arange(2 * n, dtype=torch.int32, device="cuda").view(torch.complex64)
    d_out = torch.empty_like(d_in)
    wall, ev = timed(torch, lambda: qbe.qbe_permute(ctx, d_in, d_out, r, perm, 1), steps, 2)
    # sampled check against the definition: output index o holds the input
    # entry whose bit perm[j] is o's bit j
    o = rng.integers(0, n, 4096, dtype=np.int64)
    i = np.zeros_like(o)
    for j in range(r):
        i |= ((o >> j) & 1) << perm[j]
    got = d_out.view(torch.int64)[torch.from_numpy(o).cuda()].cpu().numpy()
    want = d_in.view(torch.int64)[torch.from_numpy(i).cuda()].cpu().numpy()
    copy_wall, copy_ev = timed(torch, lambda: d_out.copy_(d_in), steps, 2)
    nbytes = 2 * n * 8
    gbs = nbytes / (ev * 1e-3) / 1e9
    return {"workload": f"permute_r{r}_complex64", "ms": ev, "GB_per_s": gbs, "copy_ms": copy_ev,
            "copy_GB_per_s": nbytes / (copy_ev * 1e-3) / 1e9, "sampled_exact": bool(np.array_equal(got, want)),
            "roofline": {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": gbs / HBM_PEAK_GBS,
                         "traffic": PERMUTE_TRAFFIC["bytes"] if r == 28 and source_digest(PERMUTE_SOURCES) ==
                         PERMUTE_TRAFFIC["sources_sha256"] else None,
                         "algorithmic_bytes": nbytes,
                         "copy_peak": copy_peak_gbs(torch), "frac_vs_copy": gbs / copy_peak_gbs(torch),
                         "note": "algorithmic bytes = read + write of the tensor once; traffic: FETCH_SIZE and "
                                 "WRITE_SIZE counters per dispatch with the copy calibration"}}


def bench_learned(qbe, net, train_info):
    """The learned proposal at the 8x8 / depth-32 scale: the trained network
    against tree-trimming on 10 held-out circuits under a 4 GiB per-slice
    memory cap, judged by exact total FLOPs (the heuristic is the fallback)."""
    import numpy as np
    from circuitgen import circuit_model, random_grid_circuit
    from paper_2004_10892_amd import learned as L
    t2 = time.perf_counter()
    rows, gains, best = [], [], []
    for k in range(10):
        qm = qbe.Model.from_circuitgen(circuit_model(random_grid_circuit(8, 8, 32, 5000 + k)))
        res = L.compare(qm, net, mem_cap=L.MEM_CAP)
        rows.append(res)
        gains.append(res["log2_gain"])
        best.append(res["log2_gain_best_of_both"])
    elim = []
    for k in range(10):
        qm = qbe.Model.from_circuitgen(circuit_model(random_grid_circuit(8, 8, 32, 5000 + k)))
        r = L.compare_order(qm, net)
        r.pop("order")
        elim.append(r)
    t3 = time.perf_counter()
    out = dict(train_info, workload="learned_6x6-8x8_d16-32_eval_8x8_d32", eval_s=t3 - t2, mem_cap_bytes=L.MEM_CAP,
               elimination={"mean_log2_gain_raw": float(np.mean([r["log2_gain_raw"] for r in elim])),
                            "mean_log2_gain_with_fallback": float(np.mean([r["log2_gain"] for r in elim])),
                            "learned_chosen": sum(r["chosen"] == "learned" for r in elim),
                            "per_circuit": [{k: (round(v, 3) if isinstance(v, float) else v) for k, v in r.items()}
                                            for r in elim]},
               mean_log2_gain=float(np.mean(gains)), mean_log2_gain_best_of_both=float(np.mean(best)),
               learned_chosen=sum(r["chosen"] == "learned" for r in rows),
               per_circuit=[{"heuristic_m": r["heuristic"]["m"], "learned_m": r["learned"]["m"],
                             "heuristic_log2_flops": round(r["heuristic"]["log2_total_flops"], 3),
                             "learned_log2_flops": round(r["learned"]["log2_total_flops"], 3),
                             "chosen": r["chosen"], "heuristic_plan_ms": round(r["heuristic"]["plan_ms"], 1),
                             "learned_plan_ms": round(r["learned"]["plan_ms"], 1)} for r in rows])
    return out




def bench_fused_c2(torch, qbe, ctx, steps, warmup):
    """5x5 depth-16 circuit, 64 slices: one LDS-resident fused launch per
    amplitude (issued directly or from a HIP graph) vs one launch per bucket."""
    name = "grid5x5_d16_m6"
    want = golden(name)
    plan, plan_ms, cfg = build_plan(qbe, ctx, name, "fused")
    st = plan.stats()
    ws = plan.workspace()
    out = torch.zeros(2, dtype=torch.float64, device="cuda")
    fn = lambda: qbe.qbe_contract_async(ctx, plan, ws, out)  # noqa: E731
    g = graph_of(torch, qbe, ctx, fn)
    forms = {}
    for form, call in (("fused", fn), ("fused+hipgraph", g.replay)):
        out.zero_()
        wall_f, ev_f = timed(torch, call, steps, warmup)
        got_f = complex(*out.cpu().numpy())
        forms[form] = {"ms_per_step": ev_f, "wall_ms_per_step": wall_f, "value": 1e3 / ev_f,
                       "rel_err": abs(got_f - want) / abs(want)}
    chosen = min(forms, key=lambda f: forms[f]["ms_per_step"])
    ev = forms[chosen]["ms_per_step"]
    plan_p, _, _ = build_plan(qbe, ctx, name, "per_step", merge=False)
    ws_p = plan_p.workspace()
    out_p = torch.zeros(2, dtype=torch.float64, device="cuda")
    wall_p, ev_p = timed(torch, lambda: qbe.qbe_contract_async(ctx, plan_p, ws_p, out_p), max(1, steps // 4), 1)
    err_p = abs(complex(*out_p.cpu().numpy()) - want) / abs(want)
    flops = st["flops_per_slice"] * plan.n_slices
    achieved = flops / (ev * 1e-3) / 1e12
    return {"workload": name, "form": chosen, "ms_per_amplitude": ev, "amplitudes_per_s": 1e3 / ev,
            "rel_err": forms[chosen]["rel_err"], "forms": forms, "planning_ms": plan_ms, "config": cfg,
            "plain_fp32": {"ms_per_amplitude": ev_p, "amplitudes_per_s": 1e3 / ev_p, "rel_err": err_p},
            "speedup_vs_plain": ev_p / ev,
            "roofline": {"bound": "alu", "achieved": achieved, "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                         "frac": achieved / FP32_PEAK_TFLOPS, "traffic": fused_traffic(), "kernel": "fused_kernel",
                         "algorithmic_flops_per_launch": flops,
                         "note": "LDS-resident: operands and intermediates stay on chip; bounded by the chain of "
                                 "dependent bucket levels (latency), not by HBM or ALU throughput"}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-extra", action="store_true", help="headline line only")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-learned", action="store_true", help="headline without the learned proposal")
    ap.add_argument("--only", choices=["headline", "c2", "batch", "many", "learned", "permute"],
                    help="run just one workload")
    ap.add_argument("--pmc-workload", action="store_true",
                    help="for hardware-counter runs: a device-to-device copy of 256 MiB (three times, the "
                         "calibration of the byte counters) and 20 launches of the 5x5 fused kernel")
    ap.add_argument("--pmc-c3", choices=["fp32", "bf16x6", "bf16x3", "plain_fp32"],
                    help="for hardware-counter runs: the copy calibration, then the headline plan in this form "
                         "(sliced set from --mu, else tree-trimming), autotuned, and two contractions")
    ap.add_argument("--plan", default="min_fill+tt_rec2_t16_s5+segments+sums2",
                    help="for --pmc-c3: a candidate plan of the headline search without the network "
                         "(min_fill or anytime8, + tt or tt_rec<k>_t<tries>_s<seed>), optionally followed by "
                         "+prefix or +segments")
    ap.add_argument("--reps", type=int, default=2, help="contractions in a --pmc-c3 run")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only: the contraction runs on a single MI355X "
              f"(--gpus {args.gpus} is not supported)", file=sys.stderr)
        sys.exit(2)

    if args.only == "headline":
        args.no_extra = args.no_cpu = True

    import torch

    import paper_2004_10892_amd as qbe

    ctx = qbe.Context(0)
    if args.pmc_workload or args.pmc_c3:
        src = torch.ones(64 << 20, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
    if args.pmc_workload:
        name = "grid5x5_d16_m6"
        plan, _, _ = build_plan(qbe, ctx, name, "fused")
        ws = plan.workspace()
        out = torch.zeros(2, dtype=torch.float64, device="cuda")
        for _ in range(20):
            qbe.qbe_contract_async(ctx, plan, ws, out)
        torch.cuda.synchronize()
        got = complex(*out.cpu().numpy())
        log(f"[bench] pmc workload done, rel err {abs(got - golden(name)) / abs(golden(name)):.2e}")
        return
    if args.pmc_c3:
        qm, m = c3_model(qbe)
        cands = plan_candidates(qbe, qm, m, None)
        base, use_prefix, use_segments, use_sums = split_plan_name(args.plan)
        if base not in cands:
            raise SystemExit(f"--plan must be one of {sorted(cands)}, optionally followed by +prefix or +segments "
                             "and +sums<N>")
        mu, pi, _ = cands[base]
        plain = args.pmc_c3 == "plain_fp32"
        plan = qbe.Plan(qm, pi, mu, ctx=ctx, exec="per_step", precision="fp32" if plain else args.pmc_c3,
                        merge=not plain, fused_prefix=use_prefix and not plain,
                        fused_segments=use_segments and not plain, fold_inputs=not plain,
                        max_sums=0 if plain else use_sums)
        ws = plan.workspace()
        out = torch.zeros(2, dtype=torch.float64, device="cuda")
        if not plain:
            plan.autotune(ws)
        torch.cuda.synchronize()
        for _ in range(args.reps):
            qbe.qbe_contract_async(ctx, plan, ws, out)
        torch.cuda.synchronize()
        got = complex(*out.cpu().numpy())
        log(f"[bench] pmc c3 {args.pmc_c3} plan {args.plan} mu {mu}: {plan.stats()['n_launches'] + 2} dispatches "
            f"per contraction, rel err {abs(got - golden(C3)) / abs(golden(C3)):.2e}")
        return
    if args.only == "c2":
        print(json.dumps(bench_fused_c2(torch, qbe, ctx, args.steps, args.warmup)), flush=True)
        return
    if args.only == "batch":
        print(json.dumps(bench_batch(torch, qbe, ctx, args.steps)), flush=True)
        return
    if args.only == "many":
        print(json.dumps(bench_many(torch, qbe, ctx, args.steps)), flush=True)
        return
    if args.only == "permute":
        print(json.dumps(bench_permute(torch, qbe, ctx, args.steps)), flush=True)
        return

    net, train_info = (None, None)
    if not args.no_learned or args.only == "learned":
        log("[bench] training the learned proposal's network ...")
        net, train_info = train_net(qbe, ctx)
        log(f"[bench] {train_info['labels']} labels, train {train_info['train_s']:.1f} s, loss "
            f"{train_info['loss_first_epoch']:.3f} -> {train_info['loss_last_epoch']:.3f}")
    if args.only == "learned":
        print(json.dumps(bench_learned(qbe, net, train_info)), flush=True)
        return

    h = bench_headline(torch, qbe, ctx, args.steps, args.warmup, net)
    ev = h["ev"]
    line = {
        "metric": METRIC, "value": 1e3 / ev, "unit": "amplitudes/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ev, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32" if h["chosen"] == "fp32" else "bf16",
        "data": "synthetic", "config": h["config"],
        "rel_err": h["rel_err"], "precision": h["chosen"],
        "mfma_util": h["mfma"]["value"], "mfma_util_plain_fp32": h["mfma"]["plain_fp32"],
        "mfma_util_source": h["mfma"]["source"],
        "plain_fp32": h["plain"], "speedup_vs_plain": h["plain"]["ms_per_amplitude"] / ev,
        "forms": h["forms"],
        "planning_ms": h["planning_ms"], "amplitudes_per_s_with_planning": 1e3 / (ev + h["planning_ms"]),
        "note_planning": "host planning of the chosen plan (its order and sliced set, schedule); the plan search "
                         "over candidate plans (plans) is a one-time cost per circuit; the plan is cached across "
                         "amplitudes in the timed loop",
        "plan": h["mu_source"], "plan_search_s": h["plan_search_s"], "plans": h["plans"], "mu": h["mu"],
        "combined_form": h["combined"],
        "roofline": h["roofline"], "launches_top": h["launches_top"],
    }
    if train_info:
        line["learned_training"] = train_info
    if not args.no_cpu:
        log("[bench] cpu baseline (oracle, sampled slices) ...")
        line["cpu_baseline"] = cpu_baseline_slices(C3)
    if not args.no_extra:
        log("[bench] 5x5 d16 fused ...")
        line["c2_fused"] = bench_fused_c2(torch, qbe, ctx, 100, 10)
        log("[bench] batch of 512 ...")
        line["batch_workload"] = bench_batch(torch, qbe, ctx, 20)
        log("[bench] 256 bitstrings of the 5x5 circuit ...")
        line["many_amplitudes"] = bench_many(torch, qbe, ctx, 20)
        log("[bench] stand-alone permute ...")
        line["permute_workload"] = bench_permute(torch, qbe, ctx, 10)
        if net is not None:
            log("[bench] learned proposal on 8x8 d32 ...")
            line["learned_proposal"] = bench_learned(qbe, net, train_info)
    print(json.dumps(line), flush=True)
    if h["rel_err"] > 1e-5 or h["plain"]["rel_err"] > 1e-5:
        sys.exit(1)


if __name__ == "__main__":
    main()

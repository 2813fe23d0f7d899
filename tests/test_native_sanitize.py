"""The host planner and plan compiler (planner.cpp, program.cpp,
program_check.cpp) built with AddressSanitizer and UndefinedBehaviorSanitizer
(g++, host code only) and run on circuit plans of every form the library
builds: tree-trimming with and without Alg. 2's order recomputation, merged
and one launch per bucket, the 7x7 depth-24 workload included.  Any
out-of-bounds access, use after free, overflow or other undefined behaviour
in the index arithmetic that the device programs inherit fails the test."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2004_10892_amd", "csrc")


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("no g++")
    out = str(tmp_path_factory.mktemp("asan") / "plan_sanitize")
    cmd = [gxx, "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=undefined", os.path.join(ROOT, "tests", "native", "plan_sanitize.cpp"),
           os.path.join(CSRC, "planner.cpp"), os.path.join(CSRC, "program.cpp"),
           os.path.join(CSRC, "program_check.cpp"), "-o", out]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-3000:]
    return out


def write_case(path, mod, order, mu):
    with open(path, "w") as f:
        f.write(f"{mod.n_vars} {len(mod.tensors)}\n")
        for vs, _ in mod.tensors:
            f.write(" ".join(str(v) for v in [len(vs)] + list(vs)) + "\n")
        f.write(" ".join(map(str, [len(order)] + list(order))) + "\n")
        f.write(" ".join(map(str, [len(mu)] + list(mu))) + "\n")


@pytest.mark.parametrize("rows,cols,depth,seed,m", [(4, 4, 10, 0, 0), (5, 5, 16, 1, 6), (6, 6, 20, 3, 5),
                                                    (7, 7, 24, 0, 10)])
def test_planner_and_compiler_under_sanitizers(driver, tmp_path, rows, cols, depth, seed, m):
    import paper_2004_10892_amd as qbe
    from circuitgen import circuit_model, random_grid_circuit
    mod = circuit_model(random_grid_circuit(rows, cols, depth, seed))
    qm = qbe.Model.from_circuitgen(mod)
    order = qbe.qbe_order_min_fill(qm)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    for k, kw in enumerate((dict(), dict(recompute_every=2, tries=4, seed=1))):
        mu, pi, _ = qbe.qbe_slice(qm, order, m, **kw)
        path = str(tmp_path / f"case{k}.txt")
        write_case(path, mod, pi, mu)
        r = subprocess.run([driver, path], capture_output=True, text=True, timeout=600, env=env)
        assert r.returncode == 0 and r.stdout.strip() == "ok", (r.stdout[-2000:], r.stderr[-4000:])
        assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-4000:]


def test_star_network_with_rank30_intermediate_under_sanitizers(driver, tmp_path):
    from circuitgen import star_network
    mod = star_network(30, seed=5)
    path = str(tmp_path / "star.txt")
    write_case(path, mod, list(range(31)), [])
    r = subprocess.run([driver, path], capture_output=True, text=True, timeout=600)
    assert r.returncode == 0 and r.stdout.strip() == "ok", (r.stdout, r.stderr[-4000:])

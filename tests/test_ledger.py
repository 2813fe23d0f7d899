"""Slice ledger on the host (no device): failure recovery and resume.

The slices of a plan are independent subtasks (Sec. 2.4) and the result is
their sum (Eq. 4), so a job records each slice range's partial sum as it
completes, re-runs only ranges whose result was lost or rejected, and can be
resumed from a saved ledger.  Here the partial sums are synthetic (seeded
per-slice values summed per range on the host): a failed range (a non-finite
result), a lost range (dropped after recording) and an interruption (save,
then load in a fresh ledger) are injected, and the resumed ledger's sum must
equal the range-order sum of the same partials bit for bit, and the exact
sum of the per-slice values to rounding."""
import ctypes as C
import math
import struct

import numpy as np
import pytest


@pytest.fixture(scope="module")
def qbe():
    import paper_2004_10892_amd as q
    return q


def _slices(n, seed=7):
    return np.random.default_rng(seed).standard_normal(2 * n).view(np.complex128)


def _partials(vals, n, rs):
    return [complex(vals[b:min(n, b + rs)].sum()) for b in range(0, n, rs)]


def test_ranges_cover_the_slices_with_a_ragged_tail(qbe):
    led = qbe.Ledger(1000, 128, tag=0xfeed)
    info = led.info()
    assert info == dict(n_slices=1000, range_size=128, tag=0xfeed, n_ranges=8, n_done=0)
    assert led.next() == (0, 0, 128)
    for i in range(7):
        led.record(i, complex(i, -i))
    assert led.next() == (7, 896, 1000)
    assert qbe.Ledger(1, 1).info()["n_ranges"] == 1
    assert qbe.Ledger(7, 100).next() == (0, 0, 7)


def test_failed_and_lost_ranges_rerun_and_resume_from_a_file(qbe, tmp_path):
    n, rs = 1000, 96
    vals = _slices(n)
    parts = _partials(vals, n, rs)
    led = qbe.Ledger(n, rs, tag=42)
    # first run: ranges 0..5 complete, range 3 fails (non-finite result)
    for i in range(6):
        if i == 3:
            with pytest.raises(qbe.QbeError, match="not finite"):
                led.record(i, complex(float("nan"), 0.0))
            continue
        led.record(i, parts[i])
    assert led.next()[0] == 3
    # range 1's result is judged lost; the job stops and saves
    led.drop(1)
    assert led.get(1) == (False, 0j)
    assert led.get(2) == (True, parts[2])
    path = str(tmp_path / "job.ledger")
    led.save(path)
    led.close()
    # resume in a fresh ledger: exactly ranges 1, 3 and 6.. are pending
    res = qbe.Ledger.load(path)
    info = res.info()
    assert (info["n_slices"], info["range_size"], info["tag"], info["n_done"]) == (n, rs, 42, 4)
    pending = []
    while True:
        nxt = res.next()
        if nxt is None:
            break
        i, b, e = nxt
        assert (b, e) == (i * rs, min(n, (i + 1) * rs))
        pending.append(i)
        res.record(i, parts[i])
    assert pending == [1, 3] + list(range(6, len(parts)))
    got = res.sum()
    re = im = 0.0
    for p in parts:  # range order, left to right
        re += p.real
        im += p.imag
    assert got == complex(re, im)
    exact = complex(math.fsum(vals.real), math.fsum(vals.imag))
    assert abs(got - exact) <= 1e-13 * np.abs(vals).sum()


def test_sum_refuses_pending_ranges_and_records_are_checked(qbe):
    led = qbe.Ledger(64, 16)
    led.record(0, 1 + 2j)
    with pytest.raises(qbe.QbeError, match="3 ranges pending"):
        led.sum()
    with pytest.raises(qbe.QbeError, match="already recorded"):
        led.record(0, 1j)
    for bad in (-1, 4):
        with pytest.raises(qbe.QbeError, match="out of range"):
            led.record(bad, 1j)
        with pytest.raises(qbe.QbeError, match="out of range"):
            led.drop(bad)
    with pytest.raises(qbe.QbeError, match="not finite"):
        led.record(1, complex(0.0, float("inf")))
    assert led.info()["n_done"] == 1
    for n, rs in ((0, 1), (1, 0), (-5, 3)):
        with pytest.raises(qbe.QbeError):
            qbe.Ledger(n, rs)


def test_run_checks_its_arguments_without_a_device(qbe):
    led = qbe.Ledger(16, 4)
    n = C.c_int64(5)
    rc = qbe._lib.qbe_ledger_run(None, None, led.handle, None, 0, -1, C.byref(n))
    assert qbe.ERRORS[rc] == "INVALID_ARG" and n.value == 0


def _write(path, magic=b"QBELDG01", n=10, rs=4, tag=1, ranges=None, tail=b""):
    if ranges is None:
        ranges = [(1, float(i), -float(i)) for i in range((n - 1) // rs + 1)]
    with open(path, "wb") as f:
        f.write(magic + struct.pack("<qqQ", n, rs, tag))
        for d, re, im in ranges:
            f.write(struct.pack("<qdd", d, re, im))
        f.write(tail)


def test_load_accepts_the_documented_layout_and_rejects_damage(qbe, tmp_path):
    p = str(tmp_path / "a")
    _write(p)
    led = qbe.Ledger.load(p)
    assert led.info() == dict(n_slices=10, range_size=4, tag=1, n_ranges=3, n_done=3)
    assert led.sum() == complex(3.0, -3.0)
    # the file the library writes is that layout, byte for byte
    q = str(tmp_path / "b")
    led.save(q)
    assert open(q, "rb").read() == open(p, "rb").read()
    cases = {
        "magic": dict(magic=b"QBELDG02"),
        "count": dict(ranges=[(1, 0.0, 0.0)] * 2),
        "tail": dict(tail=b"\0"),
        "flag": dict(ranges=[(1, 0.0, 0.0), (2, 0.0, 0.0), (0, 0.0, 0.0)]),
        "value": dict(ranges=[(1, 0.0, 0.0), (1, float("nan"), 0.0), (0, 0.0, 0.0)]),
        "sizes": dict(n=0, ranges=[]),
    }
    for name, kw in cases.items():
        bad = str(tmp_path / name)
        _write(bad, **kw)
        with pytest.raises(qbe.QbeError):
            qbe.Ledger.load(bad)
    with open(str(tmp_path / "short"), "wb") as f:
        f.write(b"QBELDG01" + struct.pack("<q", 10))
    with pytest.raises(qbe.QbeError, match="truncated"):
        qbe.Ledger.load(str(tmp_path / "short"))
    with pytest.raises(qbe.QbeError, match="cannot open"):
        qbe.Ledger.load(str(tmp_path / "missing"))

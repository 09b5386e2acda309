"""The correctly rounded sin, cos and log of gp_crmath.h, compiled for the
host, against the C library's double and extended-precision results (the
same decision the exception tables were built from): a strided pass over
every float, and the inputs the exception tables list.  The device copy of
the same code is compared with the oracle on every float by
tests/test_gpu_crmath.py."""
import os
import subprocess

import pytest

CSRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2110_11226_amd", "csrc")


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("crmath") / "crmath_check")
    subprocess.run(["g++", "-O2", "-std=c++17", "-ffp-contract=off", "-fopenmp", "-I", CSRC, "-o", exe,
                    os.path.join(CSRC, "crmath_check.cpp")], check=True)
    return exe


@pytest.mark.parametrize("fn", ["sin", "cos", "log"])
def test_strided_pass_over_every_binade(checker, fn):
    out = subprocess.run([checker, fn, "251"], check=True, capture_output=True, text=True).stdout
    summary = {ln.split()[1]: ln.split()[2:] for ln in out.splitlines() if ln.startswith("summary")}
    n, flagged, wrong, unflagged, undecided, entries = summary[fn]
    assert int(n) > 4_000_000
    assert int(wrong) == 0 and int(unflagged) == 0 and int(undecided) == 0, out[-2000:]
    if fn in ("sin", "cos"):
        # the negative inputs (-0, -inf and NaN among them): sin(-x) = -sin x,
        # cos(-x) = cos x bit for bit
        n, _, bad, _, _, _ = summary["sign"]
        assert int(n) > 8_000_000 and int(bad) == 0, out[-2000:]


def test_exception_entries_match_the_findings_file():
    """Every "<fn> <x> <result>" line of crmath_exceptions.txt is in the
    generated tables, and nothing else is."""
    found = set()
    for ln in open(os.path.join(CSRC, "crmath_exceptions.txt")):
        p = ln.split()
        if len(p) == 3 and p[0] in ("sin", "cos", "log"):
            found.add((p[0], int(p[1], 16), int(p[2], 16)))
    text = open(os.path.join(CSRC, "gp_crmath_tables.h")).read()
    tab = set()
    for name in ("sin", "cos", "log"):
        block = text.split(f"k{name.capitalize()}Exc[")[1].split("};")[0]
        for ln in block.splitlines():
            ln = ln.strip().strip(",").strip("{}")
            if ln.startswith("0x") and "," in ln:
                a, b = (int(v.strip().rstrip("u"), 16) for v in ln.split(","))
                if a != 0xffffffff:
                    tab.add((name, a, b))
    assert tab == found and len(found) > 0


def entries():
    rows = []
    for ln in open(os.path.join(CSRC, "crmath_exceptions.txt")):
        p = ln.split()
        if len(p) == 3 and p[0] in ("sin", "cos", "log"):
            rows.append((p[0], int(p[1], 16), int(p[2], 16)))
    return rows


@pytest.mark.parametrize("fn,x,want", entries())
def test_each_exception_entry_is_needed_and_applied(checker, fn, x, want):
    """Each listed input: its double result rounds to the wrong float (the
    entry is needed), lies near a rounding boundary (the lookup is reached),
    and the function with its tables returns the correctly rounded float."""
    out = subprocess.run([checker, fn, "1", hex(x), hex(x)], check=True, capture_output=True, text=True).stdout
    summary = {ln.split()[1]: ln.split()[2:] for ln in out.splitlines() if ln.startswith("summary")}
    n, flagged, wrong, unflagged, undecided, n_entries = summary[fn]
    assert (int(n), int(flagged), int(n_entries)) == (1, 1, 1), out
    assert int(wrong) == 0 and int(unflagged) == 0 and int(undecided) == 0, out
    assert f"{fn} {x:#010x} {want:#010x}" in out, out

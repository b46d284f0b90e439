"""The oracle's pins catch plausible mistakes (CPU only).

Each mutant is the oracle's C source with one plausible slip planted in it
(a dropped term, a wrong sign or comparison, a transposed operand, a wrong
tie rule, a missing check, a slip in assembling the hull from its hoods).  It is compiled with gcc into a temporary
library, and the pin suite below -- hand-derived fixtures, brute force on
random lattices (upper and lower hood, hull corners and their order),
closed forms and the contract's error codes -- must reject
every one of them, while accepting the unmodified source.
"""
import ctypes
import os
import subprocess

import numpy as np
import pytest

import synth
from oracle import brute, invariants
from tests import golden_io

SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                   "oracle", "hull_oracle.c")

MUTANTS = {
    "non-strict hood (pop only on > 0)": (
        "Y[rep]) >= 0)", "Y[rep]) > 0)"),
    "lower hood (flipped pop test)": (
        "Y[rep]) >= 0)", "Y[rep]) <= 0)"),
    "equal-x tie keeps highest index": (
        "if (Y[j] > Y[rep]) rep = j;", "if (Y[j] >= Y[rep]) rep = j;"),
    "equal-x keeps lowest y": (
        "if (Y[j] > Y[rep]) rep = j;", "if (Y[j] < Y[rep]) rep = j;"),
    "no equal-x reduction": (
        "while (j < n && X[j] == X[i]) {", "while (0 && j < n && X[j] == X[i]) {"),
    "dropped term in orient": (
        "return (i128)(bx - ax) * (i128)(cy - ay) - (i128)(by - ay) * (i128)(cx - ax);",
        "return (i128)(bx - ax) * (i128)(cy - ay);"),
    "transposed operand in orient": (
        "(i128)(by - ay) * (i128)(cx - ax);", "(i128)(cy - ay) * (i128)(bx - ax);"),
    "wrong sign in orient": (
        "(i128)(bx - ax) * (i128)(cy - ay) - (i128)", "(i128)(bx - ax) * (i128)(cy - ay) + (i128)"),
    "wrong stack index": (
        "int64_t a = out_idx[h - 2], b = out_idx[h - 1];",
        "int64_t a = out_idx[h - 1], b = out_idx[h - 2];"),
    "missing sortedness check": (
        "if (i > 0 && X[i] < X[i - 1]) return OR_ERR_UNSORTED;", ""),
    "missing grid check": (
        "if (t != s) return OR_ERR_GRID;", ""),
    "lower hood not mirrored": (
        "if (rc == OR_OK && lower)", "if (rc == OR_OK && 0 && lower)"),
    "hull keeps the shared right end twice": (
        "if (k == hu - 1 && up[k] == out_idx[hl - 1]) continue;", ""),
    "hull keeps the shared left end twice": (
        "if (k == 0 && up[k] == out_idx[0]) continue;", ""),
    "hull walks the upper hood left to right": (
        "out_idx[h++] = up[k];", "out_idx[h++] = up[hu - 1 - k];"),
}


def _compile(src_text, tmp_path, name):
    c = tmp_path / f"{name}.c"
    so = tmp_path / f"{name}.so"
    c.write_text(src_text)
    subprocess.check_call(["gcc", "-O1", "-std=c11", "-shared", "-fPIC", str(c),
                           "-o", str(so), "-lm"])
    lib = ctypes.CDLL(str(so))
    for name in ("oracle_upper_hull", "oracle_lower_hull", "oracle_convex_hull"):
        getattr(lib, name).argtypes = [ctypes.c_void_p, ctypes.c_int64,
                                       ctypes.c_void_p, ctypes.c_void_p]
        getattr(lib, name).restype = ctypes.c_int
    return lib


def _run(lib, xy, name="oracle_upper_hull"):
    a = np.ascontiguousarray(np.asarray(xy, np.float32).reshape(-1, 2))
    out = np.zeros(max(a.shape[0], 1), np.int32)
    cnt = ctypes.c_int64(0)
    rc = getattr(lib, name)(a.ctypes.data, a.shape[0], out.ctypes.data,
                            ctypes.addressof(cnt))
    return rc, [int(i) for i in out[:cnt.value]]


def _pins_pass(lib) -> bool:
    for path in golden_io.all_fixtures():
        xy, expect = golden_io.load(path)
        if _run(lib, xy) != (0, list(expect)):
            return False
    for seed in range(150):
        xy = synth.lattice_points(1 + seed % 12, 8, seed=77 + seed)
        if _run(lib, xy) != (0, brute.upper_hull_brute(xy)):
            return False
        if _run(lib, xy, "oracle_lower_hull") != (0, brute.lower_hull_brute(xy)):
            return False
        if seed % 3 == 0:  # the hull's brute force is O(n^4)
            rc, got = _run(lib, xy, "oracle_convex_hull")
            if rc != 0 or sorted(got) != brute.convex_hull_corners_brute(xy) or \
                    invariants.check_convex_hull(xy, got):
                return False
    if _run(lib, [[0.5, 0.0], [0.25, 0.0]])[0] != -10:
        return False
    if _run(lib, [[0.5, 2.0 ** -40]])[0] != -12:
        return False
    return True


def test_unmodified_oracle_passes(tmp_path):
    assert _pins_pass(_compile(open(SRC).read(), tmp_path, "orig"))


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(tmp_path, name):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation site not found: {old!r}"
    lib = _compile(src.replace(old, new), tmp_path, "mut")
    assert not _pins_pass(lib), f"pins did not catch: {name}"

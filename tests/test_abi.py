"""The C-ABI library loads and exports every entry point its header declares
(CPU only: no call here touches a GPU)."""
import ctypes
import os
import re

import pytest

import paper_1203_5004_amd as uh

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "wagener_hull.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^[A-Za-z_][\w \*]*?\b((?:upper|convex)_hull\w*)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("upper_hull", "upper_hull_plan_create", "upper_hull_plan_run",
                     "upper_hull_plan_destroy", "upper_hull_bridge", "upper_hull_orient",
                     "upper_hull_status_string", "convex_hull"):
        assert required in names
    assert sorted(names) == sorted(uh.EXPORTS)


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(uh.LIB_PATH):
        pytest.fail("library not built: run `python -m paper_1203_5004_amd.build`")
    return uh.load_library()


def test_every_declared_symbol_is_exported(lib):
    raw = ctypes.CDLL(uh.LIB_PATH)
    for name in declared_functions():
        assert hasattr(raw, name), name


def test_status_strings(lib):
    assert uh.upper_hull_status_string(uh.UH_OK) == "ok"
    for code in (uh.UH_ERR_ARG, uh.UH_ERR_ALLOC, uh.UH_ERR_HIP, uh.UH_ERR_CAPTURE,
                 uh.UH_ERR_WORKSPACE, uh.UH_ERR_TOO_LARGE,
                 uh.UH_ERR_UNSORTED, uh.UH_ERR_RANGE, uh.UH_ERR_GRID):
        s = uh.upper_hull_status_string(code)
        assert s and s != "unknown status"


def test_status_codes_match_the_oracle_contract():
    import oracle
    assert (uh.UH_ERR_UNSORTED, uh.UH_ERR_RANGE, uh.UH_ERR_GRID) == (
        oracle.ERR_UNSORTED, oracle.ERR_RANGE, oracle.ERR_GRID)


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    monkeypatch.setattr(uh, "_lib", None)
    monkeypatch.setattr(uh, "LIB_PATH", str(tmp_path / "nope.so"))
    with pytest.raises(RuntimeError, match="no CPU fallback"):
        uh.load_library()


def test_workspace_bytes_is_pure_arithmetic(lib):
    # callable without a GPU; monotone in both bounds; about 12 bytes a point
    # (16 with the convex hull's hood buffers); 0 for invalid bounds
    f = uh.upper_hull_workspace_bytes
    assert f(-1, 1) == 0 and f(10, 0) == 0
    prev = 0
    for m in (0, 1, 1023, 1024, 1025, 65536, 1 << 20, (1 << 20) + 1, 1 << 27):
        b = f(m, 1)
        assert b >= prev and b >= 12 * m
        assert b <= 12 * m + 64 * 1024 + m // 8, (m, b)
        assert f(m, 2) >= b + 4 * m
        prev = b
    assert f(1 << 27, 4096) > f(1 << 27, 1)
    assert f(1 << 27, 1) % 256 == 0

"""The C-ABI library loads and exports every symbol include/ozk.h declares;
host-only size/layout functions agree with the documented formulas.  No
compute calls (no GPU here)."""
import ctypes
import os
import re

import pytest

import paper_2606_25453_amd as ozk

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ozk.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ozk_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(ozk.LIB_PATH):
        pytest.skip("libozk.so not built")
    return ozk.library()


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert len(names) >= 19
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(ozk.EXPORTS) == names


def test_packed_sizes_and_k_split(lib):
    assert ozk.ozk_s1_packed_bytes(1, 1, 1) == 256 * 32
    assert ozk.ozk_s1_packed_bytes(300, 65, 8) == 512 * 96 * 8
    assert ozk.ozk_s2_packed_bytes(300, 65, 16, 1) == 512 * 96 * 16 * 3
    assert ozk.ozk_s1_packed_bytes(-1, 1, 1) == 0
    for p in range(1, 9):
        per_k = 2 ** 12 if p == 1 else (p - 1) * 2 ** 14
        k = ozk.ozk_s1_k_split(p)
        assert k % 32 == 0 and per_k * k < 2 ** 31 <= per_k * (k + 32)
    assert ozk.ozk_s1_k_split(0) == 0 and ozk.ozk_s1_k_split(9) == 0


def test_null_context_is_rejected(lib):
    assert lib.ozk_dgemm(None, 1, 4, 1, 1, 1, 1.0, None, 1, None, 1, 0.0, None, 1, None, 0, None) == \
        ozk.OZK_ERR_INVALID_ARG
    assert lib.ozk_sgemm(None, 1, 4, 1, 1, 1, 1.0, None, 1, None, 1, 0.0, None, 1, None, 0, None) == \
        ozk.OZK_ERR_INVALID_ARG
    assert lib.ozk_status_string(ozk.OZK_ERR_WORKSPACE).decode() == "workspace missing or too small"
    assert lib.ozk_version().decode().count(".") == 2
    assert lib.ozk_last_arg(None) == 0


def test_header_constants_match_the_binding():
    """Every integer #define of the header that the binding mirrors has the
    same value there."""
    import re
    text = open(os.path.join(ROOT, "include", "ozk.h")).read()
    defines = dict((k, int(v)) for k, v in re.findall(r"^#define (OZK_\w+) \(?(-?\d+)\)?", text, re.M))
    mirrored = [k for k in defines if hasattr(ozk, k)]
    assert {"OZK_S1_VARIANTS", "OZK_S2_VARIANTS", "OZK_S2_FUSED_CRT", "OZK_K_CHUNK", "OZK_ROW_ALIGN"} <= set(mirrored)
    for k in mirrored:
        assert getattr(ozk, k) == defines[k], k

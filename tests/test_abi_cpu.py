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


def _fake_ctx():
    """A Context object that was never created on a device: the binding's
    argument checks must reject the tensors below before it is used."""
    c = ozk.Context.__new__(ozk.Context)
    c.handle = None
    c.device = 0
    return c


def test_binding_rejects_bad_tensors_before_any_call():
    torch = pytest.importorskip("torch")
    ctx = _fake_ctx()
    f64 = lambda *s: torch.zeros(*s, dtype=torch.float64)  # noqa: E731
    cases = [
        (lambda: ozk.ozk_dgemm(ctx, 1, 4, f64(4, 5), f64(6, 3)), "inner dimensions"),
        (lambda: ozk.ozk_dgemm(ctx, 1, 4, f64(4, 5).float(), f64(5, 3)), "dtype"),
        (lambda: ozk.ozk_dgemm(ctx, 1, 4, f64(4, 5), f64(5, 3), C=f64(4, 2)), "shape"),
        (lambda: ozk.ozk_dgemm(ctx, 1, 4, f64(20), f64(5, 3)), "2-dimensional"),
        (lambda: ozk.ozk_dgemm(ctx, 1, 4, f64(4, 5), f64(5, 3)), "cuda:0"),
        (lambda: ozk.ozk_dgemm(ctx, 1, 4, [[1.0]], f64(5, 3)), "torch tensor"),
        (lambda: ozk.ozk_dgemm_t(ctx, 1, 4, f64(5, 4), f64(5, 3), trans_a=True, C=f64(3, 4)), "shape"),
        (lambda: ozk.ozk_sgemm(ctx, 1, 4, f64(4, 5), f64(5, 3)), "dtype"),
        (lambda: ozk.ozk_zgemm_3m(ctx, 8, f64(4, 5), f64(5, 3)), "dtype"),
        (lambda: ozk.ozk_cgemm_3m(ctx, 8, f64(4, 5).to(torch.complex128), f64(5, 3).to(torch.complex128)), "dtype"),
        (lambda: ozk.ozk_s1_dgemm_unfused(ctx, 3, f64(4, 5), f64(4, 3)), "inner dimensions"),
        (lambda: ozk.ozk_s2_split_rows(ctx, 8, f64(4, 5), complex_planes=1), "dtype"),
        (lambda: ozk.ozk_s1_diagonals(ctx, 3, 4, 4, 4, torch.zeros(10, dtype=torch.int8),
                                      torch.zeros(10, dtype=torch.int8)), "elements"),
        (lambda: ozk.BatchPlan(ctx, ozk.OZK_OP_ZGEMM, ozk.OZK_SCHEME2, 8, [(f64(2, 2), f64(2, 2), f64(2, 2))]),
         "problem 0"),
    ]
    for fn, what in cases:
        with pytest.raises(ValueError) as ei:
            fn()
        assert what in str(ei.value), (what, str(ei.value))

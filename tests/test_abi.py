"""CPU checks of the C ABI: the library loads, exports every function that
include/mor.h declares, and rejects invalid plan arguments before touching a
device (no compute calls without a GPU)."""
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "mor.h")).read()
    return sorted(set(re.findall(r"\b(mor_[a-z_]+)\s*\(", src)))


def test_every_declared_symbol_is_exported():
    import paper_2103_10203_amd as mor
    names = _declared()
    assert "mor_plan_create" in names and "mor_solve" in names
    for n in names:
        assert hasattr(mor.lib, n), n


def test_binding_covers_header():
    from paper_2103_10203_amd import _native
    assert set(_declared()) == set(_native._SIGS)


@pytest.mark.parametrize("shape,M,val,code", [
    ((16,), 3, 0, 1),            # ndim 1
    ((16, 16), 0, 0, 1),         # M < 1
    ((16, 16), 257, 0, 1),       # M > N
    ((16, 16), 5, 2, 1),         # phase value outside {0,1}
    ((14, 16), 5, 0, 6),         # 14 = 2*7 unsupported
    ((2048, 4), 5, 0, 6),        # too long an axis
])
def test_plan_create_rejects(shape, M, val, code):
    import ctypes as ct
    from paper_2103_10203_amd import _native as nat
    g = np.zeros(shape, np.uint8)
    g.flat[0] = val
    grid = nat.mor_grid()
    grid.ndim = len(shape)
    for a in range(3):
        grid.n[a] = shape[a] if a < len(shape) else 1
    h = ct.c_void_p()
    st = nat.lib.mor_plan_create(ct.byref(grid), g.ctypes.data_as(ct.c_void_p), M, None, ct.byref(h))
    assert st == code
    assert h.value is None
    assert len(nat.lib.mor_last_error()) > 0


@pytest.mark.parametrize("case,code", [
    ("negative_count", 1),
    ("null_map", 1),
    ("bad_M_in_second", 1),
    ("bad_phase_in_third", 1),
    ("unsupported_grid", 6),
])
def test_plan_create_batch_rejects(case, code):
    """mor_plan_create_batch checks every map and M before any device work;
    on error every output entry is NULL."""
    import ctypes as ct
    from paper_2103_10203_amd import _native as nat
    shape = (14, 16) if case == "unsupported_grid" else (16, 16)
    n = 3
    maps = np.zeros((n,) + shape, np.uint8)
    Ms = np.full(n, 5, np.int64)
    if case == "bad_M_in_second":
        Ms[1] = 257
    if case == "bad_phase_in_third":
        maps[2].flat[7] = 3
    count = -1 if case == "negative_count" else n
    grid = nat._grid_of(shape)
    hs = (ct.c_void_p * n)(*([ct.c_void_p(1).value] * n))
    ptrs = (ct.c_void_p * n)(*[maps[b].ctypes.data for b in range(n)])
    if case == "null_map":
        ptrs[1] = None
    st = nat.lib.mor_plan_create_batch(ct.byref(grid), count, ct.cast(ptrs, ct.c_void_p),
                                       Ms.ctypes.data_as(ct.c_void_p), None, ct.cast(hs, ct.c_void_p))
    assert st == code
    assert len(nat.lib.mor_last_error()) > 0
    if count > 0:
        assert all(h is None for h in hs)


def test_plan_create_batch_of_nothing():
    import ctypes as ct
    from paper_2103_10203_amd import _native as nat
    grid = nat._grid_of((16, 16))
    assert nat.lib.mor_plan_create_batch(ct.byref(grid), 0, None, None, None, None) == nat.MOR_OK


def test_null_arguments():
    from paper_2103_10203_amd import _native as nat
    assert nat.lib.mor_solve(None, None, 1, None, 1e-6, None, None) == nat.MOR_E_INVALID_ARG
    assert nat.lib.mor_plan_destroy(None) == nat.MOR_OK
    assert nat.lib.mor_profile_query(None, None, None, None, None) == nat.MOR_E_INVALID_ARG
    assert nat.lib.mor_profile_query(b"nope", None, None, None, None) == nat.MOR_E_INVALID_ARG


def test_tune_api_host_side():
    """Variant selection is host state: counts, get/set round trip and the
    rejected arguments (no GPU needed)."""
    import paper_2103_10203_amd as mor
    assert mor.tune_variants(2, 256) >= 2
    keep = mor.tune_get(2, 256)
    mor.tune_set(2, 256, 1)
    assert mor.tune_get(2, 256) == 1
    mor.tune_set(2, 256, keep)
    for args in [(2, 100), (4, 256), (2, 255)]:
        with pytest.raises(mor.MorError):
            mor.tune_variants(*args)
    with pytest.raises(mor.MorError):
        mor.tune_set(2, 256, mor.tune_variants(2, 256))
    with pytest.raises(mor.MorError):
        mor.tune_set(2, 256, -1)
    assert mor.tune_variants(2, 256, mor.KERNEL_COL) >= 2
    mor.tune_set(2, 256, 1, mor.KERNEL_COL)
    assert mor.tune_get(2, 256, mor.KERNEL_COL) == 1
    assert mor.tune_get(2, 256) == keep  # the row table is separate
    mor.tune_set(2, 256, 0, mor.KERNEL_COL)
    with pytest.raises(mor.MorError):
        mor.tune_variants(2, 100, mor.KERNEL_COL)
    with pytest.raises(mor.MorError):
        mor.tune_variants(2, 256, 7)
    # sub-batch limits: query, set, restore, reject
    start = mor.tune_subbatch()
    assert start[0] >= 0 and start[1] >= 1 and mor.tune_subbatch() == start
    assert mor.tune_subbatch(1 << 20, 4) == start
    assert mor.tune_subbatch(start[0], start[1]) == (1 << 20, 4)
    assert mor.tune_subbatch(-1, -1) == start
    for bad in ((-2, -1), (-1, 0), (-1, -2)):
        with pytest.raises(mor.MorError):
            mor.tune_subbatch(*bad)


def test_precision_constants_match_header():
    """The binding's precision values are the header's enum (FP32, BF16X3, FP64)."""
    import paper_2103_10203_amd as mor
    src = open(os.path.join(ROOT, "include", "mor.h")).read()
    m = re.search(r"enum\s*\{\s*MOR_PREC_FP32\s*=\s*(\d+),\s*MOR_PREC_BF16X3\s*=\s*(\d+),\s*MOR_PREC_FP64\s*=\s*(\d+)\s*\}",
                  src)
    assert m, "precision enum not found"
    assert (mor.PREC_FP32, mor.PREC_BF16X3, mor.PREC_FP64) == tuple(int(x) for x in m.groups())


def test_make_plans_checks_its_arguments():
    import paper_2103_10203_amd as mor
    g = np.zeros((16, 16), np.uint8)
    with pytest.raises(ValueError):
        mor.make_plans([g, g], [5])
    assert mor.make_plans([], 5) == []


def test_plan_arrays_cached_on_plan_lists():
    """The handle and size arrays of a PlanList are built once and rebuilt
    when a member changes or a plan is closed; a plain list is marshalled on
    every call.  (Stand-in plan objects: no device needed.)"""
    import ctypes as ct

    from paper_2103_10203_amd import _native

    class FakePlan:
        def __init__(self, h, n, nc):
            self.handle, self.N, self.n_coeff = ct.c_void_p(h), n, nc

    plans = _native.PlanList([FakePlan(16 * (i + 1), 100 + i, 7 + i) for i in range(5)])
    a = _native._plan_arrays(plans)
    assert [a[0][i] for i in range(5)] == [16 * (i + 1) for i in range(5)]
    assert a[1].tolist() == [100 + i for i in range(5)] and a[2].tolist() == [7 + i for i in range(5)]
    assert _native._plan_arrays(plans) is a
    po = np.array([4, 0, 0, 2], np.int64)
    assert _native._plan_sum(a[1], po) == 104 + 100 + 100 + 102
    assert _native._plan_sum(a[2], np.zeros(0, np.int64)) == 0
    plans[2] = FakePlan(999, 1, 2)  # a member replaced: rebuilt
    b = _native._plan_arrays(plans)
    assert b is not a and b[0][2] == 999 and b[1][2] == 1
    _native._plans_closed += 1  # as Plan.close() does: rebuilt
    try:
        assert _native._plan_arrays(plans) is not b
    finally:
        _native._plans_closed -= 1
    plain = list(plans)
    assert _native._plan_arrays(plain) is not _native._plan_arrays(plain)

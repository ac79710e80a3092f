"""The C-ABI library loads and exports every entry point include/mdpe.h
declares, and rejects bad calls without touching a GPU (host only)."""
import ctypes

import pytest

from paper_2101_10881_amd import mdpe


# the boundary's calls: plan once, evaluate per call (Section 5), batched,
# reverse pass, release, error strings
BOUNDARY = {"plan_polynomial", "plan_info", "eval_and_diff", "plan_batch", "eval_and_diff_batch", "eval_adjoint",
            "plan_destroy", "batch_destroy", "last_error_string"}


def test_header_symbols_exported():
    L = mdpe.lib()
    syms = mdpe.header_symbols()
    assert BOUNDARY <= set(syms), BOUNDARY - set(syms)
    for s in syms:
        assert hasattr(L, s), s


def test_boundary_calls_reject_null_arguments():
    L = mdpe.lib()
    assert L.eval_and_diff_batch(None, None, None, None, None, None, None) == mdpe.MDPE_EINVAL
    assert L.eval_adjoint(None, None, None, None, None, None, None) == mdpe.MDPE_EINVAL
    assert L.plan_batch(None, 0, None, None) == mdpe.MDPE_EINVAL
    L.batch_destroy(None)


def test_host_only_plan_cannot_evaluate():
    p = mdpe.Plan(3, [2], [0, 2], 4, 2, device=-1)
    rc = mdpe.lib().eval_and_diff(p.handle, None, None, None, None, None, None)
    assert rc == mdpe.MDPE_EINVAL
    assert "host-only" in mdpe.last_error_string()


def test_null_arguments():
    L = mdpe.lib()
    assert L.plan_polynomial(None, -1, None) == mdpe.MDPE_EINVAL
    assert L.plan_info(None, None) == mdpe.MDPE_EINVAL
    assert L.eval_and_diff(None, None, None, None, None, None, None) == mdpe.MDPE_EINVAL
    assert L.md_elementwise(7, 2, 4, None, None, None, None) == mdpe.MDPE_EINVAL
    assert L.md_elementwise(0, 2, 0, None, None, None, None) == mdpe.MDPE_OK   # empty: nothing to do
    L.plan_destroy(None)


def test_profiler_lifecycle_without_gpu():
    prof = mdpe.Profiler()
    t = prof.read()
    assert t["n_cnv"] == 0 and t["cnv_ms"] == 0.0
    del prof


def test_profiler_classes():
    # a mask of launch classes; unknown bits are refused without touching a GPU
    p = mdpe.Profiler(classes=mdpe.MDPE_TIME_CONV | mdpe.MDPE_TIME_ADD)
    with pytest.raises(mdpe.MdpeError) as e:
        mdpe.Profiler(classes=16)
    assert e.value.code == mdpe.MDPE_EINVAL
    assert p.read()["n_cnv"] == 0


def test_plan_info_fields():
    p = mdpe.Plan(5, [3, 2], [0, 1, 4, 2, 3], 7, 4, device=-1)
    i = p.info
    assert (i["n"], i["N"], i["d"], i["m"]) == (5, 2, 7, 4)
    assert i["workspace_bytes"] == i["n_series"] * 8 * 4 * 8

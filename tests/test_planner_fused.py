"""Fused convolution layers (MDPE_FUSED_LAYERS): the planner's split of the
convolution jobs into independent components, checked on the host.

* the fused rows hold exactly the plan's jobs, each component's in layer order;
* no slot written by a job of one component is read or written by a job of
  another (so components may run concurrently, each in one workgroup);
* running the jobs component by component on float64 series (every layer of
  component 0, then of component 1, ...) gives the bits of the layer-by-layer
  run, where any dependency across components would change the result.
"""
import numpy as np
import pytest

from paper_2101_10881_amd import mdpe
from paper_2101_10881_amd import workloads as W

CASES = [
    ("p2_1d_d8", lambda: W.p2(m=1, d=8), 0),
    ("p2_4d_d64", lambda: W.p2(), 0),
    ("p1_2d_d8", lambda: W.p1(m=2, d=8), 0),
    ("p1_keep", lambda: W.p1(m=2, d=4), mdpe.MDPE_KEEP_MONOMIAL_VALUES),
    ("p1_exponents", lambda: W.with_exponents(W.p1(m=2, d=4), 3, seed=5), 0),
    ("p1_complex", lambda: W.p1(m=1, d=4, cx=True), 0),
    ("rand3", lambda: W.rand3(), 0),
    ("p2_asap", lambda: W.p2(m=2, d=8), mdpe.MDPE_ASAP_LAYERS),
]


def _plan(w, flags):
    if w.cx:
        flags |= mdpe.MDPE_COMPLEX
    return mdpe.Plan(w.n, w.nvars, w.vars, w.d, w.m, -1, flags | mdpe.MDPE_FUSED_LAYERS, w.exps)


@pytest.mark.parametrize("name,build,flags", CASES, ids=[c[0] for c in CASES])
def test_components_are_independent_and_complete(name, build, flags):
    w = build()
    P = _plan(w, flags)
    info = P.info
    assert info["fused_components"] > 0 and 1 <= info["fused_waves"] <= 4
    rows = P.fused_jobs()
    jobs = P.conv_jobs()
    # the same jobs, with the same layers
    assert sorted(map(tuple, rows[:, 1:].tolist())) == sorted(map(tuple, jobs.tolist()))
    comp = rows[:, 0]
    assert np.all(np.diff(comp) >= 0) and comp[-1] == info["fused_components"] - 1
    for c in np.unique(comp):
        assert np.all(np.diff(rows[comp == c, 1]) >= 0)      # layers in order
    # the widest layer of a component bounds the wavefronts per workgroup
    widest = max(np.sum((comp == c) & (rows[:, 1] == L)) for c, L in set(map(tuple, rows[:, :2].tolist())))
    assert info["fused_waves"] == min(4, widest)
    # a slot written in one component is touched by no other
    owner = {}
    for c, _, t1, t2, t3 in rows.tolist():
        assert owner.setdefault(t3, c) == c
    for c, _, t1, t2, t3 in rows.tolist():
        for s in (t1, t2):
            assert owner.get(s, c) == c


def _run(P, w, order):
    """Leading limbs only, one float64 per coefficient; jobs of a layer read before any writes."""
    d1 = w.d + 1
    lead = (w.coeff[0, 0] if w.cx else w.coeff[0])
    zl = (w.z[0, 0] if w.cx else w.z[0])
    A = np.zeros((int(P.info["n_series"]), d1))
    A[: w.N + 1] = lead
    A[w.N + 1: w.N + 1 + w.n] = zl
    for batch in order:
        out = [np.convolve(A[t1], A[t2])[:d1] for t1, t2, _ in batch]
        for (_, _, t3), o in zip(batch, out):
            A[t3] = o
    return A


@pytest.mark.parametrize("name,build,flags", [c for c in CASES if not c[1]().cx], ids=[c[0] for c in CASES if not c[1]().cx])
def test_component_order_computes_the_layer_results(name, build, flags):
    w = build()
    P = _plan(w, flags)
    jobs = P.conv_jobs()
    layered = [[tuple(r[1:]) for r in jobs[jobs[:, 0] == L].tolist()] for L in range(1, P.info["n_layers"] + 1)]
    rows = P.fused_jobs()
    fused = []
    for c in np.unique(rows[:, 0]):
        mine = rows[rows[:, 0] == c]
        for L in np.unique(mine[:, 1]):
            fused.append([tuple(r[2:]) for r in mine[mine[:, 1] == L].tolist()])
    a, b = _run(P, w, layered), _run(P, w, fused)
    assert np.any(a != 0)
    assert np.array_equal(a.view(np.uint64), b.view(np.uint64))


def test_streamed_plans_do_not_fuse():
    w = W.p1(m=2, d=8)
    P = mdpe.Plan.for_workload(w, device=-1, flags=mdpe.MDPE_FUSED_LAYERS | mdpe.MDPE_STREAM_OPERANDS)
    assert P.info["streamed"] == 1 and P.info["fused_components"] == 0
    with pytest.raises(mdpe.MdpeError) as e:
        P.fused_jobs()
    assert e.value.code == mdpe.MDPE_EINVAL


def test_default_fuses_deep_plans_of_small_layers():
    # among the layered and fused launches (p2 takes the chain launch by default)
    fused = lambda w, f=mdpe.MDPE_NO_CHAIN_LAUNCH: mdpe.Plan.for_workload(w, device=-1, flags=f).info["fused_components"] > 0
    # p2: 64 layers of 378 jobs
    assert fused(W.p2(m=1, d=8)) and fused(W.p2()) and fused(W.p2(m=4, d=95)) and fused(W.p2(m=10, d=31))
    assert fused(W.p2(m=5, d=31)) and fused(W.p2(m=8, d=8))
    assert not fused(W.p2(m=10, d=32)) and not fused(W.p2(m=8, d=9))   # the boundary no longer dominates
    assert not fused(W.p2(m=4, d=152))                  # two wavefronts per job
    assert not fused(W.p1()) and not fused(W.p1(m=4, d=8))   # layers of thousands of jobs
    assert fused(W.p1(m=1, d=152)) and fused(W.p1(m=2, d=63))  # ... unless the steps are very short
    assert not fused(W.p1(m=2, d=64)) and not fused(W.p3(m=1, d=8))  # p3: two layers
    # the power table joins monomials into components of several jobs per layer
    assert not fused(W.with_exponents(W.p1(m=2, d=4), 3, seed=5))
    assert not fused(W.rand3())                         # three layers
    assert not fused(W.p2(m=1, d=8), mdpe.MDPE_LAYER_LAUNCHES)


def test_fused_and_layer_launches_exclude_each_other():
    w = W.p2(m=1, d=8)
    with pytest.raises(mdpe.MdpeError) as e:
        mdpe.Plan.for_workload(w, device=-1, flags=mdpe.MDPE_FUSED_LAYERS | mdpe.MDPE_LAYER_LAUNCHES)
    assert e.value.code == mdpe.MDPE_EINVAL

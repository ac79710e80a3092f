"""Layer balancing of the planner: convolutions with slack moved to later
layers so that layers fill whole rounds of the SIMDs.

Checked against the earliest-layer layering of Section 5 (MDPE_ASAP_LAYERS),
with a dependency analysis written here from the slot accesses, and by running
both layerings on float64 series layer by layer (every job of a layer reads
before any writes), where any broken dependency changes the result.
"""
import numpy as np
import pytest

from paper_2101_10881_amd import mdpe
from paper_2101_10881_amd import workloads as W

SIMDS = 1024


def _plans(w, flags=0):
    asap = mdpe.Plan.for_workload(w, device=-1, flags=flags | mdpe.MDPE_ASAP_LAYERS)
    bal = mdpe.Plan.for_workload(w, device=-1, flags=flags)
    return asap, bal


def _job_layers(p):
    jobs = p.conv_jobs()
    return {tuple(int(x) for x in r[1:]): int(r[0]) for r in jobs}, jobs


def _dependencies(jobs):
    """(earlier job, later job) triplets: read after write, write after write,
    write after read, from the slot accesses of a layer-ordered job list."""
    last_writer, readers, deps = {}, {}, []
    for layer in sorted(set(int(x) for x in jobs[:, 0])):
        rows = [tuple(int(x) for x in r[1:]) for r in jobs[jobs[:, 0] == layer]]
        for t in rows:
            for s in {t[0], t[1]}:
                if s in last_writer:
                    deps.append((last_writer[s], t))
            if t[2] in last_writer:
                deps.append((last_writer[t[2]], t))
            deps.extend((r, t) for r in readers.get(t[2], ()) if r != t)
        for t in rows:
            for s in {t[0], t[1]}:
                readers.setdefault(s, []).append(t)
        for t in rows:
            last_writer[t[2]] = t
            readers[t[2]] = []
    return deps


def _rounds(p):
    J, Q = p.info["jobs_per_group"], p.info["waves_per_job"]
    return sum(-(-(-(-int(c) // J) * Q) // SIMDS) for c in p.layer_sizes()[0])


def _run_float(p, w):
    """Leading limbs only, one float64 per coefficient: the plan's structure,
    not m-double arithmetic, is under test."""
    d1 = w.d + 1
    lead = w.coeff[0, 0] if w.cx else w.coeff[0]
    zl = w.z[0, 0] if w.cx else w.z[0]
    A = np.zeros((int(p.info["n_series"]), d1))
    A[: w.N + 1] = lead
    A[w.N + 1: w.N + 1 + w.n] = zl
    jobs = p.conv_jobs()
    for layer in range(1, p.info["n_layers"] + 1):
        rows = jobs[jobs[:, 0] == layer]
        out = [np.convolve(A[t1], A[t2])[:d1] for _, t1, t2, _ in rows]
        for r, o in zip(rows, out):
            A[r[3]] = o
    sc = p.scale_jobs()
    out = [A[s] * float(e) for s, _, e in sc]
    for (_, dst, _), o in zip(sc, out):
        A[dst] = o
    adds = p.add_jobs()
    for level in range(1, p.info["n_levels"] + 1):
        rows = adds[adds[:, 0] == level]
        out = [A[t2] + A[t1] for _, t1, t2 in rows]
        for r, o in zip(rows, out):
            A[r[2]] = o
    res = p.outputs()
    return np.stack([A[s] if s >= 0 else np.zeros(d1) for s in res])


CASES = [
    ("p1", lambda: W.p1(), 0),
    ("p1_keep", lambda: W.p1(), mdpe.MDPE_KEEP_MONOMIAL_VALUES),
    ("p1_streamed", lambda: W.p1(), mdpe.MDPE_STREAM_OPERANDS),
    ("p1_exponents", lambda: W.with_exponents(W.p1(m=2), 3, seed=5), 0),
    ("c4", lambda: W.p1(m=8, d=32), mdpe.MDPE_KEEP_MONOMIAL_VALUES),
    ("p1_d32", lambda: W.p1(m=2, d=32), 0),
]


def test_p1_balanced_sizes():
    asap, bal = _plans(W.p1())
    assert [int(c) for c in asap.layer_sizes()[0]] == [3640, 5460, 5460, 1820]
    assert [int(c) for c in bal.layer_sizes()[0]] == [3072, 4096, 6144, 3068]
    assert (asap.info["balanced_layers"], bal.info["balanced_layers"]) == (0, 1)
    assert (_rounds(asap), _rounds(bal)) == (18, 16)   # 16 = ceil(16380 / 1024)


@pytest.mark.parametrize("name,build,flags", CASES, ids=[c[0] for c in CASES])
def test_balanced_layering_keeps_every_dependency(name, build, flags):
    w = build()
    asap, bal = _plans(w, flags)
    assert bal.info["balanced_layers"] == 1
    assert _rounds(bal) < _rounds(asap)
    la, ja = _job_layers(asap)
    lb, _ = _job_layers(bal)
    assert sorted(la) == sorted(lb)                       # the same jobs
    assert bal.info["n_layers"] == asap.info["n_layers"]  # the same depth
    for before, after in _dependencies(ja):
        assert lb[before] < lb[after], (before, after)
    # additions, scale jobs and outputs are untouched
    assert np.array_equal(asap.add_jobs(), bal.add_jobs())
    assert np.array_equal(asap.scale_jobs(), bal.scale_jobs())
    assert np.array_equal(asap.outputs(), bal.outputs())
    for k in ("n_series", "n_conv", "n_add", "jobs_per_group", "waves_per_job", "lane_steps", "streamed"):
        assert asap.info[k] == bal.info[k], k


@pytest.mark.parametrize("name,build,flags", CASES, ids=[c[0] for c in CASES])
def test_balanced_layering_computes_the_same(name, build, flags):
    w = build()
    asap, bal = _plans(w, flags)
    a, b = _run_float(asap, w), _run_float(bal, w)
    assert np.all(np.isfinite(a)) and np.any(a != 0)
    assert np.array_equal(a.view(np.uint64), b.view(np.uint64))


def test_a_broken_layering_is_caught_by_the_float_run():
    """The float run is sensitive to a dependency broken by a layering: moving
    one f_2 job a layer earlier (beside the f_1 it reads) changes the result."""
    w = W.p1(m=1, d=8)
    asap = mdpe.Plan.for_workload(w, device=-1, flags=mdpe.MDPE_ASAP_LAYERS)
    ref = _run_float(asap, w)

    class Moved:
        info = asap.info

        def conv_jobs(self):
            jobs = asap.conv_jobs().copy()
            q = int(np.flatnonzero(jobs[:, 0] == 2)[0])
            jobs[q, 0] = 1
            return jobs

        def __getattr__(self, k):
            return getattr(asap, k)

    assert not np.array_equal(_run_float(Moved(), w), ref)


def test_small_layers_keep_the_earliest_layering():
    for w in (W.rand3(), W.p2(), W.p3(m=2)):
        asap, bal = _plans(w)
        assert bal.info["balanced_layers"] == 0
        assert np.array_equal(asap.conv_jobs(), bal.conv_jobs())

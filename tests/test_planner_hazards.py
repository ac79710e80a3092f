"""The planner's hazard checker rejects bad job lists (host only, no GPU).

Section 5 runs the jobs of one layer at once, so they must be independent:
no job may read or write a slot that another job of its layer writes, and a
job may read only what an earlier layer (or the staging) wrote.  The kernel
adds two rules of its own: a convolution never writes its second operand
(streamed while outputs are stored), nor its first when operands are
streamed or when one job is spread over several wavefronts (each wavefront
stages the first operand by itself, and the wavefronts of a job need not
share a workgroup, so one could store before another has read).

check_plan_jobs runs the checker plan_polynomial runs on every plan; the
tests feed it the rows of real plans, then the same rows with one planted
fault each.
"""
import numpy as np
import pytest

from paper_2101_10881_amd import mdpe
from paper_2101_10881_amd import workloads as W
from test_planner import _execute_exact

import exact_ref as E


def _rows(p):
    return p.conv_jobs().copy(), p.add_jobs().copy(), p.outputs().copy()


def _check(w, p, conv, add, out, extra_slots=0, **kw):
    mdpe.check_plan_jobs(w.n, w.N, p.info["n_series"] + extra_slots, conv, add, out, **kw)


def _rejected(w, p, conv, add, out, words, extra_slots=0, **kw):
    with pytest.raises(mdpe.MdpeError) as e:
        _check(w, p, conv, add, out, extra_slots, **kw)
    assert e.value.code == mdpe.MDPE_EINVAL
    msg = str(e.value)
    assert all(x in msg for x in words), msg
    return msg


def _sorted(conv):
    return conv[np.argsort(conv[:, 0], kind="stable")]


# multilinear polynomials whose monomials have at least two variables (no
# staged derivative copies), several layers deep
CASES = [
    ("worked_example", lambda: W.make("ex", 2, 3, 6, [(0, 2, 5), (0, 1, 4, 5), (1, 2, 3)], seed=4)),
    ("p1_small", lambda: W.make("p1s", 2, 4, 8, W.all_subsets(8, 4), seed=1)),
    ("p2_shape", lambda: W.p2(m=2, d=8)),
    ("rand3", lambda: W.rand3()),
]


@pytest.mark.parametrize("name,build", CASES, ids=[c[0] for c in CASES])
def test_real_plans_pass(name, build):
    w = build()
    for flags in (0, mdpe.MDPE_ASAP_LAYERS, mdpe.MDPE_STREAM_OPERANDS):
        p = mdpe.Plan.for_workload(w, device=-1, flags=flags)
        conv, add, out = _rows(p)
        _check(w, p, conv, add, out, waves_per_job=p.info["waves_per_job"], streamed=p.info["streamed"])


def _dependent_pair(conv):
    """A job of layer L+1 that reads a slot written in layer L."""
    writer = {}
    for q, (L, t1, t2, t3) in enumerate(conv):
        writer.setdefault(int(t3), []).append((int(L), q))
    for q, (L, t1, t2, t3) in enumerate(conv):
        for s in (int(t1), int(t2)):
            for Lw, qw in writer.get(s, []):
                if Lw == L - 1 and qw != q:
                    return q, qw
    raise AssertionError("no dependent pair")


@pytest.mark.parametrize("name,build", CASES, ids=[c[0] for c in CASES])
def test_read_after_write_in_one_layer_is_rejected(name, build):
    w = build()
    p = mdpe.Plan.for_workload(w, device=-1, flags=mdpe.MDPE_ASAP_LAYERS)
    conv, add, out = _rows(p)
    q, qw = _dependent_pair(conv)
    conv[q, 0] = conv[qw, 0]          # the reader joins its producer's layer
    _rejected(w, p, _sorted(conv), add, out, ["conv layer", "written in the same stage"])


@pytest.mark.parametrize("name,build", CASES, ids=[c[0] for c in CASES])
def test_read_before_write_is_rejected(name, build):
    w = build()
    p = mdpe.Plan.for_workload(w, device=-1, flags=mdpe.MDPE_ASAP_LAYERS)
    conv, add, out = _rows(p)
    q, qw = _dependent_pair(conv)
    conv[qw, 0] = conv[q, 0] + 1      # the producer now runs after its reader
    _rejected(w, p, _sorted(conv), add, out, ["conv layer", "read before write"])


@pytest.mark.parametrize("name,build", CASES, ids=[c[0] for c in CASES])
def test_two_writers_of_one_slot_are_rejected(name, build):
    w = build()
    p = mdpe.Plan.for_workload(w, device=-1, flags=mdpe.MDPE_ASAP_LAYERS)
    conv, add, out = _rows(p)
    first = conv[conv[:, 0] == 1]
    assert len(first) >= 2
    i0, i1 = np.flatnonzero(conv[:, 0] == 1)[:2]
    conv[i1, 3] = conv[i0, 3]
    _rejected(w, p, conv, add, out, ["conv layer 1", "two jobs write one slot"])


@pytest.mark.parametrize("name,build", CASES, ids=[c[0] for c in CASES])
def test_second_operand_as_output_is_rejected(name, build):
    w = build()
    p = mdpe.Plan.for_workload(w, device=-1)
    conv, add, out = _rows(p)
    conv[len(conv) // 2, 2] = conv[len(conv) // 2, 3]    # t2 = t3
    _rejected(w, p, conv, add, out, ["second operand is the output"])


def test_in_place_job_needs_one_wavefront_and_staged_operands():
    # b_{n-2} := b_{n-2} * a_k (Section 3) is in place on staged plans with one
    # wavefront per job; the same rows fail for a job over several wavefronts
    # and for streamed operands
    w = W.make("p1s", 4, 6, 8, W.all_subsets(8, 4), seed=1)
    p = mdpe.Plan.for_workload(w, device=-1, flags=mdpe.MDPE_LAYER_LAUNCHES)
    conv, add, out = _rows(p)
    assert p.info["waves_per_job"] == 1 and not p.info["streamed"]
    assert (conv[:, 1] == conv[:, 3]).sum() == w.N
    _check(w, p, conv, add, out)
    _rejected(w, p, conv, add, out, ["first operand is the output"], waves_per_job=2)
    _rejected(w, p, conv, add, out, ["first operand is the output"], streamed=True)


def test_addition_reading_a_sum_of_its_own_level_is_rejected():
    w = W.rand3()
    p = mdpe.Plan.for_workload(w, device=-1)
    conv, add, out = _rows(p)
    assert (add[:, 0] == 1).sum() >= 2
    add[1, 1] = add[0, 2]             # reads what job 0 of level 1 is updating
    _rejected(w, p, conv, add, out, ["add level 1", "written in the same stage"])


def test_addition_reading_an_unwritten_slot_is_rejected():
    w = W.rand3()
    p = mdpe.Plan.for_workload(w, device=-1)
    conv, add, out = _rows(p)
    add[0, 1] = p.info["n_series"]    # one slot more than the plan uses: never written
    _rejected(w, p, conv, add, out, ["add level 1", "read before write"], extra_slots=1)


def test_unwritten_output_slot_is_rejected():
    w = W.rand3()
    p = mdpe.Plan.for_workload(w, device=-1)
    conv, add, out = _rows(p)
    _check(w, p, conv, add, out, extra_slots=1)
    out[0] = p.info["n_series"]
    _rejected(w, p, conv, add, out, ["output slot never written"], extra_slots=1)


def test_layers_must_not_decrease():
    w = W.rand3()
    p = mdpe.Plan.for_workload(w, device=-1, flags=mdpe.MDPE_ASAP_LAYERS)
    conv, add, out = _rows(p)
    _rejected(w, p, conv[::-1].copy(), add, out, ["layers must start at 1 and not decrease"])


# ------------------------------------------- jobs over several wavefronts --

@pytest.mark.parametrize("build,m,d", [(W.p2, 1, 152), (W.p2, 2, 95), (W.p2, 4, 152), (W.p2, 10, 152)])
def test_multiwave_staged_plans_have_no_in_place_job(build, m, d):
    """A staged plan that spreads a job over several wavefronts gives the
    in-place multiplications fresh output slots (as streamed plans do)."""
    w = build(m=m, d=d)
    p = mdpe.Plan.for_workload(w, device=-1, flags=mdpe.MDPE_NO_CHAIN_LAUNCH)
    assert p.info["waves_per_job"] > 1 and not p.info["streamed"]
    conv, add, out = _rows(p)
    assert not (conv[:, 1] == conv[:, 3]).any()
    _check(w, p, conv, add, out, waves_per_job=p.info["waves_per_job"])
    # one more slot per monomial of at least three variables
    base = mdpe.Plan.for_workload(w, device=-1, flags=mdpe.MDPE_STREAM_OPERANDS)
    assert p.info["n_series"] == base.info["n_series"]


def test_multiwave_plan_of_many_long_monomials():
    # 40 monomials of 32 variables at two doubles, d = 152: three wavefronts per job
    rng = np.random.default_rng(5)
    w = W.make("long32", 2, 152, 32, W.random_supports(rng, 32, 40, [32] * 40), seed=1)
    p = mdpe.Plan.for_workload(w, device=-1)
    assert p.info["waves_per_job"] == 3
    conv, add, out = _rows(p)
    assert not (conv[:, 1] == conv[:, 3]).any()


@pytest.mark.parametrize("m,d,keep", [(1, 140, False), (1, 127, True), (4, 140, True)])
def test_multiwave_plan_jobs_compute_the_definition(m, d, keep):
    """The fresh slots are wired through: the plan's jobs, run in exact
    arithmetic, give the exact value and gradient."""
    w = W.random_poly("mw", m, d, 6, 2, [4, 3], 1)
    flags = mdpe.MDPE_LAYER_LAUNCHES | (mdpe.MDPE_KEEP_MONOMIAL_VALUES if keep else 0)
    p = mdpe.Plan.for_workload(w, device=-1, flags=flags)
    assert p.info["waves_per_job"] > 1
    val, grad = _execute_exact(p, w)
    (ev, eg), _ = E.workload_exact(w)
    assert val == ev and grad == eg

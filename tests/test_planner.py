"""Planner pins (host only, no GPU): the data staging of Section 5.

* The worked example of Section 4 / Fig. 1: 21 convolutions in layers of
  6, 9, 5, 1; 28 series; the triplet of f_{1,1} and the pair a_0 -> f_{1,3};
  addition levels 6, 1.
* The launch sizes and job counts printed for p1, p2 and p3 (Section 6.1,
  Table 2).
* eq. (6) for the slot count, 3 n_k - 3 convolutions per monomial,
  Corollary 2's depth.
* Executing the plan's jobs on exact rational series reproduces the exact
  value and gradient (the jobs compute what the paper defines).
* Invalid descriptions are rejected with the right status.
"""
import json
import os
from fractions import Fraction

import numpy as np
import pytest

import exact_ref as E
from paper_2101_10881_amd import mdpe
from paper_2101_10881_amd import workloads as W

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _plan(n, supports, d=3, m=2):
    nvars = [len(s) for s in supports]
    vars_ = [v for s in supports for v in s]
    return mdpe.Plan(n, nvars, vars_, d, m, device=-1)


def test_worked_example():
    g = json.load(open(os.path.join(GOLD, "worked_example.json")))
    sup = [tuple(v - 1 for v in s) for s in g["supports_1based"]]
    p = _plan(g["n"], sup)
    conv, add = p.layer_sizes()
    assert p.info["n_conv"] == g["n_conv"]
    assert conv == g["conv_layer_sizes"]
    assert add == g["add_level_sizes"]
    assert p.info["n_series"] == g["n_series"]
    jobs = p.conv_jobs()
    assert list(jobs[0][1:]) == g["triplet_f11_in_units_of_d_plus_1"] and jobs[0][0] == 1
    adds = p.add_jobs()
    assert list(adds[0][1:]) == g["pair_a0_into_f13_in_units_of_d_plus_1"]
    # value tree: f13 := a0 + f13, f33 := f24 + f33 (level 1), then f33 := f33 + f13 (level 2)
    slot = {"a0": 0, "f13": 12, "f24": 16, "f33": 19}
    want = [(1, slot[a], slot[b]) for a, b in g["value_tree"][:2]] + [(2, slot["f13"], slot["f33"])]
    got = [tuple(r) for r in adds if r[2] in (slot["f13"], slot["f33"])]
    assert got == want
    assert p.outputs()[0] == slot["f33"]


def test_p1_counts():
    g = json.load(open(os.path.join(GOLD, "paper_counts.json")))["p1"]
    # the paper's launch sizes are those of the earliest-layer layering
    p = mdpe.Plan.for_workload(W.p1(), device=-1, flags=mdpe.MDPE_ASAP_LAYERS)
    conv, add = p.layer_sizes()
    assert p.info["n_conv"] == g["n_conv"] and p.info["n_add"] == g["n_add"]
    assert conv == g["conv_launches"] and add == g["add_launches"]


def test_p2_counts():
    g = json.load(open(os.path.join(GOLD, "paper_counts.json")))["p2"]
    # the layered plan (the chain launch, chosen for p2 by default, relayers the cross products)
    p = mdpe.Plan.for_workload(W.p2(), device=-1, flags=mdpe.MDPE_NO_CHAIN_LAUNCH)
    conv, add = p.layer_sizes()
    assert p.info["n_conv"] == g["n_conv"] and p.info["n_add"] == g["n_add"]
    assert conv[:31] == [g["first_31_conv_launches"]] * 31
    assert p.info["n_layers"] == 64


def test_p3_additions():
    g = json.load(open(os.path.join(GOLD, "paper_counts.json")))["p3"]
    sup = W.all_subsets(128, 2)
    assert len(sup) == g["N"]
    p = _plan(128, sup, d=0, m=1)
    assert p.info["n_add"] == g["n_add"]
    assert p.info["n_conv"] == 3 * g["N"]


def test_flop_convention_of_the_paper():
    g = json.load(open(os.path.join(GOLD, "paper_counts.json")))["flops_p1_deca_d152"]
    from paper_2101_10881_amd import flops
    d = g["d"]
    assert 16380 * (d + 1) ** 2 * g["deca_mul_ops"] == g["mul_part"]
    assert (16380 * d * (d + 1) + 9084 * (d + 1)) * g["deca_add_ops"] == g["add_part"]
    assert flops.paper_convention(16380, 9084, d) == g["total"]


@pytest.mark.parametrize("seed", range(8))
def test_counts_eq6_and_corollary2(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(1, 12))
    N = int(rng.integers(0, 30))
    nk = rng.integers(1, n + 1, size=N)
    sup = W.random_supports(rng, n, N, nk)
    p = _plan(n, sup, d=int(rng.integers(0, 20)), m=int(rng.choice(W.SUPPORTED_M)))
    i = p.info
    assert i["n_series"] == 1 + N + n + sum(k + max(1, k - 2) + max(0, k - 2) for k in nk)
    assert i["n_conv"] == sum(3 * k - 3 if k >= 2 else 1 for k in nk)
    assert i["n_layers"] == (max(nk) if N else 0)
    lists = [N + 1] + [sum(1 for s in sup if v in s) for v in range(n)]
    levels = max(int(np.ceil(np.log2(L))) if L > 1 else 0 for L in lists)
    assert i["n_levels"] == levels
    assert i["n_add"] == sum(max(L - 1, 0) for L in lists)
    out = p.outputs()
    for v in range(n):
        assert (out[1 + v] == -1) == (lists[1 + v] == 0)


def _execute_exact(p, w):
    """Run the plan's jobs on exact rational series (slots hold lists of Fractions)."""
    d = w.d
    A = [None] * p.info["n_series"]
    a = E.planar_to_exact(w.coeff)
    z = E.planar_to_exact(w.z)
    for s in range(w.N + 1):
        A[s] = a[s]
    for i in range(w.n):
        A[w.N + 1 + i] = z[i]
    for k, nk in enumerate(w.nvars):   # n_k = 1: the derivative a_k, staged into its backward slot
        if nk == 1:
            base = 1 + w.N + w.n + int(sum(w.nvars)) + int(sum(max(1, int(q) - 2) for q in w.nvars[:k]))
            A[base] = a[k + 1]
    for layer, t1, t2, t3 in p.conv_jobs():
        A[t3] = E.smul(A[t1], A[t2])
    for src, dst, e in p.scale_jobs():
        A[dst] = [c * int(e) for c in A[src]]
    for level, t1, t2 in p.add_jobs():
        A[t2] = E.sadd(A[t2], A[t1])
    out = p.outputs()
    val = A[out[0]]
    grad = [A[s] if s >= 0 else [Fraction(0)] * (d + 1) for s in out[1:]]
    return val, grad


@pytest.mark.parametrize("seed", range(6))
def test_plan_jobs_compute_the_definition(seed):
    rng = np.random.default_rng(40 + seed)
    n = int(rng.integers(1, 8))
    N = int(rng.integers(0, 8))
    w = W.random_poly("plan", 1, 2, n, N, rng.integers(1, n + 1, size=N), seed)
    p = mdpe.Plan.for_workload(w, device=-1)
    val, grad = _execute_exact(p, w)
    (ev, eg), _ = E.workload_exact(w)
    assert val == ev
    assert grad == eg


def test_worked_example_jobs_compute_the_definition():
    w = W.make("ex", 1, 3, 6, [(0, 2, 5), (0, 1, 4, 5), (1, 2, 3)], seed=4)
    val, grad = _execute_exact(mdpe.Plan.for_workload(w, device=-1), w)
    (ev, eg), _ = E.workload_exact(w)
    assert val == ev and grad == eg


@pytest.mark.parametrize("build", [W.rand3, W.p1, W.p2, lambda: W.p1(m=8, d=32)],
                         ids=["rand3_2d_d8", "p1_10d_d152", "p2_4d_d64", "p1_8d_d32"])
def test_lane_schedule_is_balanced(build):
    w = build()
    i = mdpe.Plan.for_workload(w, device=-1).info
    J, d = i["jobs_per_group"], w.d
    total = J * (d + 1) * (d + 2) // 2
    assert i["lane_steps"] >= max(d + 1, -(-total // 64))
    assert i["lane_steps"] <= max(d + 1, -(-total // 64)) + 1


@pytest.mark.parametrize("bad, code", [
    (dict(n=0), mdpe.MDPE_EINVAL),
    (dict(nvars=[0]), mdpe.MDPE_EINVAL),
    (dict(nvars=[4], vars_=[0, 1, 2, 4]), mdpe.MDPE_EINVAL),       # variable out of range
    (dict(nvars=[2], vars_=[1, 1]), mdpe.MDPE_EINVAL),             # not strictly increasing
    (dict(nvars=[2], vars_=[2, 1]), mdpe.MDPE_EINVAL),
    (dict(d=-1), mdpe.MDPE_EINVAL),
    (dict(m=6), mdpe.MDPE_EUNSUPPORTED),
    (dict(m=10, d=65535), mdpe.MDPE_EUNSUPPORTED),                 # beyond the 16-bit coefficient index
])
def test_invalid_descriptions(bad, code):
    args = dict(n=4, nvars=[2], vars_=[0, 1], d=3, m=2)
    args.update(bad)
    with pytest.raises(mdpe.MdpeError) as e:
        mdpe.Plan(args["n"], args["nvars"], args["vars_"], args["d"], args["m"], device=-1)
    assert e.value.code == code
    assert mdpe.last_error_string()


@pytest.mark.parametrize("seed", range(5))
def test_keep_monomials_plan_computes_the_adjoint(seed):
    """With MDPE_KEEP_MONOMIAL_VALUES the forward jobs still compute the value and
    gradient, and the reverse jobs, run in exact arithmetic, give the adjoints."""
    rng = np.random.default_rng(90 + seed)
    n = int(rng.integers(1, 7))
    N = int(rng.integers(0, 7))
    nk = rng.integers(1, n + 1, size=N)
    w = W.random_poly("keep", 1, 2, n, N, nk, seed)
    p = mdpe.Plan.for_workload(w, device=-1, flags=mdpe.MDPE_KEEP_MONOMIAL_VALUES)
    p0 = mdpe.Plan.for_workload(w, device=-1)
    assert p.info["n_conv"] == p0.info["n_conv"] + int(np.sum(nk >= 2))
    assert p.info["n_layers"] == p0.info["n_layers"]
    present = len(set(int(v) for v in w.vars))
    assert p.info["n_reverse"] == N + present
    # exact execution: forward jobs, then the reverse correlations
    d = w.d
    A = [None] * p.info["n_series"]
    a = E.planar_to_exact(w.coeff)
    z = E.planar_to_exact(w.z)
    for s_ in range(N + 1):
        A[s_] = a[s_]
    for i in range(n):
        A[N + 1 + i] = z[i]
    for k, q in enumerate(w.nvars):
        if q == 1:
            base = 1 + N + n + int(sum(w.nvars)) + int(sum(max(1, int(r) - 2) for r in w.nvars[:k]))
            A[base] = a[k + 1]
    for layer, t1, t2, t3 in p.conv_jobs():
        A[t3] = E.smul(A[t1], A[t2])
    for level, t1, t2 in p.add_jobs():
        A[t2] = E.sadd(A[t2], A[t1])
    ybar = [Fraction(int(v)) for v in rng.integers(-3, 4, size=d + 1)]
    rj = p.reverse_jobs()
    A[rj[0][0] if len(rj) else 0] = ybar
    corr = lambda x, y: [sum((x[s + j] * y[j] for j in range(d + 1 - s)), Fraction(0)) for s in range(d + 1)]
    for t1, t2, t3 in rj:
        A[t3] = corr(A[t1], A[t2])
    (ev, eg), _ = E.workload_exact(w)
    sup = w.supports()
    outs = {tuple(r[1:]) for r in rj}
    for k, s_ in enumerate(sup):
        M = [Fraction(1)] + [Fraction(0)] * d
        for v in s_:
            M = E.smul(M, z[v])
        assert any(A[t3] == corr(ybar, M) for (t2, t3) in outs), f"abar_{k + 1}"
    for i in range(n):
        if any(i in s_ for s_ in sup):
            assert any(A[t3] == corr(ybar, eg[i]) for (t2, t3) in outs), f"zbar_{i}"


def test_complex_plan_same_jobs_double_workspace():
    w = W.random_poly("cx", 3, 9, 7, 11, [1, 2, 3, 4, 5, 3, 2, 6, 7, 2, 3], seed=4)
    p = mdpe.Plan.for_workload(w, device=-1)
    pc = mdpe.Plan.for_workload(w, device=-1, flags=mdpe.MDPE_COMPLEX)
    assert pc.info["flags"] == mdpe.MDPE_COMPLEX
    assert pc.info["workspace_bytes"] == 2 * p.info["workspace_bytes"]
    assert np.array_equal(pc.conv_jobs(), p.conv_jobs())
    assert np.array_equal(pc.add_jobs(), p.add_jobs())
    assert np.array_equal(pc.outputs(), p.outputs())


@pytest.mark.parametrize("flags, m, d, code", [
    (mdpe.MDPE_COMPLEX | mdpe.MDPE_KEEP_MONOMIAL_VALUES, 2, 3, mdpe.MDPE_EUNSUPPORTED),  # no complex reverse pass
    (1024, 2, 3, mdpe.MDPE_EINVAL),                          # unknown flag
    (mdpe.MDPE_SINGLE_LAUNCH | mdpe.MDPE_LAYER_LAUNCHES, 2, 3, mdpe.MDPE_EINVAL),
    (mdpe.MDPE_SINGLE_LAUNCH | mdpe.MDPE_CHAIN_LAUNCH, 2, 3, mdpe.MDPE_EINVAL),
    (mdpe.MDPE_CHAIN_LAUNCH | mdpe.MDPE_NO_CHAIN_LAUNCH, 2, 3, mdpe.MDPE_EINVAL),
    (mdpe.MDPE_CHAIN_LAUNCH | mdpe.MDPE_FUSED_LAYERS, 2, 3, mdpe.MDPE_EINVAL),
    (mdpe.MDPE_CHAIN_LAUNCH | mdpe.MDPE_STREAM_OPERANDS, 2, 3, mdpe.MDPE_EINVAL),
    (mdpe.MDPE_STREAM_OPERANDS | mdpe.MDPE_STAGE_OPERANDS, 2, 3, mdpe.MDPE_EINVAL),
    (mdpe.MDPE_STAGE_OPERANDS, 10, 1700, mdpe.MDPE_EUNSUPPORTED),  # does not fit in LDS
])
def test_complex_plan_limits(flags, m, d, code):
    with pytest.raises(mdpe.MdpeError) as e:
        mdpe.Plan(4, [2], [0, 1], d, m, device=-1, flags=flags)
    assert e.value.code == code
    many = dict(nvars=[2] * 5000, vars_=[0, 1] * 5000)      # layers big enough that staging pays
    assert not mdpe.Plan(4, many["nvars"], many["vars_"], 818, 10, device=-1, flags=mdpe.MDPE_COMPLEX).info["streamed"]
    assert mdpe.Plan(4, many["nvars"], many["vars_"], 819, 10, device=-1, flags=mdpe.MDPE_COMPLEX).info["streamed"]
    assert not mdpe.Plan(4, many["nvars"], many["vars_"], 819, 10, device=-1).info["streamed"]   # real: staged


@pytest.mark.parametrize("seed", range(6))
def test_plan_jobs_with_exponents_compute_the_definition(seed):
    """Power table, common factors and exponent scale jobs, run in exact
    arithmetic, give the value and gradient of sum_k a_k prod z^e."""
    rng = np.random.default_rng(140 + seed)
    n = int(rng.integers(1, 7))
    N = int(rng.integers(1, 7))
    w = W.with_exponents(W.random_poly("plan_e", 1, 3, n, N, rng.integers(1, n + 1, size=N), seed), 5, seed=seed)
    p = mdpe.Plan.for_workload(w, device=-1)
    assert p.info["n_scale"] == int(np.sum(w.exps >= 2))
    val, grad = _execute_exact(p, w)
    (ev, eg), _ = E.workload_exact(w)
    assert val == ev
    assert grad == eg


def test_unit_exponents_give_the_multilinear_plan():
    w = W.random_poly("ones", 2, 4, 6, 9, [1, 2, 3, 4, 5, 3, 2, 6, 3], seed=5)
    p0 = mdpe.Plan.for_workload(w, device=-1)
    w.exps = np.ones_like(w.vars)
    p1 = mdpe.Plan.for_workload(w, device=-1)
    assert p1.info == p0.info
    assert np.array_equal(p1.conv_jobs(), p0.conv_jobs()) and np.array_equal(p1.add_jobs(), p0.add_jobs())


def test_exponent_layers():
    # x0^3 x1 * a: the power z0^2 at layer 1, the common factor a z0^2 at layer 2,
    # then the monomial's two layers
    w = W.make("layers", 1, 2, 2, [(0, 1)], seed=1)
    w.exps = np.array([3, 1], dtype=np.int32)
    p = mdpe.Plan.for_workload(w, device=-1)
    assert p.layer_sizes()[0] == [1, 1, 2, 1]
    assert [tuple(r) for r in p.scale_jobs()] == [(p.outputs()[1], p.outputs()[1], 3)]


@pytest.mark.parametrize("exps, flags, code", [
    ([1, 0], 0, mdpe.MDPE_EINVAL),
    ([65, 1], 0, mdpe.MDPE_EINVAL),
    ([2, 1], mdpe.MDPE_KEEP_MONOMIAL_VALUES, mdpe.MDPE_EUNSUPPORTED),
])
def test_exponent_limits(exps, flags, code):
    with pytest.raises(mdpe.MdpeError) as e:
        mdpe.Plan(4, [2], [0, 1], 3, 2, device=-1, flags=flags, exps=exps)
    assert e.value.code == code
    mdpe.Plan(4, [2], [0, 1], 3, 2, device=-1, flags=mdpe.MDPE_KEEP_MONOMIAL_VALUES, exps=[1, 1])


@pytest.mark.parametrize("m,d,flags", [(10, 1637, 0), (10, 818, mdpe.MDPE_COMPLEX), (1, 8191, 0), (2, 4095, 0)])
def test_largest_staged_degrees(m, d, flags):
    # the largest d with operands staged in LDS (for layers big enough that
    # staging pays); one more must stream them
    nv, vs = [2] * 5000, [0, 1] * 5000
    p = mdpe.Plan(3, nv, vs, d, m, device=-1, flags=flags)
    q = mdpe.Plan(3, nv, vs, d + 1, m, device=-1, flags=flags)
    assert not p.info["streamed"] and q.info["streamed"]
    pairs = (d + 3) // 2                                  # coefficients k, d-k of degree d+1
    want = -(-pairs // 64) if d + 2 > 4096 else max(1, pairs // 64)
    assert q.info["waves_per_job"] == want


def test_degree_limit():
    p = mdpe.Plan(2, [2], [0, 1], 65534, 1, device=-1)
    assert p.info["streamed"] and p.info["waves_per_job"] == (65536 // 2 + 63) // 64
    assert p.info["lane_steps"] == 65536                 # one pair (k, d-k) per lane: d + 2 terms
    with pytest.raises(mdpe.MdpeError) as e:
        mdpe.Plan(2, [2], [0, 1], 65535, 1, device=-1)
    assert e.value.code == mdpe.MDPE_EUNSUPPORTED


def _streamed_slots_are_fresh(p):
    rows = p.conv_jobs()
    return all(t1 != t3 for _, t1, t2, t3 in rows)


@pytest.mark.parametrize("seed", range(6))
def test_streamed_plan_jobs_compute_the_definition(seed):
    """Streamed operands: no convolution writes its first operand, and the jobs,
    run in exact arithmetic, still give the value and gradient (with exponents)."""
    rng = np.random.default_rng(240 + seed)
    n = int(rng.integers(1, 7))
    N = int(rng.integers(1, 7))
    w = W.random_poly("stream", 1, 3, n, N, rng.integers(1, n + 1, size=N), seed)
    if seed % 2:
        w = W.with_exponents(w, 4, seed=seed)
    p = mdpe.Plan.for_workload(w, device=-1, flags=mdpe.MDPE_STREAM_OPERANDS)
    p0 = mdpe.Plan.for_workload(w, device=-1)
    assert p.info["streamed"] and not p0.info["streamed"]
    assert _streamed_slots_are_fresh(p)
    assert p.info["n_conv"] == p0.info["n_conv"] and p.info["n_layers"] == p0.info["n_layers"]
    val, grad = _execute_exact(p, w)
    (ev, eg), _ = E.workload_exact(w)
    assert val == ev and grad == eg


def test_streamed_keep_monomials_plan():
    w = W.random_poly("stream_keep", 1, 2, 6, 7, [1, 2, 3, 4, 5, 6, 3], seed=3)
    p = mdpe.Plan.for_workload(w, device=-1, flags=mdpe.MDPE_STREAM_OPERANDS | mdpe.MDPE_KEEP_MONOMIAL_VALUES)
    assert _streamed_slots_are_fresh(p)
    assert p.info["n_reverse"] == mdpe.Plan.for_workload(w, device=-1, flags=mdpe.MDPE_KEEP_MONOMIAL_VALUES).info["n_reverse"]


def test_streaming_chosen_by_cost():
    # few jobs per layer at a large degree: several wavefronts per job pay
    big = W.make("big", 4, 4000, 8, W.all_subsets(8, 4), seed=1)
    p = mdpe.Plan.for_workload(big, device=-1)
    assert p.info["streamed"] and p.info["waves_per_job"] == 31
    # c1: thousands of jobs per layer, staged
    assert not mdpe.Plan.for_workload(W.p1(), device=-1).info["streamed"]


@pytest.mark.parametrize("build,m,d,simple", [(W.p2, 1, 152, 1), (W.p2, 2, 152, 1), (W.p1, 2, 64, 0),
                                              (W.p2, 4, 152, 0), (W.p1, 10, 152, 0)])
def test_simple_dealing_choice(build, m, d, simple):
    # coefficients of at most two doubles are dealt to lanes in turn where the
    # planner estimates it faster than the lane schedule; never for more
    flags = mdpe.MDPE_NO_CHAIN_LAUNCH
    assert mdpe.Plan.for_workload(build(m=m, d=d), device=-1, flags=flags).info["simple_dealing"] == simple


@pytest.mark.parametrize("build,m,d,J,Q", [(W.p1, 10, 152, 1, 1), (W.p2, 4, 64, 2, 1),
                                           (W.p2, 10, 152, 1, 2), (W.p2, 4, 152, 1, 2),
                                           (W.p2, 1, 152, 1, 2), (W.p2, 2, 95, 1, 2),
                                           (W.p1, 2, 152, 1, 1)])
def test_jobs_and_wavefronts_per_group(build, m, d, J, Q):
    # layers with fewer wavefronts than SIMDs (p2's 378 jobs) spread a job over
    # two wavefronts, down to the longest coefficient's d+1 steps; at one or two
    # doubles per coefficient by dealing the coefficients over them
    i = mdpe.Plan.for_workload(build(m=m, d=d), device=-1, flags=mdpe.MDPE_NO_CHAIN_LAUNCH).info
    assert (i["jobs_per_group"], i["waves_per_job"]) == (J, Q)
    if Q > 1:
        assert i["lane_steps"] == d + 1


def test_single_launch_for_tiny_plans_only():
    """Plans whose ~10 dependent launches would cost more than their work run
    in one workgroup's launch: 16 monomials of 3 of 8 variables at d = 8 do,
    p1, p2, p3 and the mixed batch's instances do not; the flag forces it,
    and the per-layer flag excludes it."""
    info = lambda w, f=0: mdpe.Plan.for_workload(w, device=-1, flags=f).info
    i = info(W.rand3())
    assert i["single_launch"] == 1 and i["single_waves"] in (4, 8, 16)
    for w in (W.p1(m=2, d=8), W.p2(m=1, d=8), W.p3(m=1, d=8), W.p1()):
        assert info(w)["single_launch"] == 0
    assert all(info(w)["single_launch"] == 0 for w in W.mixed_batch(64, seed=1))
    assert info(W.rand3(), mdpe.MDPE_LAYER_LAUNCHES)["single_launch"] == 0
    forced = info(W.p1(m=2, d=8), mdpe.MDPE_SINGLE_LAUNCH)
    assert forced["single_launch"] == 1 and forced["chain_layers"] == 0 and forced["fused_components"] == 0
    # the jobs and layers are the plan's own: the single launch only changes how they are launched
    a = mdpe.Plan.for_workload(W.rand3(), device=-1, flags=mdpe.MDPE_LAYER_LAUNCHES)
    b = mdpe.Plan.for_workload(W.rand3(), device=-1)
    assert np.array_equal(a.conv_jobs(), b.conv_jobs()) and np.array_equal(a.add_jobs(), b.add_jobs())

"""GPU parity: the HIP path against the CPU oracle, bit for bit.

Both sides implement the same multiple-double specification and the same
per-job operation order, so every limb must agree exactly (integer
comparison of the binary64 bit patterns, signed zeros included).  Cases
span several workgroup tiles and ragged tails: all seven precisions,
degrees 0..255, monomials with 1..12 variables, absent variables, N = 0,
the three test polynomial shapes at sweep points, and the benchmark
workloads at full size (c1 against a digest of the
oracle's output written by tests/golden/make_digests.py).
"""
import json
import os

import numpy as np
import pytest

from gpu_util import assert_bitexact, run_gpu, sha256
from paper_2101_10881_amd import workloads as W

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _say(msg):
    print(msg, flush=True)


@pytest.mark.parametrize("m", W.SUPPORTED_M)
@pytest.mark.parametrize("op", ["add", "mul"])
def test_md_elementwise_bitexact(oracle_lib, m, op):
    import torch
    from paper_2101_10881_amd import mdpe
    _say(f"md_elementwise m={m} op={op}")
    rng = np.random.default_rng(500 + m)
    count = 20011
    x = W.md_series(rng, count, m, 0)[:, :, 0]
    y = W.md_series(rng, count, m, 0)[:, :, 0] * np.ldexp(1.0, rng.integers(-6, 6, size=count))
    q = count // 10
    y[:, :q] = -x[:, :q]
    if m > 1:
        y[m - 1, :q] = x[m - 1, :q] * 0.25
    y[:, q:2 * q] = 0.0
    x, y = np.ascontiguousarray(x), np.ascontiguousarray(y)
    want = oracle_lib.md_op(op, x, y)
    dev = torch.device("cuda", 0)
    xt, yt = torch.from_numpy(x).to(dev), torch.from_numpy(y).to(dev)
    zt = torch.empty_like(xt)
    mdpe.md_elementwise(op, xt, yt, zt)
    torch.cuda.synchronize()
    assert_bitexact(zt.cpu().numpy(), want, f"md_{op} m={m}")


def _compare(oracle_lib, w):
    _say(f"eval_and_diff {w.name}: m={w.m} d={w.d} n={w.n} N={w.N}")
    want_v, want_g = oracle_lib.eval_workload(w)
    got_v, got_g = run_gpu(w)
    assert_bitexact(got_v, want_v, f"{w.name} value")
    assert_bitexact(got_g, want_g, f"{w.name} gradient")


@pytest.mark.parametrize("m", W.SUPPORTED_M)
def test_random_polynomials_bitexact(oracle_lib, m):
    for seed in range(3):
        rng = np.random.default_rng(7000 + 10 * m + seed)
        n = int(rng.integers(1, 14))
        N = int(rng.integers(1, 40))
        d = int(rng.choice([0, 1, 2, 5, 8, 17, 33]))
        nk = rng.integers(1, min(n, 12) + 1, size=N)
        _compare(oracle_lib, W.random_poly(f"rand_m{m}_s{seed}", m, d, n, N, nk, seed))


@pytest.mark.parametrize("d", [0, 1, 7, 31, 63, 64, 65, 100, 152, 200, 255])
def test_degrees_span_tiles(oracle_lib, d):
    m = 2 if d > 100 else 3
    rng = np.random.default_rng(d)
    w = W.random_poly(f"deg{d}", m, d, 6, 7, rng.integers(1, 6, size=7), seed=d + 1)
    _compare(oracle_lib, w)


def test_many_jobs_ragged_groups(oracle_lib):
    # J jobs per workgroup with a partial last group in every layer
    w = W.random_poly("ragged", 4, 9, 12, 61, [5] * 61, seed=3)
    _compare(oracle_lib, w)


def test_edge_cases(oracle_lib):
    _compare(oracle_lib, W.make("no_monomials", 5, 6, 3, [], seed=2))
    _compare(oracle_lib, W.make("absent_vars", 4, 5, 9, [(1, 3), (3, 8), (1, 3, 8)], seed=5))
    _compare(oracle_lib, W.make("one_var", 10, 0, 1, [(0,), (0,)], seed=6))
    _compare(oracle_lib, W.make("all_vars", 2, 4, 10, [tuple(range(10)), (0, 9)], seed=7))
    _compare(oracle_lib, W.make("n_k_1_and_2", 3, 3, 4, [(0,), (1, 2), (3,), (0, 3)], seed=8))
    _compare(oracle_lib, W.make("worked_example", 10, 8, 6, [(0, 2, 5), (0, 1, 4, 5), (1, 2, 3)], seed=4))


def test_integer_inputs_exact(oracle_lib):
    rng = np.random.default_rng(9)
    w = W.random_poly("ints", 4, 6, 5, 9, rng.integers(1, 5, size=9), seed=9)
    w.coeff[:] = 0.0
    w.z[:] = 0.0
    w.coeff[0] = rng.integers(-3, 4, size=w.coeff.shape[1:])
    w.z[0] = rng.integers(-3, 4, size=w.z.shape[1:])
    _compare(oracle_lib, w)


def test_rand3_2d_d8_bitexact(oracle_lib):
    _compare(oracle_lib, W.rand3())


def test_p2_4d_d64_bitexact(oracle_lib):
    _compare(oracle_lib, W.p2())


def test_p1_8d_d32_forward_bitexact(oracle_lib):
    _compare(oracle_lib, W.p1(m=8, d=32))


def test_p3_shape_bitexact(oracle_lib):
    # all 8128 two-variable monomials of 128 variables (addition-heavy)
    _compare(oracle_lib, W.p3(m=3, d=8))


@pytest.mark.parametrize("poly,m,d", [("p1", 1, 191), ("p1", 5, 95), ("p2", 2, 31), ("p3", 8, 15), ("p1", 2, 64),
                                      ("p2", 2, 152), ("p2", 3, 152), ("p2", 1, 152), ("p2", 1, 191),
                                      ("p2", 1, 64), ("p2", 2, 66)])
def test_sweep_corners_bitexact(oracle_lib, poly, m, d):
    # points of the precision x degree sweep: other lane schedules (two jobs
    # per workgroup at d = 95; p2 at d >= 152 spreads each job over two
    # wavefronts, dealing the coefficients at m <= 2, and at d = 64 the second
    # wavefront deals a single coefficient) and precisions than the benchmark
    # configuration
    build = {"p1": W.p1, "p2": W.p2, "p3": W.p3}[poly]
    _compare(oracle_lib, build(m=m, d=d))


@pytest.mark.parametrize("m,d", [(2, 31), (2, 152), (3, 152), (2, 66), (4, 64)])
def test_p2_layered_plans_bitexact(oracle_lib, m, d):
    # p2 runs its chains of products in the chain launch by default; its
    # layered plan (two wavefronts per job at d >= 152, dealt coefficients at
    # two doubles) stays available and must give the same bits
    from paper_2101_10881_amd import mdpe
    import torch
    w = W.p2(m=m, d=d)
    P = mdpe.Polynomial.for_workload(w, torch.device("cuda", 0), chain_launch=False)
    assert P.plan.info["chain_layers"] == 0
    _say(f"layered p2 m={m} d={d}: fused={P.plan.info['fused_components'] > 0} "
         f"waves_per_job={P.plan.info['waves_per_job']}")
    want_v, want_g = oracle_lib.eval_workload(w)
    got_v, got_g = run_gpu(w, poly=P)
    assert_bitexact(got_v, want_v, "value")
    assert_bitexact(got_g, want_g, "gradient")


@pytest.mark.parametrize("case", ["p1_m2", "p1_exponents_m2", "p1_m3_d32", "p1_keep_m1"])
def test_balanced_layers_bitexact(oracle_lib, case):
    # p1's shape at these degrees plans with convolutions moved to later
    # layers to fill whole rounds of the SIMDs: the oracle's bits, and the
    # earliest-layer plan's bits
    import torch
    from paper_2101_10881_amd import mdpe
    w = {"p1_m2": lambda: W.p1(m=2), "p1_exponents_m2": lambda: W.with_exponents(W.p1(m=2), 3, seed=5),
         "p1_m3_d32": lambda: W.p1(m=3, d=32), "p1_keep_m1": lambda: W.p1(m=1)}[case]()
    keep = case.startswith("p1_keep")
    dev = torch.device("cuda", 0)
    bal = mdpe.Polynomial.for_workload(w, dev, keep_monomials=keep)
    asap = mdpe.Polynomial.for_workload(w, dev, keep_monomials=keep, asap_layers=True)
    assert bal.plan.info["balanced_layers"] == 1 and asap.plan.info["balanced_layers"] == 0
    _say(f"balanced layers {case}: {bal.plan.layer_sizes()[0]}")
    want_v, want_g = oracle_lib.eval_workload(w)
    for P in (bal, asap):
        got_v, got_g = run_gpu(w, poly=P)
        assert_bitexact(got_v, want_v, f"{case} value")
        assert_bitexact(got_g, want_g, f"{case} gradient")


@pytest.mark.parametrize("m,d,cx", [(10, 1637, False), (10, 818, True), (1, 8191, False), (2, 4095, False),
                                     (4, 2000, False)])
def test_maximum_degrees_bitexact(oracle_lib, m, d, cx):
    # the largest d whose convolution operands fit one workgroup's LDS (more
    # than 64 KB of it), staged there on request, for real and complex series
    # and both staging modes
    import torch
    from paper_2101_10881_amd import mdpe
    w = W.make(f"maxd_m{m}_d{d}", m, d, 3, [(0, 1), (0, 1, 2), (2,)], seed=3, cx=cx)
    P = mdpe.Polynomial.for_workload(w, torch.device("cuda", 0), stream_operands=False)
    assert not P.plan.info["streamed"]
    _say(f"eval_and_diff {w.name}: staged at the LDS limit")
    want_v, want_g = oracle_lib.eval_workload(w)
    got_v, got_g = run_gpu(w, poly=P)
    assert_bitexact(got_v, want_v, f"{w.name} value")
    assert_bitexact(got_g, want_g, f"{w.name} gradient")


def test_p1_10d_d152_full_size_digest():
    # full-size deca-double p1 at d = 152, in the launch configuration the benchmark times
    g = json.load(open(os.path.join(GOLD, "digests.json")))["workloads"]["p1_10d_d152"]
    w = W.p1()
    _say(f"eval_and_diff {w.name} (digest)")
    val, grad = run_gpu(w)
    assert [float(v).hex() for v in val[:, 0]] == g["value_head"]
    assert [float(v).hex() for v in grad[:, 0, 0]] == g["grad_head"]
    assert sha256(val) == g["value_sha256"]
    assert sha256(grad) == g["grad_sha256"]


def test_repeat_and_workspace_reuse(oracle_lib):
    import torch
    from paper_2101_10881_amd import mdpe
    w = W.random_poly("rep", 5, 20, 7, 15, [3] * 15, seed=12)
    P = mdpe.Polynomial.for_workload(w, torch.device("cuda", 0))
    a = run_gpu(w, poly=P)
    w2 = W.random_poly("rep2", 5, 20, 7, 15, [3] * 15, seed=13)   # same shape, other data, same workspace
    run_gpu(w2, poly=P)
    b = run_gpu(w, poly=P)
    assert_bitexact(a[0], b[0], "repeat value")
    assert_bitexact(a[1], b[1], "repeat grad")
    want_v, want_g = oracle_lib.eval_workload(w)
    assert_bitexact(b[0], want_v, "value")


def test_profiled_and_side_stream(oracle_lib):
    import torch
    from paper_2101_10881_amd import mdpe
    w = W.random_poly("prof", 8, 16, 6, 20, [4] * 20, seed=14)
    prof = mdpe.Profiler()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        got = run_gpu(w, profiler=prof)
    t = prof.read()
    assert t["n_cnv"] == 4 and t["n_stage"] == 1 and t["n_gather"] == 1
    assert t["cnv_ms"] > 0
    want_v, want_g = oracle_lib.eval_workload(w)
    assert_bitexact(got[0], want_v, "value")
    assert_bitexact(got[1], want_g, "grad")


@pytest.mark.parametrize("fused", [False, True])
def test_profiler_conv_launches_only(oracle_lib, fused):
    # timing only the convolution launches (five layers, or one fused launch):
    # the same outputs, no other events
    import torch
    from paper_2101_10881_amd import mdpe
    w = W.random_poly("profc", 4, 33, 7, 30, [5] * 30, seed=15)
    P = mdpe.Polynomial.for_workload(w, torch.device("cuda", 0), fused_layers=fused)
    prof = mdpe.Profiler(classes=mdpe.MDPE_TIME_CONV)
    got = run_gpu(w, profiler=prof, poly=P)
    t = prof.read()
    assert t["n_cnv"] == (1 if fused else 5) and t["n_stage"] == t["n_add"] == t["n_gather"] == 0 and t["cnv_ms"] > 0
    want_v, want_g = oracle_lib.eval_workload(w)
    assert_bitexact(got[0], want_v, "value")
    assert_bitexact(got[1], want_g, "grad")


def test_hip_graph_capture_and_replay(oracle_lib):
    # the plain path launches kernels only (no allocation, no memset, no
    # synchronisation), so a caller can capture it in a HIP graph; every
    # replay, with new inputs copied in and eager work in between, must match
    # the oracle bit for bit
    import torch
    from paper_2101_10881_amd import mdpe
    dev = torch.device("cuda", 0)
    w = W.random_poly("graph", 4, 20, 7, 25, np.random.default_rng(21).integers(1, 6, size=25), seed=21)
    P = mdpe.Polynomial.for_workload(w, dev)
    coeff = torch.from_numpy(w.coeff).to(dev)
    z = torch.from_numpy(w.z).to(dev)
    value = torch.empty((w.m, w.d + 1), dtype=torch.float64, device=dev)
    grad = torch.empty((w.m, w.n, w.d + 1), dtype=torch.float64, device=dev)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        P.eval_and_diff(coeff, z, value, grad)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        P.eval_and_diff(coeff, z, value, grad)
    other = W.random_poly("eager", 3, 9, 5, 8, [2] * 8, seed=4)
    for rep in range(4):
        _say(f"graph replay {rep}")
        rng = np.random.default_rng(600 + rep)
        w.coeff = W.md_series(rng, w.N + 1, w.m, w.d)
        w.z = W.md_series(rng, w.n, w.m, w.d)
        coeff.copy_(torch.from_numpy(w.coeff))
        z.copy_(torch.from_numpy(w.z))
        graph.replay()
        run_gpu(other)                       # eager work between replays
        torch.cuda.synchronize()
        want_v, want_g = oracle_lib.eval_workload(w)
        assert_bitexact(value.cpu().numpy(), want_v, f"replay {rep} value")
        assert_bitexact(grad.cpu().numpy(), want_g, f"replay {rep} gradient")


def test_repeated_calls_and_argument_checks(oracle_lib):
    # repeated calls on the same buffers skip the Python-side checks; new or
    # wrong tensors are still checked, and every call recomputes
    import torch
    from paper_2101_10881_amd import mdpe
    w = W.rand3()
    dev = torch.device("cuda", 0)
    P = mdpe.Polynomial.for_workload(w, dev)
    coeff = torch.from_numpy(w.coeff).to(dev)
    z = torch.from_numpy(w.z).to(dev)
    v, g = P.eval_and_diff(coeff, z)
    want_v, want_g = oracle_lib.eval_workload(w)
    for _ in range(3):
        v.fill_(0.0)
        P.eval_and_diff(coeff, z, v, g)
        torch.cuda.synchronize()
        assert_bitexact(v.cpu().numpy(), want_v, "value")
        assert_bitexact(g.cpu().numpy(), want_g, "gradient")
    with pytest.raises(ValueError):
        P.eval_and_diff(coeff[:, :-1].contiguous(), z, v, g)
    with pytest.raises(ValueError):
        P.eval_and_diff(coeff, z, v[:, :-1].contiguous(), g)
    P.eval_and_diff(coeff, z, v, g)
    torch.cuda.synchronize()
    assert_bitexact(v.cpu().numpy(), want_v, "value after the refused calls")

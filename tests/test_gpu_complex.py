"""GPU parity for complex series (MDPE_COMPLEX): the HIP path against the CPU
oracle, bit for bit.  Both sides implement the same complex product (four
m-double products, the real part adding the exactly negated xi*yi) and the
same per-job order, so every limb of both parts must agree exactly."""
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


def _compare(oracle_lib, w):
    assert w.cx
    _say(f"complex eval_and_diff {w.name}: m={w.m} d={w.d} n={w.n} N={w.N}")
    want_v, want_g = oracle_lib.eval_workload(w)
    got_v, got_g = run_gpu(w)
    assert got_v.shape == want_v.shape and got_g.shape == want_g.shape
    assert_bitexact(got_v, want_v, f"{w.name} value")
    assert_bitexact(got_g, want_g, f"{w.name} gradient")


@pytest.mark.parametrize("m", W.SUPPORTED_M)
@pytest.mark.parametrize("op", ["cadd", "cmul"])
def test_complex_md_elementwise_bitexact(oracle_lib, m, op):
    import torch
    from paper_2101_10881_amd import mdpe
    _say(f"md_elementwise m={m} op={op}")
    rng = np.random.default_rng(800 + m)
    count = 5003
    x = np.stack([W.md_series(rng, count, m, 0)[:, :, 0] for _ in range(2)])
    y = np.stack([W.md_series(rng, count, m, 0)[:, :, 0] for _ in range(2)])
    y[:, :, : count // 8] = -x[:, :, : count // 8]
    y[1, :, count // 8: count // 4] = 0.0
    x, y = np.ascontiguousarray(x), np.ascontiguousarray(y)
    want = oracle_lib.md_op(op, x, y)
    dev = torch.device("cuda", 0)
    xt, yt = torch.from_numpy(x).to(dev), torch.from_numpy(y).to(dev)
    zt = torch.empty_like(xt)
    mdpe.md_elementwise(op, xt, yt, zt)
    torch.cuda.synchronize()
    assert_bitexact(zt.cpu().numpy(), want, f"{op} m={m}")


@pytest.mark.parametrize("m", W.SUPPORTED_M)
def test_random_complex_polynomials_bitexact(oracle_lib, m):
    for seed in range(2):
        rng = np.random.default_rng(8100 + 10 * m + seed)
        n = int(rng.integers(1, 12))
        N = int(rng.integers(1, 30))
        d = int(rng.choice([0, 1, 5, 8, 17, 33]))
        nk = rng.integers(1, min(n, 9) + 1, size=N)
        _compare(oracle_lib, W.random_poly(f"crand_m{m}_s{seed}", m, d, n, N, nk, seed, cx=True))


@pytest.mark.parametrize("d", [0, 31, 64, 100, 152])
def test_complex_degrees_span_tiles(oracle_lib, d):
    rng = np.random.default_rng(d + 50)
    w = W.random_poly(f"cdeg{d}", 2, d, 6, 7, rng.integers(1, 6, size=7), seed=d + 3, cx=True)
    _compare(oracle_lib, w)


def test_complex_edge_cases(oracle_lib):
    _compare(oracle_lib, W.make("c_no_monomials", 5, 6, 3, [], seed=2, cx=True))
    _compare(oracle_lib, W.make("c_absent_vars", 4, 5, 9, [(1, 3), (3, 8), (1, 3, 8)], seed=5, cx=True))
    _compare(oracle_lib, W.make("c_n_k_1_and_2", 3, 3, 4, [(0,), (1, 2), (3,), (0, 3)], seed=8, cx=True))
    _compare(oracle_lib, W.make("c_worked_example", 10, 8, 6, [(0, 2, 5), (0, 1, 4, 5), (1, 2, 3)], seed=4, cx=True))


def test_complex_shapes_of_the_test_polynomials(oracle_lib):
    _compare(oracle_lib, W.rand3(cx=True))
    _compare(oracle_lib, W.p2(m=2, d=16, cx=True))
    _compare(oracle_lib, W.p3(m=2, d=4, cx=True))


def test_complex_p1_full_size_digest():
    # p1 in complex deca double at d = 152, against a digest of the oracle's output
    g = json.load(open(os.path.join(GOLD, "digests.json")))["workloads"]["p1_10d_d152_complex"]
    w = W.p1(cx=True)
    _say(f"complex eval_and_diff {w.name} (digest)")
    val, grad = run_gpu(w)
    assert [float(v).hex() for v in val[..., 0].ravel()] == g["value_head"]
    assert sha256(val) == g["value_sha256"]
    assert sha256(grad) == g["grad_sha256"]

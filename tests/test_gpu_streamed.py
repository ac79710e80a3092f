"""GPU parity for streamed operands (MDPE_STREAM_OPERANDS, chosen by the plan
beyond the LDS limit): both convolution operands read from global memory, a
job's coefficients spread over several wavefronts, no in-place convolution.
The operation order is unchanged, so the outputs must equal the CPU oracle's
(and the staged path's) bit for bit."""
import json
import os

import numpy as np
import pytest

from gpu_util import assert_bitexact, sha256
from paper_2101_10881_amd import workloads as W

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _run(w, stream, keep=False, ybar=None):
    import torch
    from paper_2101_10881_amd import mdpe
    dev = torch.device("cuda", 0)
    P = mdpe.Polynomial.for_workload(w, dev, keep_monomials=keep, stream_operands=stream)
    coeff = torch.from_numpy(w.coeff).to(dev)
    z = torch.from_numpy(w.z).to(dev)
    val, grad = P.eval_and_diff(coeff, z)
    out = [val, grad]
    if ybar is not None:
        out += list(P.adjoint(torch.from_numpy(np.ascontiguousarray(ybar)).to(dev), grad))
    torch.cuda.synchronize()
    return P.plan.info, [t.cpu().numpy() for t in out]


def _compare(oracle_lib, w, stream=True):  # stream: True forces, None lets the plan choose
    info, (val, grad) = _run(w, stream)
    print(f"streamed {w.name}: m={w.m} d={w.d} waves/job={info['waves_per_job']} streamed={info['streamed']}",
          flush=True)
    assert info["streamed"] == 1
    want_v, want_g = oracle_lib.eval_workload(w)
    assert_bitexact(val, want_v, f"{w.name} value")
    assert_bitexact(grad, want_g, f"{w.name} gradient")


@pytest.mark.parametrize("m", W.SUPPORTED_M)
def test_forced_streaming_random_bitexact(oracle_lib, m):
    for seed in range(2):
        rng = np.random.default_rng(9300 + 10 * m + seed)
        n = int(rng.integers(1, 10))
        N = int(rng.integers(1, 25))
        d = int(rng.choice([0, 3, 8, 33, 100]))
        nk = rng.integers(1, min(n, 7) + 1, size=N)
        w = W.random_poly(f"str_m{m}_s{seed}", m, d, n, N, nk, seed, cx=bool(seed))
        if m in (2, 5):
            w = W.with_exponents(w, 4, seed=seed)
        _compare(oracle_lib, w)


def test_forced_streaming_adjoint(oracle_lib):
    w = W.random_poly("str_adj", 4, 12, 7, 15, np.random.default_rng(3).integers(1, 7, size=15), seed=3)
    ybar = W.upstream_adjoint(4, 12, seed=2)
    info, (val, grad, cbar, zbar) = _run(w, True, keep=True, ybar=ybar)
    assert info["streamed"] == 1
    want_v, want_g = oracle_lib.eval_workload(w)
    assert_bitexact(val, want_v, "value")
    assert_bitexact(grad, want_g, "gradient")
    want_c, want_z = oracle_lib.eval_adjoint(w.m, w.d, w.n, w.nvars, w.vars, w.z, want_g, ybar)
    assert_bitexact(cbar, want_c, "coeff_bar")
    assert_bitexact(zbar, want_z, "z_bar")


def test_forced_streaming_p1_full_size_digest():
    # c1's workload with streamed operands: the same bits as the staged path
    g = json.load(open(os.path.join(GOLD, "digests.json")))["workloads"]["p1_10d_d152"]
    info, (val, grad) = _run(W.p1(), True)
    assert info["streamed"] == 1
    assert sha256(val) == g["value_sha256"]
    assert sha256(grad) == g["grad_sha256"]


@pytest.mark.parametrize("m,d,cx", [(10, 2000, False), (4, 2100, True), (2, 9000, False), (1, 20000, False)])
def test_degrees_beyond_lds_bitexact(oracle_lib, m, d, cx):
    # beyond one workgroup's LDS the plan streams by itself; at d + 1 > 4096
    # one pair of coefficients (k, d-k) per lane over many wavefronts
    w = W.make(f"big_m{m}_d{d}", m, d, 2, [(0, 1)], seed=5, cx=cx)
    _compare(oracle_lib, w, stream=None)


def _seq_conv(x, y):
    # m = 1: z_k = x_0 y_k, then += x_i y_{k-i} for i = 1..k, one float64 rounding
    # per product and per sum, vectorised over k in the same order
    acc = x[0] * y
    for i in range(1, len(x)):
        acc[i:] = acc[i:] + x[i] * y[: len(y) - i]
    return acc


def test_largest_degree_m1():
    # d = 65534, the 16-bit coefficient index's limit: p = a_0 + a_1 z_0 z_1 in
    # plain doubles against the float64 recurrence (the oracle's m = 1 pin)
    d = 65534
    w = W.make("limit_m1", 1, d, 2, [(0, 1)], seed=5)
    info, (val, grad) = _run(w, None)
    print(f"streamed limit: d={d} waves/job={info['waves_per_job']}", flush=True)
    assert info["streamed"] == 1
    a0, a1 = w.coeff[0, 0], w.coeff[0, 1]
    z0, z1 = w.z[0, 0], w.z[0, 1]
    f1 = _seq_conv(a1, z0)
    f2 = _seq_conv(f1, z1)
    b1 = _seq_conv(z1, a1)
    assert_bitexact(val[0], f2 + a0, "value")
    assert_bitexact(grad[0, 0], b1, "d/dz_0")
    assert_bitexact(grad[0, 1], f1, "d/dz_1")

"""GPU parity of the chain launch: one workgroup per chain of products,
consecutive products overlapped, first operands passed on through LDS.

Each coefficient is still one lane's sequential sum in the specified order,
so the chain launch must give the oracle's bits, and those of the layered
and fused launches, on every precision, on real and complex series, with the
monomial values kept for the reverse pass, and at the p2 size the benchmark
times.
"""
import numpy as np
import pytest

from gpu_util import assert_bitexact, require_gpu
from paper_2101_10881_amd import mdpe
from paper_2101_10881_amd import workloads as W

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)


def _run(w, **kw):
    torch = require_gpu()
    dev = torch.device("cuda", 0)
    P = mdpe.Polynomial.for_workload(w, dev, **kw)
    coeff = torch.from_numpy(w.coeff).to(dev)
    z = torch.from_numpy(w.z).to(dev)
    v, g = P.eval_and_diff(coeff, z)
    torch.cuda.synchronize()
    return P, v.cpu().numpy(), g.cpu().numpy()


def _chain_vs_oracle(oracle_lib, w):
    i = mdpe.Plan.for_workload(w, device=-1, flags=mdpe.MDPE_CHAIN_LAUNCH).info
    _say(f"chain launch {w.name}: m={w.m} d={w.d} n={w.n} N={w.N} chains={i['chain_count']} "
         f"layers={i['chain_layers']} waves={i['chain_waves']} window={i['chain_window']} ring={i['chain_ring']}")
    P, v, g = _run(w, chain_launch=True)
    assert P.plan.info["chain_layers"] > 0
    want_v, want_g = oracle_lib.eval_workload(w)
    assert_bitexact(v, want_v, f"{w.name} value")
    assert_bitexact(g, want_g, f"{w.name} gradient")


@pytest.mark.parametrize("m", W.SUPPORTED_M)
def test_p2_shape_small_degree_every_precision(oracle_lib, m):
    # p2's shape (64 variables per monomial) with 8 monomials of 40 variables
    w = W.random_poly(f"chain_m{m}", m, 8, 40, 8, [40] * 8, seed=60 + m)
    _chain_vs_oracle(oracle_lib, w)


@pytest.mark.parametrize("d", [0, 1, 31, 63, 64, 100])
def test_degrees(oracle_lib, d):
    m = 3 if d <= 64 else 2
    w = W.random_poly(f"chain_d{d}", m, d, 24, 5, [3, 9, 17, 24, 12], seed=d + 7)
    _chain_vs_oracle(oracle_lib, w)


def test_mixed_lengths_and_absent_variables(oracle_lib):
    w = W.make("chain_mixed", 4, 12, 30, [tuple(range(0, 28, 2)), (1, 3), (5,), tuple(range(1, 29)),
                                          (4, 8, 12, 16, 20)], seed=11)
    _chain_vs_oracle(oracle_lib, w)


def test_complex_series(oracle_lib):
    w = W.random_poly("chain_cx", 2, 10, 20, 4, [20, 11, 6, 15], seed=13, cx=True)
    _chain_vs_oracle(oracle_lib, w)


def test_p2_4d_d64_matches_fused_and_oracle(oracle_lib):
    w = W.p2()
    _say("chain launch p2 4d d=64 against the fused launch and the oracle")
    P, v, g = _run(w, chain_launch=True)
    _, fv, fg = _run(w, fused_layers=True)
    assert_bitexact(v, fv, "value vs fused")
    assert_bitexact(g, fg, "gradient vs fused")
    want_v, want_g = oracle_lib.eval_workload(w)
    assert_bitexact(v, want_v, "value")
    assert_bitexact(g, want_g, "gradient")


def test_kept_monomial_values_and_adjoint():
    torch = require_gpu()
    dev = torch.device("cuda", 0)
    w = W.random_poly("chain_keep", 4, 10, 20, 6, [20, 14, 9, 12, 20, 3], seed=21)
    ybar = torch.from_numpy(W.upstream_adjoint(4, 10, seed=3)).to(dev)
    out = {}
    for name, kw in (("chain", dict(chain_launch=True)), ("layers", dict(fused_layers=False))):
        _say(f"adjoint after the {name} launch")
        P = mdpe.Polynomial.for_workload(w, dev, keep_monomials=True, **kw)
        coeff = torch.from_numpy(w.coeff).to(dev)
        z = torch.from_numpy(w.z).to(dev)
        v, g = P.eval_and_diff(coeff, z)
        cb, zb = P.adjoint(ybar, g)
        torch.cuda.synchronize()
        out[name] = [t.cpu().numpy() for t in (v, g, cb, zb)]
    for a, b, what in zip(out["chain"], out["layers"], ("value", "gradient", "coeff_bar", "z_bar")):
        assert_bitexact(a, b, what)

"""GPU parity of the single launch: the whole evaluation of a small plan in one
workgroup (staging, convolution layers, scale stage, addition levels,
gather), bit for bit equal to the oracle and to the per-launch path."""
import numpy as np
import pytest

from gpu_util import assert_bitexact, require_gpu, run_gpu
from paper_2101_10881_amd import workloads as W

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)


def _poly(w, **kw):
    torch = require_gpu()
    from paper_2101_10881_amd import mdpe
    return mdpe.Polynomial.for_workload(w, torch.device("cuda", 0), **kw)


def _single_vs_oracle(oracle_lib, w, forced=True):
    P = _poly(w, single_launch=forced)
    i = P.plan.info
    assert i["single_launch"] == 1
    _say(f"single launch {w.name}: m={w.m} d={w.d} n={w.n} N={w.N} waves={i['single_waves']} "
         f"layers={i['n_layers']} levels={i['n_levels']}")
    got_v, got_g = run_gpu(w, poly=P)
    want_v, want_g = oracle_lib.eval_workload(w)
    assert_bitexact(got_v, want_v, f"{w.name} value")
    assert_bitexact(got_g, want_g, f"{w.name} gradient")
    lv, lg = run_gpu(w, poly=_poly(w, fused_layers=False))
    assert_bitexact(got_v, lv, f"{w.name} value vs per-layer launches")
    assert_bitexact(got_g, lg, f"{w.name} gradient vs per-layer launches")


def test_double_double_d8_takes_it_by_default(oracle_lib):
    # the c0 workload: 16 monomials of 3 of 8 variables, d = 8
    _single_vs_oracle(oracle_lib, W.rand3(), forced=False)


@pytest.mark.parametrize("m", W.SUPPORTED_M)
def test_every_precision(oracle_lib, m):
    w = W.random_poly(f"single_m{m}", m, 9, 10, 23, np.random.default_rng(m).integers(1, 9, size=23), seed=30 + m)
    _single_vs_oracle(oracle_lib, w)


@pytest.mark.parametrize("d", [0, 1, 31, 64, 100])
def test_degrees(oracle_lib, d):
    w = W.random_poly(f"single_d{d}", 2, d, 7, 12, np.random.default_rng(d).integers(1, 7, size=12), seed=d + 3)
    _single_vs_oracle(oracle_lib, w)


def test_edge_cases(oracle_lib):
    _single_vs_oracle(oracle_lib, W.make("single_none", 3, 4, 3, [], seed=2))               # no convolution
    _single_vs_oracle(oracle_lib, W.make("single_absent", 4, 5, 9, [(1, 3), (3, 8), (1, 3, 8)], seed=5))
    _single_vs_oracle(oracle_lib, W.make("single_one_var", 10, 0, 1, [(0,), (0,)], seed=6))
    _single_vs_oracle(oracle_lib, W.make("single_worked", 5, 8, 6, [(0, 2, 5), (0, 1, 4, 5), (1, 2, 3)], seed=4))


def test_complex_and_exponents(oracle_lib):
    _single_vs_oracle(oracle_lib, W.random_poly("single_cx", 3, 7, 6, 10, [3] * 10, seed=8, cx=True))
    # one double per part: two doubles per coefficient, staged descriptors first
    _single_vs_oracle(oracle_lib, W.random_poly("single_cx1", 1, 9, 6, 14, [3] * 14, seed=7, cx=True))
    _single_vs_oracle(oracle_lib, W.with_exponents(W.random_poly("single_e", 2, 6, 5, 9, [3] * 9, seed=9), 4, seed=2))


def test_adjoint_after_a_single_launch():
    torch = require_gpu()
    dev = torch.device("cuda", 0)
    w = W.random_poly("single_keep", 4, 10, 8, 14, [4] * 14, seed=12)
    ybar = torch.from_numpy(W.upstream_adjoint(4, 10, seed=2)).to(dev)
    outs = []
    for kw in (dict(single_launch=True), dict(fused_layers=False)):
        P = _poly(w, keep_monomials=True, **kw)
        coeff = torch.from_numpy(w.coeff).to(dev)
        z = torch.from_numpy(w.z).to(dev)
        v, g = P.eval_and_diff(coeff, z)
        cb, zb = P.adjoint(ybar, g)
        torch.cuda.synchronize()
        outs.append([t.cpu().numpy() for t in (v, g, cb, zb)])
    for a, b, what in zip(outs[0], outs[1], ("value", "gradient", "coeff_bar", "z_bar")):
        assert_bitexact(a, b, what)

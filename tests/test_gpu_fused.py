"""GPU: every convolution layer in one launch (MDPE_FUSED_LAYERS), one
workgroup per independent component, bit for bit equal to the per-layer
launches (MDPE_LAYER_LAUNCHES) and to the oracle."""
import numpy as np
import pytest

from gpu_util import assert_bitexact, run_gpu
from paper_2101_10881_amd import workloads as W

pytestmark = pytest.mark.gpu


def _layered(w):
    import torch
    from paper_2101_10881_amd import mdpe
    P = mdpe.Polynomial.for_workload(w, torch.device("cuda", 0), fused_layers=False)
    assert P.plan.info["fused_components"] == 0
    return P


def _fused(w, keep=False):
    import torch
    from paper_2101_10881_amd import mdpe
    P = mdpe.Polynomial.for_workload(w, torch.device("cuda", 0), keep_monomials=keep, fused_layers=True)
    info = P.plan.info
    assert info["fused_components"] > 0
    print(f"fused {w.name}: {info['fused_components']} components x {info['fused_waves']} wavefronts, "
          f"{info['n_layers']} layers", flush=True)
    return P


CASES = [
    ("p2_1d_d8", lambda: W.p2(m=1, d=8)),
    ("p2_2d_d63", lambda: W.p2(m=2, d=63)),
    ("p2_3d_d31", lambda: W.p2(m=3, d=31)),
    ("p2_4d_d64", lambda: W.p2()),
    ("p2_10d_d20", lambda: W.p2(m=10, d=20)),
    ("p1_10d_d8", lambda: W.p1(m=10, d=8)),
    ("p1_2d_d152", lambda: W.p1(m=2, d=152)),
    ("rand3_2d_d8", lambda: W.rand3()),
    ("p1_2d_d4_exponents", lambda: W.with_exponents(W.p1(m=2, d=4), 3, seed=5)),
    ("p1_2d_d8_complex", lambda: W.p1(m=2, d=8, cx=True)),
    ("p1_1d_d8_complex", lambda: W.p1(m=1, d=8, cx=True)),
]


@pytest.mark.parametrize("name,build", CASES, ids=[c[0] for c in CASES])
def test_fused_layers_match_per_layer_launches(name, build):
    w = build()
    want = run_gpu(w, poly=_layered(w))
    got = run_gpu(w, poly=_fused(w))
    assert_bitexact(got[0], want[0], f"{name} value")
    assert_bitexact(got[1], want[1], f"{name} grad")


@pytest.mark.parametrize("name,build", [CASES[0], CASES[3], CASES[7]], ids=["p2_1d_d8", "p2_4d_d64", "rand3_2d_d8"])
def test_fused_layers_match_oracle(oracle_lib, name, build):
    w = build()
    got = run_gpu(w, poly=_fused(w))
    v, g = oracle_lib.eval_workload(w)
    assert_bitexact(got[0], v, f"{name} value")
    assert_bitexact(got[1], g, f"{name} grad")


def test_fused_layers_keep_monomials_for_the_adjoint():
    import torch
    from paper_2101_10881_amd import mdpe
    w = W.p1(m=4, d=8)
    dev = torch.device("cuda", 0)
    ybar = torch.from_numpy(W.upstream_adjoint(4, 8, seed=3)).to(dev)
    out = []
    for fused in (False, True):
        P = mdpe.Polynomial.for_workload(w, dev, keep_monomials=True, fused_layers=fused)
        assert (P.plan.info["fused_components"] > 0) == fused
        v, g = P.eval_and_diff(torch.from_numpy(w.coeff).to(dev), torch.from_numpy(w.z).to(dev))
        cb, zb = P.adjoint(ybar, g)
        torch.cuda.synchronize()
        out.append([t.cpu().numpy() for t in (v, g, cb, zb)])
    for a, b, what in zip(out[0], out[1], ("value", "grad", "coeff_bar", "z_bar")):
        assert_bitexact(b, a, what)


@pytest.mark.parametrize("m,d,poly,expect", [(4, 127, "p2", True), (4, 128, "p2", False), (5, 31, "p2", True),
                                             (5, 32, "p2", False), (8, 8, "p2", True), (8, 9, "p2", False),
                                             (10, 31, "p2", True), (10, 32, "p2", False),
                                             (2, 63, "p1", True), (2, 64, "p1", False)])
def test_default_choice_at_its_limits(oracle_lib, m, d, poly, expect):
    # either side of the automatic rule's degree limits, bitwise against the oracle
    import torch
    from paper_2101_10881_amd import mdpe
    w = getattr(W, poly)(m=m, d=d)
    P = mdpe.Polynomial.for_workload(w, torch.device("cuda", 0), chain_launch=False)
    assert (P.plan.info["fused_components"] > 0) == expect
    print(f"{w.name}: fused={expect}", flush=True)
    got = run_gpu(w, poly=P)
    v, g = oracle_lib.eval_workload(w)
    assert_bitexact(got[0], v, f"{w.name} value")
    assert_bitexact(got[1], g, f"{w.name} grad")

"""GPU reverse pass: eval_adjoint and the torch.autograd.Function, bit for
bit against the CPU oracle, and against central finite differences of
L = sum_t ybar_t p_t on leading doubles (step 1e-6)."""
from fractions import Fraction

import numpy as np
import pytest

import exact_ref as E
from gpu_util import assert_bitexact, run_gpu
from paper_2101_10881_amd import workloads as W

pytestmark = pytest.mark.gpu


def _gpu_adjoint(w, ybar):
    import torch
    from paper_2101_10881_amd import mdpe
    dev = torch.device("cuda", 0)
    P = mdpe.Polynomial.for_workload(w, dev, keep_monomials=True)
    coeff = torch.from_numpy(w.coeff).to(dev)
    z = torch.from_numpy(w.z).to(dev)
    val, grad = P.eval_and_diff(coeff, z)
    cbar, zbar = P.adjoint(torch.from_numpy(np.ascontiguousarray(ybar)).to(dev), grad)
    torch.cuda.synchronize()
    return val.cpu().numpy(), grad.cpu().numpy(), cbar.cpu().numpy(), zbar.cpu().numpy()


def _compare(oracle_lib, w, ybar):
    print(f"adjoint {w.name}: m={w.m} d={w.d} n={w.n} N={w.N}", flush=True)
    val, grad, cbar, zbar = _gpu_adjoint(w, ybar)
    want_v, want_g = oracle_lib.eval_workload(w)
    assert_bitexact(val, want_v, "value (kept monomials)")
    assert_bitexact(grad, want_g, "gradient (kept monomials)")
    want_c, want_z = oracle_lib.eval_adjoint(w.m, w.d, w.n, w.nvars, w.vars, w.z, want_g, ybar)
    assert_bitexact(cbar, want_c, "coeff_bar")
    assert_bitexact(zbar, want_z, "z_bar")


@pytest.mark.parametrize("m", W.SUPPORTED_M)
def test_adjoint_random_bitexact(oracle_lib, m):
    for seed in range(2):
        rng = np.random.default_rng(800 + 10 * m + seed)
        n = int(rng.integers(1, 10))
        N = int(rng.integers(1, 25))
        d = int(rng.choice([0, 1, 4, 9, 40]))
        w = W.random_poly(f"adj_m{m}_{seed}", m, d, n, N, rng.integers(1, min(n, 7) + 1, size=N), seed)
        _compare(oracle_lib, w, W.md_series(rng, 1, m, d)[:, 0, :])


def test_adjoint_edge_cases(oracle_lib):
    _compare(oracle_lib, W.make("adj_absent", 3, 5, 7, [(1, 3), (0,), (1, 3, 6)], seed=3), W.upstream_adjoint(3, 5))
    _compare(oracle_lib, W.make("adj_const", 2, 4, 2, [], seed=3), W.upstream_adjoint(2, 4))
    _compare(oracle_lib, W.make("adj_ex", 10, 12, 6, [(0, 2, 5), (0, 1, 4, 5), (1, 2, 3)], seed=4),
             W.upstream_adjoint(10, 12))


@pytest.mark.parametrize("m", [1, 2])
def test_adjoint_dealt_over_wavefronts(oracle_lib, m):
    # few jobs per layer at d = 152 and one or two doubles per coefficient: the
    # plan deals each job's coefficients over several wavefronts, the reverse
    # layer's correlations too
    from paper_2101_10881_amd import mdpe
    rng = np.random.default_rng(870 + m)
    w = W.random_poly(f"adj_dealt_m{m}", m, 152, 8, 12, rng.integers(2, 6, size=12), 5)
    i = mdpe.Plan.for_workload(w, device=-1, flags=mdpe.MDPE_KEEP_MONOMIAL_VALUES).info
    assert i["simple_dealing"] == 1 and i["waves_per_job"] >= 2
    _compare(oracle_lib, w, W.md_series(rng, 1, m, 152)[:, 0, :])


def test_adjoint_reads_the_given_gradient():
    # z_bar correlates ybar with the gradient passed in: twice the gradient
    # gives exactly twice z_bar (scaling by two is exact in every md step),
    # and coeff_bar, which reads the kept monomial products, is unchanged
    import torch
    from paper_2101_10881_amd import mdpe
    w = W.random_poly("adj_grad", 4, 20, 6, 9, [2, 3, 4, 1, 3, 2, 4, 3, 2], seed=7)
    dev = torch.device("cuda", 0)
    P = mdpe.Polynomial.for_workload(w, dev, keep_monomials=True)
    _, grad = P.eval_and_diff(torch.from_numpy(w.coeff).to(dev), torch.from_numpy(w.z).to(dev))
    ybar = torch.from_numpy(W.upstream_adjoint(w.m, w.d, seed=4)).to(dev)
    cb1, zb1 = P.adjoint(ybar, grad)
    cb2, zb2 = P.adjoint(ybar, 2.0 * grad)
    torch.cuda.synchronize()
    assert_bitexact(zb2.cpu().numpy(), 2.0 * zb1.cpu().numpy(), "z_bar of twice the gradient")
    assert_bitexact(cb2.cpu().numpy(), cb1.cpu().numpy(), "coeff_bar")


def test_p1_8d_d32_adjoint_bitexact(oracle_lib):
    w = W.p1(m=8, d=32)
    _compare(oracle_lib, w, W.upstream_adjoint(w.m, w.d, seed=1))


def _autograd_check(oracle_lib, w, ybar, samples, seed):
    """poly_eval(coeff, z).backward(ybar): value, coeff.grad and z.grad bit for
    bit against the oracle; then central differences of L = sum_t ybar_t p_t on
    leading doubles (step 1e-6), through the GPU forward, at `samples` entries
    of z and of the coefficients each.  p is affine in every single input
    coefficient (eq. (3)), so the differences are exact up to md rounding."""
    import torch
    from paper_2101_10881_amd import mdpe
    from paper_2101_10881_amd.autograd import poly_eval
    print(f"autograd {w.name}: m={w.m} d={w.d} n={w.n} N={w.N}", flush=True)
    dev = torch.device("cuda", 0)
    P = mdpe.Polynomial.for_workload(w, dev, keep_monomials=True)
    coeff = torch.from_numpy(w.coeff).to(dev).requires_grad_(True)
    z = torch.from_numpy(w.z).to(dev).requires_grad_(True)
    value, grad = poly_eval(coeff, z, P)
    value.backward(torch.from_numpy(ybar).to(dev))
    torch.cuda.synchronize()
    want_v, want_g = oracle_lib.eval_workload(w)
    assert_bitexact(value.detach().cpu().numpy(), want_v, "value")
    assert_bitexact(grad.cpu().numpy(), want_g, "gradient")
    want_c, want_z = oracle_lib.eval_adjoint(w.m, w.d, w.n, w.nvars, w.vars, w.z, want_g, ybar)
    assert_bitexact(coeff.grad.cpu().numpy(), want_c, "coeff.grad")
    assert_bitexact(z.grad.cpu().numpy(), want_z, "z.grad")
    zg, cg = z.grad.cpu().numpy(), coeff.grad.cpu().numpy()

    def L(ww):
        v, _ = run_gpu(ww, poly=P)
        return sum(Fraction(float(ybar[0, t])) * E.md_value(v[:, t]) for t in range(ww.d + 1))

    rng = np.random.default_rng(seed)
    for kind in ("z", "a") * samples:
        arr = w.z if kind == "z" else w.coeff
        idx = int(rng.integers(arr.shape[1]))
        s = int(rng.integers(w.d + 1))
        x0 = arr[0, idx, s]
        out = []
        for sign in (1, -1):
            arr[0, idx, s] = x0 + sign * 1e-6
            out.append((L(w), Fraction(float(arr[0, idx, s])) - Fraction(float(x0))))
            arr[0, idx, s] = x0
        fd = (out[0][0] - out[1][0]) / (out[0][1] - out[1][1])
        adj = E.md_value((zg if kind == "z" else cg)[:, idx, s])
        assert abs(fd - adj) <= Fraction(1, 10 ** 9) * max(abs(adj), Fraction(1, 10 ** 6)), (kind, idx, s)


def test_autograd_function_matches_oracle_and_finite_differences(oracle_lib):
    w = W.random_poly("ag", 8, 10, 8, 30, [4] * 30, seed=21)
    _autograd_check(oracle_lib, w, W.upstream_adjoint(w.m, w.d, seed=2), samples=2, seed=5)


def test_autograd_function_p1_8d_d32_full_size(oracle_lib):
    # the differentiation workload itself: octo double, d = 32, all 1820
    # four-variable monomials of 16 variables, upstream adjoint uniform in [-1, 1]
    w = W.p1(m=8, d=32)
    _autograd_check(oracle_lib, w, W.upstream_adjoint(w.m, w.d, seed=1), samples=8, seed=7)

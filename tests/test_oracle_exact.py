"""Pins for the oracle's polynomial evaluation and differentiation (CPU only).

Everything here is checked against something other than the oracle itself:

* exact rational brute force (value and every partial derivative, written
  from the definition of eq. (3) with the truncated products of eq. (1)),
  within the bound 4(d+1) 2^(-52m) relative to the magnitude series;
* integer-valued inputs, where every operation is exact and the oracle must
  return the exact integers bit for bit;
* closed forms: z_i = 1+t gives binomial coefficients, z_i = 1/(1-t) gives
  C(j+r-1, r-1);
* Euler's identity for homogeneous polynomials, sum_i z_i * dp/dz_i = r p,
  which ties the gradient (backward and cross products) to the value
  (forward products);
* permutation symmetry of p1 (Section 6.1) with one coefficient series for
  every monomial: permuted inputs give the same value and the permuted
  gradient, within twice the bound;
* the pairwise addition tree against the paper's worked example (Section 4,
  the two steps after eq. (5)) and against the eleven addition launch sizes
  printed for p1 in Section 6.1.
"""
from fractions import Fraction
from math import comb

import numpy as np
import pytest

import exact_ref as E
from paper_2101_10881_amd import workloads as W

MS = W.SUPPORTED_M


def _check_against_exact(oracle_lib, w):
    val, grad = oracle_lib.eval_workload(w)
    (ev, eg), (mv, mg) = E.workload_exact(w)
    b = E.bound(w.m, w.d)
    assert E.max_scaled_error(val, ev, mv) <= b, "value"
    for i in range(w.n):
        assert E.max_scaled_error(grad[:, i, :], eg[i], mg[i]) <= b, f"grad {i}"
    return val, grad


@pytest.mark.parametrize("m", MS)
def test_random_tiny_polynomials_vs_rationals(oracle_lib, m):
    for seed in range(1, 7):
        rng = np.random.default_rng(1000 * m + seed)
        n = int(rng.integers(1, 6))
        N = int(rng.integers(0, 6))
        d = int(rng.integers(0, 5))
        nk = rng.integers(1, n + 1, size=N)
        _check_against_exact(oracle_lib, W.random_poly("t", m, d, n, N, nk, seed))


@pytest.mark.parametrize("m", [1, 2, 4, 10])
def test_worked_example_vs_rationals(oracle_lib, m):
    # p = a0 + a1 x1 x3 x6 + a2 x1 x2 x5 x6 + a3 x2 x3 x4   (Section 4, eq. (4)); 0-based below
    sup = [(0, 2, 5), (0, 1, 4, 5), (1, 2, 3)]
    _check_against_exact(oracle_lib, W.make("ex", m, 3, 6, sup, seed=4))


@pytest.mark.parametrize("m", [2, 3])
def test_monomial_n5_and_absent_variables(oracle_lib, m):
    # the n = 5 statement table of eq. (2), plus variables that appear nowhere
    _check_against_exact(oracle_lib, W.make("n5", m, 2, 7, [(0, 2, 3, 5, 6)], seed=9))
    _check_against_exact(oracle_lib, W.make("n6", m, 1, 8, [(1, 2, 3, 4, 6, 7), (0, 7)], seed=10))


def test_no_monomials_gives_a0_and_zero_gradient(oracle_lib):
    w = W.make("const", 4, 3, 3, [], seed=2)
    val, grad = oracle_lib.eval_workload(w)
    assert np.array_equal(val, w.coeff[:, 0, :])
    assert not np.any(grad) and not np.any(np.signbit(grad))


def _integer_workload(m, d, n, supports, rng, lo=-3, hi=4):
    w = W.make("int", m, d, n, supports, seed=1)
    w.coeff[:] = 0.0
    w.z[:] = 0.0
    w.coeff[0] = rng.integers(lo, hi, size=w.coeff.shape[1:]).astype(float)
    w.z[0] = rng.integers(lo, hi, size=w.z.shape[1:]).astype(float)
    return w


@pytest.mark.parametrize("m", MS)
def test_integer_inputs_are_exact(oracle_lib, m):
    rng = np.random.default_rng(50 + m)
    sup = W.random_supports(rng, 6, 7, rng.integers(1, 5, size=7))
    w = _integer_workload(m, 5, 6, sup, rng)
    val, grad = oracle_lib.eval_workload(w)
    (ev, eg), _ = E.workload_exact(w)
    assert list(val[0]) == [float(v) for v in ev]
    assert not np.any(val[1:])
    for i in range(w.n):
        assert list(grad[0, i]) == [float(v) for v in eg[i]]
    assert not np.any(grad[1:])


@pytest.mark.parametrize("m", [1, 2, 5, 8])
def test_closed_form_one_plus_t(oracle_lib, m):
    # z_i = 1 + t and constant coefficients c_k: value_j = a0_j + sum_k c_k C(n_k, j),
    # d/dz_i coefficient j = sum_{k contains i} c_k C(n_k - 1, j)
    rng = np.random.default_rng(7)
    n, d = 6, 6
    sup = W.random_supports(rng, n, 9, rng.integers(1, 6, size=9))
    w = W.make("1pt", m, d, n, sup, seed=1)
    w.coeff[:] = 0.0
    w.z[:] = 0.0
    c = rng.integers(-5, 6, size=len(sup)).astype(float)
    w.coeff[0, 1:, 0] = c
    w.coeff[0, 0, :] = 0.0
    w.z[0, :, 0] = 1.0
    w.z[0, :, 1] = 1.0
    val, grad = oracle_lib.eval_workload(w)
    for j in range(d + 1):
        assert val[0, j] == sum(ck * comb(len(s), j) for ck, s in zip(c, sup))
        for i in range(n):
            assert grad[0, i, j] == sum(ck * comb(len(s) - 1, j) for ck, s in zip(c, sup) if i in s)
    assert not np.any(val[1:]) and not np.any(grad[1:])


@pytest.mark.parametrize("m", [2, 4])
def test_closed_form_geometric(oracle_lib, m):
    # z_i = 1/(1-t) = 1 + t + t^2 + ...: a product of r of them has coefficients C(j+r-1, r-1)
    n, d = 5, 9
    sup = [(0, 1, 2), (1, 3), (0, 1, 2, 3, 4)]
    w = W.make("geo", m, d, n, sup, seed=1)
    w.coeff[:] = 0.0
    w.z[:] = 0.0
    w.coeff[0, 1:, 0] = 1.0
    w.z[0] = 1.0
    val, grad = oracle_lib.eval_workload(w)
    for j in range(d + 1):
        assert val[0, j] == sum(comb(j + len(s) - 1, len(s) - 1) for s in sup)
        assert grad[0, 1, j] == sum(comb(j + len(s) - 2, len(s) - 2) for s in sup)


@pytest.mark.parametrize("m", [2, 3, 4])
def test_euler_identity_homogeneous(oracle_lib, m):
    # homogeneous of degree r with a_0 = 0:  sum_i z_i * dp/dz_i = r p  (exact in the truncated ring)
    r, n, d = 4, 8, 6
    rng = np.random.default_rng(21 + m)
    sup = W.random_supports(rng, n, 12, [r] * 12)
    w = W.make("euler", m, d, n, sup, seed=5)
    w.coeff[:, 0, :] = 0.0
    val, grad = oracle_lib.eval_workload(w)
    z = E.planar_to_exact(w.z)
    lhs = [Fraction(0)] * (d + 1)
    for i in range(n):
        lhs = E.sadd(lhs, E.smul(z[i], E.series_to_exact(grad[:, i, :])))
    rhs = [r * v for v in E.series_to_exact(val)]
    _, (mv, _) = E.workload_exact(w)
    tol = E.bound(m, d) * 3 * r
    for j in range(d + 1):
        assert abs(lhs[j] - rhs[j]) <= tol * mv[j]


def test_m1_against_numpy_float64(oracle_lib):
    # m = 1 is plain float64: compare with numpy products in another order, to rounding
    rng = np.random.default_rng(4)
    w = W.random_poly("np", 1, 7, 5, 9, rng.integers(1, 5, size=9), seed=4)
    val, grad = oracle_lib.eval_workload(w)
    d = w.d
    trunc = lambda a, b: np.convolve(a, b)[: d + 1]
    v = w.coeff[0, 0].copy()
    for k, s in enumerate(w.supports()):
        t = w.coeff[0, k + 1]
        for j in s:
            t = trunc(t, w.z[0, j])
        v = v + t
    assert np.allclose(val[0], v, rtol=0, atol=1e-13)


def test_tree_schedule_matches_worked_example(oracle_lib):
    # value list [a0, f13, f24, f33]: f13 := a0 + f13 and f33 := f24 + f33, then f33 := f33 + f13
    assert oracle_lib.tree_schedule(4) == [[(0, 1), (2, 3)], [(1, 3)]]
    assert oracle_lib.tree_schedule(2) == [[(0, 1)]]   # d/dz1 = b11 + b22
    assert oracle_lib.tree_schedule(1) == []
    assert oracle_lib.tree_schedule(0) == []


def test_tree_launch_sizes_match_p1(oracle_lib):
    # p1: value list of 1 + 1820 entries, 16 gradient lists of C(15,3) = 455 entries.
    # Section 6.1 prints the addition launches: 4542, 2279, 1140, 562, 281, 140, 78, 39, 20, 2, 1.
    val = [len(r) for r in oracle_lib.tree_schedule(1821)]
    gr = [len(r) for r in oracle_lib.tree_schedule(455)]
    total = [val[i] + 16 * (gr[i] if i < len(gr) else 0) for i in range(len(val))]
    assert total == [4542, 2279, 1140, 562, 281, 140, 78, 39, 20, 2, 1]
    assert sum(total) == 9084


@pytest.mark.parametrize("m,d", [(1, 4), (2, 3), (3, 3), (10, 2)])
def test_p1_permutation_symmetry(oracle_lib, m, d):
    # p1 with equal a_k is symmetric in its 16 variables: permuting the inputs
    # leaves the value and permutes the gradient (Section 6.1's p1 shape)
    assert E.permutation_symmetry_holds(oracle_lib.eval_workload, m, d, seed=3)

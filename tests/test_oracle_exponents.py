"""Pins for the oracle's general exponents (CPU only).

A monomial a_k prod_j z_{i_j}^{e_j} is evaluated as the multilinear monomial
F_k prod_j z_{i_j} with the common factor F_k = a_k prod_j z_{i_j}^{e_j - 1}
taken from a table of powers (Section 3), and every partial derivative is e_j
times the multilinear one.  Checked against

* exact rational brute force written from the definition (value and every
  partial derivative of sum_k a_k prod z^e), real and complex, within
  4(d+1) 2^(-52m) of the magnitude series;
* closed forms: (1+t)^e and its derivative e (1+t)^(e-1), integer-exact;
* integer inputs with exponents, exact bit for bit;
* all exponents one, which must reproduce the multilinear path bit for bit;
* the rejection of exponents outside 1..64.
"""
from math import comb

import numpy as np
import pytest

import exact_ref as E
from paper_2101_10881_amd import workloads as W


def _check(oracle_lib, w):
    val, grad = oracle_lib.eval_workload(w)
    (ev, eg), (mv, mg) = E.workload_exact(w)
    b = E.bound(w.m, w.d)
    assert E.max_scaled_error(val, ev, mv) <= b, "value"
    for i in range(w.n):
        assert E.max_scaled_error(grad[..., i, :], eg[i], mg[i]) <= b, f"grad {i}"
    return val, grad


@pytest.mark.parametrize("m", W.SUPPORTED_M)
@pytest.mark.parametrize("cx", [False, True])
def test_random_polynomials_with_exponents_vs_rationals(oracle_lib, m, cx):
    for seed in range(1, 4):
        rng = np.random.default_rng(700 + 10 * m + seed)
        n = int(rng.integers(1, 5))
        N = int(rng.integers(1, 5))
        d = int(rng.integers(0, 4))
        w = W.random_poly("e", m, d, n, N, rng.integers(1, n + 1, size=N), seed, cx=cx)
        _check(oracle_lib, W.with_exponents(w, 4, seed=seed))


def test_worked_example_with_exponents(oracle_lib):
    w = W.make("ex", 3, 5, 6, [(0, 2, 5), (0, 1, 4, 5), (1, 2, 3), (4,)], seed=4)
    w.exps = np.array([2, 1, 3, 1, 2, 1, 4, 5, 1, 1, 3], dtype=np.int32)
    _check(oracle_lib, w)


@pytest.mark.parametrize("m", [1, 2, 4])
@pytest.mark.parametrize("e", [1, 2, 3, 7])
def test_closed_form_power_of_one_plus_t(oracle_lib, m, e):
    d = 9
    w = W.make("pow", m, d, 2, [(1,)], seed=1)
    w.exps = np.array([e], dtype=np.int32)
    w.coeff[:] = 0.0
    w.coeff[0, 1, 0] = 1.0            # a_1 = 1, a_0 = 0
    w.z[:] = 0.0
    w.z[0, :, 0] = 1.0
    w.z[0, :, 1] = 1.0                # z = 1 + t
    val, grad = oracle_lib.eval_workload(w)
    assert [float(v) for v in val[0]] == [comb(e, j) for j in range(d + 1)]
    assert [float(v) for v in grad[0, 1]] == [e * comb(e - 1, j) for j in range(d + 1)]
    assert not val[1:].any() and not grad[1:].any() and not grad[:, 0].any()


@pytest.mark.parametrize("m", [1, 3])
def test_integer_inputs_with_exponents_exact(oracle_lib, m):
    rng = np.random.default_rng(31 + m)
    w = W.random_poly("ints", m, 4, 4, 6, rng.integers(1, 4, size=6), seed=31)
    w = W.with_exponents(w, 3, seed=2)
    w.coeff[:] = 0.0
    w.z[:] = 0.0
    w.coeff[0] = rng.integers(-2, 3, size=w.coeff.shape[1:])
    w.z[0] = rng.integers(-1, 2, size=w.z.shape[1:])
    val, grad = oracle_lib.eval_workload(w)
    (ev, eg), _ = E.workload_exact(w)
    assert [float(v) for v in val[0]] == [float(x) for x in ev] and not val[1:].any()
    for i in range(w.n):
        assert [float(v) for v in grad[0, i]] == [float(x) for x in eg[i]] and not grad[1:, i].any()


@pytest.mark.parametrize("cx", [False, True])
def test_unit_exponents_reproduce_multilinear_path(oracle_lib, cx):
    w = W.random_poly("ones", 4, 6, 6, 9, [1, 2, 3, 4, 5, 3, 2, 6, 3], seed=5, cx=cx)
    v0, g0 = oracle_lib.eval_workload(w)
    w.exps = np.ones_like(w.vars)
    v1, g1 = oracle_lib.eval_workload(w)
    assert np.array_equal(v0.view(np.int64), v1.view(np.int64))
    assert np.array_equal(g0.view(np.int64), g1.view(np.int64))


@pytest.mark.parametrize("e", [0, -1, 65])
def test_bad_exponents_rejected(oracle_lib, e):
    w = W.make("bad", 2, 2, 3, [(0, 2)], seed=1)
    w.exps = np.array([1, e], dtype=np.int32)
    with pytest.raises(ValueError):
        oracle_lib.eval_workload(w)

"""Pins for the oracle's complex series (CPU only).

Complex coefficients keep real and imaginary parts in separate arrays
(Sections 2 and 5).  The oracle's complex product is (xr yr - xi yi) +
(xr yi + xi yr) i with every product an md_mul and the two sums md_adds (the
difference adds the exactly negated product).  Checked against

* exact complex rational arithmetic, per operation and for whole tiny
  polynomials with their gradients, within 4(d+1) 2^(-52m) relative to the
  magnitude series taken with the L1 modulus |re| + |im|;
* Gaussian-integer inputs, where every operation is exact and the oracle must
  return the exact integers bit for bit;
* zero imaginary parts, which must reproduce the real path bit for bit (the
  negated zero products and the zero imaginary sums change no bit);
* conjugate symmetry: with real coefficients, p(conj z) = conj(p(z)) and the
  same for every partial derivative, value for value (every rounding is
  symmetric under negation).
"""
from fractions import Fraction

import numpy as np
import pytest

import exact_ref as E
from paper_2101_10881_amd import workloads as W

MS = W.SUPPORTED_M


def _cmd(rng, count, m):
    re = W.md_series(rng, count, m, 0)[:, :, 0]
    im = W.md_series(rng, count, m, 0)[:, :, 0]
    return np.ascontiguousarray(np.stack([re, im]))


def _cval(arr, i):
    return E.CF(E.md_value(arr[0, :, i]), E.md_value(arr[1, :, i]))


@pytest.mark.parametrize("m", MS)
@pytest.mark.parametrize("op", ["cadd", "cmul"])
def test_complex_md_ops_vs_rationals(oracle_lib, m, op):
    rng = np.random.default_rng(40 + m)
    count = 300
    x = _cmd(rng, count, m)
    y = _cmd(rng, count, m) * np.ldexp(1.0, rng.integers(-4, 4, size=count))
    y[:, :, :30] = -x[:, :, :30]                       # cancellation
    z = oracle_lib.md_op(op, x, y)
    eps = Fraction(1, 2 ** (52 * m))
    for i in range(count):
        a, b, got = _cval(x, i), _cval(y, i), _cval(z, i)
        want = a + b if op == "cadd" else a * b
        scale = abs(a) + abs(b) if op == "cadd" else 2 * abs(a) * abs(b)
        assert abs(got.re - want.re) <= eps * scale and abs(got.im - want.im) <= eps * scale, (op, m, i)


@pytest.mark.parametrize("m", MS)
def test_random_tiny_complex_polynomials_vs_rationals(oracle_lib, m):
    for seed in range(1, 4):
        rng = np.random.default_rng(900 + 10 * m + seed)
        n = int(rng.integers(1, 6))
        N = int(rng.integers(1, 6))
        d = int(rng.integers(0, 4))
        w = W.random_poly("cx", m, d, n, N, rng.integers(1, n + 1, size=N), seed, cx=True)
        val, grad = oracle_lib.eval_workload(w)
        assert val.shape == (2, m, d + 1) and grad.shape == (2, m, n, d + 1)
        (ev, eg), (mv, mg) = E.workload_exact(w)
        b = E.bound(m, d)
        assert E.max_scaled_error(val, ev, mv) <= b, "value"
        for i in range(n):
            assert E.max_scaled_error(grad[:, :, i, :], eg[i], mg[i]) <= b, f"grad {i}"


def test_worked_example_complex_vs_rationals(oracle_lib):
    w = W.make("ex", 4, 5, 6, [(0, 2, 5), (0, 1, 4, 5), (1, 2, 3)], seed=4, cx=True)
    val, grad = oracle_lib.eval_workload(w)
    (ev, eg), (mv, mg) = E.workload_exact(w)
    assert E.max_scaled_error(val, ev, mv) <= E.bound(4, 5)
    for i in range(6):
        assert E.max_scaled_error(grad[:, :, i, :], eg[i], mg[i]) <= E.bound(4, 5)


@pytest.mark.parametrize("m", [1, 2, 5, 10])
def test_gaussian_integer_inputs_exact(oracle_lib, m):
    rng = np.random.default_rng(60 + m)
    w = W.random_poly("gint", m, 4, 5, 7, rng.integers(1, 5, size=7), seed=11, cx=True)
    w.coeff[:] = 0.0
    w.z[:] = 0.0
    w.coeff[:, 0] = rng.integers(-3, 4, size=w.coeff[:, 0].shape)
    w.z[:, 0] = rng.integers(-2, 3, size=w.z[:, 0].shape)
    val, grad = oracle_lib.eval_workload(w)
    (ev, eg), _ = E.workload_exact(w)
    for c in range(w.d + 1):
        e = E.CF._lift(ev[c])
        assert val[0, 0, c] == e.re and val[1, 0, c] == e.im
        assert not val[:, 1:, c].any()                  # exact integers: lower limbs zero
    for i in range(w.n):
        for c in range(w.d + 1):
            e = E.CF._lift(eg[i][c])
            assert grad[0, 0, i, c] == e.re and grad[1, 0, i, c] == e.im


@pytest.mark.parametrize("m", [1, 2, 4, 10])
def test_zero_imaginary_parts_reproduce_real_path(oracle_lib, m):
    wr = W.random_poly("r", m, 7, 6, 9, [1, 2, 3, 4, 3, 2, 5, 6, 3], seed=5)
    wc = W.random_poly("r", m, 7, 6, 9, [1, 2, 3, 4, 3, 2, 5, 6, 3], seed=5, cx=True)
    assert np.array_equal(wc.coeff[0], wr.coeff) and np.array_equal(wc.z[0], wr.z)
    wc.coeff[1] = 0.0
    wc.z[1] = 0.0
    vr, gr = oracle_lib.eval_workload(wr)
    vc, gc = oracle_lib.eval_workload(wc)
    assert np.array_equal(vc[0].view(np.int64), vr.view(np.int64))
    assert np.array_equal(gc[0].view(np.int64), gr.view(np.int64))
    assert not vc[1].any() and not gc[1].any()


@pytest.mark.parametrize("m", [2, 3, 8])
def test_conjugate_symmetry(oracle_lib, m):
    w = W.random_poly("conj", m, 6, 7, 12, [1, 2, 3, 4, 5, 3, 2, 4, 3, 6, 2, 3], seed=13, cx=True)
    w.coeff[1] = 0.0                                    # real coefficients
    val, grad = oracle_lib.eval_workload(w)
    w.z[1] = -w.z[1]                                    # conj z (exact)
    cval, cgrad = oracle_lib.eval_workload(w)
    assert np.array_equal(cval[0], val[0]) and np.array_equal(cval[1], -val[1])
    assert np.array_equal(cgrad[0], grad[0]) and np.array_equal(cgrad[1], -grad[1])

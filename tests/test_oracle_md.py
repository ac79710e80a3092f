"""Pins for the oracle's multiple-double operations (CPU only).

* two_sum / two_prod are error-free: hi + lo equals the exact sum / product
  and hi is the rounded result (Knuth; Dekker/FMA).
* md_add / md_mul agree with exact rational arithmetic to within
  2^(-52m) times the operand magnitude (|x|+|y| for add, |x||y| for mul), on
  random, cancelling and power-of-two-scaled operands, for every m.
* m = 1 reduces to plain binary64 + and *.
* Results are normalised expansions: |z_{j+1}| <= ulp(z_j)/2 on random inputs.
* The double-operation counts of one md op agree with the closed forms the
  benchmark uses for its flop accounting.
"""
from fractions import Fraction

import numpy as np
import pytest

from exact_ref import md_value
from paper_2101_10881_amd import workloads as W

MS = W.SUPPORTED_M


def _operands(rng, m, count):
    x = W.md_series(rng, count, m, 0)[:, :, 0]
    y = W.md_series(rng, count, m, 0)[:, :, 0]
    y = y * np.ldexp(1.0, rng.integers(-4, 4, size=count))  # exact rescaling
    q = count // 8
    y[:, :q] = -x[:, :q]                     # exact cancellation of the leading limbs
    if m > 1:
        y[m - 1, :q] = x[m - 1, :q] * 0.5    # ... leaving a tiny remainder
    y[:, q:2 * q] = x[:, q:2 * q]            # doubling
    return np.ascontiguousarray(x), np.ascontiguousarray(y)


def test_two_sum_two_prod_exact(oracle_lib):
    rng = np.random.default_rng(11)
    a = rng.uniform(-1, 1, 4000) * np.ldexp(1.0, rng.integers(-60, 60, 4000))
    b = rng.uniform(-1, 1, 4000) * np.ldexp(1.0, rng.integers(-60, 60, 4000))
    a[:10] = [0.0, -0.0, 1.0, 2.0 ** 53, 1e300, -1e-300, 3.0, 0.1, 1.0, -2.0]
    b[:10] = [0.0, 0.0, 2.0 ** -60, 1.0, 1e300, 1e-300, -3.0, 0.2, -1.0, 2.0 ** -1074 * 3]
    hi, lo = oracle_lib.eft("two_sum", a, b)
    for i in range(a.size):
        assert Fraction(hi[i]) + Fraction(lo[i]) == Fraction(a[i]) + Fraction(b[i])
        assert hi[i] == a[i] + b[i]
    hi, lo = oracle_lib.eft("two_prod", a[10:], b[10:])
    for i in range(hi.size):
        assert Fraction(hi[i]) + Fraction(lo[i]) == Fraction(a[10 + i]) * Fraction(b[10 + i])
        assert hi[i] == a[10 + i] * b[10 + i]


@pytest.mark.parametrize("m", MS)
@pytest.mark.parametrize("op", ["add", "mul"])
def test_md_op_vs_rationals(oracle_lib, m, op):
    rng = np.random.default_rng(100 + m)
    x, y = _operands(rng, m, 600)
    z = oracle_lib.md_op(op, x, y)
    tol = Fraction(1, 2 ** (52 * m))
    for i in range(x.shape[1]):
        X, Y, Z = md_value(x[:, i]), md_value(y[:, i]), md_value(z[:, i])
        exact = X + Y if op == "add" else X * Y
        mag = abs(X) + abs(Y) if op == "add" else abs(X) * abs(Y)
        assert abs(Z - exact) <= tol * mag, (m, op, i)


@pytest.mark.parametrize("m", [m for m in MS if m > 1])
def test_md_results_normalised(oracle_lib, m):
    rng = np.random.default_rng(7 + m)
    x = W.md_series(rng, 800, m, 0)[:, :, 0]
    y = W.md_series(rng, 800, m, 0)[:, :, 0]
    for op in ("add", "mul"):
        z = oracle_lib.md_op(op, x, y)
        for j in range(m - 1):
            nz = z[j] != 0
            assert np.all(np.abs(z[j + 1][nz]) <= np.spacing(np.abs(z[j][nz])) / 2)


def test_m1_is_plain_binary64(oracle_lib):
    rng = np.random.default_rng(3)
    x = rng.uniform(-1, 1, (1, 1000))
    y = rng.uniform(-1, 1, (1, 1000))
    assert np.array_equal(oracle_lib.md_op("add", x, y), x + y)
    assert np.array_equal(oracle_lib.md_op("mul", x, y), x * y)


def test_integer_operands_exact(oracle_lib):
    for m in MS:
        x = np.zeros((m, 3)); y = np.zeros((m, 3))
        x[0] = [3.0, -7.0, 2.0 ** 40]
        y[0] = [5.0, 7.0, 2.0 ** 12]
        s = oracle_lib.md_op("add", x, y)
        p = oracle_lib.md_op("mul", x, y)
        assert list(s[0]) == [8.0, 0.0, 2.0 ** 40 + 2.0 ** 12]
        assert list(p[0]) == [15.0, -49.0, 2.0 ** 52]
        assert not np.any(s[1:]) and not np.any(p[1:])


@pytest.mark.parametrize("m", MS)
def test_op_counts_match_flop_formula(oracle_lib, m):
    from paper_2101_10881_amd import flops
    for op in ("add", "mul"):
        c = oracle_lib.op_counts(op, m)
        f = flops.md_op_counts(op, m)
        assert (c["add"], c["mul"], c["fma"]) == (f["add"], f["mul"], f["fma"]), (op, m, c, f)

"""Pins for the oracle's reverse pass (CPU only).

L = sum_t ybar_t p_t.  The adjoints are checked
* against exact rational brute force: abar_k[s] = sum_t ybar_t (prod_{j in k} z_j)_{t-s},
  zbar_i[s] = sum_t ybar_t (dp/dz_i)_{t-s}, abar_0 = ybar, within 8(d+1) 2^(-52m)
  relative to the same sums taken over absolute values;
* against central finite differences of L on leading doubles (step 1e-6): p is
  affine in every single coefficient, so the difference quotient is the exact
  derivative up to the multiple-double rounding of L.
"""
from fractions import Fraction

import numpy as np
import pytest

import exact_ref as E
from paper_2101_10881_amd import workloads as W


def _exact_adjoint(w, ybar):
    a = E.planar_to_exact(w.coeff)
    z = E.planar_to_exact(w.z)
    yb = E.series_to_exact(ybar)
    d = w.d
    sup = w.supports()
    (val, grad), (mval, mgrad) = E.workload_exact(w)

    def corr(x, y):
        return [sum((x[s + j] * y[j] for j in range(d + 1 - s)), Fraction(0)) for s in range(d + 1)]

    absy = [abs(v) for v in yb]
    prods, mprods = [], []
    for s_ in sup:
        t = [Fraction(1)] + [Fraction(0)] * d
        tm = list(t)
        for v in s_:
            t = E.smul(t, z[v])
            tm = E.smul(tm, [abs(c) for c in z[v]])
        prods.append(t)
        mprods.append(tm)
    cbar = [list(yb)] + [corr(yb, M) for M in prods]
    cmag = [absy] + [corr(absy, M) for M in mprods]
    zbar = [corr(yb, g) for g in grad]
    zmag = [corr(absy, g) for g in mgrad]
    return cbar, cmag, zbar, zmag


def _check(oracle_lib, w, ybar):
    cbar, zbar = oracle_lib.adjoint_workload(w, ybar)
    ec, mc, ez, mz = _exact_adjoint(w, ybar)
    tol = 2 * E.bound(w.m, w.d)
    for k in range(w.N + 1):
        assert E.max_scaled_error(cbar[:, k, :], ec[k], mc[k]) <= tol, f"abar {k}"
    for i in range(w.n):
        assert E.max_scaled_error(zbar[:, i, :], ez[i], mz[i]) <= tol, f"zbar {i}"
    return cbar, zbar


@pytest.mark.parametrize("m", W.SUPPORTED_M)
def test_adjoint_vs_rationals(oracle_lib, m):
    for seed in range(1, 4):
        rng = np.random.default_rng(300 + 10 * m + seed)
        n = int(rng.integers(1, 6))
        N = int(rng.integers(0, 6))
        d = int(rng.integers(0, 5))
        w = W.random_poly("adj", m, d, n, N, rng.integers(1, n + 1, size=N), seed)
        ybar = W.md_series(np.random.default_rng(seed), 1, m, d)[:, 0, :]
        _check(oracle_lib, w, ybar)


def test_adjoint_worked_example_and_absent(oracle_lib):
    w = W.make("ex", 4, 4, 8, [(0, 2, 5), (0, 1, 4, 5), (1, 2, 3), (6,)], seed=4)
    cbar, zbar = _check(oracle_lib, w, W.upstream_adjoint(4, 4, seed=3))
    assert not np.any(zbar[:, 7, :]) and not np.any(np.signbit(zbar[:, 7, :]))   # variable 8 is absent
    assert np.array_equal(cbar[:, 0, :], W.upstream_adjoint(4, 4, seed=3))        # abar_0 = ybar


def _L(oracle_lib, w, ybar):
    val, _ = oracle_lib.eval_workload(w)
    return sum(Fraction(float(ybar[0, t])) * E.md_value(val[:, t]) for t in range(w.d + 1))   # ybar has one limb


@pytest.mark.parametrize("m", [2, 8])
def test_adjoint_vs_central_differences(oracle_lib, m):
    w = W.random_poly("fd", m, 6, 6, 10, [3, 4, 2, 4, 3, 1, 4, 3, 2, 4], seed=8)
    ybar = W.upstream_adjoint(m, 6, seed=5)          # leading limb uniform in [-1, 1), lower limbs 0
    cbar, zbar = oracle_lib.adjoint_workload(w, ybar)
    rng = np.random.default_rng(2)
    h = 1e-6
    picks = [("z", int(rng.integers(w.n)), int(rng.integers(w.d + 1))) for _ in range(4)]
    picks += [("a", int(rng.integers(w.N + 1)), int(rng.integers(w.d + 1))) for _ in range(4)]
    for kind, idx, s in picks:
        arr = w.z if kind == "z" else w.coeff
        x0 = arr[0, idx, s]
        vals = []
        for sign in (1, -1):
            arr[0, idx, s] = x0 + sign * h
            step = Fraction(float(arr[0, idx, s])) - Fraction(float(x0))
            vals.append((_L(oracle_lib, w, ybar), step))
            arr[0, idx, s] = x0
        fd = (vals[0][0] - vals[1][0]) / (vals[0][1] - vals[1][1])
        adj = E.md_value((zbar if kind == "z" else cbar)[:, idx, s])
        assert abs(fd - adj) <= Fraction(1, 10 ** 9) * max(abs(adj), Fraction(1, 10 ** 6)), (kind, idx, s)

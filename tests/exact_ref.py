"""Exact rational reference (Python fractions) for the oracle's pins.

A multiple double x = (x_0, ..., x_{m-1}) denotes the exact rational sum of
its limbs.  Everything here is exact: truncated power-series products
(eq. (1) of the paper) and the polynomial of eq. (3) with its gradient,
written directly from the definitions, with no ordering or rounding.
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np


def md_value(limbs) -> Fraction:
    """Exact value of one multiple double given its limbs."""
    return sum((Fraction(float(v)) for v in limbs), Fraction(0))


class CF:
    """An exact complex rational re + im i (pairs of Fractions).  abs() is the
    L1 modulus |re| + |im|, which bounds both parts of a product:
    |re(xy)|, |im(xy)| <= abs(x) abs(y)."""

    __slots__ = ("re", "im")

    def __init__(self, re, im=Fraction(0)):
        self.re, self.im = Fraction(re), Fraction(im)

    @staticmethod
    def _lift(v):
        return v if isinstance(v, CF) else CF(v)

    def __add__(self, o):
        o = CF._lift(o)
        return CF(self.re + o.re, self.im + o.im)

    __radd__ = __add__

    def __sub__(self, o):
        o = CF._lift(o)
        return CF(self.re - o.re, self.im - o.im)

    def __mul__(self, o):
        o = CF._lift(o)
        return CF(self.re * o.re - self.im * o.im, self.re * o.im + self.im * o.re)

    __rmul__ = __mul__

    def __abs__(self):
        return abs(self.re) + abs(self.im)

    def __eq__(self, o):
        o = CF._lift(o)
        return self.re == o.re and self.im == o.im

    def conj(self):
        return CF(self.re, -self.im)


def planar_to_exact(arr):
    """[m][count][d+1] planar limbs -> list (count) of lists (d+1) of Fractions;
    complex [2][m][count][d+1] -> lists of CF."""
    if arr.ndim == 4:
        re, im = planar_to_exact(arr[0]), planar_to_exact(arr[1])
        return [[CF(a, b) for a, b in zip(r, i)] for r, i in zip(re, im)]
    m, count, d1 = arr.shape
    return [[md_value(arr[:, s, c]) for c in range(d1)] for s in range(count)]


def series_to_exact(arr):
    """[m][d+1] -> list of Fractions."""
    return [md_value(arr[:, c]) for c in range(arr.shape[1])]


def smul(x, y):
    """Truncated product of two exact series of equal length."""
    d1 = len(x)
    return [sum((x[i] * y[k - i] for i in range(k + 1)), Fraction(0)) for k in range(d1)]


def sadd(x, y):
    return [a + b for a, b in zip(x, y)]


def spow(x, e):
    """x^e, truncated, by repeated products (e >= 0)."""
    out = [Fraction(1)] + [Fraction(0)] * (len(x) - 1)
    for _ in range(e):
        out = smul(out, x)
    return out


def poly_exact(supports, a, z, exps=None):
    """Exact value and gradient of p = a_0 + sum_k a_k prod_{j in S_k} z_j^{e_{k,j}}.

    a: list of N+1 exact series (a_0 first); z: list of n exact series;
    exps: None (every exponent one) or per monomial a tuple of exponents.
    Returns (value, [grad_0, ..., grad_{n-1}]).
    """
    d1 = len(a[0])
    zero = [Fraction(0)] * d1
    value = list(a[0])
    grad = [list(zero) for _ in z]
    for k, sup in enumerate(supports):
        ek = exps[k] if exps is not None else (1,) * len(sup)
        term = list(a[k + 1])
        for v, e in zip(sup, ek):
            term = smul(term, spow(z[v], e))
        value = sadd(value, term)
        for i, ei in zip(sup, ek):
            g = [c * ei for c in a[k + 1]]
            for v, e in zip(sup, ek):
                g = smul(g, spow(z[v], e - 1 if v == i else e))
            grad[i] = sadd(grad[i], g)
    return value, grad


def poly_magnitude(supports, a, z, exps=None):
    """The same computation on |coefficients|: the magnitude series used by the error bound."""
    aa = [[abs(c) for c in s] for s in a]
    zz = [[abs(c) for c in s] for s in z]
    return poly_exact(supports, aa, zz, exps)


def workload_exact(w):
    """Exact value/gradient and magnitudes for a workloads.Workload."""
    a = planar_to_exact(w.coeff)
    z = planar_to_exact(w.z)
    sup = w.supports()
    exps = None
    if getattr(w, "exps", None) is not None:
        exps, pos = [], 0
        for s_ in sup:
            exps.append(tuple(int(e) for e in w.exps[pos:pos + len(s_)]))
            pos += len(s_)
    return poly_exact(sup, a, z, exps), poly_magnitude(sup, a, z, exps)


def bound(m: int, d: int) -> Fraction:
    """Relative bound 4(d+1) 2^(-52m) per coefficient, relative to the magnitude series."""
    return Fraction(4 * (d + 1), 2 ** (52 * m))


def max_scaled_error(got_planar, exact, mag):
    """max_k |got_k - exact_k| / mag_k over coefficients with mag_k > 0 (got: [m][d+1]);
    complex got ([2][m][d+1]) against CF exact values: both parts, each against mag_k."""
    if got_planar.ndim == 3:
        exact = [CF._lift(e) for e in exact]
        return max(max_scaled_error(got_planar[0], [e.re for e in exact], mag),
                   max_scaled_error(got_planar[1], [e.im for e in exact], mag))
    worst = Fraction(0)
    for c in range(got_planar.shape[1]):
        g = md_value(got_planar[:, c])
        err = abs(g - exact[c])
        if mag[c] == 0:
            if err != 0:
                return Fraction(10 ** 9)
            continue
        worst = max(worst, err / mag[c])
    return worst


def permutation_symmetry_holds(eval_workload, m: int, d: int, seed: int) -> bool:
    """p1 (every product of four of 16 variables) with one coefficient series
    shared by all monomials is a symmetric function of its variables.  So
    evaluating at the permuted inputs z'_i = z_{pi(i)} must give the same value
    and dp/dz'_i = dp/dz_{pi(i)} at the original inputs.  The summation order
    differs between the two runs, so each result is compared within twice the
    bound 4(d+1) 2^(-52m), relative to the magnitude series (computed here in
    float64 from the leading limbs, padded for its own rounding).  Exact
    differences of the multiple doubles are taken with fractions."""
    import dataclasses
    from paper_2101_10881_amd import workloads as W
    w = W.p1(seed=seed, m=m, d=d)
    w.coeff[:, 2:, :] = w.coeff[:, 1:2, :]            # a_1 = ... = a_N; a_0 stays its own
    pi = np.random.default_rng(seed).permutation(w.n)
    w_perm = dataclasses.replace(w, z=np.ascontiguousarray(w.z[:, pi, :]))
    val, grad = eval_workload(w)
    val_p, grad_p = eval_workload(w_perm)
    # magnitude series from |leading limbs|
    trunc = lambda x, y: np.convolve(x, y)[: d + 1]
    a = np.abs(w.coeff[0])
    z = np.abs(w.z[0])
    mag_val = a[0].copy()
    mag_grad = np.zeros((w.n, d + 1))
    for k, s in enumerate(w.supports()):
        t = a[k + 1]
        for j in s:
            t = trunc(t, z[j])
        mag_val += t
        for i in s:
            g = a[k + 1]
            for j in s:
                if j != i:
                    g = trunc(g, z[j])
            mag_grad[i] += g
    tol = 2 * bound(m, d) * Fraction(1 + 2 ** -30)

    def close(x, y, mag):
        for c in range(d + 1):
            if abs(md_value(x[:, c]) - md_value(y[:, c])) > tol * Fraction(float(mag[c])):
                return False
        return True

    if not close(val, val_p, mag_val):
        return False
    return all(close(grad_p[:, i, :], grad[:, pi[i], :], mag_grad[pi[i]]) for i in range(w.n))

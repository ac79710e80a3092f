"""Seeded synthetic workloads: polynomial supports and multiple-double input series.

This module is shared by the test suite (which feeds the same arrays to the
CPU oracle and to the HIP path) and by the benchmark.  It holds no
multiple-double arithmetic: limbs are drawn directly in a normalised form
(each lower limb is a uniform multiple of half an ulp of the limb above it),
so no renormalisation is needed and nothing here depends on the method.

Layouts (all C-contiguous float64 numpy arrays, limb 0 most significant):

* ``coeff``: ``[m][N+1][d+1]`` -- a_0 first, then a_1..a_N (eq. (3) of the paper);
* ``z``:     ``[m][n][d+1]``   -- the n input series z_1..z_n;
* complex workloads carry a leading axis of two, real parts then imaginary
  parts (``[2][m][N+1][d+1]`` and ``[2][m][n][d+1]``), the separate real and
  imaginary arrays of Sections 2 and 5;
* supports: ``nvars[N]`` (int32) and ``vars[sum nvars]`` (int32, 0-based,
  strictly increasing inside each monomial);
* ``exps``: None (every exponent one), or ``[sum nvars]`` int32 exponents
  aligned with ``vars`` (monomial k is a_k prod_j z_{i_j}^{e_j}).

The shapes follow the paper's test polynomials (Section 6.1, Table 2):
p1 = all 1820 products of four of 16 variables; p2 = 128 monomials of 64 of
128 variables; p3 = all 8128 products of two of 128 variables.
"""
from __future__ import annotations

import itertools
from dataclasses import dataclass, field

import numpy as np

SUPPORTED_M = (1, 2, 3, 4, 5, 8, 10)


@dataclass
class Workload:
    """One polynomial instance with its input series."""

    name: str
    m: int
    d: int
    n: int
    nvars: np.ndarray  # int32 [N]
    vars: np.ndarray   # int32 [sum nvars]
    coeff: np.ndarray  # float64 [m][N+1][d+1], or [2][m][N+1][d+1] (complex)
    z: np.ndarray      # float64 [m][n][d+1], or [2][m][n][d+1] (complex)
    meta: dict = field(default_factory=dict)
    exps: np.ndarray = None  # int32 [sum nvars], or None: every exponent one

    @property
    def N(self) -> int:
        return int(self.nvars.shape[0])

    @property
    def cx(self) -> bool:
        """Complex coefficients and inputs (real and imaginary parts)."""
        return self.coeff.ndim == 4

    def supports(self):
        """List of tuples of 0-based variable indices, one per monomial."""
        out, pos = [], 0
        for k in range(self.N):
            nk = int(self.nvars[k])
            out.append(tuple(int(v) for v in self.vars[pos:pos + nk]))
            pos += nk
        return out


def md_series(rng: np.random.Generator, count: int, m: int, d: int) -> np.ndarray:
    """Draw ``count`` random series of d+1 m-double coefficients, shape [m][count][d+1].

    Limb 0 is uniform in [-1, 1).  Limb k (k >= 1) is u * h where u is uniform in
    [-1, 1) and h is half an ulp of limb k-1 (zero below a zero limb), so
    |x_k| <= ulp(x_{k-1}) / 2: a normalised expansion whose limb k is of order
    2^(-53k), as the workload recipe asks, without any rounding arithmetic.
    Scaling by a power of two is exact, so every limb is an exact double.
    """
    out = np.empty((m, count, d + 1), dtype=np.float64)
    out[0] = rng.uniform(-1.0, 1.0, size=(count, d + 1))
    for k in range(1, m):
        u = rng.uniform(-1.0, 1.0, size=(count, d + 1))
        prev = out[k - 1]
        _, ex = np.frexp(prev)           # prev = f * 2^ex, 0.5 <= |f| < 1, so ulp = 2^(ex-53)
        half_ulp = np.ldexp(1.0, ex - 54)
        limb = np.ldexp(u, ex - 54)      # exact: u times a power of two
        limb = np.where(prev == 0.0, 0.0, limb)
        # guard the (practically impossible) subnormal range so limbs stay exact
        limb = np.where(half_ulp < 2.0 ** -1000, 0.0, limb)
        out[k] = limb
    return np.ascontiguousarray(out)


def _pack_supports(supports):
    nvars = np.array([len(s) for s in supports], dtype=np.int32)
    flat = [v for s in supports for v in s]
    vars_ = np.array(flat, dtype=np.int32) if flat else np.zeros(0, dtype=np.int32)
    return nvars, vars_


def random_supports(rng: np.random.Generator, n: int, N: int, nk) -> list:
    """N supports; monomial k has nk[k] distinct variables drawn uniformly, sorted."""
    out = []
    for k in range(N):
        s = np.sort(rng.choice(n, size=int(nk[k]), replace=False))
        out.append(tuple(int(v) for v in s))
    return out


def all_subsets(n: int, r: int) -> list:
    """Every r-subset of n variables in lexicographic order (p1: n=16, r=4)."""
    return [tuple(c) for c in itertools.combinations(range(n), r)]


def _draw_series(rng, N, n, m, d, cx):
    """a_0..a_N, then z_1..z_n; complex: then the imaginary parts, in the same order."""
    coeff = md_series(rng, N + 1, m, d)
    z = md_series(rng, n, m, d)
    if cx:
        coeff = np.ascontiguousarray(np.stack([coeff, md_series(rng, N + 1, m, d)]))
        z = np.ascontiguousarray(np.stack([z, md_series(rng, n, m, d)]))
    return coeff, z


def make(name: str, m: int, d: int, n: int, supports, seed: int = 1, meta=None, cx: bool = False) -> Workload:
    """Build a workload from explicit supports: a_0..a_N first, then z_1..z_n
    (complex: the real parts are those of the real workload with the same seed)."""
    if m not in SUPPORTED_M:
        raise ValueError(f"m={m} not in {SUPPORTED_M}")
    rng = np.random.default_rng(seed)
    nvars, vars_ = _pack_supports(supports)
    coeff, z = _draw_series(rng, len(supports), n, m, d, cx)
    return Workload(name, m, d, n, nvars, vars_, coeff, z, dict(meta or {}))


def random_poly(name: str, m: int, d: int, n: int, N: int, nk, seed: int = 1, cx: bool = False) -> Workload:
    """Supports drawn first from the same generator, then the series."""
    rng = np.random.default_rng(seed)
    if np.isscalar(nk):
        nk = [int(nk)] * N
    supports = random_supports(rng, n, N, nk)
    nvars, vars_ = _pack_supports(supports)
    coeff, z = _draw_series(rng, N, n, m, d, cx)
    return Workload(name, m, d, n, nvars, vars_, coeff, z, {"seed": seed})


# ----- the benchmark workloads ----------------------------------------------------------

def with_exponents(w: Workload, emax: int, seed: int = 1, frac: float = 0.5) -> Workload:
    """The same workload with exponents: each occurrence of a variable gets,
    with probability frac, an exponent drawn uniformly from 2..emax (else 1)."""
    rng = np.random.default_rng(seed)
    q = w.vars.shape[0]
    e = np.where(rng.uniform(size=q) < frac, rng.integers(2, emax + 1, size=q), 1).astype(np.int32)
    return Workload(w.name + f"_e{emax}", w.m, w.d, w.n, w.nvars, w.vars, w.coeff, w.z, dict(w.meta), e)


def _cname(name, cx):
    return name + "_complex" if cx else name


def rand3(seed: int = 1, cx: bool = False) -> Workload:
    """Double double, d=8: n=8, 16 monomials of 3 distinct variables each."""
    return random_poly(_cname("rand3_2d_d8_n8_N16", cx), 2, 8, 8, 16, 3, seed, cx)


def p1(seed: int = 1, m: int = 10, d: int = 152, cx: bool = False) -> Workload:
    """p1 (all 1820 4-subsets of 16 variables); deca double at d=152 is the
    workload of Table 3, octo double at d=32 the differentiation one."""
    return make(_cname(f"p1_{m}d_d{d}", cx), m, d, 16, all_subsets(16, 4), seed, {"seed": seed}, cx)


def p2(seed: int = 1, m: int = 4, d: int = 64, cx: bool = False) -> Workload:
    """p2 shape: n=128, 128 monomials of 64 distinct variables, quad double, d=64."""
    return random_poly(_cname(f"p2_{m}d_d{d}", cx), m, d, 128, 128, 64, seed, cx)


def p3(seed: int = 1, m: int = 10, d: int = 152, cx: bool = False) -> Workload:
    """p3: all 8128 products of two of 128 variables."""
    return make(_cname(f"p3_{m}d_d{d}", cx), m, d, 128, all_subsets(128, 2), seed, {"seed": seed}, cx)


def batch_instances(count: int = 512, seed: int = 1):
    """Instance parameters of the batched workload (drawn, not built)."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        n = int(rng.integers(8, 65))
        N = int(rng.integers(16, 1025))
        d = int(rng.choice([8, 16, 32, 64, 128]))
        m = int(rng.choice([2, 4]))
        nk = rng.integers(2, 9, size=N)
        nk = np.minimum(nk, n)
        out.append(dict(n=n, N=N, d=d, m=m, nk=nk.astype(np.int32), seed=int(rng.integers(1, 2**31 - 1))))
    return out


def upstream_adjoint(m: int, d: int, seed: int = 1) -> np.ndarray:
    """Upstream adjoint series: leading limb uniform in [-1, 1), lower limbs zero; [m][d+1]."""
    rng = np.random.default_rng(seed)
    out = np.zeros((m, d + 1), dtype=np.float64)
    out[0] = rng.uniform(-1.0, 1.0, size=d + 1)
    return out


def mixed_batch(count: int = 512, seed: int = 1):
    """The batched workload: `count` instances with parameters drawn by
    batch_instances(count, seed), each built from its own seed."""
    out = []
    for q, par in enumerate(batch_instances(count, seed)):
        out.append(random_poly(f"batch{q}_m{par['m']}_d{par['d']}", par["m"], par["d"], par["n"], par["N"],
                               par["nk"], par["seed"]))
    return out

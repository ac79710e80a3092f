"""The oracle's pins are sensitive: plant one plausible mistake at a time in a
copy of the oracle (on the CPU), rebuild it, and check that the exact
rational pins reject it.  The mistakes cover a wrong variable index, a wrong
backward-product index (including the literal index printed in Section 3's
statement list, which the design reads as b_{n-2-j}), dropped terms in the
multiple-double operations, a sign error in two_sum, a dropped carry in the
addition tree, a mis-assigned partial derivative, in the complex product a
lost sign, a wrong cross term and a dropped imaginary sum, and for general
exponents a dropped or wrong exponent factor, a wrong power table and a
skipped common factor.
"""
import os
import subprocess

import numpy as np
import pytest

import exact_ref as E
from oracle import build as obuild
from oracle import oracle as O
from paper_2101_10881_amd import workloads as W

MUTANTS = {
    "forward_chain_wrong_variable": ("conv(m, cx, d, F(j - 1), ZS(I(j)), F(j), tmp);",
                                     "conv(m, cx, d, F(j - 1), ZS(I(j - 1)), F(j), tmp);"),
    "cross_product_literal_index": ("conv(m, cx, d, F(j), B(n - 2 - j), C(j), tmp);",
                                    "conv(m, cx, d, F(j), B(n - 3 - j), C(j), tmp);"),
    "cross_product_off_by_one": ("conv(m, cx, d, F(j), B(n - 2 - j), C(j), tmp);",
                                 "conv(m, cx, d, F(j), B(n - 1 - j), C(j), tmp);"),
    "backward_start_wrong": ("conv(m, cx, d, ZS(I(n)), ZS(I(n - 1)), B(1), tmp);",
                             "conv(m, cx, d, ZS(I(n)), ZS(I(n - 2)), B(1), tmp);"),
    "md_add_drops_last_limb": ("for (int k = 0; k < m; ++k)\n        deposit(m, S, k, y[k]);",
                               "for (int k = 0; k < m - 1; ++k)\n        deposit(m, S, k, y[k]);"),
    "md_mul_drops_low_parts": ("deposit(m, S, k + 1, E[k]);", "(void)E[k];"),
    "md_mul_drops_last_level": ("S[m - 1] = fma(x[i], y[m - 1 - i], S[m - 1]);", "(void)i;"),
    "two_prod_no_error": ("*e = fma(a, b, -pp);", "*e = 0.0;"),
    "two_sum_sign": ("double err = (a - (ss - bb)) + (b - bb);", "double err = (a - (ss - bb)) - (b - bb);"),
    "renorm_skips_top_down": ("two_sum(e, u[j + 1], &r[j], &e);", "r[j] = u[j + 1];"),
    "conv_skips_first_term": ("for (int i = 1; i <= k; ++i) {\n            coef_mul(m, cx, x + (size_t)i * w",
                              "for (int i = 2; i <= k; ++i) {\n            coef_mul(m, cx, x + (size_t)i * w"),
    "tree_drops_carry": ("        if (r % 2)\n            live[w++] = live[r - 1];\n        r = w;\n    }\n    free(live);\n}\n\n/* The schedule",
                         "        r = w;\n    }\n    free(live);\n}\n\n/* The schedule"),
    "complex_real_part_sign": ("ii[l] = -ii[l];", "ii[l] = ii[l];"),
    "complex_cross_term_wrong": ("md_mul(m, x + m, y, ir);", "md_mul(m, x, y, ir);"),
    "complex_add_drops_imaginary": ("md_add(m, x + m, y + m, z + m);", "memcpy(z + m, x + m, sizeof(double) * m);"),
    "exponent_scaling_dropped": ("coef_scale(m, cx, der[j] + (size_t)c * nl, e[j]);", "(void)c;"),
    "exponent_scaling_off_by_one": ("coef_scale(m, cx, der[j] + (size_t)c * nl, e[j]);",
                                    "coef_scale(m, cx, der[j] + (size_t)c * nl, e[j] - 1);"),
    "power_table_wrong_base": ("conv(m, cx, d, P1 + (size_t)(p - 2) * S, Z + (size_t)i * S,",
                               "conv(m, cx, d, P1, Z + (size_t)i * S,"),
    "common_factor_skipped": ("conv(m, cx, d, F, Pt + (powoff[v[j]] + (size_t)(e[j] - 2)) * S, F,",
                              "if (0) conv(m, cx, d, F, Pt + (powoff[v[j]] + (size_t)(e[j] - 2)) * S, F,"),
    "last_partial_misassigned": ("memcpy(der[n - 1], F(n - 1), sizeof(double) * S);",
                                 "memcpy(der[n - 1], F(n - 2), sizeof(double) * S);"),
}


def _pins_pass(L) -> bool:
    """Run a battery of exact pins against library L; False as soon as one fails."""
    cases = []
    for m in (1, 2, 3):
        for seed in range(1, 6):
            rng = np.random.default_rng(77 * m + seed)
            n = int(rng.integers(2, 7))
            N = int(rng.integers(1, 7))
            nk = rng.integers(1, n + 1, size=N)
            cases.append(W.random_poly("mut", m, int(rng.integers(1, 4)), n, N, nk, seed))
        cases.append(W.make("ex", m, 3, 6, [(0, 2, 5), (0, 1, 4, 5), (1, 2, 3)], seed=4))
        cases.append(W.make("n5", m, 2, 7, [(0, 2, 3, 5, 6)], seed=9))
        cases.append(W.make("ex_cx", m, 2, 6, [(0, 2, 5), (0, 1, 4, 5), (1, 2, 3)], seed=4, cx=True))
        ex = W.make("ex_e", m, 3, 6, [(0, 2, 5), (0, 1, 4, 5), (1, 2, 3), (3,)], seed=6)
        ex.exps = np.array([2, 1, 4, 1, 3, 1, 2, 5, 1, 1, 4], dtype=np.int32)
        cases.append(ex)
    for w in cases:
        val, grad = O.eval_workload(w, L=L)
        (ev, eg), (mv, mg) = E.workload_exact(w)
        b = E.bound(w.m, w.d)
        if E.max_scaled_error(val, ev, mv) > b:
            return False
        for i in range(w.n):
            if E.max_scaled_error(grad[..., i, :], eg[i], mg[i]) > b:
                return False
    return True


def test_unmutated_oracle_passes_battery(oracle_lib):
    assert _pins_pass(O.lib())


def _build_mutant(tmp_path, name):
    src = open(obuild.SRC).read()
    old, new = MUTANTS[name]
    assert src.count(old) >= 1, f"mutation site for {name} not found"
    mutant = src.replace(old, new, 1)
    c = tmp_path / "mutant.c"
    c.write_text(mutant)
    so = tmp_path / "libmutant.so"
    subprocess.run(["gcc", *obuild.CFLAGS, str(c), "-o", str(so), "-lm"], check=True)
    return O.bind(str(so))


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(tmp_path, name):
    L = _build_mutant(tmp_path, name)
    assert not _pins_pass(L), f"planted mistake {name} was not caught"


@pytest.mark.parametrize("name", ["forward_chain_wrong_variable", "backward_start_wrong",
                                  "cross_product_off_by_one", "last_partial_misassigned"])
def test_structural_mutant_breaks_permutation_symmetry(tmp_path, name):
    """The symmetry pin, with no exact reference at all, also rejects the
    mistakes that depend on a variable's position inside its monomial."""
    L = _build_mutant(tmp_path, name)
    assert not E.permutation_symmetry_holds(lambda w: O.eval_workload(w, L=L), 2, 3, seed=3)

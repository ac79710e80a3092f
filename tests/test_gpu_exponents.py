"""GPU parity for general exponents (Section 3: a table of powers and the
common factor a_k prod z^(e-1), derivatives scaled by the exponent): the HIP
path against the CPU oracle, bit for bit, real and complex."""
import numpy as np
import pytest

from gpu_util import assert_bitexact, run_gpu
from paper_2101_10881_amd import workloads as W

pytestmark = pytest.mark.gpu


def _compare(oracle_lib, w):
    print(f"eval_and_diff {w.name}: m={w.m} d={w.d} n={w.n} N={w.N} cx={w.cx} "
          f"max exponent {int(w.exps.max()) if w.exps is not None and w.exps.size else 1}", flush=True)
    want_v, want_g = oracle_lib.eval_workload(w)
    got_v, got_g = run_gpu(w)
    assert_bitexact(got_v, want_v, f"{w.name} value")
    assert_bitexact(got_g, want_g, f"{w.name} gradient")


@pytest.mark.parametrize("m", W.SUPPORTED_M)
@pytest.mark.parametrize("cx", [False, True])
def test_random_polynomials_with_exponents_bitexact(oracle_lib, m, cx):
    for seed in range(2):
        rng = np.random.default_rng(9100 + 10 * m + seed)
        n = int(rng.integers(1, 10))
        N = int(rng.integers(1, 25))
        d = int(rng.choice([0, 3, 8, 17]))
        nk = rng.integers(1, min(n, 6) + 1, size=N)
        w = W.random_poly(f"exp_m{m}_s{seed}", m, d, n, N, nk, seed, cx=cx)
        _compare(oracle_lib, W.with_exponents(w, int(rng.integers(2, 7)), seed=seed))


def test_exponent_edge_cases(oracle_lib):
    w = W.make("univariate_powers", 4, 12, 3, [(0,), (0,), (1,), (0, 2)], seed=3)
    w.exps = np.array([5, 1, 64, 2, 7], dtype=np.int32)     # n_k = 1 with and without a factor
    _compare(oracle_lib, w)
    w = W.make("shared_powers", 3, 9, 4, [(0, 1, 2, 3), (0, 2), (1, 3), (0, 1, 3)], seed=6, cx=True)
    w.exps = np.array([3, 2, 4, 1, 3, 4, 2, 5, 1, 1, 2], dtype=np.int32)
    _compare(oracle_lib, w)


def test_p1_with_exponents(oracle_lib):
    # p1's supports in quad double at d = 32, half of the occurrences raised to 2..4
    _compare(oracle_lib, W.with_exponents(W.p1(m=4, d=32), 4, seed=1))

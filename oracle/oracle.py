"""ctypes wrapper around oracle/liboracle.so (see oracle.c for what it computes).

TEST INFRASTRUCTURE ONLY.  All arrays are float64 numpy arrays in the
limb-planar layouts of the C file: series batches [m][count][d+1]; complex
data has a leading axis of two (real parts, then imaginary parts), which is
the C file's 2m planes.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int)
_lp = ctypes.POINTER(ctypes.c_long)


def bind(path):
    """Load an oracle shared library from ``path`` and declare its signatures."""
    L = ctypes.CDLL(path)
    L.oracle_eval_and_diff.argtypes = [ctypes.c_int] * 4 + [_ip, _ip, _dp, _dp, _dp, _dp, ctypes.c_int]
    L.oracle_eval_and_diff_general.argtypes = [ctypes.c_int] * 5 + [_ip, _ip, _ip, _dp, _dp, _dp, _dp, ctypes.c_int]
    L.oracle_md_op.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_long, _dp, _dp, _dp]
    L.oracle_eft.argtypes = [ctypes.c_int, ctypes.c_long, _dp, _dp, _dp, _dp]
    L.oracle_op_counts.argtypes = [ctypes.c_int, ctypes.c_int, _lp]
    L.oracle_tree_schedule.argtypes = [ctypes.c_int, _ip, _ip, ctypes.c_int]
    L.oracle_eval_adjoint.argtypes = [ctypes.c_int] * 4 + [_ip, _ip, _dp, _dp, _dp, _dp, _dp, ctypes.c_int]
    return L


def lib():
    global _LIB
    if _LIB is None:
        path = os.path.join(_HERE, "liboracle.so")
        if not os.path.exists(path):
            from . import build as _b
            _b.build()
        _LIB = bind(path)
    return _LIB


def _d(a):
    return a.ctypes.data_as(_dp)


def _i(a):
    return a.ctypes.data_as(_ip)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def eval_and_diff(m, d, n, nvars, vars_, coeff, z, nthreads=0, L=None, exps=None):
    """Return (value [m][d+1], grad [m][n][d+1]); complex inputs ([2][m][...])
    give complex outputs ([2][m][d+1], [2][m][n][d+1]).  exps: None (every
    exponent one) or one exponent per entry of vars_.
    ``L``: an alternative library from bind()."""
    nvars, vars_ = _i32(nvars), _i32(vars_)
    N = int(nvars.shape[0])
    coeff, z = _f64(coeff), _f64(z)
    cx = coeff.ndim == 4
    lead = (2, m) if cx else (m,)
    assert coeff.shape == lead + (N + 1, d + 1), coeff.shape
    assert z.shape == lead + (n, d + 1), z.shape
    if exps is not None:
        exps = _i32(exps)
        assert exps.shape == vars_.shape
    value = np.empty(lead + (d + 1,))
    grad = np.empty(lead + (n, d + 1))
    rc = (L or lib()).oracle_eval_and_diff_general(m, int(cx), d, n, N, _i(nvars), _i(vars_),
                                                   _i(exps) if exps is not None else None, _d(coeff), _d(z),
                                                   _d(value), _d(grad), int(nthreads))
    if rc != 0:
        raise ValueError("oracle: invalid polynomial description")
    return value, grad


def eval_workload(w, nthreads=0, L=None):
    return eval_and_diff(w.m, w.d, w.n, w.nvars, w.vars, w.coeff, w.z, nthreads, L, getattr(w, "exps", None))


def md_op(op, x, y, L=None):
    """op 'add' or 'mul' on planar [m][count] arrays; 'cadd' or 'cmul' on
    complex [2][m][count] arrays."""
    x, y = _f64(x), _f64(y)
    code = {"add": 0, "mul": 1, "cadd": 2, "cmul": 3}[op]
    m, count = x.shape[-2], x.shape[-1]
    assert x.shape == y.shape and x.ndim == (3 if code >= 2 else 2)
    z = np.empty_like(x)
    if (L or lib()).oracle_md_op(code, m, count, _d(x), _d(y), _d(z)) != 0:
        raise ValueError("oracle: bad md op")
    return z


def eft(op, a, b):
    a, b = _f64(a), _f64(b)
    hi, lo = np.empty_like(a), np.empty_like(a)
    lib().oracle_eft({"two_sum": 0, "two_prod": 1}[op], a.size, _d(a), _d(b), _d(hi), _d(lo))
    return hi, lo


def op_counts(op, m):
    """{add, mul, fma, two_sum} double-operation counts of one md op."""
    c = np.zeros(4, dtype=np.int64)
    lib().oracle_op_counts({"add": 0, "mul": 1}[op], m, c.ctypes.data_as(_lp))
    return dict(add=int(c[0]), mul=int(c[1]), fma=int(c[2]), two_sum=int(c[3]))


def tree_schedule(length):
    """Rounds of (input index, updated index) pairs of the pairwise tree sum."""
    pairs = np.zeros(2 * max(length, 1), dtype=np.int32)
    sizes = np.zeros(64, dtype=np.int32)
    nr = lib().oracle_tree_schedule(int(length), _i(pairs), _i(sizes), 64)
    out, pos = [], 0
    for r in range(nr):
        out.append([(int(pairs[2 * (pos + p)]), int(pairs[2 * (pos + p) + 1])) for p in range(sizes[r])])
        pos += int(sizes[r])
    return out


def eval_adjoint(m, d, n, nvars, vars_, z, grad, ybar, nthreads=0, L=None):
    """Adjoints (coeff_bar [m][N+1][d+1], z_bar [m][n][d+1]) of L = sum_t ybar_t p_t.
    grad: the oracle's gradient for the same inputs."""
    nvars, vars_ = _i32(nvars), _i32(vars_)
    N = int(nvars.shape[0])
    z, grad, ybar = _f64(z), _f64(grad), _f64(ybar)
    assert ybar.shape == (m, d + 1) and z.shape == (m, n, d + 1) and grad.shape == z.shape
    cbar = np.empty((m, N + 1, d + 1))
    zbar = np.empty((m, n, d + 1))
    rc = (L or lib()).oracle_eval_adjoint(m, d, n, N, _i(nvars), _i(vars_), _d(z), _d(grad), _d(ybar), _d(cbar),
                                          _d(zbar), int(nthreads))
    if rc != 0:
        raise ValueError("oracle: invalid polynomial description")
    return cbar, zbar


def adjoint_workload(w, ybar, nthreads=0, L=None):
    """Forward gradient then adjoints, for a workloads.Workload."""
    _, grad = eval_workload(w, nthreads, L)
    return eval_adjoint(w.m, w.d, w.n, w.nvars, w.vars, w.z, grad, ybar, nthreads, L)

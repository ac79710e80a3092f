"""Work accounting for the benchmark: double-operation counts of the
multiple-double operations and of the convolution / addition jobs.

Counts are closed forms of the project's multiple-double algorithms
(two_sum = 6 additions/subtractions, two_prod = 1 multiplication + 1 FMA):

* md_add(m): y_k is added at level k of m running sums; every level above
  the last costs one two_sum, the last level one plain addition; then the
  two renormalisation passes ((m-1) + (m-2) two_sums for m >= 2).
* md_mul(m): exact products x_i*y_j (two_prod) for levels i+j <= m-2, plain
  products/FMAs for levels m-1 and m, every exact part deposited as in md_add,
  then the same renormalisation.

FLOPs count an FMA as two operations, like the FP64 peak they are compared
with; "instructions" counts each FP64 VALU operation once.

Per convolution job (eq. (1) of the paper, computed without the zero terms):
(d+1)(d+2)/2 md_mul and d(d+1)/2 md_add.  Per addition job: d+1 md_add.
Complex series (cx=True): a complex multiplication is four md_mul and two
md_add, a complex addition two md_add.
The paper's own convention (Section 6.2) charges the zero-inserted square,
(d+1)^2 md_mul and d(d+1) md_add, at 3089 and 397 double operations per
deca-double multiplication and addition; ``paper_convention`` reproduces it.
"""
from __future__ import annotations


def _renorm_two_sums(m: int) -> int:
    return 2 * m - 3 if m >= 2 else 0


def md_op_counts(op: str, m: int) -> dict:
    """{'add', 'mul', 'fma'} double operations of one md_add / md_mul."""
    if op == "add":
        ts = m * (m - 1) // 2 + _renorm_two_sums(m)
        return dict(add=6 * ts + m, mul=0, fma=0)
    if op == "mul":
        n_tp = (m - 1) + (m - 2) * (m - 1) // 2 if m >= 2 else 0
        ts_e = (m - 2) * (m - 1) // 2 if m >= 2 else 0
        ts_p = sum(k * (2 * m - 3 - 2 * k) for k in range(1, m - 1))
        adds_plain = (m - 1) + sum(2 * k for k in range(1, m - 1))
        ts = ts_e + ts_p + _renorm_two_sums(m)
        return dict(add=6 * ts + adds_plain, mul=n_tp + 1, fma=n_tp + 2 * (m - 1))
    raise ValueError(op)


def md_flops(op: str, m: int) -> int:
    c = md_op_counts(op, m)
    return c["add"] + c["mul"] + 2 * c["fma"]


def md_instructions(op: str, m: int) -> int:
    c = md_op_counts(op, m)
    return c["add"] + c["mul"] + c["fma"]


def conv_md_ops(d: int):
    """(md_mul, md_add) of one truncated convolution, zero terms skipped."""
    return (d + 1) * (d + 2) // 2, d * (d + 1) // 2


def coef_flops(op: str, m: int, cx: bool = False) -> int:
    """FLOPs of one coefficient multiplication or addition (real or complex)."""
    if not cx:
        return md_flops(op, m)
    if op == "mul":
        return 4 * md_flops("mul", m) + 2 * md_flops("add", m)
    return 2 * md_flops("add", m)


def conv_flops(m: int, d: int, cx: bool = False) -> int:
    nm, na = conv_md_ops(d)
    return nm * coef_flops("mul", m, cx) + na * coef_flops("add", m, cx)


def add_flops(m: int, d: int, cx: bool = False) -> int:
    return (d + 1) * coef_flops("add", m, cx)


def conv_bytes(m: int, d: int, cx: bool = False) -> int:
    """Algorithmic HBM bytes of one convolution job: read two series, write one."""
    return 3 * (d + 1) * m * 8 * (2 if cx else 1)


def add_bytes(m: int, d: int, cx: bool = False) -> int:
    return 3 * (d + 1) * m * 8 * (2 if cx else 1)


PAPER_DECA_COST = {"mul": 3089, "add": 397}


def paper_convention(n_conv: int, n_add: int, d: int) -> int:
    """Double operations as counted in Section 6.2 for deca doubles."""
    mul = n_conv * (d + 1) ** 2
    add = n_conv * d * (d + 1) + n_add * (d + 1)
    return mul * PAPER_DECA_COST["mul"] + add * PAPER_DECA_COST["add"]

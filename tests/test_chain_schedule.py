"""The chain launch on the host: lane schedules, their checker, chain plans.

A chain is a run of products where each job's first operand is the previous
job's output (Section 3: f_j = f_{j-1} * z_{i_j}, b_j = b_{j-1} * z_{i_{n-j}}).
The chain kernel overlaps a chain's products: coefficient i of a product is
final after its own i+1 terms, and the next product reads its first operand
in increasing i.  Those coefficients pass through LDS slots, ordered only by
a workgroup barrier after every `window` steps, so a schedule is correct
exactly when each read of a first-operand coefficient sees the previous
product's value.  Here a plain simulation of the kernel's memory (a read sees
what was committed at the last barrier; a read and a write of one LDS
coefficient between two barriers is a race) checks the schedules the planner
builds, independently of the library's own checker, and planted mistakes are
rejected by both.  Chain plans, run job by job in exact rationals, compute
the polynomial's value and gradient.
"""
from fractions import Fraction

import numpy as np
import pytest

import exact_ref as E
from paper_2101_10881_amd import mdpe
from paper_2101_10881_amd import workloads as W

IDLE = 0x7FFF


def _rows(codes):
    """Per thread: list of (start step, job or None, k, length)."""
    out = []
    for row in codes:
        t, items = 0, []
        for c in row:
            if c < 0:
                break
            j, k = int(c) >> 16, int(c) & 0xFFFF
            if j == IDLE:
                t += k + 1
                continue
            items.append((t, j, k))
            t += k + 1
        out.append((items, t))
    return out


def simulate(L, d, waves, window, ring, steps, codes):
    """Run the chain kernel's LDS traffic step by step; return '' or the first fault.

    Iteration s stores the coefficients whose last step is s and reads the
    first-operand coefficient of step s+1 (the prologue, iteration -1, reads
    step 0's).  A barrier follows iteration s when (s+1) % window == 0.
    """
    assert codes.shape[0] == 64 * waves
    rows = _rows(codes)
    done = {}
    events = {}   # iteration -> list of ("r", slot, pos, want) / ("w", slot, pos, tag)
    for items, end in rows:
        if end > steps:
            return "row longer than the steps"
        for (t, j, k) in items:
            if j >= L or k > d:
                return "code out of range"
            if (j, k) in done:
                return "coefficient twice"
            done[(j, k)] = t
            for i in range(k + 1):
                want = ("staged",) if j == 0 else (j - 1, i)
                events.setdefault(t + i - 1, []).append(("r", j % ring, i, want))
            if j + 1 < L:
                events.setdefault(t + k, []).append(("w", (j + 1) % ring, k, (j, k)))
    if len(done) != L * (d + 1):
        return "coefficient missing"
    committed = {(0, i): ("staged",) for i in range(d + 1)}
    touched_r, pending = set(), {}
    for it in range(-1, steps):
        for ev in events.get(it, []):
            kind, slot, pos, val = ev
            if kind == "r":
                if (slot, pos) in pending:
                    return f"iteration {it}: read and write of one coefficient between barriers"
                if committed.get((slot, pos)) != val:
                    return f"iteration {it}: read {committed.get((slot, pos))} where {val} is due"
                touched_r.add((slot, pos))
            else:
                if (slot, pos) in touched_r or (slot, pos) in pending:
                    return f"iteration {it}: write of a coefficient read or written between the same barriers"
                pending[(slot, pos)] = val
        if it == -1 or (it + 1) % window == 0:   # the staging barrier, then one per window
            committed.update(pending)
            pending.clear()
            touched_r.clear()
    # the stores of the last window are not read in the kernel
    return ""


@pytest.mark.parametrize("L, d", [(1, 0), (2, 0), (3, 1), (5, 8), (64, 64), (63, 64), (20, 130), (40, 31),
                                  (8, 200)])
@pytest.mark.parametrize("waves, window", [(4, 1), (4, 2), (4, 4), (8, 1), (8, 3), (12, 2), (16, 1)])
def test_schedules_pass_both_checks(L, d, waves, window):
    for ring in sorted({2, 3, max(2, min(L, 46)), max(2, L)}):
        codes, steps = mdpe.chain_schedule(L, d, waves, window, ring)
        assert steps % window == 0 and steps % 2 == 0
        mdpe.check_chain_schedule(L, d, waves, window, ring, steps, codes)
        assert simulate(L, d, waves, window, ring, steps, codes) == ""


def test_p2_shape_fills_the_lanes():
    # quad double p2 at d = 64: 64 products per chain, 2145 multiply-adds each;
    # on four wavefronts the chain takes under 600 steps (64 layers of one
    # job per wavefront take over 4000), over 90% of lane-steps doing work
    codes, steps = mdpe.chain_schedule(64, 64, 4, 2, 46)
    assert steps < 600
    assert 64 * 2145 / (256 * steps) > 0.9


def _first_job_step(codes, j, k):
    for r, row in enumerate(codes):
        t = 0
        for e, c in enumerate(row):
            if c < 0:
                break
            jj, kk = int(c) >> 16, int(c) & 0xFFFF
            if jj == j and kk == k:
                return r, e, t
            t += kk + 1
    raise KeyError((j, k))


def _plant(codes, how):
    c = codes.copy()
    if how == "early":
        # start coefficient 5 of product 3 one step earlier: take a step off the idle stretch before it
        r, e, t = _first_job_step(c, 3, 5)
        assert e > 0 and (int(c[r, e - 1]) >> 16) == IDLE
        g = (int(c[r, e - 1]) & 0xFFFF) + 1
        if g == 1:
            c[r, e - 1:-1] = c[r, e:].copy()
        else:
            c[r, e - 1] = (IDLE << 16) | (g - 2)
    elif how == "twice":
        r, e, _ = _first_job_step(c, 2, 4)
        r2 = (r + 1) % c.shape[0]
        end = int(np.argmax(c[r2] < 0))
        c[r2, end] = c[r, e]
    elif how == "missing":
        r, e, _ = _first_job_step(c, 4, 0)
        c[r, e] = (IDLE << 16) | 0
    elif how == "range":
        r, e, _ = _first_job_step(c, 1, 1)
        c[r, e] = (99 << 16) | 1
    return c


@pytest.mark.parametrize("how", ["early", "twice", "missing", "range"])
def test_planted_mistakes_are_rejected(how):
    L, d, waves, window, ring = 12, 20, 4, 2, 6
    codes, steps = mdpe.chain_schedule(L, d, waves, window, ring)
    bad = _plant(codes, how)
    with pytest.raises(mdpe.MdpeError) as e:
        mdpe.check_chain_schedule(L, d, waves, window, ring, steps, bad)
    assert e.value.code == mdpe.MDPE_EINVAL
    assert simulate(L, d, waves, window, ring, steps, bad) != ""


def _hand_schedule():
    """Three products of degree 1 on four wavefronts, a barrier every step:
    product 0's coefficient 1 starts late (step 20), while product 1's
    coefficient 0 is stored early (iteration 2) into the slot of product 2's
    first operand."""
    def idle(g):
        return (IDLE << 16) | (g - 1)

    rows = [[idle(20), (0 << 16) | 1],       # reads x_0, x_1 in iterations 19, 20; stores at 21
            [(0 << 16) | 0],                 # stored at 0
            [idle(2), (1 << 16) | 0],        # reads x_0 at 1 (stored at 0); stores at 2
            [idle(22), (1 << 16) | 1],       # reads x_1 at 22 (stored at 21); stores at 23
            [idle(4), (2 << 16) | 0],        # reads x_0 at 3 (stored at 2)
            [idle(24), (2 << 16) | 1]]       # reads x_1 at 24 (stored at 23)
    codes = np.full((256, 3), -1, dtype=np.int32)
    for r, row in enumerate(rows):
        codes[r, :len(row)] = row
    return codes, 26


def test_hand_schedule_needs_its_slots_and_window():
    codes, steps = _hand_schedule()
    mdpe.check_chain_schedule(3, 1, 4, 1, 3, steps, codes)
    assert simulate(3, 1, 4, 1, 3, steps, codes) == ""
    # two slots: product 1 overwrites product 0's first operand (slot 0) at
    # iteration 2, before the late read of iteration 19
    with pytest.raises(mdpe.MdpeError) as e:
        mdpe.check_chain_schedule(3, 1, 4, 1, 2, steps, codes)
    assert "overwritten" in str(e.value)
    assert simulate(3, 1, 4, 1, 2, steps, codes) != ""
    # a barrier every second step: the read of iteration 1 shares a window with the store of iteration 0
    with pytest.raises(mdpe.MdpeError) as e:
        mdpe.check_chain_schedule(3, 1, 4, 2, 3, steps, codes)
    assert "before the barrier" in str(e.value)
    assert simulate(3, 1, 4, 2, 3, steps, codes) != ""


def test_schedule_arguments_are_checked():
    with pytest.raises(mdpe.MdpeError):
        mdpe.chain_schedule(0, 4, 4, 1, 2)
    with pytest.raises(mdpe.MdpeError):
        mdpe.chain_schedule(4, 4, 6, 1, 2)      # 4, 8, 12 or 16 wavefronts
    with pytest.raises(mdpe.MdpeError):
        mdpe.chain_schedule(4, 4, 4, 1, 1)      # at least two slots


def _execute_exact(p, w):
    """Run the plan's convolution layers, scale and addition jobs on exact rationals."""
    A = [None] * p.info["n_series"]
    a = E.planar_to_exact(w.coeff)
    z = E.planar_to_exact(w.z)
    for s in range(w.N + 1):
        A[s] = a[s]
    for i in range(w.n):
        A[w.N + 1 + i] = z[i]
    for layer, t1, t2, t3 in p.conv_jobs():
        A[t3] = E.smul(A[t1], A[t2])
    for level, t1, t2 in p.add_jobs():
        A[t2] = E.sadd(A[t2], A[t1])
    out = p.outputs()
    return A[out[0]], [A[s] if s >= 0 else [Fraction(0)] * (w.d + 1) for s in out[1:]]


@pytest.mark.parametrize("nk, keep", [(3, False), (7, False), (12, False), (12, True), (2, False)])
def test_chain_plans_compute_the_definition(nk, keep):
    w = W.random_poly("chain", 1, 4, 14, 5, nk, seed=nk)
    flags = mdpe.MDPE_CHAIN_LAUNCH | (mdpe.MDPE_KEEP_MONOMIAL_VALUES if keep else 0)
    p = mdpe.Plan.for_workload(w, device=-1, flags=flags)
    i = p.info
    assert i["chain_layers"] >= 1 and i["chain_count"] >= 1 and i["chain_waves"] in (4, 8)
    val, grad = _execute_exact(p, w)
    (ev, eg), _ = E.workload_exact(w)
    assert val == ev
    assert grad == eg


def test_chain_rows_are_chains_over_staged_second_operands():
    w = W.p2(m=4, d=8)
    p = mdpe.Plan.for_workload(w, device=-1, flags=mdpe.MDPE_CHAIN_LAUNCH)
    i = p.info
    rows = p.chain_jobs()
    conv = p.conv_jobs()
    # forward (64 products) and backward (62 and b * a) chains of every monomial
    assert i["chain_count"] == 2 * w.N and i["chain_layers"] == 64
    assert len(rows) == w.N * (64 + 63)
    written = set(conv[:, 3].tolist())
    staged = 1 + w.N + w.n
    layers = {tuple(r[1:]): r[0] for r in conv}
    for c in range(i["chain_count"]):
        ch = rows[rows[:, 0] == c]
        assert list(ch[:, 1]) == list(range(len(ch)))
        assert ch[0, 2] < staged
        assert all(t2 not in written for t2 in ch[:, 3])
        assert all(ch[q, 2] == ch[q - 1, 4] for q in range(1, len(ch)))
        for q, (_, _, t1, t2, t3) in enumerate(ch):
            assert layers[(t1, t2, t3)] == q + 1
    # after the chains, every cross product in one layer; no product in place
    assert i["n_layers"] == 65
    assert not np.any(conv[:, 1] == conv[:, 3])
    sizes, _ = p.layer_sizes()
    assert sizes[64] == w.N * 62


def test_chain_launch_only_where_asked_or_worth_it():
    shallow = W.p1(m=2, d=8)
    with pytest.raises(mdpe.MdpeError) as e:
        mdpe.Plan.for_workload(W.make("one", 2, 4, 3, [(0,), (1,)], seed=1), device=-1,
                               flags=mdpe.MDPE_CHAIN_LAUNCH | mdpe.MDPE_STREAM_OPERANDS)
    assert e.value.code == mdpe.MDPE_EINVAL
    assert mdpe.Plan.for_workload(shallow, device=-1).info["chain_layers"] == 0
    assert mdpe.Plan.for_workload(W.p2(m=4, d=64), device=-1,
                                  flags=mdpe.MDPE_LAYER_LAUNCHES).info["chain_layers"] == 0


def test_chain_launch_default_at_one_and_two_doubles():
    # the layers after the chains (p2's cross products) are weighed as the plan
    # without the chain launch weighs its dealt steps; measured on MI355X, the
    # chain launch wins at one double for d = 31..152 (not at d = 127, 0.88 of
    # the dealt plan's time against an estimate of 0.98) and at two doubles for
    # every degree, d = 191 included (0.94 against 1.92 ms); at one double and
    # d = 191 it loses (7%)
    def chained(m, d):
        return mdpe.Plan.for_workload(W.p2(m=m, d=d), device=-1).info["chain_layers"] > 0
    assert all(chained(1, d) for d in (31, 63, 95, 152))
    assert not chained(1, 191)
    assert all(chained(2, d) for d in (31, 63, 95, 127, 152, 191))

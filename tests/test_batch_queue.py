"""Host-only checks of the batched executor's task queue (no GPU):
every job and addition item is covered exactly once, each instance's tasks
appear in pipeline order, and every task waits only for tasks of its own
instance that come earlier in the queue -- the property that makes the
persistent kernel deadlock-free."""
import numpy as np
import pytest

from paper_2101_10881_amd import mdpe
from paper_2101_10881_amd import workloads as W


def _batch(ws, tiles=None):
    plans = [mdpe.Plan.for_workload(w, device=-1) for w in ws]
    return plans, mdpe.Batch(plans, tiles)


@pytest.mark.parametrize("tiles", [None, [{"m": 2, "d": 8, "jobs_per_group": 5, "groups_per_task": 3,
                                           "add_items_per_task": 100}]])
def test_queue_covers_and_orders(tiles):
    rng = np.random.default_rng(4)
    ws = []
    for q in range(12):
        n = int(rng.integers(2, 12))
        N = int(rng.integers(0, 30))
        m = int(rng.choice([2, 4]))
        d = int(rng.choice([0, 8, 20]))
        ws.append(W.random_poly(f"b{q}", m, d, n, N, rng.integers(1, min(n, 6) + 1, size=N), q))
    plans, B = _batch(ws, tiles)
    rows = B.tasks()
    assert B.info()["m1"] == 2 and B.info()["m2"] == 4
    seen_before = {}
    queue_of = {}
    for inst, kind, need, count, first, queue in rows:
        # waits only for earlier tasks of its own instance, all in one queue
        assert need <= seen_before.get(inst, 0)
        seen_before[inst] = seen_before.get(inst, 0) + 1
        assert queue_of.setdefault(inst, queue) == queue
    assert list(rows[:, 5]) == sorted(rows[:, 5])
    for p, w in enumerate(ws):
        mine = rows[rows[:, 0] == p]
        kinds = list(mine[:, 1])
        assert kinds == sorted(kinds, key=lambda k: {0: 0, 1: 1, 2: 2, 3: 3}[k])
        # need = number of this instance's tasks of earlier stages
        info = plans[p].info
        d1 = w.d + 1
        conv = mine[mine[:, 1] == 1]
        covered = np.zeros(info["n_conv"], dtype=int)
        for _, _, _, c, f, _ in conv:
            covered[f:f + c] += 1
        assert np.all(covered == 1)
        add = mine[mine[:, 1] == 2]
        items = np.zeros(info["n_add"] * d1, dtype=int)
        for _, _, _, c, f, _ in add:
            items[f:f + c] += 1
        assert np.all(items == 1)
        st = mine[mine[:, 1] == 0]
        assert st[:, 3].sum() == (1 + w.N + w.n + int(np.sum(w.nvars == 1))) * d1
        ga = mine[mine[:, 1] == 3]
        assert ga[:, 3].sum() == (1 + w.n) * d1
        assert ga[:, 2].min() == len(mine) - len(ga)   # gather waits for everything else


def test_batch_rejects_mixed_precisions():
    ws = [W.random_poly("a", 2, 3, 4, 3, [2, 2, 2], 1), W.random_poly("b", 8, 3, 4, 3, [2, 2, 2], 2)]
    with pytest.raises(mdpe.MdpeError) as e:
        _batch(ws)
    assert e.value.code == mdpe.MDPE_EUNSUPPORTED

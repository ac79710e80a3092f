"""Host-only checks of the batched executor's task queues (no GPU):
every job and addition item is covered exactly once, each queue is ordered by
pipeline depth, and every task waits only for tasks of its own instance of
smaller depth -- the property that makes the persistent kernel deadlock-free.
An instance costing more than an eighth of the batch is dealt over all eight
queues; the others keep one queue each."""
import numpy as np
import pytest

from paper_2101_10881_amd import mdpe
from paper_2101_10881_amd import workloads as W


def _batch(ws, tiles=None):
    plans = [mdpe.Plan.for_workload(w, device=-1) for w in ws]
    return plans, mdpe.Batch(plans, tiles)


def _depths(rows):
    """Pipeline depth of each task within its instance: the rank of its wait
    count among the instance's distinct wait counts (one per stage)."""
    dep = np.zeros(len(rows), dtype=int)
    for p in np.unique(rows[:, 0]):
        idx = np.flatnonzero(rows[:, 0] == p)
        rank = {v: i for i, v in enumerate(sorted(set(rows[idx, 2].tolist())))}
        dep[idx] = [rank[v] for v in rows[idx, 2].tolist()]
    return dep


def _check_deadlock_free(rows):
    dep = _depths(rows)
    assert list(rows[:, 5]) == sorted(rows[:, 5])          # queues are contiguous, in order
    for q in np.unique(rows[:, 5]):
        assert np.all(np.diff(dep[rows[:, 5] == q]) >= 0)   # each queue in depth order
    for i, r in enumerate(rows):                            # waits for smaller depths only
        mine = rows[:, 0] == r[0]
        assert r[2] == np.sum(mine & (dep < dep[i]))


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
    _check_deadlock_free(rows)
    dep = _depths(rows)
    assert len(np.unique(rows[:, 5])) == 8
    for p, w in enumerate(ws):
        mine = rows[rows[:, 0] == p]
        kinds = mine[np.argsort(dep[rows[:, 0] == p], kind="stable"), 1]
        assert np.all(np.diff(kinds) >= 0)                 # stage, conv, add, gather by depth
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


def test_batch_of_one_is_dealt_over_every_queue():
    for w in (W.p2(m=1, d=8), W.p1(m=2, d=8)):
        _, B = _batch([w])
        rows = B.tasks()
        _check_deadlock_free(rows)
        per_queue = np.bincount(rows[:, 5], minlength=8)
        assert len(per_queue) == 8 and per_queue.max() - per_queue.min() <= 1
        conv = rows[rows[:, 1] == 1]
        J = B.info()["n_conv_tasks"]
        assert J == len(conv) and conv[:, 3].max() <= 16   # one group of jobs per task


def test_equal_instances_keep_one_queue_each():
    ws = [W.random_poly(f"e{q}", 2, 8, 6, 20, 3, seed=1) for q in range(16)]
    _, B = _batch(ws)
    rows = B.tasks()
    _check_deadlock_free(rows)
    for p in range(16):
        assert len(np.unique(rows[rows[:, 0] == p, 5])) == 1
    assert np.all(np.bincount(rows[:, 5], minlength=8) > 0)


# ------------------------------------------------------- the tune cache --
# plan_batch reads the autotuner's JSON cache itself, so a C caller gets the
# tuned tiles; the tiles it finds must give the same task table as passing
# them directly (plan_batch_tiles).

def _mixed(count=24, seed=9):
    rng = np.random.default_rng(seed)
    ws = []
    for q in range(count):
        m = int(rng.choice([2, 4]))
        d = int(rng.choice([8, 16, 64, 128]))
        n = int(rng.integers(4, 12))
        N = int(rng.integers(4, 40))
        ws.append(W.random_poly(f"t{q}", m, d, n, N, rng.integers(2, min(n, 6) + 1, size=N), q))
    return ws


def test_plan_batch_reads_the_committed_tune_cache():
    import json
    ws = _mixed()
    plans = [mdpe.Plan.for_workload(w, device=-1) for w in ws]
    tiles = json.load(open(mdpe.TUNE_CACHE))["gfx950"]["tiles"]
    a = mdpe.Batch(plans, tune_cache=mdpe.TUNE_CACHE)
    b = mdpe.Batch(plans, tiles=tiles)
    c = mdpe.Batch(plans)
    assert np.array_equal(a.tasks(), b.tasks())
    assert not np.array_equal(a.tasks(), c.tasks())     # the cache changes the tiles of its buckets


def test_tune_cache_without_this_architecture_gives_the_defaults(tmp_path):
    ws = _mixed(8)
    plans = [mdpe.Plan.for_workload(w, device=-1) for w in ws]
    f = tmp_path / "cache.json"
    f.write_text('{"gfx942": {"tiles": [{"m": 2, "d": 8, "jobs_per_group": 3}]}, "note": [1, 2.5, true, null]}')
    assert np.array_equal(mdpe.Batch(plans, tune_cache=str(f)).tasks(), mdpe.Batch(plans).tasks())


@pytest.mark.parametrize("text,words", [
    (None, "cannot read"),
    ("{not json", "not a JSON object"),
    ('[1, 2]', "not a JSON object"),
    ('{"gfx950": {"tiles": 3}}', "no tile list"),
    ('{"gfx950": {"tiles": [{"d": 8, "jobs_per_group": 2}]}}', "integer m, d"),
    ('{"gfx950": {"tiles": [{"m": 2, "d": 8, "jobs_per_group": 2.5}]}}', "integer m, d"),
    ('{"gfx950": {"tiles": [{"m": 2, "d": 8, "deal": 3}]}}', "deal 0, 1 or 2"),
])
def test_bad_tune_caches_are_rejected(tmp_path, text, words):
    ws = _mixed(4)
    plans = [mdpe.Plan.for_workload(w, device=-1) for w in ws]
    f = tmp_path / "cache.json"
    if text is not None:
        f.write_text(text)
    with pytest.raises(mdpe.MdpeError) as e:
        mdpe.Batch(plans, tune_cache=str(f))
    assert e.value.code == mdpe.MDPE_EINVAL and words in str(e.value)


def test_batch_workspace_is_the_instances_parts():
    ws = _mixed(10)
    plans = [mdpe.Plan.for_workload(w, device=-1) for w in ws]
    B = mdpe.Batch(plans)
    want = sum((p.info["workspace_bytes"] + 255) // 256 * 256 for p in plans)
    assert B.info()["workspace_bytes"] == want


def test_deal_tile_field_changes_no_task():
    # the coefficient order inside a group (schedule or dealt) changes neither
    # the tasks nor, on the GPU, the bits (tests/test_gpu_batch.py)
    ws = _mixed(6)
    plans = [mdpe.Plan.for_workload(w, device=-1) for w in ws]
    base = mdpe.Batch(plans, tiles=[]).tasks()
    for deal in (1, 2):
        tiles = [{"m": 2, "d": w.d, "deal": deal} for w in ws if w.m == 2]
        assert np.array_equal(mdpe.Batch(plans, tiles=tiles).tasks(), base)
    with pytest.raises(mdpe.MdpeError):
        mdpe.Batch(plans, tiles=[{"m": 2, "d": 8, "deal": 5}])

"""GPU batched executor: one persistent launch (plain or hipGraph-replayed)
over many polynomials of different sizes, degrees and precisions, bit for
bit equal to evaluating each instance with eval_and_diff (and to the
oracle), for several tile choices."""
import numpy as np
import pytest

from gpu_util import assert_bitexact
from paper_2101_10881_amd import workloads as W

pytestmark = pytest.mark.gpu


def _instances(count, seed, ms=(2, 4), ds=(0, 3, 8, 16, 33, 64)):
    rng = np.random.default_rng(seed)
    out = []
    for q in range(count):
        n = int(rng.integers(2, 20))
        N = int(rng.integers(0, 60))
        m = int(rng.choice(ms))
        d = int(rng.choice(ds))
        out.append(W.random_poly(f"b{seed}_{q}_m{m}_d{d}", m, d, n, N, rng.integers(1, min(n, 8) + 1, size=N),
                                 1000 * seed + q))
    return out


def _plain(ws):
    import torch
    from paper_2101_10881_amd import mdpe
    dev = torch.device("cuda", 0)
    out = []
    for w in ws:
        P = mdpe.Polynomial.for_workload(w, dev)
        v, g = P.eval_and_diff(torch.from_numpy(w.coeff).to(dev), torch.from_numpy(w.z).to(dev))
        out.append((v, g))
    torch.cuda.synchronize()
    return [(v.cpu().numpy(), g.cpu().numpy()) for v, g in out]


def _batched(ws, tiles=None, graph=False, replays=1, mutate=None, grid=0):
    import torch
    from paper_2101_10881_amd import mdpe
    dev = torch.device("cuda", 0)
    B = mdpe.BatchedPolynomials(ws, dev, tiles)
    if grid:
        B.batch.set_grid(grid)
    coeffs = [torch.from_numpy(w.coeff).to(dev) for w in ws]
    zs = [torch.from_numpy(w.z).to(dev) for w in ws]
    B.bind(coeffs, zs)
    results = []
    for r in range(replays):
        print(f"batch launch {r} graph={graph} instances={len(ws)}", flush=True)
        vals, grads = B.run(graph=graph)
        torch.cuda.synchronize()
        B.batch.status()
        results.append([(v.cpu().numpy(), g.cpu().numpy()) for v, g in zip(vals, grads)])
        if mutate is not None:
            mutate(r, coeffs)
        _ = torch.ones(1000, device=dev).sum()   # eager work between replays
        torch.cuda.synchronize()
    return results, B


def _check(got, want, what):
    for q, ((gv, gg), (wv, wg)) in enumerate(zip(got, want)):
        assert_bitexact(gv, wv, f"{what} instance {q} value")
        assert_bitexact(gg, wg, f"{what} instance {q} grad")


def test_batch_matches_plain_and_oracle(oracle_lib):
    ws = _instances(24, 1)
    want = _plain(ws)
    got, B = _batched(ws)
    assert B.batch.info()["grid"] > 0
    _check(got[0], want, "batch")
    for q in (0, 5, 17):
        v, g = oracle_lib.eval_workload(ws[q])
        assert_bitexact(got[0][q][0], v, f"oracle value {q}")
        assert_bitexact(got[0][q][1], g, f"oracle grad {q}")


def test_batch_graph_replays_follow_inputs():
    import torch
    ws = _instances(16, 2)

    def mutate(r, coeffs):
        # next replay sees new coefficients through the same pointers
        for q, c in enumerate(coeffs):
            c[0] *= -1.0
            ws[q].coeff[0] *= -1.0

    got, _ = _batched(ws, graph=True, replays=3, mutate=None)
    want = _plain(ws)
    for r in range(3):
        _check(got[r], want, f"graph replay {r}")
    ws2 = _instances(10, 3)
    ws = ws2
    got2, _ = _batched(ws2, graph=True, replays=2, mutate=mutate)
    # replay 0 read the original inputs, replay 1 the negated leading limbs of a_0..a_N;
    # the host copies were flipped after each replay, so they hold the originals again
    want0 = _plain(ws2)
    _check(got2[0], want0, "replay 0")
    for q in range(len(ws2)):
        ws2[q].coeff[0] *= -1.0
    want1 = _plain(ws2)
    _check(got2[1], want1, "replay 1 (new inputs)")


@pytest.mark.parametrize("tiles", [
    [{"m": 2, "d": 16, "jobs_per_group": 11, "groups_per_task": 1, "add_items_per_task": 64},
     {"m": 4, "d": 33, "jobs_per_group": 2, "groups_per_task": 5, "add_items_per_task": 333}],
    [{"m": m, "d": d, "jobs_per_group": 1, "groups_per_task": 1, "add_items_per_task": 4096}
     for m in (2, 4) for d in (0, 3, 8, 16, 33, 64)],
    # double doubles forced onto the lane schedule, and dealt to lanes in turn
    [{"m": 2, "d": d, "jobs_per_group": 3, "groups_per_task": 2, "add_items_per_task": 1000, "deal": 1}
     for d in (0, 3, 8, 16, 33, 64)],
    [{"m": 2, "d": d, "jobs_per_group": 5, "groups_per_task": 3, "add_items_per_task": 777, "deal": 2}
     for d in (0, 3, 8, 16, 33, 64)],
])
def test_tiles_do_not_change_bits(tiles):
    ws = _instances(12, 4)
    want = _plain(ws)
    got, _ = _batched(ws, tiles=tiles)
    _check(got[0], want, "tiled batch")


def test_homogeneous_deca_double_batch():
    ws = _instances(6, 5, ms=(10,), ds=(4, 40))
    want = _plain(ws)
    got, _ = _batched(ws, graph=True, replays=2)
    _check(got[0], want, "m=10 batch")
    _check(got[1], want, "m=10 batch replay")


@pytest.mark.parametrize("grid", [8, 64])
def test_wavefronts_running_many_tasks(grid):
    # a small persistent grid makes every wavefront claim and run many tasks in turn
    # (one per XCD at grid 8), the regime of the full 512-instance batch
    ws = _instances(12, 6)
    small = [{"m": m, "d": d, "groups_per_task": 1, "add_items_per_task": 64} for m in (2, 4)
             for d in (0, 3, 8, 16, 33, 64)]
    want = _plain(ws)
    got, _ = _batched(ws, tiles=small, grid=grid, graph=True, replays=2)
    _check(got[0], want, f"grid {grid}")
    _check(got[1], want, f"grid {grid} replay")


def test_mixed_batch_512_full_size(oracle_lib):
    # the batched configuration as the benchmark times it: 512 instances,
    # autotuned tiles, one graph launch; every instance bitwise equal to its
    # plain evaluation, and one instance of each (m, d) bucket to the oracle
    import os
    import sys
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import bench
    ws = W.mixed_batch(512, seed=1)
    got, B = _batched(ws, tiles=bench.load_tiles(), graph=True)
    want = _plain(ws)
    _check(got[0], want, "config 3")
    first = {}
    for q, w in enumerate(ws):
        first.setdefault((w.m, w.d), q)
    for (m, d), q in sorted(first.items()):
        print(f"oracle check: instance {q} m={m} d={d} N={ws[q].N}", flush=True)
        v, g = oracle_lib.eval_workload(ws[q])
        assert_bitexact(got[0][q][0], v, f"oracle value {q}")
        assert_bitexact(got[0][q][1], g, f"oracle grad {q}")


@pytest.mark.parametrize("name,build,grid", [
    ("p2_1d_d8", lambda: W.p2(m=1, d=8), 0),
    ("p2_2d_d64", lambda: W.p2(m=2, d=64), 0),
    ("p2_4d_d64", lambda: W.p2(), 0),
    ("p1_4d_d8", lambda: W.p1(m=4, d=8), 0),
    ("rand3_2d_d8", lambda: W.rand3(), 0),
    ("p2_1d_d8_grid8", lambda: W.p2(m=1, d=8), 8),
])
def test_batch_of_one_dealt_over_every_xcd(name, build, grid):
    # one instance is dealt over all eight XCD queues; each layer's results
    # cross XCDs through the agent-scope fences
    ws = [build()]
    want = _plain(ws)
    got, B = _batched(ws, graph=True, replays=2, grid=grid)
    assert len(np.unique(B.batch.tasks()[:, 5])) == 8
    _check(got[0], want, name)
    _check(got[1], want, name + " replay")


def test_eval_and_diff_batch_rebinds_on_the_stream(oracle_lib):
    """eval_and_diff_batch through the C ABI, with the tiles plan_batch reads
    from the tune cache: three calls without a host synchronisation between
    them -- new input buffers on the second (the pointer table is rebound on
    the stream), the first buffers again on the third -- each bit for bit equal
    to eval_and_diff of every instance."""
    import torch
    from paper_2101_10881_amd import mdpe
    dev = torch.device("cuda", 0)
    ws = _instances(20, 11, ds=(0, 8, 16, 33, 64, 128))
    B = mdpe.BatchedPolynomials(ws, dev, tune_cache=mdpe.TUNE_CACHE)
    c1 = [torch.from_numpy(w.coeff).to(dev) for w in ws]
    z1 = [torch.from_numpy(w.z).to(dev) for w in ws]
    c2 = [-c for c in c1]                     # exact: every limb negated
    z2 = [z.clone() for z in z1]
    print(f"eval_and_diff_batch: {len(ws)} instances, workspace {B.batch.info()['workspace_bytes']} bytes", flush=True)
    outs = []
    for cs, zs in ((c1, z1), (c2, z2), (c1, z1)):
        vals, grads = B.eval_and_diff(cs, zs)
        outs.append(([v.clone() for v in vals], [g.clone() for g in grads]))   # stream-ordered copies
    torch.cuda.synchronize()
    B.batch.status()
    want1 = _plain(ws)
    for w in ws:
        w.coeff = -w.coeff
    want2 = _plain(ws)
    for w in ws:
        w.coeff = -w.coeff
    for r, want in ((0, want1), (1, want2), (2, want1)):
        got = [(v.cpu().numpy(), g.cpu().numpy()) for v, g in zip(*outs[r])]
        _check(got, want, f"eval_and_diff_batch call {r}")
    v, g = oracle_lib.eval_workload(ws[3])
    assert_bitexact(outs[0][0][3].cpu().numpy(), v, "oracle value 3")
    assert_bitexact(outs[0][1][3].cpu().numpy(), g, "oracle grad 3")


def test_default_grid_fills_whole_simds():
    # the persistent grid is the resident one-wavefront workgroups per CU rounded
    # down to a multiple of the CU's four SIMDs (equal wavefronts per SIMD)
    import torch
    ws = _instances(6, 9)
    want = _plain(ws)
    got, B = _batched(ws)
    _check(got[0], want, "default grid")
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    grid = B.batch.info()["grid"]
    assert grid % cus == 0, (grid, cus)
    per_cu = grid // cus
    assert per_cu <= 4 or per_cu % 4 == 0, per_cu

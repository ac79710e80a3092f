#!/usr/bin/env python3
"""Benchmark: evaluation + full gradient of p1 in deca-double precision at
degree 152 (the paper's Table 3 workload) on one MI355X.

One step = one eval_and_diff: staging, the four convolution launches, the
eleven addition launches and the gather, with inputs already in HBM.

Prints one JSON line.  `value` is the FP64 operation rate of the whole step
in GFLOP/s, counting the double operations the project's multiple-double
algorithms execute (FMA = 2) on the convolution jobs without zero terms and
on the addition jobs.  `roofline` reports the convolution kernel, timed with
HIP events around each of its launches inside the timed region, against the
FP64 vector peak.  `cpu_baseline` is the CPU oracle on a bounded sample of
the same workload, on all host cores.
"""
import argparse
import hashlib
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP64_PEAK_TFLOPS = 78.6      # MI355X FP64 vector, FMA counted as two operations
HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=10.0, help="target wall time of the CPU sample")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="run one torch copy of this size before timing (for HBM counter calibration)")
    ap.add_argument("--no-check", dest="check", action="store_false",
                    help="skip comparing the output digest with the oracle's (compared by default)")
    ap.add_argument("--workload", default="p1", choices=["p1", "batch", "sweep", "rand3", "p2", "autograd"],
                    help="p1: deca double d=152 (the headline); batch: 512 mixed instances vs separate launches; "
                         "sweep: the paper's precision x degree tables for p1, p2, p3")
    ap.add_argument("--polys", default="p1,p2,p3", help="sweep: test polynomials")
    ap.add_argument("--ms", default="1,2,3,4,5,8,10", help="sweep: precisions")
    ap.add_argument("--ds", default="0,8,15,31,63,95,127,152,159,191", help="sweep: degrees")
    ap.add_argument("--complex", action="store_true", help="sweep: complex series")
    ap.add_argument("--layer-launches", action="store_true",
                    help="sweep: one launch per convolution layer even where the plan would fuse them")
    ap.add_argument("--emax", type=int, default=1,
                    help="sweep: raise half of the variable occurrences to exponents 2..emax")
    ap.add_argument("--instances", type=int, default=512, help="batch: number of instances")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the other workloads and side measurements (double double d=8, quad double p2, "
                         "the batch, the autograd pass, complex, streamed, layering, seeds)")
    ap.add_argument("--workload-steps", type=int, default=20, help="timed steps of each of the other workloads")
    return ap.parse_args()


def progress(msg):
    """A progress line on stderr (the result is the one JSON line on stdout)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_source_digest():
    h = hashlib.sha256()
    for f in ("md.hpp", "conv_core.hpp", "kernels.hip", "plan.cpp", "plan.hpp"):
        h.update(open(os.path.join(ROOT, "paper_2101_10881_amd", "csrc", f), "rb").read())
    return h.hexdigest()


def traffic_from_profile(digest, launches_per_step):
    """HBM bytes per convolution launch from the committed PMC summary, if it
    was taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", "conv_layer_kernel_p1_10d_d152_traffic.json")
    try:
        t = json.load(open(path))
    except (OSError, ValueError):
        return None
    if t.get("kernel_source_sha256") != digest:
        return None
    return t.get("hbm_bytes_per_launch")


def cpu_baseline(target_s):
    """The oracle, as it stands, on the first K monomials of p1 (m=10, d=152)."""
    import numpy as np

    from oracle import oracle as O
    from paper_2101_10881_amd import flops, mdpe
    from paper_2101_10881_amd import workloads as W

    cores = len(os.sched_getaffinity(0))
    cpu_model = None
    try:
        with open("/proc/cpuinfo") as f:
            cpu_model = next((l.split(":", 1)[1].strip() for l in f if l.startswith("model name")), None)
    except OSError:
        pass
    full = W.p1()

    def sample(K, threads):
        sup = full.supports()[:K]
        w = W.make(f"p1_first{K}", 10, 152, 16, sup, seed=1)
        t0 = time.perf_counter()
        O.eval_workload(w, nthreads=threads)
        dt = time.perf_counter() - t0
        i = mdpe.Plan.for_workload(w, device=-1).info
        work = i["n_conv"] * flops.conv_flops(10, 152) + i["n_add"] * flops.add_flops(10, 152)
        return dt, work

    K0 = max(cores, 8)
    dt0, _ = sample(K0, cores)
    K = int(min(1820, max(K0, K0 * target_s / max(dt0, 1e-3))))
    dt, work = sample(K, cores)
    # one thread, on a few monomials (a couple of seconds)
    K1 = 48
    dt1, work1 = sample(K1, 1)
    return {"value": work / dt / 1e9, "unit": "GFLOP/s", "cores": cores, "cpu_model": cpu_model, "kind": "oracle",
            "sample": f"first {K} of the 1820 monomials of p1, m=10, d=152, seed 1 ({dt:.1f} s wall, "
                      f"{cores} OpenMP threads, same flop accounting as value)",
            "seconds": dt,
            "single_thread": {"value": round(work1 / dt1 / 1e9, 3), "unit": "GFLOP/s",
                              "sample": f"first {K1} monomials, 1 thread ({dt1:.1f} s wall)"}}


def _cpu_info():
    cores = len(os.sched_getaffinity(0))
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            model = next((l.split(":", 1)[1].strip() for l in f if l.startswith("model name")), None)
    except OSError:
        pass
    return cores, model


def _step_times(fn, steps, warmup):
    """Per-step milliseconds of fn() from HIP events between consecutive steps
    on the current stream (inputs resident, no host synchronisation inside)."""
    import torch
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    marks = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    marks[0].record(stream)
    for k in range(steps):
        fn()
        marks[k + 1].record(stream)
    torch.cuda.synchronize()
    per = sorted(marks[k].elapsed_time(marks[k + 1]) for k in range(steps))
    return {"median": round(statistics.median(per), 4), "min": round(per[0], 4), "max": round(per[-1], 4),
            "mean": round(marks[0].elapsed_time(marks[-1]) / steps, 4), "steps": steps}


def _rate(flop, ms):
    return {"GFLOPs": round(flop / (ms * 1e-3) / 1e9, 2), "frac_fp64_peak": round(flop / (ms * 1e-3) / 1e12 /
                                                                                    FP64_PEAK_TFLOPS, 5)}


def _oracle_timed(fn, reps=3):
    """Median wall seconds of fn() over reps runs (the CPU oracle, all host cores)."""
    times, out = [], None
    for _ in range(reps):
        t0 = time.perf_counter()
        out = fn()
        times.append(time.perf_counter() - t0)
    return statistics.median(times), out


def _bits_equal(gpu, want):
    import numpy as np
    g = np.ascontiguousarray(gpu.detach().cpu().numpy(), dtype=np.float64).view(np.uint64)
    return bool(np.array_equal(g, np.ascontiguousarray(want, dtype=np.float64).view(np.uint64)))


def measure_plain_workload(w, steps, warmup, with_oracle=True):
    """One plain workload: eval_and_diff per step, event-timed, beside the
    oracle on all host cores for the same inputs; outputs compared bitwise."""
    import torch

    from oracle import oracle as O
    from paper_2101_10881_amd import flops, mdpe

    dev = torch.device("cuda", 0)
    P = mdpe.Polynomial.for_workload(w, dev)
    coeff = torch.from_numpy(w.coeff).to(dev)
    z = torch.from_numpy(w.z).to(dev)
    value, grad = P.eval_and_diff(coeff, z)
    ms = _step_times(lambda: P.eval_and_diff(coeff, z, value, grad), steps, warmup)
    info = P.plan.info
    work = info["n_conv"] * flops.conv_flops(w.m, w.d) + info["n_add"] * flops.add_flops(w.m, w.d)
    chain = info["chain_layers"] > 0
    launches = (1 if info["fused_components"] else
                (1 + info["n_layers"] - info["chain_layers"]) if chain else info["n_layers"])
    out = {"workload": w.name, "m": w.m, "d": w.d, "n": w.n, "N": w.N, "n_conv": info["n_conv"],
           "n_add": info["n_add"], "conv_launches": launches,
           "fused_layers": bool(info["fused_components"]), "ms_per_step": ms, "flop_per_step": work,
           **_rate(work, ms["median"])}
    if chain:
        out["chain_launch"] = {k: info[k] for k in ("chain_layers", "chain_count", "chain_waves", "chain_window",
                                                    "chain_ring")}
    if not with_oracle:
        return out
    cores, model = _cpu_info()
    sec, (ov, og) = _oracle_timed(lambda: O.eval_workload(w, nthreads=cores))
    out["bitexact_vs_oracle"] = _bits_equal(value, ov) and _bits_equal(grad, og)
    out["cpu_oracle"] = {"seconds": round(sec, 5), **_rate(work, sec * 1e3), "cores": cores, "cpu_model": model,
                         "sample": "the whole workload, median of 3 runs"}
    out["gpu_vs_cpu"] = round(sec * 1e3 / ms["median"], 1)
    return out


def measure_autograd_workload(steps, warmup, with_oracle=True):
    """The differentiation workload: octo-double p1 at d = 32 through
    torch.autograd.Function (forward keeping the monomial products, backward
    the adjoint kernel), beside the oracle's value, gradient and adjoints."""
    import torch

    from oracle import oracle as O
    from paper_2101_10881_amd import flops, mdpe
    from paper_2101_10881_amd import workloads as W
    from paper_2101_10881_amd.autograd import poly_eval

    dev = torch.device("cuda", 0)
    w = W.p1(m=8, d=32)
    P = mdpe.Polynomial.for_workload(w, dev, keep_monomials=True)
    coeff = torch.from_numpy(w.coeff).to(dev)
    z = torch.from_numpy(w.z).to(dev)
    ybar_np = W.upstream_adjoint(w.m, w.d, seed=1)
    ybar = torch.from_numpy(ybar_np).to(dev)
    value, grad = P.eval_and_diff(coeff, z)
    fwd = _step_times(lambda: P.eval_and_diff(coeff, z, value, grad), steps, warmup)
    rev = _step_times(lambda: P.adjoint(ybar, grad), steps, warmup)
    cr = coeff.clone().requires_grad_(True)
    zr = z.clone().requires_grad_(True)

    def step():
        cr.grad = None
        zr.grad = None
        v, _ = poly_eval(cr, zr, P)
        v.backward(ybar)

    ag = _step_times(step, steps, warmup)
    info = P.plan.info
    fwd_work = info["n_conv"] * flops.conv_flops(w.m, w.d) + info["n_add"] * flops.add_flops(w.m, w.d)
    rev_work = info["n_reverse"] * flops.conv_flops(w.m, w.d)

    def oracle():
        ov, og = O.eval_workload(w, nthreads=cores)
        oc, oz = O.eval_adjoint(w.m, w.d, w.n, w.nvars, w.vars, w.z, og, ybar_np, nthreads=cores)
        return ov, og, oc, oz

    work = fwd_work + rev_work
    if not with_oracle:
        return {"workload": w.name + "_autograd", "forward_ms": fwd, "reverse_ms": rev, "autograd_step_ms": ag,
                **_rate(work, ag["median"]), "flop_per_step": work}
    cores, model = _cpu_info()
    sec, (ov, og, oc, oz) = _oracle_timed(oracle)
    exact = (_bits_equal(value, ov) and _bits_equal(grad, og) and _bits_equal(cr.grad, oc) and
             _bits_equal(zr.grad, oz))
    return {"workload": w.name + "_autograd", "m": w.m, "d": w.d, "n": w.n, "N": w.N,
            "forward_conv_jobs": info["n_conv"], "reverse_jobs": info["n_reverse"],
            "forward_ms": fwd, **{"forward_" + k: v for k, v in _rate(fwd_work, fwd["median"]).items()},
            "reverse_ms": rev, **{"reverse_" + k: v for k, v in _rate(rev_work, rev["median"]).items()},
            "autograd_step_ms": ag, **_rate(work, ag["median"]), "flop_per_step": work,
            "bitexact_vs_oracle": exact,
            "cpu_oracle": {"seconds": round(sec, 5), **_rate(work, sec * 1e3), "cores": cores, "cpu_model": model,
                           "sample": "value, gradient and adjoints of the whole workload, median of 3 runs"},
            "gpu_vs_cpu": round(sec * 1e3 / ag["median"], 1)}


def measure_batch(instances, steps, warmup):
    """The batched workload: `instances` polynomials (n 8..64, N 16..1024,
    2..8 variables per monomial, d in {8,16,32,64,128}, m in {2,4}) in one
    persistent launch (plain and hipGraph-replayed) against one eval_and_diff
    per instance on one stream.  Outputs must agree bit for bit."""
    import torch

    from paper_2101_10881_amd import flops, mdpe
    from paper_2101_10881_amd import workloads as W

    dev = torch.device("cuda", 0)
    t0 = time.perf_counter()
    ws = W.mixed_batch(instances, seed=1)
    B = mdpe.BatchedPolynomials(ws, dev, tune_cache=mdpe.TUNE_CACHE)
    coeffs = [torch.from_numpy(w.coeff).to(dev) for w in ws]
    zs = [torch.from_numpy(w.z).to(dev) for w in ws]
    B.bind(coeffs, zs)
    setup_s = time.perf_counter() - t0
    work = sum(P.plan.info["n_conv"] * flops.conv_flops(P.m, P.d) + P.plan.info["n_add"] * flops.add_flops(P.m, P.d)
               for P in B.polys)
    pv = [torch.empty_like(v) for v in B.values]
    pg = [torch.empty_like(g) for g in B.grads]
    stream = torch.cuda.current_stream()

    def plain():
        for P, c, z, v, g in zip(B.polys, coeffs, zs, pv, pg):
            P.eval_and_diff(c, z, v, g)

    def timed(fn, reps):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    ms_plain = timed(plain, max(1, steps // 4))
    ms_batch = timed(lambda: B.run(graph=False), steps)
    B.batch.status()
    ms_graph = timed(lambda: B.run(graph=True), steps)
    B.batch.status()
    same = all(torch.equal(x.view(torch.int64), y.view(torch.int64))
               for x, y in zip(B.values + B.grads, pv + pg))
    # the boundary's batched call: one graph replay per step over one workspace
    ms_call = _step_times(lambda: B.eval_and_diff(coeffs, zs), steps, warmup)
    same_call = all(torch.equal(x.view(torch.int64), y.view(torch.int64))
                    for x, y in zip(B.values + B.grads, pv + pg))
    info = B.batch.info()
    # the default tiles on the same kernel, for the tuner's gain
    D = mdpe.BatchedPolynomials(ws, dev)
    D.bind(coeffs, zs)
    ms_default = timed(lambda: D.run(graph=True), steps)
    D.batch.status()
    same_default = all(torch.equal(x.view(torch.int64), y.view(torch.int64))
                       for x, y in zip(D.values + D.grads, pv + pg))
    del D
    return {
        "workload": f"mixed_batch_{instances}", "instances": instances, "seed": 1,
        "GFLOPs": round(work / (ms_graph * 1e-3) / 1e9, 1),
        "frac_fp64_peak": round(work / (ms_graph * 1e-3) / 1e12 / FP64_PEAK_TFLOPS, 5),
        "flop_per_step": work,
        "batched_ms": {"graph": round(ms_graph, 4), "launch": round(ms_batch, 4)},
        "eval_and_diff_batch_ms": ms_call,
        "plain_ms": round(ms_plain, 4),
        "speedup_vs_plain": round(ms_plain / ms_graph, 3),
        "bitexact_vs_plain": bool(same and same_call and same_default),
        "tiles": {"tuned_ms": round(ms_graph, 4), "default_ms": round(ms_default, 4),
                  "tuned_speedup": round(ms_default / ms_graph, 3), "cache": os.path.relpath(mdpe.TUNE_CACHE, ROOT)},
        "precisions": sorted({P.m for P in B.polys}), "degrees": sorted({P.d for P in B.polys}),
        "n_conv": sum(P.plan.info["n_conv"] for P in B.polys), "n_add": sum(P.plan.info["n_add"] for P in B.polys),
        "tasks": info["n_tasks"], "persistent_workgroups": info["grid"],
        "setup_s": round(setup_s, 1),
        "_outputs": (ws, B),
    }


def batch_cpu_baseline(r, every=8):
    """The oracle on every `every`-th instance of the batch (a bounded
    sample), all host cores; sampled outputs compared bitwise with the batch's."""
    from oracle import oracle as O
    from paper_2101_10881_amd import flops

    ws, B = r.pop("_outputs")
    cores, model = _cpu_info()
    idx = list(range(0, len(ws), every))
    work, exact = 0, True
    t0 = time.perf_counter()
    outs = [O.eval_workload(ws[q], nthreads=cores) for q in idx]
    sec = time.perf_counter() - t0
    for q, (ov, og) in zip(idx, outs):
        P = B.polys[q]
        work += P.plan.info["n_conv"] * flops.conv_flops(P.m, P.d) + P.plan.info["n_add"] * flops.add_flops(P.m, P.d)
        exact &= _bits_equal(B.values[q], ov) and _bits_equal(B.grads[q], og)
    r["bitexact_vs_oracle_sample"] = bool(exact)
    r["cpu_oracle"] = {"seconds": round(sec, 3), **_rate(work, sec * 1e3), "cores": cores, "cpu_model": model,
                       "sample": f"{len(idx)} of the {len(ws)} instances (every {every}th), one run"}
    gpu_rate = r["flop_per_step"] / (r["batched_ms"]["graph"] * 1e-3)
    r["gpu_vs_cpu"] = round(gpu_rate / (work / sec), 1)
    return r


def run_batch(a):
    if a.copy_calibration_mib:
        copy_calibration(a.copy_calibration_mib)
    r = measure_batch(a.instances, a.steps, a.warmup)
    r.pop("_outputs")
    out = {
        "metric": "FP64 GFLOP/s (multi-double ops) for eval+gradient; % FP64 peak; batched vs plain",
        "value": r["GFLOPs"], "unit": "GFLOP/s",
        "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": r["batched_ms"]["graph"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic (seeded random instances)",
        "config": {"workload": r["workload"]},
        "batched": r,
    }
    print(json.dumps(out), flush=True)


def measure_complex(steps, warmup, m=10, d=152):
    """p1 with complex coefficients and inputs (real and imaginary parts in
    separate limb planes), the headline precision and degree."""
    import torch

    from paper_2101_10881_amd import flops, mdpe
    from paper_2101_10881_amd import workloads as W

    dev = torch.device("cuda", 0)
    w = W.p1(m=m, d=d, cx=True)
    P = mdpe.Polynomial.for_workload(w, dev)
    coeff = torch.from_numpy(w.coeff).to(dev)
    z = torch.from_numpy(w.z).to(dev)
    v, g = P.eval_and_diff(coeff, z)
    for _ in range(warmup):
        P.eval_and_diff(coeff, z, v, g)
    torch.cuda.synchronize()
    prof = mdpe.Profiler()
    for _ in range(steps):
        P.eval_and_diff(coeff, z, v, g, profiler=prof)
    t = prof.read()
    info = P.plan.info
    cnv, add = t["cnv_ms"] / steps, t["add_ms"] / steps
    conv_f = info["n_conv"] * flops.conv_flops(m, d, cx=True)
    work = conv_f + info["n_add"] * flops.add_flops(m, d, cx=True)
    return {"workload": w.name, "cnv_ms": round(cnv, 4), "add_ms": round(add, 4),
            "GFLOPs": round(work / ((cnv + add) * 1e-3) / 1e9, 1),
            "conv_TFLOPs": round(conv_f / (cnv * 1e-3) / 1e12, 3)}


def measure_streamed(steps, warmup):
    """Streamed operands (both read from global memory, several wavefronts per
    job): p1 in deca double at d = 152 forced to stream (its plan stages), and a large degree
    (all 4-subsets of 8 variables, quad double, d = 4000) where the plan
    streams by itself, beside the same plan forced to stage."""
    import torch

    from paper_2101_10881_amd import flops, mdpe
    from paper_2101_10881_amd import workloads as W

    dev = torch.device("cuda", 0)
    out = {}
    big = W.make("p_8_4_4d_d4000", 4, 4000, 8, W.all_subsets(8, 4), seed=1)
    for key, w, force in (("p1_10d_d152_forced", W.p1(), True), ("degree_4000_staged", big, False),
                          ("degree_4000", big, None)):
        P = mdpe.Polynomial.for_workload(w, dev, stream_operands=force)
        coeff = torch.from_numpy(w.coeff).to(dev)
        z = torch.from_numpy(w.z).to(dev)
        v, g = P.eval_and_diff(coeff, z)
        for _ in range(warmup):
            P.eval_and_diff(coeff, z, v, g)
        torch.cuda.synchronize()
        prof = mdpe.Profiler()
        for _ in range(steps):
            P.eval_and_diff(coeff, z, v, g, profiler=prof)
        t = prof.read()
        info = P.plan.info
        cnv = t["cnv_ms"] / steps
        conv_f = info["n_conv"] * flops.conv_flops(w.m, w.d)
        out[key] = {"workload": w.name, "streamed": bool(info["streamed"]), "waves_per_job": info["waves_per_job"],
                    "lane_steps": info["lane_steps"], "cnv_ms": round(cnv, 4),
                    "conv_TFLOPs": round(conv_f / (cnv * 1e-3) / 1e12, 3)}
        del P, coeff, z, v, g
    return out


def measure_layering(steps, warmup):
    """p1 in deca double at d = 152 with the earliest-layer layering of
    Section 5 (MDPE_ASAP_LAYERS: 3640/5460/5460/1820 jobs, 18 rounds of the
    1024 SIMDs) beside the default balanced one (3072/4096/6144/3068, 16
    rounds); outputs compared bitwise."""
    import torch

    from paper_2101_10881_amd import mdpe
    from paper_2101_10881_amd import workloads as W

    dev = torch.device("cuda", 0)
    w = W.p1()
    coeff = torch.from_numpy(w.coeff).to(dev)
    z = torch.from_numpy(w.z).to(dev)
    out, bits = {}, []
    for key, asap in (("earliest", True), ("balanced", False)):
        P = mdpe.Polynomial.for_workload(w, dev, asap_layers=asap)
        v, g = P.eval_and_diff(coeff, z)
        for _ in range(warmup):
            P.eval_and_diff(coeff, z, v, g)
        torch.cuda.synchronize()
        prof = mdpe.Profiler()
        for _ in range(steps):
            P.eval_and_diff(coeff, z, v, g, profiler=prof)
        t = prof.read()
        bits.append((v.view(torch.int64).clone(), g.view(torch.int64).clone()))
        out[key] = {"conv_launches": [int(x) for x in P.plan.layer_sizes()[0]],
                    "cnv_ms": round(t["cnv_ms"] / steps, 4)}
        del P, v, g
    out["workload"] = w.name
    out["bitexact"] = bool(torch.equal(bits[0][0], bits[1][0]) and torch.equal(bits[0][1], bits[1][1]))
    return out


def measure_seeds(P, steps):
    """The step time of p1 in deca double at d = 152 for the input seeds
    2..10 with the same plan (p1's supports do not depend on the seed; the
    series values do), the spread the paper reports over seeds (Table 8)."""
    import torch

    from paper_2101_10881_amd import workloads as W

    dev = P.workspace.device
    ms = {}
    for seed in range(2, 11):
        w = W.p1(seed=seed)
        coeff = torch.from_numpy(w.coeff).to(dev)
        z = torch.from_numpy(w.z).to(dev)
        v, g = P.eval_and_diff(coeff, z)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            P.eval_and_diff(coeff, z, v, g)
        e1.record()
        torch.cuda.synchronize()
        ms[seed] = round(e0.elapsed_time(e1) / steps, 4)
    vals = sorted(ms.values())
    return {"workload": "p1_10d_d152", "steps_per_seed": steps, "ms_per_step": ms,
            "median": vals[len(vals) // 2], "min": vals[0], "max": vals[-1]}


def sweep_workload(poly, m, d, cx=False, emax=1):
    from paper_2101_10881_amd import workloads as W
    w = {"p1": W.p1, "p2": W.p2, "p3": W.p3}[poly](seed=1, m=m, d=d, cx=cx)
    return W.with_exponents(w, emax, seed=1) if emax > 1 else w


def run_sweep(a):
    """The structure of the paper's appendix tables: for each test polynomial,
    precision and degree, the summed convolution and addition kernel times,
    their sum and the wall time of one evaluation, in milliseconds."""
    import torch

    from paper_2101_10881_amd import flops, mdpe

    dev = torch.device("cuda", 0)
    rows = []
    for poly in a.polys.split(","):
        for m in (int(x) for x in a.ms.split(",")):
            for d in (int(x) for x in a.ds.split(",")):
                w = sweep_workload(poly, m, d, a.complex, a.emax)
                P = mdpe.Polynomial.for_workload(w, dev, fused_layers=False if a.layer_launches else None)
                coeff = torch.from_numpy(w.coeff).to(dev)
                z = torch.from_numpy(w.z).to(dev)
                v, g = P.eval_and_diff(coeff, z)
                torch.cuda.synchronize()
                reps = max(1, a.steps)
                prof = mdpe.Profiler()
                t0 = time.perf_counter()
                for _ in range(reps):
                    P.eval_and_diff(coeff, z, v, g, profiler=prof)
                torch.cuda.synchronize()
                wall = (time.perf_counter() - t0) * 1e3 / reps
                t = prof.read()
                info = P.plan.info
                work = (info["n_conv"] * flops.conv_flops(m, d, a.complex)
                        + info["n_add"] * flops.add_flops(m, d, a.complex)
                        + info["n_scale"] * (d + 1) * flops.md_flops("mul", m) * (2 if a.complex else 1))
                row = {"poly": poly, "complex": a.complex, "emax": a.emax, "m": m, "d": d, "cnv_ms": round(t["cnv_ms"] / reps, 4),
                       "add_ms": round(t["add_ms"] / reps, 4), "sum_ms": round((t["cnv_ms"] + t["add_ms"]) / reps, 4),
                       "wall_ms": round(wall, 4), "n_conv": info["n_conv"], "n_add": info["n_add"],
                       "fused_layers": int(info["fused_components"] > 0),
                       "TFLOPs": round(work / (t["cnv_ms"] + t["add_ms"]) * reps / 1e9, 3)}
                rows.append(row)
                print(json.dumps(row), flush=True)
                del P, coeff, z, v, g
                torch.cuda.empty_cache()
    print(json.dumps({"sweep": rows}), flush=True)


def copy_calibration(mib):
    """One plain device copy of `mib` MiB, so that a counter profile of the run
    shows what FETCH_SIZE / WRITE_SIZE read for a known number of bytes."""
    import torch
    nbytes = mib << 20
    src = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst


def run_single(a):
    """One of the other workloads on its own (for profiling): double double at
    d = 8 (rand3), quad double p2 at d = 64, or the octo-double autograd pass;
    the oracle beside it unless --no-cpu-baseline."""
    from paper_2101_10881_amd import workloads as W
    if a.copy_calibration_mib:
        copy_calibration(a.copy_calibration_mib)
    if a.workload == "autograd":
        r = measure_autograd_workload(a.steps, a.warmup, not a.no_cpu_baseline)
        ms = r["autograd_step_ms"]["median"]
    else:
        w = W.rand3() if a.workload == "rand3" else W.p2()
        r = measure_plain_workload(w, a.steps, a.warmup, not a.no_cpu_baseline)
        ms = r["ms_per_step"]["median"]
    out = {"metric": "FP64 GFLOP/s (multi-double ops) for eval+gradient; % FP64 peak; batched vs plain",
           "value": r["GFLOPs"], "unit": "GFLOP/s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
           "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
           "data": "synthetic (seeded random series)", "config": {"workload": r["workload"]}, "result": r}
    print(json.dumps(out), flush=True)


def load_tiles():
    """Autotuned tiles for the batched executor, if a cache for this device exists."""
    path = os.path.join(ROOT, "paper_2101_10881_amd", "tune_cache.json")
    try:
        cache = json.load(open(path))
    except (OSError, ValueError):
        return None
    return cache.get("gfx950", {}).get("tiles")


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": f"--gpus {a.gpus}: this benchmark runs on one GPU only (the path would shard "
                                   "by monomial ranges with one all-gather of partial series; no multi-GPU run "
                                   "is implemented)"}))
        sys.exit(2)
    if a.workload == "batch":
        return run_batch(a)
    if a.workload == "sweep":
        return run_sweep(a)
    if a.workload in ("rand3", "p2", "autograd"):
        return run_single(a)
    import torch

    from paper_2101_10881_amd import flops, mdpe
    from paper_2101_10881_amd import workloads as W

    dev = torch.device("cuda", 0)
    w = W.p1()
    P = mdpe.Polynomial.for_workload(w, dev)
    info = P.plan.info
    conv_sizes, add_sizes = P.plan.layer_sizes()
    coeff = torch.from_numpy(w.coeff).to(dev)
    z = torch.from_numpy(w.z).to(dev)
    value = torch.empty((w.m, w.d + 1), dtype=torch.float64, device=dev)
    grad = torch.empty((w.m, w.n, w.d + 1), dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream()

    if a.copy_calibration_mib:
        copy_calibration(a.copy_calibration_mib)

    for _ in range(a.warmup):
        P.eval_and_diff(coeff, z, value, grad)
    torch.cuda.synchronize()

    # inside the timed region only the convolution launches (the roofline's
    # kernel) carry event pairs; the other launches are timed afterwards
    prof = mdpe.Profiler(classes=mdpe.MDPE_TIME_CONV)
    # one event between consecutive steps: the whole region and each step's time
    marks = [torch.cuda.Event(enable_timing=True) for _ in range(a.steps + 1)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    marks[0].record(stream)
    for k in range(a.steps):
        P.eval_and_diff(coeff, z, value, grad, profiler=prof)
        marks[k + 1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    total_ms = marks[0].elapsed_time(marks[-1])
    per_step = sorted(marks[k].elapsed_time(marks[k + 1]) for k in range(a.steps))
    kt = prof.read()
    # breakdown of the other launches: a few untimed steps with every launch timed
    bsteps = 5
    bprof = mdpe.Profiler()
    for _ in range(bsteps):
        P.eval_and_diff(coeff, z, value, grad, profiler=bprof)
    bt = bprof.read()

    m, d = w.m, w.d
    step_flops = info["n_conv"] * flops.conv_flops(m, d) + info["n_add"] * flops.add_flops(m, d)
    ms_per_step = total_ms / a.steps
    gflops = step_flops / (ms_per_step * 1e-3) / 1e9
    conv_flops_total = info["n_conv"] * flops.conv_flops(m, d) * a.steps
    conv_ms = kt["cnv_ms"]
    achieved = conv_flops_total / (conv_ms * 1e-3) / 1e12
    launches = kt["n_cnv"]
    digest = kernel_source_digest()
    traffic = traffic_from_profile(digest, len(conv_sizes))
    n_mac = info["n_conv"] * (d + 1) * (d + 2) // 2
    paper_ops = flops.paper_convention(info["n_conv"], info["n_add"], d)

    out = {
        "metric": "FP64 GFLOP/s (multi-double ops) for eval+gradient; % FP64 peak; batched vs plain",
        "value": round(gflops, 1),
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "step_ms": {"median": round(statistics.median(per_step), 4), "min": round(per_step[0], 4),
                    "max": round(per_step[-1], 4)},
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded random deca-double series; p1 supports)",
        "config": {"workload": w.name, "polynomial": "p1: all 1820 products of 4 of 16 variables",
                   "m": m, "d": d, "n": w.n, "N": w.N, "seed": 1,
                   "n_conv": info["n_conv"], "n_add": info["n_add"],
                   "conv_launches": [int(x) for x in conv_sizes], "add_launches": [int(x) for x in add_sizes]},
        "roofline": {
            "kernel": "conv_layer_kernel<10>",
            "bound": "alu",
            "achieved": round(achieved, 3),
            "peak": FP64_PEAK_TFLOPS,
            "unit": "TFLOP/s",
            "frac": round(achieved / FP64_PEAK_TFLOPS, 4),
            "traffic": traffic,
            "algorithmic_flops_per_job": flops.conv_flops(m, d),
            "avg_launch_ms": round(conv_ms / max(launches, 1), 4),
            "avg_jobs_per_launch": info["n_conv"] / len(conv_sizes),
            "algorithmic_hbm_GBs": round(info["n_conv"] * flops.conv_bytes(m, d) * a.steps / (conv_ms * 1e-3) / 1e9, 1),
        },
        "times_ms_per_step": {"stage": round(bt["stage_ms"] / bsteps, 4), "cnv": round(conv_ms / a.steps, 4),
                              "add": round(bt["add_ms"] / bsteps, 4), "gather": round(bt["gather_ms"] / bsteps, 4),
                              "sum": round(conv_ms / a.steps + bt["add_ms"] / bsteps, 4),
                              "wall": round(wall * 1e3 / a.steps, 4),
                              "note": "cnv from the timed steps (conv launches timed only); stage, add, gather "
                                      f"from {bsteps} further steps with every launch timed"},
        "md_mac_per_s": round(n_mac / (ms_per_step * 1e-3), 1),
        "paper_convention_TFLOPs": round(paper_ops / (ms_per_step * 1e-3) / 1e12, 3),
        "kernel_source_sha256": digest[:16],
    }
    if a.check:
        # the digests of the oracle's output for this workload, written by
        # tests/golden/make_digests.py
        g = json.load(open(os.path.join(ROOT, "tests", "golden", "digests.json")))["workloads"]["p1_10d_d152"]
        h = lambda t: hashlib.sha256(t.cpu().numpy().astype("<f8").tobytes()).hexdigest()
        out["check"] = {"value_matches_oracle_digest": h(value) == g["value_sha256"],
                        "grad_matches_oracle_digest": h(grad) == g["grad_sha256"]}
    if not a.no_extras:
        # the other workloads, each beside the oracle on the host cores
        ks = max(10, a.workload_steps)
        wl = {}
        for wk in (W.rand3(), W.p2()):
            progress(f"workload {wk.name}")
            wl[wk.name] = measure_plain_workload(wk, ks, 3)
        progress(f"workload mixed_batch_{a.instances}")
        r = measure_batch(a.instances, ks, 2)
        wl[r["workload"]] = batch_cpu_baseline(r)
        progress("workload p1_8d_d32 autograd")
        r = measure_autograd_workload(ks, 3)
        wl[r["workload"]] = r
        out["workloads"] = wl
        progress("side measurements")
        out["complex_p1"] = measure_complex(5, 1)
        out["streamed_operands"] = measure_streamed(3, 1)
        out["layer_balancing"] = measure_layering(5, 1)
        out["seed_spread"] = measure_seeds(P, 3)
    if not a.no_cpu_baseline:
        progress("CPU baseline")
        out["cpu_baseline"] = cpu_baseline(a.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

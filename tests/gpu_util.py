"""Helpers for the GPU tests: run the HIP path through the C ABI binding."""
import hashlib

import numpy as np


def require_gpu():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("GPU test needs an MI355X")
    return torch


def run_gpu(w, profiler=None, stream=None, poly=None):
    """Evaluate workload w with the HIP path; returns numpy (value, grad)."""
    torch = require_gpu()
    from paper_2101_10881_amd import mdpe
    dev = torch.device("cuda", 0)
    P = poly or mdpe.Polynomial.for_workload(w, dev)
    coeff = torch.from_numpy(w.coeff).to(dev)
    z = torch.from_numpy(w.z).to(dev)
    val, grad = P.eval_and_diff(coeff, z, stream=stream, profiler=profiler)
    torch.cuda.synchronize()
    return val.cpu().numpy(), grad.cpu().numpy()


def bits(a):
    return np.ascontiguousarray(a, dtype=np.float64).view(np.uint64)


def assert_bitexact(got, want, what=""):
    g, w = bits(got), bits(want)
    if not np.array_equal(g, w):
        bad = np.argwhere(g != w)
        i = tuple(bad[0])
        raise AssertionError(f"{what}: {len(bad)} of {g.size} limbs differ; first at {i}: "
                             f"got {got[i]!r} want {want[i]!r}")


def sha256(a):
    return hashlib.sha256(np.ascontiguousarray(a, dtype="<f8").tobytes()).hexdigest()

"""Host-side checks of the benchmark's contract (no GPU): the one-GPU refusal,
the flop accounting it reports, and the profile lookup that fills
roofline.traffic only for the kernel source it was measured on."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_2101_10881_amd import flops  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU only" in msg["error"]


def test_flop_accounting_closed_forms():
    # per convolution: (d+1)(d+2)/2 md_mul and d(d+1)/2 md_add (eq. (1), zero terms skipped)
    m, d = 10, 152
    assert flops.conv_md_ops(d) == (11781, 11628)
    assert flops.conv_flops(m, d) == 11781 * flops.md_flops("mul", m) + 11628 * flops.md_flops("add", m)
    assert flops.conv_flops(m, d) == 25588791                 # the figure bench.py reports per job of p1, deca double, d = 152
    # complex: 4 md_mul + 2 md_add per product, 2 md_add per sum
    assert flops.coef_flops("mul", m, True) == 4 * flops.md_flops("mul", m) + 2 * flops.md_flops("add", m)
    # the paper's convention for deca doubles (Section 6.2) on p1 at d = 152
    assert flops.paper_convention(16380, 9084, 152) == 1336226651784


def test_traffic_only_for_the_profiled_source(tmp_path, monkeypatch):
    digest = bench.kernel_source_digest()
    t = json.load(open(os.path.join(ROOT, "profiles", "conv_layer_kernel_p1_10d_d152_traffic.json")))
    got = bench.traffic_from_profile(digest, 4)
    if t["kernel_source_sha256"] == digest:
        assert got == t["hbm_bytes_per_launch"]
    else:
        assert got is None
    assert bench.traffic_from_profile("0" * 64, 4) is None

"""Write tests/golden/digests.json: SHA-256 of the oracle's value and gradient
for the full-size workloads whose oracle run is too slow for a test.

Calls only the CPU oracle (oracle/) and the seeded input generator; nothing
here comes from the HIP path.  Run:  python tests/golden/make_digests.py
"""
import hashlib
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402
from paper_2101_10881_amd import workloads as W  # noqa: E402


def digest(a) -> str:
    return hashlib.sha256(a.astype("<f8").tobytes()).hexdigest()


def main():
    out = {"_source": "oracle/oracle.c via tests/golden/make_digests.py; inputs from paper_2101_10881_amd.workloads",
           "workloads": {}}
    for name, w in (("p1_10d_d152", W.p1()), ("p1_10d_d152_complex", W.p1(cx=True))):
        t = time.time()
        val, grad = O.eval_workload(w, nthreads=os.cpu_count())
        out["workloads"][name] = {
            "name": w.name, "m": w.m, "d": w.d, "n": w.n, "N": w.N, "seed": 1,
            "value_sha256": digest(val), "grad_sha256": digest(grad),
            "value_head": [float(v).hex() for v in val[..., 0].ravel()],
            "grad_head": [float(v).hex() for v in grad[..., 0, 0].ravel()],
        }
        print(name, "%.1fs" % (time.time() - t), flush=True)
    with open(os.path.join(HERE, "digests.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()

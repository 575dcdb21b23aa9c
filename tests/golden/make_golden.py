"""Write tests/golden/plain_small_digest.json.

Calls only graphgen (inputs) and oracle (expected values).  The digest pins
the seeded ER n=512 workload (p=0.05, int32 weights U{1..100}) and the
oracle's solution of it, so that an accidental change to either shows up.
"""
import hashlib
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import graphgen as gg  # noqa: E402
import oracle  # noqa: E402


def main():
    W, _ = gg.plain_small(0)
    D = oracle.fw(W, threads=4).astype(np.int32)
    out = {
        "_source": "graphgen.plain_small(0) solved by oracle.fw; written by make_golden.py",
        "n": int(W.shape[0]),
        "input_sha256": hashlib.sha256(np.ascontiguousarray(W).tobytes()).hexdigest(),
        "output_sha256": hashlib.sha256(D.tobytes()).hexdigest(),
        "sum": int(D.astype(np.int64).sum()),
        "max": int(D.max()),
    }
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "plain_small_digest.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=2)
        f.write("\n")
    print(path)


if __name__ == "__main__":
    main()

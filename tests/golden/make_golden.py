"""Write tests/golden/structure.json from the FP64 oracle alone.

For each named workload this records the basis dimension, the number of stored
entries and SHA-256 digests of the full upper-triangle structure (row_ptr as
little-endian int64, col as little-endian int32) and of the two-body key list
(little-endian int32 [n_tbme][4]).  The oracle finds every row's columns by
testing all j >= i, so this takes a few minutes on 8 cores for the largest
workload.  Run:  python tests/golden/make_golden.py
"""
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import seeded_inputs as si  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "structure.json")


def digest(a: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def main(names):
    data = {}
    if os.path.exists(OUT):
        with open(OUT) as f:
            data = json.load(f)
    for name in names:
        p = si.WORKLOADS[name]["problem"]
        t = time.time()
        o = oracle.Oracle(oracle.Problem(*p))
        rows = np.arange(o.dim, dtype=np.int64)
        counts = o.row_counts(rows)
        rp = np.zeros(o.dim + 1, np.int64)
        rp[1:] = np.cumsum(counts)
        _, cols, _ = o.rows(rows, values=False)
        data[name] = {
            "problem": list(p),
            "dim": o.dim,
            "nnz": int(rp[-1]),
            "n_tbme": o.n_tbme,
            "row_ptr_sha256": digest(rp.astype("<i8")),
            "col_sha256": digest(cols.astype("<i4")),
            "tbme_keys_sha256": digest(o.tbme_keys().astype("<i4")),
        }
        print(name, data[name], "%.1fs" % (time.time() - t), flush=True)
        with open(OUT, "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)


if __name__ == "__main__":
    main(sys.argv[1:] or ["he4_nmax2", "li6_nmax6", "b10_nmax4"])

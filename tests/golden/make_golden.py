"""Write tests/golden/full_size.json: the CPU oracle's kappa on the full-size
workloads, as digests (the arrays themselves are hundreds of MB).

Calls only ``oracle`` (Alg. Peeling) and ``synth`` (the seeded inputs); no
value comes from the HIP library.  Usage, from the repository root:

    python tests/golden/make_golden.py cl20 cl23 [sbm] [--threads 8]

Each entry records the r-clique count, the digest of kappa as little-endian
int32 in lexicographic r-clique order, and a few summaries (max, sum, the
number of r-cliques per kappa value) that help when a digest differs.
"""

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
from synth import WORKLOADS, workload  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "full_size.json")


def digest(kappa: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(kappa, dtype="<i4").tobytes()).hexdigest()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("names", nargs="+", choices=sorted(WORKLOADS))
    ap.add_argument("--threads", type=int, default=oracle.default_threads())
    args = ap.parse_args()
    data = json.load(open(OUT)) if os.path.exists(OUT) else {}
    for name in args.names:
        kind = WORKLOADS[name]["kind"]
        r, s = oracle.KINDS[kind]
        t0 = time.time()
        raw = workload(name)
        og = oracle.Graph.from_raw(raw)
        kappa = og.peel(r, s, threads=args.threads)
        vals, counts = np.unique(kappa, return_counts=True)
        data[name] = {
            "kind": kind,
            "generator": raw.name,
            "n_rcliques": int(kappa.size),
            "kappa_sha256": digest(kappa),
            "kappa_max": int(kappa.max()) if kappa.size else 0,
            "kappa_sum": int(kappa.astype(np.int64).sum()),
            "kappa_histogram": {int(v): int(c) for v, c in zip(vals, counts)},
            "oracle_seconds": round(time.time() - t0, 1),
        }
        json.dump(data, open(OUT, "w"), indent=1, sort_keys=True)
        print(name, data[name]["n_rcliques"], data[name]["kappa_sha256"],
              data[name]["oracle_seconds"], "s", flush=True)


if __name__ == "__main__":
    main()

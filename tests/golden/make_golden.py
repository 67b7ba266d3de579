"""Write tests/golden/full_size.json: the CPU oracle's kappa on the full-size
workloads, as digests (the arrays themselves are hundreds of MB).

Calls only ``oracle`` (Alg. Peeling) and ``synth`` (the seeded inputs); no
value comes from the HIP library.  Usage, from the repository root:

    python tests/golden/make_golden.py cl20 cl23 [sbm] [--threads 8]

Each entry records the r-clique count, the digest of kappa as little-endian
int32 in lexicographic r-clique order, and a few summaries (max, sum, the
number of r-cliques per kappa value) that help when a digest differs.

The (3,4) block-model workload (4.2*10^8 triangles) is too slow for one
sequential Alg. Peeling, so it is split, exactly: Alg. Peeling runs on the
subgraph induced by each community (a process pool), and each community's
result is placed at its triangles' ids in the whole graph's lexicographic
triangle list.  This is the whole graph's kappa when every 4-clique lies
inside one community: then the s-cliques of the whole graph are those of
the communities, a triangle's S-degree and every step of the peeling only
involve its own community's 4-cliques, and the triangles outside every
community are in no 4-clique (kappa 0).  The script checks that condition:
the sum of d_4 over the whole graph (the oracle's S-degree count) must equal
the sum over the communities, and fails otherwise.
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


def _community_kappa(task):
    """Alg. Peeling (3,4) on one community's induced subgraph; returns its
    triangles (global vertex ids), their kappa and the sum of their d_4."""
    verts, src, dst = task
    og = oracle.Graph(verts.size, np.searchsorted(verts, src),
                      np.searchsorted(verts, dst))
    tri = og.rcliques(3)
    kap = og.peel(3, 4, threads=1)
    dsum = int(og.sdeg(3, 4, 1).astype(np.int64).sum())
    return verts[tri], kap, dsum


def kappa_by_community(raw, labels, threads):
    """kappa of the (3,4) decomposition of the whole block model from the
    oracle on each community (see the module doc for why it is exact)."""
    from concurrent.futures import ProcessPoolExecutor

    og = oracle.Graph.from_raw(raw)
    tris = og.rcliques(3)
    n = np.int64(raw.n)
    key = (tris[:, 0].astype(np.int64) * n + tris[:, 1]) * n + tris[:, 2]
    del tris
    assert np.all(key[1:] > key[:-1]), "triangles not in lexicographic order"
    total = int(og.sdeg(3, 4, threads).astype(np.int64).sum())
    del og
    intra = labels[raw.src] == labels[raw.dst]
    es, ed = raw.src[intra], raw.dst[intra]
    el = labels[es]
    order = np.argsort(el, kind="stable")
    es, ed, el = es[order], ed[order], el[order]
    vorder = np.argsort(labels, kind="stable")
    ncomm = int(labels.max()) + 1
    vb = np.searchsorted(labels[vorder], np.arange(ncomm + 1))
    eb = np.searchsorted(el, np.arange(ncomm + 1))
    tasks = [(np.sort(vorder[vb[c]:vb[c + 1]]).astype(np.int32),
              es[eb[c]:eb[c + 1]], ed[eb[c]:eb[c + 1]]) for c in range(ncomm)]
    kappa = np.zeros(key.size, np.int32)
    got = 0
    with ProcessPoolExecutor(threads) as ex:
        for g, kap, dsum in ex.map(_community_kappa, tasks, chunksize=8):
            k = (g[:, 0].astype(np.int64) * n + g[:, 1]) * n + g[:, 2]
            idx = np.searchsorted(key, k)
            assert np.array_equal(key[idx], k), "community triangle not found"
            kappa[idx] = kap
            got += dsum
    if got != total:
        raise RuntimeError(f"4-cliques span communities ({got} != {total} "
                           "incidences): run the whole-graph peeling instead")
    return kappa


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
        if name == "sbm":
            from synth import sbm
            raw, labels = sbm(seed=4, with_communities=True)
            raw.name = name + ":" + raw.name
            kappa = kappa_by_community(raw, labels, args.threads)
        else:
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

"""Benchmark: (3,4)-nucleus decomposition of a stochastic block model
(5000 communities of U{50..400} vertices, p_in 0.3, p_out 2e-6; 1.13M
vertices, 4.2e8 triangles, 3.6e9 triangle-4-clique incidences) on one
MI355X -- the largest single-GPU configuration of the workloads.

One step is the whole path on a graph whose raw edge list is already in HBM:
canonical CSR -> edge and triangle numbering -> 4-clique incidence lists ->
d_s -> SND sweeps (notification frontier on) until a sweep changes nothing.
``value`` is the r-clique h-index evaluations the step performs (the
frontier skips r-cliques that cannot change; the iterates are those of
plain SND) per second of step time; the step time itself is the
time-to-exact-convergence including preparation.

Also reported on the same line:
  * ``roofline``: the update kernel in full sweeps (every r-clique with
    d_s > 0 recomputed) on the same prepared graph: algorithmic bytes (see
    sweep_bytes) over its device time per sweep (HIP events on the
    library's stream), against the 8 TB/s HBM peak; ``traffic`` from the
    committed rocprofv3 counters when they were taken on the current sweep
    kernels (else null);
  * ``ceilings``: a streaming read, a streaming copy and the sweep's gather
    pattern alone (its id stream and tau gathers, no h-index) measured on
    this device, with the update kernel's fraction of each;
  * ``and``: the same graph decomposed by AND;
  * ``truss_cl20`` / ``core_cl23``: the k-truss (Chung-Lu 2^20) and k-core
    (Chung-Lu 2^23) workloads: SND and AND time to exact with and without
    preparation, full-sweep roofline; for k-core the fraction of exact
    values and of active r-cliques after every sweep;
  * ``stream`` / ``small_graphs``: batched and served k-truss against one
    graph per launch on a sample of the request-stream workload;
  * ``ego``: PartialAND estimates on ego networks of random cl20 edges;
  * ``cpu_baseline``: the CPU oracle's update operator timed on the host
    over a bounded sample of the block model's triangles.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu]
"""

from __future__ import annotations

import argparse
import ctypes
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
HEADLINE = "sbm"
HEADLINE_KIND = "nucleus34"
STREAM_BUDGET = 96 << 30  # device-memory budget of the served stream
K_OF = {"core": 1, "truss": 2, "nucleus34": 3}
TAU_CTYPE = {1: "u8", 2: "u16", 4: "i32"}


def progress(msg: str) -> None:
    """A line on stderr when a step or leg has finished (stdout carries only
    the result line)."""
    print(f"bench: {msg}", file=sys.stderr, flush=True)


def sweep_bytes(P: int, nr_eval: int, k: int, tb: int) -> int:
    """Algorithmic bytes of one full sweep over the nr_eval r-cliques with
    d_s > 0: the id stream (4 bytes x kP), one tau gather per id (tb x kP,
    tb = bytes per stored tau), int64 offsets (8 per r-clique), own tau read
    and new tau written (2 tb per r-clique)."""
    return (4 + tb) * k * P + (8 + 2 * tb) * nr_eval


def cpu_baseline(budget_s=10.0, seed=4):
    """The oracle's update operator on the triangles of whole communities of
    the block model, taken as one graph: the disjoint union of the sampled
    communities' induced subgraphs.  No 4-clique of this workload leaves a
    community (the full-size digest checks it), so U on those triangles is
    the same there as in the whole graph.  Communities are drawn at random;
    their number is calibrated so that U takes about budget_s."""
    import numpy as np

    import oracle
    from synth import sbm

    raw, labels = sbm(seed=seed, with_communities=True)
    threads = oracle.default_threads()
    intra = labels[raw.src] == labels[raw.dst]
    es, ed, el = raw.src[intra], raw.dst[intra], labels[raw.src[intra]]
    ncomm = int(labels.max()) + 1
    order = np.random.default_rng(seed + 1).permutation(ncomm)

    def union_of(comms):
        pick = np.isin(el, comms)
        s, d = es[pick], ed[pick]
        verts = np.unique(np.concatenate([s, d]))
        return (verts.size, np.searchsorted(verts, s).astype(np.int32),
                np.searchsorted(verts, d).astype(np.int32))

    def time_u(comms):
        n, s, d = union_of(comms)
        og = oracle.Graph(n, s, d)
        ds = og.sdeg(3, 4, threads)
        t = time.perf_counter()
        og.update(3, 4, ds, threads=threads)
        dt = time.perf_counter() - t
        return int(np.count_nonzero(ds)), dt, og.num_rcliques(3)

    def time_peel(comms):  # the oracle's Alg. Peeling, S-degrees included
        n, s, d = union_of(comms)
        og = oracle.Graph(n, s, d)
        inc = int(og.sdeg(3, 4, threads).sum())
        t = time.perf_counter()
        og.peel(3, 4, threads)
        return time.perf_counter() - t, og.num_rcliques(3), inc

    upd0, dt0, _ = time_u(order[:20])
    want = int(min(ncomm, max(20, 20 * budget_s / max(dt0, 1e-6))))
    upd, dt, nt = time_u(order[:want])
    pt, pnt, pinc = time_peel(order[:3])
    want_p = int(min(ncomm, max(3, 3 * budget_s / max(pt, 1e-6))))
    if want_p > 3:
        pt, pnt, pinc = time_peel(order[:want_p])
    return {"value": upd / dt, "unit": "r-clique h-index updates/s",
            "cores": threads, "kind": "oracle",
            "sample": f"U applied to the {nt} triangles ({upd} with d_s > 0, "
                      f"tau = d_s) of {want} of the {ncomm} communities "
                      f"(random, seed {seed + 1}) in {dt:.1f} s",
            "peeling": {"s": pt, "triangles": pnt, "incidence_P": pinc,
                        "incidence_per_s": pinc / pt, "cores": threads,
                        "sample": f"Alg. Peeling (S-degrees, then bucket peeling) "
                                  f"of the {pnt} triangles of {want_p} communities "
                                  f"(the same draw)"}}


def sweep_source_hash() -> str:
    """Hash of the sources that define the sweep kernels and the r-clique
    order they gather in."""
    import hashlib
    h = hashlib.sha256()
    for f in ("sweep.hip", "sweep_dev.h", "layout.hip"):
        with open(os.path.join(ROOT, "paper_1704_00386_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_sweep_sbm_nucleus34.json")


def measured_traffic():
    """HBM bytes per full sweep of the headline workload from the committed
    rocprofv3 counter record, or None when it is missing or was taken on
    different sweep kernels."""
    try:
        rec = json.load(open(TRAFFIC_FILE))
    except (OSError, ValueError):
        return None
    if rec.get("sweep_source_sha256") != sweep_source_hash():
        return None
    return rec.get("hbm_bytes_per_sweep")


FULL_SWEEP_SUFFIX = ", false, false>"  # k_sweep_*<..., AND, frontier>
HEADLINE_FLAGS = "--only-headline --steps 2 --warmup 1 --calib-copy"


def _short_kernel(name: str) -> str:
    name = name.replace("void ", "").replace("nd::(anonymous namespace)::", "")
    i = name.find(">(")
    return name[:i + 1] if i >= 0 else name


def _profile_command(args_extra: str, out: str) -> str:
    return (f"rocprofv3 {args_extra} --output-format csv -d $OUT/{out} -o {out} "
            f"-- python3 $R/bench.py {HEADLINE_FLAGS}")


def summarize_profiles(trace_csv: str, fetch_csv: str, write_csv: str) -> None:
    """Write the committed profile summaries of the headline workload from
    the CSV output of three rocprofv3 runs of `bench.py --only-headline`
    (see the commands recorded in them): the kernel trace statistics, and
    FETCH_SIZE / WRITE_SIZE per dispatch, scaled by what the same counters
    read for the 1 GiB device copy that --calib-copy makes first."""
    import csv
    import statistics

    out_dir = os.path.join(ROOT, "profiles")
    rows = list(csv.DictReader(open(trace_csv)))
    tot = sum(float(r["TotalDurationNs"]) for r in rows)
    lines = ["# Kernel trace: the headline leg ((3,4) SND on the block model)", "",
             "Command (run from /tmp, `TMPDIR=/tmp`, repo at `$R`, output under `$OUT`):", "", "```",
             _profile_command("--kernel-trace --stats", "kt"), "```", "",
             "The run holds a 1 GiB device copy, one warm-up and two timed steps (build + prepare +",
             "SND with the notification frontier until exact), the full-sweep roofline leg (4 SND",
             "sweeps recomputing every r-clique), AND with the frontier, and the ceiling kernels.",
             "`k_sweep_small<k, tau type, AND, frontier>` sweeps the bins of at most 16 values per",
             "lane (d_s 1..1024) in one launch; `<3, unsigned char, false, false>` is the full sweep",
             "(tau in 8 bits: every d_s of this workload is below 256).", "",
             "| % | calls | total ms | avg us | kernel |", "|---:|---:|---:|---:|---|"]
    full_avg = 0.0
    for r in sorted(rows, key=lambda r: -float(r["TotalDurationNs"]))[:36]:
        name = _short_kernel(r["Name"])
        avg = float(r["AverageNs"]) / 1e3
        if name.startswith("k_sweep_") and name.endswith(FULL_SWEEP_SUFFIX):
            full_avg += avg
        lines.append(f"| {100 * float(r['TotalDurationNs']) / tot:.1f} | {r['Calls']} | "
                     f"{float(r['TotalDurationNs']) / 1e6:.2f} | {avg:.1f} | `{name}` |")
    lines += ["", f"Full sweep = the `k_sweep_*<..., false, false>` launches of a sweep: "
              f"{full_avg:.0f} us per sweep (sum of their averages)."]
    open(os.path.join(out_dir, "kernel_trace_sbm_nucleus34.md"), "w").write("\n".join(lines) + "\n")

    def per_kernel(path, counter):
        vals, copy = {}, []
        for r in csv.DictReader(open(path)):
            if r["Counter_Name"] != counter:
                continue
            name = _short_kernel(r["Kernel_Name"])
            v = float(r["Counter_Value"])
            if "copyBuffer" in name:
                copy.append(v)
            vals.setdefault(name, []).append(v)
        return vals, max(copy)

    fetch, fcopy = per_kernel(fetch_csv, "FETCH_SIZE")
    write, wcopy = per_kernel(write_csv, "WRITE_SIZE")
    gib_kib = float(1 << 20)  # the copy moves 1 GiB each way
    fscale, wscale = gib_kib / fcopy, gib_kib / wcopy
    full = sorted(k for k in fetch if k.startswith("k_sweep_") and k.endswith(FULL_SWEEP_SUFFIX))
    f_kib = sum(statistics.mean(fetch[k]) for k in full)
    w_kib = sum(statistics.mean(write.get(k, [0.0])) for k in full)
    rec = {
        "workload": "(3,4) SND, full sweeps, block model (5000 communities of U{50..400}, "
                    "p_in 0.3, p_out 2e-6, seed 4)",
        "kernels": full,
        "fetch_bytes_per_sweep": f_kib * 1024 * fscale,
        "write_bytes_per_sweep": w_kib * 1024 * wscale,
        "hbm_bytes_per_sweep": (f_kib * fscale + w_kib * wscale) * 1024,
        "fetch_scale": fscale, "write_scale": wscale,
        "scale_from": "1 GiB device-to-device copy (__amd_rocclr_copyBuffer) in the same run",
        "sweep_source_sha256": sweep_source_hash(),
        "commands": [_profile_command("--pmc FETCH_SIZE", "pf"),
                     _profile_command("--pmc WRITE_SIZE", "pw")],
    }
    json.dump(rec, open(TRAFFIC_FILE, "w"), indent=1)
    md = ["# HBM-side traffic of one full sweep ((3,4) SND, block model)", "",
          "Counters per dispatch (KiB), averaged over the full sweeps of the roofline leg and summed over",
          "the bin kernels of a sweep, then scaled by what the same counter reads for a 1 GiB",
          f"device-to-device copy in the same run (FETCH_SIZE reads {fcopy / 1024:.0f} MiB for it, "
          f"WRITE_SIZE {wcopy / 1024:.0f} MiB):", "",
          f"- fetch scale {fscale:.3f}, write scale {wscale:.3f}",
          f"- FETCH per sweep: {rec['fetch_bytes_per_sweep'] / 2**30:.2f} GiB",
          f"- WRITE per sweep: {rec['write_bytes_per_sweep'] / 2**30:.3f} GiB", "",
          "Per kernel (unscaled KiB averages):", "", "| kernel | FETCH_SIZE KiB | WRITE_SIZE KiB |",
          "|---|---:|---:|"]
    for k in full:
        md.append(f"| `{k}` | {statistics.mean(fetch[k]):.0f} | {statistics.mean(write.get(k, [0.0])):.0f} |")
    md += ["", "Commands (run from /tmp, `TMPDIR=/tmp`, repo at `$R`, output under `$OUT`), then "
           "`python bench.py --summarize-profiles <trace stats csv> <fetch csv> <write csv>`:", "", "```",
           *rec["commands"], "```", "",
           "These counters measure L2-to-fabric traffic, which includes Infinity Cache (MALL) hits,",
           "so they bound DRAM bytes from above."]
    open(os.path.join(out_dir, "traffic_sweep_sbm_nucleus34.md"), "w").write("\n".join(md) + "\n")

    # preparation: every kernel that is neither a sweep nor a ceiling or copy
    # kernel, by total time, with its scaled traffic per dispatch
    skip = ("k_sweep_", "k_gather", "k_read", "k_copy", "__amd", "at::",
            "k_incidence_original", "k_to_original")

    def is_prep(r):
        return not _short_kernel(r["Name"]).replace(
            "(anonymous namespace)::", "").startswith(skip)

    prep = [r for r in rows if is_prep(r)]
    prep.sort(key=lambda r: -float(r["TotalDurationNs"]))
    pm = ["# Preparation kernels: time and HBM-side traffic ((3,4), block model)", "",
          "Per dispatch, from the same three runs as the sweep's traffic record: the kernel-trace",
          "average duration, FETCH_SIZE and WRITE_SIZE averaged over the dispatches and scaled",
          f"by the 1 GiB copy (fetch x{fscale:.3f}, write x{wscale:.3f}), and their sum over the",
          "duration. Each step (the warm-up and two timed) prepares the graph once.",
          "`k_n34_vertex<D, pass>`: pass 0 bit rows and triangle counts, 1 triangles, 2 S-degrees",
          "and local counts, 3 the 4-cliques' entries (D: the degree class).", "",
          "| kernel | calls | avg ms | FETCH GB | WRITE GB | GB/s |", "|---|---:|---:|---:|---:|---:|"]
    for r in prep[:16]:
        name = _short_kernel(r["Name"])
        avg_ms = float(r["AverageNs"]) / 1e6
        fb = statistics.mean(fetch.get(name, [0.0])) * 1024 * fscale / 1e9
        wb = statistics.mean(write.get(name, [0.0])) * 1024 * wscale / 1e9
        pm.append(f"| `{name}` | {r['Calls']} | {avg_ms:.2f} | {fb:.2f} | {wb:.2f} | "
                  f"{(fb + wb) / (avg_ms * 1e-3):.0f} |")
    pm += ["", "Commands: the three of the sweep's traffic record, then "
           "`python bench.py --summarize-profiles <trace stats csv> <fetch csv> <write csv>`:", "", "```",
           _profile_command("--kernel-trace --stats", "kt"), *rec["commands"], "```"]
    open(os.path.join(out_dir, "traffic_prep_sbm_nucleus34.md"), "w").write("\n".join(pm) + "\n")
    print(f"full sweep {full_avg:.0f} us; HBM-side {rec['hbm_bytes_per_sweep'] / 1e9:.2f} GB per sweep")


def summarize_quality(json_path: str) -> None:
    """profiles/quality_<workload>_<kind>.md from the JSON line printed by
    `python bench.py --quality <workload>`."""
    q = json.loads(open(json_path).read().strip().splitlines()[-1])
    name, kind = q["workload"], q["kind"]
    L = [f"# Accuracy per sweep: {kind} on the `{name}` workload ({q['n_rcliques']} r-cliques)", "",
         f"Command (repo root): `python bench.py --quality {name}`", "",
         "`fraction_exact`: share of all r-cliques with tau_t = kappa.  `kendall_tau`: scipy's tau-b of",
         f"tau_t against kappa on a uniform sample of {q['kendall_sample']} r-cliques.  `active`: share of",
         "all r-cliques that the notifications flag for the next sweep (the indicator of Section",
         "5.1.4).  `changed`: share that changed in the sweep.  `ms_cum`: summed device time of",
         "sweeps 1..t (events around each sweep's launches; sweeps run one at a time and count the",
         "active flags here).", "",
         f"Degree levels (Defn. 4; the bound on SND sweeps): {q['degree_levels']}.  "
         f"SND sweeps: {len(q['snd']['rows']) - 1}; AND sweeps: {len(q['and']['rows']) - 1}."]
    for mode in ("snd", "and"):
        m = q[mode]
        L += ["", f"## {mode.upper()}", "",
              "Stops: after the first sweep whose active (paper's indicator) or changed share falls",
              "below the ratio:", "",
              "| ratio | by | sweep | ms | fraction exact | Kendall-Tau |",
              "|---:|---|---:|---:|---:|---:|"]
        for by in ("active", "changed"):
            for ratio, st in m[f"{by}_ratio_stops"].items():
                L.append(f"| {ratio} | {by} | {st['sweep']} | {st['ms_cum']:.2f} | "
                         f"{st['fraction_exact']:.4f} | {st['kendall_tau']:.4f} |")
        L += ["", "| sweep | active | changed | ms (cum.) | fraction exact | Kendall-Tau |",
              "|---:|---:|---:|---:|---:|---:|"]
        nr = q["n_rcliques"]
        for r in m["rows"]:
            a = "" if r["active"] is None else f"{r['active'] / nr:.5f}"
            c = "" if r["changed"] is None else f"{r['changed'] / nr:.5f}"
            L.append(f"| {r['sweep']} | {a} | {c} | {r['ms_cum']:.2f} | {r['fraction_exact']:.5f} | "
                     f"{r['kendall_tau']:.5f} |")
    path = os.path.join(ROOT, "profiles", f"quality_{name}_{kind}.md")
    open(path, "w").write("\n".join(L) + "\n")
    print(path)


TRACE_RUNS = {
    "stream_truss": ("batched and served k-truss on a sample of the request-stream workload "
                     "(the stream leg alone)", "--only-stream"),
}


def summarize_trace(stats_csv: str, name: str) -> None:
    """profiles/kernel_trace_<name>.md from the kernel-stats CSV of
    `rocprofv3 --kernel-trace --stats -- python3 bench.py <flags>`."""
    import csv

    what, flags = TRACE_RUNS[name]
    rows = list(csv.DictReader(open(stats_csv)))
    tot = sum(float(r["TotalDurationNs"]) for r in rows)
    lines = [f"# Kernel trace: {name}", "", what + ".", "",
             "Command (run from /tmp, `TMPDIR=/tmp`, repo at `$R`, output under `$OUT`):", "", "```",
             f"rocprofv3 --kernel-trace --stats --output-format csv -d $OUT/{name} "
             f"-o {name} -- python3 $R/bench.py {flags}", "```", "",
             f"Total kernel time {tot / 1e6:.1f} ms.", "",
             "| % | calls | total ms | avg us | kernel |", "|---:|---:|---:|---:|---|"]
    for r in sorted(rows, key=lambda r: -float(r["TotalDurationNs"]))[:30]:
        lines.append(f"| {100 * float(r['TotalDurationNs']) / tot:.1f} | {r['Calls']} | "
                     f"{float(r['TotalDurationNs']) / 1e6:.2f} | "
                     f"{float(r['AverageNs']) / 1e3:.1f} | `{_short_kernel(r['Name'])}` |")
    path = os.path.join(ROOT, "profiles", f"kernel_trace_{name}.md")
    open(path, "w").write("\n".join(lines) + "\n")
    print(path)


# ----------------------------------------------------------------- legs


def device_edges(raw):
    import torch
    src = torch.from_numpy(raw.src).cuda()
    dst = torch.from_numpy(raw.dst).cuda()
    torch.cuda.synchronize()
    return src, dst


def timed_steps(nd, ctx, raw, src, dst, kind, steps, warmup, mode="snd"):
    """Build + prepare + decompose (frontier on) from the edge list in HBM,
    `warmup` untimed then `steps` timed; returns (last graph, kappa, results,
    step times in ms)."""
    import torch

    def step():
        g = nd.Graph.from_edges(ctx, raw.n, src, dst)
        kappa, res = g.decompose(kind, mode, use_frontier=True)
        return g, kappa, res

    for _ in range(warmup):
        g, _, _ = step()
        g.close()
    torch.cuda.synchronize()
    times, results = [], []
    g = kappa = None
    for i in range(steps):
        if g is not None:
            g.close()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g, kappa, res = step()
        torch.cuda.synchronize()
        times.append(1e3 * (time.perf_counter() - t0))
        results.append(res)
        progress(f"{raw.name} {kind} {mode} step {i + 1}/{steps}: {times[-1]:.1f} ms")
    return g, kappa, results, times


def full_sweep_roofline(g, kind, res, sweeps=None):
    """Full SND sweeps (every r-clique with d_s > 0 recomputed) on a prepared
    graph, each timed with HIP events on the library's stream (nd_iter_info.ms);
    algorithmic bytes per sweep over the mean sweep time."""
    import numpy as np

    nr_eval = int(np.count_nonzero(g.sdegree(kind).cpu().numpy()))
    ms = []

    def collect(info):
        ms.append(info.ms)
        return 0

    kfull, rfull = g.decompose(kind, "snd", on_iter=collect,
                               max_iters=-1 if sweeps is None else sweeps,
                               allow_not_converged=True)
    B = sweep_bytes(res["n_incidence"], nr_eval, K_OF[kind], res["tau_bytes"])
    avg = sum(ms) / len(ms)
    return {"nr_eval": nr_eval, "bytes_per_sweep": B, "avg_sweep_ms": avg,
            "sweeps_timed": len(ms), "achieved_GBs": B / (avg * 1e-3) / 1e9,
            "kappa": kfull, "res": rfull}


def _ceiling_lib():
    lib = ctypes.CDLL(os.path.join(ROOT, "paper_1704_00386_amd", "libndceil.so"))
    lib.ndc_read.restype = ctypes.c_float
    lib.ndc_read.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                             ctypes.c_void_p]
    lib.ndc_copy.restype = ctypes.c_float
    lib.ndc_copy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                             ctypes.c_void_p]
    lib.ndc_gather.restype = ctypes.c_float
    lib.ndc_gather.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int,
                               ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p,
                               ctypes.c_void_p]
    return lib


def gather_ceiling(g, kind, tau_bytes):
    """The gather pattern alone (the id stream and one tau gather per id, min
    per s-clique, no h-index) over the incidence as exported: r-cliques in
    their original order, ids original.  GB/s of (4 + tau bytes) per
    incidence id, best of 3, timed with events on the current stream by
    libndceil.so."""
    import torch

    lib = _ceiling_lib()
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    sink = torch.zeros(1, dtype=torch.int64, device="cuda")
    off, ids = g.incidence(kind)
    k = ids.shape[1]
    ds = g.sdegree(kind)
    tau = {1: torch.uint8, 2: torch.int16, 4: torch.int32}[tau_bytes]
    tau = ds.to(tau)
    del off
    nsets = ids.shape[0]
    gathers = [lib.ndc_gather(ids.data_ptr(), nsets, k, tau.data_ptr(),
                              tau_bytes, sink.data_ptr(), st)
               for _ in range(3)]
    del ids, tau
    torch.cuda.synchronize()
    gb = (4 + tau_bytes) * k * nsets
    return {"gather_GBs": gb / (min(gathers) * 1e-3) / 1e9,
            "gather_bytes": gb, "gather_ms": min(gathers)}


def ceilings(nd, g, kind, tau_bytes):
    """Streaming read, streaming copy and the sweep's gather pattern (its id
    stream and tau gathers without the h-index) on this device, timed with
    events on the current stream by libndceil.so."""
    import torch

    lib = _ceiling_lib()
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    sink = torch.zeros(1, dtype=torch.int64, device="cuda")
    nbytes = 8 << 30
    a = torch.empty(nbytes // 4, dtype=torch.int32, device="cuda").fill_(1)
    b = torch.empty_like(a)
    reads = [lib.ndc_read(a.data_ptr(), nbytes, sink.data_ptr(), st) for _ in range(3)]
    copies = [lib.ndc_copy(a.data_ptr(), b.data_ptr(), nbytes, st) for _ in range(3)]
    del a, b, sink
    torch.cuda.synchronize()
    out = {"read_GBs": nbytes / (min(reads) * 1e-3) / 1e9,
           "copy_GBs": 2 * nbytes / (min(copies) * 1e-3) / 1e9}
    out.update(gather_ceiling(g, kind, tau_bytes))
    out["what"] = ("8 GiB streamed with 16-byte loads (read) and loads+stores "
                   "(copy); the incidence as exported (original r-clique order "
                   "and ids, each workgroup streaming contiguous runs of 32768 "
                   f"lists) with one {tau_bytes}-byte tau gather per id, min per "
                   "s-clique (gather); best of 3 each")
    return out


def headline_leg(nd, ctx, args):
    """The headline: (3,4) SND with the frontier on the block model, then the
    full-sweep roofline, AND and the ceilings on the prepared graph."""
    import numpy as np
    import torch

    from synth import workload

    raw = workload(HEADLINE)
    src, dst = device_edges(raw)
    g, kappa, results, times = timed_steps(nd, ctx, raw, src, dst, HEADLINE_KIND,
                                           args.steps, args.warmup)
    del src, dst
    res = results[-1]
    ms_step = sum(times) / len(times)
    nr_eval = int(np.count_nonzero(g.sdegree(HEADLINE_KIND).cpu().numpy()))
    roof = full_sweep_roofline(g, HEADLINE_KIND, res, sweeps=4)
    kand, rand = g.decompose(HEADLINE_KIND, "and", use_frontier=True)
    out = {"raw": raw, "g": g, "kappa": kappa, "res": res, "times": times,
           "ms_step": ms_step, "nr_eval": nr_eval, "roof": roof,
           "and": {"sweeps": rand["sweeps"], "ms_iterate": rand["ms_iterate"],
                   "frontier": True,
                   "kappa_equals_snd": bool(torch.equal(kand, kappa))}}
    del kand
    progress("headline roofline and AND legs done")
    if not args.no_ceilings:
        out["ceilings"] = ceilings(nd, g, HEADLINE_KIND, res["tau_bytes"])
        progress("ceilings done")
    return out


def workload_leg(nd, ctx, name, kind, quality=False):
    """One of the other single-GPU workloads: SND and AND (frontier) time to
    exact with and without preparation (one warm step, then one timed), the
    full-sweep roofline, and with `quality` the fraction of exact values and
    of active r-cliques after every SND sweep."""
    import numpy as np
    import torch

    from synth import workload

    raw = workload(name)
    src, dst = device_edges(raw)
    out = {"workload": raw.name, "kind": kind}
    g = kappa = None
    for mode in ("snd", "and"):
        if g is not None:
            g.close()
        g, k, results, times = timed_steps(nd, ctx, raw, src, dst, kind, 1, 1,
                                           mode=mode)
        r = results[-1]
        out[mode] = {"time_to_exact_ms": times[-1], "ms_iterate": r["ms_iterate"],
                     "ms_prep": times[-1] - r["ms_iterate"], "sweeps": r["sweeps"],
                     "evaluated_updates": r["updates"],
                     "evaluated_updates_per_s": r["updates"] / (times[-1] * 1e-3)}
        if kappa is None:
            kappa = k
        else:
            out["kappa_and_equals_snd"] = bool(torch.equal(k, kappa))
    del src, dst
    res = results[-1]
    roof = full_sweep_roofline(g, kind, res)
    out["n_rcliques"] = res["n_rcliques"]
    out["incidence_P"] = res["n_incidence"]
    out["tau_bytes"] = res["tau_bytes"]
    nre = roof["nr_eval"]
    out["snd"]["full_sweep_equivalent_updates_per_s"] = (
        nre * out["snd"]["sweeps"] / (out["snd"]["time_to_exact_ms"] * 1e-3))
    out["full_sweep"] = {"avg_ms": roof["avg_sweep_ms"],
                         "bytes_per_sweep": roof["bytes_per_sweep"],
                         "achieved_GBs": roof["achieved_GBs"],
                         "frac_of_hbm_peak": roof["achieved_GBs"] / HBM_PEAK_GBS,
                         "kappa_equals_frontier": bool(torch.equal(roof["kappa"], kappa))}
    gc = gather_ceiling(g, kind, res["tau_bytes"])
    out["full_sweep"]["gather_original_order_GBs"] = gc["gather_GBs"]
    out["full_sweep"]["sweep_over_original_order_gather"] = (
        roof["achieved_GBs"] / gc["gather_GBs"])
    out["full_sweep"]["gather_what"] = (
        "the gather pattern alone (ids and tau gathers, no h-index) over the "
        "incidence in original r-clique order with original ids; the sweep "
        "runs in the internal (sweep bin, id) numbering, which packs the "
        "values of high-degree r-cliques together, so on power-law graphs it "
        "beats this figure: a measure of what the layout gains, not a bound")
    if quality:
        nr = kappa.numel()
        snap = torch.empty(max(nr, 1), dtype=torch.int32, device="cuda")
        curve = []

        def on_iter(info):
            rc = nd._hip.hipMemcpy(snap.data_ptr(), info.tau_dev, 4 * nr, 3)
            if rc != 0:
                raise RuntimeError(f"hipMemcpy failed ({rc})")
            curve.append({"sweep": int(info.iter),
                          "fraction_exact": int((snap[:nr] == kappa).sum()) / nr,
                          "active": int(info.active_next) / nr,
                          "changed": int(info.changed) / nr})
            return 0

        g.decompose(kind, "snd", use_frontier=True, count_active=True,
                    on_iter=on_iter)
        out["snd_per_sweep"] = curve
    progress(f"{name} leg done")
    return out, g, kappa


def stream_leg(nd, ctx, count, seed=5, n_lo=1000, n_hi=200000, serve=True,
               group=None):
    """Batched and served k-truss against one graph per launch, on `count`
    graphs of the request-stream workload (Chung-Lu, n ~ U{n_lo..n_hi},
    mean degree ~ U[8,64], exponent ~ U[2.0,2.5]).  Edge lists are resident
    in HBM before timing; every path builds, prepares and decomposes its
    graphs (frontier SND, the same iterates as plain SND).  The server runs
    on a context with a device-memory budget of STREAM_BUDGET bytes and
    admits requests by it.  The batched path takes the graphs `group` at a
    time (default: all at once up to 512 graphs, else 256), since all of a
    call's graphs are prepared and resident together."""
    import concurrent.futures as cf

    import numpy as np
    import torch

    from synth import chung_lu, request_stream

    specs = request_stream(count=count, n_lo=n_lo, n_hi=n_hi, seed=seed)
    progress(f"generating {count} stream graphs")
    dev = []
    with cf.ThreadPoolExecutor(8) as ex:
        for a in range(0, count, 256):
            for r in ex.map(lambda sp: chung_lu(sp["n"], sp["beta"], sp["mean"],
                                                sp["seed"]), specs[a:a + 256]):
                dev.append((r.n, torch.from_numpy(r.src).cuda(),
                            torch.from_numpy(r.dst).cuda()))
            if count > 256:
                progress(f"generated {len(dev)} of {count}")
    if group is None:
        group = count if count <= 512 else 256
    kind = "truss"
    updates = 0
    alg_bytes = 0.0
    for n, s, d in dev[:4]:  # warm the allocator and kernels once
        nd.Graph.from_edges(ctx, n, s, d).decompose(kind, "snd", use_frontier=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    solo, solo_ms = [], []
    for n, s, d in dev:
        t1 = time.perf_counter()
        g = nd.Graph.from_edges(ctx, n, s, d)
        k, r = g.decompose(kind, "snd", use_frontier=True)
        solo.append(k)
        updates += r["updates"]
        # algorithmic bytes of the evaluations (ids, tau gathers, offsets and
        # own tau per update, each evaluated r-clique taken at its graph's
        # mean list length)
        if r["n_rcliques"]:
            tb = r["tau_bytes"]
            alg_bytes += r["updates"] * ((4 + tb) * 2 * r["n_incidence"] / r["n_rcliques"]
                                         + 8 + 2 * tb)
        g.close()
        torch.cuda.synchronize()
        solo_ms.append(1e3 * (time.perf_counter() - t1))
    t_solo = time.perf_counter() - t0
    solo = [k.cpu() for k in solo]  # keep HBM for the other paths
    t_built, t_batch, same = 0.0, 0.0, True
    for a in range(0, count, group):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        gs = nd.graphs_from_edges(ctx, dev[a:a + group])
        t_built += time.perf_counter() - t0
        ks, rs = nd.batch_decompose(ctx, gs, kind, "snd", use_frontier=True)
        for g in gs:
            g.close()
        torch.cuda.synchronize()
        t_batch += time.perf_counter() - t0
        same &= all(torch.equal(x.cpu(), y) for x, y in zip(ks, solo[a:a + group]))
        del gs, ks
        if count > group:
            progress(f"batched {min(a + group, count)} of {count}")
    out = {
        "graphs": count,
        "workload": f"request stream of Chung-Lu k-truss graphs, n ~ U{{{n_lo}.."
                    f"{n_hi}}}, mean ~ U[8,64], exponent ~ U[2.0,2.5], seed {seed}",
        "one_per_launch_graphs_per_s": count / t_solo,
        "batched_graphs_per_s": count / t_batch,
        "batched_speedup": t_solo / t_batch,
        "batch_group": group,
        "batched_split_s": {"graph_from_edges": t_built,
                            "batch_decompose": t_batch - t_built},
        "updates": updates,
        "aggregate_algorithmic_GBs": {
            "one_per_launch": alg_bytes / t_solo / 1e9,
            "batched": alg_bytes / t_batch / 1e9,
            "what": "the evaluated h-index updates' algorithmic bytes (id stream, "
                    "tau gathers, offsets and own tau), each evaluated r-clique at "
                    "its graph's mean list length, over the path's wall time "
                    "(build and preparation included); HBM peak 8000 GB/s"},
    }
    if serve:
        # served: Poisson arrivals at 80% of the one-graph-per-launch rate
        sctx = nd.Context(0, hbm_budget_bytes=STREAM_BUDGET)
        rate = 0.8 * count / t_solo
        gaps = np.random.default_rng(seed).exponential(1.0 / rate, size=count)
        arrive = np.cumsum(gaps) - gaps[0]
        import queue
        import threading
        srv = nd.Server(sctx, max_slots=64)
        lag, got, pending = [], [], queue.Queue()

        def collect():  # the results, in submission order, as they finish
            for _ in range(count):
                got.append(srv.wait(pending.get()))

        consumer = threading.Thread(target=collect)
        t0 = time.perf_counter()
        consumer.start()
        for i, (n, s, d) in enumerate(dev):
            while time.perf_counter() - t0 < arrive[i]:
                time.sleep(0.0002)
            pending.put(srv.submit(nd.Graph.from_edges(sctx, n, s, d), kind,
                                   use_frontier=True))
            lag.append(1e3 * (time.perf_counter() - t0 - arrive[i]))
        consumer.join()
        t_srv = time.perf_counter() - t0
        sizes = np.array([int(s.numel()) for _, s, _ in dev])
        lats, slow, joined, peak, prep_overlap = [], [], 0, 0, 0
        for (kappa, r, info), want, ms in zip(got, solo, solo_ms):
            lats.append(info["latency_ms"])
            slow.append(info["latency_ms"] / ms)
            joined += info["joined_running"]
            peak = max(peak, info["peak_members"])
            prep_overlap += info["epochs_during_prep"] > 0
            same &= bool(torch.equal(kappa, want))
        del got
        srv.close()
        del sctx
        out["aggregate_algorithmic_GBs"]["served"] = alg_bytes / t_srv / 1e9
        out["served"] = {"arrival_rate_per_s": rate, "graphs_per_s": count / t_srv,
                         "p50_ms": float(np.percentile(lats, 50)),
                         "p99_ms": float(np.percentile(lats, 99)),
                         # latency over the same graph's one-per-launch time
                         # (the request sizes differ 200-fold, so raw
                         # latency percentiles mostly reflect the sizes)
                         "slowdown_p50": float(np.percentile(slow, 50)),
                         "slowdown_p99": float(np.percentile(slow, 99)),
                         # how far the caller's submissions (graph build
                         # included) fell behind the arrival times
                         # within each half of the requests by edge count
                         "by_size": {
                             h: {"p50_ms": float(np.percentile(np.array(lats)[sel], 50)),
                                 "p99_ms": float(np.percentile(np.array(lats)[sel], 99))}
                             for h, sel in (("smaller_half", sizes <= np.median(sizes)),
                                            ("larger_half", sizes > np.median(sizes)))
                             if sel.any()},
                         "submit_lag_ms_p50": float(np.percentile(lag, 50)),
                         "submit_lag_ms_max": float(np.max(lag)),
                         "hbm_budget_bytes": STREAM_BUDGET,
                         "joined_running_batch": joined,
                         "peak_requests_per_epoch": peak,
                         "prepared_while_sweeping": prep_overlap}
    out["results_identical"] = bool(same)
    progress(f"stream leg ({count} graphs) done")
    return out


def ego_leg(nd, g, kappa, kind, count, seed=13):
    """PartialAND estimates on the ego networks of `count` random r-cliques
    of the prepared graph, all in one call: throughput, and accuracy against
    the exact kappa (share exact, mean relative error) -- the comparison of
    the application of Section 5.3."""
    import numpy as np
    import torch

    nr = kappa.numel()
    q = torch.from_numpy(np.random.default_rng(seed).integers(
        0, nr, size=count).astype(np.int32)).cuda()
    g.ego_estimate(kind, q[:64])  # warm
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    est, sw = g.ego_estimate(kind, q)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    k = kappa[q.long()].to(torch.float64)
    e = est.to(torch.float64)
    rel = ((e - k) / torch.clamp(k, min=1.0)).mean().item()
    return {"queries": count, "ms": 1e3 * dt, "queries_per_s": count / dt,
            "fraction_exact": (est == kappa[q.long()]).double().mean().item(),
            "mean_relative_error": rel,
            "mean_sweeps": sw.double().mean().item(),
            "max_sweeps": int(sw.max().item())}


def quality_leg(nd, name, sample=1_000_000, seed=9):
    """Per-sweep accuracy of the iterates against the exact result (the
    approximation trade-off of Sections 5.1.4 and 5.2.3): fraction of
    r-cliques whose tau_t equals kappa (all of them), the Kendall-Tau
    similarity of tau_t and kappa (scipy's tau-b on a uniform sample of
    r-cliques), the share of active r-cliques (flagged by the
    notifications for the next sweep) and of changed ones, with each
    sweep's device time, for SND and AND on one of the named workloads; and
    the stop points of the active-ratio control at 40% / 10% / 1%, by active
    share (the paper's indicator) and by changed share."""
    import numpy as np
    import scipy.stats
    import torch

    from synth import WORKLOADS, workload

    kind = WORKLOADS[name]["kind"]
    raw = workload(name)
    ctx = nd.Context(0)
    g = nd.Graph.from_edges(ctx, raw.n, torch.from_numpy(raw.src).cuda(),
                            torch.from_numpy(raw.dst).cuda())
    g.prepare(kind)
    _, n_levels = g.levels(kind)
    kappa, _ = g.decompose(kind, "snd", use_frontier=True)
    kap = kappa.cpu().numpy()
    nr = kap.size
    idx = np.random.default_rng(seed).choice(nr, size=min(sample, nr),
                                             replace=False)
    out = {"workload": name, "kind": kind, "n_rcliques": int(nr),
           "kendall_sample": int(idx.size), "degree_levels": n_levels}
    for mode in ("snd", "and"):
        its, stats = [], []
        g.decompose(kind, mode, keep_iterates=its, keep_stats=stats,
                    count_active=True)
        tau0 = g.sdegree(kind).cpu().numpy()
        rows, t_cum = [], 0.0
        seq = [tau0] + [t.cpu().numpy() for _, t in its]
        for t, tau in enumerate(seq):
            st = stats[t - 1] if t > 0 else None
            if st:
                t_cum += st["ms"]
            exact = float(np.count_nonzero(tau == kap)) / max(nr, 1)
            kt = float(scipy.stats.kendalltau(tau[idx], kap[idx]).statistic)
            rows.append({"sweep": t, "changed": st["changed"] if st else None,
                         "active": st["active_next"] if st else None,
                         "ms_cum": t_cum, "fraction_exact": exact,
                         "kendall_tau": kt})
        res = {"rows": rows}
        for by in ("active", "changed"):
            stops = {}
            for ratio in (0.4, 0.1, 0.01):
                hit = next((r for r in rows[1:] if r[by] < ratio * nr), rows[-1])
                stops[str(ratio)] = {k: hit[k] for k in ("sweep", "ms_cum",
                                                         "fraction_exact",
                                                         "kendall_tau")}
            res[f"{by}_ratio_stops"] = stops
        out[mode] = res
    g.close()
    return out


def recorded_peeling(name: str):
    """Seconds the oracle's peeling took on a workload when its full-size
    digest was recorded, or None."""
    try:
        rec = json.load(open(os.path.join(ROOT, "tests", "golden",
                                          "full_size.json")))
        return float(rec[name]["oracle_seconds"])
    except (OSError, ValueError, KeyError):
        return None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=10.0)
    ap.add_argument("--calib-copy", action="store_true",
                    help="first copy 1 GiB device-to-device (a known-size "
                         "kernel for scaling hardware byte counters)")
    ap.add_argument("--no-ceilings", action="store_true")
    ap.add_argument("--stream-graphs", type=int, default=256,
                    help="graphs in the batched/served comparison (0: skip)")
    ap.add_argument("--stream-group", type=int, default=None,
                    help="graphs per batched call in the stream leg (default: "
                         "all up to 512, else 256)")
    ap.add_argument("--small-graphs", type=int, default=512,
                    help="graphs in the small-graph batched comparison "
                         "(0: skip)")
    ap.add_argument("--ego-queries", type=int, default=4096,
                    help="random edges for the ego-estimate leg (0: skip)")
    ap.add_argument("--no-workloads", action="store_true",
                    help="skip the k-truss (cl20) and k-core (cl23) legs")
    ap.add_argument("--only-headline", action="store_true",
                    help="run only the headline leg (for the profiles)")
    ap.add_argument("--only-stream", action="store_true",
                    help="run only the stream leg and print its JSON")
    ap.add_argument("--quality", default=None,
                    help="only run the per-sweep accuracy leg on this "
                         "workload (e.g. cl23) and print its JSON")
    ap.add_argument("--summarize-quality", default=None, metavar="JSON",
                    help="write profiles/quality_*.md from the output of "
                         "--quality and exit")
    ap.add_argument("--summarize-trace", nargs=2, default=None,
                    metavar=("STATS_CSV", "NAME"),
                    help="write profiles/kernel_trace_NAME.md from a "
                         "rocprofv3 kernel-stats CSV and exit")
    ap.add_argument("--summarize-profiles", nargs=3, default=None,
                    metavar=("TRACE_STATS_CSV", "FETCH_CSV", "WRITE_CSV"),
                    help="write the profiles/ summaries from rocprofv3 output "
                         "and exit (no GPU needed)")
    args = ap.parse_args()
    if args.summarize_profiles:
        summarize_profiles(*args.summarize_profiles)
        return
    if args.summarize_trace:
        summarize_trace(*args.summarize_trace)
        return
    if args.summarize_quality:
        summarize_quality(args.summarize_quality)
        return
    if args.gpus != 1:
        print("bench.py measures one GPU only: no part of this path runs on "
              "several GPUs here (the sharding is a design note)",
              file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_1704_00386_amd as nd

    if args.quality:
        print(json.dumps(quality_leg(nd, args.quality)), flush=True)
        return
    ctx = nd.Context(0)
    if args.only_stream:
        out = {}
        if args.stream_graphs > 0:
            out["stream"] = stream_leg(nd, ctx, args.stream_graphs,
                                       group=args.stream_group)
        if args.small_graphs > 0:
            out["small_graphs"] = stream_leg(nd, ctx, args.small_graphs, seed=7,
                                             n_lo=1000, n_hi=5000, serve=False)
        print(json.dumps(out), flush=True)
        return
    if args.calib_copy:
        a = torch.ones(1 << 28, dtype=torch.int32, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    h = headline_leg(nd, ctx, args)
    res, roof, raw = h["res"], h["roof"], h["raw"]
    ms_step = h["ms_step"]
    h["g"].close()
    traffic = measured_traffic()
    line = {
        "metric": "r-clique h-index updates/sec + time-to-exact-convergence "
                  "vs CPU peeling",
        "value": res["updates"] / (ms_step * 1e-3),
        "unit": "r-clique h-index updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": "(3,4)-nucleus SND on the stochastic block model: "
                               "5000 communities of U{50..400} vertices, p_in 0.3, "
                               "p_out 2e-6, seed 4; triangles as r-cliques",
                   "n": raw.n, "raw_pairs": raw.m, "triangles": res["n_rcliques"],
                   "incidence_P": res["n_incidence"],
                   "swept_per_sweep": h["nr_eval"],
                   "tau_bytes": res["tau_bytes"], "kind": HEADLINE_KIND,
                   "mode": "snd", "frontier": True},
        "updates_counted": "h-index evaluations the step performs (r-cliques "
                           "the frontier recomputes, summed over sweeps)",
        "time_to_exact_ms": ms_step,
        "time_to_exact_no_prep_ms": res["ms_iterate"],
        "ms_prep": ms_step - res["ms_iterate"],
        "ms_iterate": res["ms_iterate"],
        "step_ms_all": h["times"],
        "sweeps": res["sweeps"],
        "t_star": res["sweeps"] - 1,  # first t with tau_t = kappa
        "evaluated_updates": res["updates"],
        "evaluated_updates_per_s_of_sweep_time": res["updates"] / (res["ms_iterate"] * 1e-3),
        "full_sweep_equivalent_updates_per_s": h["nr_eval"] * res["sweeps"] / (ms_step * 1e-3),
        "roofline": {"bound": "hbm", "achieved": roof["achieved_GBs"],
                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": roof["achieved_GBs"] / HBM_PEAK_GBS,
                     "traffic": traffic,
                     "kernel": "full sweep: one application of U to every "
                               "r-clique with d_s > 0 (k_sweep_small<3, "
                               f"{TAU_CTYPE[res['tau_bytes']]}>)",
                     "bytes_per_launch": roof["bytes_per_sweep"],
                     "avg_launch_ms": roof["avg_sweep_ms"],
                     "sweeps_timed": roof["sweeps_timed"]},
        "and": h["and"],
    }
    if "ceilings" in h:
        c = h["ceilings"]
        c["update_kernel_frac_of_read"] = roof["achieved_GBs"] / c["read_GBs"]
        c["update_kernel_frac_of_gather"] = roof["achieved_GBs"] / c["gather_GBs"]
        line["ceilings"] = c
    del h
    line["paper_context"] = {
        "hardware": "2 x 12-core Intel Ivy Bridge at 2.4 GHz, 24 threads, "
                    "C++/OpenMP (Section 5)",
        "published_updates_per_s": None,
        "derived_and_updates_per_s": {
            "k_truss": [3.7e6, 1.5e7], "nucleus34": [1.1e6, 3.1e6]},
        "derived_from": "|R| x AND iterations (Table 3, sequential runs) / "
                        "AND time on 24 threads (Table 4) for the facebook and "
                        "web-Google graphs (Table 2); order of magnitude only",
    }
    if not args.only_headline:
        if not args.no_workloads:
            tr, g, kappa = workload_leg(nd, ctx, "cl20", "truss")
            line["truss_cl20"] = tr
            if args.ego_queries > 0:
                line["ego"] = ego_leg(nd, g, kappa, "truss", args.ego_queries)
            g.close()
            del kappa
            line["core_cl23"], g, _ = workload_leg(nd, ctx, "cl23", "core",
                                                   quality=True)
            g.close()
        if args.stream_graphs > 0:
            line["stream"] = stream_leg(nd, ctx, args.stream_graphs,
                                        group=args.stream_group)
        if args.small_graphs > 0:
            line["small_graphs"] = stream_leg(nd, ctx, args.small_graphs, seed=7,
                                              n_lo=1000, n_hi=5000, serve=False)
    if not args.no_cpu:
        progress("cpu baseline (oracle) starts")
        cb = cpu_baseline(args.cpu_budget)
        # the step's h-index evaluations at the oracle's update rate
        cb["time_to_exact_s_est"] = res["updates"] / cb["value"]
        cb["time_to_exact_s_est_is"] = ("the step's evaluated updates divided "
                                        "by the oracle's rate")
        pe = cb["peeling"]
        pe["full_workload_s_est"] = res["n_incidence"] / pe["incidence_per_s"]
        pe["full_workload_s_est_is"] = ("the workload's incidence pairs divided by "
                                        "the sample's peeling rate (peeling is "
                                        "linear in them)")
        pe["step_speedup_est"] = pe["full_workload_s_est"] / (ms_step * 1e-3)
        line["cpu_baseline"] = cb
    peel = recorded_peeling(HEADLINE)
    if peel is not None:
        line["cpu_peeling_recorded"] = {
            "s": peel, "step_speedup": peel / (ms_step * 1e-3),
            "what": "the oracle's Alg. Peeling on this workload, split exactly "
                    "by community over a pool of 8 processes (parallel S-degree "
                    "count, sequential peeling per community), timed when the "
                    "full-size kappa digests in tests/golden/full_size.json were "
                    "written, on that machine's cores (not this run's host): "
                    "context, not the baseline"}
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()

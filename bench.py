"""Benchmark: Lloyd iterations of inverted-file spherical k-means on one MI355X.

One step = one whole Lloyd iteration (assignment walk + certification + FP64
re-scores + objective, then the update: exact member sums, FP64 norms and the
inverted-file rebuild) over the full synthetic object set, which is resident
in HBM before the timed region starts.

Default workload: 8,000,000 synthetic Zipf tf-idf documents over 140,000 terms
(Poisson(60) nonzeros clipped to [3, 1000], Zipf s = 1.1), k = 10,000, FP32
inverted-file values.  Prints ONE JSON line on stdout; progress goes to stderr.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Lloyd iter/s and sparse mult-adds/s at 8M docs×140k terms, k=10k; HBM GB/s"
HBM_PEAK_GBPS = 8000.0
COPY_BYTES = 1 << 30
ENTRY_BYTES = {"f32": 8, "bf16": 4, "f16": 4}   # (cluster id, value) per posting entry


def log(msg):
    print("[bench %7.1fs] %s" % (time.perf_counter() - T0, msg), file=sys.stderr, flush=True)


T0 = time.perf_counter()


def walk_bytes(m, nnz, n, ranges, valtype):
    """Algorithmic bytes of one walk launch: every posting entry walked (cluster
    id + value: 8 B for FP32 values, 4 B for 16-bit local ids and values);
    per cluster range, each object nonzero (term id + value, 8 B) with its
    slice descriptor (two int32, 8 B), the object row pointers (8 B) and the
    object's range record written (16 B)."""
    return ENTRY_BYTES[valtype] * m + ranges * (16 * nnz + 8 * (n + 1) + 16 * n)


def iteration_bytes(m, nnz, n, ranges, nnz_means, valtype):
    """Algorithmic bytes of one Lloyd iteration: the walk, the assignment
    read/write, and the update (the object entries grouped by cluster: key,
    position, term, value; FP64 mean entries written; inverted file written)."""
    return (walk_bytes(m, nnz, n, ranges, valtype) + 8 * n + 16 * nnz
            + nnz_means * (12 + 12 + ENTRY_BYTES[valtype]))


def kernel_hash(sources=("assign.hip", "invfile.hip", "plan.hip")):
    """Hash of a kernel's sources and the shared headers: by default the
    walk's kernels, the inverted-file layout they read (slabs, postings) and
    the planner that picks their plan."""
    h = hashlib.sha256()
    for f in (*sources, "kernels.h", "ivf_internal.h"):
        with open(os.path.join(ROOT, "paper_2002_09094_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


# Working sets of the read-ceiling probes: (bytes, mode, passes).  mode 0:
# every workgroup reads the whole buffer (resident in each XCD's L2); mode 1:
# the buffer split among the workgroups and swept `passes` times (128 MiB:
# beyond the L2s, inside the 256 MB Infinity Cache; 4 GiB: HBM).
CEILINGS = {"l2": (2 << 20, 0, 40), "infinity_cache": (128 << 20, 1, 100),
            "hbm": (4 << 30, 1, 3)}
# Launch shapes each level is timed with, (loads in flight per lane,
# workgroups per CU); a level's ceiling is the best of them.  The first shape
# is also the one whose counters calibrate bytes per request.
PROBE_SHAPES = [(4, 8), (8, 8), (16, 8), (4, 16), (8, 16), (16, 16)]


def probe_bytes(level, cus, wgs_per_cu=PROBE_SHAPES[0][1]):
    """Bytes one timed probe launch reads at `level`."""
    nbytes, mode, passes = CEILINGS[level]
    n16 = nbytes // 16
    if mode == 0:
        return cus * wgs_per_cu * n16 * 16 * passes
    return n16 * 16 * passes


def read_ceilings():
    """Measured read bandwidth (GB/s) of working sets resident in L2, in the
    Infinity Cache and in HBM: the roofs the walk's counted traffic is placed
    against.  Each level is read by the library's streaming probe in every
    shape of PROBE_SHAPES (one warm-up and one timed launch each) and takes
    the best.  Returns (ceilings, per-shape rates)."""
    import torch

    import paper_2002_09094_amd as ivf

    out, shapes = {}, {}
    for level, (nbytes, mode, passes) in CEILINGS.items():
        buf = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda:0")
        torch.cuda.synchronize()
        rates = [ivf.read_ceiling(buf, mode, passes, unroll=u, wgs_per_cu=w)
                 for u, w in PROBE_SHAPES]
        shapes[level] = {"%dx%d" % sh: r for sh, r in zip(PROBE_SHAPES, rates)}
        out[level] = max(rates)
        del buf
    torch.cuda.empty_cache()
    log("read ceilings (GB/s, best of %d shapes): " % len(PROBE_SHAPES)
        + ", ".join("%s %.0f" % kv for kv in out.items()))
    log("per shape (loads in flight x workgroups per CU): %s" % json.dumps(
        {k: {s: round(r) for s, r in v.items()} for k, v in shapes.items()}))
    return out, shapes


def level_counters(kernel, workload, valtype):
    """Per-launch bytes of the walk at each level of the memory hierarchy,
    from the committed rocprofv3 counter summary, if it was taken on the
    current kernel source (else None)."""
    path = os.path.join(ROOT, "profiles", "%s_%s_%s_levels.json"
                        % (kernel[2:] if kernel.startswith("k_") else kernel, workload, valtype))
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    if t.get("kernel_hash") != kernel_hash(KERNEL_SOURCE[kernel]):
        return None
    return t


def traffic_counters(kernel, workload, valtype):
    """Calibrated FETCH_SIZE / WRITE_SIZE bytes per launch of `kernel`, from the
    committed counter summary, if it was taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", "%s_%s_%s_traffic.json"
                        % (kernel[2:] if kernel.startswith("k_") else kernel, workload, valtype))
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    if t.get("kernel_hash") != kernel_hash(KERNEL_SOURCE[kernel]):
        return None
    return t


def walk_roofline(kernel, workload, valtype, walk_s, alg_bytes, ceilings, copy_gbps, add_gbps,
                  probe_shapes=None):
    """The walk against the roof it hits.  The method's algorithmic bytes
    charge every posting read to memory (the paper's per-access model), but
    the caches serve most of them, so those bytes per second are reported as
    an effective rate only.  The roof is set from counters: the bytes the
    walk moved from L2 into the compute units (L1 -> L2 read requests) and
    from the memory side into L2 (L2 -> fabric read requests, Infinity-Cache
    hits included), each against the read ceiling measured in this run for a
    working set resident at that level; the bound is the level with the
    larger fraction.  The fabric bytes against the published 8 TB/s are an
    upper bound of the walk's HBM share."""
    out = {"kernel": kernel, "unit": "GB/s",
           "algorithmic_bytes_per_launch": alg_bytes,
           "effective_gbps_algorithmic": alg_bytes / walk_s / 1e9,
           "ceilings_gbps": ceilings, "ceilings_by_probe_shape": probe_shapes,
           "hbm_peak_published_gbps": HBM_PEAK_GBPS,
           "stream_copy_gbps": copy_gbps, "stream_add_gbps": add_gbps}
    lv = level_counters(kernel, workload, valtype)
    if lv is None:
        out.update({"bound": None, "achieved": None, "peak": None, "frac": None,
                    "traffic": None,
                    "note": "no counter summary taken on the current kernel source"})
        return out
    levels = {
        "l2": (lv["l2_read_bytes"] / walk_s / 1e9, ceilings["l2"]),
        "infinity_cache": (lv["fabric_read_bytes"] / walk_s / 1e9, ceilings["infinity_cache"]),
    }
    tr = traffic_counters(kernel, workload, valtype)
    write_bytes = tr["write_bytes"] if tr else 0.0
    fr = {k: a / p for k, (a, p) in levels.items()}
    bound = max(fr, key=fr.get)
    a, p = levels[bound]
    out.update({
        "bound": bound, "achieved": a, "peak": p, "frac": a / p,
        "peak_kind": "measured read ceiling of a working set resident at that level",
        "traffic": lv["fabric_read_bytes"] + write_bytes,
        "traffic_unit": ("bytes per launch between L2 and the memory side: reads (counted "
                         "requests) + writes (calibrated WRITE_SIZE)" if write_bytes else
                         "bytes per launch read by L2 from the memory side"),
        "levels": {k: {"achieved": a_, "peak": p_, "frac": a_ / p_}
                   for k, (a_, p_) in levels.items()},
        "hbm_upper_bound": {"achieved": lv["fabric_read_bytes"] / walk_s / 1e9,
                            "peak": HBM_PEAK_GBPS,
                            "frac": lv["fabric_read_bytes"] / walk_s / 1e9 / HBM_PEAK_GBPS},
        "l2_hit_rate": lv.get("l2_hit_rate"),
        "mfma_instructions": lv.get("mfma_instructions"),
        "counters_source": lv.get("source")})
    return out


def cpu_baseline(x, w, valtype, check, target_s):
    """The FP64 oracle on this host's cores, on a bounded sample of the state
    the GPU assigned outside the timed region (the chain's means after the
    timed iterations and its previous assignment): the oracle's assignment
    walk over a seeded sample of S objects, S grown until the walk takes
    about target_s / 2, scaled to the whole set by the exact mult-add count;
    plus its update step over the whole set.  The same oracle results check
    the GPU on the sample: identical assignments, and the largest relative
    error of the FP32 tile scores (top-1: the tile's winner against that
    cluster's FP64 score; top-2: the tile's best other score against the
    oracle's, where the two winners agree)."""
    import numpy as np

    import datagen
    import oracle
    import paper_2002_09094_amd as ivf

    cores = len(os.sched_getaffinity(0))
    threads = int(os.environ.get("OMP_NUM_THREADS", cores))
    ptr, idx, val = check["means"]
    means = oracle.Means(w.k, w.d, ptr, idx, val)
    prev, got = check["prev"], check["assign"]
    m_full = int(check["stats"]["mult_adds"])
    s = min(x.n, 20_000)
    while True:
        samp = np.sort(datagen.perm_prefix(x.n, s, w.seed, stream=23))
        xs = x.subset(samp)
        t = time.perf_counter()
        r = oracle.assign(xs, means, prev[samp], threads=threads)
        dt = time.perf_counter() - t
        log("cpu baseline: oracle walk of %d objects, %.3e mult-adds in %.2fs" % (s, r.mult_adds, dt))
        if dt >= 0.5 * target_s or s >= x.n:
            break
        s = int(min(x.n, max(2 * s, s * 0.5 * target_s / max(dt, 1e-3))))
    rate = r.mult_adds / dt
    t = time.perf_counter()
    oracle.update(x, w.k, got, means, threads=threads)
    t_update = time.perf_counter() - t
    log("cpu baseline: oracle update of all %d objects in %.2fs" % (x.n, t_update))
    t_iter = m_full / rate + t_update
    base = {
        "value": 1.0 / t_iter,
        "unit": "iter/s",
        "cores": threads,
        "kind": "oracle",
        "sample": ("FP64 oracle on the GPU chain's state after the timed iterations: its "
                   "assignment walk over a seeded sample of %d of %d objects (%.1fs, scaled to "
                   "the whole set by the exact mult-add count %d) plus its update of all "
                   "objects (%.1fs)" % (s, x.n, dt, m_full, t_update)),
        "assign_mult_adds_per_s": rate,
        "update_s": t_update,
        "cpu_model": cpu_model(),
        "nproc": os.cpu_count(),
    }
    base.update(single_core_small())
    # the GPU on the same sample
    gs = got[samp]
    best, bid, sec = (check[k][samp] for k in ("best", "best_id", "second"))
    same = (bid == r.assign) & (r.rho > 0)
    e1 = np.abs(best[same].astype(np.float64) - r.rho[same]) / r.rho[same]
    other = np.nonzero((bid >= 0) & ~same)[0]
    if len(other):   # FP32 winners the FP64 re-score overturned: their own FP64 scores
        r64 = oracle.scores(x, means, samp[other], bid[other])
        e1 = np.concatenate([e1, np.abs(best[other].astype(np.float64) - r64) / r64])
    two = same & (r.rho2 > 0)
    e2 = np.abs(sec[two].astype(np.float64) - r.rho2[two]) / r.rho2[two]
    nmax = int(np.max(np.diff(x.indptr)))
    c, a, g = ivf.cert_bound(valtype, nmax, float(x.values.max()))
    st = check["stats"]
    prec = {"sample_objects": int(s), "identical": int(np.sum(gs == r.assign)),
            "max_rel_err_top1": float(e1.max()) if len(e1) else 0.0,
            "max_rel_err_top2": float(e2.max()) if len(e2) else 0.0,
            "top1_pairs": int(len(e1)), "top2_pairs": int(two.sum()),
            "bound_c_longest_row": c,
            "certified_fraction": st["certified"] / x.n, "rescored": st["rescored"],
            "sample_rescored": int(np.sum(check["flags"][samp] & 2)),
            "max_rel_err_rescored": st["max_rel_err_rescored"]}
    log("precision check: %d of %d sampled objects identical to the oracle; max rel err "
        "top-1 %.3g, top-2 %.3g" % (prec["identical"], s, prec["max_rel_err_top1"],
                                    prec["max_rel_err_top2"]))
    return base, prec


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def single_core_small():
    """The oracle on one core over the small workload (20,000 documents,
    k = 100): the second Lloyd iteration's assignment + update, beside the
    paper's single-thread figures."""
    import numpy as np

    import datagen
    import oracle

    w = datagen.WORKLOADS["small"]
    x = w.generate()
    seeds = w.seeds(x)
    means = oracle.initial_means(x, seeds)
    prev = np.full(x.n, -1, np.int32)
    times = []
    for _ in range(2):
        t = time.perf_counter()
        r = oracle.assign(x, means, prev, threads=1)
        means, _ = oracle.update(x, w.k, r.assign, means, threads=1)
        times.append(time.perf_counter() - t)
        prev = r.assign
    log("cpu baseline: small workload on one core, %.3f s per iteration" % times[-1])
    return {"single_core_small_s_per_iter": times[-1], "single_core_small_mult_adds": r.mult_adds}


def stream_gbps(nbytes=2 << 30, reps=5):
    """Streaming bandwidth of this GPU, bytes read + written per second over
    2 GiB arrays: a copy (c = a) and STREAM's add (c = a + b), the practical
    HBM ceilings next to the nominal 8 TB/s."""
    import torch

    a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda:0").fill_(1.0)
    b = torch.empty_like(a).fill_(2.0)
    c = torch.empty_like(a)

    def timed(f):
        for _ in range(2):
            f()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            f()
        e1.record()
        e1.synchronize()
        return e0.elapsed_time(e1) / 1e3

    copy = 2.0 * nbytes * reps / timed(lambda: c.copy_(a)) / 1e9
    add = 3.0 * nbytes * reps / timed(lambda: torch.add(a, b, out=c)) / 1e9
    del a, b, c
    torch.cuda.empty_cache()
    log("stream: copy %.1f GB/s, add %.1f GB/s (read + write)" % (copy, add))
    return copy, add


def _csv_rows(path):
    import csv
    with open(path, newline="") as f:
        return list(csv.DictReader(f))


def summarize_trace(stats_csv, out_txt, command, note=""):
    """Text summary of a rocprofv3 --kernel-trace --stats run."""
    rows = _csv_rows(stats_csv)
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    lines = ["# rocprofv3 kernel statistics", "# command: " + command]
    if note:
        lines.append("# " + note)
    lines += ["",
             "%-40s %6s %14s %14s %7s" % ("kernel", "calls", "total_ms", "avg_ms", "pct")]
    for r in rows[:25]:
        name = r["Name"].replace("ivf::(anonymous namespace)::", "").split("(")[0]
        lines.append("%-40s %6s %14.3f %14.3f %7.2f" % (
            name[:40], r["Calls"], float(r["TotalDurationNs"]) / 1e6,
            float(r["AverageNs"]) / 1e6, float(r["Percentage"])))
    trace_csv = stats_csv.replace("kernel_stats", "kernel_trace")
    if os.path.exists(trace_csv):
        top = rows[0]["Name"]
        launches = [r for r in _csv_rows(trace_csv) if r["Kernel_Name"] == top]
        if not launches:   # a trace of another run
            raise ValueError("%s holds no launch of %s" % (trace_csv, top))
        ms = [(int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e6 for r in launches]
        short = top.replace("ivf::(anonymous namespace)::", "").split("(")[0]
        lines += ["", "%s launches in order (ms): %s" % (short, ", ".join("%.3f" % v for v in ms))]
        if len(ms) > 1 and "::k_walk<" in top:
            lines.append("%s average over the launches after the first (the first iteration "
                         "starts from the seed means): %.3f ms" % (short, sum(ms[1:]) / (len(ms) - 1)))
        elif ms:
            lines.append("%s average over all launches: %.3f ms" % (short, sum(ms) / len(ms)))
        r0 = launches[0]
        lines.append("%s resources: VGPR %s, AGPR %s, SGPR %s, LDS %s bytes, workgroup %s, grid %s"
                     % (short, r0["VGPR_Count"], r0["Accum_VGPR_Count"], r0["SGPR_Count"],
                        r0["LDS_Block_Size"], r0["Workgroup_Size_X"], r0["Grid_Size_X"]))
    with open(out_txt, "w") as f:
        f.write("\n".join(lines) + "\n")


def summarize_update_trace(trace_csv, out_txt, command, top=12):
    """Per-iteration kernel times of the update from a rocprofv3 kernel trace
    (columns Kernel_Name, Start_Timestamp, End_Timestamp): the launches
    between one walk launch and the next are that iteration's merge, update
    and rebuild; the merge of the ranges and the objective belong to the
    assignment step and are left out of the update's busy time."""
    import re
    rows = _csv_rows(trace_csv)
    rows.sort(key=lambda r: int(r["Start_Timestamp"]))
    assign_side = ("k_merge", "k_rescore", "k_objective", "k_sum_final")
    iters, cur = [], None
    for r in rows:
        name = r["Kernel_Name"]
        if "copyBuffer" in name or "k_read" in name:
            continue
        if re.search(r"::k_walk", name):
            if cur is not None:
                iters.append(cur)
            cur = []
            continue
        if cur is not None:
            cur.append(r)
    if cur:
        iters.append(cur)
    lines = ["# rocprofv3 kernel trace: update kernels per Lloyd iteration",
             "# command: " + command,
             "# iteration i: the launches after walk launch i (the first walk starts from "
             "the seed means); busy = summed kernel time of the update and rebuild", ""]
    for i, it in enumerate(iters):
        agg = {}
        for r in it:
            m = re.search(r"(k_[a-z0-9_]+)", r["Kernel_Name"])
            key = m.group(1) if m else r["Kernel_Name"][:30]
            a = agg.setdefault(key, [0, 0.0])
            a[0] += 1
            a[1] += (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e6
        busy = sum(v[1] for k, v in agg.items() if k not in assign_side)
        if busy == 0.0:
            continue
        lines.append("iteration %d: update busy %.2f ms" % (i + 1, busy))
        for k, v in sorted(agg.items(), key=lambda x: -x[1][1])[:int(top)]:
            if k in assign_side:
                continue
            lines.append("    %-24s x%-3d %8.3f ms" % (k, v[0], v[1]))
    with open(out_txt, "w") as f:
        f.write("\n".join(lines) + "\n")


# the walk's counters also depend on the plan (range width, slab threshold),
# which the planner in plan.hip chooses
KERNEL_SOURCE = {"k_walk": ("assign.hip", "invfile.hip", "plan.hip"),
                 "k_walk_batch": ("assign.hip", "invfile.hip", "plan.hip"),
                 "k_ivfd_walk": ("ivfd.hip",)}


def _last_dispatch_values(rows, match):
    """Counter values of the last dispatch whose kernel name contains `match`."""
    sel = [r for r in rows if match(r["Kernel_Name"])]
    if not sel:
        return {}
    last = max(int(r["Dispatch_Id"]) for r in sel)
    return {r["Counter_Name"]: float(r["Counter_Value"]) for r in sel
            if int(r["Dispatch_Id"]) == last}


def summarize_levels(workload, valtype, out_json, out_txt, command, kernel, cus, *csvs):
    """Bytes the walk moved at each level of the memory hierarchy, from
    rocprofv3 --pmc passes over a run that first times the read probes (three
    levels, a warm-up and a timed launch per shape of PROBE_SHAPES, in the
    order of CEILINGS) and
    then the walk: L1 -> L2 read requests (TCP_TCC_READ_REQ_sum) and L2 ->
    fabric read requests (TCC_EA0_RDREQ_sum) of the last walk launch, each
    scaled to bytes by what the same counter reads for the timed probe of
    known size (the L2-resident probe and the HBM-resident one)."""
    import collections
    rows = []
    for path in csvs:
        rows += _csv_rows(path)
    probes = collections.OrderedDict()
    for r in rows:
        if "k_read" in r["Kernel_Name"]:
            probes.setdefault(int(r["Dispatch_Id"]), {})[r["Counter_Name"]] = float(r["Counter_Value"])
    # per counter: the probe dispatches that carry it, in order (each pass has its own ids)
    by_counter = collections.defaultdict(list)
    for did in sorted(probes):
        for name, v in probes[did].items():
            by_counter[name].append(v)
    levels = list(CEILINGS)

    def timed_probe(counter, level):
        # per level: (warm-up, timed) per shape; the first shape's timed launch
        vals = by_counter[counter]
        return vals[2 * len(PROBE_SHAPES) * levels.index(level) + 1]

    walk = {}
    for path in csvs:
        walk.update(_last_dispatch_values(_csv_rows(path),
                                          lambda n: ("::%s<" % kernel) in n))
    l2_bpr = probe_bytes("l2", cus) / timed_probe("TCP_TCC_READ_REQ_sum", "l2")
    fab_bpr = probe_bytes("hbm", cus) / timed_probe("TCC_EA0_RDREQ_sum", "hbm")
    out = {"kernel": kernel, "workload": workload, "valtype": valtype,
           "kernel_hash": kernel_hash(KERNEL_SOURCE[kernel]),
           "l2_bytes_per_request": l2_bpr, "fabric_bytes_per_request": fab_bpr,
           "l2_read_bytes": walk["TCP_TCC_READ_REQ_sum"] * l2_bpr,
           "fabric_read_bytes": walk["TCC_EA0_RDREQ_sum"] * fab_bpr,
           "counters": walk, "probe_counters": {k: v for k, v in by_counter.items()},
           "source": os.path.basename(out_txt), "command": command}
    if "TCC_HIT_sum" in walk and "TCC_MISS_sum" in walk:
        h, m = walk["TCC_HIT_sum"], walk["TCC_MISS_sum"]
        out["l2_hit_rate"] = h / (h + m)
    mf = [v for k, v in walk.items() if "MFMA" in k]
    out["mfma_instructions"] = sum(mf) if mf else None
    with open(out_json, "w") as f:
        json.dump(out, f, indent=1)
    lines = ["# rocprofv3 counters of the steady-state %s launch and of the read probes" % kernel,
             "# command: " + command, "",
             "walk counters (last dispatch):"]
    lines += ["  %-34s %.4e" % kv for kv in walk.items()]
    lines += ["", "probe counters (warm-up, timed) x (%s):" % ", ".join(levels)]
    lines += ["  %-34s %s" % (k, ", ".join("%.4e" % x for x in v)) for k, v in by_counter.items()]
    lines += ["",
              "bytes per L1->L2 read request (L2 probe: %.4e B read): %.1f"
              % (probe_bytes("l2", cus), l2_bpr),
              "bytes per L2->fabric read request (HBM probe: %.4e B read): %.1f"
              % (probe_bytes("hbm", cus), fab_bpr),
              "walk: L2 -> CU read bytes per launch %.4e" % out["l2_read_bytes"],
              "walk: memory side -> L2 read bytes per launch %.4e" % out["fabric_read_bytes"]]
    if "l2_hit_rate" in out:
        lines.append("walk: L2 hit rate (requests) %.3f" % out["l2_hit_rate"])
    if out["mfma_instructions"] is not None:
        lines.append("walk: MFMA instructions %d" % out["mfma_instructions"])
    with open(out_txt, "w") as f:
        f.write("\n".join(lines) + "\n")
    return out


def summarize_counters(fetch_csv, write_csv, workload, valtype, out_json, command,
                       kernel="k_walk"):
    """Memory-side traffic of the last launch of `kernel` from FETCH_SIZE and
    WRITE_SIZE runs (KiB per dispatch), each scaled so that the calibration
    copy of COPY_BYTES reads and writes exactly COPY_BYTES.  fetch_csv "-":
    writes only."""
    def pick(path, counter):
        rows = [r for r in _csv_rows(path) if r["Counter_Name"] == counter]
        copies = [float(r["Counter_Value"]) for r in rows
                  if "copyBuffer" in r["Kernel_Name"] and float(r["Counter_Value"]) > 1e5][:3]
        walks = [r for r in rows if "::%s<" % kernel in r["Kernel_Name"]]
        return copies, walks
    wc, ww = pick(write_csv, "WRITE_SIZE")
    w_scale = COPY_BYTES / (1024.0 * sum(wc) / len(wc))
    write = float(ww[-1]["Counter_Value"]) * 1024.0 * w_scale
    if fetch_csv == "-":   # the read side taken from request counters instead
        fc, f_scale, fetch, fraw = None, None, None, None
    else:
        fc, fw = pick(fetch_csv, "FETCH_SIZE")
        f_scale = COPY_BYTES / (1024.0 * sum(fc) / len(fc))
        fraw = float(fw[-1]["Counter_Value"])
        fetch = fraw * 1024.0 * f_scale
    out = {"kernel": kernel, "workload": workload, "valtype": valtype,
           "kernel_hash": kernel_hash(KERNEL_SOURCE[kernel]), "fetch_bytes": fetch,
           "write_bytes": write,
           "hbm_bytes_per_launch": (fetch + write) if fetch is not None else None,
           "fetch_scale": f_scale,
           "write_scale": w_scale, "copy_fetch_kib": fc, "copy_write_kib": wc,
           "walk_fetch_kib_raw": fraw,
           "walk_write_kib_raw": float(ww[-1]["Counter_Value"]), "command": command}
    with open(out_json, "w") as f:
        json.dump(out, f, indent=1)
    return out


def summarize_pmc(out_txt, command, *csvs):
    """Text summary of rocprofv3 --pmc passes over the walk: the counters of
    its last dispatch in each pass and the ratios read from them."""
    import collections
    vals = collections.OrderedDict()
    for path in csvs:
        rows = [r for r in _csv_rows(path) if "k_walk" in r["Kernel_Name"]]
        last = max(int(r["Dispatch_Id"]) for r in rows)
        for r in rows:
            if int(r["Dispatch_Id"]) == last:
                vals[r["Counter_Name"]] = float(r["Counter_Value"])
    lines = ["# rocprofv3 counters of the steady-state walk launch (last k_walk dispatch of each pass)",
             "# commands: " + command, ""]
    for k, v in vals.items():
        lines.append("%-34s %.4e" % (k, v))
    g = vals.get
    lines.append("")
    if g("TCC_HIT_sum") is not None and g("TCC_MISS_sum") is not None:
        h, m = g("TCC_HIT_sum"), g("TCC_MISS_sum")
        lines.append("L2 hit rate (requests): %.3f" % (h / (h + m)))
    if g("SQ_WAIT_ANY") and g("SQ_WAVE_CYCLES"):
        lines.append("wave cycles waiting (SQ_WAIT_ANY / SQ_WAVE_CYCLES): %.3f"
                     % (g("SQ_WAIT_ANY") / g("SQ_WAVE_CYCLES")))
    if g("SQ_WAIT_INST_LDS") and g("SQ_WAVE_CYCLES"):
        lines.append("wave cycles waiting on LDS: %.3f" % (g("SQ_WAIT_INST_LDS") / g("SQ_WAVE_CYCLES")))
    if g("SQ_LDS_BANK_CONFLICT") and g("SQ_LDS_IDX_ACTIVE"):
        lines.append("LDS bank-conflict cycles / LDS active cycles: %.3f"
                     % (g("SQ_LDS_BANK_CONFLICT") / g("SQ_LDS_IDX_ACTIVE")))
    if g("TCP_TCC_READ_REQ_LATENCY_sum") and g("TCP_TCC_READ_REQ_sum"):
        lines.append("average L2 read latency seen by L1 (cycles): %.0f"
                     % (g("TCP_TCC_READ_REQ_LATENCY_sum") / g("TCP_TCC_READ_REQ_sum")))
    if g("TCP_TCC_READ_REQ_sum") and g("TCP_TOTAL_CACHE_ACCESSES_sum"):
        lines.append("L1 accesses that go to L2: %.3f"
                     % (g("TCP_TCC_READ_REQ_sum") / g("TCP_TOTAL_CACHE_ACCESSES_sum")))
    with open(out_txt, "w") as f:
        f.write("\n".join(lines) + "\n")


def run_figures(args):
    """Per-iteration quantities behind the paper's figures on means and
    multiplications, measured on synthetic data: for several k on 1,000,000
    documents shaped like the paper's 1M-document PubMed sample (140,000
    terms, Poisson(60) nonzeros in [3, 1000], Zipf s = 1.1), every Lloyd
    iteration's distinct terms in the means, their nonzeros sum_j (ntm)_j (the
    inverted file's size), the mult-adds M of the assignment (Eq. ivf_mult),
    the changes and the walk time, from the seeded initial state until an
    assignment changes nothing (at most --steps + 10 iterations)."""
    import numpy as np
    import torch

    import datagen
    import paper_2002_09094_amd as ivf

    dev = "cuda:0"
    n, d, seed = 1_000_000, 140_000, 9
    x = datagen.generate(n, d, 60.0, 3, 1000, 1.1, seed)
    xd = (torch.from_numpy(x.indptr).to(dev), torch.from_numpy(x.indices).to(dev),
          torch.from_numpy(x.values).to(dev))
    log("generated pubmed_1m: n=%d d=%d nnz=%d" % (n, d, x.nnz))
    out = {"metric": "per-iteration means and mult-adds vs k (synthetic)",
           "workload": "pubmed_1m", "n": n, "d": d, "lambda": 60.0, "zipf_s": 1.1, "seed": seed,
           "nnz": x.nnz, "valtype": args.valtype, "runs": []}
    for k in (1000, 2000, 5000, 10000, 20000):
        km = ivf.IVFKMeans(*xd, d, k, valtype=args.valtype)
        km.init_seeds(torch.from_numpy(datagen.seed_objects(x, k, seed).astype(np.int32)).to(dev))
        a = torch.full((n,), -1, dtype=torch.int32, device=dev)
        run = {"k": k, "iters": []}
        for r in range(args.steps + 10):
            sa = km.assign(a)
            su = km.update(a)
            idx = km.get_means()[1]
            distinct = int(torch.unique(idx).numel())
            run["iters"].append({"iter": r + 1, "changed": sa["changed"], "mult_adds": sa["mult_adds"],
                                 "walk_ms": sa["walk_ms"], "nnz_means": su["nnz_means"],
                                 "distinct_terms": distinct, "objective": su["objective_exact"]})
            log("k=%d iter %d: changed %d, M %.3e, nnz(means) %d, distinct terms %d, walk %.1f ms"
                % (k, r + 1, sa["changed"], sa["mult_adds"], su["nnz_means"], distinct,
                   sa["walk_ms"]))
            if sa["changed"] == 0:
                break
        km.close()
        out["runs"].append(run)
    print(json.dumps(out), flush=True)


def calibration_copies():
    """Three plain device copies of COPY_BYTES: the reference dispatches the
    counter summaries scale FETCH_SIZE and WRITE_SIZE by."""
    import torch

    src = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst
    log("copy calibration: 3 x %d bytes" % COPY_BYTES)


def _ivfd_compare(km, a, iters, n_r, tag):
    """`iters` Lloyd iterations; each assignment runs twice from the same
    means and previous partition: the means-inverted walk, then IVFD.  The
    two partitions and multiplication counts must agree."""
    import torch

    rows = []
    for r in range(iters):
        prev = a.clone()
        sa = km.assign(a)
        b = prev.clone()
        sd = km.assign_ivfd(b, objects_per_range=n_r)
        same = bool(torch.equal(a, b))
        if not same or sa["mult_adds"] != sd["mult_adds"]:
            raise SystemExit("%s iteration %d: IVFD and IVF disagree" % (tag, r + 1))
        km.update(a)
        rows.append({"iter": r + 1, "mult_adds": sa["mult_adds"], "changed": sa["changed"],
                     "ivf_walk_ms": sa["walk_ms"], "ivfd_walk_ms": sd["walk_ms"],
                     "ivf_assign_ms": sa["assign_ms"], "ivfd_assign_ms": sd["assign_ms"],
                     "ivfd_rescored": sd["rescored"], "ivf_rescored": sa["rescored"]})
        log("%s iter %d: M %.3e, IVF walk %.1f ms, IVFD walk %.1f ms (x%.2f), same partition"
            % (tag, r + 1, sa["mult_adds"], sa["walk_ms"], sd["walk_ms"],
               sd["walk_ms"] / max(sa["walk_ms"], 1e-9)))
    return rows


def run_ivfd(args):
    """Which side to invert (the paper's IVFD against IVF): the assignment
    step with the objects inverted (each mean a query over them) against the
    means inverted, on the same means, partition checked equal every
    iteration.  First on the 8M-document workload at k = 10,000, then on the
    1M-document PubMed-shaped set for k = 1,000 .. 20,000 (the paper's k
    sweep).  Iterations after the first (which starts from seed means)."""
    import numpy as np
    import torch

    import datagen
    import paper_2002_09094_amd as ivf

    dev = "cuda:0"
    if args.calibrate_copy:
        calibration_copies()
    n_r = args.ivfd_range
    out = {"metric": "IVFD vs IVF assignment walk time (same means, same partition)",
           "objects_per_range": n_r, "runs": []}
    sets = [("pubmed_8m", datagen.WORKLOADS["pubmed_8m"], [10000])]
    if not args.ivfd_8m_only:
        sets.append(("pubmed_1m", datagen.Workload("pubmed_1m", 1_000_000, 140_000, 60.0, 3, 1000,
                                                   1.1, 0, 0, 9),
                     [1000, 2000, 5000, 10000, 20000]))
    for name, w, ks in sets:
        x = w.generate()
        xd = (torch.from_numpy(x.indptr).to(dev), torch.from_numpy(x.indices).to(dev),
              torch.from_numpy(x.values).to(dev))
        log("generated %s: n=%d d=%d nnz=%d" % (name, x.n, x.d, x.nnz))
        for k in ks:
            km = ivf.IVFKMeans(*xd, x.d, k)
            km.init_seeds(torch.from_numpy(datagen.seed_objects(x, k, w.seed).astype(np.int32))
                          .to(dev))
            a = torch.full((x.n,), -1, dtype=torch.int32, device=dev)
            km.assign(a)          # first iteration from the seed means: not timed
            km.update(a)
            rows = _ivfd_compare(km, a, args.steps, n_r, "%s k=%d" % (name, k))
            ivf_ms = float(np.mean([r["ivf_walk_ms"] for r in rows]))
            ivfd_ms = float(np.mean([r["ivfd_walk_ms"] for r in rows]))
            out["runs"].append({"workload": name, "n": x.n, "d": x.d, "nnz": x.nnz, "k": k,
                                "ivf_walk_ms": ivf_ms, "ivfd_walk_ms": ivfd_ms,
                                "ratio": ivfd_ms / ivf_ms, "iters": rows})
            km.close()
        del xd
        torch.cuda.empty_cache()
    print(json.dumps(out), flush=True)


BATCH_METRIC = "aggregate sparse mult-adds/s, 96 batched instances (uneven N, D, k; restarts)"


def run_batched(args):
    """The many-instance workload: 96 instances (48 object sets once, 6 sets
    with 8 restarts each), N, D, lambda, s and k drawn per set; one batched
    walk launch per Lloyd iteration, the iteration replayed from HIP graphs.
    One step = one iteration of all 96 instances.  The warmup covers the two
    eager iterations, the tile autotuner and the recording of the graphs."""
    import numpy as np
    import torch

    import datagen
    import paper_2002_09094_amd as ivf

    dev = "cuda:0"
    copy_gbps, add_gbps = stream_gbps()
    inst = datagen.batched_instances()
    data = {}
    for w, _ in inst:
        if w.name not in data:
            x = w.generate()
            xd = (torch.from_numpy(x.indptr).to(dev), torch.from_numpy(x.indices).to(dev),
                  torch.from_numpy(x.values).to(dev))
            data[w.name] = (x, xd)
    nnz_total = sum(data[w.name][0].nnz for w, _ in inst)
    log("generated %d object sets for %d instances, %d objects, %d nonzeros over instances"
        % (len(data), len(inst), sum(w.n for w, _ in inst), nnz_total))
    b = ivf.IVFBatch([(*data[w.name][1], w.d) for w, _ in inst], [w.k for w, _ in inst],
                     valtype=args.valtype, cluster_range=args.cluster_range,
                     waves_per_wg=args.waves)
    b.init_seeds([torch.from_numpy(w.seeds(data[w.name][0], restart=r).astype(np.int32)).to(dev)
                  for w, r in inst])
    assigns = [torch.full((w.n,), -1, dtype=torch.int32, device=dev) for w, _ in inst]
    warmup = max(args.warmup, 3)
    for r in range(warmup):
        st = b.iterate(1, assigns)[0]
        log("warmup %d: batch iteration %.1f ms (walk %.1f), M=%.3e, plan %s"
            % (r, st[0]["assign_ms"], st[0]["walk_ms"], sum(s["mult_adds"] for s in st), b.plan))
    torch.cuda.synchronize()
    per = []
    t_start = time.perf_counter()
    for r in range(args.steps):
        st = b.iterate(1, assigns)[0]
        per.append(st)
        log("step %d: batch iteration %.1f ms (walk %.1f), M=%.3e, changed=%d, rescored=%d"
            % (r, st[0]["assign_ms"], st[0]["walk_ms"], sum(s["mult_adds"] for s in st),
               sum(s["changed"] for s in st), sum(s["rescored"] for s in st)))
    torch.cuda.synchronize()
    t_total = time.perf_counter() - t_start
    plan = b.plan
    tuning = b.tuning
    log("autotuner (clusters per tile, waves, walk ms): %s" % tuning)
    thetas = b.threshold_tuning
    log("autotuner (dense-slab threshold, walk ms): %s" % thetas)

    mult = sum(s["mult_adds"] for st in per for s in st)
    walk_avg_s = sum(st[0]["walk_ms"] for st in per) / len(per) / 1e3
    kr = plan["kr_max"]
    wb = [sum(walk_bytes(s["mult_adds"], data[w.name][0].nnz, w.n, -(-w.k // kr), args.valtype)
              for s, (w, _) in zip(st, inst)) for st in per]
    ceilings, probe_shapes = read_ceilings()

    # the state after the timed iterations, for the oracle leg: every
    # instance's means and assignment, then one more iteration
    before = []
    for i, (w, _) in enumerate(inst):
        ptr, idx, val = (t.cpu().numpy() for t in b.get_means(i))
        before.append(((ptr, idx, val), assigns[i].cpu().numpy()))
    b.iterate(1, assigns)
    after = [t.cpu().numpy() for t in assigns]
    out = {
        "metric": BATCH_METRIC,
        "value": mult / t_total,
        "unit": "mult-adds/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": warmup,
        "ms_per_step": 1e3 * t_total / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.valtype,
        "data": "synthetic",
        "config": {"workload": "batched96", "instances": len(inst), "object_sets": len(data),
                   "objects": sum(w.n for w, _ in inst), "nnz": nnz_total,
                   "k_range": [min(w.k for w, _ in inst), max(w.k for w, _ in inst)],
                   "valtype": args.valtype, "plan": plan,
                   "autotuner": [{"clusters_per_tile": t[0], "waves": t[1], "walk_ms": t[2]}
                                 for t in tuning],
                   "autotuner_dense_threshold": [{"threshold": round(t, 4), "walk_ms": ms}
                                                 for (t, ms) in thetas]},
        "iter_per_s": args.steps / t_total,
        "mult_adds_per_iter": mult / len(per),
        "walk_ms": 1e3 * walk_avg_s,
        "iteration_ms": sum(st[0]["assign_ms"] for st in per) / len(per),
        "certified_fraction": (sum(s["certified"] for st in per for s in st)
                               / (len(per) * sum(w.n for w, _ in inst))),
        "roofline": walk_roofline("k_walk_batch", "batched96", args.valtype, walk_avg_s,
                                  sum(wb) / len(wb), ceilings, copy_gbps, add_gbps,
                                  probe_shapes),
    }
    b.close()
    if not args.no_cpu_baseline:
        out["cpu_baseline"], out["oracle_check"] = batched_cpu_baseline(inst, data, before, after,
                                                                       args.cpu_seconds)
    print(json.dumps(out), flush=True)


def batched_cpu_baseline(inst, data, before, after, target_s):
    """The FP64 oracle on this host's cores over the batched instances' state
    after the timed iterations: its assignment walk over the first objects of
    successive instances (from their means and previous assignment) until
    about target_s of CPU work; the same results check the GPU's next
    iteration on a seeded sample of 96 objects of every instance."""
    import numpy as np

    import datagen
    import oracle

    threads = int(os.environ.get("OMP_NUM_THREADS", len(os.sched_getaffinity(0))))
    exact, sampled = 0, 0
    for i, (w, r) in enumerate(inst):
        x = data[w.name][0]
        m = min(w.n, 96)
        rows = np.sort(datagen.perm_prefix(w.n, m, w.seed + 1000 * r, stream=7))
        means = oracle.Means(w.k, w.d, *before[i][0])
        ar = oracle.assign(x.subset(rows), means, before[i][1][rows], threads=threads)
        exact += int(np.array_equal(after[i][rows], ar.assign))
        sampled += m
    log("oracle check: %d of %d instances identical on %d sampled objects"
        % (exact, len(inst), sampled))
    cm, ct, used, objs = 0, 0.0, 0, 0
    for i, (w, _) in enumerate(inst):
        x = data[w.name][0]
        m = min(w.n, 4000)
        rows = np.arange(m)
        means = oracle.Means(w.k, w.d, *before[i][0])
        t = time.perf_counter()
        ar = oracle.assign(x.subset(rows), means, before[i][1][rows], threads=threads)
        ct += time.perf_counter() - t
        cm += ar.mult_adds
        used += 1
        objs += m
        if ct >= target_s:
            break
    log("cpu baseline: %d objects of %d instances, %.3e mult-adds in %.1fs" % (objs, used, cm, ct))
    base = {"value": cm / ct, "unit": "mult-adds/s", "cores": threads, "kind": "oracle",
            "sample": "FP64 oracle assignment walk of the first %d objects of each of the "
                      "first %d instances (%d objects) against their means after the timed "
                      "iterations, %.1fs" % (4000, used, objs, ct)}
    return base, {"instances_identical_to_oracle": exact, "instances": len(inst),
                  "oracle_sampled_objects": sampled}


def main():
    if len(sys.argv) > 1 and sys.argv[1] == "summarize-trace":
        summarize_trace(*sys.argv[2:6])
        return
    if len(sys.argv) > 1 and sys.argv[1] == "summarize-update-trace":
        summarize_update_trace(*sys.argv[2:5])
        return
    if len(sys.argv) > 1 and sys.argv[1] == "summarize-pmc":
        summarize_pmc(*sys.argv[2:])
        return
    if len(sys.argv) > 1 and sys.argv[1] == "summarize-counters":
        print(json.dumps(summarize_counters(*sys.argv[2:9])))
        return
    if len(sys.argv) > 1 and sys.argv[1] == "summarize-levels":
        a = sys.argv[2:]
        print(json.dumps(summarize_levels(a[0], a[1], a[2], a[3], a[4], a[5], int(a[6]),
                                          *a[7:])))
        return
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="pubmed_8m")
    ap.add_argument("--valtype", default="f32", choices=sorted(ENTRY_BYTES))
    ap.add_argument("--cluster-range", type=int, default=0)
    ap.add_argument("--waves", type=int, default=0)
    ap.add_argument("--chunk", type=int, default=0)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--ivfd-range", type=int, default=16384,
                    help="IVFD workload: objects per LDS tile (4096, 8192 or 16384)")
    ap.add_argument("--ivfd-8m-only", action="store_true",
                    help="IVFD workload: only the 8M-document set")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first run a plain 1 GiB device copy 3 times (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)
    if args.workload == "batched96":
        run_batched(args)
        return
    if args.workload == "figures":
        run_figures(args)
        return
    if args.workload == "ivfd":
        run_ivfd(args)
        return

    run_single(args)


def run_single(args):
    """One workload on one handle: the benchmark's Lloyd chain (default: 8M
    documents x 140k terms, k = 10,000)."""
    import numpy as np
    import torch

    import datagen
    import paper_2002_09094_amd as ivf

    if args.calibrate_copy:
        calibration_copies()
    copy_gbps, add_gbps = stream_gbps()
    ceilings, probe_shapes = read_ceilings()
    w = datagen.WORKLOADS[args.workload]
    log("generating %s: n=%d d=%d lambda=%g k=%d" % (w.name, w.n, w.d, w.lam, w.k))
    x = w.generate()
    seeds = w.seeds(x)
    log("generated nnz=%d" % x.nnz)
    dev = "cuda:0"
    xd = (torch.from_numpy(x.indptr).to(dev), torch.from_numpy(x.indices).to(dev),
          torch.from_numpy(x.values).to(dev))
    km = ivf.IVFKMeans(*xd, w.d, w.k, valtype=args.valtype, cluster_range=args.cluster_range,
                       waves_per_wg=args.waves, objects_per_item=args.chunk)
    km.init_seeds(torch.from_numpy(seeds.astype(np.int32)).to(dev))
    a = torch.full((w.n,), -1, dtype=torch.int32, device=dev)
    plan = km.plan
    log("built; plan %s" % plan)
    for r in range(args.warmup):
        sa = km.assign(a)
        su = km.update(a)
        log("warmup %d: assign %.1f ms (walk %.1f), update %.1f ms, M=%.3e, rescored=%d"
            % (r, sa["assign_ms"], sa["walk_ms"], su["update_ms"], sa["mult_adds"],
               sa["rescored"]))
    torch.cuda.synchronize()
    per = []
    step_ms = []
    snaps = []
    t_start = time.perf_counter()
    for r in range(args.steps):
        t0 = time.perf_counter()
        sa = km.assign(a)
        snaps.append(a.clone())   # for the per-iteration hashes, read after the timed region
        su = km.update(a)         # both calls synchronise: the step's wall time
        step_ms.append(1e3 * (time.perf_counter() - t0))
        per.append((sa, su))
        log("step %d: assign %.1f ms (walk %.1f), update %.1f ms, M=%.3e, certified=%d, "
            "rescored=%d, changed=%d" % (r, sa["assign_ms"], sa["walk_ms"], su["update_ms"],
                                         sa["mult_adds"], sa["certified"], sa["rescored"],
                                         sa["changed"]))
    torch.cuda.synchronize()
    t_total = time.perf_counter() - t_start
    hashes = [hashlib.sha256(t.cpu().numpy().tobytes()).hexdigest() for t in snaps]
    del snaps

    # one more assignment outside the timed region: the state the oracle checks
    means = km.get_means()
    check = {"means": tuple(t.cpu().numpy() for t in means), "prev": a.cpu().numpy()}
    del means
    sc = km.assign(a)
    best, best_id, second, _, flags = (t.cpu().numpy() for t in km.get_scores())
    check.update({"stats": sc, "assign": a.cpu().numpy(), "best": best, "best_id": best_id,
                  "second": second, "flags": flags})

    R = plan["ranges"]
    mult = sum(p[0]["mult_adds"] for p in per)
    walk_s = sum(p[0]["walk_ms"] for p in per) / 1e3
    assign_s = sum(p[0]["assign_ms"] for p in per) / 1e3
    bytes_iter = sum(iteration_bytes(p[0]["mult_adds"], x.nnz, x.n, R, p[1]["nnz_means"],
                                     args.valtype) for p in per)
    wb = [walk_bytes(p[0]["mult_adds"], x.nnz, x.n, R, args.valtype) for p in per]
    walk_avg_s = walk_s / len(per)
    algorithmic = (sum(wb) / len(wb)) / walk_avg_s / 1e9
    out = {
        "metric": METRIC,
        "value": args.steps / t_total,
        "unit": "iter/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * t_total / args.steps,
        "median_ms_per_step": float(np.median(step_ms)),
        "step_ms": step_ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.valtype,
        "data": "synthetic",
        "config": {"workload": w.name, "n": w.n, "d": w.d, "k": w.k, "nnz": x.nnz,
                   "lambda": w.lam, "zipf_s": w.s, "seed": w.seed, "valtype": args.valtype,
                   "plan": plan},
        "mult_adds_per_s": mult / t_total,
        "mult_adds_per_s_walk": mult / walk_s,
        "mult_adds_per_iter": mult / len(per),
        "gbps_algorithmic_iteration": bytes_iter / t_total / 1e9,
        "assign_ms": 1e3 * assign_s / len(per),
        "walk_ms": 1e3 * walk_avg_s,
        "update_ms": sum(p[1]["update_ms"] for p in per) / len(per),
        "walk_ms_per_step": [p[0]["walk_ms"] for p in per],
        "update_ms_per_step": [p[1]["update_ms"] for p in per],
        "certified_fraction": sum(p[0]["certified"] for p in per) / (len(per) * x.n),
        "rescored_per_iter": sum(p[0]["rescored"] for p in per) / len(per),
        "max_rel_err_rescored": max(p[0]["max_rel_err_rescored"] for p in per),
        "assign_sha256_per_step": hashes,
        "changed_per_step": [p[0]["changed"] for p in per],
        "objective": per[-1][1]["objective_exact"],
        "roofline": walk_roofline("k_walk", w.name, args.valtype, walk_avg_s,
                                  sum(wb) / len(wb), ceilings, copy_gbps, add_gbps,
                                  probe_shapes),
    }
    km.close()
    del xd, a
    torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        out["cpu_baseline"], out["precision_check"] = cpu_baseline(
            x, w, args.valtype, check, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

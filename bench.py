#!/usr/bin/env python3
"""Throughput of the batched GPU search on the mid-size workload, one JSON line.

Workload (the paper's mid-size plain method): a 200,000-sequence data bank
(log-normal lengths, median 1,000 bp, about 275 Mbp, per-sequence GC 0.35-0.65)
and 1,000 queries, log-uniform 80-10,000 bp, half planted homologs at 70-99%
identity with 1% indels; k = 11, +1/-3, gap 5 + 2g, band 32, X-drop 20, top 50.

A step is one gg_search_batch_device call over all 1,000 queries: every stage of
the path, with the queries already resident in GPU memory and the hits written
to GPU memory, its waves replayed from the library's captured HIP graph.  The
call returns only when its results are complete.

``--workload large-batched`` times the same step over 100,000 short queries
(100-250 bp, 80% bank regions with 1-3% substitutions, top 20) against the large
bank (500,000 sequences, about 3 Gbp, with tandem and interspersed repeats);
``--workload large-served`` serves queries of 50-20,000 bp against the large bank
at 50, 200 and 1,000 arrivals/s and times the batched step over 2,000 of them.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from paper_1507_02987_amd import gg, synth  # noqa: E402

METRIC = "queries/s and DB-Gbp·query-kbp/s at 1 GPU; p50/p99 latency under load"
HBM_PEAK_GBS = 8000.0
# 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz: int32 vector lane-operations per second
VALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12
CAP = 64
# int32 operations one banded Smith-Waterman cell needs: E and F (2 subtractions,
# 1 max and 1 start select each), G (compare, select, add), H (3 max), the start
# of H (2 compares, 2 selects) and the best-cell update (compare, 3 selects)
ALIGN_OPS_PER_CELL = 22


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in ("gg_kernels.hip", "gg_internal.h"):
        with open(os.path.join(ROOT, "paper_1507_02987_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_for(stage: str, workload: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary for this
    kernel, if the counters were taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", f"traffic_{stage}_{workload}.txt")
    if not os.path.exists(path):
        return None
    fields = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line:
                key, val = line.split(":", 1)
                fields[key.strip()] = val.strip()
    if fields.get("kernel_source") != kernel_source_hash():
        return None
    return int(fields["bytes_per_launch"]) if "bytes_per_launch" in fields else None


def cpu_baseline(db, qs, max_hits: int, min_seconds: float = 8.0):
    """The oracle, untuned, over all queries on the host cores (index excluded)."""
    sys.path.insert(0, os.path.join(ROOT, "oracle"))
    import ggo  # checker / baseline only
    from concurrent.futures import ThreadPoolExecutor

    ggo.build()
    cores = min(16, len(os.sched_getaffinity(0)))
    oix = ggo.Index(db.seqs, db.off, 11)
    prm = ggo.params(max_hits)
    queries = [bytes(qs.query(i)) for i in range(qs.n)]

    def run(q):
        return oix.search(q, prm, cap=CAP)[0]

    done, t0 = 0, time.perf_counter()
    chunk = 4 * cores
    with ThreadPoolExecutor(max_workers=cores) as ex:
        while True:
            part = [queries[(done + j) % len(queries)] for j in range(chunk)]
            rcs = list(ex.map(run, part))
            assert all(r in (0, 5) for r in rcs)
            done += len(part)
            if time.perf_counter() - t0 >= min_seconds:
                break
    dt = time.perf_counter() - t0
    return {"value": done / dt, "unit": "queries/s", "cores": cores, "kind": "oracle",
            "sample": f"the workload's queries in order, {done} searched ({done / len(queries):.2f} "
                      f"of the set), {dt:.1f} s wall on {cores} threads (index build excluded)"}


def serve_leg(gix, db, prm, rate: float, n: int) -> dict:
    """Open-loop Poisson arrivals at `rate` queries/s into the continuous-batching
    server; latency = completion time - scheduled arrival time.  The first 32
    served results are checked against the one-query form."""
    import threading

    qs = synth.large_served_queries(db, n=n)
    arr = synth.served_arrivals(rate, n)
    want = {}
    for i in range(min(32, n)):
        rc, h, _ = gix.search(qs.query(i), prm, cap=CAP)
        want[i] = h.tobytes()
    sv = gg.Server(gix, prm, hit_budget_bytes=0, max_slots=256)
    tickets = [None] * n
    done = [0.0] * n
    submitted = [0]
    lock = threading.Lock()
    status = []

    def collector():
        pending = set()
        nxt = 0
        while nxt < n or pending:
            with lock:
                upto = submitted[0]
            while nxt < upto:
                pending.add(nxt)
                nxt += 1
            for i in list(pending):
                rc, h, m = sv.poll(tickets[i], cap=CAP, timeout_us=0)
                if rc != gg.GG_EAGAIN:
                    done[i] = time.perf_counter()
                    status.append(rc)
                    pending.discard(i)
                    if i in want:
                        assert h.tobytes() == want[i], f"served query {i} differs"
            time.sleep(0.0001)

    th = threading.Thread(target=collector)
    th.start()
    t0 = time.perf_counter()
    for i in range(n):
        target = t0 + arr[i]
        while True:
            now = time.perf_counter()
            if now >= target:
                break
            time.sleep(min(target - now, 0.0005))
        tickets[i] = sv.submit(qs.query(i))
        with lock:
            submitted[0] = i + 1
    th.join()
    t_end = max(done)
    sv.close()
    assert all(r in (gg.GG_OK, gg.GG_ETRUNC) for r in status)
    lat = np.array([done[i] - (t0 + arr[i]) for i in range(n)]) * 1e3
    return {"rate_per_s": rate, "requests": n, "p50_ms": round(float(np.percentile(lat, 50)), 3),
            "p99_ms": round(float(np.percentile(lat, 99)), 3),
            "achieved_qps": round(n / (t_end - t0), 1)}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--workload", choices=("mid", "large-batched", "large-served"), default="mid")
    ap.add_argument("--queries", type=int, default=0, help="queries per step (0: the workload's)")
    ap.add_argument("--no-serve", action="store_true", help="skip the served-form latency leg")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="BYTES",
                    help="only copy BYTES device-to-device three times (counter calibration)")
    ap.add_argument("--no-tune", action="store_true",
                    help="keep the library's default launch choices (for profiler runs)")
    ap.add_argument("--no-plain", action="store_true",
                    help="skip the one-query-at-a-time comparison (for kernel-trace runs)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the search would shard by query or by data-bank range)", file=sys.stderr)
        return 2

    gg.lib()  # the compiled HIP library, or a loud failure
    if args.calibrate_copy:
        a, b = gg.DeviceBuffer(args.calibrate_copy), gg.DeviceBuffer(args.calibrate_copy)
        for _ in range(3):
            b.copy_from(a, args.calibrate_copy)
        log(f"copied {args.calibrate_copy} bytes device-to-device 3 times")
        return 0
    t = time.perf_counter()
    if args.workload == "mid":
        cfg, db = 1, synth.mid_db()
        qs = synth.mid_queries(db, n=args.queries or 1000)
        desc = "mid-size: 200,000-seq bank (~275 Mbp), 1,000 queries 80-10,000 bp, k=11, top 50"
    else:
        db = synth.large_db()
        if args.workload == "large-batched":
            cfg, qs = 3, synth.large_short_queries(db, n=args.queries or 100_000)
            desc = ("large bank, short queries: 500,000-seq bank (~3 Gbp, repeats), 100,000 "
                    "queries 100-250 bp, "
                    "k=11, top 20")
        else:
            cfg, qs = 4, synth.large_served_queries(db, n=args.queries or 2000)
            desc = ("large bank, served: 500,000-seq bank (~3 Gbp, repeats), queries 50-20,000 "
                    "bp, k=11, "
                    "top 50, served at 50/200/1,000 per s")
    if args.queries:
        desc = desc.replace(f"{qs.n:,}", str(qs.n))
    workload = {1: "mid", 3: "large_short", 4: "large_served"}[cfg]
    log(f"workload: {db.n_seqs} seqs, {db.total_bp / 1e6:.1f} Mbp, {qs.n} queries, "
        f"{qs.lengths().sum()} query bp ({time.perf_counter() - t:.1f} s)")
    max_hits = synth.TOP_N[cfg]
    prm = gg.params(max_hits)

    t = time.perf_counter()
    gix = gg.Index(db.seqs, db.off, 11, device=0)
    build_s = time.perf_counter() - t
    log(f"index built on GPU 0 in {build_s:.1f} s: {gix.info()}")

    # launch choices picked by the library's autotuner on the workload's batch (on
    # its first 48 queries for the large workloads, whose batches take seconds)
    t = time.perf_counter()
    if args.no_tune:
        tuning = gix.tuning()
    else:
        sample = qs if cfg == 1 else qs.subset(np.arange(min(48, qs.n)))
        log(f"autotuning on {sample.n} queries ...")
        tuning = gix.autotune(sample.buf, sample.off, prm)
        log(f"autotuned on {sample.n} queries in {time.perf_counter() - t:.1f} s: {tuning}")

    # inputs resident in HBM before the timed region
    dq = gg.DeviceBuffer(max(len(qs.buf), 1))
    dq.upload(qs.buf)
    dout = gg.DeviceBuffer(qs.n * CAP * gg.HIT_DTYPE.itemsize)
    dn = gg.DeviceBuffer(qs.n * 4)

    def step():
        rc, _ = gix.search_batch_device(dq, qs.off, prm, dout, dn, CAP)
        if rc not in (gg.GG_OK, gg.GG_ETRUNC):
            raise gg.GGError(rc, "gg_search_batch_device")

    for _ in range(args.warmup):
        step()
    log(f"warmup {args.warmup} done")
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    dt = time.perf_counter() - t0
    qps = qs.n * args.steps / dt
    gbp_kbp = (db.total_bp / 1e9) * (qs.lengths().sum() / 1e3) * args.steps / dt
    log(f"timed {args.steps} steps: {dt * 1e3 / args.steps:.3f} ms/step, {qps:.0f} queries/s")
    # the same steps with every wave launched kernel by kernel (no captured graph);
    # the large workloads' queries exceed a graph wave, so they never use it
    nograph_ms, graph_waves = None, 0
    if args.workload == "mid":
        os.environ["GG_GRAPH"] = "0"
        t1 = time.perf_counter()
        for _ in range(args.steps):
            step()
        nograph_ms = (time.perf_counter() - t1) * 1e3 / args.steps
        del os.environ["GG_GRAPH"]
        gix.profile(True)
        step()
        graph_waves = gix.profile_read("graph")["units"]
        gix.profile(False)
        log(f"without the wave graph: {nograph_ms:.3f} ms/step; graph waves per step: "
            f"{graph_waves}")

    # device results equal the host-buffer form (PCIe-inclusive rate measured here
    # too); the large workloads skip this second full pass
    pcie_qps = None
    if args.workload == "mid":
        got_n = dn.download(np.zeros(qs.n, np.int32))
        got = dout.download(np.zeros(qs.n * CAP, gg.HIT_DTYPE))
        t1 = time.perf_counter()
        rc, res, n_host, _ = gix.search_batch(qs.buf, qs.off, prm, cap=CAP, stats=True)
        pcie_qps = qs.n / (time.perf_counter() - t1)
        assert rc in (gg.GG_OK, gg.GG_ETRUNC)
        assert np.array_equal(got_n, n_host)
        for i in range(qs.n):
            m = min(int(n_host[i]), CAP)
            assert got[i * CAP: i * CAP + m].tobytes() == res[i].tobytes(), i

    # per-kernel GPU time, HIP events on the library's stream, over profiled steps
    nprof = 3 if args.workload == "mid" else 1
    gix.profile(True)
    for _ in range(nprof):
        rc, stats = gix.search_batch_device(dq, qs.off, prm, dout, dn, CAP, stats=True)
        assert rc in (gg.GG_OK, gg.GG_ETRUNC)
    stages = {s: gix.profile_read(s) for s in (
        "encode", "scan", "gather_prep", "probe", "gather_count", "gather", "group", "filter",
        "filter_compact", "sort_hist", "sort_scan", "sort_scatter", "chain", "chain_write",
        "extend", "merge", "merge_sweep", "select", "align", "report")}
    gix.profile(False)
    step_ms = {s: v["ms"] / nprof for s, v in stages.items()}
    cells = int(stats["n_cells"].sum())
    hits = int(stats["n_hits"].sum())
    # Algorithmic work per launch of each modelled kernel:
    #  probe   - HBM: the 8 B posting of every hit plus 16 B per query position
    #            (hit offset, list head, query id, window code); neighbour-window
    #            probes are cache traffic and not counted
    #  gather  - HBM: 8 B posting read + 8 B key write per hit
    #  filter  - HBM: 8 B key read per hit (the kept few are written back)
    #  sort_*  - HBM: 16 B per key per scatter pass, 8 B per histogram pass
    #  align   - integer ALU: ALIGN_OPS_PER_CELL int32 operations per in-band cell
    positions = int(qs.lengths().sum())
    model = {
        "probe": ("hbm", lambda st: 8 * st["units"] + 16 * positions * st["launches"]),
        "gather": ("hbm", lambda st: 16 * st["units"]),
        "filter": ("hbm", lambda st: 8 * st["units"]),
        "sort_scatter": ("hbm", lambda st: 16 * st["units"]),
        "sort_hist": ("hbm", lambda st: 8 * st["units"]),
        "align": ("alu", lambda st: ALIGN_OPS_PER_CELL * cells * nprof),
    }
    kernel_name = {"probe": "k_probe_chain", "gather": "k_gather", "filter": "k_hit_filter",
                   "sort_scatter": "k_rs_scatter",
                   "sort_hist": "k_rs_hist", "align": "k_bsw"}
    cand = {s: stages[s] for s in model if stages[s]["launches"]}

    def roofline_of(stage):
        st = cand[stage]
        bound, work_fn = model[stage]
        per_launch = work_fn(st) / st["launches"]
        avg_s = st["ms"] / 1e3 / st["launches"]
        if bound == "hbm":
            achieved, peak, unit = per_launch / avg_s / 1e9, HBM_PEAK_GBS, "GB/s"
        else:
            achieved, peak, unit = per_launch / avg_s / 1e12, VALU_PEAK_TOPS, "TOP/s"
        # traffic: HBM bytes per launch from the committed counter summary (also for
        # the ALU-bound aligner, where it shows how little memory it moves)
        return {"bound": bound, "kernel": kernel_name[stage], "achieved": round(achieved, 2),
                "peak": peak, "unit": unit, "frac": round(achieved / peak, 4),
                "traffic": traffic_for(stage, workload),
                "avg_launch_us": round(avg_s * 1e6, 2),
                "algorithmic_work_per_launch": int(per_launch)}

    dom = max(cand, key=lambda s: cand[s]["ms"])
    roofline = roofline_of(dom)
    other_rooflines = [roofline_of(s) for s in sorted(cand, key=lambda s: -cand[s]["ms"])
                       if s != dom]
    al = stages["align"]
    align_gcups = cells / (al["ms"] / nprof / 1e3) / 1e9 if al["ms"] > 0 else None

    # the plain one-query-at-a-time loop on the same GPU, for comparison
    plain_qps = None
    if not args.no_plain:
        n_plain = min(200 if cfg != 3 else 2000, qs.n)
        t1 = time.perf_counter()
        for i in range(n_plain):
            rc, _, _ = gix.search(qs.query(i), prm, cap=CAP)
            assert rc in (gg.GG_OK, gg.GG_ETRUNC)
        plain_qps = n_plain / (time.perf_counter() - t1)
    log(f"plain per-query loop: {plain_qps} queries/s; PCIe-inclusive batch: {pcie_qps}")

    serve = []
    if not args.no_serve and cfg != 3:
        # served form: queries shaped like the serving workload (log-uniform 50-20,000
        # bp, 60% planted homologs) against the resident bank, Poisson arrivals
        legs = ((50.0, 2000), (200.0, 2000), (1000.0, 2000)) if cfg == 4 else \
            ((200.0, 400), (1000.0, 1000), (5000.0, 2000))
        for rate, n in legs:
            serve.append(serve_leg(gix, db, prm, rate, n))
            log(f"served at {rate:.0f}/s: {serve[-1]}")

    cpu = None
    if not args.no_cpu:
        log("oracle CPU baseline ...")
        cpu = cpu_baseline(db, qs, max_hits)
        log(f"oracle: {cpu['value']:.0f} queries/s on {cpu['cores']} threads")

    line = {
        "metric": METRIC, "value": round(qps, 1), "unit": "queries/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(dt * 1e3 / args.steps, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": desc + ", batched", "db_bp": db.total_bp,
                   "queries": qs.n, "query_bp": int(qs.lengths().sum()), "k": 11,
                   "max_hits": max_hits, "parallelism": "single GPU"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "extra": {
            "db_gbp_query_kbp_per_s": round(gbp_kbp, 2),
            "plain_per_query_qps": round(plain_qps, 1) if plain_qps else None,
            "pcie_inclusive_batch_qps": round(pcie_qps, 1) if pcie_qps else None,
            "index_build_s": round(build_s, 2),
            "tuning": tuning,
            "graph_waves_per_step": graph_waves,
            "ms_per_step_without_graph": round(nograph_ms, 4) if nograph_ms else None,
            "stage_ms_per_step": {s: round(v, 4) for s, v in step_ms.items()},
            "other_rooflines": other_rooflines,
            "hits_per_step": hits,
            "align_cells_per_step": cells,
            "align_gcups": round(align_gcups, 2) if align_gcups else None,
            "valu_peak_tops": round(VALU_PEAK_TOPS, 1),
            "served": serve,
        },
    }
    print(json.dumps(line), flush=True)
    for b in (dq, dout, dn):
        b.close()
    gix.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())

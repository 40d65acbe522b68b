#!/usr/bin/env python3
"""Throughput of the batched GPU search on the large resident bank, one JSON line.

Headline workload (the paper's scale: a ~3 Gbp data bank): 500,000 bank
sequences, log-normal lengths with median 4,000 bp (about 3.0 Gbp), 10% of the
bases in tandem repeats and 5% in interspersed repeat families; 2,000 queries,
log-uniform 500-5,000 bp, half planted homologs at 75-99% identity with 1%
indels; k = 11, +1/-3, gap 5 + 2g, band 32, X-drop 20, top 100.

A step is one gg_search_batch call over all 2,000 queries: query bytes in host
memory through every stage of the path to the hits in host memory.  The index is
resident in HBM; its build is timed apart.  Every step returns only when its hits
are in host memory.

After the timed steps, `extra` holds, on the same GPU:
* `mid`: the mid-size bank (200,000 sequences, ~275 Mbp; 1,000 queries of
  80-10,000 bp, top 50), timed device-resident (queries and hits in HBM), with
  its kernels' rooflines;
* `short`: 100,000 short queries (100-250 bp, top 20) against the large bank in
  one batched call, beside the plain one-query-at-a-time loop;
* `served`: queries of 50-20,000 bp (top 50) arriving Poisson at 50, 200 and
  1,000 per second into the continuous-batching server under a 16 GiB hit
  budget, with p50/p99 latency (first 10% of each rate dropped as warm-up).
`cpu_baseline` is the oracle on this host's cores over a seeded sample of the
headline queries, and on one thread.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import platform
import queue
import sys
import threading
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from paper_1507_02987_amd import gg, synth  # noqa: E402

METRIC = "queries/s and DB-Gbp·query-kbp/s at 1 GPU; p50/p99 latency under load"
HBM_PEAK_GBS = 8000.0
# 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz: int32 vector lane-operations per second
VALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12
# int32 operations one banded Smith-Waterman cell needs: E and F (2 subtractions,
# 1 max and 1 start select each), G (compare, select, add), H (3 max), the start
# of H (2 compares, 2 selects) and the best-cell update (compare, 3 selects)
ALIGN_OPS_PER_CELL = 22
SERVE_BUDGET = 16 << 30  # hit-buffer bytes of the served form (16 GiB)
# Launch choices each workload runs with: grouping, X-drop lane steps, wave size
# (log2 hits, 0 = the default), graph replay on/off, and the largest query (log2
# hits) a replayed wave takes (0 = any that fits a wave).  Picked by measurement on
# each workload (`--autotune` reruns gg_index_autotune instead); profiles taken
# with the same table agree.  On the 3 Gbp bank, graph waves limited to queries of
# at most 2^18 hits match the plain loop (long queries) or beat it (short ones),
# while taking every query that fits loses 10%.
TUNING = {"large": ("sort", 256, 0, 1, 18), "mid": ("sort", 256, 0, 1, 0),
          "short": ("sort", 256, 0, 1, 18), "served": ("sort", 256, 0, 1, 18)}


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
    kernel and workload, if the counters were taken on the current kernel source."""
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


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def oracle_rate(oix, prm, queries, order, threads: int, seconds: float, cap: int):
    """Searches queries[order[0]], queries[order[1]], ... with the oracle on
    `threads` threads until `seconds` of wall time; returns (completed, elapsed,
    hits of the completed ones).  Searches still running at the deadline are left
    to finish in the background and not counted."""
    import ggo  # checker / baseline only

    todo = queue.Queue()
    for i in order:
        todo.put(int(i))
    done = []
    lock = threading.Lock()
    stop = threading.Event()

    def worker():
        while not stop.is_set():
            try:
                i = todo.get_nowait()
            except queue.Empty:
                return
            rc, _, _, st = oix.search(queries[i], prm, cap=cap)
            assert rc in (0, 5)
            with lock:
                if not stop.is_set():
                    done.append((i, int(st["n_hits"])))

    t0 = time.perf_counter()
    ths = [threading.Thread(target=worker, daemon=True) for _ in range(threads)]
    for t in ths:
        t.start()
    deadline = t0 + seconds
    for t in ths:
        t.join(max(0.0, deadline - time.perf_counter()))
    stop.set()
    elapsed = min(time.perf_counter(), deadline) - t0
    with lock:
        got = list(done)
    _ = ggo
    return len(got), elapsed, sum(h for _, h in got)


def cpu_baseline(db, qs, max_hits: int, cap: int, hits_per_query: np.ndarray):
    """The oracle, untuned, on the host cores: the headline's queries in a seeded
    random order, as many as finish in 20 s on all threads, then in 15 s on one."""
    sys.path.insert(0, os.path.join(ROOT, "oracle"))
    import ggo  # checker / baseline only

    ggo.build()
    t = time.perf_counter()
    oix = ggo.Index(db.seqs, db.off, 11)
    build_s = time.perf_counter() - t
    prm = ggo.params(max_hits)
    queries = [bytes(qs.query(i)) for i in range(qs.n)]
    order = np.random.default_rng([synth.ROOT_SEED, 2]).permutation(qs.n)
    # one GPU's share of the host: at most 16 threads
    cores = min(16, len(os.sched_getaffinity(0)))
    n_all, dt_all, h_all = oracle_rate(oix, prm, queries, order, cores, 20.0, cap)
    n_one, dt_one, h_one = oracle_rate(oix, prm, queries, order[::-1], 1, 15.0, cap)
    mean_h = float(hits_per_query.mean())
    return {
        "value": round(n_all / dt_all, 3), "unit": "queries/s", "cores": cores,
        "kind": "oracle",
        "sample": (f"headline queries in a seeded random order on {cores} threads, {n_all} "
                   f"finished in {dt_all:.1f} s (mean {h_all / max(n_all, 1) / 1e6:.2f} M hits "
                   f"each, workload mean {mean_h / 1e6:.2f} M); searches running at the "
                   f"deadline not counted; oracle index build {build_s:.0f} s excluded"),
        "cpu_model": cpu_model(),
        "one_thread": {"value": round(n_one / dt_one, 3), "unit": "queries/s",
                       "sample": f"reverse of the same order, {n_one} finished in {dt_one:.1f} s "
                                 f"(mean {h_one / max(n_one, 1) / 1e6:.2f} M hits each)"},
        "oracle_hits_per_s_all_threads": round(h_all / dt_all),
    }


# Algorithmic work per launch of each modelled kernel:
#  gather  - HBM: 8 B posting read + 8 B key write per hit
#  filter  - HBM: 8 B key read per hit (the kept few are written back)
#  sort_*  - HBM: 16 B per key per scatter pass, 8 B per histogram pass
#  align   - integer ALU: ALIGN_OPS_PER_CELL int32 operations per in-band cell
KERNEL = {"gather": "k_gather", "filter": "k_hit_filter", "gather_filter": "k_gather_filter",
          "sort_scatter": "k_rs_scatter_seg",
          "sort_hist": "k_rs_hist_seg", "align": "k_bsw"}


def rooflines(stages: dict, cells: int, nprof: int, workload: str):
    model = {
        "gather": ("hbm", lambda st: 16 * st["units"]),
        "filter": ("hbm", lambda st: 8 * st["units"]),
        # one posting entry read per hit; the kept keys it writes are a few per mille
        "gather_filter": ("hbm", lambda st: 8 * st["units"]),
        "sort_scatter": ("hbm", lambda st: 16 * st["units"]),
        "sort_hist": ("hbm", lambda st: 8 * st["units"]),
        "align": ("alu", lambda st: ALIGN_OPS_PER_CELL * cells * nprof),
    }
    cand = {s: stages[s] for s in model if stages.get(s, {}).get("launches")}

    def one(stage):
        st = cand[stage]
        bound, work_fn = model[stage]
        per_launch = work_fn(st) / st["launches"]
        avg_s = st["ms"] / 1e3 / st["launches"]
        if bound == "hbm":
            achieved, peak, unit = per_launch / avg_s / 1e9, HBM_PEAK_GBS, "GB/s"
        else:
            achieved, peak, unit = per_launch / avg_s / 1e12, VALU_PEAK_TOPS, "TOP/s"
        return {"bound": bound, "kernel": KERNEL[stage], "achieved": round(achieved, 2),
                "peak": peak, "unit": unit, "frac": round(achieved / peak, 4),
                "traffic": traffic_for(stage, workload), "avg_launch_us": round(avg_s * 1e6, 2),
                "launches": st["launches"] // nprof,
                "algorithmic_work_per_launch": int(per_launch)}

    order = sorted(cand, key=lambda s: -cand[s]["ms"])
    return [one(s) for s in order]


STAGES = ("encode", "scan", "gather_prep", "probe", "gather_count", "gather", "group",
          "gather_filter", "filter",
          "filter_compact", "sort_hist", "sort_scan", "sort_scatter", "chain", "chain_write",
          "extend", "merge", "merge_sweep", "select", "align", "report", "graph")


def profile_steps(gix, run, nprof: int):
    """Per-stage GPU time (HIP events on the library's stream) over nprof steps;
    run(stats) performs one step and returns the per-query stats."""
    gix.profile(True)
    stats = None
    for _ in range(nprof):
        stats = run(True)
    stages = {s: gix.profile_read(s) for s in STAGES}
    gix.profile(False)
    return stages, stats


def set_tuning(gix, which: str, args, sample=None, prm=None) -> dict:
    if args.autotune and sample is not None:
        t = time.perf_counter()
        tun = gix.autotune(sample.buf, sample.off, prm)
        log(f"autotuned on {sample.n} queries in {time.perf_counter() - t:.1f} s: {tun}")
        return tun
    grouping, lane_steps, wave_log2, graph, graph_qlog2 = TUNING[which]
    gix.set_tuning(grouping, lane_steps, wave_log2, graph, graph_qlog2)
    return gix.tuning()


def mid_leg(args) -> dict:
    """The mid-size bank, device-resident batched steps (queries and hits in HBM)."""
    db = synth.mid_db()
    qs = synth.mid_queries(db, n=1000)
    cap = prm_n = synth.TOP_N[1]
    prm = gg.params(prm_n)
    gix = gg.Index(db.seqs, db.off, 11, device=0)
    tun = set_tuning(gix, "mid", args, qs, prm)
    dq = gg.DeviceBuffer(max(len(qs.buf), 1))
    dq.upload(qs.buf)
    dout = gg.DeviceBuffer(qs.n * cap * gg.HIT_DTYPE.itemsize)
    dn = gg.DeviceBuffer(qs.n * 4)

    def run(stats=False):
        rc, st = gix.search_batch_device(dq, qs.off, prm, dout, dn, cap, stats=stats)
        if rc not in (gg.GG_OK, gg.GG_ETRUNC):
            raise gg.GGError(rc, "gg_search_batch_device")
        return st

    for _ in range(3):
        run()
    steps = 20
    t0 = time.perf_counter()
    for _ in range(steps):
        run()
    dt = (time.perf_counter() - t0) / steps
    gix.profile(True)
    run()
    graph_waves = gix.profile_read("graph")["units"]
    gix.profile(False)
    stages, st = profile_steps(gix, run, 3)
    cells = int(st["n_cells"].sum())
    out = {"workload": "mid-size bank: 200,000 seqs (~275 Mbp), 1,000 queries 80-10,000 bp, "
                       "k=11, top 50, device-resident",
           "queries_per_s": round(qs.n / dt, 1), "ms_per_step": round(dt * 1e3, 4),
           "db_gbp_query_kbp_per_s": round(db.total_bp / 1e9 * qs.lengths().sum() / 1e3 / dt, 1),
           "graph_waves_per_step": graph_waves, "tuning": tun,
           "hits_per_step": int(st["n_hits"].sum()), "align_cells_per_step": cells,
           "stage_ms_per_step": {s: round(v["ms"] / 3, 4) for s, v in stages.items() if v["ms"]},
           "rooflines": rooflines(stages, cells, 3, "mid")}
    for b in (dq, dout, dn):
        b.close()
    gix.close()
    return out


def aligner_probe(L: int) -> None:
    """One query copying L bases of a random bank sequence, with substitutions at
    2% of its positions: the search ends in one L x L box, whose banded DP is one
    serial chain of about L pair steps (the aligner's time per pair step)."""
    rng = np.random.default_rng(3)
    acgt = np.frombuffer(b"ACGT", np.uint8)
    bank = acgt[rng.integers(0, 4, L + 1000)]
    q = bank[500:500 + L].copy()
    pos = rng.choice(L, L // 50, replace=False)
    q[pos] = acgt[(np.searchsorted(acgt, q[pos]) + 1) % 4]
    gix = gg.Index(bank, np.array([0, len(bank)], np.int64), 11, device=0)
    prm = gg.params(10)
    for _ in range(5):
        rc, hits, n = gix.search(q.tobytes(), prm, cap=10)
    log(f"aligner probe: status {rc}, {n} hit(s), first box "
        f"{(int(hits[0]['box_q_end']) - int(hits[0]['box_q_start'])) if n else 0} query bases")


def short_leg(db, gix, args) -> dict:
    """100,000 short queries against the large bank in one batched call, beside
    the plain one-query-at-a-time loop over 2,000 of them."""
    t = time.perf_counter()
    qs = synth.large_short_queries(db, n=args.short_queries)
    log(f"short queries: {qs.n} ({time.perf_counter() - t:.1f} s)")
    cap = synth.TOP_N[3]
    prm = gg.params(cap)
    tun = set_tuning(gix, "short", args)
    out = np.zeros(qs.n * cap, gg.HIT_DTYPE)
    nout = np.zeros(qs.n, np.int32)
    warm = qs.subset(np.arange(min(500, qs.n)))
    gix.search_batch_into(warm.buf, warm.off, prm, out, nout, cap)
    gix.profile(True)
    t0 = time.perf_counter()
    rc = gix.search_batch_into(qs.buf, qs.off, prm, out, nout, cap)
    dt = time.perf_counter() - t0
    graph = gix.profile_read("graph")
    gix.profile(False)
    assert rc in (gg.GG_OK, gg.GG_ETRUNC), gg.STATUS[rc]
    n_plain = min(2000, qs.n)
    t1 = time.perf_counter()
    for i in range(n_plain):
        rc, _, _ = gix.search(qs.query(i), prm, cap=cap)
        assert rc in (gg.GG_OK, gg.GG_ETRUNC)
    plain_qps = n_plain / (time.perf_counter() - t1)
    return {"workload": "large bank, short queries: 100,000 queries 100-250 bp (80% bank regions "
                        "with 1-3% substitutions), k=11, top 20, one batched call, host buffers",
            "queries": qs.n, "queries_per_s": round(qs.n / dt, 1), "wall_s": round(dt, 2),
            "graph_waves": graph["units"], "graph_ms": round(graph["ms"], 1),
            "plain_per_query_qps": round(plain_qps, 1), "plain_sample": n_plain, "tuning": tun,
            "alignments": int(np.minimum(nout, cap).sum())}


def serve_leg(gix, qs, prm, cap: int, rate: float, n: int, check: dict) -> dict:
    """Open-loop Poisson arrivals at `rate` queries/s into the continuous-batching
    server; latency = completion time - scheduled arrival time, the first 10% of
    requests dropped as warm-up.  Queries in `check` must equal their one-query
    results."""
    arr = synth.served_arrivals(rate, n)
    sv = gg.Server(gix, prm, hit_budget_bytes=SERVE_BUDGET, max_slots=256)
    tickets = [None] * n
    done = [0.0] * n
    submitted = [0]
    lock = threading.Lock()
    status = []
    bad = []

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
                rc, h, m = sv.poll(tickets[i], cap=cap, timeout_us=0)
                if rc != gg.GG_EAGAIN:
                    done[i] = time.perf_counter()
                    status.append(rc)
                    pending.discard(i)
                    if i in check and h.tobytes() != check[i]:
                        bad.append(i)
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
    assert not bad, f"served queries differ from their one-query results: {bad[:5]}"
    assert all(r in (gg.GG_OK, gg.GG_ETRUNC) for r in status)
    lat = np.array([done[i] - (t0 + arr[i]) for i in range(n)]) * 1e3
    kept = lat[n // 10:]
    return {"rate_per_s": rate, "requests": n, "warmup_dropped": n // 10,
            "p50_ms": round(float(np.percentile(kept, 50)), 3),
            "p99_ms": round(float(np.percentile(kept, 99)), 3),
            "achieved_qps": round(n / (t_end - t0), 1)}


def served_legs(db, gix, args) -> list:
    qs = synth.large_served_queries(db, n=args.served_queries)
    cap = synth.TOP_N[4]
    prm = gg.params(cap)
    set_tuning(gix, "served", args)
    check = {}
    for i in range(min(16, qs.n)):
        rc, h, _ = gix.search(qs.query(i), prm, cap=cap)
        check[i] = h.tobytes()
    out = []
    for rate in (50.0, 200.0, 1000.0):
        out.append(serve_leg(gix, qs, prm, cap, rate, qs.n, check))
        log(f"served at {rate:.0f}/s: {out[-1]}")
    return out


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--queries", type=int, default=0, help="headline queries (0: all 2,000)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the mid, short-query and served legs (for profiler runs)")
    ap.add_argument("--no-mid", action="store_true")
    ap.add_argument("--no-short", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--short-queries", type=int, default=100_000)
    ap.add_argument("--served-queries", type=int, default=2000)
    ap.add_argument("--autotune", action="store_true",
                    help="run gg_index_autotune instead of the fixed launch choices")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="BYTES",
                    help="only copy BYTES device-to-device three times (counter calibration)")
    ap.add_argument("--calibrate-read", type=int, default=0, metavar="BYTES",
                    help="only stream-read BYTES three times (counter calibration)")
    ap.add_argument("--only-mid", action="store_true",
                    help="only the mid-size device-resident leg, printed as JSON (profiler runs)")
    ap.add_argument("--aligner-probe", type=int, default=0, metavar="L",
                    help="only search, 5 times, one query copying L bases of a bank sequence "
                         "with 2%% substitutions: one L x L box for the aligner (profiler runs)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the search would shard by query or by data-bank range)", file=sys.stderr)
        return 2

    gg.lib()  # the compiled HIP library, or a loud failure
    if args.calibrate_copy or args.calibrate_read:
        nb = args.calibrate_copy or args.calibrate_read
        a, b = gg.DeviceBuffer(nb), gg.DeviceBuffer(nb)
        for _ in range(3):
            if args.calibrate_copy:
                b.copy_from(a, nb)
            else:
                a.read_sum(nb)
        log(f"{'copied' if args.calibrate_copy else 'stream-read'} {nb} bytes 3 times")
        return 0

    if args.only_mid:
        print(json.dumps(mid_leg(args)), flush=True)
        return 0
    if args.aligner_probe:
        aligner_probe(args.aligner_probe)
        return 0

    t = time.perf_counter()
    db = synth.large_db()
    qs = synth.large_queries(db, n=args.queries or 2000)
    log(f"workload: {db.n_seqs} seqs, {db.total_bp / 1e6:.1f} Mbp, {qs.n} queries, "
        f"{qs.lengths().sum()} query bp ({time.perf_counter() - t:.1f} s)")
    cap = synth.TOP_N[2]
    prm = gg.params(cap)
    desc = ("large bank: 500,000-seq bank (~3.0 Gbp, 10% tandem + 5% interspersed repeats), "
            f"{qs.n:,} queries 500-5,000 bp (half planted homologs), k=11, top 100, "
            "host buffers in and out")

    t = time.perf_counter()
    gix = gg.Index(db.seqs, db.off, 11, device=0)
    build_s = time.perf_counter() - t
    log(f"index built on GPU 0 in {build_s:.2f} s: {gix.info()}")
    tuning = set_tuning(gix, "large", args, qs.subset(np.arange(min(48, qs.n))), prm)

    out = np.zeros(qs.n * cap, gg.HIT_DTYPE)
    nout = np.zeros(qs.n, np.int32)

    def step():
        rc = gix.search_batch_into(qs.buf, qs.off, prm, out, nout, cap)
        if rc not in (gg.GG_OK, gg.GG_ETRUNC):
            raise gg.GGError(rc, "gg_search_batch")

    for i in range(args.warmup):
        step()
        log(f"warmup step {i + 1}/{args.warmup}")
    t0 = time.perf_counter()
    for i in range(args.steps):
        step()
        if (i + 1) % 5 == 0:
            log(f"timed step {i + 1}/{args.steps}")
    dt = time.perf_counter() - t0
    # --steps 0 (profiler runs): only the per-stage step below runs on the GPU
    qps = qs.n * args.steps / dt
    gbp_kbp = (db.total_bp / 1e9) * (qs.lengths().sum() / 1e3) * args.steps / dt
    log(f"timed {args.steps} steps: {dt * 1e3 / max(args.steps, 1):.1f} ms/step, "
        f"{qps:.1f} queries/s")

    # per-stage GPU time over one more step, with per-query work counts
    def run(stats=False):
        rc, res, n_h, st = gix.search_batch(qs.buf, qs.off, prm, cap=cap, stats=stats)
        assert rc in (gg.GG_OK, gg.GG_ETRUNC)
        return st

    stages, st = profile_steps(gix, run, 1)
    cells = int(st["n_cells"].sum())
    hits = st["n_hits"].astype(np.int64)
    roofs = rooflines(stages, cells, 1, "large")
    roofline = roofs[0] if roofs else None
    log(f"stages (ms): { {s: round(v['ms'], 1) for s, v in stages.items() if v['ms']} }")

    extra = {"db_gbp_query_kbp_per_s": round(gbp_kbp, 2), "index_build_s": round(build_s, 2),
             "tuning": tuning, "hits_per_step": int(hits.sum()),
             "max_hits_one_query": int(hits.max()),
             "runs_per_step": int(st["n_cands"].sum()), "align_cells_per_step": cells,
             "stage_ms_per_step": {s: round(v["ms"], 3) for s, v in stages.items() if v["ms"]},
             "other_rooflines": roofs[1:], "valu_peak_tops": round(VALU_PEAK_TOPS, 1)}
    if not args.no_extra and not args.no_mid:
        extra["mid"] = mid_leg(args)
        log(f"mid: {extra['mid']['queries_per_s']} queries/s device-resident")
    if not args.no_extra and not args.no_short:
        extra["short"] = short_leg(db, gix, args)
        log(f"short: {extra['short']}")
    if not args.no_extra and not args.no_serve:
        extra["served"] = served_legs(db, gix, args)

    cpu = None
    if not args.no_cpu:
        log("oracle CPU baseline ...")
        cpu = cpu_baseline(db, qs, cap, cap, hits)
        log(f"oracle: {cpu['value']} queries/s on {cpu['cores']} threads, "
            f"{cpu['one_thread']['value']} on one")

    line = {
        "metric": METRIC, "value": round(qps, 2), "unit": "queries/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(dt * 1e3 / max(args.steps, 1), 2),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": desc, "db_bp": db.total_bp, "queries": qs.n,
                   "query_bp": int(qs.lengths().sum()), "k": 11, "max_hits": cap,
                   "parallelism": "single GPU"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "extra": extra,
    }
    print(json.dumps(line), flush=True)
    gix.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())

"""Benchmark of the free-Boolean-generator path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload c1|c3]

Default workload: random 3-CNF model counting, n = 32 variables, m = 136
clauses (ratio 4.25), 16 seeded instances (seeds 0..15), full 2^32 valuation
space each.  One step is the whole hot path over that batch, with the
programs resident on the device:

  * compile       residency lookup of the 16 compiled programs
  * evaluate      one persistent batched launch over all 16 programs:
                  generator synthesis, evaluation, the 2^32-bit DNF vector of
                  every instance (512 MiB each), its model count and the
                  model count of every tile
  * enumerate     one batched enumeration: a scan over the tile counts of all
                  instances and one compaction launch that reads the DNF
                  vectors only in tiles holding models

value = 16 * 2^32 valuations per step / step time.  The JSON line also
carries the roofline of the dominant kernel (the batched evaluator, measured
with HIP events on the launch stream: bound by the HBM write of the DNF
vectors, 1/8 byte per valuation), the batched versus per-formula ("plain")
count rates, the CPU oracle timed on a bounded sample on this host, and a
"c3" block: the 4096-formula batch (one batched count per step replayed from
a HIP graph against 4096 plain launches, and the unspecialized interpreter's
fraction of the VALU bitwise peak on the programs that have a general part).

Workload c3: the same 4096-formula block as the line's workload.
Workload c4: the serving loop (Poisson arrivals, continuous batching),
reporting p50/p99 latency beside valuations/s.
Workload posets: labeled partial orders through the c-partition counting
procedure (bounded posets on --posets-n elements).
Workload theories: one count of each propositional theory of the paper's
examples, at every tiling, with and without the uniform-cofactor variant.
Workload unlabeled: non-isomorphic partial orders (7 elements) and graphs (7
vertices) by the Frobenius-Burnside lemma.
Workload copy: a 1 GiB device copy, the calibration kernel for the HBM byte
counters, and an 8 GiB fill (the write ceiling).
Workload valu: the attainable v_bitop3 issue rate (independent chains on a
full grid), the check of the VALU peak the bitwise fractions are quoted
against.
"""

import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# MI355X: 256 CUs x 64 lanes x 32 bits x 2.4 GHz, one 2-input bitwise
# operation per 32-bit lane per clock.
VALU_BITWISE_PEAK = 256 * 64 * 32 * 2.4e9
METRIC = "valuations/sec and % VALU bitwise peak (batched vs plain, bit-exact counts)"
HBM_PEAK = 8e12  # bytes/s

# The paper's own figure for this path, on its hardware (Section 2.3): a term
# of 2^17 nodes over 30 variables in about 1 s on a PC with two GPUs of 2^11
# 32-bit cores each (OpenCL) -- 2^30 valuations/s, 2^47 node-bit-ops/s.
PAPER_CONTEXT = {"valuations_per_s": 2.0 ** 30, "node_bit_ops_per_s": 2.0 ** 47,
                 "hardware": "PC with 2 GPUs x 2^11 32-bit cores, OpenCL (GPUs not named)",
                 "workload": "30 variables, 2^17-node term, about 1 s (Section 2.3)"}

# HBM bytes of one launch of the dominant kernel, from the FETCH_SIZE and
# WRITE_SIZE counters (rocprofv3 --pmc, one counter per run), each scaled by
# the reading of the same counter for a device copy of 1 GiB (FETCH_SIZE reads
# half the bytes copied, WRITE_SIZE all of them), for k_batch_direct<5> (16
# DNF vectors + tile counts), together with the SHA-1 of the kernel sources
# (their code, comments left out) the counters were taken on.  The bench line
# reports the bytes only while the sources still have that digest, and null
# otherwise.
C1_TRAFFIC = {"bytes": 8606066816, "kernel_sources_sha1": "f9c1039855fcdb7cf1166deeffbccc7ce8e7d404"}
KERNEL_SOURCES = ("fbg_device.h", "fbg_asm16.h", "fbg_isa.h", "fbg_kernels.h", "batch.hip")


def code_of(text):
    """C/HIP source without its comments and blank space, so that an edit of
    comments alone keeps the digest (string literals hold no comment marks)."""
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    return " ".join(text.split())


def kernel_sources_sha1():
    h = hashlib.sha1()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1310_6978_amd", "csrc", name), encoding="utf-8") as f:
            h.update(code_of(f.read()).encode())
    return h.hexdigest()


def c1_traffic():
    if C1_TRAFFIC["bytes"] is None or C1_TRAFFIC["kernel_sources_sha1"] != kernel_sources_sha1():
        return None
    return C1_TRAFFIC["bytes"]


class ProgramCache:
    """Compiled programs stay resident, keyed by (text hash, n)."""

    def __init__(self, fbg):
        self.fbg = fbg
        self.progs = {}
        self.compile_s = 0.0

    def get(self, text, n):
        key = (hashlib.sha1(text.encode()).hexdigest(), n)
        p = self.progs.get(key)
        if p is None:
            t0 = time.perf_counter()
            p = self.fbg.Program(text, n)
            self.compile_s += time.perf_counter() - t0
            self.progs[key] = p
        return p


def ev_ms(a, b):
    return a.elapsed_time(b)


def host_cpu():
    """Model name of the host CPU (from /proc/cpuinfo) and its logical CPUs."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"model": model, "nproc": os.cpu_count()}


def cpu_bitparallel(text, n):
    """The oracle's blocked evaluation of Section 2.3 (64 valuations per
    word, generator blocks from the definition of M) over the whole valuation
    space of one instance: the paper-style CPU path, as a cross-check."""
    import oracle
    threads = min(os.cpu_count() or 1, 16)
    t0 = time.perf_counter()
    c = oracle.bitpar_count(text, n, threads)
    dt = time.perf_counter() - t0
    return {"value": float(1 << n) / dt, "unit": "valuations/s", "cores": threads, "kind": "oracle-bitparallel",
            "sample": "all 2^%d valuations of seed 0 (%.1f s, %d models)" % (n, dt, c), "count": c}


def cpu_baseline(text, n, target_s=15.0):
    """The oracle, as it stands, on a contiguous sample of the valuation
    space of one instance; scaled to valuations/s."""
    import oracle
    threads = min(os.cpu_count() or 1, 16)
    lo = 0
    size = 1 << 22
    t0 = time.perf_counter()
    oracle.count_range(text, n, lo, lo + size, threads)
    dt = time.perf_counter() - t0
    # grow the sample to about target_s seconds of work
    size2 = int(size * max(1.0, target_s / max(dt, 1e-3)))
    size2 = max(size, min(size2, (1 << n) - lo))
    size2 -= size2 % 64
    t0 = time.perf_counter()
    c = oracle.count_range(text, n, lo, lo + size2, threads)
    dt = time.perf_counter() - t0
    return {"value": size2 / dt, "unit": "valuations/s", "cores": threads, "kind": "oracle",
            "sample": "per-valuation oracle over valuations [0, %d) of seed 0 (%.1f s, %d models)"
                      % (size2, dt, c)}


def golden_c1():
    """Oracle counts and model lists of the 16 instances (tests/golden)."""
    path = os.path.join(ROOT, "tests", "golden", "c1_3cnf_n32.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        g = json.load(f)
    return {int(s): r for s, r in g["seeds"].items()}


def bench_c1(args, torch, fbg):
    import workloads
    seeds = list(range(16))
    texts = [workloads.random_3cnf(32, 136, s) for s in seeds]
    cache = ProgramCache(fbg)
    progs = [cache.get(t, n) for t, n in texts]
    cold_compile_s = cache.compile_s
    n = 32
    words = 1 << (n - 6)
    batch = fbg.Batch(progs)
    counts = torch.empty(len(progs), dtype=torch.int64, device="cuda")
    dnfs = [torch.empty(words, dtype=torch.int64, device="cuda") for _ in progs]
    batch.set_dnf_outputs(dnfs)
    cap = 4096
    idx = [torch.empty(cap, dtype=torch.int64, device="cuda") for _ in progs]
    batch.set_enum_outputs(idx)
    stream = torch.cuda.current_stream()
    ev = []

    def step(record):
        for t, nn in texts:                                          # compile (resident lookup)
            cache.get(t, nn)
        if record:
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record(stream)
        batch.eval_dnf(counts=counts, stream=stream)                 # evaluate + DNF + count, batched
        if record:
            b.record(stream)
            ev.append((a, b))
        batch.enumerate(stream=stream)                               # models of all, from the DNF vectors

    for _ in range(args.warmup):
        step(False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step(True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_step = (t1 - t0) * 1e3 / args.steps

    got = counts.cpu().numpy().view("uint64").tolist()
    lists = [ii.cpu().numpy().view("uint64")[:min(c, cap)].tolist() for ii, c in zip(idx, got)]
    gold = golden_c1()
    exact = None
    if gold is not None and all(s in gold for s in seeds):
        exact = all(got[i] == gold[s]["count"] and lists[i] == gold[s]["models"][:cap]
                    for i, s in enumerate(seeds))
    k_ms = sum(ev_ms(a, b) for a, b in ev) / len(ev)

    # counting alone: one batched launch vs 16 plain launches, and the
    # uniform-cofactor variant of the batched count
    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(reps):
            fn()
        b.record(stream)
        torch.cuda.synchronize()
        return ev_ms(a, b) / reps

    reps = max(args.steps, 3)
    bc = torch.empty(len(progs), dtype=torch.int64, device="cuda")
    batch_ms = timed(lambda: batch.count(out=bc, stream=stream), reps)
    batch_same = bc.cpu().numpy().view("uint64").tolist() == got
    plain_out = torch.empty(1, dtype=torch.int64, device="cuda")

    def plain():
        for p in progs:
            fbg.count(p, out=plain_out, stream=stream)
    plain_ms = timed(plain, 3)
    cbatch = fbg.Batch(progs, cofactor=True)
    cof_ms = timed(lambda: cbatch.count(out=bc, stream=stream), reps)
    cof_same = bc.cpu().numpy().view("uint64").tolist() == got
    cbatch.free()

    vals = len(progs) * float(1 << n)
    dnf_bytes = vals / 8  # the DNF vectors, 1/8 byte per valuation
    l2in = sum(p.info["l2in"] for p in progs)
    achieved = l2in * float(1 << n) / (k_ms / 1e3)
    res = {
        "metric": METRIC,
        "value": vals / (ms_step / 1e3),
        "unit": "valuations/s",
        "ms_per_step": ms_step,
        "dtype": "u32",
        "config": {"workload": "random 3-CNF model counting, n=32, m=136 (ratio 4.25), seeds 0-15; per step: "
                               "one batched launch writing the 2^32-bit DNF vector and the per-tile model "
                               "counts of every instance, the counts summed from the tile counts, then one "
                               "batched enumeration of all models from the DNF vectors",
                   "n": n, "clauses": 136, "instances": len(progs),
                   "words_per_lane": progs[0].info["words_per_lane"]},
        "roofline": {"bound": "hbm", "achieved": dnf_bytes / (k_ms / 1e3) / 1e9, "peak": HBM_PEAK / 1e9,
                     "unit": "GB/s", "frac": dnf_bytes / (k_ms / 1e3) / HBM_PEAK, "traffic": c1_traffic(),
                     "kernel": "k_batch_direct<5> (16 programs: evaluation, DNF write-out, tile counts; "
                               "with the per-program sums of k_sum_tile_counts in the timed call)",
                     "avg_ms": k_ms, "algorithmic_bytes_per_launch": dnf_bytes,
                     "algorithmic_bitops_per_launch": l2in * float(1 << n),
                     "algorithmic_bitop_rate_T": achieved / 1e12,
                     "valu_bitwise_peak_T": VALU_BITWISE_PEAK / 1e12},
        "batched_vs_plain": {"batched_count_ms": batch_ms, "plain_count_ms": plain_ms,
                             "batched_valuations_per_s": vals / (batch_ms / 1e3),
                             "plain_valuations_per_s": vals / (plain_ms / 1e3),
                             "speedup": plain_ms / batch_ms, "counts_equal": batch_same},
        "dnf_write_out": {"bytes_per_launch": len(progs) * float(1 << n) / 8,
                          "gb_per_s": len(progs) * float(1 << n) / 8 / (k_ms / 1e3) / 1e9,
                          "frac_of_hbm_peak": len(progs) * float(1 << n) / 8 / (k_ms / 1e3) / HBM_PEAK},
        "paper_context": PAPER_CONTEXT,
        "cofactor": {"batched_count_ms": cof_ms, "valuations_per_s": vals / (cof_ms / 1e3),
                     "speedup_vs_full_evaluation": batch_ms / cof_ms, "counts_equal": cof_same},
        # The clause block factors the clauses over the index classes (one
        # per-lane product per group of clauses, a product tree over the
        # words), so this C1 figure is the factored path's algorithmic rate
        # over the bitwise peak, not a roofline: it exceeds 1.  The
        # unspecialized interpreter's fraction is c3.general_plans below.
        "factored_algorithmic_rate_over_valu_peak": achieved / VALU_BITWISE_PEAK,
        "counts": got,
        "bit_exact_vs_oracle": exact,
        "cold_compile_ms_per_program": cold_compile_s * 1e3 / len(progs),
    }
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline(texts[0][0], n)
        res["cpu_bitparallel"] = cpu_bitparallel(texts[0][0], n)
        res["cpu_bitparallel"]["count_equal"] = res["cpu_bitparallel"]["count"] == got[0]
        res["host"] = host_cpu()
    return res


def c3_block(args, torch, fbg):
    """The 4096 random DAG formulas (n in [10,30], 50..2000 ops, seed 0):
    one batched count per step replayed from a captured HIP graph, against
    4096 plain single-program launches; and the unspecialized interpreter's
    algorithmic fraction: sum of L_2in 2^n over the programs that have a
    general part (every program operation on every word), over the time of
    their own batched launch, over the VALU bitwise peak."""
    from workloads.formulas import random_dag_batch
    from paper_1310_6978_amd import autotune
    log = lambda m: print("c3: " + m, file=sys.stderr, flush=True)  # noqa: E731
    batch_f = random_dag_batch(4096, 0)
    t0 = time.perf_counter()
    progs = [fbg.Program(t, n) for t, n in batch_f]
    compile_ms = (time.perf_counter() - t0) * 1e3
    vals = float(sum(1 << n for _, n in batch_f))
    tuner = autotune.Tuner()
    wpl = tuner.tune_batch(progs)                       # cached per device and program set
    tuned = tuner.table.get(tuner.last_key, {})
    log("%d programs compiled in %.0f ms, %d words per lane" % (len(progs), compile_ms, wpl))
    stream = torch.cuda.current_stream()

    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(reps):
            fn()
        b.record(stream)
        torch.cuda.synchronize()
        return a.elapsed_time(b) / reps

    reps = max(args.steps, 3)
    b = fbg.Batch(progs, words_per_lane=wpl)
    counts = torch.empty(len(progs), dtype=torch.int64, device="cuda")
    eager_ms = timed(lambda: b.count(out=counts, stream=stream), reps)
    graph_ms = timed(lambda: b.count(out=counts, stream=stream, graph=True), reps)
    got = counts.cpu().numpy().view("uint64").tolist()
    outs = torch.empty(len(progs), dtype=torch.int64, device="cuda")

    def plain():
        for i, p in enumerate(progs):
            fbg.count(p, out=outs[i:i + 1], stream=stream)
    plain_ms = timed(plain, 1)
    log("batched %.2f ms (graph) / %.2f ms (eager), plain %.1f ms" % (graph_ms, eager_ms, plain_ms))
    same = got == outs.cpu().numpy().view("uint64").tolist()
    exact = None
    path = os.path.join(ROOT, "tests", "golden", "c3_dag_batch.json")
    if os.path.exists(path):
        with open(path) as f:
            exact = [r["count"] for r in json.load(f)["formulas"]] == got
    # the programs with a general part, as a batch of their own
    gen = [p for p in progs if p.info["n_instr"] > p.info["n_clause_instr"]]
    gen_l2in = sum(p.info["l2in"] * 2.0 ** p.n for p in gen)
    gb = fbg.Batch(gen, words_per_lane=wpl)
    gout = torch.empty(len(gen), dtype=torch.int64, device="cuda")
    gen_ms = timed(lambda: gb.count(out=gout, stream=stream), reps)
    gen_rate = gen_l2in / (gen_ms / 1e3)
    gb.free()
    # the small and the large formulas apart: each set as a batch of its own
    # and as plain launches
    by_n = {}
    for name, sel in (("n<=20", lambda n: n <= 20), ("n>=28", lambda n: n >= 28)):
        part = [p for p in progs if sel(p.n)]
        pb = fbg.Batch(part, words_per_lane=wpl)
        pout = torch.empty(len(part), dtype=torch.int64, device="cuda")
        p_ms = timed(lambda: pb.count(out=pout, stream=stream), reps)
        pb.free()

        def plain_part():
            for i, p in enumerate(part):
                fbg.count(p, out=pout[i:i + 1], stream=stream)
        pp_ms = timed(plain_part, 1)
        pv = float(sum(1 << p.n for p in part))
        by_n[name] = {"formulas": len(part), "batched_ms": p_ms, "plain_ms": pp_ms,
                      "batched_valuations_per_s": pv / (p_ms / 1e3), "plain_valuations_per_s": pv / (pp_ms / 1e3)}
    b.free()
    l2in = sum(p.info["l2in"] * 2.0 ** p.n for p in progs)
    return {
        "formulas": len(progs), "words_per_lane": wpl, "autotune_ms": tuned.get("ms"),
        "compile_ms": compile_ms,
        "batched_step_ms_graph": graph_ms, "batched_step_ms_eager": eager_ms,
        "plain_4096_launches_ms": plain_ms, "speedup_batched_vs_plain": plain_ms / graph_ms,
        "valuations_per_s": vals / (graph_ms / 1e3),
        "algorithmic_bitops_per_step": l2in,
        "general_plans": {"programs": len(gen), "sum_l2in_2n": gen_l2in, "ms": gen_ms,
                          "algorithmic_rate_T": gen_rate / 1e12,
                          "frac_of_valu_bitwise_peak": gen_rate / VALU_BITWISE_PEAK},
        "by_n": by_n,
        "counts_equal_oracle": exact, "batched_equals_plain": same,
    }


def bench_c3(args, torch, fbg):
    r = c3_block(args, torch, fbg)
    ms = r["batched_step_ms_graph"]
    g = r["general_plans"]
    return {
        "metric": METRIC, "value": r["valuations_per_s"], "unit": "valuations/s", "ms_per_step": ms,
        "dtype": "u32",
        "config": {"workload": "4096 random DAG formulas, n in [10,30], 50-2000 ops, seed 0; per step one "
                               "batched count replayed from a HIP graph",
                   "formulas": r["formulas"], "words_per_lane": r["words_per_lane"]},
        "roofline": {"bound": "alu", "achieved": g["algorithmic_rate_T"], "peak": VALU_BITWISE_PEAK / 1e12,
                     "unit": "Tbitop/s", "frac": g["frac_of_valu_bitwise_peak"], "traffic": None,
                     "kernel": "the batched count of the %d programs with a general part" % g["programs"]},
        "c3": r,
        "bit_exact_vs_oracle": r["counts_equal_oracle"],
    }


def bench_c4(args, torch, fbg):
    """Serving: Poisson arrivals of model-counting requests (90% random 3-CNF
    with n uniform in [12,36] and ratio 4.25, 10% the theories of the k=9
    equivalence, 5x5 permutation and k=8 triangle-free workloads), continuous
    batching.  First a burst (every request arriving at once), then the
    saturation rate: the rate served while real-time arrivals come at 1.25 x
    the burst rate; then one timed run per load level, arrivals at that
    fraction of the saturation rate.  Results are checked against the
    theories' closed forms and against the stored oracle counts of the
    stream's 3-CNF requests with n <= 20 (tests/golden/c4_requests.json)."""
    from paper_1310_6978_amd.serve import ServeLoop
    from workloads.serving import request_stream

    def log(msg):
        print(msg, file=sys.stderr, flush=True)

    loop = ServeLoop(words_per_lane=16, slice_words=args.slice_words, max_active=256)
    warm = request_stream(50, 0.0, seed=99)
    loop.run(warm, realtime=False, log=log)
    log("c4: burst run, %d requests at once" % args.sat_requests)
    burst = loop.run(request_stream(args.sat_requests, 0.0, seed=1), realtime=False, log=log)
    # Requests that are all there at once batch better than arrivals spread
    # in time, so the burst rate overstates what the loop sustains: the
    # saturation rate is the rate served while real-time arrivals come faster
    # than that (1.25 x the burst rate), and the load levels are fractions of it.
    over = 1.25 * burst["requests_per_s"]
    log("c4: burst %.1f req/s; overload run, %d requests at %.1f req/s" % (burst["requests_per_s"],
                                                                          args.sat_requests * 4, over))
    sat = loop.run(request_stream(args.sat_requests * 4, over, seed=2), realtime=True, log=log)
    rate = sat["requests_per_s"]
    closed = {"equivalence_k9": 21147, "permutations_k5": 120, "triangle_free_k8": 4682270}
    with open(os.path.join(ROOT, "tests", "golden", "c4_requests.json")) as f:
        stored = json.load(f)["counts"]
    runs = []
    ok = True
    checked = 0
    for load in [float(x) for x in args.loads.split(",")]:
        qps = load * rate
        log("c4: saturation %.1f req/s; timed run of %d requests at %.1f req/s (%.2f x)"
            % (rate, args.requests, qps, load))
        reqs = request_stream(args.requests, qps, seed=0)
        res = loop.run(reqs, realtime=True, log=log)
        n_ok = 0
        for r in reqs:
            c = res["counts"][r["id"]]
            if r["kind"] in closed:
                ok = ok and c == closed[r["kind"]]
                checked += 1
            elif str(r["id"]) in stored and n_ok < 400:
                rec = stored[str(r["id"])]
                ok = ok and rec["n"] == r["n"] and c == rec["count"]
                checked += 1
                n_ok += 1
        runs.append({"load": load, "qps": qps, "latency_p50_ms": res["latency_p50_ms"],
                     "latency_p99_ms": res["latency_p99_ms"], "latency_mean_ms": res["latency_mean_ms"],
                     "requests_per_s": res["requests_per_s"], "valuations_per_s": res["valuations_per_s"],
                     "gpu_busy": res["gpu_busy"], "slices": res["slices"], "wall_s": res["wall_s"]})
    loop.close()
    mid = runs[len(runs) // 2]
    return {
        "metric": METRIC, "value": mid["valuations_per_s"], "unit": "valuations/s",
        "ms_per_step": mid["wall_s"] * 1e3, "dtype": "u32",
        "config": {"workload": "serving: %d requests per load level, Poisson arrivals at %s x saturation; 90%% "
                               "random 3-CNF n in [12,36] ratio 4.25, 10%% theories (equivalence k=9, 5x5 "
                               "permutations, triangle-free k=8)" % (args.requests, args.loads),
                   "requests": args.requests, "loads": args.loads},
        "serving": {"saturation_requests_per_s": rate, "saturation_valuations_per_s": sat["valuations_per_s"],
                    "saturation_offered_requests_per_s": over,
                    "burst_requests_per_s": burst["requests_per_s"], "burst_valuations_per_s": burst["valuations_per_s"],
                    "runs": runs},
        "bit_exact_vs_oracle": ok, "requests_checked": checked,
    }


def bench_posets(args, torch, fbg):
    """Labeled partial orders on n-2 elements by the counting procedure of
    Section 3.4 (bounded posets of Section 5.2): one program per layering,
    all counted in one batched launch, combined by formula (ltn).  The
    whole theory has (n-2)(n-3) letters (56 at n = 10, beyond one
    evaluation); a layering leaves at most C(n-2, 2)."""
    import workloads
    from paper_1310_6978_amd import tba
    n = args.posets_n
    text, nl = workloads.bounded_posets(n)
    parts = list(tba.bounded_poset_parts(n))
    t0 = time.perf_counter()
    res = tba.bounded_posets(n, text, nl)                     # includes compiling every part
    torch.cuda.synchronize()
    wall_first = time.perf_counter() - t0
    times = {}
    for cof in (True, False):
        progs = [fbg.compile_assume(text + extra, nl, assume) for _, assume, extra in parts]
        b = fbg.Batch(progs, cofactor=cof)
        out = torch.empty(len(progs), dtype=torch.int64, device="cuda")
        for _ in range(args.warmup):
            b.count(out=out)
        s = torch.cuda.current_stream()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s)
        for _ in range(args.steps):
            b.count(out=out)
        e1.record(s)
        torch.cuda.synchronize()
        times[cof] = e0.elapsed_time(e1) / args.steps
        assert out.cpu().numpy().view("uint64").tolist() == [q.count for q in res.parts]
        b.free()
    vals = float(sum(2 ** q.n_free for q in res.parts))
    return {"metric": "labeled partial orders counted by c-partitions (valuations/s of the batched count)",
            "value": vals / (times[True] / 1e3), "unit": "valuations/s", "ms_per_step": times[True],
            "dtype": "u32",
            "config": {"workload": "bounded partial orders n=%d (labeled posets on %d elements), %d layerings"
                                   % (n, n - 2, len(parts)), "letters": nl,
                       "max_free_letters": max(q.n_free for q in res.parts)},
            "labeled_posets": res.total, "batched_count_ms_cofactor": times[True],
            "batched_count_ms_full_evaluation": times[False], "first_run_wall_s_with_compile": wall_first}


def bench_theories(args, torch, fbg):
    """The propositional theories of the paper's examples: one count per
    theory at every tiling, full evaluation and uniform cofactor, against
    their closed-form counts."""
    import workloads
    cases = [("equivalence relations k=9 (Bell 9)", workloads.equivalence_relations(9), 21147),
             ("triangle-free graphs k=8", workloads.triangle_free(8), 4682270),
             ("5x5 permutation matrices", workloads.permutation_matrices(5), 120),
             ("equivalence relations k=6", workloads.equivalence_relations(6), 203)]
    stream = torch.cuda.current_stream()
    out = torch.empty(1, dtype=torch.int64, device="cuda")
    rows, enum_rows, ok, vals, best_total = [], [], True, 0.0, 0.0
    for name, (text, n), want in cases:
        p = fbg.Program(text, n)
        best = None
        for w in (8, 16, 32):
            for cof in (False, True):
                fbg.count(p, out=out, stream=stream, words_per_lane=w, cofactor=cof)
                torch.cuda.synchronize()
                a = torch.cuda.Event(enable_timing=True)
                b = torch.cuda.Event(enable_timing=True)
                a.record(stream)
                for _ in range(args.steps):
                    fbg.count(p, out=out, stream=stream, words_per_lane=w, cofactor=cof)
                b.record(stream)
                torch.cuda.synchronize()
                ms = a.elapsed_time(b) / args.steps
                got = int(out.cpu().numpy().view("uint64")[0])
                ok = ok and got == want
                rows.append({"theory": name, "n": n, "words_per_lane": w, "cofactor": cof, "ms": ms,
                             "alg_frac": p.info["l2in"] * 2.0 ** n / (ms / 1e3) / VALU_BITWISE_PEAK, "count": got})
                if not cof and (best is None or ms < best):
                    best = ms
        vals += 2.0 ** n
        best_total += best
        # every model listed (two passes: tile counts and scan, then the
        # compaction of the tiles that hold models), at the library's tiling
        # (then again with the uniform cofactor at the same tiling: the same
        # list, element by element)
        cap = want
        first = None
        for cof in (False, True):
            if cof:
                p.set_tuning(p.info["words_per_lane"], cofactor=True)
            idx, tot = fbg.enumerate_models(p, cap, stream=stream)
            torch.cuda.synchronize()
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record(stream)
            for _ in range(args.steps):
                fbg.enumerate_models(p, cap, out=idx, total=tot, stream=stream)
            b.record(stream)
            torch.cuda.synchronize()
            ok = ok and int(tot.cpu().numpy().view("uint64")[0]) == want
            got = idx[:want].cpu()
            if first is None:
                first = got
            else:
                ok = ok and bool(torch.equal(got, first))
            enum_rows.append({"theory": name, "models": want, "cofactor": cof,
                              "words_per_lane": p.info["words_per_lane"], "ms": a.elapsed_time(b) / args.steps,
                              "list_bytes": 8 * want})
    return {"metric": "valuations/s of one full-evaluation count per theory (best tiling)",
            "value": vals / (best_total / 1e3), "unit": "valuations/s", "ms_per_step": best_total, "dtype": "u32",
            "config": {"workload": "propositional theories: equivalence k=9 and k=6, triangle-free k=8, "
                                   "5x5 permutations; one count each"},
            "counts_match_closed_forms": ok, "runs": rows, "enumerate": enum_rows}


def bench_c0(args, torch, fbg):
    """Equivalence relations on 6 elements (n = 15, 60 clauses): a launch-
    bound size, so what is reported is the latency of one call from the
    host, synchronised, for the count, the DNF vector and the enumeration,
    each against the stored oracle values (tests/golden/c0_equivalence_k6.json)
    and the closed form B_6 = 203."""
    import numpy as np
    import workloads
    text, n = workloads.equivalence_relations(6)
    p = fbg.Program(text, n)
    stream = torch.cuda.current_stream()
    out = torch.empty(1, dtype=torch.int64, device="cuda")
    dnf = torch.empty(fbg.dnf_words(n), dtype=torch.int64, device="cuda")
    idx = torch.empty(256, dtype=torch.int64, device="cuda")
    tot = torch.empty(1, dtype=torch.int64, device="cuda")
    calls = {"count": lambda: fbg.count(p, out=out, stream=stream),
             "dnf": lambda: fbg.eval_dnf(p, out=dnf, stream=stream),
             "enumerate": lambda: fbg.enumerate_models(p, 256, out=idx, total=tot, stream=stream)}
    reps = max(args.steps, 1) * 40
    lat = {}
    for name, fn in calls.items():
        for _ in range(max(args.warmup, 1) * 10):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
            torch.cuda.synchronize()
        lat[name] = (time.perf_counter() - t0) * 1e6 / reps
    with open(os.path.join(ROOT, "tests", "golden", "c0_equivalence_k6.json")) as f:
        g = json.load(f)
    want_dnf = np.array([int(x, 16) for x in g["dnf_words_hex"]], dtype=np.uint64)
    models = np.array(g["models"], dtype=np.uint64)
    ok = (g["count"] == 203 and int(out.cpu().numpy().view("uint64")[0]) == 203
          and np.array_equal(dnf.cpu().numpy().view(np.uint64), want_dnf)
          and int(tot.cpu().numpy().view("uint64")[0]) == 203
          and np.array_equal(idx.cpu().numpy().view(np.uint64)[:203], models))
    return {"metric": "latency of one call (us, host to result, synchronised)", "value": lat["count"],
            "unit": "us", "ms_per_step": lat["count"] / 1e3, "dtype": "u32",
            "config": {"workload": "equivalence relations k=6: n=15, 60 clauses; count, DNF (512 words), "
                                   "enumeration (203 models)", "n": n},
            "higher_is_better": False, "latency_us": lat, "bit_exact_vs_oracle": ok}


def bench_unlabeled(args, torch, fbg):
    """Non-isomorphic models by the Frobenius-Burnside lemma: one batched
    count of the fixed-point theories of every cycle type."""
    from paper_1310_6978_amd import frontend, unlabeled
    posets = ("S = range({n})\nS2 = perm(S, 2)\nS3 = perm(S, 3)\n"
              "anti = A[i,j:S2] (~p(i,j) | ~p(j,i))\n"
              "trans = A[i,j,k:S3] (~(p(i,j) & p(j,k)) | p(i,k))\n"
              "assumptions = {{p(i,i): 1 for i in S}}\n")
    graphs = ("S = range({n})\nS2 = perm(S, 2)\nsym = A[i,j:S2] (~e(i,j) | e(j,i))\n"
              "assumptions = {{e(i,i): 0 for i in S}}\n")
    rows, total_ms = [], 0.0
    for name, script, n in (("partial orders", posets, 7), ("graphs", graphs, 7)):
        tr = frontend.translate(script.format(n=n))
        t0 = time.perf_counter()
        res = unlabeled.count_translation(tr, range(n), cofactor=True)
        torch.cuda.synchronize()
        first = (time.perf_counter() - t0) * 1e3
        t0 = time.perf_counter()
        for _ in range(args.steps):
            res = unlabeled.count_translation(tr, range(n), cofactor=True)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / args.steps
        total_ms += ms
        rows.append({"structures": name, "n": n, "letters": tr.n, "cycle_types": len(res.terms),
                     "unlabeled": res.unlabeled, "labeled": res.labeled, "ms_with_compile": ms,
                     "first_ms": first})
    return {"metric": "non-isomorphic models counted per second (Frobenius-Burnside, one batched count)",
            "value": len(rows) / (total_ms / 1e3), "unit": "theories/s", "ms_per_step": total_ms, "dtype": "u32",
            "config": {"workload": "unlabeled partial orders on 7 elements and graphs on 7 vertices"},
            "runs": rows}


def bench_valu(args, torch):
    """The attainable integer-bitwise VALU rate (independent v_bitop3 chains,
    full grid): the check of the denominator of the algorithmic fraction."""
    import ctypes
    lib = ctypes.CDLL(os.path.join(ROOT, "paper_1310_6978_amd", "libfbg_probe.so"))
    lib.fbg_probe_valu_peak.restype = ctypes.c_int
    lib.fbg_probe_valu_peak.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_uint32, ctypes.c_uint32,
                                        ctypes.c_void_p]
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    blocks = cus * 8                       # 8 waves per SIMD
    iters = 4096
    out = torch.empty(blocks * 256, dtype=torch.int32, device="cuda")
    stream = torch.cuda.current_stream()

    def launch():
        rc = lib.fbg_probe_valu_peak(ctypes.c_void_p(out.data_ptr()), blocks, iters, 12345,
                                     ctypes.c_void_p(stream.cuda_stream))
        if rc != 0:
            raise RuntimeError("probe launch failed: %d" % rc)
    for _ in range(max(args.warmup, 1)):
        launch()
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record(stream)
    for _ in range(args.steps):
        launch()
    b.record(stream)
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / args.steps
    lane_instr = float(blocks) * 256 * iters * 64
    rate = lane_instr / (ms / 1e3)
    spec = cus * 64 * 2.4e9                # one VALU instruction per lane per clock
    return {"metric": "attainable v_bitop3 rate (VALU peak probe)", "value": rate, "unit": "lane-instr/s",
            "ms_per_step": ms, "dtype": "u32",
            "config": {"workload": "%d blocks x 256 threads, 8 independent v_bitop3 chains, %d x 64 per lane"
                                   % (blocks, iters)},
            "fraction_of_spec": rate / spec, "spec_lane_instr_per_s": spec,
            "bitops_per_s_2input": rate * 32, "valu_bitwise_peak_2input": VALU_BITWISE_PEAK}


def bench_copy(args, torch):
    """A plain device-to-device copy of 1 GiB: the calibration kernel for the
    FETCH_SIZE / WRITE_SIZE counters (it must read and write 1 GiB)."""
    nbytes = 1 << 30
    src = torch.empty(nbytes // 8, dtype=torch.int64, device="cuda").fill_(7)
    dst = torch.empty_like(src)
    for _ in range(args.warmup):
        dst.copy_(src)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        dst.copy_(src)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / args.steps
    # the write ceiling the DNF write-out is compared with: torch's fill of a
    # buffer as large as the 16 C1 DNF vectors (8 GiB), timed with HIP events
    big = torch.empty(8 << 30, dtype=torch.uint8, device="cuda")
    stream = torch.cuda.current_stream()
    big.fill_(1)
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record(stream)
    for _ in range(args.steps):
        big.fill_(1)
    b.record(stream)
    torch.cuda.synchronize()
    fill_ms = a.elapsed_time(b) / args.steps
    return {"metric": "copy bandwidth (counter calibration)", "value": 2 * nbytes / (ms / 1e3) / 1e9,
            "unit": "GB/s", "ms_per_step": ms, "dtype": "u64",
            "config": {"workload": "device copy of 1 GiB (reads 1 GiB, writes 1 GiB)", "bytes": nbytes},
            "fill_8GiB": {"ms": fill_ms, "gb_per_s": (8 << 30) / (fill_ms / 1e3) / 1e9}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="c1",
                    choices=["c0", "c1", "c3", "c4", "posets", "theories", "unlabeled", "copy", "valu"])
    ap.add_argument("--posets-n", type=int, default=11, help="posets: bounded posets on n elements")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-c3", action="store_true", help="c1: leave out the 4096-formula batch block")
    ap.add_argument("--requests", type=int, default=20000, help="c4: requests in the timed run")
    ap.add_argument("--sat-requests", type=int, default=1000, help="c4: requests of the burst run (the overload run takes 4 x as many)")
    ap.add_argument("--loads", default="0.3,0.6,0.9", help="c4: arrival rates as fractions of saturation")
    ap.add_argument("--slice-words", type=float, default=2.5e11, help="c4: clause-word work per slice")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: a formula's valuation space would be cut into contiguous "
              "index ranges, one per GPU, with a single 8-byte sum per count; only the one-GPU kernel "
              "is measured here.", file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a HIP device", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    from paper_1310_6978_amd import fbg
    if args.workload == "c1":
        res = bench_c1(args, torch, fbg)
        if not args.no_c3:
            res["c3"] = c3_block(args, torch, fbg)
    elif args.workload == "c0":
        res = bench_c0(args, torch, fbg)
    elif args.workload == "c3":
        res = bench_c3(args, torch, fbg)
    elif args.workload == "c4":
        res = bench_c4(args, torch, fbg)
    elif args.workload == "posets":
        res = bench_posets(args, torch, fbg)
    elif args.workload == "theories":
        res = bench_theories(args, torch, fbg)
    elif args.workload == "unlabeled":
        res = bench_unlabeled(args, torch, fbg)
    elif args.workload == "valu":
        res = bench_valu(args, torch)
    else:
        res = bench_copy(args, torch)
    out = {"metric": res.pop("metric"), "value": res.pop("value"), "unit": res.pop("unit"), "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": res.pop("ms_per_step"),
           "higher_is_better": res.pop("higher_is_better", True), "scaling": "weak", "vs_baseline": None,
           "dtype": res.pop("dtype"),
           "data": "synthetic (seeded SplitMix64 formulas)", "config": res.pop("config")}
    out.update(res)
    print(json.dumps(out))


if __name__ == "__main__":
    main()

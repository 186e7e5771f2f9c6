"""Serving loop: admission logic on the CPU; on the GPU, every request's count
in a mixed, continuously batched run equals its count alone and the oracle's
(the tolerance is zero: counts are integers)."""

import random

import pytest

import oracle
import workloads
from workloads.serving import request_stream


def test_admission_budget():
    from paper_1310_6978_amd.serve import Admission
    a = Admission(100)
    assert a.try_reserve(60)
    assert not a.try_reserve(50)     # would exceed the arena: wait
    assert a.try_reserve(40)
    a.release(60)
    assert a.try_reserve(50)
    with pytest.raises(ValueError):
        a.try_reserve(101)           # never fits


def test_request_stream_is_seeded_and_poisson():
    a = request_stream(400, 100.0, seed=3)
    b = request_stream(400, 100.0, seed=3)
    assert [r["text"] for r in a] == [r["text"] for r in b]
    assert all(x["arrival"] <= y["arrival"] for x, y in zip(a, a[1:]))
    mean_gap = a[-1]["arrival"] / len(a)
    assert 0.007 < mean_gap < 0.013          # rate 100/s
    kinds = [r["kind"] for r in a]
    assert 0.05 < sum(k != "3cnf" for k in kinds) / len(kinds) < 0.16
    assert all(12 <= r["n"] <= 36 for r in a if r["kind"] == "3cnf")
    assert request_stream(5, 0.0)[-1]["arrival"] == 0.0


def test_deferred_release_runs_once_across_threads():
    # compile threads and the loop's thread sweep the deferred-release list
    # together; every entry must be released exactly once
    import collections
    import threading
    import time
    from paper_1310_6978_amd import fbg

    class Done:
        def query(self):
            return True

    calls = collections.Counter()
    lock = threading.Lock()

    def release(i):
        time.sleep(0)                # let another thread run mid-release
        with lock:
            calls[i] += 1

    with fbg._grave_lock:
        for i in range(3000):
            fbg._graveyard.append((lambda i=i: release(i), [Done()], ()))
    start = threading.Barrier(8)

    def work():
        start.wait()
        for _ in range(20):
            fbg._sweep()

    threads = [threading.Thread(target=work) for _ in range(8)]
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    assert not fbg._graveyard
    assert calls == collections.Counter(range(3000))


@pytest.mark.gpu
def test_mixed_requests_match_alone_and_oracle():
    import numpy as np
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU test needs a HIP device")
    from paper_1310_6978_amd import fbg
    from paper_1310_6978_amd.serve import ServeLoop
    reqs = request_stream(120, 2000.0, seed=11, n_lo=12, n_hi=24, theory_share=0.0)
    rng = random.Random(1)
    # a few theory requests of the affordable kinds, repeated (resident programs)
    for i in range(12):
        text, n = workloads.triangle_free(6) if i % 2 else workloads.permutation_matrices(4)
        reqs.append({"id": 120 + i, "arrival": rng.random() * 0.05, "kind": "theory", "text": text, "n": n})
    loop = ServeLoop(words_per_lane=16, slice_words=2e8, max_active=32)
    res = loop.run(reqs, realtime=True)
    loop.close()
    assert res["requests"] == len(reqs)
    for r in reqs:
        want = oracle.count(r["text"], r["n"])
        assert res["counts"][r["id"]] == want, r["id"]
    # alone: one program, one launch
    for r in reqs[:20]:
        p = fbg.Program(r["text"], r["n"])
        alone = int(fbg.count(p).cpu().numpy().view(np.uint64)[0])
        assert alone == res["counts"][r["id"]]
    assert res["cache_hits"] >= 10          # the repeated theories stayed resident
    assert res["latency_p99_ms"] >= res["latency_p50_ms"] > 0


@pytest.mark.gpu
def test_tiny_arena_still_serves_everything():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU test needs a HIP device")
    from paper_1310_6978_amd import fbg
    from paper_1310_6978_amd.serve import ServeLoop, program_bytes
    reqs = request_stream(30, 0.0, seed=5, n_lo=12, n_hi=20, theory_share=0.0)
    # room for a handful of requests at a time: admission has to wait
    loop = ServeLoop(words_per_lane=8, slice_words=1e7, arena_bytes=2 * 200000, max_active=8)
    res = loop.run(reqs, realtime=False)
    loop.close()
    for r in reqs:
        assert res["counts"][r["id"]] == oracle.count(r["text"], r["n"])
    # admission bound the number of requests held at once, so the 30
    # requests needed several slices
    smallest = min(program_bytes(fbg.Program(r["text"], r["n"]).info) + 8 for r in reqs)
    assert 1 <= res["peak_admitted"] <= (2 * 200000) // smallest < 30
    assert res["slices"] >= -(-30 // res["peak_admitted"])

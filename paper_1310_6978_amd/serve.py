"""Continuous-batching serving loop for model-counting requests on one GPU.

Requests arrive over time (Poisson arrivals in the benchmark).  Each request
is compiled on admission (programs of repeated texts stay resident), reserves
its device bytes against an arena budget, and gets a count slot.  The GPU runs
a sequence of *slices*: one persistent batched launch (fbg_server_launch) over
work items taken round-robin from every admitted request, a bounded amount of
work per slice, on alternating streams.  A request that arrives while slices
are running joins the next slice as soon as it is admitted, so its work
overlaps on the device with the work of the requests already there; large
requests are spread over many slices while small ones finish in one.  A
request completes when every slice that carried its tiles has finished; its
count is then read from its slot.

Counts are exact: a request's count is the same alone and in any mix (the
items of one slot add up the same tiles whatever else shares the launch).
"""

import collections
import hashlib
import time

import numpy as np

from . import fbg


class Admission:
    """Reservation of device bytes against a fixed arena budget, first come
    first served."""

    def __init__(self, budget_bytes):
        self.budget = int(budget_bytes)
        self.used = 0

    def try_reserve(self, nbytes):
        nbytes = int(nbytes)
        if nbytes > self.budget:
            raise ValueError("request needs %d bytes, arena holds %d" % (nbytes, self.budget))
        if self.used + nbytes > self.budget:
            return False
        self.used += nbytes
        return True

    def release(self, nbytes):
        self.used -= int(nbytes)
        assert self.used >= 0


class ProgramCache:
    """Compiled programs kept resident, keyed by the hash of the text and n;
    least recently used entries beyond `capacity` are freed.  `flags` are the
    compile flags (the loop encodes only the server's tiling)."""

    def __init__(self, capacity=64, flags=0):
        self.capacity = capacity
        self.flags = int(flags)
        self.entries = collections.OrderedDict()
        self.hits = 0
        self.misses = 0

    def get(self, text, n):
        key = (hashlib.sha1(text.encode()).hexdigest(), n)
        p = self.entries.get(key)
        if p is not None:
            self.entries.move_to_end(key)
            self.hits += 1
            return p
        self.misses += 1
        p = fbg.Program(text, n, self.flags)
        self.entries[key] = p
        while len(self.entries) > self.capacity:
            self.entries.popitem(last=False)
        return p


def program_bytes(info):
    """Device bytes a compiled program holds (its code arena block)."""
    return int(info["code_bytes"])


class _Req:
    __slots__ = ("rid", "arrival", "n", "text", "kind", "prog", "ntiles", "nins", "next_tile", "slot", "deps",
                 "bytes", "admitted_at", "done_at", "count")

    def __init__(self, r):
        self.rid = r["id"]
        self.arrival = r["arrival"]
        self.n = r["n"]
        self.text = r["text"]
        self.kind = r.get("kind", "")
        self.prog = None
        self.deps = []
        self.next_tile = 0
        self.count = None


class ServeLoop:
    """The serving loop.  `slice_words` bounds the clause-word work of one
    slice (a clause applied to one 32-bit word is one unit): a longer slice
    spreads the host's work per launch over more requests, a shorter one lets
    a small request that arrives behind a large one finish sooner.  `cofactor`
    runs the slices with the uniform-cofactor test (a tile on which a clause
    made only of tile literals is false is skipped); counts are the same
    either way."""

    def __init__(self, words_per_lane=16, slice_words=2.5e11, arena_bytes=4 << 30, max_active=256,
                 max_items=16384, nstreams=2, cache_capacity=64, cofactor=True):
        import torch
        self.torch = torch
        self.W = int(words_per_lane)
        self.slice_words = float(slice_words)
        self.admission = Admission(arena_bytes)
        self.max_active = int(max_active)
        self.max_items = int(max_items)
        self.max_requests_per_slice = max(1, int(max_items) // 4)
        self.streams = [torch.cuda.Stream() for _ in range(nstreams)]
        self.copy_stream = torch.cuda.Stream()
        self.server = fbg.Server(max_programs=max_active, max_items=max_items, words_per_lane=self.W,
                                 nbuf=2 * nstreams + 2, cofactor=cofactor)
        self.cache = ProgramCache(cache_capacity, flags=fbg.compile_wpl(self.W))

    def run(self, requests, realtime=True, log=None):
        torch = self.torch
        reqs = [_Req(r) for r in sorted(requests, key=lambda r: r["arrival"])]
        nslots = max(r.rid for r in reqs) + 1
        counts = torch.zeros(nslots, dtype=torch.int64, device="cuda")
        host_counts = torch.zeros(nslots, dtype=torch.int64).pin_memory()
        torch.cuda.synchronize()
        pending = collections.deque(reqs)
        waiting = collections.deque()
        active = []                       # admitted, tiles left to issue
        issued = []                       # all tiles issued, slices in flight
        inflight = collections.deque()    # (end event, timing start event, stream index)
        done = []
        slice_ms = []
        peak = 0                          # most requests admitted at once
        t0 = time.perf_counter()
        k = 0
        last_log = 0.0

        def now():
            return time.perf_counter() - t0

        while pending or waiting or active or issued:
            t = now()
            while pending and (not realtime or pending[0].arrival <= t):
                waiting.append(pending.popleft())
            # ---- admission: compile, reserve bytes, take a slot
            while waiting and len(active) + len(issued) < self.max_active:
                r = waiting[0]
                if r.prog is None:
                    r.prog = self.cache.get(r.text, r.n)
                    r.nins = max(1, r.prog.info["n_instr"])
                    r.ntiles = fbg.program_tiles(r.prog, self.W)
                    r.bytes = program_bytes(r.prog.info) + 8
                if not self.admission.try_reserve(r.bytes):
                    break
                waiting.popleft()
                r.admitted_at = now()
                r.slot = r.rid
                active.append(r)
                peak = max(peak, len(active) + len(issued))
            # ---- one slice over the admitted requests
            launched = False
            if active and len(inflight) < len(self.streams):
                items, progs, local = [], [], {}
                share = self.slice_words / len(active)
                words_per_tile = 64 * self.W
                still = []
                for r in active:
                    if len(items) >= self.max_requests_per_slice or len(progs) >= self.max_active:
                        still.append(r)
                        continue
                    chunk = max(1, int(share // (r.nins * words_per_tile)))
                    t1 = min(r.ntiles, r.next_tile + chunk)
                    if id(r.prog) not in local:
                        local[id(r.prog)] = len(progs)
                        progs.append(r.prog)
                    # one item per request; the server cuts long items into
                    # pieces so that the slice occupies every compute unit
                    items.append((local[id(r.prog)], r.slot, r.next_tile, t1))
                    r.next_tile = t1
                    (issued if t1 >= r.ntiles else still).append(r)
                    r.deps.append(k)
                active = still
                s = self.streams[k % len(self.streams)]
                start = torch.cuda.Event(enable_timing=True)
                end = torch.cuda.Event(enable_timing=True)
                start.record(s)
                self.server.launch(progs, items, counts, stream=s)
                end.record(s)
                inflight.append((k, start, end))
                k += 1
                launched = True
            # ---- retire finished slices, complete requests
            finished = set()
            while inflight and inflight[0][2].query():
                kk, a, b = inflight.popleft()
                slice_ms.append(a.elapsed_time(b))
                finished.add(kk)
            oldest = inflight[0][0] if inflight else k
            ready = [r for r in issued if max(r.deps) < oldest]
            if ready:
                # read back only the slots from the first ready one to the last
                lo = min(r.slot for r in ready)
                hi = max(r.slot for r in ready) + 1
                with torch.cuda.stream(self.copy_stream):
                    host_counts[lo:hi].copy_(counts[lo:hi], non_blocking=True)
                self.copy_stream.synchronize()
                hc = host_counts.numpy().view(np.uint64)
                tt = now()
                for r in ready:
                    r.count = int(hc[r.slot])
                    r.done_at = tt
                    self.admission.release(r.bytes)
                    r.prog = None
                    done.append(r)
                issued = [r for r in issued if r.count is None]
            if log is not None and now() - last_log >= 10.0:
                last_log = now()
                log("serve: %.1f s, %d of %d requests done, %d slices, %d waiting, %d active"
                    % (last_log, len(done), len(reqs), k, len(waiting), len(active) + len(issued)))
            if not launched and not ready:
                if inflight and (not pending or pending[0].arrival > now()):
                    inflight[0][2].synchronize()
                elif not inflight and pending and realtime and not waiting and not active:
                    time.sleep(max(0.0, min(0.0005, pending[0].arrival - now())))
        wall = now()
        torch.cuda.synchronize()
        lat = np.array([r.done_at - r.arrival for r in done])
        vals = float(sum(2.0 ** r.n for r in done))
        return {
            "requests": len(done),
            "wall_s": wall,
            "valuations_per_s": vals / wall if wall > 0 else 0.0,
            "requests_per_s": len(done) / wall if wall > 0 else 0.0,
            "latency_p50_ms": float(np.percentile(lat, 50) * 1e3) if len(lat) else 0.0,
            "latency_p99_ms": float(np.percentile(lat, 99) * 1e3) if len(lat) else 0.0,
            "latency_mean_ms": float(lat.mean() * 1e3) if len(lat) else 0.0,
            "slices": k,
            "peak_admitted": peak,
            "gpu_busy": float(sum(slice_ms) / 1e3 / wall) if wall > 0 else 0.0,
            "cache_hits": self.cache.hits,
            "cache_misses": self.cache.misses,
            "counts": {r.rid: r.count for r in done},
        }

    def close(self):
        self.server.free()

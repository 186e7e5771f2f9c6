"""Autotuner for the evaluator's tiling.

The evaluator's cost per clause per tile is a fixed scalar part (instruction
fetch, the lane and tile parts of the literal set) plus one VALU operation
per word, so more words per lane amortise the fixed part, while fewer words
per lane give small valuation spaces more tiles (and so more waves).  For a
program with clauses the uniform-cofactor test is a second dimension: it
skips every tile on which a clause made only of tile variables is false,
which pays where such clauses kill most tiles (the theories) and costs a
little where they do not.  The tuner times fbg_count on the candidate
tilings, with and without the test, with HIP events, keeps the fastest, and
caches the choice per (device architecture, n, program-size bucket,
clause-only or not) in a JSON file (FBG_TUNE_CACHE, default
~/.cache/fbg/tune.json).  It then makes the choice the program's default
through fbg_program_set_tuning (counts, DNF vectors and enumerations then use
it; results are the same either way).
"""

import hashlib
import json
import math
import os

from . import fbg

CANDIDATES = (4, 8, 16, 32)


def _cache_path():
    return os.environ.get("FBG_TUNE_CACHE", os.path.join(os.path.expanduser("~"), ".cache", "fbg", "tune.json"))


def _arch():
    import torch
    try:
        return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    except Exception:
        return "unknown"


def key_of(prog):
    info = prog.info
    size = max(1, int(info["n_instr"]))
    general = int(info["n_instr"]) > int(info["n_clause_instr"])
    return "%s|n=%d|L=%d|gen=%d" % (_arch(), prog.n, int(math.log2(size)), int(general))


class Tuner:
    def __init__(self, path=None, candidates=CANDIDATES, reps=3):
        self.path = path or _cache_path()
        self.candidates = tuple(candidates)
        self.reps = reps
        self.table = {}
        self.last_key = None   # cache key of the last tune_batch
        if os.path.exists(self.path):
            try:
                with open(self.path) as f:
                    self.table = json.load(f)
            except (OSError, ValueError):
                self.table = {}

    def measure(self, prog):
        """{(words_per_lane, cofactor): ms} for one count of `prog` at each
        candidate (the cofactor only for programs with clauses)."""
        import torch
        out = torch.empty(1, dtype=torch.int64, device="cuda")
        res = {}
        cofs = (False, True) if int(prog.info["n_clause_instr"]) > 0 else (False,)
        for w in self.candidates:
            for cof in cofs:
                try:
                    fbg.count(prog, out=out, words_per_lane=w, cofactor=cof)  # warm-up
                except fbg.FbgError:
                    break  # registers do not fit at this tiling
                torch.cuda.synchronize()
                a = torch.cuda.Event(enable_timing=True)
                b = torch.cuda.Event(enable_timing=True)
                a.record()
                for _ in range(self.reps):
                    fbg.count(prog, out=out, words_per_lane=w, cofactor=cof)
                b.record()
                torch.cuda.synchronize()
                res[(w, cof)] = a.elapsed_time(b) / self.reps
        return res

    def apply(self, prog, save=True):
        """Set the program's default tiling and cofactor choice from the cache,
        measuring on a miss.  Returns the chosen words per lane."""
        k = key_of(prog)
        entry = self.table.get(k, {})
        w = entry.get("words_per_lane")
        cof = bool(entry.get("cofactor", False))
        if w is None:
            times = self.measure(prog)
            w, cof = min(times, key=times.get)
            self.table[k] = {"words_per_lane": w, "cofactor": cof,
                             "ms": {"%d%s" % (x, "c" if c else ""): t for (x, c), t in times.items()}}
            if save:
                self.save()
        prog.set_tuning(w, cofactor=cof)
        return w

    def tune_batch(self, progs, candidates=(0, 4, 8, 16, 32), save=True):
        """Words per lane for a batch (0: each plan takes the tiling of its
        largest program).  Times one batched count per candidate, caches the
        fastest per (architecture, multiset of program keys) and returns it."""
        import torch
        digest = hashlib.sha1("\n".join(sorted(key_of(p) for p in progs)).encode()).hexdigest()[:16]
        k = "%s|batch=%s|%d" % (_arch(), digest, len(progs))
        self.last_key = k
        hit = self.table.get(k, {}).get("words_per_lane")
        if hit is not None:
            return hit
        out = torch.empty(len(progs), dtype=torch.int64, device="cuda")
        times = {}
        for w in candidates:
            try:
                b = fbg.Batch(progs, words_per_lane=w)
            except fbg.FbgError:
                continue  # registers do not fit at this tiling
            b.count(out=out)  # warm-up
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(self.reps):
                b.count(out=out)
            e1.record()
            torch.cuda.synchronize()
            times[w] = e0.elapsed_time(e1) / self.reps
            b.free()
        w = min(times, key=times.get)
        self.table[k] = {"words_per_lane": w, "ms": times}
        if save:
            self.save()
        return w

    def save(self):
        d = os.path.dirname(self.path)
        if d:
            os.makedirs(d, exist_ok=True)
        tmp = self.path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(self.table, f, indent=1, sort_keys=True)
        os.replace(tmp, self.path)

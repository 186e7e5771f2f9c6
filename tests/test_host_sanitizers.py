"""The host compiler and encoder under AddressSanitizer and
UndefinedBehaviorSanitizer (CPU only): a driver built from compiler.cpp alone
with g++ -fsanitize=address,undefined compiles random formulas, encodes them
at every tiling, lists them and emulates them; every emulated DNF vector must
equal the oracle's, and random malformed text (a parser fuzz) must end in a
parse error, never in a sanitizer report."""

import os
import random
import shutil
import subprocess

import numpy as np
import pytest

import oracle
import workloads
from tests.formula_gen import many_registers, random_cnf, random_program

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1310_6978_amd", "csrc")


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not found")
    out = str(tmp_path_factory.mktemp("sanitize") / "driver")
    cmd = [gxx, "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-I", CSRC, "-I", os.path.join(ROOT, "include"),
           os.path.join(ROOT, "tests", "sanitize", "driver.cpp"), os.path.join(CSRC, "compiler.cpp"),
           "-lpthread", "-o", out]
    subprocess.check_call(cmd)
    return out


def run(driver, cases):
    data = b"".join(b"%d %d\n" % (n, len(t.encode())) + t.encode() for t, n in cases)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:halt_on_error=1:detect_stack_use_after_return=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    env.pop("LD_PRELOAD", None)
    r = subprocess.run([driver], input=data, capture_output=True, env=env, timeout=600)
    assert r.returncode == 0, r.stderr.decode(errors="replace")[-4000:]
    assert b"runtime error" not in r.stderr and b"AddressSanitizer" not in r.stderr, r.stderr[-4000:]
    return r.stdout.decode().splitlines()


def test_random_formulas_under_sanitizers(driver):
    rng = random.Random(77)
    cases = []
    for k in range(40):
        n = rng.choice([0, 1, 3, 5, 6, 9, 12, 13, 16])
        if k % 4 == 0:
            text = random_cnf(rng, max(n, 3), rng.randrange(1, 40))
            n = max(n, 3)
        elif k % 4 == 1:
            text = many_registers(rng, max(n, 6), rng.choice([3, 6, 10]))
            n = max(n, 6)
        else:
            _, text = random_program(rng, max(n, 1))
            n = max(n, 1)
        cases.append((text, n))
    cases.append(workloads.random_dag(14, 600, 3))
    cases.append(workloads.equivalence_relations(5))
    lines = run(driver, cases)
    it = iter(lines)
    for text, n in cases:
        want = oracle.dnf(text, n)
        for _ in range(12):            # 6 tilings x 2 variants
            f = next(it).split()
            assert f[0] != "ERR", (f, text[:200])
            got = np.array([int(x, 16) for x in f[2:]], dtype=np.uint64)
            assert np.array_equal(got, want), (f[:2], text[:200])


def test_exchanged_variables_give_the_xcd_local_layout(driver):
    """The second encoding of the batched DNF write-out: the program with its
    variables renamed, emulated at 32 words per lane, and each word (tile t,
    word i, lane l) put where the write-out kernel stores it (piece p(t) or
    p(t) + 8 by i >> 4, 1 KiB unit (i >> 2) & 3, 16-byte group of lane l,
    word i & 3) gives the DNF vector.  Clause-only formulas (the write-out's
    programs) and general ones, n = 21 and 22."""
    rng = random.Random(2101)
    cases = [workloads.random_3cnf(21, 89, 4), workloads.random_3cnf(22, 94, 5),
             (random_cnf(rng, 22, 60), 22), (random_program(rng, 21)[1], 21)]
    lines = run(driver, cases)
    xs = [l for l in lines if l.startswith("X")]
    assert len(xs) == len(cases)
    for (text, n), line in zip(cases, xs):
        got = np.array([int(x, 16) for x in line.split()[1:]], dtype=np.uint64)
        assert np.array_equal(got, oracle.dnf(text, n)), text[:200]


def test_parser_fuzz_under_sanitizers(driver):
    rng = random.Random(5)
    alphabet = "x0123456789 ~&^|()=\n;#abt_"
    cases = []
    for _ in range(300):
        text = "".join(rng.choice(alphabet) for _ in range(rng.randrange(0, 80)))
        cases.append((text, rng.randrange(0, 12)))
    # deep nesting and long operator chains
    cases.append(("(" * 3000 + "x0" + ")" * 3000, 1))
    cases.append((" & ".join("x%d" % (i % 7) for i in range(5000)), 7))
    cases.append(("~" * 2000 + "x1", 2))
    lines = run(driver, cases)
    assert len(lines) >= len(cases)

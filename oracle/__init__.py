"""CPU oracle for the free-Boolean-generator path -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The product library never loads it.

The C source (``oracle.c``) evaluates a formula valuation by valuation
(Proposition 2.2: bit mu of t(b_1..b_n) is t at mu) and, as a cross-check, by
the blocked bitwise evaluation of Section 2.3.  This module only marshals
arguments through ctypes.
"""

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(verbose=False):
    """Compile oracle.c with gcc into liboracle.so (always rebuilds)."""
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-pthread", "-Wall", "-Wextra",
           "-o", _LIB + ".tmp", _SRC]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build()
    lib = ctypes.CDLL(_LIB)
    u64p = ctypes.POINTER(ctypes.c_uint64)
    lib.orc_error.restype = ctypes.c_char_p
    lib.orc_count.argtypes = [ctypes.c_char_p, ctypes.c_int, ctypes.c_int, u64p]
    lib.orc_dnf.argtypes = [ctypes.c_char_p, ctypes.c_int, ctypes.c_int, u64p, ctypes.c_uint64]
    lib.orc_models.argtypes = [ctypes.c_char_p, ctypes.c_int, ctypes.c_int, u64p, ctypes.c_uint64, u64p]
    lib.orc_eval_at.argtypes = [ctypes.c_char_p, ctypes.c_int, u64p, ctypes.c_uint64,
                                ctypes.POINTER(ctypes.c_uint8)]
    lib.orc_count_range.argtypes = [ctypes.c_char_p, ctypes.c_int, ctypes.c_uint64, ctypes.c_uint64,
                                    ctypes.c_int, u64p]
    lib.orc_describe.argtypes = [ctypes.c_char_p] + [ctypes.POINTER(ctypes.c_int)] * 3
    lib.orc_bitpar_count.argtypes = [ctypes.c_char_p, ctypes.c_int, ctypes.c_int, u64p]
    lib.orc_bitpar_dnf.argtypes = [ctypes.c_char_p, ctypes.c_int, ctypes.c_int, u64p, ctypes.c_uint64]
    for f in ("orc_count", "orc_count_range", "orc_dnf", "orc_models", "orc_eval_at", "orc_describe",
              "orc_bitpar_count", "orc_bitpar_dnf"):
        getattr(lib, f).restype = ctypes.c_int
    _lib = lib
    return lib


class OracleError(RuntimeError):
    pass


def _check(rc):
    if rc != 0:
        raise OracleError(_load().orc_error().decode())


def _b(src):
    return src.encode() if isinstance(src, str) else src


def _u64p(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))


def dnf_words(n):
    return 1 if n < 6 else 1 << (n - 6)


def count(src, n, threads=0):
    """Number of models: valuations mu in 2^n with t(mu) = 1."""
    out = ctypes.c_uint64(0)
    _check(_load().orc_count(_b(src), n, threads, ctypes.byref(out)))
    return out.value


def count_range(src, n, lo, hi, threads=0):
    """Number of models mu with lo <= mu < hi."""
    out = ctypes.c_uint64(0)
    _check(_load().orc_count_range(_b(src), n, int(lo), int(hi), threads, ctypes.byref(out)))
    return out.value


def dnf(src, n, threads=0):
    """The 2^n-bit DNF vector as uint64 words (bit mu&63 of word mu>>6)."""
    out = np.zeros(dnf_words(n), dtype=np.uint64)
    _check(_load().orc_dnf(_b(src), n, threads, _u64p(out), out.size))
    return out


def models(src, n, cap=None, threads=0):
    """(ascending model indices, at most ``cap`` of them; total model count)."""
    if cap is None:
        cap = count(src, n, threads)
    buf = np.zeros(max(int(cap), 1), dtype=np.uint64)
    total = ctypes.c_uint64(0)
    _check(_load().orc_models(_b(src), n, threads, _u64p(buf), int(cap), ctypes.byref(total)))
    return buf[: min(int(cap), total.value)].copy(), total.value


def eval_at(src, n, idx):
    """t(mu) for each mu in ``idx`` as a uint8 array of 0/1."""
    idx = np.ascontiguousarray(np.asarray(idx, dtype=np.uint64))
    out = np.zeros(idx.size, dtype=np.uint8)
    _check(_load().orc_eval_at(_b(src), n, _u64p(idx), idx.size,
                               out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))))
    return out


def describe(src):
    """(1 + largest variable index, number of assertions, number of temporaries)."""
    a, b, c = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    _check(_load().orc_describe(_b(src), ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
    return a.value, b.value, c.value


def bitpar_count(src, n, threads=0):
    """Model count by the blocked evaluation of Section 2.3 (64-bit blocks)."""
    out = ctypes.c_uint64(0)
    _check(_load().orc_bitpar_count(_b(src), n, threads, ctypes.byref(out)))
    return out.value


def bitpar_dnf(src, n, threads=0):
    """DNF vector by the blocked evaluation of Section 2.3."""
    out = np.zeros(dnf_words(n), dtype=np.uint64)
    _check(_load().orc_bitpar_dnf(_b(src), n, threads, _u64p(out), out.size))
    return out


def orbits(src, n, perms, threads=0):
    """(number of orbits of the models under the permutations of the
    letters in ``perms`` -- a whole group, one row per element; number of
    models).  With the group of all relabelings of a domain this is the
    number of non-isomorphic models (Section 3.2, kappa)."""
    perms = np.ascontiguousarray(np.asarray(perms, dtype=np.int32))
    if perms.ndim != 2 or perms.shape[1] != n:
        raise OracleError("perms must have shape (group size, n)")
    lib = _load()
    lib.orc_orbits.argtypes = [ctypes.c_char_p, ctypes.c_int, ctypes.POINTER(ctypes.c_int32), ctypes.c_int,
                               ctypes.c_int, ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(ctypes.c_uint64)]
    lib.orc_orbits.restype = ctypes.c_int
    o, t = ctypes.c_uint64(0), ctypes.c_uint64(0)
    _check(lib.orc_orbits(_b(src), n, perms.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), perms.shape[0],
                          threads, ctypes.byref(o), ctypes.byref(t)))
    return o.value, t.value

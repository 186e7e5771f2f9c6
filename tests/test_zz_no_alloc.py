"""The entry point that allocates nothing (fbg_enumerate_noalloc), through
the C ABI, against the allocating fbg_enumerate and the oracle: two calls in
a row on one device, the second with a smaller input, so that whatever the
first call left in the shared static scratch cannot leak into the second."""

import ctypes

import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def F():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")
    from paper_1310_6978_amd import fbg
    return fbg


def host(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy().view(np.uint64)


def both(F, p, cap):
    """(models, total) from fbg_enumerate_noalloc and from fbg_enumerate."""
    import torch
    out = torch.full((max(cap, 1),), -1, dtype=torch.int64, device="cuda")[:cap]
    tot = torch.full((1,), -1, dtype=torch.int64, device="cuda")
    F.enumerate_models_noalloc(p, out, tot)
    t_na = int(host(tot)[0])
    m_na = host(out)[:min(t_na, cap)].copy()
    ref, rt = F.enumerate_models(p, cap)
    t_ref = int(host(rt)[0])
    m_ref = host(ref)[:min(t_ref, cap)].copy()
    return (m_na, t_na), (m_ref, t_ref)


def test_two_calls_second_smaller(F):
    big_text, big_n = workloads.equivalence_relations(7)      # 21 letters, 877 models
    small_text, small_n = workloads.equivalence_relations(5)  # 10 letters, 52 models
    big = F.Program(big_text, big_n)
    small = F.Program(small_text, small_n)
    want_big, want_big_c = oracle.models(big_text, big_n)
    want_small, want_small_c = oracle.models(small_text, small_n)
    print("noalloc: k=7 equivalence then k=5", flush=True)
    (m1, t1), (r1, rt1) = both(F, big, 1000)
    assert t1 == rt1 == want_big_c == 877
    assert np.array_equal(m1, r1) and np.array_equal(m1, want_big)
    (m2, t2), (r2, rt2) = both(F, small, 1000)
    assert t2 == rt2 == want_small_c == 52
    assert np.array_equal(m2, r2) and np.array_equal(m2, want_small)


def test_truncation_and_zero_capacity(F):
    text, n = workloads.triangle_free(6)  # 15 letters, 5789 models
    p = F.Program(text, n)
    want, wc = oracle.models(text, n)
    print("noalloc: triangle-free k=6, capacities 100 and 0", flush=True)
    (m, t), (r, rt) = both(F, p, 100)
    assert t == rt == wc == 5789 and np.array_equal(m, r) and np.array_equal(m, want[:100])
    (m, t), (r, rt) = both(F, p, 0)
    assert t == rt == wc and m.size == 0


def test_larger_than_the_scratch_is_refused(F):
    import torch
    p = F.Program("x0 | x39", 40)       # 2^24 tiles at 32 words per lane
    out = torch.empty(1, dtype=torch.int64, device="cuda")
    tot = torch.empty(1, dtype=torch.int64, device="cuda")
    st = F.lib.fbg_enumerate_noalloc(p.handle, ctypes.c_void_p(out.data_ptr()), 1,
                                     ctypes.c_void_p(tot.data_ptr()), ctypes.c_void_p(0))
    assert st == F.FBG_E_RANGE
    assert "static" in F.lib.fbg_last_error().decode()
    # the device is still usable and the next call exact
    small_text, small_n = workloads.equivalence_relations(4)  # 6 letters, 15 models
    (m, t), (r, rt) = both(F, F.Program(small_text, small_n), 64)
    assert t == rt == 15 and np.array_equal(m, r)

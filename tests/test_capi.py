"""The C-ABI library loads and exports every symbol include/fbg.h declares;
calls that need a device fail loudly without one."""

import ctypes
import os
import re

import pytest

from paper_1310_6978_amd import fbg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "fbg.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fbg_[a-z_0-9]+)\s*\(", text)))


def test_every_declared_symbol_is_exported():
    lib = ctypes.CDLL(fbg.LIB_PATH)
    names = declared_symbols()
    assert len(names) >= 15
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(fbg.EXPORTED)


def test_one_hip_runtime_in_the_process():
    # libfbg must use torch's HIP runtime, not load a second one
    maps = open("/proc/self/maps").read()
    libs = set(line.split()[-1] for line in maps.splitlines() if "libamdhip64" in line)
    assert len(libs) == 1, libs


def test_version():
    assert "gfx950" in fbg.version()


def test_library_is_the_in_tree_build():
    assert os.path.dirname(fbg.LIB_PATH) == os.path.join(ROOT, "paper_1310_6978_amd")


def test_device_calls_fail_without_device():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    p = fbg.Program("x0 | x1", 4)
    st = fbg.lib.fbg_count(p.handle, ctypes.c_void_p(8), ctypes.c_void_p(0))
    assert st == fbg.FBG_E_DEVICE
    assert "without a HIP device" in fbg.lib.fbg_last_error().decode()


def test_null_arguments():
    assert fbg.lib.fbg_count(None, None, None) == fbg.FBG_E_INVAL
    assert fbg.lib.fbg_program_info(None, None) == fbg.FBG_E_INVAL
    assert fbg.lib.fbg_program_get_info(None, None) == fbg.FBG_E_INVAL
    out = ctypes.c_void_p()
    assert fbg.lib.fbg_compile(None, 3, 0, ctypes.byref(out)) == fbg.FBG_E_INVAL
    assert fbg.lib.fbg_compile(b"x0", 3, 0x40, ctypes.byref(out)) == fbg.FBG_E_INVAL
    assert "flags" in fbg.lib.fbg_last_error().decode()
    fbg.lib.fbg_program_free(None)
    fbg.lib.fbg_batch_free(None)


def test_program_info_through_the_c_abi():
    """fbg_program_info fills the struct in full: n, L_2in, L_valu, tiling."""
    info = fbg.ProgramInfo()
    p = fbg.Program("a = x0 & x1\na ^ x2\nx3 | ~x4", 7)
    assert fbg.lib.fbg_program_info(p.handle, ctypes.byref(info)) == fbg.FBG_OK
    assert info.n_vars == 7 and info.l2in == 4 and info.dnf_words == 2
    assert info.words_per_lane in (1, 2, 4, 8, 16, 32)
    # one clause (x3 | ~x4) and a general part: at least one VALU
    # instruction per slice for each of its operations
    assert 2.0 <= info.l_valu < 40.0
    old = fbg.ProgramInfo()
    assert fbg.lib.fbg_program_get_info(p.handle, ctypes.byref(old)) == fbg.FBG_OK
    assert old.l_valu == info.l_valu and old.l2in == info.l2in
    assert p.info["l_valu"] == info.l_valu


def test_compile_only_some_tilings():
    """FBG_COMPILE_WPL: the program is encoded for the tilings asked for; the
    results there are those of a full compile, every other tiling is refused."""
    text, n = "a = x0 & x1\nb = a ^ x5\nb | (x2 & ~x7)\nx3 | ~x4 | x6", 8
    full = fbg.Program(text, n)
    part = fbg.Program(text, n, fbg.compile_wpl(4, 16))
    assert fbg.compile_wpl(1, 2, 4, 8, 16, 32) == fbg.COMPILE_WPL_MASK
    with pytest.raises(ValueError):
        fbg.compile_wpl(3)
    assert part.info["words_per_lane"] in (4, 16)
    assert part.info["code_bytes"] <= full.info["code_bytes"]
    assert part.info["n_instr"] == full.info["n_instr"] and part.info["l2in"] == full.info["l2in"]
    for w in (4, 16):
        d0, c0 = full.emulate(w)
        d1, c1 = part.emulate(w)
        assert c0 == c1 and (d0 == d1).all()
        assert part.disasm(w) == full.disasm(w)
    for w in (1, 2, 8, 32):
        with pytest.raises(fbg.FbgError) as e:
            part.emulate(w)
        assert e.value.status == fbg.FBG_E_INVAL and "words per lane" in str(e.value)
        assert fbg.lib.fbg_program_disasm(part.handle, w, None, 0) == -1
        t = fbg.Tune(w, 0, 0, 0)
        assert fbg.lib.fbg_program_set_tuning(part.handle, ctypes.byref(t)) == fbg.FBG_E_INVAL
    part.set_tuning(4)
    assert part.info["words_per_lane"] == 4
    # the default tiling of a one-tiling program is that tiling
    one = fbg.Program(text, n, fbg.compile_wpl(2))
    assert one.info["words_per_lane"] == 2
    assert one.emulate(2)[1] == full.emulate(2)[1]


def test_compile_flags_for_assume_and_subst():
    """The tiling flags act the same through fbg_compile_assume and
    fbg_compile_subst; unknown bits are refused by all three calls."""
    text, n = "a = x0 & x3\na | (x1 ^ x5) | ~x6\nx2 | x4 | x7", 8
    assume = [-1, 1, -1, 0, -1, -1, -1, -1]
    full = fbg.compile_assume(text, n, assume)
    part = fbg.compile_assume(text, n, assume, fbg.compile_wpl(8))
    assert part.info["words_per_lane"] == 8 and part.n == full.n == 6
    assert part.emulate(8)[1] == full.emulate(8)[1]
    with pytest.raises(fbg.FbgError):
        part.emulate(4)
    subst = [0, 1, 2, 0, -2, 3, 4, 1]  # x4 := 1; x3 = x0, x7 = x1
    full = fbg.compile_subst(text, n, subst, 5)
    part = fbg.compile_subst(text, n, subst, 5, fbg.compile_wpl(1, 32))
    assert part.info["words_per_lane"] in (1, 32)
    for w in (1, 32):
        assert part.emulate(w)[1] == full.emulate(w)[1]
    with pytest.raises(fbg.FbgError):
        part.emulate(2)
    for call in (lambda: fbg.compile_assume(text, n, assume, 0x80),
                 lambda: fbg.compile_subst(text, n, subst, 5, 0x100)):
        with pytest.raises(fbg.FbgError) as e:
            call()
        assert e.value.status == fbg.FBG_E_INVAL

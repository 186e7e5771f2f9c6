"""ctypes binding of libfbg (include/fbg.h).

Argument marshalling only: every step of the path runs in the library's HIP
kernels.  Device buffers are torch tensors on the current HIP device (int64
storage, read back as uint64), streams are torch streams.  If libfbg.so has
not been built, importing this module raises: there is no fallback.
"""

import ctypes
import os
import threading
import weakref

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfbg.so")

FBG_OK = 0
FBG_E_INVAL = -1
FBG_E_PARSE = -2
FBG_E_RANGE = -3
FBG_E_NOMEM = -4
FBG_E_DEVICE = -5
_STATUS = {0: "FBG_OK", -1: "FBG_E_INVAL", -2: "FBG_E_PARSE", -3: "FBG_E_RANGE",
           -4: "FBG_E_NOMEM", -5: "FBG_E_DEVICE"}

MAX_VARS = 48
MAX_DNF_VARS = 40
MAX_WORDS_PER_LANE = 32
COMPILE_WPL_MASK = 0x3F


def compile_wpl(*words_per_lane):
    """Compile flags that encode a program only for these tilings (words
    per lane); a call at any other tiling then fails with FBG_E_INVAL."""
    f = 0
    for w in words_per_lane:
        w = int(w)
        if w < 1 or w > MAX_WORDS_PER_LANE or w & (w - 1):
            raise ValueError(f"words per lane {w}: not one of 1, 2, 4, 8, 16, 32")
        f |= 1 << (w.bit_length() - 1)
    return f


class FbgError(RuntimeError):
    def __init__(self, status, message, offset=-1):
        super().__init__("%s: %s" % (_STATUS.get(status, status), message))
        self.status = status
        self.offset = offset


class ProgramInfo(ctypes.Structure):
    _fields_ = [("n_vars", ctypes.c_int32), ("const_value", ctypes.c_int32), ("l2in", ctypes.c_uint64),
                ("n_instr", ctypes.c_int32), ("n_regs", ctypes.c_int32), ("n_clause_instr", ctypes.c_int32),
                ("words_per_lane", ctypes.c_int32), ("dnf_words", ctypes.c_uint64),
                ("code_bytes", ctypes.c_uint64), ("l_valu", ctypes.c_double)]


class Tune(ctypes.Structure):
    _fields_ = [("words_per_lane", ctypes.c_int32), ("grid_blocks", ctypes.c_int32),
                ("flags", ctypes.c_int32), ("direct_run", ctypes.c_int32)]


TUNE_COFACTOR = 1


class Item(ctypes.Structure):
    _fields_ = [("prog", ctypes.c_int32), ("slot", ctypes.c_int32), ("tile_begin", ctypes.c_uint64),
                ("tile_end", ctypes.c_uint64)]


# fbg_item as a numpy record: work items marshalled in one step
ITEM_DTYPE = np.dtype([("prog", "<i4"), ("slot", "<i4"), ("tile_begin", "<u8"), ("tile_end", "<u8")])
assert ITEM_DTYPE.itemsize == ctypes.sizeof(Item)


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError("libfbg.so is not built (run __graft_entry__.build() or "
                          "python paper_1310_6978_amd/build.py)")
    # torch ships its own HIP runtime with the same soname as the system one;
    # loading torch first makes libfbg bind to that runtime, so device
    # pointers and streams from torch are valid in libfbg's calls (loading
    # libfbg first would bring a second runtime into the process)
    import torch  # noqa: F401
    lib = ctypes.CDLL(LIB_PATH)
    vp, u64, i32, u32 = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int32, ctypes.c_uint32
    u64p = ctypes.POINTER(ctypes.c_uint64)
    sigs = {
        "fbg_compile": (i32, [ctypes.c_char_p, i32, u32, ctypes.POINTER(vp)]),
        "fbg_compile_assume": (i32, [ctypes.c_char_p, i32, ctypes.POINTER(ctypes.c_int8), u32, ctypes.POINTER(vp)]),
        "fbg_compile_subst": (i32, [ctypes.c_char_p, i32, ctypes.POINTER(ctypes.c_int32), i32, u32,
                                    ctypes.POINTER(vp)]),
        "fbg_program_free": (None, [vp]),
        "fbg_program_info": (i32, [vp, ctypes.POINTER(ProgramInfo)]),
        "fbg_program_get_info": (i32, [vp, ctypes.POINTER(ProgramInfo)]),
        "fbg_program_set_tuning": (i32, [vp, ctypes.POINTER(Tune)]),
        "fbg_eval_dnf": (i32, [vp, vp, u64, vp]),
        "fbg_eval_dnf_tuned": (i32, [vp, vp, u64, ctypes.POINTER(Tune), vp]),
        "fbg_count": (i32, [vp, vp, vp]),
        "fbg_count_tuned": (i32, [vp, vp, ctypes.POINTER(Tune), vp]),
        "fbg_enumerate": (i32, [vp, vp, u64, vp, vp]),
        "fbg_enumerate_noalloc": (i32, [vp, vp, u64, vp, vp]),
        "fbg_batch_create": (i32, [ctypes.POINTER(vp), i32, ctypes.POINTER(Tune), ctypes.POINTER(vp)]),
        "fbg_batch_count": (i32, [vp, vp, vp]),
        "fbg_batch_count_graph": (i32, [vp, vp, vp]),
        "fbg_batch_set_dnf_outputs": (i32, [vp, ctypes.POINTER(vp), ctypes.POINTER(ctypes.c_uint64)]),
        "fbg_batch_eval_dnf": (i32, [vp, vp, vp]),
        "fbg_batch_set_enum_outputs": (i32, [vp, ctypes.POINTER(vp), ctypes.POINTER(ctypes.c_uint64)]),
        "fbg_batch_enumerate": (i32, [vp, vp]),
        "fbg_batch_free": (None, [vp]),
        "fbg_count_batch": (i32, [ctypes.POINTER(vp), i32, vp, ctypes.POINTER(Tune), vp]),
        "fbg_enumerate_dnf": (i32, [vp, i32, vp, u64, vp, vp]),
        "fbg_program_tiles": (u64, [vp, i32]),
        "fbg_server_create": (i32, [i32, i32, i32, i32, i32, ctypes.POINTER(vp)]),
        "fbg_server_launch": (i32, [vp, ctypes.POINTER(vp), i32, ctypes.POINTER(Item), i32, vp, i32, vp]),
        "fbg_server_free": (None, [vp]),
        "fbg_program_emulate": (i32, [vp, i32, u64p, u64, u64p]),
        "fbg_program_disasm": (ctypes.c_int64, [vp, i32, ctypes.c_char_p, ctypes.c_int64]),
        "fbg_last_error": (ctypes.c_char_p, []),
        "fbg_last_error_offset": (ctypes.c_int64, []),
        "fbg_version": (ctypes.c_char_p, []),
    }
    for name, (res, args) in sigs.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


lib = _load()

# every symbol include/fbg.h declares
EXPORTED = ("fbg_compile", "fbg_compile_assume", "fbg_compile_subst", "fbg_program_free", "fbg_program_info",
            "fbg_program_get_info", "fbg_program_set_tuning",
            "fbg_eval_dnf", "fbg_eval_dnf_tuned",
            "fbg_count", "fbg_count_tuned", "fbg_enumerate", "fbg_enumerate_noalloc", "fbg_enumerate_dnf", "fbg_batch_create",
            "fbg_batch_count", "fbg_batch_count_graph", "fbg_batch_set_dnf_outputs", "fbg_batch_eval_dnf",
            "fbg_batch_set_enum_outputs", "fbg_batch_enumerate",
            "fbg_batch_free", "fbg_count_batch", "fbg_program_tiles", "fbg_server_create",
            "fbg_server_launch", "fbg_server_free", "fbg_program_emulate", "fbg_program_disasm",
            "fbg_last_error", "fbg_last_error_offset", "fbg_version")


def _check(st):
    if st != FBG_OK:
        raise FbgError(st, lib.fbg_last_error().decode(errors="replace"), lib.fbg_last_error_offset())


def _tune(words_per_lane=0, grid_blocks=0, cofactor=False, direct_run=0):
    if not words_per_lane and not grid_blocks and not cofactor and not direct_run:
        return None
    return ctypes.byref(Tune(int(words_per_lane), int(grid_blocks), TUNE_COFACTOR if cofactor else 0,
                             int(direct_run)))


def _torch_stream(stream):
    """The torch stream object of `stream` (None: the current stream; an
    integer: a caller-owned hipStream_t)."""
    import torch
    if stream is None:
        return torch.cuda.current_stream()
    if hasattr(stream, "cuda_stream"):
        return stream
    return torch.cuda.ExternalStream(int(stream))


def _stream(stream):
    return ctypes.c_void_p(_torch_stream(stream).cuda_stream)


# Deferred release.  A launch reads a program's code (and a batch its work
# tables) until it finishes, but the library returns a freed block to its
# arena at once, where the next compile may overwrite it.  So an object that
# was launched is not freed directly: free() records an event on every
# stream it was launched on and parks the handle here; it is released once
# all those events have completed (checked whenever objects are created or
# freed).  Objects may be created and freed on several threads (a serving
# loop compiles on a thread pool): the list changes only under _grave_lock,
# and an entry is taken off it before it is released, so it is released once.
_graveyard = []
_grave_lock = threading.Lock()


def _sweep():
    with _grave_lock:
        done, keep = [], []
        for entry in _graveyard:
            (done if all(e.query() for e in entry[1]) else keep).append(entry)
        _graveyard[:] = keep
    for release, _, _ in done:
        release()


def _release_after(streams, release, keepalive=()):
    import torch
    events = []
    for s in streams.values():
        e = torch.cuda.Event()
        e.record(s)
        events.append(e)
    with _grave_lock:
        _graveyard.append((release, events, tuple(keepalive)))
    _sweep()


def _used_on(objs, stream):
    """Note that a launch on `stream` uses every object of `objs`."""
    s = _torch_stream(stream)
    for o in objs:
        o._streams[s.cuda_stream] = s


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _device_u64(nelem, like=None):
    import torch
    return torch.empty(max(int(nelem), 1), dtype=torch.int64, device="cuda")


def as_u64(t):
    """Device or host int64 tensor -> numpy uint64 array (host copy)."""
    return t.detach().cpu().numpy().view(np.uint64)


def dnf_words(n):
    return 1 if n < 6 else 1 << (n - 6)


class Program:
    """A compiled formula, resident on the device it was compiled on."""

    def __init__(self, src, n, flags=0, assume=None, subst=None, n_free=0):
        h = ctypes.c_void_p()
        if isinstance(src, str):
            src = src.encode()
        if subst is not None:
            a = np.ascontiguousarray(subst, dtype=np.int32)
            if a.shape != (int(n),):
                raise ValueError("subst needs %d entries, got shape %s" % (int(n), a.shape))
            _check(lib.fbg_compile_subst(src, int(n), a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                         int(n_free), int(flags), ctypes.byref(h)))
        elif assume is None:
            _check(lib.fbg_compile(src, int(n), int(flags), ctypes.byref(h)))
        else:
            a = np.ascontiguousarray(assume, dtype=np.int8)
            if a.shape != (int(n),):
                raise ValueError("assume needs %d entries, got shape %s" % (int(n), a.shape))
            _check(lib.fbg_compile_assume(src, int(n), a.ctypes.data_as(ctypes.POINTER(ctypes.c_int8)),
                                          int(flags), ctypes.byref(h)))
        self._h = h
        self._streams = {}
        self._batches = weakref.WeakSet()   # batches holding this program (their launches read it too)
        _sweep()
        info = ProgramInfo()
        _check(lib.fbg_program_info(h, ctypes.byref(info)))
        self.info = {f: getattr(info, f) for f, _ in ProgramInfo._fields_}
        self.n = int(info.n_vars)

    @property
    def handle(self):
        if self._h is None:
            raise FbgError(FBG_E_INVAL, "program was freed")
        return self._h

    def free(self):
        """Release the program once every launch that used it has finished
        (launches are asynchronous; see _release_after)."""
        h = getattr(self, "_h", None)
        if h is None:
            return
        self._h = None
        streams, self._streams = self._streams, {}
        for b in list(self._batches):
            streams.update(b._streams)
        if streams:
            _release_after(streams, lambda: lib.fbg_program_free(h))
        else:
            lib.fbg_program_free(h)

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass

    def set_tuning(self, words_per_lane, cofactor=False):
        """Default words per lane and evaluation variant for this program
        (fbg_program_set_tuning)."""
        t = Tune(int(words_per_lane), 0, TUNE_COFACTOR if cofactor else 0, 0)
        _check(lib.fbg_program_set_tuning(self.handle, ctypes.byref(t)))
        info = ProgramInfo()
        _check(lib.fbg_program_info(self.handle, ctypes.byref(info)))
        self.info = {f: getattr(info, f) for f, _ in ProgramInfo._fields_}

    def emulate(self, words_per_lane=1):
        """Host interpretation of the encoded program: (dnf uint64 array, count).
        Reads it the way the uniform-cofactor kernels do when the program's
        default tuning selects them (set_tuning(..., cofactor=True))."""
        out = np.zeros(dnf_words(self.n), dtype=np.uint64)
        cnt = ctypes.c_uint64(0)
        _check(lib.fbg_program_emulate(self.handle, int(words_per_lane),
                                       out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)), out.size,
                                       ctypes.byref(cnt)))
        return out, cnt.value

    def disasm(self, words_per_lane=0):
        size = lib.fbg_program_disasm(self.handle, int(words_per_lane), None, 0)
        buf = ctypes.create_string_buffer(int(size) + 1)
        lib.fbg_program_disasm(self.handle, int(words_per_lane), buf, int(size) + 1)
        return buf.value.decode()


def compile(src, n, flags=0):  # noqa: A001 - the boundary's name
    return Program(src, n, flags)


def compile_assume(src, n, assume, flags=0):
    """fbg_compile_assume: assume[k] in {-1, 0, 1} (-1 free); the program's
    variables are the free ones, renumbered in increasing order."""
    return Program(src, n, flags, assume=assume)


def compile_subst(src, n, subst, n_free, flags=0):
    """fbg_compile_subst: subst[k] = -1 / -2 (constant 0 / 1) or the
    program variable j < n_free that xk becomes."""
    return Program(src, n, flags, subst=subst, n_free=n_free)


def eval_dnf(prog, out=None, stream=None, words_per_lane=0, grid_blocks=0, cofactor=False):
    """fbg_eval_dnf: the DNF vector as an int64 device tensor of uint64 words."""
    words = dnf_words(prog.n)
    if out is None:
        out = _device_u64(words)
    tune = _tune(words_per_lane, grid_blocks, cofactor)
    if tune is None:
        _check(lib.fbg_eval_dnf(prog.handle, _ptr(out), out.numel(), _stream(stream)))
    else:
        _check(lib.fbg_eval_dnf_tuned(prog.handle, _ptr(out), out.numel(), tune, _stream(stream)))
    _used_on([prog], stream)
    return out


def count(prog, out=None, stream=None, words_per_lane=0, grid_blocks=0, cofactor=False):
    """fbg_count: one-element int64 device tensor holding the model count."""
    if out is None:
        out = _device_u64(1)
    tune = _tune(words_per_lane, grid_blocks, cofactor)
    if tune is None:
        _check(lib.fbg_count(prog.handle, _ptr(out), _stream(stream)))
    else:
        _check(lib.fbg_count_tuned(prog.handle, _ptr(out), tune, _stream(stream)))
    _used_on([prog], stream)
    return out


def enumerate_models(prog, capacity, out=None, total=None, stream=None):
    """fbg_enumerate: (device tensor of the first min(total, capacity) model
    indices, ascending; one-element device tensor with the total)."""
    if out is None:
        out = _device_u64(capacity)
    if total is None:
        total = _device_u64(1)
    ptr = _ptr(out) if capacity > 0 else ctypes.c_void_p(0)
    _check(lib.fbg_enumerate(prog.handle, ptr, int(capacity), _ptr(total), _stream(stream)))
    _used_on([prog], stream)
    return out, total


def enumerate_models_noalloc(prog, out, total, stream=None):
    """fbg_enumerate_noalloc: as enumerate_models into caller-given device
    tensors (out: capacity int64 words, may be empty; total: one word), with
    the temporaries in the library's static device scratch."""
    ptr = _ptr(out) if out.numel() > 0 else ctypes.c_void_p(0)
    _check(lib.fbg_enumerate_noalloc(prog.handle, ptr, int(out.numel()), _ptr(total), _stream(stream)))
    _used_on([prog], stream)
    return out, total


def enumerate_dnf(dnf, n, capacity, out=None, total=None, stream=None):
    """fbg_enumerate_dnf: the models read off a stored DNF vector (device
    tensor of max(1, 2^(n-6)) words)."""
    if out is None:
        out = _device_u64(capacity)
    if total is None:
        total = _device_u64(1)
    ptr = _ptr(out) if capacity > 0 else ctypes.c_void_p(0)
    _check(lib.fbg_enumerate_dnf(_ptr(dnf), int(n), ptr, int(capacity), _ptr(total), _stream(stream)))
    return out, total


def program_tiles(prog, words_per_lane):
    """Tiles of 64 * words_per_lane words covering the program's valuations."""
    return int(lib.fbg_program_tiles(prog.handle, int(words_per_lane)))


class Server:
    """fbg_server: launches over explicit work items that add into count
    slots, with pinned staging buffers reused round-robin."""

    def __init__(self, max_programs, max_items, words_per_lane, nbuf=4, cofactor=False):
        h = ctypes.c_void_p()
        _check(lib.fbg_server_create(int(max_programs), int(max_items), int(words_per_lane), int(nbuf),
                                     TUNE_COFACTOR if cofactor else 0, ctypes.byref(h)))
        self._h = h
        self.words_per_lane = int(words_per_lane)
        self.max_programs = int(max_programs)
        self.max_items = int(max_items)

    def launch(self, progs, items, counts, stream=None):
        """progs: list of Program; items: (prog index, slot, tile_begin,
        tile_end) tuples, or a numpy array of ITEM_DTYPE; counts: int64 device
        tensor of slots (added to)."""
        arr = (ctypes.c_void_p * len(progs))(*[p.handle.value for p in progs])
        its = np.ascontiguousarray(np.asarray(items, dtype=ITEM_DTYPE) if not isinstance(items, np.ndarray)
                                   else items.astype(ITEM_DTYPE, copy=False))
        _check(lib.fbg_server_launch(self._h, arr, len(progs), its.ctypes.data_as(ctypes.POINTER(Item)), len(its),
                                     _ptr(counts), counts.numel(), _stream(stream)))
        _used_on(progs, stream)

    def free(self):
        if getattr(self, "_h", None) is not None:
            lib.fbg_server_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


class Batch:
    """A work plan for counting many programs in one persistent launch."""

    def __init__(self, progs, words_per_lane=0, grid_blocks=0, cofactor=False, direct_run=0):
        self._progs = list(progs)  # keep the programs alive
        arr = (ctypes.c_void_p * len(self._progs))(*[p.handle.value for p in self._progs])
        h = ctypes.c_void_p()
        _check(lib.fbg_batch_create(arr, len(self._progs),
                                    _tune(words_per_lane, grid_blocks, cofactor, direct_run), ctypes.byref(h)))
        self._h = h
        self._streams = {}
        for p in self._progs:
            p._batches.add(self)

    def __len__(self):
        return len(self._progs)

    def count(self, out=None, stream=None, graph=False):
        """Counts of all programs; graph=True replays a captured HIP graph
        (fbg_batch_count_graph)."""
        if out is None:
            out = _device_u64(len(self._progs))
        f = lib.fbg_batch_count_graph if graph else lib.fbg_batch_count
        _check(f(self._h, _ptr(out), _stream(stream)))
        _used_on([self], stream)
        return out

    def set_dnf_outputs(self, outs):
        """outs: one int64 device tensor per program (at least its dnf_words)."""
        if len(outs) != len(self._progs):
            raise ValueError("need %d output tensors" % len(self._progs))
        self._outs = list(outs)  # the buffers must outlive the launches
        ptrs = (ctypes.c_void_p * len(outs))(*[o.data_ptr() for o in outs])
        sizes = (ctypes.c_uint64 * len(outs))(*[o.numel() for o in outs])
        _check(lib.fbg_batch_set_dnf_outputs(self._h, ptrs, sizes))

    def set_enum_outputs(self, outs):
        """outs: one int64 device tensor per program (its capacity), or
        None for capacity 0."""
        if len(outs) != len(self._progs):
            raise ValueError("need %d output tensors" % len(self._progs))
        self._enum_outs = list(outs)
        ptrs = (ctypes.c_void_p * len(outs))(*[o.data_ptr() if o is not None else None for o in outs])
        caps = (ctypes.c_uint64 * len(outs))(*[o.numel() if o is not None else 0 for o in outs])
        _check(lib.fbg_batch_set_enum_outputs(self._h, ptrs, caps))

    def enumerate(self, stream=None):
        """Models of every program into its enumeration output, ascending
        (after eval_dnf on the same stream)."""
        _check(lib.fbg_batch_enumerate(self._h, _stream(stream)))
        _used_on([self], stream)

    def eval_dnf(self, counts=None, stream=None):
        """Every program's DNF vector into its output tensor and its count
        into counts, computing each word once (fbg_batch_eval_dnf: one launch
        per plan, plus a sum of tile counts for plans written one run of
        tiles per wave)."""
        if counts is None:
            counts = _device_u64(len(self._progs))
        _check(lib.fbg_batch_eval_dnf(self._h, _ptr(counts), _stream(stream)))
        _used_on([self], stream)
        return counts

    def free(self):
        """Release the plan once its launches have finished; the programs
        stay alive until then."""
        h = getattr(self, "_h", None)
        if h is None:
            return
        self._h = None
        streams = dict(self._streams)   # kept: the programs' own free() still waits for these launches
        if streams:
            _release_after(streams, lambda: lib.fbg_batch_free(h), keepalive=self._progs)
        else:
            lib.fbg_batch_free(h)

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def count_batch(progs, out=None, stream=None, words_per_lane=0, grid_blocks=0, cofactor=False):
    """fbg_count_batch: counts of all programs (one persistent launch)."""
    progs = list(progs)
    if out is None:
        out = _device_u64(len(progs))
    arr = (ctypes.c_void_p * len(progs))(*[p.handle.value for p in progs])
    _check(lib.fbg_count_batch(arr, len(progs), _ptr(out), _tune(words_per_lane, grid_blocks, cofactor),
                               _stream(stream)))
    return out


def version():
    return lib.fbg_version().decode()

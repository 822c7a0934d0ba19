"""ctypes binding of libecc (include/ecc.h).

Argument marshalling only: every step of the computation runs in the HIP
library.  torch supplies device memory and streams.  If libecc.so has not been
built the import of this module still works, but every call raises
:class:`EccLibraryMissing`; there is no fallback computation.
"""
from __future__ import annotations

import ctypes
import os
from typing import Iterable, Sequence

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libecc.so")

ECC_OK, ECC_ERR_INVALID_ARG, ECC_ERR_UNSUPPORTED, ECC_ERR_OUT_OF_MEMORY, ECC_ERR_DEVICE, ECC_ERR_BUSY = range(6)
ECC_U8, ECC_U16, ECC_F32 = 1, 2, 3
ECC_SUBLEVEL, ECC_SUPERLEVEL = 0, 1

# public C entry points (kept in step with include/ecc.h)
EXPORTS = (
    "ecc_create", "ecc_destroy", "ecc_last_error", "ecc_status_string",
    "ecc_curves_compute", "ecc_curves_compute_noalloc", "ecc_curves_compute_streamed", "ecc_curves_compute_batch",
    "ecc_curves_compute_4d",
    "ecc_batch_plan_tune",
    "ecc_vertex_table", "ecc_vertex_classes_compute", "ecc_vertex_class_table",
    "ecc_validate_field", "ecc_profile_enable", "ecc_profile_read",
    "ecc_server_create", "ecc_server_submit", "ecc_server_poll", "ecc_server_drain",
    "ecc_server_destroy",
)


class EccLibraryMissing(RuntimeError):
    pass


class EccError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{_status_name(status)}: {message}")
        self.status = status
        self.message = message


class Field(ctypes.Structure):
    _fields_ = [("ndim", ctypes.c_int32), ("dtype", ctypes.c_int32), ("shape", ctypes.c_int64 * 3),
                ("data", ctypes.c_void_p), ("n_levels", ctypes.c_int32),
                ("connectivity", ctypes.c_int32), ("thresholds", ctypes.c_void_p),
                ("filtration", ctypes.c_int32)]


class Field4(ctypes.Structure):
    _fields_ = [("dtype", ctypes.c_int32), ("shape", ctypes.c_int64 * 4), ("data", ctypes.c_void_p),
                ("n_levels", ctypes.c_int32), ("connectivity", ctypes.c_int32), ("thresholds", ctypes.c_void_p),
                ("filtration", ctypes.c_int32)]


class Curves(ctypes.Structure):
    _fields_ = [("ec", ctypes.c_void_p), ("perimeter", ctypes.c_void_p), ("area", ctypes.c_void_p),
                ("volume", ctypes.c_void_p)]


class ServerConfig(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_size_t), ("max_slots", ctypes.c_int32),
                ("max_batch", ctypes.c_int32)]


_lib = None


def load(path: str = LIB_PATH):
    """Open libecc.so and declare the C signatures."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise EccLibraryMissing(f"{path} is not built; run `python -m paper_2311_11740_amd.build`")
    # libecc binds to the HIP runtime already present in the process.  torch
    # ships its own copy of that runtime: loading torch first makes libecc use
    # the same one, so torch's device pointers and streams are valid in libecc
    # (loaded the other way round, two runtimes would compete for the device).
    import torch  # noqa: F401
    lib = ctypes.CDLL(path)
    vp, i32, i64p = ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_int64)
    sig = {
        "ecc_create": ([ctypes.c_int, ctypes.POINTER(vp)], ctypes.c_int),
        "ecc_destroy": ([vp], ctypes.c_int),
        "ecc_last_error": ([], ctypes.c_char_p),
        "ecc_status_string": ([ctypes.c_int], ctypes.c_char_p),
        "ecc_curves_compute": ([vp, ctypes.POINTER(Field), ctypes.POINTER(Curves), vp], ctypes.c_int),
        "ecc_curves_compute_noalloc": ([vp, ctypes.POINTER(Field), ctypes.POINTER(Curves), vp], ctypes.c_int),
        "ecc_curves_compute_streamed": ([vp, ctypes.POINTER(Field), ctypes.POINTER(Curves), ctypes.c_size_t, vp],
                                        ctypes.c_int),
        "ecc_curves_compute_batch": ([vp, i32, ctypes.POINTER(Field), ctypes.POINTER(Curves), vp],
                                     ctypes.c_int),
        "ecc_batch_plan_tune": ([vp, i32, ctypes.POINTER(Field), vp], ctypes.c_int),
        "ecc_curves_compute_4d": ([vp, ctypes.POINTER(Field4), vp, vp, vp, vp], ctypes.c_int),
        "ecc_vertex_table": ([i32, i32, ctypes.POINTER(ctypes.c_int32)], ctypes.c_int),
        "ecc_vertex_classes_compute": ([vp, ctypes.POINTER(Field), vp, vp], ctypes.c_int),
        "ecc_vertex_class_table": ([i32, ctypes.POINTER(ctypes.c_int32)], ctypes.c_int),
        "ecc_validate_field": ([ctypes.POINTER(Field), ctypes.POINTER(Curves)], ctypes.c_int),
        "ecc_profile_enable": ([vp, i32], ctypes.c_int),
        "ecc_profile_read": ([vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64), i32],
                             ctypes.c_int),
        "ecc_server_create": ([vp, ctypes.POINTER(ServerConfig), ctypes.POINTER(vp)], ctypes.c_int),
        "ecc_server_submit": ([vp, ctypes.POINTER(Field), ctypes.POINTER(Curves),
                               ctypes.POINTER(ctypes.c_uint64)], ctypes.c_int),
        "ecc_server_poll": ([vp, ctypes.c_uint64, ctypes.POINTER(ctypes.c_int32)], ctypes.c_int),
        "ecc_server_drain": ([vp], ctypes.c_int),
        "ecc_server_destroy": ([vp], ctypes.c_int),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    _ = i64p
    _lib = lib
    return lib


def _status_name(s: int) -> str:
    names = ["ECC_OK", "ECC_ERR_INVALID_ARG", "ECC_ERR_UNSUPPORTED", "ECC_ERR_OUT_OF_MEMORY",
             "ECC_ERR_DEVICE", "ECC_ERR_BUSY"]
    return names[s] if 0 <= s < len(names) else f"status {s}"


def check(status: int):
    if status != ECC_OK:
        msg = load().ecc_last_error().decode(errors="replace")
        raise EccError(status, msg)


def vertex_table(ndim: int, connectivity: int = 0):
    """The library's per-vertex contribution table as nested lists (host call)."""
    lib = load()
    n = 16 if ndim == 2 else 256
    buf = (ctypes.c_int32 * (n * 4))()
    check(lib.ecc_vertex_table(ndim, connectivity, buf))
    return [list(buf[4 * m:4 * m + 4]) for m in range(n)]


def vertex_class_table(ndim: int = 2):
    """Class of each vertex mask as the library counts it (-1 empty): 16 masks
    and classes 0..4 in 2D, 256 masks and classes 0..20 in 3D."""
    lib = load()
    n = 16 if ndim == 2 else 256
    buf = (ctypes.c_int32 * n)()
    check(lib.ecc_vertex_class_table(ndim, buf))
    return list(buf)


VERTEX_CLASSES_2D = ("one", "adjacent", "diagonal", "three", "four")


# ----------------------------------------------------------------------------
# torch-facing helpers (torch only supplies device memory and streams)
# ----------------------------------------------------------------------------
def _torch():
    import torch
    return torch


def _dtype_code(t) -> int:
    torch = _torch()
    if t.dtype == torch.uint8:
        return ECC_U8
    if t.dtype == torch.uint16:
        return ECC_U16
    if t.dtype == torch.float32:
        return ECC_F32
    raise TypeError(f"unsupported field dtype {t.dtype}")


def _stream_ptr(stream):
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream()
    if isinstance(stream, int):
        return stream or None
    return stream.cuda_stream or None


CHANNELS_2D = ("ec", "perimeter", "area")
CHANNELS_3D = ("ec", "perimeter", "area", "volume")


def make_field(t, n_levels: int, thresholds=None, connectivity: int = 0, superlevel: bool = False):
    """Build the C field descriptor for a contiguous device tensor.  The returned
    tuple keeps the host threshold buffer alive.  `superlevel` selects the
    filtration by {value >= t_l} over non-increasing thresholds."""
    import numpy as np
    if not t.is_contiguous():
        raise ValueError("field must be contiguous (C order)")
    if t.dim() not in (2, 3):
        raise ValueError("field must be 2D or 3D")
    f = Field()
    f.ndim = t.dim()
    f.dtype = _dtype_code(t)
    for k in range(3):
        f.shape[k] = int(t.shape[k]) if k < t.dim() else 0
    f.data = t.data_ptr()
    f.n_levels = int(n_levels)
    f.connectivity = int(connectivity or 0)
    f.filtration = ECC_SUPERLEVEL if superlevel else ECC_SUBLEVEL
    keep = None
    if thresholds is not None:
        keep = np.ascontiguousarray(np.asarray(thresholds, dtype=np.float32))
        if keep.size != n_levels:
            raise ValueError("thresholds must have n_levels entries")
        f.thresholds = keep.ctypes.data
    else:
        f.thresholds = None
    return f, keep


def alloc_curves(ndim: int, n_levels: int, device, channels: Iterable[str] | None = None):
    torch = _torch()
    allowed = CHANNELS_2D if ndim == 2 else CHANNELS_3D
    channels = allowed if channels is None else tuple(channels)
    for c in channels:
        if c not in allowed:
            raise ValueError(f"channel {c!r} not available for {ndim}D fields")
    out = {c: torch.empty(n_levels, dtype=torch.int64, device=device) for c in channels}
    cv = Curves()
    for c in ("ec", "perimeter", "area", "volume"):
        setattr(cv, c, out[c].data_ptr() if c in out else None)
    return out, cv


class Context:
    """A libecc context on one HIP device."""

    def __init__(self, device: int = 0):
        self._lib = load()
        h = ctypes.c_void_p()
        check(self._lib.ecc_create(int(device), ctypes.byref(h)))
        self.handle = h
        self.device = device

    def close(self):
        if getattr(self, "handle", None):
            check(self._lib.ecc_destroy(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def profile(self, on: bool = True):
        check(self._lib.ecc_profile_enable(self.handle, 1 if on else 0))

    def profile_read(self, reset: bool = True):
        """(total milliseconds, launches) of the field-reading kernel since the last reset."""
        ms = ctypes.c_double()
        n = ctypes.c_int64()
        check(self._lib.ecc_profile_read(self.handle, ctypes.byref(ms), ctypes.byref(n), 1 if reset else 0))
        return ms.value, n.value

    def compute(self, field, n_levels: int, thresholds=None, connectivity: int = 0,
                channels: Sequence[str] | None = None, stream=None, out=None, noalloc: bool = False,
                superlevel: bool = False):
        """Curves of one device field: dict channel -> int64 device tensor (async on `stream`).
        `out` may supply preallocated curves (dict channel -> int64 tensor of n_levels).
        `noalloc` calls ecc_curves_compute_noalloc (the library allocates no
        device memory for the call; `out` avoids torch's allocation too).
        `superlevel` selects the superlevel filtration (ECC_SUPERLEVEL)."""
        f, keep = make_field(field, n_levels, thresholds, connectivity, superlevel)
        if out is None:
            out, cv = alloc_curves(field.dim(), n_levels, field.device, channels)
        else:
            cv = Curves()
            for c in ("ec", "perimeter", "area", "volume"):
                setattr(cv, c, out[c].data_ptr() if c in out else None)
        fn = self._lib.ecc_curves_compute_noalloc if noalloc else self._lib.ecc_curves_compute
        check(fn(self.handle, ctypes.byref(f), ctypes.byref(cv), _stream_ptr(stream)))
        del keep
        return out

    def compute_streamed(self, field, n_levels: int, thresholds=None, connectivity: int = 0,
                         channels: Sequence[str] | None = None, slab_bytes: int = 0, stream=None,
                         superlevel: bool = False):
        """Curves of a field in host memory (numpy array), streamed through the
        device in slabs of at most `slab_bytes` (0: the library's default).
        Blocking; returns dict channel -> int64 numpy array."""
        import numpy as np
        a = np.ascontiguousarray(field)
        if a.ndim not in (2, 3):
            raise ValueError("field must be 2D or 3D")
        codes = {np.dtype(np.uint8): ECC_U8, np.dtype(np.uint16): ECC_U16, np.dtype(np.float32): ECC_F32}
        if a.dtype not in codes:
            raise TypeError(f"unsupported field dtype {a.dtype}")
        f = Field()
        f.ndim = a.ndim
        f.dtype = codes[a.dtype]
        for k in range(3):
            f.shape[k] = int(a.shape[k]) if k < a.ndim else 0
        f.data = a.ctypes.data
        f.n_levels = int(n_levels)
        f.connectivity = int(connectivity or 0)
        f.filtration = ECC_SUPERLEVEL if superlevel else ECC_SUBLEVEL
        keep = None
        if thresholds is not None:
            keep = np.ascontiguousarray(np.asarray(thresholds, dtype=np.float32))
            if keep.size != n_levels:
                raise ValueError("thresholds must have n_levels entries")
            f.thresholds = keep.ctypes.data
        allowed = CHANNELS_2D if a.ndim == 2 else CHANNELS_3D
        channels = allowed if channels is None else tuple(channels)
        out = {c: np.zeros(n_levels, dtype=np.int64) for c in channels}
        cv = Curves()
        for c in ("ec", "perimeter", "area", "volume"):
            setattr(cv, c, out[c].ctypes.data if c in out else None)
        check(self._lib.ecc_curves_compute_streamed(self.handle, ctypes.byref(f), ctypes.byref(cv),
                                                    int(slab_bytes), _stream_ptr(stream)))
        del keep, a
        return out

    def vertex_classes(self, field, n_levels: int, thresholds=None, stream=None, out=None,
                       superlevel: bool = False):
        """Counts of lattice vertices per neighbourhood class and level: int64
        device tensor [5, n_levels] (2D, rows in VERTEX_CLASSES_2D order) or
        [21, n_levels] (3D, classes as vertex_class_table(3)), async on
        `stream`.  `out` may supply that tensor."""
        torch = _torch()
        f, keep = make_field(field, n_levels, thresholds, 0, superlevel)
        nc = 5 if field.dim() == 2 else 21
        if out is None:
            out = torch.empty((nc, n_levels), dtype=torch.int64, device=field.device)
        elif tuple(out.shape) != (nc, n_levels) or out.dtype != torch.int64 or not out.is_contiguous():
            raise ValueError(f"out must be a contiguous int64 tensor of shape ({nc}, n_levels)")
        check(self._lib.ecc_vertex_classes_compute(self.handle, ctypes.byref(f), out.data_ptr(),
                                                   _stream_ptr(stream)))
        del keep
        return out

    def compute_4d(self, field, n_levels: int, thresholds=None, connectivity: int = 0,
                   channels: Sequence[str] | None = None, stream=None, superlevel: bool = False):
        """Curves of a 4D device field (a, d, h, w): dict with ec, boundary
        (unit 3-faces with one active hypercube) and volume, int64 device
        tensors (async on `stream`).  connectivity 80 (default) or 8."""
        import numpy as np
        torch = _torch()
        if not field.is_contiguous() or field.dim() != 4:
            raise ValueError("field must be a contiguous 4D tensor")
        f = Field4()
        f.dtype = _dtype_code(field)
        for k in range(4):
            f.shape[k] = int(field.shape[k])
        f.data = field.data_ptr()
        f.n_levels = int(n_levels)
        f.connectivity = int(connectivity or 0)
        f.filtration = ECC_SUPERLEVEL if superlevel else ECC_SUBLEVEL
        keep = None
        if thresholds is not None:
            keep = np.ascontiguousarray(np.asarray(thresholds, dtype=np.float32))
            if keep.size != n_levels:
                raise ValueError("thresholds must have n_levels entries")
            f.thresholds = keep.ctypes.data
        names = ("ec", "boundary", "volume")
        channels = names if channels is None else tuple(channels)
        for c in channels:
            if c not in names:
                raise ValueError(f"channel {c!r} not available for 4D fields")
        out = {c: torch.empty(int(n_levels), dtype=torch.int64, device=field.device) for c in channels}
        ptr = [out[c].data_ptr() if c in out else None for c in names]
        check(self._lib.ecc_curves_compute_4d(self.handle, ctypes.byref(f), ptr[0], ptr[1], ptr[2],
                                              _stream_ptr(stream)))
        del keep
        return out

    def batch(self, fields, n_levels, thresholds=None, connectivity=0, channels=None, superlevel=False):
        """A reusable batched call over `fields` (device tensors); see Batch."""
        return Batch(self, fields, n_levels, thresholds, connectivity, channels, superlevel)

    def compute_batch(self, fields, n_levels, thresholds=None, connectivity=0,
                      channels: Sequence[str] | None = None, stream=None, superlevel=False):
        """Curves of many device fields in one batched call; list of dicts."""
        b = Batch(self, fields, n_levels, thresholds, connectivity, channels, superlevel)
        b.run(stream)
        return b.outputs

    def tune_batch(self, fields, n_levels, thresholds=None, connectivity=0, stream=None, superlevel=False):
        """Run the autotuner for this mix of fields (synchronises `stream`)."""
        Batch(self, fields, n_levels, thresholds, connectivity, (), superlevel).tune(stream)


class Batch:
    """Descriptors of a batched call, built once and run many times.

    fields: device tensors (2D or 3D, any mix); n_levels, thresholds,
    connectivity and superlevel: one value for all fields or a list with one
    per field.
    `outputs[i]` maps each wanted channel to an int64 device tensor of that
    field's n_levels (views into one allocation)."""

    def __init__(self, ctx, fields, n_levels, thresholds=None, connectivity=0, channels=None, superlevel=False):
        torch = _torch()
        n = len(fields)

        def per(v):
            return list(v) if isinstance(v, (list, tuple)) else [v] * n

        n_levels, connectivity, superlevel = per(n_levels), per(connectivity), per(superlevel)
        if thresholds is None or not isinstance(thresholds, (list, tuple)):
            thresholds = [thresholds] * n
        self.ctx = ctx
        self.n = n
        self.fields = list(fields)
        self.farr = (Field * max(n, 1))()
        self.carr = (Curves * max(n, 1))()
        self._keep = []
        chans = []
        total = 0
        for i, t in enumerate(self.fields):
            allowed = CHANNELS_2D if t.dim() == 2 else CHANNELS_3D
            ch = allowed if channels is None else tuple(c for c in channels if c in allowed)
            chans.append(ch)
            total += len(ch) * int(n_levels[i])
        dev = self.fields[0].device if n else "cpu"
        self.buffer = torch.empty(max(total, 1), dtype=torch.int64, device=dev)
        self.outputs = []
        off = 0
        for i, t in enumerate(self.fields):
            f, keep = make_field(t, n_levels[i], thresholds[i], connectivity[i], superlevel[i])
            self.farr[i] = f
            self._keep.append(keep)
            o = {}
            cv = Curves()
            for c in ("ec", "perimeter", "area", "volume"):
                if c in chans[i]:
                    o[c] = self.buffer[off:off + int(n_levels[i])]
                    off += int(n_levels[i])
                    setattr(cv, c, o[c].data_ptr())
                else:
                    setattr(cv, c, None)
            self.carr[i] = cv
            self.outputs.append(o)

    def run(self, stream=None):
        """Queue the batched call on `stream` (asynchronous)."""
        check(self.ctx._lib.ecc_curves_compute_batch(self.ctx.handle, self.n, self.farr, self.carr,
                                                     _stream_ptr(stream)))
        return self.outputs

    def run_per_field(self, stream=None):
        """The same fields with one single-field call each (the plain path the
        batched call is compared with)."""
        lib, h, sp = self.ctx._lib, self.ctx.handle, _stream_ptr(stream)
        f, c = ctypes.byref, self.carr
        for i in range(self.n):
            check(lib.ecc_curves_compute(h, f(self.farr[i]), f(c[i]), sp))
        return self.outputs

    def tune(self, stream=None):
        """Autotune the launch geometry for this mix (synchronises `stream`)."""
        check(self.ctx._lib.ecc_batch_plan_tune(self.ctx.handle, self.n, self.farr, _stream_ptr(stream)))


class Server:
    """A serving loop on one context: requests are host arrays, results host
    int64 arrays (see ecc_server_* in the C header)."""

    def __init__(self, ctx, hbm_budget_bytes: int, max_slots: int = 256, max_batch: int = 256):
        self.ctx = ctx
        self._lib = ctx._lib
        cfg = ServerConfig()
        cfg.hbm_budget_bytes = int(hbm_budget_bytes)
        cfg.max_slots = int(max_slots)
        cfg.max_batch = int(max_batch)
        h = ctypes.c_void_p()
        check(self._lib.ecc_server_create(ctx.handle, ctypes.byref(cfg), ctypes.byref(h)))
        self.handle = h
        self._pending = {}

    def submit(self, array, n_levels: int, thresholds=None, connectivity: int = 0, channels=None,
               superlevel: bool = False):
        """Submit a host numpy field; returns the ticket, or None when the server
        is full right now (retry after a poll)."""
        import numpy as np
        a = np.ascontiguousarray(array)
        if a.ndim not in (2, 3):
            raise ValueError("field must be 2D or 3D")
        f = Field()
        f.ndim = a.ndim
        f.dtype = {np.dtype(np.uint8): ECC_U8, np.dtype(np.uint16): ECC_U16,
                   np.dtype(np.float32): ECC_F32}[a.dtype]
        for k in range(3):
            f.shape[k] = a.shape[k] if k < a.ndim else 0
        f.data = a.ctypes.data
        f.n_levels = int(n_levels)
        f.connectivity = int(connectivity or 0)
        f.filtration = ECC_SUPERLEVEL if superlevel else ECC_SUBLEVEL
        keep = None
        if thresholds is not None:
            keep = np.ascontiguousarray(np.asarray(thresholds, dtype=np.float32))
            f.thresholds = keep.ctypes.data
        allowed = CHANNELS_2D if a.ndim == 2 else CHANNELS_3D
        chans = allowed if channels is None else tuple(c for c in channels if c in allowed)
        out = {c: np.empty(int(n_levels), np.int64) for c in chans}
        cv = Curves()
        for c in ("ec", "perimeter", "area", "volume"):
            setattr(cv, c, out[c].ctypes.data if c in out else None)
        t = ctypes.c_uint64()
        st = self._lib.ecc_server_submit(self.handle, ctypes.byref(f), ctypes.byref(cv), ctypes.byref(t))
        if st == ECC_ERR_BUSY:
            return None
        check(st)
        self._pending[t.value] = out
        return t.value

    def poll(self, ticket: int):
        """The result dict once the request is complete, else None."""
        d = ctypes.c_int32()
        check(self._lib.ecc_server_poll(self.handle, ctypes.c_uint64(ticket), ctypes.byref(d)))
        if d.value:
            return self._pending.pop(ticket)
        return None

    def drain(self):
        check(self._lib.ecc_server_drain(self.handle))

    def close(self):
        if getattr(self, "handle", None):
            check(self._lib.ecc_server_destroy(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

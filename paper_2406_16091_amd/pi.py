"""ctypes binding of libpi.so (include/pi.h).  Argument marshalling only:
every step of binning and the sweep runs in the library's HIP kernels.

Functions keep the C names (``pi_bin``, ``pi_interact``, ...) and accept
torch CUDA tensors (or raw integer device pointers) for device buffers and a
torch stream (or a raw hipStream_t integer) for ``stream``.  A non-OK status
raises :class:`PiError`.  If the library is missing the import of this module
fails loudly: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

import torch  # loaded first so that libpi.so binds to torch's HIP runtime

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpi.so")

PI_OK, PI_EINVAL, PI_ENOMEM, PI_ERANGE, PI_EDEVICE, PI_EAGAIN, PI_ENOTFOUND, PI_ESTATE = \
    0, -1, -2, -3, -4, -5, -6, -7
PI_PREC_COMPENSATED, PI_PREC_PLAIN, PI_PREC_FP64ACC = 0, 1, 2
PI_SWEEP_AUTO, PI_SWEEP_NOLDS, PI_SWEEP_PENCIL, PI_SWEEP_SUBBOX = 0, 1, 2, 3
PI_ORDER_SORTED, PI_ORDER_ORIGINAL = 0, 1

PRECISIONS = {"compensated": PI_PREC_COMPENSATED, "plain": PI_PREC_PLAIN, "fp64acc": PI_PREC_FP64ACC}
SWEEPS = {"auto": PI_SWEEP_AUTO, "nolds": PI_SWEEP_NOLDS, "pencil": PI_SWEEP_PENCIL,
          "subbox": PI_SWEEP_SUBBOX}


class PiError(RuntimeError):
    def __init__(self, status, what=""):
        self.status = int(status)
        msg = _lib().pi_status_str(self.status).decode() if _LIB is not None else str(status)
        super().__init__(f"{what}: {msg}" if what else msg)


class pi_grid(ctypes.Structure):
    _fields_ = [("origin", ctypes.c_float * 3), ("dims", ctypes.c_int32 * 3),
                ("cell_w", ctypes.c_float), ("rc", ctypes.c_float)]


class pi_cells_view(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("n_cells", ctypes.c_int64), ("grid", pi_grid),
                ("counts", ctypes.c_void_p), ("offsets", ctypes.c_void_p),
                ("perm", ctypes.c_void_p), ("cell", ctypes.c_void_p),
                ("xs", ctypes.c_void_p), ("ys", ctypes.c_void_p), ("zs", ctypes.c_void_p),
                ("ws", ctypes.c_void_p), ("max_per_cell", ctypes.c_void_p)]


class pi_interact_opts(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("sweep", ctypes.c_int32),
                ("order", ctypes.c_int32), ("tile", ctypes.c_int32 * 3)]


class pi_invariants(ctypes.Structure):
    _fields_ = [("pairs", ctypes.c_int64), ("net", ctypes.c_double * 3),
                ("scale", ctypes.c_double), ("rho_sum", ctypes.c_double)]


class pi_kernel_time(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 48), ("launches", ctypes.c_int64), ("total_ms", ctypes.c_double)]


INV_BYTES = ctypes.sizeof(pi_invariants)

_LIB = None

# (name, restype, argtypes)
_P = ctypes.c_void_p
_SIGS = [
    ("pi_status_str", ctypes.c_char_p, [ctypes.c_int32]),
    ("pi_version", ctypes.c_char_p, []),
    ("pi_ctx_create", ctypes.c_int32, [ctypes.c_int32, ctypes.POINTER(_P)]),
    ("pi_ctx_destroy", ctypes.c_int32, [_P]),
    ("pi_cells_create", ctypes.c_int32, [_P, ctypes.POINTER(_P)]),
    ("pi_cells_destroy", ctypes.c_int32, [_P]),
    ("pi_bin", ctypes.c_int32, [_P, _P, _P, _P, _P, _P, ctypes.c_int64, ctypes.POINTER(pi_grid), _P]),
    ("pi_cells_get_view", ctypes.c_int32, [_P, ctypes.POINTER(pi_cells_view)]),
    ("pi_interact", ctypes.c_int32, [_P, _P, ctypes.POINTER(pi_interact_opts), _P, _P, _P, _P, _P, _P, _P]),
    ("pi_sync", ctypes.c_int32, [_P, _P, _P]),
    ("pi_timing_enable", ctypes.c_int32, [_P, ctypes.c_int32]),
    ("pi_timing_read", ctypes.c_int32, [_P, ctypes.POINTER(pi_kernel_time), ctypes.c_int32,
                                        ctypes.POINTER(ctypes.c_int32)]),
    ("pi_timing_reset", ctypes.c_int32, [_P]),
]

# Every symbol include/pi.h declares (checked by the CPU test suite).
EXPORTS = [s[0] for s in _SIGS]


def _lib():
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_2406_16091_amd.build` (no CPU fallback exists)")
        lib = ctypes.CDLL(LIB_PATH)
        for name, res, args in _SIGS:
            f = getattr(lib, name)
            f.restype = res
            f.argtypes = args
        _LIB = lib
    return _LIB


def load():
    """Load libpi.so (raises ImportError if it is missing)."""
    return _lib()


def _ptr(t):
    if t is None:
        return None
    if isinstance(t, int):
        return t
    if isinstance(t, torch.Tensor):
        if not t.is_cuda:
            raise ValueError("device buffers must be CUDA (HIP) tensors")
        if not t.is_contiguous():
            raise ValueError("device buffers must be contiguous")
        return t.data_ptr()
    raise TypeError(f"not a device buffer: {type(t)}")


def _stream(s):
    if s is None:
        return torch.cuda.current_stream().cuda_stream
    if isinstance(s, int):
        return s
    return s.cuda_stream


def _check(st, what):
    if st != PI_OK:
        raise PiError(st, what)


def make_grid(origin, dims, cell_w, rc) -> pi_grid:
    g = pi_grid()
    for a in range(3):
        g.origin[a] = float(origin[a])
        g.dims[a] = int(dims[a])
    g.cell_w = float(cell_w)
    g.rc = float(rc)
    return g


def pi_version() -> str:
    return _lib().pi_version().decode()


def pi_ctx_create(device: int = 0):
    h = _P()
    _check(_lib().pi_ctx_create(int(device), ctypes.byref(h)), "pi_ctx_create")
    return h


def pi_ctx_destroy(ctx):
    _check(_lib().pi_ctx_destroy(ctx), "pi_ctx_destroy")


def pi_cells_create(ctx):
    h = _P()
    _check(_lib().pi_cells_create(ctx, ctypes.byref(h)), "pi_cells_create")
    return h


def pi_cells_destroy(cells):
    _check(_lib().pi_cells_destroy(cells), "pi_cells_destroy")


def pi_bin(ctx, cells, x, y, z, w, n, grid: pi_grid, stream=None):
    _check(_lib().pi_bin(ctx, cells, _ptr(x), _ptr(y), _ptr(z), _ptr(w), int(n),
                         ctypes.byref(grid), _stream(stream)), "pi_bin")


def pi_cells_get_view(cells) -> pi_cells_view:
    v = pi_cells_view()
    _check(_lib().pi_cells_get_view(cells, ctypes.byref(v)), "pi_cells_get_view")
    return v


def make_opts(precision="compensated", sweep="auto", order="sorted", tile=(0, 0, 0)):
    o = pi_interact_opts()
    o.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    o.sweep = SWEEPS[sweep] if isinstance(sweep, str) else int(sweep)
    o.order = {"sorted": PI_ORDER_SORTED, "original": PI_ORDER_ORIGINAL}[order] \
        if isinstance(order, str) else int(order)
    for a in range(3):
        o.tile[a] = int(tile[a])
    return o


def pi_interact(ctx, cells, opts, rho, gx, gy, gz, count, inv=None, stream=None):
    _check(_lib().pi_interact(ctx, cells, ctypes.byref(opts) if opts is not None else None,
                              _ptr(rho), _ptr(gx), _ptr(gy), _ptr(gz), _ptr(count), _ptr(inv),
                              _stream(stream)), "pi_interact")


def pi_sync(ctx, cells=None, stream=None):
    _check(_lib().pi_sync(ctx, cells, _stream(stream)), "pi_sync")


def pi_timing_enable(ctx, on=True):
    _check(_lib().pi_timing_enable(ctx, 1 if on else 0), "pi_timing_enable")


def pi_timing_reset(ctx):
    _check(_lib().pi_timing_reset(ctx), "pi_timing_reset")


def pi_timing_read(ctx, max_kernels=64) -> dict:
    """{kernel name: (launches, total_ms)} since the last reset (waits for
    the recorded events)."""
    buf = (pi_kernel_time * max_kernels)()
    n = ctypes.c_int32(0)
    _check(_lib().pi_timing_read(ctx, buf, max_kernels, ctypes.byref(n)), "pi_timing_read")
    return {buf[i].name.decode(): (int(buf[i].launches), float(buf[i].total_ms)) for i in range(n.value)}


def pi_status_str(st: int) -> str:
    return _lib().pi_status_str(int(st)).decode()


def read_invariants(inv_tensor) -> dict:
    """Decode a device pi_invariants buffer (uint8 tensor of INV_BYTES)."""
    raw = bytes(inv_tensor.cpu().numpy().tobytes())
    s = pi_invariants.from_buffer_copy(raw[:INV_BYTES])
    return {"pairs": int(s.pairs), "net": [s.net[0], s.net[1], s.net[2]],
            "scale": float(s.scale), "rho_sum": float(s.rho_sum)}

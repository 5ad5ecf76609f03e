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

PI_OK, PI_EINVAL, PI_ENOMEM, PI_ERANGE, PI_EDEVICE, PI_EAGAIN, PI_ENOTFOUND, PI_ESTATE, PI_ESTEP = \
    0, -1, -2, -3, -4, -5, -6, -7, -8
PI_PREC_COMPENSATED, PI_PREC_PLAIN, PI_PREC_FP64ACC = 0, 1, 2
PI_SWEEP_AUTO, PI_SWEEP_NOLDS, PI_SWEEP_PENCIL, PI_SWEEP_SUBBOX, PI_SWEEP_STREAM, PI_SWEEP_PENCILREG, PI_SWEEP_CELL = \
    0, 1, 2, 3, 4, 5, 6
PI_ORDER_SORTED, PI_ORDER_ORIGINAL = 0, 1
PI_NOALLOC_SCRATCH_RECORDS = 1 << 19
PI_PAIRFN_LJ, PI_PAIRFN_LOWFLOP, PI_PAIRFN_HIGHFLOP = 1, 2, 3
PAIRFNS = {"lj": PI_PAIRFN_LJ, "lowflop": PI_PAIRFN_LOWFLOP, "highflop": PI_PAIRFN_HIGHFLOP}

PRECISIONS = {"compensated": PI_PREC_COMPENSATED, "plain": PI_PREC_PLAIN, "fp64acc": PI_PREC_FP64ACC}
SWEEPS = {"auto": PI_SWEEP_AUTO, "nolds": PI_SWEEP_NOLDS, "pencil": PI_SWEEP_PENCIL,
          "subbox": PI_SWEEP_SUBBOX, "stream": PI_SWEEP_STREAM, "pencilreg": PI_SWEEP_PENCILREG,
          "cell": PI_SWEEP_CELL}


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


class pi_pairfn_opts(ctypes.Structure):
    _fields_ = [("kernel", ctypes.c_int32), ("precision", ctypes.c_int32), ("sweep", ctypes.c_int32),
                ("order", ctypes.c_int32), ("tile", ctypes.c_int32 * 3), ("sigma", ctypes.c_float),
                ("eps", ctypes.c_float), ("e0", ctypes.c_float)]


class pi_step_opts(ctypes.Structure):
    _fields_ = [("dt", ctypes.c_float), ("kappa", ctypes.c_float), ("lattice", ctypes.c_float),
                ("precision", ctypes.c_int32), ("sweep", ctypes.c_int32), ("tile", ctypes.c_int32 * 3)]


class pi_invariants(ctypes.Structure):
    _fields_ = [("pairs", ctypes.c_int64), ("net", ctypes.c_double * 3),
                ("scale", ctypes.c_double), ("rho_sum", ctypes.c_double)]


class pi_system_desc(ctypes.Structure):
    _fields_ = [("offset", ctypes.c_int64), ("n", ctypes.c_int64), ("grid", pi_grid)]


class pi_server_opts(ctypes.Structure):
    _fields_ = [("hbm_budget", ctypes.c_int64), ("max_slots", ctypes.c_int32), ("n_streams", ctypes.c_int32),
                ("queue_capacity", ctypes.c_int32), ("pad", ctypes.c_int32)]


class pi_request(ctypes.Structure):
    _fields_ = [("x", ctypes.c_void_p), ("y", ctypes.c_void_p), ("z", ctypes.c_void_p), ("w", ctypes.c_void_p),
                ("n", ctypes.c_int64), ("grid", pi_grid), ("n_sweeps", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("sweep", ctypes.c_int32), ("jitter_sigma", ctypes.c_float),
                ("lattice", ctypes.c_float), ("pad", ctypes.c_int32), ("seed", ctypes.c_uint64)]


class pi_result(ctypes.Structure):
    _fields_ = [("done", ctypes.c_int32), ("status", ctypes.c_int32), ("n", ctypes.c_int64),
                ("sweeps", ctypes.c_int32), ("pad", ctypes.c_int32), ("pairs_total", ctypes.c_int64),
                ("t_submit", ctypes.c_double), ("t_start", ctypes.c_double), ("t_done", ctypes.c_double),
                ("rho", ctypes.c_void_p), ("gx", ctypes.c_void_p), ("gy", ctypes.c_void_p),
                ("gz", ctypes.c_void_p), ("count", ctypes.c_void_p), ("x", ctypes.c_void_p),
                ("y", ctypes.c_void_p), ("z", ctypes.c_void_p), ("invariants", ctypes.c_void_p)]


class pi_server_stats_t(ctypes.Structure):
    _fields_ = [("queued", ctypes.c_int32), ("running", ctypes.c_int32), ("hbm_in_use", ctypes.c_int64)]


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
    ("pi_interact_noalloc", ctypes.c_int32, [_P, _P, ctypes.POINTER(pi_interact_opts), _P, _P, _P, _P, _P, _P,
                                             _P]),
    ("pi_interact_pairfn", ctypes.c_int32, [_P, _P, ctypes.POINTER(pi_pairfn_opts), _P, _P, _P, _P]),
    ("pi_state_set_velocity", ctypes.c_int32, [_P, _P, _P, _P, _P, _P]),
    ("pi_step", ctypes.c_int32, [_P, _P, ctypes.POINTER(pi_step_opts), _P, _P]),
    ("pi_state_get", ctypes.c_int32, [_P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P]),
    ("pi_sync", ctypes.c_int32, [_P, _P, _P]),
    ("pi_batch_create", ctypes.c_int32, [_P, ctypes.POINTER(_P)]),
    ("pi_batch_destroy", ctypes.c_int32, [_P]),
    ("pi_batch_run", ctypes.c_int32, [_P, _P, ctypes.c_int32, ctypes.POINTER(pi_system_desc), _P, _P, _P, _P,
                                      ctypes.POINTER(pi_interact_opts), _P, _P, _P, _P, _P, _P, _P]),
    ("pi_batch_get_view", ctypes.c_int32, [_P, ctypes.POINTER(pi_cells_view), ctypes.POINTER(ctypes.c_int64),
                                           ctypes.c_int32]),
    ("pi_batch_sync", ctypes.c_int32, [_P, _P, _P]),
    ("pi_server_create", ctypes.c_int32, [_P, ctypes.POINTER(pi_server_opts), ctypes.POINTER(_P)]),
    ("pi_server_destroy", ctypes.c_int32, [_P]),
    ("pi_submit", ctypes.c_int32, [_P, ctypes.POINTER(pi_request), ctypes.POINTER(ctypes.c_uint64)]),
    ("pi_poll", ctypes.c_int32, [_P, ctypes.c_uint64, ctypes.POINTER(pi_result)]),
    ("pi_wait", ctypes.c_int32, [_P, ctypes.c_uint64, ctypes.POINTER(pi_result)]),
    ("pi_release", ctypes.c_int32, [_P, ctypes.c_uint64]),
    ("pi_server_stats", ctypes.c_int32, [_P, ctypes.POINTER(pi_server_stats_t)]),
    ("pi_tuner_mode", ctypes.c_int32, [_P, ctypes.c_int32]),
    ("pi_tuner_choice", ctypes.c_int32, [_P, _P, ctypes.c_int32, ctypes.POINTER(pi_interact_opts), _P]),
    ("pi_timing_enable", ctypes.c_int32, [_P, ctypes.c_int32]),
    ("pi_timing_read", ctypes.c_int32, [_P, ctypes.POINTER(pi_kernel_time), ctypes.c_int32,
                                        ctypes.POINTER(ctypes.c_int32)]),
    ("pi_timing_reset", ctypes.c_int32, [_P]),
    ("pi_timing_only", ctypes.c_int32, [_P, ctypes.c_char_p]),
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


def pi_interact_noalloc(ctx, cells, opts, rho, gx, gy, gz, count, inv=None, stream=None):
    _check(_lib().pi_interact_noalloc(ctx, cells, ctypes.byref(opts) if opts is not None else None,
                                      _ptr(rho), _ptr(gx), _ptr(gy), _ptr(gz), _ptr(count), _ptr(inv),
                                      _stream(stream)), "pi_interact_noalloc")


def make_pairfn_opts(kernel="lj", precision="compensated", sweep="auto", order="sorted", tile=(0, 0, 0),
                     sigma=0.0, eps=0.0, e0=0.0):
    o = pi_pairfn_opts()
    o.kernel = PAIRFNS[kernel] if isinstance(kernel, str) else int(kernel)
    o.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    o.sweep = SWEEPS[sweep] if isinstance(sweep, str) else int(sweep)
    o.order = {"sorted": PI_ORDER_SORTED, "original": PI_ORDER_ORIGINAL}[order] \
        if isinstance(order, str) else int(order)
    for a in range(3):
        o.tile[a] = int(tile[a])
    o.sigma, o.eps, o.e0 = float(sigma), float(eps), float(e0)
    return o


def pi_interact_pairfn(ctx, cells, opts, v, count=None, inv=None, stream=None):
    _check(_lib().pi_interact_pairfn(ctx, cells, ctypes.byref(opts), _ptr(v), _ptr(count), _ptr(inv),
                                     _stream(stream)), "pi_interact_pairfn")


def make_step_opts(dt, kappa, lattice=0.0, precision="compensated", sweep="auto", tile=(0, 0, 0)):
    o = pi_step_opts()
    o.dt, o.kappa, o.lattice = float(dt), float(kappa), float(lattice)
    o.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    o.sweep = SWEEPS[sweep] if isinstance(sweep, str) else int(sweep)
    for a in range(3):
        o.tile[a] = int(tile[a])
    return o


def pi_state_set_velocity(ctx, cells, vx, vy, vz, stream=None):
    _check(_lib().pi_state_set_velocity(ctx, cells, _ptr(vx), _ptr(vy), _ptr(vz), _stream(stream)),
           "pi_state_set_velocity")


def pi_step(ctx, cells, opts, inv=None, stream=None):
    _check(_lib().pi_step(ctx, cells, ctypes.byref(opts), _ptr(inv), _stream(stream)), "pi_step")


def pi_state_get(ctx, cells, x=None, y=None, z=None, vx=None, vy=None, vz=None, rho=None, gx=None, gy=None,
                 gz=None, stream=None):
    _check(_lib().pi_state_get(ctx, cells, _ptr(x), _ptr(y), _ptr(z), _ptr(vx), _ptr(vy), _ptr(vz), _ptr(rho),
                               _ptr(gx), _ptr(gy), _ptr(gz), _stream(stream)), "pi_state_get")


def pi_sync(ctx, cells=None, stream=None):
    _check(_lib().pi_sync(ctx, cells, _stream(stream)), "pi_sync")


def pi_batch_create(ctx):
    h = _P()
    _check(_lib().pi_batch_create(ctx, ctypes.byref(h)), "pi_batch_create")
    return h


def pi_batch_destroy(batch):
    _check(_lib().pi_batch_destroy(batch), "pi_batch_destroy")


def make_system_descs(systems):
    """pi_system_desc array for systems concatenated in order."""
    arr = (pi_system_desc * len(systems))()
    off = 0
    for i, s in enumerate(systems):
        arr[i].offset = off
        arr[i].n = s.n
        arr[i].grid = make_grid(s.origin, s.dims, s.cell_w, s.rc)
        off += s.n
    return arr


def pi_batch_run(ctx, batch, descs, x, y, z, w, opts, rho, gx, gy, gz, count, inv=None, stream=None):
    _check(_lib().pi_batch_run(ctx, batch, len(descs), descs, _ptr(x), _ptr(y), _ptr(z), _ptr(w),
                               ctypes.byref(opts) if opts is not None else None, _ptr(rho), _ptr(gx),
                               _ptr(gy), _ptr(gz), _ptr(count), _ptr(inv), _stream(stream)), "pi_batch_run")


def pi_batch_get_view(batch, nsys):
    v = pi_cells_view()
    cb = (ctypes.c_int64 * nsys)()
    _check(_lib().pi_batch_get_view(batch, ctypes.byref(v), cb, nsys), "pi_batch_get_view")
    return v, [cb[i] for i in range(nsys)]


def pi_batch_sync(ctx, batch, stream=None):
    _check(_lib().pi_batch_sync(ctx, batch, _stream(stream)), "pi_batch_sync")


PI_TUNE_STATIC, PI_TUNE_TIMED = 0, 1


def pi_tuner_mode(ctx, mode):
    _check(_lib().pi_tuner_mode(ctx, int(mode)), "pi_tuner_mode")


def pi_tuner_choice(ctx, cells, precision="compensated", stream=None) -> pi_interact_opts:
    o = pi_interact_opts()
    prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    _check(_lib().pi_tuner_choice(ctx, cells, prec, ctypes.byref(o), _stream(stream)), "pi_tuner_choice")
    return o


def pi_server_create(ctx, hbm_budget=64 << 30, max_slots=8, n_streams=4, queue_capacity=1024):
    o = pi_server_opts(hbm_budget, max_slots, n_streams, queue_capacity, 0)
    h = _P()
    _check(_lib().pi_server_create(ctx, ctypes.byref(o), ctypes.byref(h)), "pi_server_create")
    return h


def pi_server_destroy(server):
    _check(_lib().pi_server_destroy(server), "pi_server_destroy")


def make_request(system, n_sweeps=1, precision="compensated", sweep="auto", jitter_sigma=0.0, lattice=0.0,
                 seed=0):
    """pi_request for a synth.System (the numpy arrays must stay alive until
    pi_submit returns; they are copied there)."""
    import numpy as np
    arrs = [np.ascontiguousarray(getattr(system, k), dtype=np.float32) for k in ("x", "y", "z", "w")]
    r = pi_request()
    r.x, r.y, r.z, r.w = (a.ctypes.data for a in arrs)
    r.n = system.n
    r.grid = make_grid(system.origin, system.dims, system.cell_w, system.rc)
    r.n_sweeps = int(n_sweeps)
    r.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    r.sweep = SWEEPS[sweep] if isinstance(sweep, str) else int(sweep)
    r.jitter_sigma = float(jitter_sigma)
    r.lattice = float(lattice)
    r.seed = int(seed)
    r._keep = arrs
    return r


def pi_submit(server, req) -> int:
    t = ctypes.c_uint64(0)
    _check(_lib().pi_submit(server, ctypes.byref(req), ctypes.byref(t)), "pi_submit")
    return int(t.value)


def pi_submit_status(server, req):
    """(status, ticket) without raising (for PI_EAGAIN / PI_ENOMEM handling)."""
    t = ctypes.c_uint64(0)
    st = _lib().pi_submit(server, ctypes.byref(req), ctypes.byref(t))
    return int(st), int(t.value)


def _result_dict(r: pi_result, copy=True):
    import numpy as np
    out = {"done": bool(r.done), "status": int(r.status), "n": int(r.n), "sweeps": int(r.sweeps),
           "pairs_total": int(r.pairs_total), "t_submit": r.t_submit, "t_start": r.t_start,
           "t_done": r.t_done}
    if r.done and r.status == PI_OK:
        n = int(r.n)

        def arr(ptr, ct, dt):
            if n == 0 or not ptr:
                return np.zeros(0, dt)
            a = np.ctypeslib.as_array(ctypes.cast(ptr, ctypes.POINTER(ct)), shape=(n,))
            return a.copy() if copy else a
        for k in ("rho", "gx", "gy", "gz", "x", "y", "z"):
            out[k] = arr(getattr(r, k), ctypes.c_float, np.float32)
        out["count"] = arr(r.count, ctypes.c_int32, np.int32)
        inv = ctypes.cast(r.invariants, ctypes.POINTER(pi_invariants))
        out["pairs_per_sweep"] = [int(inv[i].pairs) for i in range(int(r.sweeps))]
    return out


def pi_poll(server, ticket, copy=True) -> dict:
    r = pi_result()
    _check(_lib().pi_poll(server, ctypes.c_uint64(ticket), ctypes.byref(r)), "pi_poll")
    return _result_dict(r, copy)


def pi_wait(server, ticket, copy=True) -> dict:
    r = pi_result()
    _check(_lib().pi_wait(server, ctypes.c_uint64(ticket), ctypes.byref(r)), "pi_wait")
    return _result_dict(r, copy)


def pi_release(server, ticket):
    _check(_lib().pi_release(server, ctypes.c_uint64(ticket)), "pi_release")


def pi_server_stats(server) -> dict:
    st = pi_server_stats_t()
    _check(_lib().pi_server_stats(server, ctypes.byref(st)), "pi_server_stats")
    return {"queued": st.queued, "running": st.running, "hbm_in_use": st.hbm_in_use}


def pi_timing_enable(ctx, on=True):
    _check(_lib().pi_timing_enable(ctx, 1 if on else 0), "pi_timing_enable")


def pi_timing_only(ctx, name=None):
    """Time only the launches of kernel `name` (None: every launch)."""
    _check(_lib().pi_timing_only(ctx, name.encode() if name else None), "pi_timing_only")


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

"""Device-side plumbing around the C ABI: upload a system into torch CUDA
tensors, call pi_bin / pi_interact on a stream, read results back.
Marshalling only -- no arithmetic of the method happens here."""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import pi


class Context:
    """A pi_ctx on one device (created once per process and device)."""
    _cache: dict = {}

    def __init__(self, device: int = 0):
        self.device = device
        self.handle = pi.pi_ctx_create(device)

    @classmethod
    def get(cls, device: int = 0) -> "Context":
        if device not in cls._cache:
            cls._cache[device] = Context(device)
        return cls._cache[device]


class DeviceSystem:
    """One particle system resident on the GPU with its pi_cells object."""

    def __init__(self, system, device: int = 0, ctx: Context | None = None):
        self.sys = system
        self.ctx = ctx or Context.get(device)
        self.dev = torch.device("cuda", device)
        self.x = torch.from_numpy(np.ascontiguousarray(system.x)).to(self.dev)
        self.y = torch.from_numpy(np.ascontiguousarray(system.y)).to(self.dev)
        self.z = torch.from_numpy(np.ascontiguousarray(system.z)).to(self.dev)
        self.w = torch.from_numpy(np.ascontiguousarray(system.w)).to(self.dev)
        self.grid = pi.make_grid(system.origin, system.dims, system.cell_w, system.rc)
        self.cells = pi.pi_cells_create(self.ctx.handle)
        n = system.n
        f = dict(dtype=torch.float32, device=self.dev)
        self.rho = torch.empty(max(n, 1), **f)
        self.gx = torch.empty(max(n, 1), **f)
        self.gy = torch.empty(max(n, 1), **f)
        self.gz = torch.empty(max(n, 1), **f)
        self.count = torch.empty(max(n, 1), dtype=torch.int32, device=self.dev)
        self.inv = torch.zeros(pi.INV_BYTES, dtype=torch.uint8, device=self.dev)

    def close(self):
        if self.cells is not None:
            pi.pi_cells_destroy(self.cells)
            self.cells = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def bin(self, stream=None):
        pi.pi_bin(self.ctx.handle, self.cells, self.x, self.y, self.z, self.w, self.sys.n,
                  self.grid, stream)

    def interact(self, precision="compensated", sweep="auto", order="sorted", tile=(0, 0, 0),
                 invariants=True, stream=None, floats=True):
        opts = pi.make_opts(precision, sweep, order, tile)
        pi.pi_interact(self.ctx.handle, self.cells, opts,
                       self.rho if floats else None, self.gx if floats else None,
                       self.gy if floats else None, self.gz if floats else None,
                       self.count, self.inv if invariants else None, stream)

    def interact_pairfn(self, kernel="lj", precision="compensated", sweep="auto", order="sorted",
                        tile=(0, 0, 0), sigma=0.0, eps=0.0, e0=0.0, invariants=True, stream=None):
        """The timing-experiment pair kernels: v into self.rho, candidate
        counts into self.count."""
        opts = pi.make_pairfn_opts(kernel, precision, sweep, order, tile, sigma, eps, e0)
        pi.pi_interact_pairfn(self.ctx.handle, self.cells, opts, self.rho, self.count,
                              self.inv if invariants else None, stream)

    def set_velocity(self, vx, vy, vz, stream=None):
        """Velocities (numpy, input order) for time stepping."""
        self.vx, self.vy, self.vz = (torch.from_numpy(np.ascontiguousarray(v, dtype=np.float32)).to(self.dev)
                                     for v in (vx, vy, vz))
        pi.pi_state_set_velocity(self.ctx.handle, self.cells, self.vx, self.vy, self.vz, stream)

    def step(self, dt, kappa, lattice=0.0, precision="compensated", sweep="auto", tile=(0, 0, 0),
             invariants=True, stream=None):
        pi.pi_step(self.ctx.handle, self.cells, pi.make_step_opts(dt, kappa, lattice, precision, sweep, tile),
                   self.inv if invariants else None, stream)

    def state(self, forces=False):
        """Positions and velocities after the last step (numpy, input order);
        with forces, the sweep outputs of that step too."""
        n = self.sys.n
        f = dict(dtype=torch.float32, device=self.dev)
        out = {k: torch.empty(max(n, 1), **f) for k in ("x", "y", "z", "vx", "vy", "vz")}
        extra = {k: torch.empty(max(n, 1), **f) for k in ("rho", "gx", "gy", "gz")} if forces else {}
        pi.pi_state_get(self.ctx.handle, self.cells, out["x"], out["y"], out["z"], out["vx"], out["vy"],
                        out["vz"], *(extra[k] for k in ("rho", "gx", "gy", "gz")) if forces else (None,) * 4)
        pi.pi_sync(self.ctx.handle, self.cells)
        out.update(extra)
        return {k: v[:n].cpu().numpy() for k, v in out.items()}

    def sync(self, stream=None):
        pi.pi_sync(self.ctx.handle, self.cells, stream)

    def results(self):
        n = self.sys.n
        return {k: getattr(self, k)[:n].cpu().numpy() for k in ("rho", "gx", "gy", "gz", "count")}

    def invariants(self):
        return pi.read_invariants(self.inv)

    def binned(self):
        """Copies of the binned arrays (counts, offsets, perm, cell, xs, ys,
        zs, ws, max_per_cell) as numpy."""
        v = pi.pi_cells_get_view(self.cells)
        n, nc = int(v.n), int(v.n_cells)
        out = {}
        for name, cnt, dt in (("counts", nc, torch.int32), ("offsets", nc + 1, torch.int32),
                              ("perm", n, torch.int32), ("cell", n, torch.int32),
                              ("xs", n, torch.float32), ("ys", n, torch.float32),
                              ("zs", n, torch.float32), ("ws", n, torch.float32),
                              ("max_per_cell", 1, torch.int32)):
            t = torch.empty(max(cnt, 1), dtype=dt, device=self.dev)
            ptr = getattr(v, name)
            if cnt > 0:
                nbytes = cnt * 4
                # device-to-device copy through the HIP runtime torch uses
                torch.cuda.synchronize(self.dev)
                _copy_d2d(t.data_ptr(), ptr, nbytes)
            out[name] = t[:cnt].cpu().numpy()
        out["max_per_cell"] = int(out["max_per_cell"][0])
        return out


_hip = None


def _copy_d2d(dst: int, src: int, nbytes: int):
    """hipMemcpy device-to-device between two raw pointers (the view's
    buffers belong to the library, not to torch)."""
    global _hip
    if _hip is None:
        import os
        lib = None
        for cand in ("libamdhip64.so.7", "libamdhip64.so"):
            try:
                lib = ctypes.CDLL(cand)
                break
            except OSError:
                continue
        if lib is None:
            tl = os.path.join(os.path.dirname(torch.__file__), "lib", "libamdhip64.so")
            lib = ctypes.CDLL(tl)
        lib.hipMemcpy.restype = ctypes.c_int
        lib.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
        _hip = lib
    st = _hip.hipMemcpy(ctypes.c_void_p(dst), ctypes.c_void_p(src), ctypes.c_size_t(nbytes), 3)
    if st != 0:
        raise RuntimeError(f"hipMemcpy failed: {st}")


class DeviceBatch:
    """Many systems concatenated on the GPU and run through pi_batch_run."""

    def __init__(self, systems, device: int = 0, ctx: Context | None = None):
        self.systems = list(systems)
        self.ctx = ctx or Context.get(device)
        self.dev = torch.device("cuda", device)
        cat = lambda k: torch.from_numpy(np.ascontiguousarray(
            np.concatenate([getattr(s, k) for s in self.systems]).astype(np.float32))).to(self.dev)
        self.x, self.y, self.z, self.w = cat("x"), cat("y"), cat("z"), cat("w")
        self.descs = pi.make_system_descs(self.systems)
        self.offsets = [int(self.descs[i].offset) for i in range(len(self.systems))]
        n = sum(s.n for s in self.systems)
        self.n = n
        f = dict(dtype=torch.float32, device=self.dev)
        self.rho = torch.empty(max(n, 1), **f)
        self.gx = torch.empty(max(n, 1), **f)
        self.gy = torch.empty(max(n, 1), **f)
        self.gz = torch.empty(max(n, 1), **f)
        self.count = torch.empty(max(n, 1), dtype=torch.int32, device=self.dev)
        self.inv = torch.zeros(pi.INV_BYTES * len(self.systems), dtype=torch.uint8, device=self.dev)
        self.batch = pi.pi_batch_create(self.ctx.handle)

    def close(self):
        if self.batch is not None:
            pi.pi_batch_destroy(self.batch)
            self.batch = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def run(self, precision="compensated", sweep="auto", order="original", tile=(0, 0, 0), stream=None):
        opts = pi.make_opts(precision, sweep, order, tile)
        pi.pi_batch_run(self.ctx.handle, self.batch, self.descs, self.x, self.y, self.z, self.w, opts,
                        self.rho, self.gx, self.gy, self.gz, self.count, self.inv, stream)

    def sync(self, stream=None):
        pi.pi_batch_sync(self.ctx.handle, self.batch, stream)

    def results(self):
        """Per-system dicts of numpy outputs (original order)."""
        allr = {k: getattr(self, k)[:self.n].cpu().numpy() for k in ("rho", "gx", "gy", "gz", "count")}
        out = []
        for s, off in zip(self.systems, self.offsets):
            out.append({k: v[off:off + s.n] for k, v in allr.items()})
        return out

    def invariants(self):
        raw = self.inv.cpu().numpy().tobytes()
        res = []
        for i in range(len(self.systems)):
            r = pi.pi_invariants.from_buffer_copy(raw[i * pi.INV_BYTES:(i + 1) * pi.INV_BYTES])
            res.append({"pairs": int(r.pairs), "net": [r.net[0], r.net[1], r.net[2]],
                        "scale": float(r.scale), "rho_sum": float(r.rho_sum)})
        return res

    def binned(self):
        """Concatenated binned arrays and each system's first global cell."""
        v, cell_base = pi.pi_batch_get_view(self.batch, len(self.systems))
        n, nc = int(v.n), int(v.n_cells)
        out = {}
        torch.cuda.synchronize(self.dev)
        for name, cnt, dt in (("counts", nc, torch.int32), ("offsets", nc + 1, torch.int32),
                              ("perm", n, torch.int32), ("cell", n, torch.int32),
                              ("xs", n, torch.float32), ("ys", n, torch.float32),
                              ("zs", n, torch.float32), ("ws", n, torch.float32)):
            t = torch.empty(max(cnt, 1), dtype=dt, device=self.dev)
            if cnt > 0:
                _copy_d2d(t.data_ptr(), getattr(v, name), cnt * 4)
            out[name] = t[:cnt].cpu().numpy()
        out["cell_base"] = cell_base
        return out

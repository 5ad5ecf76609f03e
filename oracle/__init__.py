"""FP64 CPU oracle (test infrastructure only).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product library never does; it
shares no code with it.  The arithmetic lives in ``oracle.c`` (plain C, FP64,
OpenMP over targets); this module only builds and marshals.

Functions follow the paper (arXiv 2406.16091):
  * :func:`bin_particles` -- Sec. 2 binning (cell id, counts, exclusive prefix
    sum of Fig. 1, stable scatter into cell-sorted order);
  * :func:`sweep` -- the 27-neighbour-cell sweep of Sec. 2 / Algorithm 1 with
    the cubic B-spline kernel, over all targets or a subset;
  * :func:`brute` -- the plain O(N^2) definition of Sec. 2 (all pairs i != j
    with r_ij < r_c), no grid;
  * :func:`kernel` -- the B-spline W(r) and dW/dr;
  * :func:`sweep_pairfn` / :func:`brute_pairfn` -- the kernels of the paper's
    timing experiments (Sec. 7.1 Lennard-Jones with softening, Fig. 8's low-
    and high-FLOP kernels) over every candidate of the 27-cell stencil;
  * :func:`euler_step` / :func:`pair_energy` -- the position update that ends
    the pipeline of Sec. 2 (one symplectic Euler step with the B-spline as a
    soft pair potential) and that potential's energy.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

OK, EINVAL, ERANGE = 0, -1, -3


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so with gcc (no fast-math, no FMA
    contraction: float32 decisions must round exactly as written)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-std=gnu11", "-fPIC", "-shared", "-fopenmp",
               "-ffp-contract=off", "-fno-fast-math", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None

# A test that plants mistakes in the oracle (tests/test_oracle_mutants.py)
# compiles altered copies of oracle.c elsewhere and points this variable at
# one of them, to show that the pins fail on it.
_OVERRIDE = "ORACLE_LIBRARY"


def _load():
    global _lib
    if _lib is None:
        path = os.environ.get(_OVERRIDE)
        if not path:
            path = _LIB
            if not os.path.exists(path):
                build()
        lib = ctypes.CDLL(path)
        P = ctypes.c_void_p
        I64 = ctypes.c_int64
        lib.oracle_kernel.argtypes = [ctypes.c_double, ctypes.c_double, P, P]
        lib.oracle_kernel.restype = None
        lib.oracle_cells.argtypes = [I64, P, P, P, P, P, ctypes.c_float, P]
        lib.oracle_cells.restype = ctypes.c_int
        lib.oracle_bin.argtypes = [I64, P, P, P, P, P, P, ctypes.c_float, ctypes.c_float,
                                   P, P, P, P, P, P, P, P, P]
        lib.oracle_bin.restype = ctypes.c_int
        lib.oracle_sweep.argtypes = [I64, P, P, P, P, P, ctypes.c_float, P, P, P,
                                     I64, P, P, P, P, P, P, P, P, ctypes.c_int]
        lib.oracle_sweep.restype = ctypes.c_int
        lib.oracle_brute.argtypes = [I64, P, P, P, P, ctypes.c_float, I64, P,
                                     P, P, P, P, P, P, ctypes.c_int]
        lib.oracle_brute.restype = ctypes.c_int
        lib.oracle_sweep_pairfn.argtypes = [ctypes.c_int, I64, P, P, P, P, ctypes.c_double, ctypes.c_double,
                                            ctypes.c_double, P, P, P, I64, P, P, P, P, ctypes.c_int]
        lib.oracle_sweep_pairfn.restype = ctypes.c_int
        lib.oracle_brute_pairfn.argtypes = [ctypes.c_int, I64, P, P, P, P, ctypes.c_double, ctypes.c_double,
                                            ctypes.c_double, P, I64, P, P, P, P, ctypes.c_int]
        lib.oracle_brute_pairfn.restype = ctypes.c_int
        lib.oracle_max_threads.argtypes = []
        lib.oracle_max_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


class OracleError(RuntimeError):
    def __init__(self, status):
        super().__init__(f"oracle status {status}")
        self.status = status


def max_threads() -> int:
    return int(_load().oracle_max_threads())


def kernel(r: float, h: float):
    """(W(r), dW/dr) of the cubic B-spline with support h."""
    W = ctypes.c_double()
    dW = ctypes.c_double()
    _load().oracle_kernel(float(r), float(h), ctypes.byref(W), ctypes.byref(dW))
    return W.value, dW.value


def cells(x, y, z, origin, dims, cell_w):
    x, y, z = _f32(x), _f32(y), _f32(z)
    n = x.shape[0]
    o = _f32(origin)
    d = np.ascontiguousarray(dims, dtype=np.int32)
    out = np.empty(n, dtype=np.int32)
    st = _load().oracle_cells(n, _p(x), _p(y), _p(z), _p(o), _p(d), float(cell_w), _p(out))
    return st, out


@dataclass
class Binned:
    cell: np.ndarray      # int32 [n]  cell of each particle (original order)
    counts: np.ndarray    # int32 [n_cells]
    offsets: np.ndarray   # int32 [n_cells + 1], exclusive, last = n
    perm: np.ndarray      # int32 [n]  original index of the k-th sorted particle
    xs: np.ndarray        # float32 [n] cell-relative, sorted order
    ys: np.ndarray
    zs: np.ndarray
    ws: np.ndarray
    max_per_cell: int


def bin_particles(x, y, z, w, origin, dims, cell_w, rc) -> Binned:
    x, y, z, w = _f32(x), _f32(y), _f32(z), _f32(w)
    n = x.shape[0]
    o = _f32(origin)
    d = np.ascontiguousarray(dims, dtype=np.int32)
    nc = int(d[0]) * int(d[1]) * int(d[2])
    cell = np.empty(n, np.int32)
    counts = np.empty(max(nc, 0), np.int32)
    offsets = np.empty(max(nc, 0) + 1, np.int32)
    perm = np.empty(n, np.int32)
    xs, ys, zs, ws = (np.empty(n, np.float32) for _ in range(4))
    mc = ctypes.c_int32(0)
    st = _load().oracle_bin(n, _p(x), _p(y), _p(z), _p(w), _p(o), _p(d),
                            float(cell_w), float(rc), _p(cell), _p(counts), _p(offsets),
                            _p(perm), _p(xs), _p(ys), _p(zs), _p(ws), ctypes.byref(mc))
    if st != OK:
        raise OracleError(st)
    return Binned(cell, counts, offsets, perm, xs, ys, zs, ws, int(mc.value))


@dataclass
class SweepOut:
    rho: np.ndarray     # float64 [t]
    gx: np.ndarray
    gy: np.ndarray
    gz: np.ndarray
    ascale: np.ndarray  # float64 [t]  sum_j w_j |W'(r_ij)|
    count: np.ndarray   # int64 [t]
    cand: np.ndarray | None  # int64 [t] candidates in the clipped 27-cell stencil


def sweep(x, y, z, w, dims, rc, binned: Binned, targets=None, nthreads: int = 0) -> SweepOut:
    x, y, z, w = _f32(x), _f32(y), _f32(z), _f32(w)
    n = x.shape[0]
    d = np.ascontiguousarray(dims, dtype=np.int32)
    tg = None if targets is None else np.ascontiguousarray(targets, dtype=np.int64)
    nt = n if tg is None else tg.shape[0]
    rho, gx, gy, gz, a = (np.empty(nt, np.float64) for _ in range(5))
    cnt = np.empty(nt, np.int64)
    cand = np.empty(nt, np.int64)
    st = _load().oracle_sweep(n, _p(x), _p(y), _p(z), _p(w), _p(d), float(rc),
                              _p(binned.cell), _p(binned.offsets), _p(binned.perm),
                              nt, _p(tg), _p(rho), _p(gx), _p(gy), _p(gz), _p(a),
                              _p(cnt), _p(cand), int(nthreads))
    if st != OK:
        raise OracleError(st)
    return SweepOut(rho, gx, gy, gz, a, cnt, cand)


def brute(x, y, z, w, rc, targets=None, nthreads: int = 0) -> SweepOut:
    x, y, z, w = _f32(x), _f32(y), _f32(z), _f32(w)
    n = x.shape[0]
    tg = None if targets is None else np.ascontiguousarray(targets, dtype=np.int64)
    nt = n if tg is None else tg.shape[0]
    rho, gx, gy, gz, a = (np.empty(nt, np.float64) for _ in range(5))
    cnt = np.empty(nt, np.int64)
    st = _load().oracle_brute(n, _p(x), _p(y), _p(z), _p(w), float(rc), nt, _p(tg),
                              _p(rho), _p(gx), _p(gy), _p(gz), _p(a), _p(cnt), int(nthreads))
    if st != OK:
        raise OracleError(st)
    return SweepOut(rho, gx, gy, gz, a, cnt, None)


PAIRFN = {"lj": 1, "lowflop": 2, "highflop": 3}


@dataclass
class PairfnOut:
    v: np.ndarray       # float64 [t]  sum_j K(i, j) over the candidates
    ascale: np.ndarray  # float64 [t]  sum_j |terms| (condition scale)
    cand: np.ndarray    # int64 [t]    candidates j != i in the clipped 27-cell stencil


def sweep_pairfn(kind, x, y, z, dims, sigma, eps, e0, binned: Binned, targets=None,
                 nthreads: int = 0) -> PairfnOut:
    """The paper's timing-experiment kernels (Sec. 7.1 Lennard-Jones with
    softening; Fig. 8's low- and high-FLOP kernels) over every candidate of
    the 27-cell stencil, cell-list order."""
    x, y, z = _f32(x), _f32(y), _f32(z)
    n = x.shape[0]
    d = np.ascontiguousarray(dims, dtype=np.int32)
    tg = None if targets is None else np.ascontiguousarray(targets, dtype=np.int64)
    nt = n if tg is None else tg.shape[0]
    v, a = np.empty(nt, np.float64), np.empty(nt, np.float64)
    cand = np.empty(nt, np.int64)
    st = _load().oracle_sweep_pairfn(PAIRFN[kind], n, _p(x), _p(y), _p(z), _p(d), float(sigma), float(eps),
                                     float(e0), _p(binned.cell), _p(binned.offsets), _p(binned.perm),
                                     nt, _p(tg), _p(v), _p(a), _p(cand), int(nthreads))
    if st != OK:
        raise OracleError(st)
    return PairfnOut(v, a, cand)


def brute_pairfn(kind, x, y, z, dims, sigma, eps, e0, cell, targets=None, nthreads: int = 0) -> PairfnOut:
    """The same sums from the neighbour-cell definition, O(N^2), no cell list."""
    x, y, z = _f32(x), _f32(y), _f32(z)
    n = x.shape[0]
    d = np.ascontiguousarray(dims, dtype=np.int32)
    c = np.ascontiguousarray(cell, dtype=np.int32)
    tg = None if targets is None else np.ascontiguousarray(targets, dtype=np.int64)
    nt = n if tg is None else tg.shape[0]
    v, a = np.empty(nt, np.float64), np.empty(nt, np.float64)
    cand = np.empty(nt, np.int64)
    st = _load().oracle_brute_pairfn(PAIRFN[kind], n, _p(x), _p(y), _p(z), _p(d), float(sigma), float(eps),
                                     float(e0), _p(c), nt, _p(tg), _p(v), _p(a), _p(cand), int(nthreads))
    if st != OK:
        raise OracleError(st)
    return PairfnOut(v, a, cand)


def euler_step(x, y, z, vx, vy, vz, gx, gy, gz, dt, kappa, origin, dims, cell_w, lattice=0.0):
    """One time step (Sec. 2: interactions, then the positions are updated)
    in FP64 from the FP64 sweep outputs G at the current positions, with the
    B-spline taken as a soft pair potential E = (kappa/2) sum_i sum_{j!=i}
    w_i w_j W(r_ij) and w_i the mass: the acceleration is -kappa G_i.
    Symplectic Euler per axis: v' = v - dt kappa G, displacement dt v' cut to
    half a cell width, reflection at the box faces (the velocity flips), the
    coordinate measured from the origin rounded down to the lattice (if > 0)
    and kept at most one lattice step below the far face.  Returns
    (positions, velocities, cut) as float64 arrays [3, n] and a bool array of
    particles whose displacement was cut."""
    L = np.asarray(dims, np.float64) * float(cell_w)
    o = np.asarray(origin, np.float64)
    pos = np.stack([np.asarray(a, np.float64) for a in (x, y, z)])
    vel = np.stack([np.asarray(a, np.float64) for a in (vx, vy, vz)])
    acc = -float(kappa) * np.stack([np.asarray(a, np.float64) for a in (gx, gy, gz)])
    vel = vel + float(dt) * acc
    d = float(dt) * vel
    half = 0.5 * float(cell_w)
    cut = np.abs(d) > half
    d = np.where(cut, np.copysign(half, d), d)
    u = pos - o[:, None] + d
    low = u < 0
    u = np.where(low, -u, u)
    vel = np.where(low, -vel, vel)
    high = u >= L[:, None]
    u = np.where(high, 2 * L[:, None] - u, u)
    vel = np.where(high, -vel, vel)
    if lattice > 0:
        u = np.floor(u / lattice) * lattice
        u = np.clip(u, 0.0, L[:, None] - lattice)
    return o[:, None] + u, vel, cut.any(axis=0)


def pair_energy(w, rho, kappa):
    """E = (kappa/2) sum_i w_i rho_i: the soft pair potential of the time
    step, from the sweep's rho_i = sum_{j != i} w_j W(r_ij)."""
    return 0.5 * float(kappa) * float(np.dot(np.asarray(w, np.float64), np.asarray(rho, np.float64)))


def invariants(w, out: SweepOut):
    """Global invariants of a full sweep (targets in original order):
    P = sum_i count_i, F = sum_i w_i G_i (zero by Newton's third law on the
    antisymmetric pair terms), S = sum_i w_i A_i (scale for F)."""
    w = np.asarray(w, dtype=np.float64)
    P = int(out.count.sum())
    F = np.array([(w * out.gx).sum(), (w * out.gy).sum(), (w * out.gz).sum()])
    S = float((w * out.ascale).sum())
    return P, F, S

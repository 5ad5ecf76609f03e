"""The method's edge cases through the HIP path (C ABI), element by element
against the FP64 oracle, for every sweep organisation and every precision.

Geometries (Sec. 2: every pair i != j with r_ij < r_c, strict):
  * pairs at r = r_c exactly -- on an axis, in a plane (3-4-5) and along a
    3-D diagonal (2-3-6-7) -- which must be excluded, and the same pairs one
    lattice step closer, which must be included;
  * coincident distinct particles (r = 0): they count and add w_j W(0) to
    rho, with no gradient term;
  * 3,000 lattice pairs within a few lattice steps of the cutoff shell, so
    that the float32 filter's exact in-band test decides many pairs;
  * particles exactly on cell faces and at the box's far corner;
  * a cutoff smaller than the cell width (the reach trimming of the tiles).
All of them sit on one power-of-two lattice with a cell width that is a
multiple of it, so the exact predicate applies: counts and the pair total are
compared bit for bit.

A second group sweeps a cell width of 0.1 with off-lattice float32
positions.  There the cell-relative coordinates are rounded (once in the
binning, once more where a tile stages them relative to its halo corner), so
each organisation computes the pair differences with an absolute error of at
most delta per pair (derived in _frame_band from the extent of the frame it
computes in).  Every count must then lie between the oracle's counts at
r_c -+ delta, and the floats within the tolerance widened by what a
displacement of delta can change: delta A* for rho, 24 (sigma/h^2) delta
sum_j w_j for a component of G (|W''| and |W'/r| are both at most
12 sigma/h^2), plus the terms of pairs inside the band.

Tolerances (per output; starred values are the oracle's, A* the condition
scale sum_j w_j |W'(r_ij)|):
  COMPENSATED, FP64ACC: |rho - rho*| <= 1e-5 rho*, |G_a - G_a*| <= 1e-5 A*.
  PLAIN: its 1 - q is taken from q = sqrt(fl(r^2)) / h with an absolute error
  of at most about 5u (u = 2^-24), so W = 2 sigma (1-q)^3 is off by at most
  about 5u h |W'| per pair and each gradient component by about
  30u (sigma / h) w_j; with a margin of four:
  |rho - rho*| <= 1e-5 rho* + 2^-19 h A*,
  |G_a - G_a*| <= 1e-5 A* + 2^-16 (sigma / h) count max(w).
"""
import math
import sys

import numpy as np
import pytest

import oracle
from paper_2406_16091_amd import synth

TOL = 1e-5
SWEEPS = [("nolds", (0, 0, 0)), ("stream", (0, 0, 0)), ("pencil", (254, 1, 1)), ("pencil", (62, 1, 1)),
          ("pencil", (30, 1, 1)), ("subbox", (8, 8, 3)), ("subbox", (6, 6, 6)), ("subbox", (4, 4, 4)),
          ("subbox", (4, 4, 2)), ("subbox", (16, 4, 3)), ("subbox", (7, 7, 5)),
          ("pencilreg", (8, 8, 4)), ("pencilreg", (4, 4, 2)),
          ("cell", (1, 1, 1)), ("cell", (4, 1, 1)), ("cell", (2, 16, 1)), ("cell", (2, 32, 1)),
          ("cell", (2, 64, 1))]
PRECISIONS = ["compensated", "fp64acc", "plain"]


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2406_16091_amd import device, pi
    pi.load()
    return device


# ---------------------------------------------------------------- geometries

# cutoff = cell width = 35 * 2^-5: a multiple of 5 and of 7, so pairs at
# exactly r_c exist on the 2^-5 lattice along an axis (35, 0, 0), in a plane
# (21, 28, 0) and along a diagonal (10, 15, 30) (2-3-6-7)
RC_UNITS = 35
P_LAT = 19           # coordinates are multiples of 2^-19
G = 16               # 16^3 cells, box [0, 17.5)^3 -> indices < 17.5 * 2^19 < 2^24
EXACT_OFFSETS = [(35, 0, 0), (0, 0, 35), (21, 28, 0), (0, 21, 28), (10, 15, 30), (30, 10, 15)]
# with r_c = 0.8 of the cell width = 28 * 2^-5: axis and 2-3-6-7 diagonals
EXACT_OFFSETS_28 = [(28, 0, 0), (0, 28, 0), (8, 12, 24), (24, 8, 12)]


def _edge_system(seed, rc_scale=1.0, name="edges"):
    """The edge geometries of the module docstring in one system (indices on
    the 2^-19 lattice); rc = rc_scale * cell width."""
    rng = np.random.default_rng(seed)
    cw = RC_UNITS * 2.0 ** -5
    rc = cw * rc_scale
    unit = 1 << (P_LAT - 5)            # one 2^-5 step in lattice units
    k_rc = int(round(rc * 2 ** P_LAT))
    hi = G * RC_UNITS * unit           # box end in lattice units
    pts = []
    # exact-r_c pairs (excluded) and the same one lattice step closer (included)
    for (a, b, c) in (EXACT_OFFSETS if rc_scale == 1.0 else EXACT_OFFSETS_28):
        off = np.array([a, b, c], np.int64) * unit
        assert a * a + b * b + c * c == (k_rc // unit) ** 2
        for closer in (0, 1):
            base = rng.integers(2 * k_rc, hi - 2 * k_rc, size=3)
            part = base + off
            if closer:
                ax = int(np.argmax(off))
                part[ax] -= 1
            pts += [base, part]
    # coincident distinct particles: a pair and a triple
    for mult in (2, 3):
        base = rng.integers(0, hi, size=3)
        pts += [base.copy() for _ in range(mult)]
    # near-shell lattice pairs: distance within a few lattice steps of r_c
    n_shell = 3000
    base = rng.integers(2 * k_rc, hi - 2 * k_rc, size=(n_shell, 3))
    d = rng.standard_normal((n_shell, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    off = np.round(d * k_rc).astype(np.int64) + rng.integers(-2, 3, size=(n_shell, 3))
    pts += list(base) + list(np.clip(base + off, 0, hi - 1))
    # particles on cell faces and at the far corner
    cell = RC_UNITS * unit
    for k in range(0, G + 1):
        v = min(k * cell, hi - 1)
        pts.append(np.array([v, rng.integers(0, hi), rng.integers(0, hi)]))
        pts.append(np.array([rng.integers(0, hi), v, v]))
    pts.append(np.array([hi - 1, hi - 1, hi - 1]))
    pts.append(np.array([hi - 1, hi - 1, hi - 2]))
    pts.append(np.array([0, 0, 0]))
    # a uniform background
    pts += list(rng.integers(0, hi, size=(1500, 3)))
    m = np.array(pts, np.int64)
    m = m[rng.permutation(len(m))]
    x, y, z = (m.T.astype(np.float64) * 2.0 ** -P_LAT).astype(np.float32)
    assert np.all(np.float64(x) * 2 ** P_LAT == m[:, 0])  # exact in float32
    w = (0.5 + rng.integers(0, 1 << 23, size=len(m)) * 2.0 ** -23).astype(np.float32)
    return synth.System(name, x, y, z, w, (0.0, 0.0, 0.0), (G, G, G), cw, rc)


EDGE = {
    "edges_rc_eq_w": lambda: _edge_system(501),
    "edges_rc_lt_w": lambda: _edge_system(502, rc_scale=0.8),
}


def _oracle(s, rc=None):
    b = oracle.bin_particles(s.x, s.y, s.z, s.w, s.origin, s.dims, s.cell_w, s.rc)
    return b, oracle.sweep(s.x, s.y, s.z, s.w, s.dims, s.rc if rc is None else rc, b)


def _check(res, ref, s, precision):
    cnt = res["count"].astype(np.int64)
    bad = np.nonzero(cnt != ref.count)[0]
    assert bad.size == 0, f"count mismatch at {bad[:10]}: {cnt[bad[:10]]} vs {ref.count[bad[:10]]}"
    rho = res["rho"].astype(np.float64)
    h = float(s.rc)
    sigma = 8.0 / (math.pi * h ** 3)
    extra_rho = 0.0 if precision != "plain" else 2.0 ** -19 * h * ref.ascale
    extra_g = 0.0 if precision != "plain" else 2.0 ** -16 * sigma / h * ref.count * float(np.max(s.w))
    e = np.abs(rho - ref.rho)
    assert np.all(e <= TOL * ref.rho + extra_rho), \
        f"rho: worst {np.max(e - TOL * ref.rho - extra_rho)} over the bound"
    assert np.all(rho[ref.count == 0] == 0)
    for k in ("gx", "gy", "gz"):
        e = np.abs(res[k].astype(np.float64) - getattr(ref, k))
        assert np.all(e <= TOL * ref.ascale + extra_g), f"{k}: worst {np.max(e - TOL * ref.ascale - extra_g)}"


def test_edge_geometries_reach_the_oracle_pins(oracle_lib):
    """CPU check of the inputs themselves: the exact-r_c pairs are excluded
    and their one-step-closer twins included, and the shell pairs straddle
    the cutoff (so the in-band test is exercised)."""
    s = EDGE["edges_rc_eq_w"]()
    _, ref = _oracle(s)
    br = oracle.brute(s.x, s.y, s.z, s.w, s.rc)
    assert (br.count == ref.count).all()
    m = np.stack([np.float64(v) * 2 ** P_LAT for v in (s.x, s.y, s.z)], 1).astype(np.int64)
    k_rc = RC_UNITS << (P_LAT - 5)
    # count lattice pairs at exactly r_c, and within 3 steps of the shell
    from scipy.spatial import cKDTree
    t = cKDTree(m.astype(np.float64))
    pairs = t.query_pairs(k_rc + 3, output_type="ndarray")
    dd = m[pairs[:, 0]] - m[pairs[:, 1]]
    d2 = (dd * dd).sum(1)
    assert int((d2 == k_rc * k_rc).sum()) >= len(EXACT_OFFSETS)
    near = np.abs(np.sqrt(d2.astype(np.float64)) - k_rc) <= 3
    assert int(near.sum()) > 500


@pytest.mark.gpu
@pytest.mark.parametrize("case", list(EDGE))
def test_edge_cases_every_organisation_and_precision(dev, case):
    s = EDGE[case]()
    _say(f"[edges] {case} n={s.n} dims={s.dims} rc={s.rc} w={s.cell_w}")
    b, ref = _oracle(s)
    P, F, S = oracle.invariants(s.w, ref)
    ds = dev.DeviceSystem(s)
    ds.bin()
    ds.sync()
    got = ds.binned()
    assert (got["offsets"] == b.offsets).all() and (got["perm"] == b.perm).all()
    for precision in PRECISIONS:
        first = None
        for sweep, tile in SWEEPS:
            _say(f"[edges] {case} {precision} {sweep} {tile}")
            ds.interact(precision=precision, sweep=sweep, tile=tile, order="original")
            ds.sync()
            res = ds.results()
            _check(res, ref, s, precision)
            assert ds.invariants()["pairs"] == P
            if first is None:
                first = res
            else:  # lattice inputs: organisations agree bit for bit
                for k in ("rho", "gx", "gy", "gz", "count"):
                    assert (res[k].view(np.uint32) == first[k].view(np.uint32)).all(), (precision, sweep, k)
    ds.close()


@pytest.mark.gpu
def test_exact_cutoff_pairs_through_the_gpu(dev):
    """Two particles at r = r_c exactly (axis, plane, diagonal) do not
    interact; one lattice step closer they do, with rho = w_j W(r) and the
    counts the brute force gives."""
    cw = RC_UNITS * 2.0 ** -5
    unit = 1 << (P_LAT - 5)
    for (a, b, c) in EXACT_OFFSETS:
        for closer in (0, 1):
            base = np.array([3, 4, 5], np.int64) * RC_UNITS * unit + 1234
            part = base + np.array([a, b, c], np.int64) * unit
            if closer:
                part[int(np.argmax([a, b, c]))] -= 1
            m = np.stack([base, part])
            x, y, z = (m.T.astype(np.float64) * 2.0 ** -P_LAT).astype(np.float32)
            w = np.array([0.75, 1.25], np.float32)
            s = synth.System("pair", x, y, z, w, (0.0, 0.0, 0.0), (G, G, G), cw, cw)
            _, ref = _oracle(s)
            assert ref.count.tolist() == ([1, 1] if closer else [0, 0])
            ds = dev.DeviceSystem(s)
            ds.bin()
            for sweep, tile in SWEEPS:
                ds.interact(sweep=sweep, tile=tile, order="original")
                ds.sync()
                _check(ds.results(), ref, s, "compensated")
            ds.close()


# ---------------------------------------------------------------- off-lattice input

def _off_lattice(seed, n, g, cw, rc):
    rng = np.random.default_rng(seed)
    L = np.float32(g * cw)
    x, y, z = (rng.random((3, n)) * float(L)).astype(np.float32)
    w = (0.5 + rng.random(n)).astype(np.float32)
    s = synth.System("offlattice", x, y, z, w, (0.0, 0.0, 0.0), (g, g, g), cw, rc)
    st, cells = oracle.cells(x, y, z, s.origin, s.dims, s.cell_w)
    keep = cells >= 0   # float32 cell decision: drop the few on the far face
    return synth.System("offlattice", x[keep], y[keep], z[keep], w[keep], s.origin, s.dims, cw, rc)


OFF = {
    "w0.1_rc0.1": lambda: _off_lattice(601, 60000, 30, 0.1, 0.1),
    "w0.1_rc0.07": lambda: _off_lattice(602, 60000, 30, 0.1, 0.07),
    "w0.3_rc0.3_dense": lambda: _off_lattice(603, 80000, 20, 0.3, 0.3),
}


def _ulp(v):
    return 2.0 ** (math.floor(math.log2(v)) - 23)


def _frame_band(sweep, tile, cw):
    """Bound on |computed - exact| of a pair's difference vector for one
    organisation, with the origin at zero.  Each stored cell-relative
    coordinate fl(x - i w) is off by at most ulp(w) (its value lies within
    about [0, w]).  The no-LDS, stream and cell-SM walks shift the target by
    -+w and subtract, two roundings of values below 2w: at most 2 ulp(w) more
    per axis.  A tile stages both particles at fl(c w + x_rel) with c up to the
    halo's extent E_a = (T_a + 2) w, a rounding of ulp(E_a)/2 each, and then
    subtracts exactly (both on the ulp(E_a) grid, difference below 2w)."""
    if sweep in ("nolds", "stream", "cell"):
        e = [4 * _ulp(cw)] * 3
    else:
        e = [2 * _ulp(cw) + _ulp((t + 2) * cw) for t in tile]
    return math.sqrt(sum(v * v for v in e))


@pytest.mark.gpu
@pytest.mark.parametrize("case", list(OFF))
def test_off_lattice_counts_within_the_rounding_band(dev, case):
    """Off-lattice positions and a cell width that is not a power of two:
    each organisation's counts lie between the oracle's at r_c -+ delta, and
    its floats within the tolerance widened by what a displacement of delta
    changes (module docstring).  The walks that compute in the target's cell
    frame (no-LDS, stream, cell-SM) take the same roundings in the same
    order, so their outputs are bitwise equal even here."""
    s = OFF[case]()
    b, ref = _oracle(s)
    h = float(s.rc)
    sigma = 8.0 / (math.pi * h ** 3)
    wmax = float(np.max(s.w))
    ds = dev.DeviceSystem(s)
    ds.bin()
    ds.sync()
    got = ds.binned()
    assert (got["offsets"] == b.offsets).all() and (got["perm"] == b.perm).all()
    bands = {}
    differ, margin = {}, {}
    for sweep, tile in SWEEPS:
        delta = _frame_band(sweep, tile, s.cell_w)
        if delta not in bands:
            lo = oracle.sweep(s.x, s.y, s.z, s.w, s.dims, np.float32(h - delta), b).count
            hi = oracle.sweep(s.x, s.y, s.z, s.w, s.dims, np.float32(h + delta), b).count
            bands[delta] = (lo, hi)
        lo, hi = bands[delta]
        ds.interact(sweep=sweep, tile=tile, order="original")
        ds.sync()
        res = ds.results()
        cnt = res["count"].astype(np.int64)
        assert np.all(cnt >= lo) and np.all(cnt <= hi), (sweep, tile, delta)
        if sweep == "nolds":
            cell_frame = res
        elif sweep in ("stream", "cell"):
            for k in ("rho", "gx", "gy", "gz", "count"):
                assert (res[k].view(np.uint32) == cell_frame[k].view(np.uint32)).all(), (sweep, tile, k)
        differ[f"{sweep}{tile}"] = int((cnt != ref.count).sum())
        nband = (hi - lo).astype(np.float64)
        sw = wmax * ref.count
        rho_tol = (TOL * ref.rho + delta * ref.ascale + 12 * sigma / h ** 2 * delta ** 2 * sw
                   + nband * 2 * sigma * (2 * delta / h) ** 3 * wmax + 1e-30)
        g_tol = (TOL * ref.ascale + 24 * sigma / h ** 2 * delta * sw
                 + nband * 6 * sigma / h * (2 * delta / h) ** 2 * wmax + 1e-30)
        e = np.abs(res["rho"].astype(np.float64) - ref.rho)
        assert np.all(e <= rho_tol), (sweep, tile, float(np.max(e / rho_tol)))
        worst = float(np.max(e / rho_tol))
        for k in ("gx", "gy", "gz"):
            e = np.abs(res[k].astype(np.float64) - getattr(ref, k))
            assert np.all(e <= g_tol), (sweep, tile, k, float(np.max(e / g_tol)))
            worst = max(worst, float(np.max(e / g_tol)))
        margin[f"{sweep}{tile}"] = round(worst, 3)
    _say(f"[offlattice] {case}: counts differing from the exact predicate: {differ}; "
         f"largest error / bound: {margin}")


# ---------------------------------------------------------------- object state

@pytest.mark.gpu
def test_failed_bin_leaves_no_binned_system(dev):
    """A binning that fails leaves the object unbinned: the sweep and the
    view report PI_ESTATE and launch nothing; a later good binning works."""
    from paper_2406_16091_amd import pi
    s = synth.box_system(3000, 8, seed=611, lattice_log2=18)
    ds = dev.DeviceSystem(s)
    ds.bin()
    ds.interact(order="original")
    ds.sync()
    good = ds.results()
    bad = pi.make_grid((0, 0, 0), (8, 8, 8), 1.0, 1.5)  # cell narrower than the cutoff
    with pytest.raises(pi.PiError) as e:
        pi.pi_bin(ds.ctx.handle, ds.cells, ds.x, ds.y, ds.z, ds.w, s.n, bad)
    assert e.value.status == pi.PI_EINVAL
    with pytest.raises(pi.PiError) as e:
        pi.pi_interact(ds.ctx.handle, ds.cells, pi.make_opts(), ds.rho, ds.gx, ds.gy, ds.gz, ds.count)
    assert e.value.status == pi.PI_ESTATE
    with pytest.raises(pi.PiError) as e:
        pi.pi_cells_get_view(ds.cells)
    assert e.value.status == pi.PI_ESTATE
    with pytest.raises(pi.PiError) as e:
        pi.pi_tuner_choice(ds.ctx.handle, ds.cells)
    assert e.value.status == pi.PI_ESTATE
    ds.bin()
    ds.interact(order="original")
    ds.sync()
    again = ds.results()
    for k in ("rho", "gx", "gy", "gz", "count"):
        assert (again[k].view(np.uint32) == good[k].view(np.uint32)).all()
    ds.close()

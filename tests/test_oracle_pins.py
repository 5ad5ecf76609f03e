"""Pins of the FP64 oracle against facts fixed outside the oracle itself.

Each test names what fixes the expected value: the paper's worked examples
(Fig. 1, the Sec. 6 scan example, Table 1's first column), closed forms of the
B-spline, its unit integral, exact integer arithmetic on the input lattice,
Newton's third law, brute force, and statistical means of uniform systems.
"""
import math
import os

import numpy as np
import pytest
from scipy import integrate

import oracle
from paper_2406_16091_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _read_golden(name):
    out = {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            k, v = line.split(":", 1) if ":" in line else (None, line)
            if k is None:
                out.setdefault("rows", []).append([float(t) for t in v.split()])
            else:
                out.setdefault(k.strip(), []).append([float(t) for t in v.split()])
    return out


# ---------------------------------------------------------------- Fig. 1

def test_fig1_counts_and_offsets(oracle_lib):
    g = _read_golden("fig1_binning.txt")
    pts = np.array(g["particle"], dtype=np.float32)
    origin = g["origin"][0]
    dims = [int(v) for v in g["dims"][0]]
    cw = g["cell_w"][0][0]
    b = oracle.bin_particles(pts[:, 0], pts[:, 1], pts[:, 2], np.ones(len(pts)),
                             origin, dims, cw, cw)
    assert b.counts.tolist() == [int(v) for v in g["counts"][0]]
    assert b.offsets.tolist() == [int(v) for v in g["offsets"][0]]
    assert b.max_per_cell == 3
    # stable order inside each cell: ascending index of the figure's drawing order
    assert b.perm.tolist() == [0, 1, 2, 3, 4, 5, 7, 8, 6]


# ---------------------------------------------------------------- Sec. 6 scan

def _paper_tree_scan(a, downward_init_div):
    """The in-place upward/downward tree scan of Sec. 6, sequential form.
    downward_init_div = 2 is the appendix listing's restart of the downward
    pass, 4 the algorithm box's.  Returns (final, states)."""
    p = list(a)
    n = len(p)
    states = []
    js = 2
    while js <= n:
        h = js // 2
        for i in range(js - 1, n, js):
            p[i] += p[i - h]
        states.append(list(p))
        js *= 2
    js = max(4, js // downward_init_div)
    while js > 1:
        h = js // 2
        for i in range(js + h - 1, n, js):
            p[i] += p[i - h]
        states.append(list(p))
        js = h
    return p, states


def test_scan_worked_example():
    g = _read_golden("scan_vectors.txt")
    final, states = _paper_tree_scan([int(v) for v in g["input"][0]], 2)
    want = [g[k][0] for k in ("up1", "up2", "up3")]
    assert [s for s in states[:3]] == [[int(v) for v in w] for w in want]
    # the downward pass of the listing visits the 4-step level first; it is a
    # no-op on 8 entries (index 5 is the first updated), matching down1
    assert states[-2] == [int(v) for v in g["down1"][0]]
    assert final == [int(v) for v in g["down2"][0]]


def test_scan_erratum_algorithm_box():
    """The algorithm box restarts the downward pass at js/4 and leaves the
    last entry wrong for 12 ones (it stays 4); the listing (js/2) is right."""
    ones = [1] * 12
    good, _ = _paper_tree_scan(ones, 2)
    bad, _ = _paper_tree_scan(ones, 4)
    assert good == list(range(1, 13))
    assert bad[-1] == 4


def test_oracle_offsets_equal_paper_scan(oracle_lib):
    """The oracle's exclusive offsets equal the listing's inclusive tree scan
    shifted by one, for many lengths and count vectors."""
    rng = np.random.default_rng(7)
    for ncell in list(range(1, 40)) + [63, 64, 65, 127, 128, 200, 1000]:
        counts = rng.integers(0, 4, size=ncell)
        # one particle row per cell along x, cell width 1, rc = 1
        xs = np.repeat(np.arange(ncell), counts).astype(np.float64) + 0.5
        n = xs.size
        b = oracle.bin_particles(xs, np.full(n, 0.5), np.full(n, 0.5), np.ones(n),
                                 (0, 0, 0), (ncell, 1, 1), 1.0, 1.0)
        incl, _ = _paper_tree_scan(counts.tolist(), 2)
        assert b.counts.tolist() == counts.tolist()
        assert b.offsets.tolist() == [0] + incl


# ---------------------------------------------------------------- Table 1

def _table1_rows():
    rows = []
    with open(os.path.join(GOLDEN, "table1_candidates.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                d, p, v = line.split()
                rows.append((int(d), int(p), float(v)))
    return rows


@pytest.mark.parametrize("d,p,printed", [r for r in _table1_rows() if r[0] ** 3 * r[1] <= 500_000])
def test_table1_candidates(oracle_lib, d, p, printed):
    n = d ** 3 * p
    rng = np.random.default_rng(1000 + d * 7 + p)
    m = rng.integers(0, 1 << 24, size=(3, n))
    x, y, z = (m.astype(np.float64) * 2.0 ** -24).astype(np.float32)
    w = np.ones(n, np.float32)
    rc = 1.0 / d
    b = oracle.bin_particles(x, y, z, w, (0, 0, 0), (d, d, d), rc, rc)
    s = oracle.sweep(x, y, z, w, (d, d, d), rc, b)
    mean = s.cand.mean()
    if d == 2:
        # every particle's clipped stencil covers the whole 2x2x2 grid
        assert (s.cand == n - 1).all() and int(round(printed)) == n - 1
    else:
        expect = (n - 1) * ((3 * d - 2) / d ** 2) ** 3   # non-periodic clipping
        tol = 0.02 if n >= 4096 else 0.15
        assert abs(mean - printed) / printed < tol
        assert abs(mean - expect) / expect < tol


# ---------------------------------------------------------------- kernel

SIG = 8.0 / math.pi  # sigma at h = 1


@pytest.mark.parametrize("q,w_over_sigma,dw_h_over_sigma", [
    (0.0, 1.0, 0.0), (0.25, 0.71875, -1.875), (0.5, 0.25, -1.5),
    (0.75, 1.0 / 32.0, -0.375), (1.0, 0.0, 0.0), (1.5, 0.0, 0.0)])
def test_kernel_closed_forms(oracle_lib, q, w_over_sigma, dw_h_over_sigma):
    for h in (1.0, 2.0 ** -5, 3.0):
        sigma = 8.0 / (math.pi * h ** 3)
        W, dW = oracle.kernel(q * h, h)
        assert W == pytest.approx(sigma * w_over_sigma, rel=1e-14, abs=1e-300)
        assert dW == pytest.approx(sigma / h * dw_h_over_sigma, rel=1e-14, abs=1e-300)


def test_kernel_unit_integral(oracle_lib):
    for h in (1.0, 2.0 ** -5, 0.37):
        val, err = integrate.quad(lambda r: 4.0 * math.pi * r * r * oracle.kernel(r, h)[0],
                                  0.0, h, points=[0.5 * h], epsabs=0, epsrel=1e-13)
        assert val == pytest.approx(1.0, rel=1e-11)


def test_kernel_derivative_matches_finite_difference(oracle_lib):
    h = 1.0
    for r in np.linspace(0.01, 0.99, 97):
        if abs(r - 0.5) < 1e-3:
            continue
        e = 1e-6
        fd = (oracle.kernel(r + e, h)[0] - oracle.kernel(r - e, h)[0]) / (2 * e)
        assert oracle.kernel(r, h)[1] == pytest.approx(fd, rel=1e-7, abs=1e-9)


def test_kernel_continuous_at_half(oracle_lib):
    a = oracle.kernel(0.5 - 1e-12, 1.0)
    b = oracle.kernel(0.5 + 1e-12, 1.0)
    assert a[0] == pytest.approx(b[0], rel=1e-9)
    assert a[1] == pytest.approx(b[1], rel=1e-9)


# ---------------------------------------------------------------- closed-form systems

def _run(x, y, z, w, dims, cw, rc, origin=(0, 0, 0)):
    b = oracle.bin_particles(x, y, z, w, origin, dims, cw, rc)
    return b, oracle.sweep(x, y, z, w, dims, rc, b)


def test_two_particles_quarter_support(oracle_lib):
    # r = h/4 along x; h = rc = 1, unit cells, box [0,4)^3
    x = np.array([1.5, 1.75], np.float32)
    y = np.array([2.0, 2.0], np.float32)
    z = np.array([2.0, 2.0], np.float32)
    w = np.array([0.75, 1.25], np.float32)
    _, s = _run(x, y, z, w, (4, 4, 4), 1.0, 1.0)
    assert s.count.tolist() == [1, 1]
    assert s.rho[0] == pytest.approx(1.25 * SIG * 0.71875, rel=1e-14)
    assert s.rho[1] == pytest.approx(0.75 * SIG * 0.71875, rel=1e-14)
    # gradient of particle 0 points toward particle 1 (+x): -w1 W'(h/4)
    assert s.gx[0] == pytest.approx(1.25 * SIG * 1.875, rel=1e-14)
    assert s.gx[1] == pytest.approx(-0.75 * SIG * 1.875, rel=1e-14)
    assert s.gy.tolist() == [0.0, 0.0] and s.gz.tolist() == [0.0, 0.0]
    assert s.ascale[0] == pytest.approx(1.25 * SIG * 1.875, rel=1e-14)


def test_two_particles_diagonal_three_quarter(oracle_lib):
    # separation (0.375, 0.5, 0) * 1.2 -> r = 0.75 with h = 1
    x = np.array([1.0, 1.45], np.float32)
    y = np.array([1.0, 1.6], np.float32)
    z = np.array([1.0, 1.0], np.float32)
    dx, dy = float(x[0]) - float(x[1]), float(y[0]) - float(y[1])
    r = math.hypot(dx, dy)
    w = np.array([1.0, 1.0], np.float32)
    _, s = _run(x, y, z, w, (3, 3, 3), 1.0, 1.0)
    q = r
    W = 2 * SIG * (1 - q) ** 3
    dW = -6 * SIG * (1 - q) ** 2
    assert s.rho[0] == pytest.approx(W, rel=1e-12)
    assert s.gx[0] == pytest.approx(dW * dx / r, rel=1e-12)
    assert s.gy[0] == pytest.approx(dW * dy / r, rel=1e-12)


def test_coincident_particles(oracle_lib):
    x = np.array([0.5, 0.5, 2.5], np.float32)
    w = np.array([1.0, 2.0, 1.0], np.float32)
    _, s = _run(x, x, x, w, (3, 3, 3), 1.0, 1.0)
    assert s.count.tolist() == [1, 1, 0]
    assert s.rho[0] == pytest.approx(2.0 * SIG, rel=1e-15)
    assert s.rho[1] == pytest.approx(1.0 * SIG, rel=1e-15)
    assert s.rho[2] == 0.0
    assert s.gx.tolist() == [0.0, 0.0, 0.0]


def test_cutoff_is_strict_exact(oracle_lib):
    # rc = 0.625 = 5/8; (0.375, 0.5) is a 3-4-5 triangle with r == rc exactly
    rc = 0.625
    x = np.array([1.0, 1.375, 1.0, 1.625, 1.0], np.float32)
    y = np.array([1.0, 1.5, 2.5, 2.5, 3.75], np.float32)
    z = np.array([1.0, 1.0, 1.0, 1.0, 1.0], np.float32)
    # pairs: (0,1) r = rc exactly -> excluded; (2,3) r = rc on axis -> excluded
    w = np.ones(5, np.float32)
    _, s = _run(x, y, z, w, (8, 8, 8), rc, rc)
    assert s.count.tolist() == [0, 0, 0, 0, 0]
    assert oracle.brute(x, y, z, w, rc).count.tolist() == [0, 0, 0, 0, 0]
    # one lattice step closer on each: included
    u = 2.0 ** -20
    x2 = x.copy()
    x2[1] = np.float32(1.375 - u)
    x2[3] = np.float32(1.625 - u)
    _, s2 = _run(x2, y, z, w, (8, 8, 8), rc, rc)
    assert s2.count.tolist() == [1, 1, 1, 1, 0]
    assert oracle.brute(x2, y, z, w, rc).count.tolist() == [1, 1, 1, 1, 0]


def test_predicate_exact_on_lattice(oracle_lib):
    """Near-shell pairs: the oracle's FP64 test equals exact integer
    arithmetic on the lattice indices (no rounding decides a count)."""
    rng = np.random.default_rng(11)
    p = 24
    rc = 2.0 ** -5
    k_rc = int(rc * 2 ** p)
    n = 3000
    base = rng.integers(4 * k_rc, (1 << p) - 4 * k_rc, size=(n, 3))
    # partner at distance ~rc along a random direction, jittered by a few units
    d = rng.standard_normal((n, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    off = np.round(d * k_rc).astype(np.int64) + rng.integers(-2, 3, size=(n, 3))
    m = np.concatenate([base, base + off])
    m = np.clip(m, 0, (1 << p) - 1)
    x, y, z = (m.T.astype(np.float64) * 2.0 ** -p).astype(np.float32)
    w = np.ones(2 * n, np.float32)
    s = oracle.brute(x, y, z, w, rc)
    mi = np.stack([(np.float64(v) * 2 ** p).astype(np.int64) for v in (x, y, z)], 1)
    want = np.zeros(2 * n, np.int64)
    for i in range(2 * n):
        dd = mi - mi[i]
        d2 = (dd * dd).sum(1)
        d2[i] = k_rc * k_rc  # exclude self
        want[i] = int((d2 < k_rc * k_rc).sum())
    assert (s.count == want).all()


# ---------------------------------------------------------------- brute vs cells

@pytest.mark.parametrize("case", ["uniform", "clustered", "wide_cells", "offset_origin", "flat"])
def test_cells_match_brute(oracle_lib, case):
    if case == "uniform":
        s = synth.uniform_unit_cube(4096, -4, seed=3)
        sysx = (s.x, s.y, s.z, s.w, s.origin, s.dims, s.cell_w, s.rc)
    elif case == "clustered":
        s = synth.clustered(n=3000, n_blobs=4, rc_log2=-4, seed=9)
        sysx = (s.x, s.y, s.z, s.w, s.origin, s.dims, s.cell_w, s.rc)
    elif case == "wide_cells":
        s = synth.box_system(2500, 6, seed=5, lattice_log2=18)
        sysx = (s.x, s.y, s.z, s.w, s.origin, s.dims, 1.0, 0.8)
    elif case == "offset_origin":
        s = synth.box_system(2000, 7, seed=6, lattice_log2=18)
        sh = np.float32(-3.0)
        sysx = (s.x + sh, s.y + sh, s.z + sh, s.w, (-3.0, -3.0, -3.0), s.dims, 1.0, 1.0)
    else:
        s = synth.box_system(2000, 12, seed=8, lattice_log2=18)
        sysx = (s.x, s.y, (s.z * np.float32(1 / 12.0)).astype(np.float32) * 0,
                s.w, s.origin, (12, 12, 1), 1.0, 1.0)
    x, y, z, w, origin, dims, cw, rc = sysx
    b = oracle.bin_particles(x, y, z, w, origin, dims, cw, rc)
    c = oracle.sweep(x, y, z, w, dims, rc, b)
    r = oracle.brute(x, y, z, w, rc)
    assert (c.count == r.count).all()
    assert c.count.sum() > 0
    for a, bb, sc in ((c.rho, r.rho, r.rho), (c.gx, r.gx, r.ascale),
                      (c.gy, r.gy, r.ascale), (c.gz, r.gz, r.ascale)):
        assert np.all(np.abs(a - bb) <= 1e-12 * sc + 1e-300)


# ---------------------------------------------------------------- definitions

@pytest.mark.parametrize("shift", [0.0, -3.0])
def test_binning_matches_independent_definition(oracle_lib, shift):
    s = synth.box_system(5000, 9, seed=12, lattice_log2=18)
    sh = np.float32(shift)
    x, y, z = (s.x + sh, s.y + 2 * sh, s.z + 3 * sh)   # exact: lattice values
    origin = (float(sh), float(2 * sh), float(3 * sh))
    b = oracle.bin_particles(x, y, z, s.w, origin, s.dims, s.cell_w, s.rc)
    # cell: float32 floor((x - o) / w), X fastest
    ix, iy, iz = (np.floor((v - np.float32(o)) / np.float32(s.cell_w)).astype(np.int64)
                  for v, o in ((x, origin[0]), (y, origin[1]), (z, origin[2])))
    cell = ix + s.dims[0] * (iy + s.dims[1] * iz)
    assert (b.cell == cell).all()
    counts = np.bincount(cell, minlength=s.n_cells)
    assert (b.counts == counts).all()
    assert (b.offsets == np.concatenate([[0], np.cumsum(counts)])).all()
    perm = np.argsort(cell, kind="stable")
    assert (b.perm == perm).all()
    assert b.max_per_cell == counts.max()
    # cell-relative coordinates: exact in float64, and exactly representable
    # in float32 on this lattice
    for rel, v, o, i in ((b.xs, x, origin[0], ix), (b.ys, y, origin[1], iy), (b.zs, z, origin[2], iz)):
        want = (v.astype(np.float64) - o - i * float(s.cell_w))[perm].astype(np.float32)
        assert (rel == want).all()
    assert (b.ws == s.w[perm]).all()


def test_out_of_box_and_bad_grid(oracle_lib):
    x = np.array([0.5, 1.0], np.float32)  # 1.0 is on the far face: outside [0, 1)
    y = np.array([0.5, 0.5], np.float32)
    with pytest.raises(oracle.OracleError) as e:
        oracle.bin_particles(x, y, y, y, (0, 0, 0), (2, 2, 2), 0.5, 0.5)
    assert e.value.status == oracle.ERANGE
    with pytest.raises(oracle.OracleError) as e:
        oracle.bin_particles(np.array([np.nan], np.float32), y[:1], y[:1], y[:1],
                             (0, 0, 0), (2, 2, 2), 0.5, 0.5)
    assert e.value.status == oracle.ERANGE
    with pytest.raises(oracle.OracleError) as e:  # cell width below the cutoff
        oracle.bin_particles(x[:1], y[:1], y[:1], y[:1], (0, 0, 0), (2, 2, 2), 0.5, 0.6)
    assert e.value.status == oracle.EINVAL
    with pytest.raises(oracle.OracleError) as e:
        oracle.bin_particles(x[:1], y[:1], y[:1], y[:1], (0, 0, 0), (0, 2, 2), 0.5, 0.5)
    assert e.value.status == oracle.EINVAL


def test_empty_system(oracle_lib):
    e = np.zeros(0, np.float32)
    b = oracle.bin_particles(e, e, e, e, (0, 0, 0), (3, 2, 1), 1.0, 1.0)
    assert b.counts.tolist() == [0] * 6 and b.offsets.tolist() == [0] * 7
    s = oracle.sweep(e, e, e, e, (3, 2, 1), 1.0, b)
    assert s.count.size == 0


# ---------------------------------------------------------------- invariants

def test_newton_third_law_and_symmetry(oracle_lib):
    s = synth.clustered(n=20000, n_blobs=8, rc_log2=-5, seed=21)
    b = oracle.bin_particles(s.x, s.y, s.z, s.w, s.origin, s.dims, s.cell_w, s.rc)
    o = oracle.sweep(s.x, s.y, s.z, s.w, s.dims, s.rc, b)
    P, F, S = oracle.invariants(s.w, o)
    assert P % 2 == 0 and P > 0
    assert np.all(np.abs(F) <= 1e-13 * S)


def test_translation_and_permutation_invariance(oracle_lib):
    s = synth.box_system(3000, 8, seed=22, lattice_log2=18)
    b = oracle.bin_particles(s.x, s.y, s.z, s.w, s.origin, s.dims, 1.0, 1.0)
    o = oracle.sweep(s.x, s.y, s.z, s.w, s.dims, 1.0, b)
    # shift by whole cells into a larger box
    sh = np.float32(2.0)
    b2 = oracle.bin_particles(s.x + sh, s.y, s.z + sh, s.w, (0, 0, 0), (11, 8, 12), 1.0, 1.0)
    o2 = oracle.sweep(s.x + sh, s.y, s.z + sh, s.w, (11, 8, 12), 1.0, b2)
    assert (o.count == o2.count).all()
    assert np.all(np.abs(o.rho - o2.rho) <= 1e-13 * o.rho)
    # permute the input order
    pi = np.random.default_rng(1).permutation(s.n)
    b3 = oracle.bin_particles(s.x[pi], s.y[pi], s.z[pi], s.w[pi], s.origin, s.dims, 1.0, 1.0)
    o3 = oracle.sweep(s.x[pi], s.y[pi], s.z[pi], s.w[pi], s.dims, 1.0, b3)
    assert (o3.count == o.count[pi]).all()
    assert (b3.offsets == b.offsets).all()
    assert np.all(np.abs(o3.gx - o.gx[pi]) <= 1e-13 * o.ascale[pi] + 1e-300)


# ---------------------------------------------------------------- statistics

def test_uniform_statistics_tiny(oracle_lib):
    """Uniform unit cube, 32^3 cells, r_c = 1/32: interior particles see on
    average (N-1)(4 pi/3) r_c^3 neighbours and rho = (N-1) E[w] (unit
    integral of W); the total ordered pair count is about 1.325e5."""
    s = synth.tiny()
    b = oracle.bin_particles(s.x, s.y, s.z, s.w, s.origin, s.dims, s.cell_w, s.rc)
    o = oracle.sweep(s.x, s.y, s.z, s.w, s.dims, s.rc, b)
    rc = s.rc
    inner = ((s.x >= rc) & (s.x < 1 - rc) & (s.y >= rc) & (s.y < 1 - rc)
             & (s.z >= rc) & (s.z < 1 - rc))
    n = s.n
    assert o.count[inner].mean() == pytest.approx((n - 1) * 4 * math.pi / 3 * rc ** 3, rel=0.02)
    assert o.rho[inner].mean() == pytest.approx((n - 1) * 1.0, rel=0.02)
    assert o.count.sum() == pytest.approx(1.325e5, rel=0.02)
    assert o.cand.mean() == pytest.approx((n - 1) * ((3 * 32 - 2) / 32 ** 2) ** 3, rel=0.01)


# ---------------------------------------------------------------- timing-experiment kernels
# Sec. 7.1 (Lennard-Jones with softening) and Fig. 8 (5- and 168-FLOP
# kernels), evaluated on every candidate of the 27-cell stencil.

K6 = 2.0 ** -6


def _pair_system(points, dims=(8, 8, 8), cw=2.0 ** -3):
    p = np.array(points, np.float64)
    x, y, z = (p.T).astype(np.float32)
    assert np.all(np.float64(x) == p[:, 0])  # exact in float32
    w = np.ones(len(p), np.float32)
    b = oracle.bin_particles(x, y, z, w, (0, 0, 0), dims, cw, cw)
    return x, y, z, dims, b


def _lj(kind, pts, sigma, eps, e0, **kw):
    x, y, z, dims, b = _pair_system(pts, **kw)
    return oracle.sweep_pairfn(kind, x, y, z, dims, sigma, eps, e0, b)


def test_lj_zero_where_softened_distance_is_sigma(oracle_lib):
    """3-4-5: r = 4k on an axis, eps = 3k, sigma = 5k gives r^2 + eps^2 =
    sigma^2, u = 1 and K = 4 e0 (1 - 1) = 0; the condition scale is 8 e0."""
    base = np.array([3, 3, 3]) * 2.0 ** -3 + 2.0 ** -5
    for ax in range(3):
        pts = [base, base.copy()]
        pts[1][ax] += 4 * K6
        o = _lj("lj", pts, 5 * K6, 3 * K6, 0.75)
        assert o.v.tolist() == [0.0, 0.0]
        assert o.ascale.tolist() == [6.0, 6.0]
        assert o.cand.tolist() == [1, 1]


def test_lj_closed_form_value(oracle_lib):
    """r = k, eps = k, sigma = 2k: u = 4k^2 / 2k^2 = 2 and
    K = 4 e0 (2^6 - 2^3) = 224 e0, A = 4 e0 (2^6 + 2^3) = 288 e0."""
    base = np.array([2, 5, 1]) * 2.0 ** -3 + 2.0 ** -4
    pts = [base, base + np.array([0, 0, K6])]
    o = _lj("lj", pts, 2 * K6, K6, 0.75)
    assert o.v.tolist() == [224 * 0.75] * 2
    assert o.ascale.tolist() == [288 * 0.75] * 2


def test_lj_softening_keeps_coincident_pairs_finite(oracle_lib):
    """r = 0: u = sigma^2 / eps^2 = 4, K = 4 e0 (4096 - 64) = 16128 e0."""
    base = np.array([1, 1, 1]) * 2.0 ** -3 + 2.0 ** -5
    o = _lj("lj", [base, base], 2 * K6, K6, 1.0)
    assert o.v.tolist() == [16128.0, 16128.0]


def test_lj_minimum_depth_and_place(oracle_lib):
    """K(s) = 4 e0 ((sigma/s)^12 - (sigma/s)^6) with s^2 = r^2 + eps^2 has
    its minimum -e0 at s = 2^(1/6) sigma: sample two-particle systems
    across r and find both."""
    sigma, eps, e0 = 0.04, 0.01, 1.25
    rs = np.arange(1, 4000) * 2.0 ** -16      # r in (0, 0.061], exact in float32
    base = np.array([2, 2, 2]) * 2.0 ** -3
    vals = []
    for r in rs:
        o = _lj("lj", [base, base + np.array([r, 0, 0])], sigma, eps, e0)
        vals.append(o.v[0])
    vals = np.array(vals)
    k = int(np.argmin(vals))
    s_min = math.sqrt(rs[k] ** 2 + eps ** 2)
    assert abs(s_min - 2.0 ** (1 / 6) * sigma) < 2.0 ** -15
    assert vals[k] == pytest.approx(-e0, rel=1e-6)
    # repulsive inside s = sigma, attractive outside, tending to 0
    s = np.sqrt(rs ** 2 + eps ** 2)
    assert np.all(vals[s < sigma * (1 - 1e-6)] > 0) and np.all(vals[s > sigma * (1 + 1e-6)] < 0)
    assert np.all(np.diff(vals[k:]) > 0) and np.all(np.diff(vals[:k + 1]) < 0)


def test_lj_equilateral_triangle(oracle_lib):
    """k (1,1,0), k (1,0,1), k (0,1,1) are pairwise sqrt(2) k apart: each
    target sums two equal terms; with eps = k, sigma = 2k: s^2 = 3k^2,
    u = 4/3, v = 2 * 4 e0 ((4/3)^6 - (4/3)^3)."""
    from fractions import Fraction
    base = np.array([3, 4, 5]) * 2.0 ** -3 + 2.0 ** -5
    pts = [base + K6 * np.array(d) for d in ((1, 1, 0), (1, 0, 1), (0, 1, 1))]
    o = _lj("lj", pts, 2 * K6, K6, 1.0)
    u = Fraction(4, 3)
    expect = float(2 * 4 * (u ** 6 - u ** 3))
    assert np.allclose(o.v, expect, rtol=1e-14, atol=0)


def test_lowflop_closed_form_and_antisymmetry(oracle_lib):
    """v_i = sum_j (x_i - x_j) + (y_i - y_j) + (z_i - z_j): two particles
    give +-(dx + dy + dz); over a system the sum of v is exactly 0 (each
    term is exact in double on the lattice and cancels with its mirror)."""
    base = np.array([1, 2, 3]) * 2.0 ** -3 + 2.0 ** -5
    d = np.array([3, -5, 7]) * 2.0 ** -9
    o = _lj("lowflop", [base, base + d], 1.0, 1.0, 1.0)
    assert o.v.tolist() == [-(3 - 5 + 7) * 2.0 ** -9, (3 - 5 + 7) * 2.0 ** -9]
    assert o.ascale.tolist() == [15 * 2.0 ** -9] * 2
    s = synth.box_system(4000, 9, seed=31, lattice_log2=18)
    b = oracle.bin_particles(s.x, s.y, s.z, s.w, s.origin, s.dims, s.cell_w, s.rc)
    o = oracle.sweep_pairfn("lowflop", s.x, s.y, s.z, s.dims, 1, 1, 1, b)
    assert float(o.v.sum()) == 0.0 and np.abs(o.v).max() > 1.0


def test_highflop_equals_lj(oracle_lib):
    """The high-FLOP kernel's 75 multiply-adds with a = 1, b = 0 leave the
    Lennard-Jones value unchanged."""
    s = synth.box_system(3000, 8, seed=32, lattice_log2=18)
    b = oracle.bin_particles(s.x, s.y, s.z, s.w, s.origin, s.dims, s.cell_w, s.rc)
    a = oracle.sweep_pairfn("lj", s.x, s.y, s.z, s.dims, 0.45, 0.2, 1.0, b)
    h = oracle.sweep_pairfn("highflop", s.x, s.y, s.z, s.dims, 0.45, 0.2, 1.0, b)
    assert (a.v == h.v).all() and (a.ascale == h.ascale).all() and (a.cand == h.cand).all()


@pytest.mark.parametrize("case", ["uniform", "clustered", "flat_grid"])
def test_pairfn_cell_list_equals_neighbour_cell_definition(oracle_lib, case):
    """The cell-list sweep against the definition with no cell list (every
    j != i whose cell is within one cell on each axis), and its candidate
    counts against the B-spline sweep's (pinned by Table 1)."""
    if case == "uniform":
        s = synth.box_system(3000, 7, seed=33, lattice_log2=18)
    elif case == "clustered":
        s = synth.box_system(3000, 9, seed=34, lattice_log2=18, clustered_blobs=3)
    else:
        s0 = synth.box_system(2500, 9, seed=35, lattice_log2=18)
        keep = s0.z < 2.0
        s = synth.System("flat", s0.x[keep], s0.y[keep], s0.z[keep], s0.w[keep], (0, 0, 0), (9, 9, 2), 1.0, 1.0)
    b = oracle.bin_particles(s.x, s.y, s.z, s.w, s.origin, s.dims, s.cell_w, s.rc)
    ref = oracle.sweep(s.x, s.y, s.z, s.w, s.dims, s.rc, b)
    for kind, (sg, ep) in (("lj", (0.5, 0.25)), ("lowflop", (1, 1)), ("highflop", (0.3, 0.3))):
        cl = oracle.sweep_pairfn(kind, s.x, s.y, s.z, s.dims, sg, ep, 0.9, b)
        br = oracle.brute_pairfn(kind, s.x, s.y, s.z, s.dims, sg, ep, 0.9, b.cell)
        assert (cl.cand == br.cand).all() and (cl.cand == ref.cand).all()
        assert np.all(np.abs(cl.v - br.v) <= 1e-13 * br.ascale + 1e-300)
        assert np.allclose(cl.ascale, br.ascale, rtol=1e-13, atol=0)


# ---------------------------------------------------------------- time stepping
# The position update that ends the pipeline (Sec. 2), with the B-spline as a
# soft pair potential E = (kappa/2) sum_i sum_{j != i} w_i w_j W(r_ij).

def _step_system(pts, vel, w, dims=(8, 8, 8), cw=1.0):
    p = np.asarray(pts, np.float64)
    x, y, z = p.T.astype(np.float32)
    v = np.asarray(vel, np.float64).T
    w = np.asarray(w, np.float32)
    b = oracle.bin_particles(x, y, z, w, (0, 0, 0), dims, cw, cw)
    g = oracle.sweep(x, y, z, w, dims, cw, b)
    return x, y, z, w, v, g


def test_step_free_particle_moves_by_dt_v(oracle_lib):
    """No neighbour: G = 0, so v' = v and x' = x + dt v (exact in binary)."""
    x, y, z, w, v, g = _step_system([[2.5, 3.25, 4.0]], [[0.5, -0.25, 0.125]], [1.0])
    pos, vel, cut = oracle.euler_step(x, y, z, *v, g.gx, g.gy, g.gz, 0.25, 3.0, (0, 0, 0), (8, 8, 8), 1.0)
    assert pos[:, 0].tolist() == [2.625, 3.1875, 4.03125] and vel[:, 0].tolist() == [0.5, -0.25, 0.125]
    assert not cut.any()


def test_step_reflects_at_both_faces_and_cuts_long_moves(oracle_lib):
    pts = [[0.0625, 4.5, 4.5], [7.9375, 1.5, 1.5], [4.5, 4.5, 1.5]]
    vel = [[-0.5, 0, 0], [0.5, 0, 0], [0, 0, 8.0]]
    x, y, z, w, v, g = _step_system(pts, vel, [1, 1, 1])
    pos, v2, cut = oracle.euler_step(x, y, z, *v, g.gx, g.gy, g.gz, 0.25, 1.0, (0, 0, 0), (8, 8, 8), 1.0)
    assert pos[0, 0] == 0.0625 and v2[0, 0] == 0.5          # 0.0625 - 0.125 -> -0.0625 -> 0.0625
    assert pos[0, 1] == 7.9375 and v2[0, 1] == -0.5         # 7.9375 + 0.125 -> 8.0625 -> 7.9375
    assert cut.tolist() == [False, False, True] and pos[2, 2] == 2.0  # dt v = 2 cut to half a cell


def test_step_repulsion_and_momentum_of_a_pair(oracle_lib):
    """Two particles at rest 0.625 h apart on x: the B-spline decreases with r,
    so the pair force pushes them apart, with equal and opposite momenta
    (w1 v1 = -w2 v2) along the line joining them."""
    x, y, z, w, v, g = _step_system([[3.25, 4.5, 4.5], [3.875, 4.5, 4.5]], [[0, 0, 0], [0, 0, 0]], [0.75, 1.25])
    pos, vel, _ = oracle.euler_step(x, y, z, *v, g.gx, g.gy, g.gz, 0.01, 2.0, (0, 0, 0), (8, 8, 8), 1.0)
    assert vel[0, 0] < 0 < vel[0, 1] and np.all(vel[1:] == 0)
    assert 0.75 * vel[0, 0] + 1.25 * vel[0, 1] == pytest.approx(0.0, abs=1e-15)
    # magnitude: dt kappa w_j |W'(0.625)|
    _, dW = oracle.kernel(0.625, 1.0)
    assert vel[0, 1] == pytest.approx(0.01 * 2.0 * 0.75 * abs(dW), rel=1e-12)


def test_step_momentum_conserved_away_from_walls(oracle_lib):
    s = synth.box_system(400, 10, seed=51, lattice_log2=18, clustered_blobs=2)
    inner = np.all([(a > 2) & (a < 8) for a in (s.x, s.y, s.z)], axis=0)
    x, y, z, w = s.x[inner], s.y[inner], s.z[inner], s.w[inner]
    rng = np.random.default_rng(5)
    v = rng.normal(0, 0.05, (3, x.size))
    b = oracle.bin_particles(x, y, z, w, (0, 0, 0), s.dims, 1.0, 1.0)
    g = oracle.sweep(x, y, z, w, s.dims, 1.0, b)
    _, vel, _ = oracle.euler_step(x, y, z, *v, g.gx, g.gy, g.gz, 0.02, 1.5, (0, 0, 0), s.dims, 1.0)
    p0 = (np.asarray(w, np.float64) * v).sum(axis=1)
    p1 = (np.asarray(w, np.float64) * vel).sum(axis=1)
    assert np.all(np.abs(p1 - p0) <= 1e-12 * (np.asarray(w, np.float64) * np.abs(vel)).sum(axis=1))


def test_step_energy_error_is_first_order(oracle_lib):
    """Symplectic Euler on the soft potential: the total energy after a fixed
    time stays close to the start, and halving dt halves the error (first
    order), which a wrong force factor or sign would break."""
    s = synth.box_system(300, 6, seed=52, lattice_log2=18)
    rng = np.random.default_rng(6)
    v0 = rng.normal(0, 0.02, (3, s.n))
    kappa, T = 0.02, 2.0

    def run(dt):
        x, y, z = (np.asarray(a, np.float64) for a in (s.x, s.y, s.z))
        v = v0.copy()
        w64 = np.asarray(s.w, np.float64)

        def energy(x, y, z, v):
            b = oracle.bin_particles(x, y, z, s.w, (0, 0, 0), s.dims, 1.0, 1.0)
            o = oracle.sweep(x, y, z, s.w, s.dims, 1.0, b)
            return 0.5 * float((w64 * (v * v).sum(axis=0)).sum()) + oracle.pair_energy(s.w, o.rho, kappa), o

        e0, o = energy(x, y, z, v)
        for _ in range(int(round(T / dt))):
            pos, v, cut = oracle.euler_step(x, y, z, *v, o.gx, o.gy, o.gz, dt, kappa, (0, 0, 0), s.dims, 1.0)
            assert not cut.any()
            x, y, z = pos
            e, o = energy(x, y, z, v)
        return abs(e - e0) / abs(e0)

    e1, e2 = run(0.1), run(0.05)
    assert e1 < 2e-2 and 1.4 < e1 / e2 < 2.8, (e1, e2)

"""Batched binning + sweep (pi_batch_run) against the FP64 oracle, system by
system, and against the single-system path: each system's result must be the
same alone and in the batch, and every replay of the captured graph must
reproduce the direct launch bit for bit."""
import sys

import numpy as np
import pytest

import oracle
from paper_2406_16091_amd import synth

pytestmark = pytest.mark.gpu
TOL = 1e-5


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


def _mixed_systems(count=24, seed=77):
    """Small uneven systems: uniform and clustered, different grids, cutoffs
    and cell widths, one empty system."""
    rng = np.random.default_rng(seed)
    out = []
    for k in range(count):
        g = int(rng.integers(3, 14))
        n = int(rng.integers(0, 6 * g ** 3)) if k != 5 else 0
        blobs = 3 if k % 3 == 0 else 0
        s = synth.box_system(n, g, seed=seed * 100 + k, lattice_log2=18, clustered_blobs=blobs)
        if k % 4 == 1:   # cutoff below the cell width
            s = synth.System(s.name, s.x, s.y, s.z, s.w, s.origin, s.dims, 1.0, 0.8)
        out.append(s)
    return out


def _ref(s):
    b = oracle.bin_particles(s.x, s.y, s.z, s.w, s.origin, s.dims, s.cell_w, s.rc)
    return b, oracle.sweep(s.x, s.y, s.z, s.w, s.dims, s.rc, b)


def _check(res, ref):
    assert (res["count"].astype(np.int64) == ref.count).all()
    rho = res["rho"].astype(np.float64)
    assert np.all(np.abs(rho - ref.rho) <= TOL * ref.rho)
    for k in ("gx", "gy", "gz"):
        assert np.all(np.abs(res[k].astype(np.float64) - getattr(ref, k)) <= TOL * ref.ascale)


@pytest.mark.parametrize("sweep,tile", [("auto", (0, 0, 0)), ("nolds", (0, 0, 0)), ("stream", (0, 0, 0)),
                                        ("subbox", (4, 4, 4)), ("pencil", (30, 1, 1)), ("subbox", (6, 6, 6)),
                                        ("pencilreg", (4, 4, 2)), ("cell", (4, 1, 1)), ("cell", (2, 32, 1))])
def test_batch_matches_oracle_per_system(dev, sweep, tile):
    systems = _mixed_systems()
    db = dev.DeviceBatch(systems)
    db.run(sweep=sweep, tile=tile)
    db.sync()
    res = db.results()
    inv = db.invariants()
    binned = db.binned()
    for i, s in enumerate(systems):
        b, ref = _ref(s)
        _check(res[i], ref)
        assert inv[i]["pairs"] == int(ref.count.sum())
        # binning of this system: its slice of the concatenated arrays
        off, nc, cb = db.offsets[i], s.n_cells, binned["cell_base"][i]
        assert (binned["counts"][cb:cb + nc] == b.counts).all()
        assert (binned["offsets"][cb:cb + nc + 1] - off == b.offsets).all()
        assert (binned["perm"][off:off + s.n] - off == b.perm).all()
        assert (binned["cell"][off:off + s.n] == b.cell[b.perm]).all()
        assert (binned["xs"][off:off + s.n].view(np.uint32) == b.xs.view(np.uint32)).all()


def test_alone_and_in_the_mix_are_identical(dev):
    systems = _mixed_systems(seed=78)
    db = dev.DeviceBatch(systems)
    db.run()
    db.sync()
    mix = db.results()
    for i in (0, 3, 7, 11, 20):
        ds = dev.DeviceSystem(systems[i])
        ds.bin()
        ds.interact(order="original")
        ds.sync()
        alone = ds.results()
        for k in ("rho", "gx", "gy", "gz", "count"):
            assert (alone[k].view(np.uint32) == mix[i][k].view(np.uint32)).all(), (i, k)


def test_graph_replays_reproduce_direct_launch(dev):
    import torch
    systems = _mixed_systems(seed=79)
    db = dev.DeviceBatch(systems)
    db.run(stream=0)           # null stream: direct launches, no graph
    db.sync()
    ref = [{k: v.copy() for k, v in r.items()} for r in db.results()]
    s = torch.cuda.Stream()
    for rep in range(4):       # first call captures, later calls replay
        junk = torch.randn(1 << 16, device="cuda")
        (junk * 2).sum().item()  # eager work between replays
        db.rho.fill_(-1.0)
        db.count.fill_(-1)
        s.wait_stream(torch.cuda.current_stream())
        db.run(stream=s)
        s.synchronize()
        db.sync()
        got = db.results()
        for i in range(len(systems)):
            for k in ("rho", "gx", "gy", "gz", "count"):
                assert (got[i][k].view(np.uint32) == ref[i][k].view(np.uint32)).all(), (rep, i, k)


def test_batch_of_512_systems_pair_counts(dev):
    """The 512-system batch workload: every system's neighbour counts and
    pair total bit-exact against the oracle."""
    systems = synth.batch_systems()
    _say(f"[batch512] total particles {sum(s.n for s in systems)}")
    db = dev.DeviceBatch(systems)
    db.run()
    db.sync()
    res = db.results()
    inv = db.invariants()
    for i, s in enumerate(systems):
        b, ref = _ref(s)
        assert (res[i]["count"].astype(np.int64) == ref.count).all(), i
        assert inv[i]["pairs"] == int(ref.count.sum()), i
        if i % 64 == 0:
            _check(res[i], ref)


def test_batch_of_many_tiny_systems(dev):
    """600 systems of 1 or 8 cells holding 0-12 particles: one 1024-cell
    block of the cell-to-system index, and one 4096-particle sort tile, span
    hundreds of systems.  Binning and sweep checked system by system."""
    rng = np.random.default_rng(80)
    systems = []
    for k in range(600):
        g = 1 if k % 3 else 2
        n = int(rng.integers(0, 13))
        systems.append(synth.box_system(n, g, seed=8000 + k, lattice_log2=18))
    _say(f"[tiny600] particles {sum(s.n for s in systems)}, cells {sum(s.n_cells for s in systems)}")
    db = dev.DeviceBatch(systems)
    db.run()
    db.sync()
    res = db.results()
    inv = db.invariants()
    binned = db.binned()
    for i, s in enumerate(systems):
        b, ref = _ref(s)
        _check(res[i], ref)
        assert inv[i]["pairs"] == int(ref.count.sum()), i
        off, nc, cb = db.offsets[i], s.n_cells, binned["cell_base"][i]
        assert (binned["counts"][cb:cb + nc] == b.counts).all(), i
        assert (binned["offsets"][cb:cb + nc + 1] - off == b.offsets).all(), i
        assert (binned["perm"][off:off + s.n] - off == b.perm).all(), i
        assert (binned["cell"][off:off + s.n] == b.cell[b.perm]).all(), i
        assert (binned["xs"][off:off + s.n].view(np.uint32) == b.xs.view(np.uint32)).all(), i

"""pi_interact_noalloc: the sweep without any allocation (invariant partials in
a fixed per-device array) against pi_interact on the same binned systems,
through the C ABI.  Two calls in a row, the second on a smaller system, each
bit for bit equal to pi_interact (floats, counts, invariants) and with counts
equal to the FP64 oracle's; a call whose invariants need more records than
the fixed array holds is refused before anything is queued."""
import sys

import numpy as np
import pytest

import oracle
from paper_2406_16091_amd import synth

ORGS = [("subbox", (6, 6, 6)), ("nolds", (0, 0, 0)), ("pencil", (62, 1, 1)), ("auto", (0, 0, 0))]


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


def _run_both(dev, ds, precision, sweep, tile):
    """pi_interact then pi_interact_noalloc on the same binned system; returns
    both result sets and invariants."""
    import torch
    from paper_2406_16091_amd import pi
    ctx = ds.ctx.handle
    opts = pi.make_opts(precision, sweep, "original", tile)
    ds.interact(precision=precision, sweep=sweep, tile=tile, order="original")
    ds.sync()
    ref, ref_inv = ds.results(), ds.invariants()
    n = ds.sys.n
    f = dict(dtype=torch.float32, device=ds.dev)
    out = {k: torch.full((max(n, 1),), -7.0, **f) for k in ("rho", "gx", "gy", "gz")}
    cnt = torch.full((max(n, 1),), -7, dtype=torch.int32, device=ds.dev)
    inv = torch.zeros(pi.INV_BYTES, dtype=torch.uint8, device=ds.dev)
    pi.pi_interact_noalloc(ctx, ds.cells, opts, out["rho"], out["gx"], out["gy"], out["gz"], cnt, inv)
    pi.pi_sync(ctx, ds.cells)
    got = {k: v[:n].cpu().numpy() for k, v in out.items()}
    got["count"] = cnt[:n].cpu().numpy()
    return ref, ref_inv, got, pi.read_invariants(inv)


@pytest.mark.gpu
def test_noalloc_equals_interact_on_two_calls_the_second_smaller(dev):
    from paper_2406_16091_amd import pi
    big = synth.uniform_unit_cube(120_000, -5, seed=801, name="noalloc_big")   # 32^3 cells, ~3.7 per cell
    small = synth.box_system(9_000, 14, seed=802, lattice_log2=18)           # 14^3 cells
    pi.pi_tuner_mode(dev.Context.get(0).handle, pi.PI_TUNE_STATIC)
    try:
        for s in (big, small):
            b = oracle.bin_particles(s.x, s.y, s.z, s.w, s.origin, s.dims, s.cell_w, s.rc)
            ref_o = oracle.sweep(s.x, s.y, s.z, s.w, s.dims, s.rc, b)
            ds = dev.DeviceSystem(s)
            ds.bin()
            ds.sync()
            for precision in ("compensated", "plain"):
                for sweep, tile in ORGS:
                    _say(f"[noalloc] {s.name} n={s.n} dims={s.dims} {precision} {sweep} {tile}")
                    ref, ref_inv, got, inv = _run_both(dev, ds, precision, sweep, tile)
                    for k in ("rho", "gx", "gy", "gz", "count"):
                        assert (got[k].view(np.uint32) == ref[k].view(np.uint32)).all(), (s.name, sweep, k)
                    assert (got["count"].astype(np.int64) == ref_o.count).all()
                    assert inv == ref_inv
                    assert inv["pairs"] == int(ref_o.count.sum())
            ds.close()
    finally:
        pi.pi_tuner_mode(dev.Context.get(0).handle, pi.PI_TUNE_TIMED)


@pytest.mark.gpu
def test_noalloc_refuses_more_records_than_the_fixed_array(dev):
    """A 30-cell pencil tiling of a 256^3 grid takes 9 x 256 x 256 = 589,824
    workgroups, more records than the fixed array holds: PI_ENOMEM, nothing
    queued (the outputs keep their fill); AUTO and a count-only call (no
    invariants, no records) still run."""
    import torch
    from paper_2406_16091_amd import pi
    s = synth.uniform_unit_cube(6_000, -8, seed=803, name="noalloc_sparse")  # 256^3 cells
    ds = dev.DeviceSystem(s)
    ds.bin()
    ds.sync()
    ctx = ds.ctx.handle
    n = s.n
    rho = torch.full((n,), -7.0, dtype=torch.float32, device=ds.dev)
    gx, gy, gz = (torch.full((n,), -7.0, dtype=torch.float32, device=ds.dev) for _ in range(3))
    cnt = torch.full((n,), -7, dtype=torch.int32, device=ds.dev)
    inv = torch.zeros(pi.INV_BYTES, dtype=torch.uint8, device=ds.dev)
    assert 9 * 256 * 256 > pi.PI_NOALLOC_SCRATCH_RECORDS
    opts = pi.make_opts("compensated", "pencil", "original", (30, 1, 1))
    with pytest.raises(pi.PiError) as e:
        pi.pi_interact_noalloc(ctx, ds.cells, opts, rho, gx, gy, gz, cnt, inv)
    assert e.value.status == pi.PI_ENOMEM
    torch.cuda.synchronize()
    assert (cnt.cpu().numpy() == -7).all()
    # the same tiling without invariants needs no records
    pi.pi_interact_noalloc(ctx, ds.cells, opts, rho, gx, gy, gz, cnt, None)
    pi.pi_sync(ctx, ds.cells)
    b = oracle.bin_particles(s.x, s.y, s.z, s.w, s.origin, s.dims, s.cell_w, s.rc)
    ref_o = oracle.sweep(s.x, s.y, s.z, s.w, s.dims, s.rc, b)
    assert (cnt.cpu().numpy().astype(np.int64) == ref_o.count).all()
    ref, ref_inv, got, got_inv = _run_both(dev, ds, "compensated", "auto", (0, 0, 0))
    for k in ("rho", "gx", "gy", "gz", "count"):
        assert (got[k].view(np.uint32) == ref[k].view(np.uint32)).all(), k
    assert got_inv["pairs"] == int(ref_o.count.sum())
    ds.close()

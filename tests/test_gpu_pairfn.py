"""GPU parity of the timing-experiment pair kernels (Sec. 7.1 Lennard-Jones
with softening; Fig. 8's 5- and 168-FLOP kernels) through the C ABI
(pi_interact_pairfn), against the FP64 oracle on Table 1's workloads: d^3
cells (d = 2 .. 16) with 1, 10 or 100 particles per cell, uniform in the unit
cube, cell width = r_c = 1/d; plus a clustered system.

Bars:
  * candidate counts: bit for bit (every j != i in the clipped 27-cell
    stencil); the invariants' pair total equals their sum;
  * v: |v - v*| <= 1e-5 A* with compensated sums, A* = sum_j |terms| (the
    FP32 term is within about 40 u of its own magnitude, u = 2^-24: the
    softened distance s^2 = r^2 + eps^2 takes 3 roundings, u = sigma^2 / s^2
    two more, u^3 two, the u^6 - u^3 difference and the factor two; Kahan
    accumulation adds at most 2 u A*); plain sums add the recursive-summation
    bound, count u A*;
  * on these lattice inputs every organisation gives bit-identical outputs,
    and the high-FLOP kernel equals Lennard-Jones bit for bit.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_2406_16091_amd import synth

U = 2.0 ** -24
ORGS = [("nolds", (0, 0, 0)), ("pencil", (0, 0, 0)), ("pencil", (1, 1, 1)), ("pencil", (6, 1, 1)),
        ("pencil", (30, 1, 1)), ("subbox", (0, 0, 0)), ("subbox", (2, 2, 2)), ("subbox", (0, 4, 4)),
        ("subbox", (3, 4, 4)), ("auto", (0, 0, 0))]


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


def _table1(d, ppc, seed):
    return synth.uniform_unit_cube(d ** 3 * ppc, -int(np.log2(d)), seed=seed, name=f"t1-{d}-{ppc}")


CASES = {f"d{d}_p{p}": (lambda d=d, p=p: _table1(d, p, 700 + 10 * d + p))
         for d, p in ((2, 1), (4, 1), (8, 1), (16, 1), (2, 10), (4, 10), (8, 10), (16, 10),
                      (2, 100), (4, 100), (8, 100))}
CASES["clustered"] = lambda: synth.box_system(40_000, 12, seed=790, lattice_log2=18, clustered_blobs=4)


def _check(res, ref, precision, tag):
    cnt = res["count"].astype(np.int64)
    assert (cnt == ref.cand).all(), f"{tag}: candidate counts differ"
    tol = 1e-5 * ref.ascale
    if precision == "plain":
        tol = tol + ref.cand * U * ref.ascale
    e = np.abs(res["rho"].astype(np.float64) - ref.v)
    assert np.all(e <= tol + 1e-30), f"{tag}: worst {float(np.max(e / (tol + 1e-30)))} of the bound"
    return float(np.max(e / (tol + 1e-30)))


@pytest.mark.gpu
@pytest.mark.parametrize("case", list(CASES))
def test_pairfn_parity_every_organisation(dev, case):
    s = CASES[case]()
    sig, eps, e0 = 0.5 * s.rc, 0.25 * s.rc, 0.75
    _say(f"[pairfn] {case} n={s.n} dims={s.dims}")
    b = oracle.bin_particles(s.x, s.y, s.z, s.w, s.origin, s.dims, s.cell_w, s.rc)
    ds = dev.DeviceSystem(s)
    ds.bin()
    ds.sync()
    worst = {}
    for kind in ("lj", "lowflop", "highflop"):
        ref = oracle.sweep_pairfn(kind, s.x, s.y, s.z, s.dims, sig, eps, e0, b)
        for precision in ("compensated", "plain"):
            first = None
            for sweep, tile in ORGS:
                tag = f"{case} {kind} {precision} {sweep}{tile}"
                ds.interact_pairfn(kind, precision, sweep, "original", tile, sig, eps, e0)
                ds.sync()
                res = ds.results()
                worst[f"{kind}/{precision}"] = max(worst.get(f"{kind}/{precision}", 0.0),
                                                  _check(res, ref, precision, tag))
                inv = ds.invariants()
                assert inv["pairs"] == int(ref.cand.sum()), tag
                if first is None:
                    first = res
                else:
                    for k in ("rho", "count"):
                        assert (res[k].view(np.uint32) == first[k].view(np.uint32)).all(), (tag, k)
            if kind == "lj":
                worst[f"lj_{precision}_bits"] = first["rho"].view(np.uint32).copy()
            elif kind == "highflop":
                assert (first["rho"].view(np.uint32) == worst[f"lj_{precision}_bits"]).all(), \
                    "high-FLOP kernel differs from Lennard-Jones"
    _say(f"[pairfn] {case}: largest error / bound "
         f"{ {k: round(v, 4) for k, v in worst.items() if not k.endswith('_bits')} }")
    ds.close()


@pytest.mark.gpu
def test_pairfn_rejects_bad_options(dev):
    from paper_2406_16091_amd import pi
    s = _table1(4, 1, 799)
    ds = dev.DeviceSystem(s)
    ds.bin()
    ctx = ds.ctx.handle
    for bad in (dict(kernel=0), dict(kernel=4), dict(precision="fp64acc"), dict(sweep="stream"),
                dict(sweep="pencil", tile=(255, 1, 1)), dict(sweep="pencil", tile=(4, 2, 1)),
                dict(sweep="subbox", tile=(4, 1, 1)), dict(sweep="subbox", tile=(4, 3, 3)),
                dict(sweep="subbox", tile=(4, 2, 4)), dict(sigma=-1.0)):
        kw = dict(kernel="lj")
        kw.update(bad)
        opts = pi.make_pairfn_opts(**kw)
        with pytest.raises(pi.PiError) as e:
            pi.pi_interact_pairfn(ctx, ds.cells, opts, ds.rho, ds.count, ds.inv)
        assert e.value.status == pi.PI_EINVAL, bad
    with pytest.raises(pi.PiError) as e:
        pi.pi_interact_pairfn(ctx, ds.cells, pi.make_pairfn_opts("lj"), None, ds.count, None)
    assert e.value.status == pi.PI_EINVAL
    ds.close()

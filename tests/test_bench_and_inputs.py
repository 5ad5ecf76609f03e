"""CPU checks of the measurement bookkeeping in bench.py and of the seeded
input recipes (sizes, occupancy and lattice of each workload)."""
import numpy as np
import pytest

import bench
import oracle
from paper_2406_16091_amd import synth


def test_kernel_key_matches_library_and_profiler_names():
    # the library's timing name and rocprofv3's demangled name map to one key
    assert bench.kernel_key("k_sweep_tile<6,6,6>") == "k_sweep_tile<6,6,6>"
    assert bench.kernel_key("k_sweep_tile<6, 6, 6, 768, 8, 0, true, false>") == "k_sweep_tile<6,6,6>"
    assert bench.kernel_key("k_radix_scatter<true, false>") == "k_radix_scatter<true,false>"
    assert bench.kernel_key("k_cell_ranges") == "k_cell_ranges"


def test_profile_lines_match_only_the_current_sources(tmp_path, monkeypatch):
    """Traffic and VALU-issue figures come from the committed summaries only
    while the kernel sources are those they were taken on; a timing name
    without template arguments matches its instances, the instance with the
    invariants on and not the batch form first."""
    h = bench.source_hash()
    prof = tmp_path / "profiles"
    prof.mkdir()
    (prof / "traffic_x.md").write_text(
        f"TRAFFIC k_sweep_tile<6, 6, 6, 768, 4, 0, false, false> 1.0e8 {h}\n"
        f"TRAFFIC k_sweep_tile<6, 6, 6, 768, 4, 0, true, false> 2.0e8 {h}\n"
        f"TRAFFIC k_sweep_nolds<0, true, false> 3.0e8 0000000000000000\n")
    (prof / "sqcounters_x.md").write_text(f"VALUISSUE k_sweep_tile<6, 6, 6, 768, 4, 0, true, false> 1052.5 {h}\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "source_hash", lambda: h)
    assert bench.measured_traffic("k_sweep_tile<6,6,6>") == 2.0e8
    assert bench.measured_traffic("k_sweep_tile<6,6,6>", inv=False) == 1.0e8
    assert bench.measured_traffic("k_sweep_nolds") is None  # taken on other sources
    assert bench.measured_valu_issue("k_sweep_tile<6,6,6>") == 1052.5
    assert bench.measured_valu_issue("k_sweep_stream") is None


def test_candidate_count_is_the_clipped_stencil_sum():
    # brute force on a small occupancy field: sum over cells of
    # count * (sources in the clipped 27-cell block) minus the targets themselves
    rng = np.random.default_rng(5)
    dims = (5, 4, 3)
    counts = rng.integers(0, 4, size=dims[0] * dims[1] * dims[2])
    c3 = counts.reshape(dims[2], dims[1], dims[0])
    want = 0
    for z in range(dims[2]):
        for y in range(dims[1]):
            for x in range(dims[0]):
                nb = c3[max(z - 1, 0):z + 2, max(y - 1, 0):y + 2, max(x - 1, 0):x + 2].sum()
                want += int(c3[z, y, x]) * int(nb)
    want -= int(counts.sum())
    assert bench.candidates_from_counts(counts, dims) == want


def test_candidate_count_matches_the_oracle():
    s = synth.tiny()
    b = oracle.bin_particles(s.x, s.y, s.z, s.w, s.origin, s.dims, s.cell_w, s.rc)
    ref = oracle.sweep(s.x, s.y, s.z, s.w, s.dims, s.rc, b)
    assert bench.candidates_from_counts(b.counts, s.dims) == int(ref.cand.sum())


@pytest.mark.parametrize("name", ["tiny", "scale_1ppc", "scale_8ppc"])
def test_uniform_recipes(name):
    s = getattr(synth, name)()
    n_cells = int(np.prod(s.dims))
    # sizes and occupancy as stated for the configurations
    assert s.n == {"tiny": 32768, "scale_1ppc": 1 << 24, "scale_8ppc": 1 << 24}[name]
    assert s.n / n_cells == {"tiny": 1.0, "scale_1ppc": 1.0, "scale_8ppc": 8.0}[name]
    assert s.cell_w >= s.rc
    # every coordinate on the 2^-24 lattice inside the unit cube; weights in [0.5, 1.5)
    for v in (s.x[:4096], s.y[:4096], s.z[:4096]):
        m = v.astype(np.float64) * 2.0 ** 24
        assert np.all(m == np.floor(m)) and np.all(v >= 0) and np.all(v < 1)
    assert np.all(s.w[:4096] >= 0.5) and np.all(s.w[:4096] < 1.5)


def test_batch_recipe_sizes_and_grids():
    systems = synth.batch_systems()
    assert len(systems) == 512
    ns = np.array([s.n for s in systems])
    assert ns.min() >= 1000 and ns.max() <= 200000
    for s in systems:
        g = s.dims[0]
        assert 10 <= g <= 58 and s.dims == (g, g, g)
        assert 0.5 <= s.n / g ** 3 <= 8.0


def test_seeded_generators_are_reproducible():
    a, b = synth.tiny(), synth.tiny()
    for k in ("x", "y", "z", "w"):
        assert (getattr(a, k).view(np.uint32) == getattr(b, k).view(np.uint32)).all()

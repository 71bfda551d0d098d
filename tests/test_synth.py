"""Input generators: paper-printed geometry values and RNG sanity (CPU)."""
import json
import os

import numpy as np

from paper_2011_11120_amd import synth

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _load(name):
    with open(os.path.join(GOLD, name)) as fh:
        return json.load(fh)


def test_decimation_counts_match_table1():
    t1 = _load("table1_geometries.json")
    nx, ny = t1["grid"]
    for row in t1["rows"]:
        if row["decimation"] in (1, 2, 4):
            assert synth.decimation_mask(nx, ny, row["decimation"]).sum() == row["traces"]


def test_decimation_spacing_matches_table1():
    """Sub2 is 21 x 21 m and Sub4 21 x 42 m on a 15 m grid (Table 1, spatial sampling)."""
    gx, gy = synth.grid_xy(20, 20, 15.0)
    for d, want in ((2, (21, 21)), (4, (21, 42))):
        m = synth.decimation_mask(20, 20, d)
        px, py = gx[m], gy[m]
        # distances from an interior kept trace to its kept neighbours along the diagonals
        c = np.argmin((px - 150) ** 2 + (py - 150) ** 2)
        dist = np.hypot(px - px[c], py - py[c])
        diag = dist[(np.abs(px - px[c]) == np.abs(py - py[c])) & (dist > 0)]
        anti = dist[((px - px[c]) == -(py - py[c])) & (dist > 0)]
        main = dist[((px - px[c]) == (py - py[c])) & (dist > 0)]
        assert int(main.min()) == want[0]
        assert int(anti.min()) == want[1]
        assert diag.size > 0


def test_table1_sizes_from_dimensions():
    t1 = _load("table1_geometries.json")
    for row in t1["rows"]:
        n = row["traces"]
        # the table prints whole GB (rounded or truncated): within one unit of the exact size
        assert abs(t1["nt_time"] * n * n * 4 / 1e9 - row["time_GB"]) < 1.0
        assert abs(t1["nfmax"] * n * n * 8 / 1e9 - row["freq_GB"]) < 1.0


def test_middle_receiver_and_mdd_grid():
    pc = _load("paper_constants.json")
    nx, ny = pc["grid"]
    gx, gy = synth.grid_xy(nx, ny, 1.0)
    assert gx[pc["middle_receiver"]] == (nx - 1) / 2 and gy[pc["middle_receiver"]] == (ny - 1) / 2
    x0, x1, dxf = pc["mdd_x"]
    y0, y1, dyf = pc["mdd_y"]
    assert ((x1 - x0) // dxf + 1) * ((y1 - y0) // dyf + 1) == pc["mdd_points"]
    assert 4 * pc["spacing_full_m"] ** 2 == pc["area_sub4_m2"]


def test_rng_uniform_and_normal_moments():
    u = synth.rng_uniform(0, 1, np.arange(200000))
    assert 0.0 < u.min() and u.max() < 1.0
    assert abs(u.mean() - 0.5) < 3e-3 and abs(u.var() - 1 / 12) < 2e-3
    z = synth.rng_normal(0, 2, np.arange(200000))
    assert abs(z.mean()) < 1e-2 and abs(z.std() - 1) < 1e-2


def test_rng_known_values():
    """SplitMix64 finaliser reference value (mix64(0x9E3779B97F4A7C15) of the published generator)."""
    # First output of SplitMix64 seeded with 0 is 0xE220A8397B1DCDAF.
    assert int(synth._mix64(np.uint64(0x9E3779B97F4A7C15))) == 0xE220A8397B1DCDAF


def test_kernel_block_is_consistent_with_full():
    spec = synth.KernelSpec(nt=64, nfmax=10, nx=3)
    K = synth.kernel_full(spec)
    sub = synth.kernel_block(spec, [2, 7], [1, 8], [0, 4, 5])
    assert np.array_equal(sub, K[np.ix_([2, 7], [1, 8], [0, 4, 5])])
    # noise breaks the complex symmetry K_f = K_f^T of the noise-free hyperbolic kernel
    assert np.abs(K - K.transpose(0, 2, 1)).max() > 1e-3 * np.abs(K).max()

"""Host-side helpers of bench.py: the tile-occupancy diagnostic and the lookup
of the profiled HBM traffic of the TV pass (no GPU)."""
import torch

import bench


def test_empty_tile_fraction():
    x = torch.zeros(2, 64, 96)
    x[0, 5, 40] = 1.0      # plane 0, tile row 0, tile column 1
    x[1, 63, 95] = 2.0     # plane 1, tile row 1, tile column 2
    assert abs(bench.empty_tile_frac(torch, x, 32) - 10.0 / 12.0) < 1e-6
    assert bench.empty_tile_frac(torch, torch.zeros(1, 16, 16), 32) is None
    # a partial tile at the edge is left out, not counted
    y = torch.zeros(1, 40, 40)
    y[0, 35, 35] = 1.0
    assert bench.empty_tile_frac(torch, y, 32) == 1.0


def test_measured_traffic_lookup():
    t = bench.measured_traffic({"tv_levels": 4, "tv_blocks": 256, "col_blocks": 512})
    assert t is None or t > 6.6e9          # at least the algorithmic bytes of a pass
    assert bench.measured_traffic({"tv_levels": 2, "tv_blocks": 6144, "col_blocks": 512}) is None


def test_cpu_baseline_runs_the_oracle_on_worker_processes():
    from paper_1904_04884_amd import scenes
    cfg = scenes.config_c2()
    g = scenes.geometry_c2()
    nvox = g.nx * g.ny * g.nz
    r = bench.cpu_baseline(scenes, 100, nvox, cfg, workers=2)
    assert r["cores"] == 2 and r["kind"] == "oracle" and len(r["slab_seconds"]) == 2
    # two slabs of 8 planes, one iteration each: the rate is their voxels over the wall time
    assert r["voxel_iters_per_s"] > 0
    assert abs(r["value"] - r["voxel_iters_per_s"] / (nvox * 100)) <= 1e-12 * r["value"]


def test_prox_bytes_per_voxel_schedule():
    # first pass v in, p out; middle passes v, p in, p out; final v, p in, x out
    assert bench.prox_bytes_per_voxel(1) == 8.0
    assert bench.prox_bytes_per_voxel(2) == 16.0 + 20.0
    assert bench.prox_bytes_per_voxel(5) == 120.0

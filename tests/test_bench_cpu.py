"""Host logic of the benchmark: the algorithmic work model the roofline figure
divides by the kernel time, on a frame small enough to count by hand, and
the staleness rule of the measured-traffic figure."""

import types

import numpy as np

import bench


def _scene(width, height, march):
    return types.SimpleNamespace(width=width, height=height, params={"march": march})


def test_work_model_counts_by_hand():
    # two pixels, three samples: pixel 0 has a hit (3 iterations), an
    # off-screen ray (4 iterations) and an invalid sample; pixel 1 is background
    hits = np.array([[[5, -1, -2], [-3, -3, -3]]])
    steps = np.array([[[3, 4, 0], [0, 0, 0]]])
    w = bench.work_model(_scene(2, 1, 1), hits, steps, "f32")
    # trace: 2 depths, one normal record, 7 texels of 16 B
    assert w["bytes_trace"] == 2 * 4 + 16 + 16 * 7
    assert w["ops_trace"] == (bench.OPS_PER_HIZ_ITER * 7 + bench.OPS_PER_SAMPLE * 3
                              + bench.OPS_PER_SEGMENT * 2 + bench.OPS_PER_PIXEL_SETUP)
    # resolve: 2 outputs, one pixel's materials, the background's env texel,
    # one radiance (hit) and one environment (miss) read
    assert w["bytes_resolve"] == 2 * 12 + 32 + 12 + 12 + 12
    assert w["ops_resolve"] == (bench.OPS_PER_WEIGHT * 2 + bench.OPS_PER_HIT + bench.OPS_PER_MISS
                                + bench.OPS_PER_PIXEL_SETUP + bench.OPS_PER_PIXEL_SHADE)
    # pyramid 2x1 then 1x1: 3 texels
    assert w["bytes_hiz"] == 2 * 4 + 16 * 3
    assert (w["iterations"], w["rays"], w["mean_iters"], w["hit_frac"]) == (7, 2, 3.5, 0.5)


def test_work_model_half_storage_and_linear_march():
    hits = np.array([[[7, -4]]])
    steps = np.array([[[2, 32]]])
    w = bench.work_model(_scene(1, 1, 0), hits, steps, "f16")
    assert w["bytes_trace"] == 4 + 8 + 4 * 34
    assert w["ops_trace"] == (bench.OPS_PER_LINEAR_STEP * 34 + bench.OPS_PER_SAMPLE * 2
                              + bench.OPS_PER_SEGMENT * 2 + bench.OPS_PER_PIXEL_SETUP)
    assert w["bytes_resolve"] == 12 + 16 + 6 + 12
    assert w["bytes_hiz"] == 4 + 16


def test_skipped_samples_are_not_drawn():
    hits = np.full((1, 1, 4), -5)
    steps = np.zeros((1, 1, 4), np.int64)
    w = bench.work_model(_scene(1, 1, 1), hits, steps, "f32")
    assert w["ops_trace"] == bench.OPS_PER_PIXEL_SETUP
    assert w["rays"] == 0 and w["iterations"] == 0


def test_traffic_figure_needs_matching_sources(tmp_path, monkeypatch):
    good = tmp_path / "summary.md"
    good.write_text("traffic_bytes_per_launch = 123\n\nsources_sha256 = "
                    + bench.kernel_sources_digest() + "\n")
    monkeypatch.setattr(bench, "COUNTER_SUMMARY", str(good))
    assert bench.measured_traffic() == 123
    stale = tmp_path / "stale.md"
    stale.write_text("traffic_bytes_per_launch = 123\n\nsources_sha256 = 00\n")
    monkeypatch.setattr(bench, "COUNTER_SUMMARY", str(stale))
    assert bench.measured_traffic() is None
    monkeypatch.setattr(bench, "COUNTER_SUMMARY", str(tmp_path / "absent.md"))
    assert bench.measured_traffic() is None

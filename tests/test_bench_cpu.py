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
    # frame: P (48 + 12) + P 16/3 + 4 B per iteration + 12 B per hit or miss
    assert w["frame_bytes"] == 2 * (48 + 12) + (2 * 16) // 3 + 4 * 7 + 12 + 12
    # the trace's share: depth and normal record per pixel, 4 B per iteration
    assert w["trace_bytes"] == 2 * (4 + 16) + 4 * 7
    # 200 per sample (every sample of the frame) + 25 per iteration
    assert w["alu_ops"] == 200 * 2 * 3 + 25 * 7
    assert w["impl_ops_trace"] == (bench.OPS_PER_HIZ_ITER * 7 + bench.OPS_PER_SAMPLE * 3
                                   + bench.OPS_PER_SEGMENT * 2 + bench.OPS_PER_PIXEL_SETUP)
    assert (w["iterations"], w["rays"], w["mean_iters"], w["hit_frac"]) == (7, 2, 3.5, 0.5)


def test_work_model_half_storage_and_linear_march():
    hits = np.array([[[7, -4]]])
    steps = np.array([[[2, 32]]])
    w = bench.work_model(_scene(1, 1, 0), hits, steps, "f16")
    # B_g 26, a 6 B radiance read at the hit, 12 B of environment for the cap
    assert w["frame_bytes"] == (26 + 12) + 16 // 3 + 4 * 34 + 6 + 12
    assert w["trace_bytes"] == 4 + 8 + 4 * 34
    assert w["impl_ops_trace"] == (bench.OPS_PER_LINEAR_STEP * 34 + bench.OPS_PER_SAMPLE * 2
                                   + bench.OPS_PER_SEGMENT * 2 + bench.OPS_PER_PIXEL_SETUP)


def test_skipped_samples_are_not_drawn():
    hits = np.full((1, 1, 4), -5)
    steps = np.zeros((1, 1, 4), np.int64)
    w = bench.work_model(_scene(1, 1, 1), hits, steps, "f32")
    assert w["impl_ops_trace"] == bench.OPS_PER_PIXEL_SETUP
    assert w["rays"] == 0 and w["iterations"] == 0


def test_error_report_by_hand():
    # 1 sampled row of 3 pixels, 2 samples: pixel 0 agrees (rel err 1e-5),
    # pixel 1 disagrees on one marched sample, pixel 2 is background
    sample = dict(rows=np.array([0]),
                  out=np.array([[[1.0, 2.0, 4.0], [1.0, 1.0, 1.0], [3.0, 3.0, 3.0]]]),
                  hits=np.array([[[5, -2], [7, -1], [-3, -3]]]))
    img = np.array([[[1.00001, 2.0, 4.0], [1.5, 1.0, 1.0], [3.0, 3.0, 3.0]]], np.float32)
    codes = np.array([[[5, -2], [8, -1], [-3, -3]]])
    r = bench.error_report(img, codes, sample, 1e-4)
    assert r["pixels"] == 3
    assert r["hit_agreement"] == 2 / 3            # marched samples: 5, 7/8, -1
    assert abs(r["pixels_all_agree"] - 2 / 3) < 1e-12
    assert abs(r["rel_max"] - 1e-5) < 1e-7         # pixel 0, float32-rounded (pixel 2 exact)
    assert r["frac_within_0.0001"] == 1.0
    want_l1 = (1.00001 - 1.0 + 0.5) / (7.0 + 3.0)  # foreground pixels 0 and 1
    assert abs(r["image_rel_l1"] - want_l1) < 1e-6


def test_traffic_figure_needs_matching_sources(tmp_path, monkeypatch):
    good = tmp_path / "summary.md"
    good.write_text("traffic_bytes_per_launch = 123\n\nl2_hit_rate = 0.5\n\nvalu_busy = 0.25\n\n"
                    "valu_lane_utilisation = 0.75\n\nsources_sha256 = "
                    + bench.kernel_sources_digest() + "\n")
    monkeypatch.setattr(bench, "COUNTER_SUMMARY", str(good))
    assert bench.measured_traffic() == 123
    c = bench.measured_counters()
    assert (c["l2_hit_rate"], c["valu_busy"], c["valu_lane_utilisation"]) == (0.5, 0.25, 0.75)
    partial = tmp_path / "partial.md"
    partial.write_text("traffic_bytes_per_launch = 123\n\nsources_sha256 = "
                       + bench.kernel_sources_digest() + "\n")
    monkeypatch.setattr(bench, "COUNTER_SUMMARY", str(partial))
    assert bench.measured_traffic() == 123 and bench.measured_counters() is None
    stale = tmp_path / "stale.md"
    stale.write_text("traffic_bytes_per_launch = 123\n\nsources_sha256 = 00\n")
    monkeypatch.setattr(bench, "COUNTER_SUMMARY", str(stale))
    assert bench.measured_traffic() is None and bench.measured_counters() is None
    monkeypatch.setattr(bench, "COUNTER_SUMMARY", str(tmp_path / "absent.md"))
    assert bench.measured_traffic() is None

"""The seeded input generator: determinism, FP32 hits and the workload's
distributions (Section 3's simplified VELO, with the sizes of the configs)."""
import numpy as np
import pytest

from paper_1709_08610_amd import events


def test_plane_positions():
    z = events.plane_z(events.load_config("c2"))
    assert z.dtype == np.float32 and z.shape == (26,)
    assert z[0] == 20.0 and z[-1] == 750.0
    np.testing.assert_allclose(np.diff(z.astype(np.float64)), 730.0 / 25, rtol=3e-6)  # FP32 spacing
    z1 = events.plane_z(events.load_config("c1"))
    assert list(z1) == [1, 2, 3, 4, 5, 6, 7, 8]


def test_event_determinism_and_independence():
    cfg = events.load_config("c3")
    a = events.make_event(cfg, 17)
    b = events.make_event(cfg, 17)
    c = events.make_event(cfg, 18)
    np.testing.assert_array_equal(a.x, b.x)
    np.testing.assert_array_equal(a.plane, b.plane)
    assert a.n_hits != c.n_hits or not np.array_equal(a.x, c.x)
    # batch slicing regenerates the same events
    bt = events.make_batch(cfg, 3, start=16)
    np.testing.assert_array_equal(bt.event(1).x, a.x)


def test_hits_are_fp32_and_on_planes():
    cfg = events.load_config("c2")
    ev = events.make_event(cfg, 0)
    assert ev.x.dtype == np.float32 and ev.y.dtype == np.float32
    assert ev.plane.min() >= 0 and ev.plane.max() < 26


def test_c2_distributions():
    cfg = events.load_config("c2")
    ev = events.make_event(cfg, 0)
    n_true = int(np.sum(ev.label >= 0))
    assert ev.truth.shape == (200, 4)
    # 10% inefficiency on 26 planes: 4680 expected true hits
    assert abs(n_true - 4680) < 5 * np.sqrt(200 * 26 * 0.09)
    assert int(np.sum(ev.label < 0)) == round(0.2 * n_true)
    assert np.all(np.abs(ev.truth[:, 2:]) <= 0.3)
    # smear: residuals of true hits about their generating line
    z = events.plane_z(cfg).astype(np.float64)[ev.plane]
    t = ev.truth[ev.label[ev.label >= 0]]
    rx = ev.x[ev.label >= 0] - t[:, 0] - t[:, 2] * z[ev.label >= 0]
    assert np.std(rx) == pytest.approx(0.012, rel=0.05)


def test_c3_uneven_batch():
    cfg = events.load_config("c3")
    b = events.make_batch(cfg, 64)
    nt = np.array([len(t) for t in b.truth])
    assert 100 < nt.mean() < 200 and nt.min() >= 1
    nh = np.diff(b.event_offsets)
    assert nh.max() > 1.2 * nh.min()


def test_c1_toy():
    cfg = events.load_config("c1")
    ev = events.make_event(cfg, 0)
    assert ev.y is None and ev.truth.shape == (10, 2)
    assert ev.n_hits == 80 + 50
    assert np.all(np.abs(ev.truth[:, 1]) <= 1.0) and np.all(np.abs(ev.truth[:, 0]) <= 0.5)


def test_track_count_scan():
    """The c7 scan: every event of point N carries exactly N true tracks, the
    points use disjoint event indices of one stream, and the geometry is c2's."""
    cfg = events.load_config("c7")
    pts = events.scan_batches(cfg, n_tracks=[50, 350], events_per_point=3)
    assert [n for n, _ in pts] == [50, 350]
    for n, b in pts:
        assert b.n_events == 3 and all(len(t) == n for t in b.truth)
        np.testing.assert_array_equal(b.plane_z, events.plane_z(events.load_config("c2")))
    a = events.scan_batches(cfg, n_tracks=[50], events_per_point=2)[0][1]
    np.testing.assert_array_equal(a.x, pts[0][1].x[: a.event_offsets[-1]])


def test_quality_eps_fake_count():
    """A found line is an eps-fake when no true track's slopes are within 1e-3."""
    from paper_1709_08610_amd import metrics
    truth = np.array([[0.0, 0.0, 0.1, 0.1], [0.0, 0.0, -0.2, 0.05]])
    found = np.array([[0.5, 0.5, 0.1004, 0.0996], [0.0, 0.0, 0.2, 0.2]])
    q = metrics.event_quality(2, found, truth, np.array([20, 20]), 0.06, 20.0, 750.0)
    assert q["n_eps"] == 1 and q["n_fake_eps"] == 1 and q["n_matched"] == 0 and q["n_fake"] == 2

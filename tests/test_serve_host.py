"""Host-side pieces of the serving workload (CPU): the request trace and the
latency summary."""
import numpy as np

from paper_2408_07967_amd import serve


def test_trace_is_poisson_with_the_resolution_mix():
    tr = serve.make_trace(rate_hz=200.0, seconds=20.0, seed=3)
    n = len(tr)
    # Poisson count: mean 4000, sd ~63
    assert abs(n - 4000) < 5 * 63
    t = np.array([q["t_ns"] for q in tr]) * 1e-9
    assert np.all(np.diff(t) >= 0) and t[-1] < 20.0
    gaps = np.diff(t)
    assert abs(gaps.mean() - 1 / 200.0) < 0.1 / 200.0
    # exponential gaps: coefficient of variation near 1
    assert abs(gaps.std() / gaps.mean() - 1.0) < 0.08
    sizes = {(q["W"], q["H"]) for q in tr}
    assert sizes == {(1280, 720), (1920, 1080), (2560, 1440), (3840, 2160)}
    frac4k = np.mean([q["W"] == 3840 for q in tr])
    assert abs(frac4k - 0.25) < 0.03
    for q in tr[:50]:
        eye = np.asarray(q["cam"].eye, np.float64)
        assert abs(np.hypot(eye[0], eye[2]) - 200.0) < 1e-3
        assert 50.0 <= eye[1] <= 150.0
    assert [q["id"] for q in tr] == list(range(n))
    assert serve.make_trace(200.0, 1.0, seed=3)[0]["t_ns"] == tr[0]["t_ns"]


def test_latency_summary():
    res = [dict(status=0, arrival_ns=i * 1000, done_ns=i * 1000 + (i + 1) * 1_000_000) for i in range(100)]
    res.append(dict(status=3, arrival_ns=0, done_ns=5))
    s = serve.latency_summary(res)
    assert s["completed"] == 100 and s["rejected"] == 1
    assert abs(s["p50_ms"] - 50.5) < 1e-9
    assert abs(s["p99_ms"] - np.percentile(np.arange(1, 101), 99)) < 1e-9
    assert abs(s["max_ms"] - 100.0) < 1e-9

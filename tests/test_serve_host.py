"""Host logic of the served stream (CPU only): the seeded Poisson arrivals and
the latency statistics."""
import numpy as np

from paper_1903_10959_amd import serve


def test_poisson_arrivals_are_seeded_and_have_the_rate():
    a = serve.make_stream(4000, 200.0, seed=5, sizes=["p0", "p1", "p2"])
    b = serve.make_stream(4000, 200.0, seed=5, sizes=["p0", "p1", "p2"])
    t = np.array([r.arrival for r in a])
    assert np.array_equal(t, [r.arrival for r in b])
    assert [r.problem for r in a] == [r.problem for r in b]
    assert np.all(np.diff(t) > 0) and t[0] > 0
    gaps = np.diff(np.concatenate([[0.0], t]))
    # exponential gaps: mean 1/rate and coefficient of variation 1 (4000 draws)
    assert abs(gaps.mean() * 200.0 - 1.0) < 0.05
    assert abs(gaps.std() / gaps.mean() - 1.0) < 0.05
    # every size drawn, about evenly
    counts = np.array([sum(r.problem == s for r in a) for s in ("p0", "p1", "p2")])
    assert np.all(np.abs(counts / 4000 - 1 / 3) < 0.03)
    assert [r.rid for r in a] == list(range(4000))


def test_latency_stats_on_constructed_timings():
    reqs = []
    for i in range(100):
        r = serve.Request(i, arrival=0.01 * i, problem=None)
        r.admitted = r.arrival + 0.001 * (i % 10)
        r.done = r.arrival + 1.0 + 0.01 * i              # end-to-end 1.00 .. 1.99 s
        r.solve_times = [0.1, 0.2]
        reqs.append(r)
    reqs[3].converged = False
    st = serve.latency_stats(reqs, wall=4.0)
    assert st["requests"] == 100
    assert abs(st["offered_rate_per_s"] - 99 / 0.99) < 1e-9
    assert st["achieved_rate_per_s"] == 25.0
    assert abs(st["e2e_p50_s"] - 1.495) < 1e-12                        # midway between 1.49 and 1.50
    assert abs(st["e2e_p99_s"] - (1.0 + 0.01 * 98.01)) < 1e-9          # linear interpolation
    assert abs(st["queue_p99_s"] - 0.009) < 1e-12
    assert abs(st["solve_p50_s"] - 0.15) < 1e-15 and not st["all_converged"]

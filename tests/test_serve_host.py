"""Host-side pieces of the serving driver."""
from paper_2006_09808_amd.serve import percentile


def test_percentile_interpolates():
    xs = [5.0, 1.0, 3.0, 2.0, 4.0]
    assert percentile(xs, 0) == 1.0
    assert percentile(xs, 50) == 3.0
    assert percentile(xs, 100) == 5.0
    assert abs(percentile(xs, 99) - 4.96) < 1e-12
    assert percentile([7.0], 99) == 7.0


class _Stack:
    """Stands in for a device tensor: the driver only asks for its size."""

    def __init__(self, n):
        self.n = n

    def numel(self):
        return self.n


class _FakeSolver:
    """Host-only stand-in for pdlib.Solver: one request served at a time,
    each taking `service_s`; request i stops after iterations[i] with
    status[i].  Completion times are computed, not waited for."""

    def __init__(self, service_s, iterations, status):
        from paper_2006_09808_amd import pdlib
        self.now = pdlib.now
        self.service = service_s
        self.iterations = iterations
        self.status = status
        self.free_at = 0.0
        self.results = {}
        self.n = 0

    def submit(self, jobs):
        out = []
        for _ in jobs:
            i = self.n
            self.n += 1
            start = max(self.now(), self.free_at)
            self.free_at = start + self.service
            self.results[i] = {"status": self.status[i], "iterations": self.iterations[i],
                               "t_start": start, "t_done": self.free_at}
            out.append(i)
        return out

    def poll(self, ticket, timeout_ms):
        return self.results[ticket]


def test_open_loop_accounting_with_a_fake_solver():
    from paper_2006_09808_amd import pdlib
    from paper_2006_09808_amd.serve import Request, run_open_loop, percentile
    arrivals = [0.0, 0.001, 0.002, 0.030, 0.031]
    iterations = [1000, 400, 1000, 250, 1000]
    status = [pdlib.PD_OK, pdlib.PD_OK, pdlib.PD_ERR_NONFINITE, pdlib.PD_OK, pdlib.PD_OK]
    sizes = [64 * 64 * 2, 128 * 128, 64 * 64, 256 * 256 * 3, 96 * 64]
    reqs = [Request(t, _Stack(n), _Stack(n), dict(max_iter=1000)) for t, n in zip(arrivals, sizes)]
    fake = _FakeSolver(0.005, iterations, status)
    summary = run_open_loop(fake, reqs)
    # latencies are completion minus arrival on the library clock; the driver
    # submits each request at its arrival, so a request waits for the ones
    # before it on the one-at-a-time fake server
    t0 = min(r.t_submit - r.t_arrival for r in reqs)        # the driver's start time, up to submit jitter
    lat = [r.result["t_done"] - (t0 + r.t_arrival) for r in reqs]
    assert summary["requests"] == 5 and summary["ok"] == 4
    assert abs(summary["p50_s"] - percentile(lat, 50)) < 2e-3
    assert abs(summary["p99_s"] - percentile(lat, 99)) < 2e-3
    assert summary["cap_hit_fraction"] == 3 / 5
    vit = sum(n * it for n, it in zip(sizes, iterations))
    assert abs(summary["voxel_iterations_per_s"] * summary["span_s"] - vit) <= 1e-6 * vit
    # queueing shows in the latencies: the third request waits for two
    assert reqs[2].result["t_done"] - reqs[0].result["t_start"] >= 3 * 0.005 - 1e-9

"""Open-loop serving driver over the library's continuous batching.

Requests arrive on a schedule (e.g. Poisson); each is submitted at its
arrival time through pd_solve_batch, the library admits it as soon as a slot
and arena space are free and iterates it together with everything already
resident (its primal, dual and exchange state stay in HBM until it stops).
Latency is the library's completion time minus the arrival time, both on
pd_now()'s clock.
"""

import time

from . import pdlib


class Request:
    """One reconstruction: device field map, device output, solver params."""

    def __init__(self, t_arrival, delta, chi, params):
        self.t_arrival = float(t_arrival)
        self.delta = delta
        self.chi = chi
        self.params = dict(params)
        self.ticket = None
        self.t_submit = None
        self.result = None

    @property
    def voxels(self):
        return int(self.delta.numel())


def percentile(xs, q):
    xs = sorted(xs)
    if not xs:
        return float("nan")
    k = (len(xs) - 1) * q / 100.0
    lo = int(k)
    hi = min(lo + 1, len(xs) - 1)
    return xs[lo] + (xs[hi] - xs[lo]) * (k - lo)


def run_open_loop(solver, requests, time_scale=1.0):
    """Submit each request at t0 + t_arrival * time_scale, then collect every
    result.  Returns a summary dict and leaves each request's .result set."""
    reqs = sorted(requests, key=lambda r: r.t_arrival)
    t0 = pdlib.now()
    for r in reqs:
        due = t0 + r.t_arrival * time_scale
        while True:
            d = due - pdlib.now()
            if d <= 0:
                break
            time.sleep(min(d, 0.002))
        r.t_submit = pdlib.now()
        (r.ticket,) = solver.submit([(r.delta, r.chi, r.params)])
    for r in reqs:
        r.result = solver.poll(r.ticket, -1)
    lat = []
    vit = 0.0
    capped = 0
    ok = 0
    t_end = t0
    for r in reqs:
        res = r.result
        if res["status"] == pdlib.PD_OK:
            ok += 1
        arrive = t0 + r.t_arrival * time_scale
        lat.append(res["t_done"] - arrive)
        vit += r.voxels * res["iterations"]
        capped += int(res["iterations"] >= r.params.get("max_iter", 0))
        t_end = max(t_end, res["t_done"])
    span = t_end - t0
    return {
        "requests": len(reqs), "ok": ok,
        "p50_s": percentile(lat, 50), "p99_s": percentile(lat, 99),
        "mean_s": sum(lat) / max(len(lat), 1), "max_s": max(lat) if lat else float("nan"),
        "voxel_iterations_per_s": vit / span if span > 0 else float("nan"),
        "span_s": span, "cap_hit_fraction": capped / max(len(reqs), 1),
    }

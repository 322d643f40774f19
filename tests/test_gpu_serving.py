"""Continuous batching: requests admitted while others run give the same
result as solved alone, admission respects the arena budget, and the
open-loop driver reports latencies."""
import numpy as np
import pytest

import _parity
import oracle
import pd_inputs

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def torch_mod():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def make(seed, nz, ny, nx, **params):
    w = pd_inputs.random_stack(seed, nz, ny, nx, **params)
    field = oracle.forward(w.chi_true)
    return w, pd_inputs.make_delta(field, w.eta, w.rho).astype(np.float32)


MIX = [(64, 64, 4, 80), (128, 128, 6, 120), (192, 192, 3, 90), (64, 96, 5, 60),
       (256, 256, 4, 70), (128, 128, 1, 45), (64, 64, 7, 100), (192, 192, 2, 30)]


def test_mix_results_equal_solo(torch_mod):
    import paper_2006_09808_amd as pd
    from paper_2006_09808_amd import serve
    torch = torch_mod
    cases = [make(100 + i, nz, ny, nx, lam=1e-3, max_iter=it, gap_tol=1e-6, check_every=10)
             for i, (ny, nx, nz, it) in enumerate(MIX)]
    with pd.Solver(arena_bytes=2 << 30, device=0) as s:
        solo = []
        for w, d in cases:
            dt = torch.from_numpy(d).to("cuda:0")
            chi, info = s.solve(dt, **w.solver_params())
            solo.append((chi.cpu().numpy(), info))
        reqs = []
        for i, (w, d) in enumerate(cases):
            dt = torch.from_numpy(d).to("cuda:0")
            reqs.append(serve.Request(0.004 * i, dt, torch.empty_like(dt), w.solver_params()))
        summary = serve.run_open_loop(s, reqs)
    _say("mix of %d requests: p50 %.1f ms p99 %.1f ms" % (len(reqs), summary["p50_s"] * 1e3,
                                                          summary["p99_s"] * 1e3))
    assert summary["ok"] == len(reqs)
    for r, (chi_solo, info_solo) in zip(reqs, solo):
        assert r.result["iterations"] == info_solo["iterations"]
        np.testing.assert_array_equal(r.chi.cpu().numpy(), chi_solo)
        assert r.result["primal"] == info_solo["primal"]


def test_admission_waits_for_arena(torch_mod):
    import paper_2006_09808_amd as pd
    from paper_2006_09808_amd import serve
    torch = torch_mod
    cases = [make(200 + i, 8, 128, 128, lam=1e-3, max_iter=40) for i in range(6)]
    need = pd.validate(128, 128, 8)
    with pd.Solver(arena_bytes=1 << 30, device=0) as probe:
        base, _, _ = probe.arena_usage()          # the context's own control block
    # room for two requests and the shape's kernel table (about 66 KB), not three
    with pd.Solver(arena_bytes=base + 2 * need + need // 2, device=0) as s:
        reqs = []
        for w, d in cases:
            dt = torch.from_numpy(d).to("cuda:0")
            reqs.append(serve.Request(0.0, dt, torch.empty_like(dt), w.solver_params()))
        summary = serve.run_open_loop(s, reqs)
        used, resident, queued = s.arena_usage()
    assert summary["ok"] == 6 and resident == 0 and queued == 0
    starts = sorted(r.result["t_start"] for r in reqs)
    dones = sorted(r.result["t_done"] for r in reqs)
    # at most two fit at once: the third starts only after the first finishes
    assert starts[2] >= dones[0] - 1e-6
    for r, (w, d) in zip(reqs, cases):
        ref, _ = oracle.solve(d.astype(np.float64), **w.solver_params())
        _parity.check(r.chi.cpu().numpy(), ref, "chi")


def test_serving_mix_sampled_against_oracle_and_under_a_small_arena(torch_mod):
    """The serving workload's request mix (Poisson arrivals at 20/s, 128^2 to
    384^2, 16-64 slices, tolerance 1e-5) on a short schedule with a 300-
    iteration cap (so the oracle check stays affordable): every 8th request's
    first slice against the oracle at the request's iteration count (slices
    are independent at a fixed count), and the same schedule again under a
    512 MiB arena (admission waits, shorter steps) with bitwise equal results."""
    import paper_2006_09808_amd as pd
    from paper_2006_09808_amd import serve
    torch = torch_mod
    sched = pd_inputs.serving_schedule(seed=5100, rate=20.0, duration=1.5)
    base = {}
    for i, n in enumerate(pd_inputs.SERVING_SIZES):
        w = pd_inputs.serving_request(5200 + i, n, 64)
        base[n] = pd_inputs.make_delta(oracle.forward(w.chi_true), w.eta, w.rho).astype(np.float32)
    params = dict(lam=1e-3, tau=1.4, sigma=1.4, theta=1.0, max_iter=300, gap_tol=1e-5, check_every=10)

    def run(arena):
        with pd.Solver(arena_bytes=arena, device=0) as s:
            reqs = []
            for (t, n, nz, seed) in sched:
                off = seed % (64 - nz + 1)
                d = torch.from_numpy(np.ascontiguousarray(base[n][off:off + nz])).to("cuda:0")
                reqs.append(serve.Request(t, d, torch.empty_like(d), params))
            summary = serve.run_open_loop(s, reqs)
        return reqs, summary

    big, sb = run(16 << 30)
    _say("serving mix: %d requests, p50 %.1f ms p99 %.1f ms" % (len(big), sb["p50_s"] * 1e3, sb["p99_s"] * 1e3))
    assert sb["ok"] == len(big) >= 10
    small, ss = run(512 << 20)
    _say("under 512 MiB: p50 %.1f ms p99 %.1f ms" % (ss["p50_s"] * 1e3, ss["p99_s"] * 1e3))
    assert ss["ok"] == len(small)
    for a, b in zip(big, small):
        assert a.result["iterations"] == b.result["iterations"]
        assert a.result["rel_gap"] == b.result["rel_gap"]
        np.testing.assert_array_equal(a.chi.cpu().numpy(), b.chi.cpu().numpy())
    for r in big[::8]:
        d = r.delta[0:1].cpu().numpy().astype(np.float64)
        ref, _ = oracle.solve(d, **dict(params, gap_tol=0.0, max_iter=r.result["iterations"]))
        got = r.chi[0:1].cpu().numpy().astype(np.float64)
        _parity.check(got, ref, "request %dx%dx%d, %d iterations, slice 0" % (
            r.delta.shape[2], r.delta.shape[1], r.delta.shape[0], r.result["iterations"]))


def test_gap_tolerance_stops_under_poisson_load(torch_mod):
    """Requests retire on their gap tolerance while others arrive and run:
    a Poisson mix (300 requests/s) in which every third request uses the
    identity kernel (its iterates reach a 1e-5 relative gap within a few
    dozen iterations, so it stops on the gap) and the rest run the dipole
    kernel to their cap.  Each gap-stopped request stops at a check within
    one period of where the oracle stops and matches the oracle's iterate at
    its own count; the capped ones run exactly to the cap."""
    import paper_2006_09808_amd as pd
    from paper_2006_09808_amd import serve
    torch = torch_mod
    rng = np.random.default_rng(77)
    t = 0.0
    reqs, refs = [], []
    for i in range(24):
        t += float(rng.exponential(1.0 / 300.0))
        n = (64, 128, 96)[i % 3]
        nz = int(rng.integers(2, 9))
        if i % 3 == 0:
            delta = rng.normal(size=(nz, n, n)).astype(np.float32)
            sp = dict(lam=0.2, tau=0.9, sigma=0.9, theta=1.0, max_iter=400, gap_tol=1e-5, check_every=5,
                      kernel="identity")
        else:
            w, delta = make(900 + i, nz, n, n, lam=1e-3, max_iter=60 + 10 * (i % 4))
            sp = dict(w.solver_params(), gap_tol=1e-5, check_every=10)
        d = torch.from_numpy(delta).to("cuda:0")
        reqs.append(serve.Request(t, d, torch.empty_like(d), sp))
        refs.append(delta)
    with pd.Solver(arena_bytes=1 << 30, device=0) as s:
        summary = serve.run_open_loop(s, reqs)
    _say("mix of %d requests: p50 %.1f ms p99 %.1f ms, cap hits %.2f" % (
        summary["requests"], summary["p50_s"] * 1e3, summary["p99_s"] * 1e3, summary["cap_hit_fraction"]))
    assert summary["ok"] == len(reqs)
    stopped = 0
    for r, delta in zip(reqs, refs):
        res = r.result
        sp = r.params
        got = r.chi.cpu().numpy().astype(np.float64)
        if sp.get("kernel") == "identity":
            base = {k: v for k, v in sp.items() if k != "kernel"}
            _, iref = oracle.solve(delta.astype(np.float64), kind="identity", **base)
            assert res["iterations"] < sp["max_iter"] and res["iterations"] % sp["check_every"] == 0
            assert res["rel_gap"] <= sp["gap_tol"]
            assert abs(res["iterations"] - iref["iterations"]) <= sp["check_every"]
            ref, _ = oracle.solve(delta.astype(np.float64), kind="identity",
                                  **dict(base, gap_tol=0.0, max_iter=res["iterations"]))
            _parity.check(got, ref, "identity %s stopped at %d" % (delta.shape, res["iterations"]))
            stopped += 1
        else:
            assert res["iterations"] == sp["max_iter"]
    assert stopped == 8

"""Continuous batching: requests admitted while others run give the same
result as solved alone, admission respects the arena budget, and the
open-loop driver reports latencies."""
import numpy as np
import pytest

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
    with pd.Solver(arena_bytes=2 * need + (4 << 20), device=0) as s:
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
        err = np.linalg.norm(r.chi.cpu().numpy() - ref) / np.linalg.norm(ref)
        assert err <= 1e-4

"""Context lifecycle and host concurrency through the C ABI: submissions and
polls from several host threads at once give each request its solo result,
and destroying a context with requests still queued or running returns
promptly and leaves the device usable."""
import threading
import time

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


def _case(seed, nz, ny, nx, iters):
    w = pd_inputs.random_stack(seed, nz, ny, nx, lam=1e-3, max_iter=iters)
    return w, pd_inputs.make_delta(oracle.forward(w.chi_true), w.eta, w.rho).astype(np.float32)


def test_concurrent_submitters_get_their_solo_results(torch_mod):
    import paper_2006_09808_amd as pd
    torch = torch_mod
    shapes = [(3, 64, 64, 40), (2, 128, 128, 30), (4, 96, 64, 35), (1, 256, 256, 25)]
    cases = [_case(700 + i, *sh) for i, sh in enumerate(shapes)]
    with pd.Solver(arena_bytes=1 << 30, device=0) as s:
        solo = []
        for w, d in cases:
            chi, info = s.solve(torch.from_numpy(d).to("cuda:0"), **w.solver_params())
            solo.append((chi.cpu().numpy(), info["iterations"]))
        results = {}
        errors = []

        def worker(k):
            try:
                for rep in range(3):
                    for i in range(len(cases)):
                        w, d = cases[(i + k) % len(cases)]
                        dt = torch.from_numpy(d).to("cuda:0")
                        out = torch.empty_like(dt)
                        (t,) = s.submit([(dt, out, w.solver_params())])
                        info = s.poll(t, -1)
                        results[(k, rep, (i + k) % len(cases))] = (out.cpu().numpy(), info)
            except Exception as e:          # reported below, in the test's thread
                errors.append(repr(e))

        threads = [threading.Thread(target=worker, args=(k,)) for k in range(4)]
        for th in threads:
            th.start()
        for th in threads:
            th.join(timeout=120)
        assert not any(th.is_alive() for th in threads)
    assert not errors, errors
    assert len(results) == 4 * 3 * len(cases)
    for (k, rep, i), (chi, info) in results.items():
        assert info["status"] == pd.PD_OK and info["iterations"] == solo[i][1]
        np.testing.assert_array_equal(chi, solo[i][0])
    _say("%d solves from 4 threads equal their solo runs" % len(results))


def test_destroy_with_requests_in_flight(torch_mod):
    import paper_2006_09808_amd as pd
    torch = torch_mod
    w, d = _case(720, 64, 256, 256, 5000)
    s = pd.Solver(arena_bytes=1 << 30, device=0)
    dt = torch.from_numpy(d).to("cuda:0")
    outs = [torch.empty_like(dt) for _ in range(3)]
    tickets = s.submit([(dt, o, w.solver_params()) for o in outs])     # more than one fits: some queue
    time.sleep(0.02)
    _, resident, queued = s.arena_usage()
    _say("in flight at destroy: %d resident, %d queued" % (resident, queued))
    assert resident + queued >= 1
    t0 = time.perf_counter()
    s.close()
    dt_close = time.perf_counter() - t0
    _say("destroy took %.1f ms" % (dt_close * 1e3))
    assert dt_close < 5.0
    assert len(tickets) == 3
    # the device and the library are still usable
    w2, d2 = _case(721, 2, 64, 64, 20)
    with pd.Solver(arena_bytes=256 << 20, device=0) as s2:
        chi, info = s2.solve(torch.from_numpy(d2).to("cuda:0"), **w2.solver_params())
    ref, _ = oracle.solve(d2.astype(np.float64), **w2.solver_params())
    assert info["status"] == pd.PD_OK
    _parity.check(chi.cpu().numpy(), ref, "chi")


def test_tune_cache_file_round_trip(torch_mod, tmp_path):
    """pd_config.tune_cache: pd_tune and pd_tune_set write the choices, a new
    context reads them back; lines that do not parse or that pd_tune_set would
    reject are skipped."""
    import paper_2006_09808_amd as pd
    path = tmp_path / "tune.txt"
    with pd.Solver(arena_bytes=1 << 30, device=0, tune_cache=str(path)) as s:
        s.tune(128, 128, 8, iters=10)
        choice = s.tune_get(128, 128)
        s.tune_set(96, 64, -1, 8, 8)
    text = path.read_text()
    _say("tune cache:\n" + text)
    assert text.count("\n") == 2 and "128 128 " in text and "96 64 " in text
    path.write_text(text + "not a choice\n128 128 99 0 0\n96 64 -1 7 0\n")
    with pd.Solver(arena_bytes=256 << 20, device=0, tune_cache=str(path)) as s2:
        assert s2.tune_get(128, 128) == choice
        got = s2.tune_get(96, 64)
        assert (got["rows"], got["cols"]) == (8, 8)


def test_resident_barrier_giveup_recovers(torch_mod):
    """A resident launch whose team barrier gives up does not end the context:
    its requests restart on the two-launch path and finish with the unforced
    run's iterates up to rounding, a request of another shape in the same
    rounds is unaffected (bitwise), and later requests of the shape keep to
    the two-launch path.  The give-up is forced from the host: the context's
    test flag makes every barrier give up at its first wait, so every
    workgroup exits through the kernel's own abort path."""
    import paper_2006_09808_amd as pd
    torch = torch_mod
    wa, da = _case(730, 6, 256, 256, 0)
    wb, db = _case(731, 3, 96, 64, 0)
    pa = dict(wa.solver_params(), max_iter=120, gap_tol=1e-12, check_every=40)
    pb = dict(wb.solver_params(), max_iter=90)
    ta, tb = torch.from_numpy(da).to("cuda:0"), torch.from_numpy(db).to("cuda:0")

    def run(s):
        oa, ob = torch.empty_like(ta), torch.empty_like(tb)
        t = s.submit([(ta, oa, pa), (tb, ob, pb)])
        ia, ib = s.poll(t[0], -1), s.poll(t[1], -1)
        assert ia["status"] == pd.PD_OK and ib["status"] == pd.PD_OK
        return oa.cpu().numpy(), ia, ob.cpu().numpy(), ib

    with pd.Solver(arena_bytes=1 << 30, device=0) as s:
        ra, ira, rb, irb = run(s)
        assert s.recovery_stats() == (0, 0)
    with pd.Solver(arena_bytes=1 << 30, device=0, barrier_giveup_test=True) as s:
        _say("PD_FLAG_TEST_BARRIER_GIVEUP: 256x256x6 (resident shape) beside 96x64x3")
        ga, iga, gb, igb = run(s)
        aborted, restarted = s.recovery_stats()
        _say("aborted rounds %d, restarted requests %d" % (aborted, restarted))
        assert aborted >= 1 and restarted >= 1
        assert iga["iterations"] == ira["iterations"] == 120 and igb["iterations"] == irb["iterations"] == 90
        _parity.check(ga, ra, "restarted request vs unforced run", rel_tol=1e-5, vox_tol=1e-5)
        assert iga["primal"] == pytest.approx(ira["primal"], rel=1e-5)
        np.testing.assert_array_equal(gb, rb)
        ref, _ = oracle.solve(da.astype(np.float64), **dict(pa, gap_tol=0.0))
        _parity.check(ga, ref, "restarted request vs oracle")
        # the shape now runs on the two-launch path: no further give-up
        ga2, iga2, _, _ = run(s)
        assert s.recovery_stats() == (aborted, restarted)
        np.testing.assert_array_equal(ga2, ga)

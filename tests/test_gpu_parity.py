"""GPU parity: the HIP solver (through the C ABI) against the FP64 oracle.

Inputs are seeded phantoms; the field map is made by the oracle's own forward
operator and rounded to FP32, and the same FP32 field map goes to both sides.
Bar (tests/_parity.py): relative L2 error on chi <= 1e-4 after a fixed
iteration count, and every voxel within 1e-4 of max|chi_oracle| (FP32 GPU
arithmetic against FP64; the observed errors are ~1e-6 of either).
"""
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


@pytest.fixture(scope="module")
def solver(torch_mod):
    import paper_2006_09808_amd as pd
    s = pd.Solver(arena_bytes=4 << 30, device=0)
    yield s
    s.close()


@pytest.fixture(scope="module")
def solver_two(torch_mod):
    """Same library, resident kernel disabled: two launches per iteration."""
    import paper_2006_09808_amd as pd
    s = pd.Solver(arena_bytes=4 << 30, device=0, resident=False)
    yield s
    s.close()


@pytest.fixture(scope="module")
def solver_fenced(torch_mod):
    """Resident kernel exchanging through agent-scope release/acquire fences
    (the protocol used when a team's workgroups are not on one XCD)."""
    import paper_2006_09808_amd as pd
    s = pd.Solver(arena_bytes=4 << 30, device=0, fenced_exchange=True, step_iters=11)
    yield s
    s.close()


@pytest.fixture(scope="module")
def solver_short(torch_mod):
    """Resident kernel with 7-iteration steps: state saved and restored
    between launches, gap checks at step ends."""
    import paper_2006_09808_amd as pd
    s = pd.Solver(arena_bytes=4 << 30, device=0, step_iters=7)
    yield s
    s.close()


def make_case(seed, nz, ny, nx, b0=(0.0, 1.0, 0.0), voxel=(1.0, 1.0), **params):
    w = pd_inputs.random_stack(seed, nz, ny, nx, **params)
    w.b0, w.voxel = b0, voxel
    field = oracle.forward(w.chi_true, b0=b0, voxel=voxel)
    delta = pd_inputs.make_delta(field, w.eta, w.rho).astype(np.float32)
    return w, delta


def gpu_solve(solver, torch, delta, **params):
    d = torch.from_numpy(np.ascontiguousarray(delta)).to("cuda:0")
    chi, info = solver.solve(d, **params)
    return chi.cpu().numpy().astype(np.float64), info


rel_l2 = _parity.rel_l2


APPLY_CASES = [
    (3, 8, 8, (0, 1, 0), (1, 1)),
    (2, 64, 64, (0, 1, 0), (1, 1)),
    (3, 64, 96, (0.3, 0.5, 0.8), (0.72, 1.0)),
    (2, 128, 192, (0, 1, 0), (1, 1)),
    (1, 384, 24, (1, 1, 0), (1, 1)),
    (2, 16, 512, (0, 1, 0), (1, 1)),
    (2, 256, 256, (0, 1, 0), (1, 1)),
    (5, 32, 48, (0, 0.6, 0.8), (1, 2)),
    (1, 384, 384, (0, 1, 0), (1, 1)),
]


@pytest.mark.parametrize("nz,ny,nx,b0,vox", APPLY_CASES)
def test_forward_operator_matches_oracle(solver, torch_mod, nz, ny, nx, b0, vox):
    _say("apply_kernel nz=%d ny=%d nx=%d b0=%s voxel=%s" % (nz, ny, nx, b0, vox))
    rng = np.random.default_rng(nz * 1000 + ny + nx)
    x = rng.normal(size=(nz, ny, nx)).astype(np.float32)
    ref = oracle.forward(x.astype(np.float64), b0=b0, voxel=vox)
    xt = torch_mod.from_numpy(x).to("cuda:0")
    out = solver.apply_kernel(xt, b0=b0, voxel=vox).cpu().numpy().astype(np.float64)
    _parity.check(out, ref, "A x", rel_tol=1e-5, vox_tol=1e-5)


SOLVE_CASES = [
    # (seed, nz, ny, nx, params)
    (1, 3, 64, 96, dict(lam=1e-3, max_iter=80, b0=(0.3, 0.5, 0.8), voxel=(0.72, 1.0))),
    (2, 2, 192, 128, dict(lam=1e-3, max_iter=60)),
    (3, 1, 24, 384, dict(lam=1e-3, max_iter=40)),
    (4, 2, 16, 512, dict(lam=1e-3, max_iter=30)),
    (5, 5, 48, 32, dict(lam=2e-3, max_iter=50, theta=0.5, tau=1.0, sigma=1.2)),
    (6, 4, 128, 128, dict(lam=1e-3, max_iter=100)),
    (7, 3, 256, 256, dict(lam=1e-3, max_iter=40)),
    (8, 5, 64, 64, dict(lam=1e-3, max_iter=45, b0=(0.6, 0.8, 0.0), theta=0.7)),
    (9, 3, 192, 192, dict(lam=1e-3, max_iter=50)),
    (10, 2, 64, 64, dict(lam=1e-3, max_iter=30, theta=0.0)),                 # no over-relaxation
    (11, 3, 48, 64, dict(lam=1e-3, max_iter=40, b0=(0.0, 0.0, 1.0))),        # B0 normal to the slices: D = 1/3 off k = 0
]


@pytest.mark.parametrize("path", ["default", "two_launch", "short_steps", "fenced"])
@pytest.mark.parametrize("seed,nz,ny,nx,params", SOLVE_CASES)
def test_fixed_iterations_match_oracle(request, torch_mod, path, seed, nz, ny, nx, params):
    solver = request.getfixturevalue({"default": "solver", "two_launch": "solver_two",
                                      "short_steps": "solver_short", "fenced": "solver_fenced"}[path])
    _say("solve [%s] seed=%d nz=%d ny=%d nx=%d %s" % (path, seed, nz, ny, nx, params))
    p = dict(params)
    b0 = p.pop("b0", (0.0, 1.0, 0.0))
    vox = p.pop("voxel", (1.0, 1.0))
    w, delta = make_case(seed, nz, ny, nx, b0=b0, voxel=vox, **p)
    sp = w.solver_params()
    got, info = gpu_solve(solver, torch_mod, delta, **sp)
    ref, iref = oracle.solve(delta.astype(np.float64), **sp)
    _say("  P %.8e (oracle %.8e)" % (info["primal"], iref["primal"]))
    assert info["iterations"] == iref["iterations"] == sp["max_iter"]
    _parity.check(got, ref, "chi")
    assert info["primal"] == pytest.approx(iref["primal"], rel=1e-4)


@pytest.mark.parametrize("path", ["default", "two_launch"])
@pytest.mark.parametrize("iters", [1, 2, 10])
@pytest.mark.parametrize("nz,ny,nx", [(2, 64, 64), (3, 256, 256), (3, 96, 64)])
def test_first_iterations_match_oracle(request, torch_mod, path, iters, nz, ny, nx):
    """The first iterates, where the over-relaxed point and the dual start
    from zero, with a gap check after every iteration (tolerance never met)."""
    solver = request.getfixturevalue({"default": "solver", "two_launch": "solver_two"}[path])
    w, delta = make_case(600 + nx + iters, nz, ny, nx, lam=1e-3, max_iter=iters, gap_tol=1e-14, check_every=1)
    sp = w.solver_params()
    got, info = gpu_solve(solver, torch_mod, delta, **sp)
    ref, iref = oracle.solve(delta.astype(np.float64), **sp)
    _say("[%s] %dx%dx%d after %d: gap %.6e (oracle %.6e)" % (path, nx, ny, nz, iters,
                                                           info["rel_gap"], iref["rel_gap"]))
    assert info["iterations"] == iref["iterations"] == iters
    _parity.check(got, ref, "chi")
    assert info["rel_gap"] == pytest.approx(iref["rel_gap"], rel=1e-4)
    assert info["primal"] == pytest.approx(iref["primal"], rel=1e-5)


def test_config1_plain_64x64(solver, torch_mod):
    w = pd_inputs.config1()
    field = oracle.forward(w.chi_true)
    delta = pd_inputs.make_delta(field, w.eta, w.rho).astype(np.float32)
    sp = w.solver_params()
    _say("config1 64x64x1, %d iterations" % sp["max_iter"])
    got, info = gpu_solve(solver, torch_mod, delta, **sp)
    ref, iref = oracle.solve(delta.astype(np.float64), **sp)
    _parity.check(got, ref, "chi")
    assert info["iterations"] == 200


@pytest.mark.parametrize("path", ["default", "two_launch", "fenced"])
@pytest.mark.parametrize("shape", [(2, 64, 64), (3, 128, 128), (2, 96, 64), (2, 256, 256)])
def test_gap_report_matches_oracle(request, torch_mod, path, shape):
    solver = request.getfixturevalue({"default": "solver", "two_launch": "solver_two",
                                      "fenced": "solver_fenced"}[path])
    w, delta = make_case(11, *shape, lam=1e-3, max_iter=40, gap_tol=1e-12, check_every=10)
    sp = w.solver_params()
    _say("gap report 64x64x2, 40 iterations, checks every 10")
    hist = []
    ref, iref = oracle.solve(delta.astype(np.float64), history=hist, **sp)
    got, info = gpu_solve(solver, torch_mod, delta, **sp)
    _say("  P %.10e / %.10e  D %.10e / %.10e  relgap %.6e / %.6e" % (
        info["primal"], iref["primal"], info["dual"], iref["dual"], info["rel_gap"], iref["rel_gap"]))
    assert info["iterations"] == 40
    assert info["primal"] == pytest.approx(iref["primal"], rel=1e-5)
    assert info["dual"] == pytest.approx(iref["dual"], rel=1e-4)
    assert abs(info["rel_gap"] - iref["rel_gap"]) <= 1e-4 * max(1.0, abs(iref["rel_gap"]))
    _parity.check(got, ref, "chi")


@pytest.mark.parametrize("shape", [(3, 32, 64), (3, 64, 64), (2, 128, 128)])
def test_identity_kernel_tolerance_stop(solver, torch_mod, shape):
    rng = np.random.default_rng(21)
    delta = rng.normal(size=shape).astype(np.float32)
    sp = dict(lam=0.2, tau=0.9, sigma=0.9, theta=1.0, max_iter=400, gap_tol=1e-5, check_every=5,
              kernel="identity")
    _say("identity kernel, gap_tol 1e-5")
    hist = []
    ref, iref = oracle.solve(delta.astype(np.float64), history=hist,
                             **{k: v for k, v in sp.items() if k != "kernel"}, kind="identity")
    got, info = gpu_solve(solver, torch_mod, delta, **sp)
    _say("  oracle stop %d relgap %.3e; gpu stop %d relgap %.3e" % (
        iref["iterations"], iref["rel_gap"], info["iterations"], info["rel_gap"]))
    assert info["iterations"] < 400 and info["iterations"] % 5 == 0
    assert info["rel_gap"] <= 1e-5
    # the stop check can differ by one check period only when the oracle's gap
    # lands within FP32 rounding of the tolerance
    assert abs(info["iterations"] - iref["iterations"]) <= 5
    ref_same, _ = oracle.solve(delta.astype(np.float64), kind="identity",
                               **dict((k, v) for k, v in sp.items() if k not in ("kernel", "gap_tol")
                                      and k != "max_iter"), max_iter=info["iterations"])
    _parity.check(got, ref_same, "chi")
    closed = np.sign(delta) * np.maximum(np.abs(delta.astype(np.float64)) - 0.2, 0.0)
    assert np.max(np.abs(got - closed)) <= 1e-3


def test_zero_iterations(solver, torch_mod):
    w, delta = make_case(12, 3, 32, 32, max_iter=0)
    sp = w.solver_params()
    got, info = gpu_solve(solver, torch_mod, delta, **sp)
    ref, iref = oracle.solve(delta.astype(np.float64), **sp)
    assert info["iterations"] == 0
    assert np.all(got == 0.0)
    assert info["primal"] == pytest.approx(iref["primal"], rel=1e-5)
    assert info["rel_gap"] == pytest.approx(1.0, abs=1e-6)


def test_batch_results_equal_solo_results(solver, torch_mod):
    import paper_2006_09808_amd as pd
    torch = torch_mod
    cases = [make_case(31, 3, 64, 64, max_iter=37), make_case(32, 2, 96, 64, max_iter=55),
             make_case(33, 1, 64, 64, max_iter=20, gap_tol=1e-9, check_every=10)]
    _say("batch of 3 requests (two shapes) vs solo")
    solo = []
    for w, d in cases:
        got, info = gpu_solve(solver, torch, d, **w.solver_params())
        solo.append((got, info))
    jobs = []
    for w, d in cases:
        dt = torch.from_numpy(d).to("cuda:0")
        jobs.append((dt, torch.empty_like(dt), w.solver_params()))
    tickets = solver.submit(jobs)
    for (dt, chi, _), t, (sgot, sinfo) in zip(jobs, tickets, solo):
        info = solver.poll(t, -1)
        assert info["status"] == pd.PD_OK
        assert info["iterations"] == sinfo["iterations"]
        np.testing.assert_array_equal(chi.cpu().numpy().astype(np.float64), sgot)


def test_staggered_gap_stops_in_one_batch_equal_solo_runs(solver, torch_mod):
    """Volumes whose gap reaches the tolerance at different checks share the
    scheduler's rounds of several steps with a volume that runs to its cap:
    launches after a mid-round stop skip the stopped volume, so every result,
    iteration count and gap equals the volume's solo run."""
    import paper_2006_09808_amd as pd
    torch = torch_mod
    rng = np.random.default_rng(401)
    cases = []
    for ts, lam in ((0.3, 0.3), (0.2, 0.05), (0.1, 0.3)):     # identity kernel: stops near 70, 120, 190
        d = rng.normal(size=(2, 32, 48)).astype(np.float32)
        cases.append((d, dict(lam=lam, tau=ts, sigma=ts, theta=1.0, max_iter=400, gap_tol=1e-5, check_every=5,
                              kernel="identity")))
    w, d = make_case(402, 3, 64, 64, max_iter=150, gap_tol=1e-5, check_every=5)
    cases.append((d, w.solver_params()))
    _say("staggered gap stops: 3 identity volumes + 1 dipole volume capped at 150")
    jobs = []
    for d, sp in cases:
        dt = torch.from_numpy(d).to("cuda:0")
        jobs.append((dt, torch.empty_like(dt), sp))
    infos = [solver.poll(t, -1) for t in solver.submit(jobs)]
    its = [i["iterations"] for i in infos]
    _say("  iterations %s" % (its,))
    assert all(i["status"] == pd.PD_OK for i in infos)
    assert its[3] == 150
    assert len(set(its[:3])) == 3 and max(its[:3]) < 400
    for (dt, chi, sp), info in zip(jobs, infos):
        solo = torch.empty_like(dt)
        (t,) = solver.submit([(dt, solo, sp)])
        sinfo = solver.poll(t, -1)
        assert sinfo["iterations"] == info["iterations"]
        assert sinfo["rel_gap"] == info["rel_gap"]
        np.testing.assert_array_equal(solo.cpu().numpy(), chi.cpu().numpy())


def test_deterministic_bitwise(solver, torch_mod):
    w, delta = make_case(41, 4, 128, 64, max_iter=30)
    a, _ = gpu_solve(solver, torch_mod, delta, **w.solver_params())
    b, _ = gpu_solve(solver, torch_mod, delta, **w.solver_params())
    np.testing.assert_array_equal(a, b)


def test_nonfinite_input_reported(solver, torch_mod):
    import paper_2006_09808_amd as pd
    delta = np.zeros((2, 32, 32), dtype=np.float32)
    delta[1, 5, 7] = np.nan
    d = torch_mod.from_numpy(delta).to("cuda:0")
    chi = torch_mod.empty_like(d)
    (t,) = solver.submit([(d, chi, dict(max_iter=20, gap_tol=1e-6, check_every=5))])
    info = solver.poll(t, -1)
    assert info["status"] == pd.PD_ERR_NONFINITE


def test_budget_and_queueing(torch_mod):
    import paper_2006_09808_amd as pd
    torch = torch_mod
    need = pd.validate(64, 64, 4)
    # room for one request at a time: the others wait in the queue
    with pd.Solver(arena_bytes=need + (need // 2) + (1 << 20), device=0) as s:
        with pytest.raises(pd.PdError) as e:
            big = torch.zeros((64, 256, 256), device="cuda:0")
            s.submit([(big, torch.empty_like(big), dict(max_iter=1))])
        assert e.value.status == pd.PD_ERR_BUDGET
        cases = [make_case(50 + i, 4, 64, 64, max_iter=25) for i in range(3)]
        jobs = []
        for w, d in cases:
            dt = torch.from_numpy(d).to("cuda:0")
            jobs.append((dt, torch.empty_like(dt), w.solver_params()))
        tickets = s.submit(jobs)
        for (dt, chi, _), t, (w, d) in zip(jobs, tickets, cases):
            info = s.poll(t, -1)
            assert info["status"] == pd.PD_OK and info["iterations"] == 25
            ref, _ = oracle.solve(d.astype(np.float64), **w.solver_params())
            _parity.check(chi.cpu().numpy().astype(np.float64), ref, "chi")


def test_batched_config_full_size_sampled(solver, torch_mod):
    """64 slices of 256x256, 500 iterations, one batched solve; in fixed-count
    mode slices are independent, so sampled slices are checked against the
    oracle solved on those slices alone."""
    w = pd_inputs.config2()
    _say("batched 256x256x64, 500 iterations (sampled slices vs oracle)")
    field = oracle.forward(w.chi_true)
    delta = pd_inputs.make_delta(field, w.eta, w.rho).astype(np.float32)
    sp = w.solver_params()
    got, info = gpu_solve(solver, torch_mod, delta, **sp)
    assert info["iterations"] == 500
    for z in (0, 37, 63):
        ref, _ = oracle.solve(delta[z:z + 1].astype(np.float64), **sp)
        _parity.check(got[z:z + 1], ref, "slice %d" % z)
    # the launch configuration the benchmark times: the autotuner's choice for
    # this shape (every resident variant does the same arithmetic, so equal bits)
    import paper_2006_09808_amd as pd
    with pd.Solver(arena_bytes=1 << 30, device=0) as tuned:
        tuned.tune(256, 256, 64, iters=50)
        choice = tuned.tune_get(256, 256)
        got_t, info_t = gpu_solve(tuned, torch_mod, delta, **sp)
    _say("  tuned choice %r" % (choice,))
    assert info_t["iterations"] == 500
    if choice["variant"] >= 0:
        np.testing.assert_array_equal(got_t, got)
    else:
        assert rel_l2(got_t, got) <= 1e-5


def test_resident_batch_split_across_launches(solver, torch_mod):
    """66 slices of 256x256 (33 pairs) exceed one co-resident launch (32 pairs
    of 8 workgroups on 256 CUs), so one volume spans two launches."""
    w, delta = make_case(61, 66, 256, 256, lam=1e-3, max_iter=30)
    sp = w.solver_params()
    _say("256x256x66, 30 iterations (two resident launches per step)")
    got, info = gpu_solve(solver, torch_mod, delta, **sp)
    assert info["iterations"] == 30
    for z in (0, 63, 64, 65):
        ref, _ = oracle.solve(delta[z:z + 1].astype(np.float64), **sp)
        _parity.check(got[z:z + 1], ref, "slice %d" % z)


@pytest.mark.parametrize("n", [64, 256])
def test_resident_short_launches_equal_one_launch(torch_mod, n):
    """Inside a launch the resident kernel hands the half-transformed field
    between its phases in a blocked layout and converts it to and from the
    [ny][nx] layout at the launch's first and last iteration.  Launches of 1,
    2 and 5 iterations (every iteration a boundary, with and without gap
    checks at launch ends) give the bits of one launch over all iterations."""
    import paper_2006_09808_amd as pd
    for gap_tol, check_every in ((0.0, 10), (1e-12, 4)):
        w, delta = make_case(81, 5, n, n, lam=1e-3, max_iter=12, gap_tol=gap_tol, check_every=check_every)
        sp = w.solver_params()
        with pd.Solver(arena_bytes=1 << 30, device=0) as s:
            ref, iref = gpu_solve(s, torch_mod, delta, **sp)
        for k in (1, 2, 5):
            with pd.Solver(arena_bytes=1 << 30, device=0, step_iters=k, time_kernels=True) as s:
                got, info = gpu_solve(s, torch_mod, delta, **sp)
                n_res, _, _ = s.kernel_time(pd.KIND_RESIDENT)
            _say("%dx%d gap_tol %g, steps of %d: %d resident launches" % (n, n, gap_tol, k, n_res))
            assert info["iterations"] == iref["iterations"] == 12 and n_res >= 12 // k
            np.testing.assert_array_equal(got, ref)
            assert info["primal"] == pytest.approx(iref["primal"], rel=1e-12)
    ref_o, _ = oracle.solve(delta.astype(np.float64), **sp)
    _parity.check(got, ref_o, "%dx%d short launches" % (n, n))


@pytest.mark.parametrize("n", [64, 128, 192, 256])
def test_resident_protocols_and_two_launch_path_agree(solver, solver_two, solver_fenced, torch_mod, n):
    """Same arithmetic in the same order: the XCD-local and fenced exchange
    give bitwise equal results; the two-launch path agrees to rounding."""
    w, delta = make_case(71, 6, n, n, lam=1e-3, max_iter=44, gap_tol=1e-9, check_every=22)
    sp = w.solver_params()
    a, ia = gpu_solve(solver, torch_mod, delta, **sp)
    f, iff = gpu_solve(solver_fenced, torch_mod, delta, **sp)
    b, ib = gpu_solve(solver_two, torch_mod, delta, **sp)
    assert ia["iterations"] == ib["iterations"] == iff["iterations"] == 44
    np.testing.assert_array_equal(a, f)
    assert rel_l2(a, b) <= 1e-5
    assert ia["primal"] == pytest.approx(ib["primal"], rel=1e-5)


@pytest.mark.parametrize("gap_tol", [0.0, 1e-9])
@pytest.mark.parametrize("ny,nx", [(96, 64), (128, 128)])
def test_graph_replay_equals_eager(torch_mod, gap_tol, ny, nx):
    """Steps replayed from a captured HIP graph give the eager result bitwise,
    on every replay, with eager work in between: the two-launch path (96x64)
    and the resident kernel (128x128, whose launches are captured too)."""
    import paper_2006_09808_amd as pd
    w, delta = make_case(81, 5, ny, nx, lam=1e-3, max_iter=300, gap_tol=gap_tol, check_every=50)
    sp = w.solver_params()
    with pd.Solver(arena_bytes=1 << 30, device=0, step_iters=50, graphs=False) as eager:
        ref, iref = gpu_solve(eager, torch_mod, delta, **sp)
        assert eager.graph_stats() == (0, 0)
    with pd.Solver(arena_bytes=1 << 30, device=0, step_iters=50) as g:
        for rep in range(3):
            got, info = gpu_solve(g, torch_mod, delta, **sp)
            np.testing.assert_array_equal(got, ref)
            assert info["iterations"] == iref["iterations"] == 300
            assert info["primal"] == iref["primal"]
            # eager work between replays: the forward operator on the device
            x = torch_mod.from_numpy(delta).to("cuda:0")
            g.apply_kernel(x)
        captures, replays = g.graph_stats()
        _say("graph captures %d replays %d" % (captures, replays))
        assert captures >= 1 and replays >= 8


@pytest.mark.parametrize("n,nz", [(256, 6), (128, 5), (64, 3), (192, 4), (96, 3), (384, 3), (512, 2)])
def test_autotune_configurations_agree(torch_mod, n, nz):
    """Every configuration the autotuner can pick.  Resident variants and tile
    sizes distribute the same arithmetic differently, so chi is bitwise
    identical across them; an FFT pass plan other than the default changes
    the rounding only, so chi stays within 1e-5 of the default plan's and
    within the parity bar of the oracle.  The choice is the fastest of each
    kind."""
    import paper_2006_09808_amd as pd
    w, delta = make_case(91, nz, n, n if n != 96 else 64, lam=1e-3, max_iter=33)
    ny, nx = delta.shape[1], delta.shape[2]
    sp = w.solver_params()
    oref, _ = oracle.solve(delta.astype(np.float64), **sp)
    with pd.Solver(arena_bytes=1 << 30, device=0) as s, \
            pd.Solver(arena_bytes=1 << 30, device=0, resident=False) as s2:
        table = s.tune(nx, ny, nz, iters=10)
        _say("tune %dx%d: %s" % (nx, ny, ["%s v%d %dx%d r%d c%d p%d %.3f ms" % (
            t["path"], t["variant"], t["team"], t["threads"], t["rows"], t["cols"], t["plan"], t["ms"])
            for t in table]))
        choice = s.tune_get(nx, ny)
        res = [t for t in table if t["path"] == "resident"]
        cols = [t for t in table if t["path"] == "column"]
        rows = [t for t in table if t["path"] == "row"]
        assert cols and rows
        if res:
            assert choice["variant"] == min(res, key=lambda t: t["ms"])["variant"]
        bc, br = min(cols, key=lambda t: t["ms"]), min(rows, key=lambda t: t["ms"])
        assert (choice["cols"], choice["plan_y"]) == (bc["cols"], bc["plan"])
        assert (choice["rows"], choice["plan_x"]) == (br["rows"], br["plan"])
        assert len({t["plan"] for t in cols}) == len({t["plan"] for t in rows}) >= (1 if n == 96 else 2)
        ref, _ = gpu_solve(s, torch_mod, delta, **sp)
        _parity.check(ref, oref, "chi, tuned choice")
        ref_plan = {}
        for t in res:
            s.tune_set(nx, ny, t["variant"])
            got, _ = gpu_solve(s, torch_mod, delta, **sp)
            ref_plan.setdefault(t["plan"], got)
            np.testing.assert_array_equal(got, ref_plan[t["plan"]])     # same plan: same bits
            assert rel_l2(got, ref) <= 1e-5
            _parity.check(got, oref, "resident v%d (plan %d)" % (t["variant"], t["plan"]))
        s2.tune_set(nx, ny)
        ref2, _ = gpu_solve(s2, torch_mod, delta, **sp)        # two-launch path, default tiles and plans
        assert rel_l2(ref2, ref) <= 1e-5
        for t in cols + rows:
            if t["path"] == "column":
                s2.tune_set(nx, ny, -1, 0, t["cols"], 0, t["plan"])
            else:
                s2.tune_set(nx, ny, -1, t["rows"], 0, t["plan"], 0)
            got, _ = gpu_solve(s2, torch_mod, delta, **sp)
            what = "%s kernel, tile %d, plan %d" % (t["path"], max(t["rows"], t["cols"]), t["plan"])
            if t["plan"] == 0:
                np.testing.assert_array_equal(got, ref2, err_msg=what)
            else:
                assert rel_l2(got, ref2) <= 1e-5, what
                _parity.check(got, oref, what)
        with pytest.raises(pd.PdError):
            s.tune_set(nx, ny, -1, 7, 0)
        with pytest.raises(pd.PdError):
            s.tune_set(nx, ny, -1, 0, 0, 5, 0)


def test_192_joins_the_multi_shape_launch_and_equals_solo(torch_mod):
    """A 192x192 volume runs as a body of the multi-shape launch next to a
    256x256 one (its body spills to scratch at two waves per SIMD); both
    equal their solo runs bitwise, and the oracle on sampled slices.  The solo
    runs use the variants whose teams the bodies have (192: 12 x 256, 256:
    16 x 256), so the FP64 gap partials are summed in the same order and the
    gap is bitwise equal too."""
    import paper_2006_09808_amd as pd
    torch = torch_mod
    cases = [make_case(1211, 6, 192, 192, lam=1e-3, max_iter=40, gap_tol=1e-12, check_every=20),
             make_case(1212, 4, 256, 256, lam=1e-3, max_iter=40)]
    with pd.Solver(arena_bytes=1 << 30, device=0, time_kernels=True) as s:
        s.tune_set(192, 192, 0)
        s.tune_set(256, 256, 1)
        solo = [gpu_solve(s, torch, d, **w.solver_params()) for w, d in cases]
        s.kernel_time_reset()
        ins = [torch.from_numpy(d).to("cuda:0") for _, d in cases]
        outs = [torch.empty_like(x) for x in ins]
        ts = s.submit([(x, o, w.solver_params()) for x, o, (w, _) in zip(ins, outs, cases)])
        infos = [s.poll(t, -1) for t in ts]
        n_multi, _, _ = s.kernel_time(pd.KIND_MULTI)
        n_single, _, _ = s.kernel_time(pd.KIND_RESIDENT)
    _say("multi-shape launches %d, single-shape resident launches %d" % (n_multi, n_single))
    assert n_multi >= 1 and n_single == 0
    for (w, d), o, info, (chi_solo, info_solo) in zip(cases, outs, infos, solo):
        assert info["status"] == pd.PD_OK and info["iterations"] == info_solo["iterations"]
        got = o.cpu().numpy().astype(np.float64)
        np.testing.assert_array_equal(got, chi_solo)
        assert info["primal"] == info_solo["primal"]
        ref, _ = oracle.solve(d[:2].astype(np.float64), **w.solver_params())
        _parity.check(got[:2], ref, "%dx%d slices 0-1" % (d.shape[1], d.shape[2]))


@pytest.mark.parametrize("v128", [0, 4])
def test_uneven_shapes_share_one_launch_and_equal_solo(torch_mod, v128):
    """Volumes of 64x64, 128x128 and 256x256 submitted together run as teams
    of one multi-shape resident launch per step (each XCD's workgroups hold
    teams of several shapes); each volume equals its solo run (its own
    single-shape launches) bitwise, and the oracle on sampled slices.  The
    128x128 volume runs the default FFT plan (variant 0) or 8 x 4 x 4
    (variant 4): the launch picks the body of the chosen variant's plan."""
    import paper_2006_09808_amd as pd
    torch = torch_mod
    cases = [make_case(1201, 5, 64, 64, lam=1e-3, max_iter=70, gap_tol=1e-12, check_every=35),
             make_case(1202, 6, 128, 128, lam=1e-3, max_iter=60),
             make_case(1203, 7, 256, 256, lam=1e-3, max_iter=50)]
    with pd.Solver(arena_bytes=1 << 30, device=0, time_kernels=True) as s:
        s.tune_set(128, 128, v128)
        s.tune_set(256, 256, 1)   # the team structure of the 256x256 body: the gap sums in the same order
        solo = [gpu_solve(s, torch, d, **w.solver_params()) for w, d in cases]
        s.kernel_time_reset()
        ins = [torch.from_numpy(d).to("cuda:0") for _, d in cases]
        outs = [torch.empty_like(x) for x in ins]
        ts = s.submit([(x, o, w.solver_params()) for x, o, (w, _) in zip(ins, outs, cases)])
        infos = [s.poll(t, -1) for t in ts]
        n_multi, ms, _ = s.kernel_time(pd.KIND_MULTI)
        n_single, _, _ = s.kernel_time(pd.KIND_RESIDENT)
    _say("multi-shape launches %d (%.2f ms), single-shape resident launches %d" % (n_multi, ms, n_single))
    assert n_multi >= 1
    for (w, d), o, info, (chi_solo, info_solo) in zip(cases, outs, infos, solo):
        assert info["status"] == pd.PD_OK and info["iterations"] == info_solo["iterations"]
        got = o.cpu().numpy().astype(np.float64)
        np.testing.assert_array_equal(got, chi_solo)
        assert info["primal"] == info_solo["primal"]
        ref, _ = oracle.solve(d[:2].astype(np.float64), **w.solver_params())
        _parity.check(got[:2], ref, "%dx%d slices 0-1" % (d.shape[1], d.shape[2]))

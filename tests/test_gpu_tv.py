"""GPU parity of the weighted TV model (Eq. (1)) through the C ABI against
the FP64 TV oracle.

Inputs are seeded device stacks with magnitude-like weights W and an
elliptical mask M; the field map is made by the oracle's forward operator and
rounded to FP32, and the same FP32 delta, W and M go to both sides.  Bar
(tests/_parity.py): relative L2 error on chi <= 1e-4 and every voxel within
1e-4 of max|chi_oracle| after a fixed iteration count (FP32 GPU arithmetic
against FP64), 1e-10 for both in the FP64 GPU build.
"""
import numpy as np
import pytest

import _parity
import oracle
import pd_inputs

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)


rel_l2 = _parity.rel_l2


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
def solver64(torch_mod):
    import paper_2006_09808_amd as pd
    s = pd.Solver(arena_bytes=4 << 30, device=0, precision="fp64")
    yield s
    s.close()


def make_tv_case(seed, nz, ny, nx, b0=(0.0, 1.0, 0.0), voxel=(1.0, 1.0), iters=40, lam=100.0):
    w = pd_inputs.tv_stack(seed, nz, ny, nx, max_iter=iters, lam=lam, b0=b0, voxel=voxel)
    # steps inside the bound tau sigma (max|W|^2 max|D|^2 + max|M|^2 (4/dx^2 + 4/dy^2)) < 1
    D = oracle.dipole_kernel(nx, ny, b0, voxel)
    L2 = oracle.kernel_norm(D) ** 2 + oracle.grad_norm_bound(voxel)
    w.tau = w.sigma = 0.95 / np.sqrt(L2)
    field = oracle.forward(w.chi_true, b0=b0, voxel=voxel)
    delta = pd_inputs.make_delta(field, w.eta, w.rho).astype(np.float32)
    return w, delta, w.weight.astype(np.float32), w.mask.astype(np.float32)


def to_dev(torch, a, dtype):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0", dtype=dtype)


def gpu_tv(solver, torch, delta, W, M, dtype=None, **params):
    dtype = dtype or torch.float32
    d, wt, mt = (to_dev(torch, a, dtype) for a in (delta, W, M))
    (t,) = solver.submit([(d, torch.empty_like(d), dict(params, model="tv", weight=wt, mask=mt))])
    info = solver.poll(t, -1)
    return info, t


def gpu_tv_solve(solver, torch, delta, W, M, dtype=None, **params):
    dtype = dtype or torch.float32
    d, wt, mt = (to_dev(torch, a, dtype) for a in (delta, W, M))
    chi = torch.empty_like(d)
    (t,) = solver.submit([(d, chi, dict(params, model="tv", weight=wt, mask=mt))])
    info = solver.poll(t, -1)
    return chi.cpu().numpy().astype(np.float64), info


TV_CASES = [
    # (seed, nz, ny, nx, b0, voxel, iters)
    (11, 2, 16, 16, (0.0, 1.0, 0.0), (1.0, 1.0), 30),
    (12, 3, 64, 64, (0.0, 1.0, 0.0), (1.0, 1.0), 60),           # odd nz: padded pair
    (13, 5, 64, 96, (0.3, 0.5, 0.8), (0.8, 1.2), 40),           # rectangular, oblique B0, anisotropic
    (14, 4, 128, 128, (0.0, 1.0, 0.0), (1.0, 1.0), 50),
    (15, 2, 192, 96, (1.0, 1.0, 0.0), (1.0, 0.7), 25),
    (16, 2, 256, 256, (0.0, 1.0, 0.0), (1.0, 1.0), 30),
    (17, 1, 384, 384, (0.0, 1.0, 0.0), (1.0, 1.0), 8),          # single slice, largest rows
]


@pytest.mark.parametrize("case", TV_CASES, ids=lambda c: "%d-%d-%d-%d" % c[:4])
def test_tv_matches_oracle_fixed_iterations(solver, torch_mod, case):
    seed, nz, ny, nx, b0, vox, iters = case
    _say("tv case nz=%d ny=%d nx=%d iters=%d" % (nz, ny, nx, iters))
    w, delta, W, M = make_tv_case(seed, nz, ny, nx, b0, vox, iters)
    sp = w.solver_params()
    chi, info = gpu_tv_solve(solver, torch_mod, delta, W, M, **sp)
    assert info["status"] == 0 and info["iterations"] == iters
    assert np.isnan(info["rel_gap"])
    ref, _ = oracle.solve_tv(delta.astype(np.float64), W.astype(np.float64), M.astype(np.float64), **sp)
    _parity.check(chi, ref, "tv chi")


@pytest.mark.parametrize("case", [TV_CASES[1], TV_CASES[2]], ids=lambda c: "%d-%d-%d-%d" % c[:4])
def test_tv_fp64_matches_oracle(solver64, torch_mod, case):
    seed, nz, ny, nx, b0, vox, iters = case
    w, delta, W, M = make_tv_case(seed, nz, ny, nx, b0, vox, iters)
    sp = w.solver_params()
    chi, info = gpu_tv_solve(solver64, torch_mod, delta.astype(np.float64), W.astype(np.float64),
                             M.astype(np.float64), dtype=torch_mod.float64, **sp)
    assert info["status"] == 0
    ref, _ = oracle.solve_tv(delta.astype(np.float64), W.astype(np.float64), M.astype(np.float64), **sp)
    _parity.check(chi, ref, "fp64 tv chi", rel_tol=1e-10, vox_tol=1e-10)


def test_tv_zero_iterations_give_zero(solver, torch_mod):
    w, delta, W, M = make_tv_case(21, 3, 32, 32, iters=0)
    chi, info = gpu_tv_solve(solver, torch_mod, delta, W, M, **w.solver_params())
    assert info["status"] == 0 and info["iterations"] == 0
    assert np.all(chi == 0)


def test_tv_step_condition_checked_on_device(solver, torch_mod):
    import paper_2006_09808_amd as pd
    w, delta, W, M = make_tv_case(22, 2, 32, 32, iters=20)
    # W = 3 everywhere: the bound grows by 9 max|D|^2 and the steps violate it
    info, _ = gpu_tv(solver, torch_mod, delta, np.full_like(W, 3.0), M, **w.solver_params())
    assert info["status"] == pd.PD_ERR_STEP and info["iterations"] == 0
    # the same steps with the generated W in [0.2, 1] are fine
    info, _ = gpu_tv(solver, torch_mod, delta, W, M, **w.solver_params())
    assert info["status"] == pd.PD_OK and info["iterations"] == 20


def test_tv_nonfinite_input_is_reported(solver, torch_mod):
    import paper_2006_09808_amd as pd
    w, delta, W, M = make_tv_case(23, 2, 32, 32, iters=10)
    M = M.copy()
    M[1, 5, 7] = np.nan
    info, _ = gpu_tv(solver, torch_mod, delta, W, M, **w.solver_params())
    assert info["status"] == pd.PD_ERR_NONFINITE and info["iterations"] == 0


def test_tv_and_l1_volumes_in_one_batch_equal_their_solo_runs(solver, torch_mod):
    torch = torch_mod
    jobs, outs = [], []
    cases = [make_tv_case(31, 3, 64, 64, iters=37), make_tv_case(32, 2, 128, 128, iters=23)]
    for w, delta, W, M in cases:
        d, wt, mt = (to_dev(torch, a, torch.float32) for a in (delta, W, M))
        chi = torch.empty_like(d)
        jobs.append((d, chi, dict(w.solver_params(), model="tv", weight=wt, mask=mt)))
        outs.append(chi)
    l1 = pd_inputs.random_stack(33, 4, 64, 64, max_iter=50)
    field = oracle.forward(l1.chi_true)
    dl1 = to_dev(torch, pd_inputs.make_delta(field, l1.eta, l1.rho).astype(np.float32), torch.float32)
    chi_l1 = torch.empty_like(dl1)
    jobs.append((dl1, chi_l1, l1.solver_params()))
    outs.append(chi_l1)
    infos = [solver.poll(t, -1) for t in solver.submit(jobs)]
    assert all(i["status"] == 0 for i in infos)
    mixed = [o.cpu().numpy() for o in outs]
    for (d, _, params), ref in zip(jobs, mixed):
        solo = torch.empty_like(d)
        (t,) = solver.submit([(d, solo, params)])
        assert solver.poll(t, -1)["status"] == 0
        np.testing.assert_array_equal(solo.cpu().numpy(), ref)


def test_tv_repeated_solves_are_bitwise_equal(solver, torch_mod):
    # the second and later runs of the same plan replay a captured HIP graph
    w, delta, W, M = make_tv_case(41, 4, 96, 96, iters=25)
    outs = []
    for _ in range(3):
        chi, info = gpu_tv_solve(solver, torch_mod, delta, W, M, **w.solver_params())
        assert info["status"] == 0
        outs.append(chi)
    np.testing.assert_array_equal(outs[0], outs[1])
    np.testing.assert_array_equal(outs[0], outs[2])


# ---------------------------------------------------------------------------
# the resident launch of the TV model (square 64², 128², 256² slices)
# ---------------------------------------------------------------------------

@pytest.fixture(scope="module")
def solver_two(torch_mod):
    import paper_2006_09808_amd as pd
    s = pd.Solver(arena_bytes=4 << 30, device=0, resident=False)
    yield s
    s.close()


@pytest.mark.parametrize("case", [(91, 3, 64, 64, 40), (92, 5, 128, 128, 33), (93, 2, 256, 256, 25),
                                  (94, 7, 256, 256, 12), (98, 1, 256, 256, 20)],
                         ids=lambda c: "%d-%d-%d" % (c[2], c[3], c[1]))
def test_tv_resident_matches_four_launch_path_and_oracle(solver, solver_two, torch_mod, case):
    """Square TV volumes of 64², 128² and 256² run as one resident launch per
    step.  Its tiles give every transform the arithmetic of the four-launch
    path's default tiles, and the updates are the same expressions, so the
    two paths agree bitwise, and both meet the oracle's bar."""
    import paper_2006_09808_amd as pd
    seed, nz, ny, nx, iters = case
    w, delta, W, M = make_tv_case(seed, nz, ny, nx, iters=iters)
    sp = w.solver_params()
    chi_r, info = gpu_tv_solve(solver, torch_mod, delta, W, M, **sp)
    chi_t, info_t = gpu_tv_solve(solver_two, torch_mod, delta, W, M, **sp)
    assert info["status"] == info_t["status"] == 0 and info["iterations"] == info_t["iterations"] == iters
    _say("  resident vs four-launch: relL2 %.3e, bitwise %s" % (rel_l2(chi_r, chi_t), np.array_equal(chi_r, chi_t)))
    np.testing.assert_array_equal(chi_r, chi_t)
    ref, _ = oracle.solve_tv(delta.astype(np.float64), W.astype(np.float64), M.astype(np.float64), **sp)
    _parity.check(chi_r, ref, "tv resident chi")
    with pd.Solver(arena_bytes=1 << 30, device=0, time_kernels=True) as s:
        gpu_tv_solve(s, torch_mod, delta, W, M, **sp)
        n_res, _, _ = s.kernel_time(pd.KIND_TV_RESIDENT)
        n_col, _, _ = s.kernel_time(pd.KIND_TV_COLUMN)
        assert n_res >= 1 and n_col == 0
    # the agent-scope exchange protocol (every barrier writes back and
    # invalidates L2) gives the same bits
    with pd.Solver(arena_bytes=1 << 30, device=0, fenced_exchange=True) as s:
        chi_f, _ = gpu_tv_solve(s, torch_mod, delta, W, M, **sp)
    np.testing.assert_array_equal(chi_f, chi_r)


@pytest.mark.timeout(600)
def test_tv_resident_bench_shape_256x256x64(solver, torch_mod):
    """The TV workload the benchmark times (64 slices of 256², all 32 pairs in
    one co-resident launch), a few iterations against the oracle over the
    whole volume."""
    w, delta, W, M = make_tv_case(6000, 64, 256, 256, iters=6)
    sp = w.solver_params()
    chi, info = gpu_tv_solve(solver, torch_mod, delta, W, M, **sp)
    assert info["status"] == 0 and info["iterations"] == 6
    _say("  GPU done; oracle")
    ref, _ = oracle.solve_tv(delta.astype(np.float64), W.astype(np.float64), M.astype(np.float64), **sp)
    _parity.check(chi, ref, "tv resident 256x256x64")
    for z in (0, 1, 62, 63):
        _parity.check(chi[z:z + 1], ref[z:z + 1], "tv resident slice %d" % z)


def test_tv_resident_barrier_giveup_recovers(torch_mod):
    """A TV resident launch whose team barrier gives up (forced from the host:
    every barrier gives up at its first wait) restarts its request on the
    four-launch path; the result equals the unforced run bitwise (the two
    paths compute the same bits)."""
    import paper_2006_09808_amd as pd
    w, delta, W, M = make_tv_case(95, 4, 128, 128, iters=30)
    sp = w.solver_params()
    with pd.Solver(arena_bytes=1 << 30, device=0) as s:
        ref, _ = gpu_tv_solve(s, torch_mod, delta, W, M, **sp)
    with pd.Solver(arena_bytes=1 << 30, device=0, barrier_giveup_test=True) as s:
        got, info = gpu_tv_solve(s, torch_mod, delta, W, M, **sp)
        aborted, restarted = s.recovery_stats()
        _say("  aborted rounds %d, restarted requests %d" % (aborted, restarted))
        assert info["status"] == 0 and info["iterations"] == 30
        assert aborted >= 1 and restarted >= 1
    np.testing.assert_array_equal(got, ref)


def test_tv_resident_more_pairs_than_one_launch_and_short_steps(solver_two, torch_mod):
    """40 slice pairs of 256² (more than one co-resident launch holds: two
    launches per step) and, on another context, steps of 7 iterations (the
    state carries over between resident launches in HBM): both equal the
    four-launch path bitwise."""
    import paper_2006_09808_amd as pd
    w, delta, W, M = make_tv_case(96, 80, 256, 256, iters=12)
    sp = w.solver_params()
    chi_t, _ = gpu_tv_solve(solver_two, torch_mod, delta, W, M, **sp)
    with pd.Solver(arena_bytes=8 << 30, device=0, time_kernels=True) as s:
        chi_r, info = gpu_tv_solve(s, torch_mod, delta, W, M, **sp)
        n_res, _, _ = s.kernel_time(pd.KIND_TV_RESIDENT)
        _say("  80 slices: %d resident launches" % n_res)
        assert info["status"] == 0 and n_res >= 2
    np.testing.assert_array_equal(chi_r, chi_t)
    w, delta, W, M = make_tv_case(97, 6, 128, 128, iters=30)
    sp = w.solver_params()
    chi_t, _ = gpu_tv_solve(solver_two, torch_mod, delta, W, M, **sp)
    with pd.Solver(arena_bytes=1 << 30, device=0, step_iters=7, time_kernels=True) as s:
        chi_r, info = gpu_tv_solve(s, torch_mod, delta, W, M, **sp)
        n_res, _, _ = s.kernel_time(pd.KIND_TV_RESIDENT)
        _say("  steps of 7: %d resident launches" % n_res)
        assert info["status"] == 0 and info["iterations"] == 30 and n_res == 5
    np.testing.assert_array_equal(chi_r, chi_t)


@pytest.mark.parametrize("n", [64, 256])
def test_tv_resident_single_iteration_launches(solver_two, torch_mod, n):
    """Steps of 1 and 3 iterations on the shapes whose resident launch keeps
    the exchange in a blocked layout inside the launch (converted at the
    launch's first and last phase): the four-launch path's bits."""
    import paper_2006_09808_amd as pd
    w, delta, W, M = make_tv_case(99, 4, n, n, iters=7)
    sp = w.solver_params()
    chi_t, _ = gpu_tv_solve(solver_two, torch_mod, delta, W, M, **sp)
    for k in (1, 3):
        with pd.Solver(arena_bytes=1 << 30, device=0, step_iters=k, time_kernels=True) as s:
            chi_r, info = gpu_tv_solve(s, torch_mod, delta, W, M, **sp)
            n_res, _, _ = s.kernel_time(pd.KIND_TV_RESIDENT)
        _say("  %dx%d steps of %d: %d resident launches" % (n, n, k, n_res))
        assert info["status"] == 0 and info["iterations"] == 7 and n_res == -(-7 // k)
        np.testing.assert_array_equal(chi_r, chi_t)

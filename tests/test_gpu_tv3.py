"""GPU parity of the weighted TV model in three dimensions (Eq. (1) with the
3-D dipole kernel and the 3-D gradient) through the C ABI against the FP64
oracle's solve_tv(kind="dipole3d").

Inputs are the TV workload's seeded device stacks (magnitude-like weights W,
elliptical mask M); the field map is the oracle's 3-D forward operator of
the phantom with noise, rounded to FP32, and the same FP32 delta, W and M go
to both sides.  Steps sit inside the 3-D bound
tau sigma (max|W|^2 max|D3|^2 + max|M|^2 (4/dx^2 + 4/dy^2 + 4/dz^2)) < 1.
Bar (tests/_parity.py): relative L2 <= 1e-4 and every voxel within 1e-4 of
max|chi_oracle| after a fixed iteration count; 1e-10 for the FP64 build.
Cases cover one pair (no neighbouring pairs), odd nz (the padded slice),
oblique B0 and anisotropic voxels, Bluestein lengths along x and along z,
and the benchmark's 256 x 256 x 64 volume.
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
    s = pd.Solver(arena_bytes=8 << 30, device=0)
    yield s
    s.close()


@pytest.fixture(scope="module")
def solver64(torch_mod):
    import paper_2006_09808_amd as pd
    s = pd.Solver(arena_bytes=4 << 30, device=0, precision="fp64")
    yield s
    s.close()


def make_tv3_case(seed, nz, ny, nx, b0=(0.0, 1.0, 0.0), voxel=(1.0, 1.0), dz=1.0, iters=30, lam=100.0):
    w = pd_inputs.tv_stack(seed, nz, ny, nx, max_iter=iters, lam=lam, b0=b0, voxel=voxel)
    D3 = oracle.dipole_kernel3(nx, ny, nz, b0, voxel, dz)
    L2 = oracle.kernel_norm(D3) ** 2 + oracle.grad3_norm_bound((voxel[0], voxel[1], dz))
    w.tau = w.sigma = 0.95 / np.sqrt(L2)
    field = oracle.forward(w.chi_true, b0=b0, voxel=voxel, kind="dipole3d", voxel_z=dz)
    delta = pd_inputs.make_delta(field, w.eta, w.rho).astype(np.float32)
    return w, delta, w.weight.astype(np.float32), w.mask.astype(np.float32)


def to_dev(torch, a, dtype):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0", dtype=dtype)


def tv3_job(torch, w, delta, W, M, dz, dtype):
    d, wt, mt = (to_dev(torch, a, dtype) for a in (delta, W, M))
    chi = torch.empty_like(d)
    params = dict(w.solver_params(), model="tv", weight=wt, mask=mt, kernel="dipole3d", voxel_z=dz)
    return (d, chi, params)


def gpu_tv3_solve(solver, torch, w, delta, W, M, dz, dtype=None):
    job = tv3_job(torch, w, delta, W, M, dz, dtype or torch.float32)
    (t,) = solver.submit([job])
    info = solver.poll(t, -1)
    return job[1].cpu().numpy().astype(np.float64), info


def oracle_tv3(w, delta, W, M, dz):
    return oracle.solve_tv(delta.astype(np.float64), W.astype(np.float64), M.astype(np.float64),
                           kind="dipole3d", voxel_z=dz, **w.solver_params())


TV3_CASES = [
    # (seed, nz, ny, nx, b0, voxel, dz, iters)
    (51, 2, 16, 16, (0.0, 1.0, 0.0), (1.0, 1.0), 1.0, 30),          # one pair
    (52, 3, 32, 32, (0.0, 0.0, 1.0), (1.0, 1.0), 1.5, 40),          # odd nz: padded slice
    (53, 8, 16, 16, (0.3, 0.5, 0.8), (1.0, 1.0), 2.0, 40),          # oblique B0
    (54, 7, 48, 32, (0.3, 0.5, 0.8), (0.8, 1.2), 0.7, 30),          # anisotropic, odd nz
    (55, 12, 64, 64, (0.0, 1.0, 0.0), (1.0, 1.0), 2.0, 25),
    (56, 6, 40, 43, (1.0, 1.0, 0.5), (1.0, 1.0), 1.0, 20),          # Bluestein rows
    (57, 43, 16, 16, (0.0, 1.0, 0.0), (1.0, 1.0), 1.0, 20),         # Bluestein along z, odd nz
    (58, 16, 128, 128, (0.0, 1.0, 0.0), (1.0, 1.0), 2.0, 15),
]


@pytest.mark.parametrize("case", TV3_CASES, ids=lambda c: "%d-%dx%dx%d" % (c[0], c[3], c[2], c[1]))
def test_tv3_matches_oracle_fixed_iterations(solver, torch_mod, case):
    seed, nz, ny, nx, b0, vox, dz, iters = case
    _say("tv3 case nx=%d ny=%d nz=%d iters=%d" % (nx, ny, nz, iters))
    w, delta, W, M = make_tv3_case(seed, nz, ny, nx, b0, vox, dz, iters)
    chi, info = gpu_tv3_solve(solver, torch_mod, w, delta, W, M, dz)
    assert info["status"] == 0 and info["iterations"] == iters
    assert np.isnan(info["rel_gap"])
    ref, _ = oracle_tv3(w, delta, W, M, dz)
    _parity.check(chi, ref, "tv3 chi")
    # slices are coupled: the 2-D model's iterate differs beyond the bar
    ref2, _ = oracle.solve_tv(delta.astype(np.float64), W.astype(np.float64), M.astype(np.float64),
                              **w.solver_params())
    assert _parity.rel_l2(chi, ref2) > 1e-3


@pytest.mark.parametrize("case", [TV3_CASES[1], TV3_CASES[3]], ids=lambda c: "%d-%dx%dx%d" % (c[0], c[3], c[2], c[1]))
def test_tv3_fp64_matches_oracle(solver64, torch_mod, case):
    seed, nz, ny, nx, b0, vox, dz, iters = case
    w, delta, W, M = make_tv3_case(seed, nz, ny, nx, b0, vox, dz, iters)
    chi, info = gpu_tv3_solve(solver64, torch_mod, w, delta.astype(np.float64), W.astype(np.float64),
                              M.astype(np.float64), dz, dtype=torch_mod.float64)
    assert info["status"] == 0
    ref, _ = oracle_tv3(w, delta, W, M, dz)
    _parity.check(chi, ref, "fp64 tv3 chi", rel_tol=1e-10, vox_tol=1e-10)


@pytest.mark.timeout(900)
def test_tv3_bench_shape_256x256x64(solver, torch_mod):
    """The benchmark's 3-D TV volume (64 slices of 256 x 256, B0 along y,
    slice thickness 2), in the launch configuration the benchmark uses (a
    default context), for a few iterations against the oracle over the whole
    volume: z transforms of length 64, 32 pairs with neighbours on both
    sides.  The oracle's dense 3-D DFT takes seconds per operator here."""
    nx = ny = 256
    nz, iters, dz = 64, 6, 2.0
    w, delta, W, M = make_tv3_case(6200, nz, ny, nx, (0.0, 1.0, 0.0), (1.0, 1.0), dz, iters)
    _say("tv3 at the benchmark shape %dx%dx%d, %d iterations" % (nx, ny, nz, iters))
    chi, info = gpu_tv3_solve(solver, torch_mod, w, delta, W, M, dz)
    assert info["status"] == 0 and info["iterations"] == iters
    _say("  GPU done; oracle solve")
    ref, _ = oracle_tv3(w, delta, W, M, dz)
    _parity.check(chi, ref, "tv3 chi, whole volume")
    for z in (0, 1, 31, 32, 62, 63):
        _parity.check(chi[z:z + 1], ref[z:z + 1], "tv3 chi, slice %d" % z)


def test_tv3_step_condition_includes_the_z_term(solver, torch_mod):
    import paper_2006_09808_amd as pd
    nz, ny, nx, dz = 4, 32, 32, 0.5
    w, delta, W, M = make_tv3_case(61, nz, ny, nx, dz=dz, iters=10)
    D3 = oracle.dipole_kernel3(nx, ny, nz, w.b0, w.voxel, dz)
    wmax, mmax = float(np.max(np.abs(W))), float(np.max(np.abs(M)))
    L2_plane = wmax ** 2 * oracle.kernel_norm(D3) ** 2 + mmax ** 2 * oracle.grad_norm_bound(w.voxel)
    L2_3d = L2_plane + mmax ** 2 * 4.0 / dz ** 2
    # steps that pass the in-plane bound but not the 3-D one
    w.tau = w.sigma = 1.0 / np.sqrt(0.5 * (L2_plane + L2_3d))
    (t,) = solver.submit([tv3_job(torch_mod, w, delta, W, M, dz, torch_mod.float32)])
    info = solver.poll(t, -1)
    assert info["status"] == pd.PD_ERR_STEP and info["iterations"] == 0
    w.tau = w.sigma = 0.99 / np.sqrt(L2_3d)
    (t,) = solver.submit([tv3_job(torch_mod, w, delta, W, M, dz, torch_mod.float32)])
    info = solver.poll(t, -1)
    assert info["status"] == pd.PD_OK and info["iterations"] == 10


def test_tv3_with_2d_tv_and_3d_l1_in_one_batch_equal_their_solo_runs(solver, torch_mod):
    torch = torch_mod
    jobs = []
    w, delta, W, M = make_tv3_case(71, 5, 64, 64, dz=1.5, iters=23)
    jobs.append(tv3_job(torch, w, delta, W, M, 1.5, torch.float32))
    w, delta, W, M = make_tv3_case(72, 8, 32, 32, dz=1.0, iters=31)
    jobs.append(tv3_job(torch, w, delta, W, M, 1.0, torch.float32))
    w2 = pd_inputs.tv_stack(73, 3, 64, 64, max_iter=17)
    D = oracle.dipole_kernel(64, 64)
    w2.tau = w2.sigma = 0.95 / np.sqrt(oracle.kernel_norm(D) ** 2 + oracle.grad_norm_bound((1.0, 1.0)))
    d2 = pd_inputs.make_delta(oracle.forward(w2.chi_true), w2.eta, w2.rho).astype(np.float32)
    dd, wt, mt = (to_dev(torch, a, torch.float32) for a in (d2, w2.weight, w2.mask))
    jobs.append((dd, torch.empty_like(dd), dict(w2.solver_params(), model="tv", weight=wt, mask=mt)))
    l1 = pd_inputs.random_stack(74, 8, 32, 32, max_iter=40)
    f3 = oracle.forward(l1.chi_true, kind="dipole3d", voxel_z=1.0)
    dl = to_dev(torch, pd_inputs.make_delta(f3, l1.eta, l1.rho).astype(np.float32), torch.float32)
    jobs.append((dl, torch.empty_like(dl), dict(l1.solver_params(), kernel="dipole3d", voxel_z=1.0)))
    infos = [solver.poll(t, -1) for t in solver.submit(jobs)]
    assert all(i["status"] == 0 for i in infos), infos
    mixed = [j[1].cpu().numpy() for j in jobs]
    for (d, _, params), ref in zip(jobs, mixed):
        solo = torch.empty_like(d)
        (t,) = solver.submit([(d, solo, params)])
        assert solver.poll(t, -1)["status"] == 0
        np.testing.assert_array_equal(solo.cpu().numpy(), ref)


def test_tv3_repeated_solves_are_bitwise_equal(solver, torch_mod):
    # the second and later runs of the same plan replay a captured HIP graph
    w, delta, W, M = make_tv3_case(81, 6, 64, 64, dz=1.0, iters=25)
    outs = []
    for _ in range(3):
        chi, info = gpu_tv3_solve(solver, torch_mod, w, delta, W, M, 1.0)
        assert info["status"] == 0
        outs.append(chi)
    np.testing.assert_array_equal(outs[0], outs[1])
    np.testing.assert_array_equal(outs[0], outs[2])

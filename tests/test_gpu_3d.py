"""GPU parity of the 3-D dipole kernel (scope-table row f3) through the C ABI
against the FP64 oracle: the whole-volume operator A = F3^-1 diag(D3) F3 and
the PD solve with it.  Inputs are seeded device stacks; the field map is the
oracle's 3-D forward operator, rounded to FP32.
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


# (nx, ny, nz, b0, voxel, voxel_z)
SHAPES = [
    (16, 16, 8, (0.0, 1.0, 0.0), (1.0, 1.0), 1.0),
    (64, 64, 16, (0.0, 0.0, 1.0), (1.0, 1.0), 2.0),      # B0 along z, thick slices
    (48, 32, 12, (0.3, 0.5, 0.8), (0.8, 1.2), 1.5),     # oblique B0, anisotropic
    (43, 20, 7, (1.0, 1.0, 1.0), (1.0, 1.0), 1.0),      # Bluestein along x and z, odd nz
    (256, 256, 8, (0.0, 1.0, 0.0), (1.0, 1.0), 2.0),
    (16, 12, 140, (0.2, 0.4, 0.9), (1.0, 1.0), 0.5),   # Bluestein z on 288 transforms, partial strips
]


def ids(c):
    return "%dx%dx%d" % c[:3]


@pytest.mark.parametrize("shape", SHAPES, ids=ids)
def test_forward_operator_3d(solver, torch_mod, shape):
    nx, ny, nz, b0, vox, dz = shape
    _say("3-D operator %s" % ids(shape))
    rng = np.random.default_rng(nx + 7 * nz)
    x = rng.normal(size=(nz, ny, nx)).astype(np.float32)
    ref = oracle.forward(x.astype(np.float64), b0=b0, voxel=vox, kind="dipole3d", voxel_z=dz)
    out = solver.apply_kernel(torch_mod.from_numpy(x).to("cuda:0"), b0=b0, voxel=vox, kernel="dipole3d",
                              voxel_z=dz).cpu().numpy()
    _parity.check(out, ref, "A3 x", rel_tol=1e-5, vox_tol=1e-5)
    # it is not the slice-wise operator
    assert rel_l2(oracle.forward(x.astype(np.float64), b0=b0, voxel=vox), ref) > 1e-2


@pytest.mark.parametrize("shape", [SHAPES[2], SHAPES[3]], ids=ids)
def test_forward_operator_3d_fp64(solver64, torch_mod, shape):
    nx, ny, nz, b0, vox, dz = shape
    rng = np.random.default_rng(3 + nx)
    x = rng.normal(size=(nz, ny, nx))
    ref = oracle.forward(x, b0=b0, voxel=vox, kind="dipole3d", voxel_z=dz)
    out = solver64.apply_kernel(torch_mod.from_numpy(x).to("cuda:0"), b0=b0, voxel=vox, kernel="dipole3d",
                                voxel_z=dz).cpu().numpy()
    _parity.check(out, ref, "fp64 A3 x %s" % ids(shape), rel_tol=1e-12, vox_tol=1e-12)


def make_case3(seed, nz, ny, nx, b0, vox, dz, **params):
    w = pd_inputs.random_stack(seed, nz, ny, nx, **params)
    field = oracle.forward(w.chi_true, b0=b0, voxel=vox, kind="dipole3d", voxel_z=dz)
    delta = pd_inputs.make_delta(field, w.eta, w.rho).astype(np.float32)
    sp = dict(w.solver_params(), b0=b0, voxel=vox)
    return sp, delta


@pytest.mark.parametrize("shape,iters", [(SHAPES[0], 40), (SHAPES[2], 30), (SHAPES[3], 30)],
                         ids=lambda v: ids(v) if isinstance(v, tuple) else str(v))
def test_l1_solve_3d_matches_oracle(solver, torch_mod, shape, iters):
    nx, ny, nz, b0, vox, dz = shape
    sp, delta = make_case3(300 + nx, nz, ny, nx, b0, vox, dz, max_iter=iters)
    _say("3-D solve %s, %d iterations" % (ids(shape), iters))
    d = torch_mod.from_numpy(np.ascontiguousarray(delta)).to("cuda:0")
    chi, info = solver.solve(d, kernel="dipole3d", voxel_z=dz, **sp)
    chi = chi.cpu().numpy().astype(np.float64)
    ref, rinfo = oracle.solve(delta.astype(np.float64), kind="dipole3d", voxel_z=dz, **sp)
    _say("  gap %.6e vs %.6e" % (info["rel_gap"], rinfo["rel_gap"]))
    assert info["iterations"] == iters
    _parity.check(chi, ref, "chi")
    assert info["primal"] == pytest.approx(rinfo["primal"], rel=1e-4)
    assert info["dual"] == pytest.approx(rinfo["dual"], rel=1e-3, abs=1e-6 * abs(rinfo["primal"]))
    assert info["rel_gap"] == pytest.approx(rinfo["rel_gap"], rel=1e-3)


def test_3d_and_2d_volumes_in_one_batch_equal_their_solo_runs(solver, torch_mod):
    torch = torch_mod
    jobs, outs = [], []
    sp3, d3 = make_case3(311, 12, 32, 48, (0.3, 0.5, 0.8), (0.8, 1.2), 1.5, max_iter=25)
    t3 = torch.from_numpy(np.ascontiguousarray(d3)).to("cuda:0")
    c3 = torch.empty_like(t3)
    jobs.append((t3, c3, dict(sp3, kernel="dipole3d", voxel_z=1.5)))
    outs.append(c3)
    w = pd_inputs.random_stack(312, 6, 32, 48, max_iter=35)
    d2 = pd_inputs.make_delta(oracle.forward(w.chi_true), w.eta, w.rho).astype(np.float32)
    t2 = torch.from_numpy(d2).to("cuda:0")
    c2 = torch.empty_like(t2)
    jobs.append((t2, c2, w.solver_params()))
    outs.append(c2)
    infos = [solver.poll(t, -1) for t in solver.submit(jobs)]
    assert all(i["status"] == 0 for i in infos)
    mixed = [o.cpu().numpy() for o in outs]
    for (d, _, params), ref in zip(jobs, mixed):
        solo = torch.empty_like(d)
        (t,) = solver.submit([(d, solo, params)])
        assert solver.poll(t, -1)["status"] == 0
        np.testing.assert_array_equal(solo.cpu().numpy(), ref)


def test_l1_solve_3d_fp64_matches_oracle(solver64, torch_mod):
    nx, ny, nz, b0, vox, dz = SHAPES[3]         # Bluestein along x and z
    sp, delta = make_case3(321, nz, ny, nx, b0, vox, dz, max_iter=25)
    d = torch_mod.from_numpy(delta.astype(np.float64)).to("cuda:0")
    chi, info = solver64.solve(d, kernel="dipole3d", voxel_z=dz, **sp)
    ref, rinfo = oracle.solve(delta.astype(np.float64), kind="dipole3d", voxel_z=dz, **sp)
    _parity.check(chi.cpu().numpy(), ref, "fp64 3-D chi", rel_tol=1e-10, vox_tol=1e-10)
    assert info["rel_gap"] == pytest.approx(rinfo["rel_gap"], rel=1e-9)


def test_gap_tolerance_stop_3d(solver, torch_mod):
    # a weak field relative to lambda: the gap reaches the tolerance within the
    # cap and both sides stop at (nearly) the same check
    rng = np.random.default_rng(330)
    nx, ny, nz, dz = 32, 32, 8, 1.0
    x = np.zeros((nz, ny, nx))
    x[2:5, 10:14, 12:15] = 1.0
    delta = (oracle.forward(x, kind="dipole3d", voxel_z=dz) + 0.01 * rng.normal(size=x.shape)).astype(np.float32)
    sp = dict(lam=0.05, tau=1.4, sigma=1.4, theta=1.0, max_iter=600, gap_tol=1e-3, check_every=10)
    d = torch_mod.from_numpy(delta).to("cuda:0")
    chi, info = solver.solve(d, kernel="dipole3d", voxel_z=dz, **sp)
    ref, rinfo = oracle.solve(delta.astype(np.float64), kind="dipole3d", voxel_z=dz, **sp)
    _say("3-D gap stop: gpu %d it relgap %.3e; oracle %d it relgap %.3e" % (
        info["iterations"], info["rel_gap"], rinfo["iterations"], rinfo["rel_gap"]))
    assert rinfo["iterations"] < 600
    assert abs(info["iterations"] - rinfo["iterations"]) <= 10
    assert info["rel_gap"] <= 1e-3


@pytest.mark.timeout(900)
def test_l1_solve_3d_bench_shape_256x256x64(solver, torch_mod):
    """The 3-D workload the benchmark times (64 slices of 256 x 256, B0 along
    y, slice thickness 2, the same seeded phantom), solved in the same launch
    configuration (a default context), for 20 iterations against the oracle
    over the whole volume: the z transforms run at full length 64 and every
    voxel is compared.  The oracle's dense 3-D DFT takes a few seconds per
    iteration here."""
    nx = ny = 256
    nz, iters, dz = 64, 20, 2.0
    w = pd_inputs.random_stack(6100, nz, ny, nx, lam=1e-3, max_iter=iters)
    sp = w.solver_params()
    _say("3-D solve at the benchmark shape %dx%dx%d, %d iterations: oracle field map" % (nx, ny, nz, iters))
    field = oracle.forward(w.chi_true, b0=sp["b0"], voxel=sp["voxel"], kind="dipole3d", voxel_z=dz)
    delta = pd_inputs.make_delta(field, w.eta, w.rho).astype(np.float32)
    d = torch_mod.from_numpy(delta).to("cuda:0")
    chi, info = solver.solve(d, kernel="dipole3d", voxel_z=dz, **sp)
    chi = chi.cpu().numpy().astype(np.float64)
    _say("  GPU done (%d iterations); oracle solve" % info["iterations"])
    ref, rinfo = oracle.solve(delta.astype(np.float64), kind="dipole3d", voxel_z=dz, **sp)
    assert info["status"] == 0 and info["iterations"] == rinfo["iterations"] == iters
    _parity.check(chi, ref, "3-D chi, whole volume")
    for z in (0, 31, 63):
        _parity.check(chi[z:z + 1], ref[z:z + 1], "3-D chi, slice %d" % z)
    _say("  P %.8e vs %.8e" % (info["primal"], rinfo["primal"]))
    assert info["primal"] == pytest.approx(rinfo["primal"], rel=1e-4)

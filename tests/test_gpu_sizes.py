"""GPU parity on slice sizes without a direct FFT plan (scope-table row f2):
lengths 2..384 run their DFTs as Bluestein (chirp-z) convolutions on the
smallest direct length >= 2n - 1, and tiles of rows/columns may be partial.
The shapes include the paper's own data sizes (256 x 258 and 128 x 132,
Sec. III); the oracle's dense DFT handles any length, so the comparison is
against the same FP64 oracle as every other shape.
"""
import numpy as np
import pytest

import _parity
import oracle
import pd_inputs
from test_gpu_parity import make_case, gpu_solve

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


# (nx, ny, nz, b0, voxel): Bluestein rows and/or columns, partial tiles
OPERATOR_SHAPES = [
    (256, 258, 2, (0.0, 1.0, 0.0), (1.0, 1.0)),      # paper's stent slices
    (132, 128, 3, (0.0, 1.0, 0.0), (1.0, 1.0)),      # paper's seed / needle slices (x = 132)
    (128, 132, 1, (0.3, 0.5, 0.8), (0.72, 0.72)),    # transposed, oblique B0
    (43, 64, 2, (1.0, 1.0, 0.0), (1.0, 2.0)),        # prime rows, partial column strips
    (64, 43, 3, (0.0, 1.0, 0.0), (1.0, 1.0)),        # prime columns, partial row groups
    (5, 3, 2, (0.0, 1.0, 0.0), (1.0, 1.0)),          # tiny
    (383, 100, 1, (0.0, 1.0, 0.0), (1.0, 1.0)),      # longest Bluestein rows (768 transforms)
    (768, 24, 2, (0.0, 1.0, 0.0), (1.0, 1.0)),       # direct 768 plan
    (40, 576, 2, (0.3, 0.5, 0.8), (1.0, 1.0)),       # direct 576 plan (24 x 24) along columns
    (288, 36, 1, (0.0, 1.0, 0.0), (1.0, 1.0)),       # longest Bluestein rows on 576 transforms
    (289, 36, 1, (0.0, 1.0, 0.0), (1.0, 1.0)),       # shortest Bluestein rows on 768 transforms
    (288, 48, 2, (0.0, 1.0, 0.0), (1.0, 1.0)),       # direct 288 plan (12 x 24)
    (48, 144, 1, (1.0, 0.0, 1.0), (1.0, 1.0)),       # longest Bluestein columns on 288 transforms
    (48, 145, 1, (1.0, 0.0, 1.0), (1.0, 1.0)),       # shortest Bluestein columns on 384 transforms
]


def ids(c):
    return "%dx%dx%d" % c[:3]


@pytest.mark.parametrize("shape", OPERATOR_SHAPES, ids=ids)
def test_forward_operator_any_size(solver, torch_mod, shape):
    nx, ny, nz, b0, vox = shape
    _say("operator nx=%d ny=%d nz=%d" % (nx, ny, nz))
    rng = np.random.default_rng(nx * 1000 + ny)
    x = rng.normal(size=(nz, ny, nx)).astype(np.float32)
    ref = oracle.forward(x.astype(np.float64), b0=b0, voxel=vox)
    out = solver.apply_kernel(torch_mod.from_numpy(x).to("cuda:0"), b0=b0, voxel=vox).cpu().numpy()
    _parity.check(out, ref, "A x", rel_tol=1e-5, vox_tol=1e-5)


@pytest.mark.parametrize("shape", [OPERATOR_SHAPES[0], OPERATOR_SHAPES[3], OPERATOR_SHAPES[6], OPERATOR_SHAPES[8],
                                   OPERATOR_SHAPES[9], OPERATOR_SHAPES[12]], ids=ids)
def test_forward_operator_any_size_fp64(solver64, torch_mod, shape):
    # FP64 Bluestein transforms agree with the dense FP64 DFT to rounding
    nx, ny, nz, b0, vox = shape
    rng = np.random.default_rng(7 + nx)
    x = rng.normal(size=(nz, ny, nx))
    ref = oracle.forward(x, b0=b0, voxel=vox)
    out = solver64.apply_kernel(torch_mod.from_numpy(x).to("cuda:0"), b0=b0, voxel=vox).cpu().numpy()
    _parity.check(out, ref, "fp64 A x %s" % ids(shape), rel_tol=1e-12, vox_tol=1e-12)


SOLVE_SHAPES = [
    (201, 256, 258, 2, 60),
    (202, 132, 128, 3, 80),
    (203, 43, 64, 2, 50),
    (204, 64, 43, 3, 50),
    (205, 7, 9, 2, 40),
]


@pytest.mark.parametrize("case", SOLVE_SHAPES, ids=lambda c: "%dx%dx%d" % c[1:4])
def test_l1_solve_any_size_matches_oracle(solver, torch_mod, case):
    seed, nx, ny, nz, iters = case
    _say("l1 solve nx=%d ny=%d nz=%d iters=%d" % (nx, ny, nz, iters))
    w, delta = make_case(seed, nz, ny, nx, max_iter=iters)
    sp = w.solver_params()
    chi, info = gpu_solve(solver, torch_mod, delta, **sp)
    assert info["status"] == 0 and info["iterations"] == iters
    ref, rinfo = oracle.solve(delta.astype(np.float64), **sp)
    _say("  gap %.6e vs %.6e" % (info["rel_gap"], rinfo["rel_gap"]))
    _parity.check(chi, ref, "chi")
    assert info["rel_gap"] == pytest.approx(rinfo["rel_gap"], rel=1e-3)


def test_tv_solve_any_size_matches_oracle(solver, torch_mod):
    from test_gpu_tv import make_tv_case, gpu_tv_solve
    w, delta, W, M = make_tv_case(206, 3, 128, 132, iters=40)
    sp = w.solver_params()
    chi, info = gpu_tv_solve(solver, torch_mod, delta, W, M, **sp)
    assert info["status"] == 0
    ref, _ = oracle.solve_tv(delta.astype(np.float64), W.astype(np.float64), M.astype(np.float64), **sp)
    _parity.check(chi, ref, "tv 132x128x3 chi")


def test_gap_stop_on_bluestein_shape(solver, torch_mod):
    # identity kernel on a 43 x 100 slice (both axes Bluestein): the gap
    # reaches the tolerance and both sides stop at (nearly) the same check
    rng = np.random.default_rng(207)
    delta = rng.normal(size=(2, 43, 100)).astype(np.float32)
    sp = dict(lam=0.2, tau=0.9, sigma=0.9, theta=1.0, max_iter=400, gap_tol=1e-5, check_every=5,
              kernel="identity")
    chi, info = gpu_solve(solver, torch_mod, delta, **sp)
    osp = dict(sp)
    osp["kind"] = osp.pop("kernel")
    ref, rinfo = oracle.solve(delta.astype(np.float64), **osp)
    _say("gap stop: gpu %d it relgap %.3e, oracle %d it relgap %.3e" % (info["iterations"], info["rel_gap"],
                                                                       rinfo["iterations"], rinfo["rel_gap"]))
    assert info["status"] == 0
    assert info["iterations"] < 400 and info["rel_gap"] <= 1e-5
    # the stop can differ by one check period only where the gap lands within
    # FP32 rounding of the tolerance
    assert abs(info["iterations"] - rinfo["iterations"]) <= 5
    osp["max_iter"], osp["gap_tol"] = info["iterations"], 0.0
    ref_same, _ = oracle.solve(delta.astype(np.float64), **osp)
    _parity.check(chi, ref_same, "chi")


def test_mixed_sizes_in_one_batch_equal_their_solo_runs(solver, torch_mod):
    torch = torch_mod
    jobs, outs = [], []
    for seed, nx, ny, nz, iters in [(211, 256, 258, 2, 30), (212, 64, 64, 3, 45), (213, 43, 64, 2, 30)]:
        w, delta = make_case(seed, nz, ny, nx, max_iter=iters)
        d = torch.from_numpy(np.ascontiguousarray(delta)).to("cuda:0")
        chi = torch.empty_like(d)
        jobs.append((d, chi, w.solver_params()))
        outs.append(chi)
    infos = [solver.poll(t, -1) for t in solver.submit(jobs)]
    assert all(i["status"] == 0 for i in infos)
    mixed = [o.cpu().numpy() for o in outs]
    for (d, _, params), ref in zip(jobs, mixed):
        solo = torch.empty_like(d)
        (t,) = solver.submit([(d, solo, params)])
        assert solver.poll(t, -1)["status"] == 0
        np.testing.assert_array_equal(solo.cpu().numpy(), ref)


def test_l1_solve_bluestein_fp64(solver64, torch_mod):
    w, delta = make_case(221, 3, 43, 100, max_iter=30)
    sp = w.solver_params()
    d = torch_mod.from_numpy(delta.astype(np.float64)).to("cuda:0")
    chi, info = solver64.solve(d, **sp)
    ref, rinfo = oracle.solve(delta.astype(np.float64), **sp)
    _parity.check(chi.cpu().numpy(), ref, "fp64 bluestein chi", rel_tol=1e-10, vox_tol=1e-10)
    assert info["rel_gap"] == pytest.approx(rinfo["rel_gap"], rel=1e-9)


def test_tv_solve_bluestein_odd_stack(solver, torch_mod):
    from test_gpu_tv import make_tv_case, gpu_tv_solve
    # 43 x 27 slices (both axes Bluestein, partial tiles), 5 slices (padded pair)
    w, delta, W, M = make_tv_case(222, 5, 27, 43, b0=(0.3, 0.5, 0.8), voxel=(0.8, 1.2), iters=35)
    sp = w.solver_params()
    chi, info = gpu_tv_solve(solver, torch_mod, delta, W, M, **sp)
    assert info["status"] == 0
    ref, _ = oracle.solve_tv(delta.astype(np.float64), W.astype(np.float64), M.astype(np.float64), **sp)
    _parity.check(chi, ref, "tv 43x27x5 chi")


def test_largest_slices_768_direct_and_383_bluestein(solver, torch_mod):
    """Maximum sizes: 768 x 768 slices (the longest direct plan on both axes)
    and 383 x 383 slices (the longest length without a direct plan, run as
    Bluestein convolutions on 768-point transforms along both axes)."""
    for nx, ny, iters in ((768, 768, 4), (383, 383, 4)):
        _say("largest: %dx%dx1, %d iterations" % (nx, ny, iters))
        w, delta = make_case(230 + nx, 1, ny, nx, max_iter=iters)
        sp = w.solver_params()
        chi, info = gpu_solve(solver, torch_mod, delta, **sp)
        assert info["status"] == 0 and info["iterations"] == iters
        ref, _ = oracle.solve(delta.astype(np.float64), **sp)
        _parity.check(chi, ref, "%dx%d chi" % (nx, ny))

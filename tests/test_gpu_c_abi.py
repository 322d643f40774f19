"""The solver through its C ABI alone: the example program
paper_2006_09808_amd/examples/pd_solve_file (C++ against include/pd.h,
device memory from hipMalloc, no Python binding and no torch in its process)
solves a seeded field map; its result is checked against the FP64 oracle and
bitwise against the Python binding's solve of the same input."""
import os
import subprocess

import numpy as np
import pytest

import _parity
import oracle
import pd_inputs

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
EXE = os.path.join(ROOT, "paper_2006_09808_amd", "examples", "pd_solve_file")


def _say(*a):
    print(*a, flush=True)


def test_c_program_matches_oracle_and_binding(tmp_path):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    if not os.path.exists(EXE):
        pytest.fail("example program not built (run the package build first)")
    import paper_2006_09808_amd as pd
    nz, ny, nx, iters, lam = 3, 96, 64, 50, 1e-3
    w = pd_inputs.random_stack(501, nz, ny, nx, lam=lam, max_iter=iters)
    delta = pd_inputs.make_delta(oracle.forward(w.chi_true), w.eta, w.rho).astype(np.float32)
    fin, fout = tmp_path / "delta.f32", tmp_path / "chi.f32"
    delta.tofile(fin)
    _say("C program: %dx%dx%d, %d iterations" % (nx, ny, nz, iters))
    p = subprocess.run([EXE, str(nx), str(ny), str(nz), repr(lam), str(iters), str(fin), str(fout)],
                       stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True, timeout=120)
    _say("  " + p.stdout.strip())
    assert p.returncode == 0
    assert "status 0 iterations %d" % iters in p.stdout
    chi_c = np.fromfile(fout, dtype=np.float32).reshape(nz, ny, nx)
    sp = dict(lam=lam, tau=1.4, sigma=1.4, theta=1.0, max_iter=iters)
    ref, _ = oracle.solve(delta.astype(np.float64), **sp)
    _parity.check(chi_c, ref, "C program chi")
    with pd.Solver(arena_bytes=256 << 20, device=0) as s:
        chi_py, _ = s.solve(torch.from_numpy(delta).to("cuda:0"), **sp)
    np.testing.assert_array_equal(chi_py.cpu().numpy(), chi_c)


def test_solve_batch_rejects_missing_device_arrays():
    """pd_validate sizes a request without its arrays; pd_solve_batch needs
    them (and W, M for the TV model) and rejects the batch otherwise."""
    import ctypes
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2006_09808_amd as pd
    with pd.Solver(arena_bytes=64 << 20, device=0) as s:
        d = torch.zeros((2, 32, 32), device="cuda:0")
        cases = [dict(delta_ptr=0, chi_ptr=d.data_ptr()), dict(delta_ptr=d.data_ptr(), chi_ptr=0),
                 dict(delta_ptr=d.data_ptr(), chi_ptr=d.data_ptr(), model="tv", lam=100.0, tau=0.3, sigma=0.3,
                      weight_ptr=0, mask_ptr=d.data_ptr())]
        for kw in cases:
            r = pd.make_request(32, 32, 2, **kw)
            tickets = (ctypes.c_uint64 * 1)()
            st = s.lib.pd_solve_batch(s._ctx, ctypes.byref(r), 1, tickets)
            assert st == pd.PD_ERR_ARG
        # the context is still usable
        chi, info = s.solve(d, max_iter=5)
        assert info["status"] == pd.PD_OK

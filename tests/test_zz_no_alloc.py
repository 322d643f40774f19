"""pd_apply_kernel_noalloc, the operator entry point that allocates nothing
(its scratch is the library's fixed device array, not the arena), against
pd_apply_kernel on the same inputs: bitwise equal, on consecutive calls whose
second is smaller than the first (the scratch keeps the last call's contents),
for the 2-D and 3-D kernels, plus the oracle's A x on sampled slices and the
size limit."""
import numpy as np
import pytest

import _parity
import oracle

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def torch_mod():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


# (nz, ny, nx, b0, voxel, kernel): each case's second call is smaller
CASES = [
    [(64, 256, 256, (0, 1, 0), (1, 1), "dipole"), (7, 96, 64, (0.3, 0.5, 0.8), (0.72, 1.0), "dipole")],
    [(3, 384, 384, (0, 1, 0), (1, 1), "dipole"), (2, 130, 132, (0, 1, 0), (1, 1), "dipole")],
    [(32, 128, 128, (0, 0.5, 0.866), (1, 1), "dipole3d"), (8, 64, 48, (0.2, 0.6, 0.77), (1, 1.5), "dipole3d")],
]


@pytest.mark.parametrize("calls", CASES)
def test_noalloc_operator_equals_arena_operator(torch_mod, calls):
    import paper_2006_09808_amd as pd
    torch = torch_mod
    with pd.Solver(arena_bytes=512 << 20, device=0) as s, pd.Solver(arena_bytes=64 << 20, device=0) as s2:
        for k, (nz, ny, nx, b0, vox, kernel) in enumerate(calls):
            _say("call %d: %s %dx%dx%d b0=%s voxel=%s" % (k, kernel, nz, ny, nx, b0, vox))
            rng = np.random.default_rng(9000 + nz * 7 + ny + nx)
            x = rng.normal(size=(nz, ny, nx)).astype(np.float32)
            xt = torch.from_numpy(x).to("cuda:0")
            ref = s.apply_kernel(xt, b0=b0, voxel=vox, kernel=kernel).cpu().numpy()
            out = torch.full_like(xt, float("nan"))
            # a context with a small arena: the operator cannot come from it
            s2.apply_kernel(xt, out=out, b0=b0, voxel=vox, kernel=kernel, noalloc=True)
            got = out.cpu().numpy()
            np.testing.assert_array_equal(got, ref)
            if kernel == "dipole3d":
                want = oracle.forward(x.astype(np.float64), b0=b0, voxel=vox, kind="dipole3d")
                _parity.check(got, want, "noalloc A3 x", rel_tol=1e-5, vox_tol=1e-5)
            else:
                for z in sorted({0, nz // 2, nz - 1}):
                    want = oracle.forward(x[z:z + 1].astype(np.float64), b0=b0, voxel=vox)
                    _parity.check(got[z:z + 1], want, "noalloc A x slice %d" % z, rel_tol=1e-5, vox_tol=1e-5)
        used, _, _ = s2.arena_usage()
        _say("small context's arena in use: %d bytes" % used)


def test_noalloc_rejects_requests_beyond_the_scratch(torch_mod):
    import paper_2006_09808_amd as pd
    torch = torch_mod
    with pd.Solver(arena_bytes=64 << 20, device=0) as s:
        x = torch.zeros((64, 768, 768), dtype=torch.float32, device="cuda:0")   # 151 MB of field
        with pytest.raises(pd.PdError) as e:
            s.apply_kernel(x, out=torch.empty_like(x), noalloc=True)
        assert e.value.status == pd.PD_ERR_SCRATCH
        # the context is still usable
        y = torch.ones((2, 64, 64), dtype=torch.float32, device="cuda:0")
        a = s.apply_kernel(y, noalloc=True).cpu().numpy()
        b = s.apply_kernel(y).cpu().numpy()
        np.testing.assert_array_equal(a, b)

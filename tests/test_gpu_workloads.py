"""Full-size workloads against the oracle on sampled slices.

In fixed-count mode slices are independent, so a slice solved alone by the
oracle for the GPU's iteration count must match the GPU's slice."""
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


rel_l2 = _parity.rel_l2


def test_uneven_batch_with_gap_tolerance(torch_mod):
    """128^2 x 32, 256^2 x 48, 384^2 x 24 in one batch, each stopping at its
    own FP64 duality gap (1e-5) or the 1000-iteration cap."""
    import paper_2006_09808_amd as pd
    torch = torch_mod
    vols = pd_inputs.config3()
    with pd.Solver(arena_bytes=8 << 30, device=0) as s:
        jobs, deltas = [], []
        for w in vols:
            field = s.apply_kernel(torch.from_numpy(w.chi_true.astype(np.float32)).to("cuda:0"))
            d = torch.from_numpy(pd_inputs.make_delta(field.cpu().numpy().astype(np.float64), w.eta, w.rho)
                                 .astype(np.float32)).to("cuda:0")
            deltas.append(d)
            jobs.append((d, torch.empty_like(d), w.solver_params()))
        t0 = pd.now()
        tickets = s.submit(jobs)
        infos = [s.poll(t, -1) for t in tickets]
        _say("uneven batch wall %.1f ms" % ((pd.now() - t0) * 1e3))
    for w, (d, chi, sp), info in zip(vols, jobs, infos):
        _say("  %s: iterations %d relgap %.4e (cap %d)" % (w.name, info["iterations"], info["rel_gap"], w.max_iter))
        assert info["status"] == pd.PD_OK
        assert info["iterations"] % 10 == 0 and info["iterations"] <= w.max_iter
        assert info["rel_gap"] <= 1e-5 or info["iterations"] == w.max_iter
        z = w.shape[0] // 2
        fixed = dict(sp, gap_tol=0.0, max_iter=info["iterations"])
        ref, _ = oracle.solve(d[z:z + 1].cpu().numpy().astype(np.float64), **fixed)
        _parity.check(chi[z:z + 1].cpu().numpy(), ref, "slice %d" % z)


def test_precision_fp32_fp64_gpu_and_oracle(torch_mod):
    """256^2 x 128 tilted needle, 0.5% noise, lambda 5e-4, 800 iterations:
    FP32 GPU, FP64 GPU (same kernels instantiated in double) and the FP64
    oracle on sampled slices."""
    import paper_2006_09808_amd as pd
    torch = torch_mod
    w = pd_inputs.config4()
    field = oracle.forward(w.chi_true)
    delta = pd_inputs.make_delta(field, w.eta, w.rho)
    d32 = delta.astype(np.float32)
    sp = w.solver_params()
    with pd.Solver(arena_bytes=4 << 30, device=0) as s:
        c32, i32 = s.solve(torch.from_numpy(d32).to("cuda:0"), **sp)
    with pd.Solver(arena_bytes=8 << 30, device=0, precision="fp64") as s:
        c64, i64 = s.solve(torch.from_numpy(d32.astype(np.float64)).to("cuda:0"), **sp)
    c32 = c32.cpu().numpy().astype(np.float64)
    c64 = c64.cpu().numpy()
    assert i32["iterations"] == i64["iterations"] == 800
    _parity.check(c32, c64, "FP32 GPU vs FP64 GPU, 128 slices")
    for z in (0, 64, 127):
        ref, _ = oracle.solve(d32[z:z + 1].astype(np.float64), **sp)
        _parity.check(c32[z:z + 1], ref, "slice %d FP32 GPU vs oracle" % z)
        _parity.check(c64[z:z + 1], ref, "slice %d FP64 GPU vs oracle" % z, rel_tol=1e-10, vox_tol=1e-10)

"""Benchmark: batched primal-dual dipole deconvolution on one MI355X.

Workload (one step = one whole solve): 64 slices of 256x256, FP32, 500
primal-dual iterations, lambda = 1e-3, tau = sigma = 1.4, theta = 1, B0 along
y; seeded synthetic needle/seed phantoms with 1% field noise.  The field map
is made on the GPU with the library's own forward operator and is resident in
HBM before timing starts.

Prints one JSON line: voxel-iterations/s of the batched solve, the plain
per-slice GPU loop (every slice solved on its own, one after another) and the
speedup, the roofline of the dominant kernel (HIP-event timed inside the
timed region), and the FP64 CPU oracle timed on a bounded sample.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

NX = NY = 256
NZ = 64
ITERS = 500
HBM_PEAK_GBS = 8000.0
# Algorithmic bytes per slice-pair point and iteration (FP32).  The whole
# iteration: read chi_n, chi_(n-1) (here: chibar's inputs), Yhat, F(delta);
# write chi, Yhat: 24 B per voxel = 48 B per pair point.  The two-launch
# kernels also move their exchange buffer, so their own algorithmic bytes are:
BYTES_PER_POINT = {
    "column": 40,    # read exchange, dual, F(delta); write dual, exchange
    "row": 32,       # read exchange, chi; write chi, exchange
    "resident": 48,  # the whole iteration's 24 B per voxel, state kept on chip
}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-per-slice", action="store_true")
    ap.add_argument("--resident-variant", type=int, default=-1,
                    help="force this resident-kernel variant instead of the autotuned choice")
    ap.add_argument("--tv-only", action="store_true",
                    help="run only the weighted-TV workload line (for profiling its kernels)")
    ap.add_argument("--volume3d-only", nargs="?", const="both", choices=("both", "tv", "l1"),
                    help="run only the workload lines in three dimensions (the TV model, the L1 model with "
                         "the 3-D kernel, or both; for profiling their kernels)")
    ap.add_argument("--no-workloads", action="store_true",
                    help="skip the single-slice, uneven-batch and 256-slice lines")
    ap.add_argument("--cpu-sample-slices", type=int, default=16)
    ap.add_argument("--cpu-sample-iters", type=int, default=60)
    ap.add_argument("--serve-seconds", type=float, default=60.0,
                    help="length of the Poisson serving run (0: skip it)")
    ap.add_argument("--serve-rate", type=float, default=20.0)
    ap.add_argument("--serve-arena-gb", type=float, default=64.0)
    ap.add_argument("--serve-stress-seconds", type=float, default=15.0,
                    help="length of a second serving run under a 2 GB arena (0, or --serve-seconds 0: skip it)")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="BYTES",
                    help="only time a plain device copy of BYTES bytes (the reference kernel for "
                         "scaling hardware byte counters) and exit")
    return ap.parse_args()


def copy_probe(nbytes, reps=5):
    import torch
    a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda:0")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    print(json.dumps({"copy_probe_bytes": nbytes, "read_plus_write_GBs": 2 * nbytes / dt / 1e9,
                      "ms": dt * 1e3}), flush=True)


KERNEL_SOURCES = {
    # the profile summaries hash the kernel sources they were taken with, and
    # the build script that holds the compiler flags
    "column": ("pd_fft.hpp", "pd_kern_impl.hpp", "pd_internal.hpp", "../build.py"),
    "row": ("pd_fft.hpp", "pd_kern_impl.hpp", "pd_internal.hpp", "../build.py"),
    "resident": ("pd_fft.hpp", "pd_kern_impl.hpp", "pd_internal.hpp", "pd_resident.hpp", "../build.py"),
    "tv_column": ("pd_fft.hpp", "pd_kern_impl.hpp", "pd_internal.hpp", "../build.py"),
    "tv_row": ("pd_fft.hpp", "pd_kern_impl.hpp", "pd_internal.hpp", "pd_tv_row.hpp", "../build.py"),
    "tv_resident": ("pd_fft.hpp", "pd_kern_impl.hpp", "pd_internal.hpp", "pd_resident.hpp", "pd_resident_tv.hpp",
                    "pd_resident_tv.hip", "../build.py"),
}
# FP32 vector ALU ceilings of MI355X.  Published: 157.3 TFLOP/s, which needs
# packed FP32 (two FMAs per lane per instruction).  The library is compiled
# without packed FP32, so the ceiling of its kernels, from the unit counts and
# the clock, is
# 256 CUs x 4 SIMDs x 16 lanes x 2 flop (one FMA) x 2.4 GHz = 78.6 TFLOP/s:
# the roofline's peak.
FP32_PEAK_TFLOPS = 157.3
FP32_NONPACKED_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12


def flops_per_voxel_iteration(n):
    """Model: one forward and one inverse 2-D FFT per iteration of a pair of
    slices, 5 M log2 M flops per M-point complex FFT, plus the point-wise
    prox/update arithmetic (about 13 flops per voxel)."""
    import math
    return 10.0 * math.log2(n) + 13.0


def measured_traffic(kernel, variant=None):
    """Scaled FETCH_SIZE + WRITE_SIZE bytes per launch of `kernel` (for the
    resident kernel: of resident variant `variant`) from the committed
    rocprofv3 summaries, with the summary's file name, or (None, None) if no
    summary was taken with the current kernel sources.  Not measured in the
    run that reports it."""
    import glob
    import hashlib
    h = hashlib.sha256()
    try:
        for f in KERNEL_SOURCES[kernel]:
            with open(os.path.join(ROOT, "paper_2006_09808_amd", "csrc", f), "rb") as fh:
                h.update(fh.read())
    except OSError:
        return None, None
    for prof in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.md"))):
        with open(prof) as fh:
            for l in fh:
                l = l.strip()
                if not l.startswith("traffic:"):
                    continue
                rec = json.loads(l[len("traffic:"):])
                if rec.get("kernel") != kernel or rec.get("sources_sha256_16") != h.hexdigest()[:16]:
                    continue
                if variant is not None and rec.get("variant") != variant:
                    continue
                return rec["read_bytes"] + rec["write_bytes"], os.path.relpath(prof, ROOT)
    return None, None


def serving(rate, seconds, arena_gb):
    """Open-loop Poisson arrivals: in-plane size uniform over 128^2, 192^2,
    256^2, 384^2, 16-64 slices, gap tolerance 1e-5 (FP64 gap every 10
    iterations), cap 1000 iterations, admission under an arena of arena_gb.
    Every request is its own seeded phantom (pd_inputs.serving_request_device:
    the batched workload's recipe, drawn on the GPU), its field map made with
    the library's forward operator plus 1% noise, all before the run starts."""
    import torch
    import pd_inputs
    import paper_2006_09808_amd as pd
    from paper_2006_09808_amd import serve

    dev = torch.device("cuda", 0)
    sched = pd_inputs.serving_schedule(rate=rate, duration=seconds)
    with pd.Solver(arena_bytes=int(arena_gb * (1 << 30)), device=0) as s:
        for n in pd_inputs.SERVING_SIZES:
            s.tune(n, n, 40, iters=20)
        params = dict(lam=1e-3, tau=1.4, sigma=1.4, theta=1.0, max_iter=1000, gap_tol=1e-5, check_every=10)
        reqs = []
        for (t, n, nz, seed) in sched:
            chi_t, eta = pd_inputs.serving_request_device(seed, n, nz, dev)
            field = s.apply_kernel(chi_t)
            d = field + 0.01 * field.abs().max() * eta
            del chi_t, eta, field
            reqs.append(serve.Request(t, d, torch.empty_like(d), params))
        torch.cuda.synchronize()
        summary = serve.run_open_loop(s, reqs)
    summary.update({"arrival_rate_per_s": rate, "duration_s": seconds, "arena_GB": arena_gb,
                    "sizes": list(pd_inputs.SERVING_SIZES), "slices": [16, 64],
                    "gap_tol": 1e-5, "max_iter": 1000, "inputs": "one seeded phantom per request"})
    return summary


def _device_delta(s, w, dev):
    import torch
    import pd_inputs
    field = s.apply_kernel(torch.from_numpy(w.chi_true.astype(np.float32)).to(dev))
    d = pd_inputs.make_delta(field.cpu().numpy().astype(np.float64), w.eta, w.rho)
    return torch.from_numpy(d.astype(np.float32)).to(dev)


def other_workloads(reps=20):
    """The single-slice latency case, the uneven batch, a stack of 256
    slices (its state, 96 MiB, no longer fits the 256 MiB last-level cache
    together with the exchange buffers), the paper's 256x258 stack and the
    FP32/FP64 precision workload, each on a fresh context."""
    import torch
    import pd_inputs
    import paper_2006_09808_amd as pd
    dev = torch.device("cuda", 0)
    out = {}
    w = pd_inputs.config1()
    with pd.Solver(arena_bytes=256 << 20, device=0) as s:
        s.tune(64, 64, 1, iters=50)          # the latency case's own launch configuration
        d = _device_delta(s, w, dev)
        chi = torch.empty_like(d)
        sp = w.solver_params()
        lat = []
        for i in range(reps + 3):
            t0 = pd.now()
            (t,) = s.submit([(d, chi, sp)])
            r = s.poll(t, -1)
            if r["status"] != pd.PD_OK:
                raise RuntimeError("single-slice solve failed: %r" % (r,))
            if i >= 3:
                lat.append(pd.now() - t0)
        lat.sort()
        out["single_64x64x1_200it"] = {"median_ms": lat[len(lat) // 2] * 1e3, "min_ms": lat[0] * 1e3,
                                       "solves": len(lat)}
    vols = pd_inputs.config3()
    with pd.Solver(arena_bytes=8 << 30, device=0) as s:
        for w in vols:                       # autotune each shape at its own slice count
            s.tune(w.shape[2], w.shape[1], w.shape[0], iters=50)
        jobs = []
        for w in vols:
            d = _device_delta(s, w, dev)
            jobs.append((d, torch.empty_like(d), w.solver_params()))
        walls = []
        for _ in range(3):
            t0 = pd.now()
            infos = [s.poll(t, -1) for t in s.submit(jobs)]
            walls.append(pd.now() - t0)
        vit = sum(int(j[0].numel()) * i["iterations"] for j, i in zip(jobs, infos))
        out["uneven_128x32_256x48_384x24_1e-5"] = {
            "wall_ms": min(walls) * 1e3, "iterations": [i["iterations"] for i in infos],
            "rel_gap": [i["rel_gap"] for i in infos], "voxel_iterations_per_s": vit / min(walls),
            "cap_hit": [i["iterations"] >= j[2]["max_iter"] for j, i in zip(jobs, infos)]}
    w = pd_inputs.random_stack(2500, 256, NY, NX, lam=1e-3, max_iter=ITERS)
    with pd.Solver(arena_bytes=4 << 30, device=0) as s:
        d = _device_delta(s, w, dev)
        chi = torch.empty_like(d)
        sp = w.solver_params()
        best = None
        for _ in range(3):
            t0 = pd.now()
            (t,) = s.submit([(d, chi, sp)])
            r = s.poll(t, -1)
            if r["status"] != pd.PD_OK:
                raise RuntimeError("256-slice solve failed")
            dt = pd.now() - t0
            best = dt if best is None else min(best, dt)
        out["batched_256x256x256_500it"] = {"ms": best * 1e3,
                                            "voxel_iterations_per_s": 256 * NX * NY * ITERS / best}
    # the paper's stent data shape (256 x 258 in-plane, 25 slices): 258 has no
    # direct FFT plan, so its transforms run as Bluestein convolutions of length 768
    w = pd_inputs.random_stack(2600, 25, 258, 256, lam=1e-3, max_iter=ITERS)
    with pd.Solver(arena_bytes=2 << 30, device=0) as s:
        d = _device_delta(s, w, dev)
        chi = torch.empty_like(d)
        sp = w.solver_params()
        best = None
        for i in range(4):                  # the second solve captures the step graphs
            t0 = pd.now()
            r = s.poll(s.submit([(d, chi, sp)])[0], -1)
            if r["status"] != pd.PD_OK:
                raise RuntimeError("256x258 solve failed")
            dt = pd.now() - t0
            if i >= 2:
                best = dt if best is None else min(best, dt)
        out["paper_shape_256x258x25_500it"] = {"ms": best * 1e3,
                                               "voxel_iterations_per_s": 25 * 256 * 258 * ITERS / best}
    # precision workload: 128 slices of 256x256 with a tilted needle, 0.5%
    # noise, lambda 5e-4, 800 iterations, FP32 and FP64 (the same kernels in
    # double) on the GPU; agreement of the two in relative L2 and ppm
    w = pd_inputs.config4()
    res = {}
    with pd.Solver(arena_bytes=1 << 30, device=0) as s:
        delta4 = _device_delta(s, w, dev).cpu().numpy()      # one FP32 field map for both runs
    for prec, dt_np in (("fp32", np.float32), ("fp64", np.float64)):
        with pd.Solver(arena_bytes=8 << 30, device=0, precision=prec) as s:
            if prec == "fp32":
                s.tune(256, 256, 128, iters=20)
            d = torch.from_numpy(delta4.astype(dt_np)).to(dev)
            chi = torch.empty_like(d)
            sp = w.solver_params()
            best = None
            for _ in range(2):
                t0 = pd.now()
                r = s.poll(s.submit([(d, chi, sp)])[0], -1)
                if r["status"] != pd.PD_OK:
                    raise RuntimeError("precision workload solve failed")
                dt = pd.now() - t0
                best = dt if best is None else min(best, dt)
            res[prec] = (chi.cpu().numpy().astype(np.float64), best)
    c32, c64 = res["fp32"][0], res["fp64"][0]
    out["precision_256x256x128_800it"] = {
        "fp32_ms": res["fp32"][1] * 1e3, "fp64_ms": res["fp64"][1] * 1e3,
        "relL2_fp32_vs_fp64": float(np.linalg.norm(c32 - c64) / np.linalg.norm(c64)),
        "max_abs_ppm_fp32_vs_fp64": float(np.abs(c32 - c64).max())}
    return out


# weighted TV model: algorithmic HBM bytes per slice-pair point of each launch
# (FP32, complex pair layout, 8 B per field): column kernel reads and writes
# the exchange field (16); dual row kernel reads ex, p, W, delta, chibar, q_x,
# q_y, M and writes p, q_x, q_y, ex (96); primal row kernel reads ex, chi, q_x,
# q_y, M and writes chi, chibar, ex (64).  Per voxel-iteration:
# (2 x 16 + 96 + 64) / 2 = 96 B.
TV_BYTES_PER_VOXEL_IT = 96.0
TV_COL_BYTES_PER_POINT = 16.0
TV_ROW_BYTES_PER_POINT = 80.0       # mean of the dual (96) and primal (64) row kernels
# the TV model's resident launch (square slices): the exchange field stays in
# the L2 of the team's XCD and the mask M in LDS for the whole launch, so per
# iteration HBM sees the row phases' other state only: dual reads p, W,
# delta, chibar, q_x, q_y and writes p, q_x, q_y (72); primal reads chi, q_x,
# q_y and writes chi, chibar (40): 112 B per slice-pair point, 56 B per
# voxel-iteration
TV_RES_BYTES_PER_POINT_IT = 112.0


def tv_workload(nz=64, n=256, iters=500, reps=3):
    """The weighted TV model of Eq. (1) on nz slices of n x n: wall time per
    solve and the kernels' HIP-event time and algorithmic bandwidth."""
    import torch
    import pd_inputs
    import paper_2006_09808_amd as pd
    dev = torch.device("cuda", 0)
    w = pd_inputs.tv_stack(6000, nz, n, n, max_iter=iters)
    # wall time on a default context (steps replayed from captured HIP
    # graphs), kernel times on a second context with HIP events per launch
    with pd.Solver(arena_bytes=4 << 30, device=0) as s:
        d = _device_delta(s, w, dev)
        W = torch.from_numpy(w.weight.astype(np.float32)).to(dev)
        M = torch.from_numpy(w.mask.astype(np.float32)).to(dev)
        chi = torch.empty_like(d)
        sp = dict(w.solver_params(), model="tv", weight=W, mask=M)
        best = None
        for i in range(reps + 2):                     # two warm-ups: the second captures the graphs
            t0 = pd.now()
            r = s.poll(s.submit([(d, chi, sp)])[0], -1)
            if r["status"] != pd.PD_OK or r["iterations"] != iters:
                raise RuntimeError("TV solve failed: %r" % (r,))
            dt = pd.now() - t0
            if i >= 2:
                best = dt if best is None else min(best, dt)
    # the four-launch path on the same input, for comparison
    with pd.Solver(arena_bytes=4 << 30, device=0, resident=False) as s:
        best4 = None
        for i in range(reps + 2):
            t0 = pd.now()
            r = s.poll(s.submit([(d, chi, sp)])[0], -1)
            if r["status"] != pd.PD_OK or r["iterations"] != iters:
                raise RuntimeError("TV solve failed: %r" % (r,))
            dt = pd.now() - t0
            if i >= 2:
                best4 = dt if best4 is None else min(best4, dt)
    kt = {}
    for resident in (True, False):
        with pd.Solver(arena_bytes=4 << 30, device=0, time_kernels=True, resident=resident) as s:
            s.poll(s.submit([(d, chi, sp)])[0], -1)
            kinds = (("tv_resident", pd.KIND_TV_RESIDENT),) if resident else \
                (("tv_column", pd.KIND_TV_COLUMN), ("tv_row", pd.KIND_TV_ROW))
            kt.update({name: s.kernel_time(kind) for name, kind in kinds})
    vit = nz * n * n * iters
    out = {"workload": "weighted TV (Eq. (1)), %d slices of %dx%d, %d iterations" % (nz, n, n, iters),
           "ms": best * 1e3, "voxel_iterations_per_s": vit / best,
           "path": "resident launch (one per step)",
           "hbm_bytes_per_voxel_iteration": TV_RES_BYTES_PER_POINT_IT / 2,
           "achieved_GBs_wall": TV_RES_BYTES_PER_POINT_IT / 2 * vit / best / 1e9,
           "four_launch": {"ms": best4 * 1e3, "voxel_iterations_per_s": vit / best4,
                           "bytes_per_voxel_iteration": TV_BYTES_PER_VOXEL_IT,
                           "achieved_GBs_wall": TV_BYTES_PER_VOXEL_IT * vit / best4 / 1e9},
           "kernels": {}}
    for name, (nl, ms, pts) in kt.items():
        if not nl:
            continue
        if name == "tv_resident":
            # pts counts iterations x pair points
            traffic, src = measured_traffic(name)
            out["kernels"][name] = {"launches": nl, "avg_ms": ms / nl,
                                    "GBs": TV_RES_BYTES_PER_POINT_IT * pts / (ms * 1e-3) / 1e9,
                                    "bytes_per_launch": TV_RES_BYTES_PER_POINT_IT * pts / nl,
                                    "traffic": traffic, "traffic_source": src,
                                    "traffic_GBs": None if traffic is None else traffic / (ms / nl * 1e-3) / 1e9}
            continue
        bpp = TV_COL_BYTES_PER_POINT if name == "tv_column" else TV_ROW_BYTES_PER_POINT
        out["kernels"][name] = {"launches": nl, "avg_ms": ms / nl, "GBs": bpp * pts / (ms * 1e-3) / 1e9,
                                "bytes_per_launch": bpp * pts / nl, "traffic": measured_traffic(name)[0]}
    return out


# weighted TV model in three dimensions: algorithmic HBM bytes per slice-pair
# point (two voxels; FP32, 8 B per complex value).  The exchange holds one
# plane per slice, so each in-place plane transform (F_y, F_y^-1) reads and
# writes two planes (32); the z-view transform reads and writes them and
# reads the 3-D D table (2 x 4 B) (40); the dual row kernel reads two
# exchange planes, p, W, delta, chibar, M, q_x, q_y, q_z and writes p, q_x,
# q_y, q_z and two planes (128); the primal row kernel reads two planes, chi,
# q_x, q_y, q_z, M and writes chi, chibar and two planes (88).  Per
# voxel-iteration: (2 x (32 + 40 + 32) + 128 + 88) / 2 = 212 B.
TV3_BYTES_PER_VOXEL_IT = 212.0
TV3_BYTES_PER_POINT = {"plane_column": 32.0, "z_transform": 40.0, "tv_row": 108.0}

# L1 model with the 3-D kernel (unpacked planes, one slice per complex plane),
# per plane point (one voxel): in-place plane transforms 16; z-view dual prox
# reads ex, Yhat, F delta, D and writes Yhat, ex (44); row kernel reads ex and
# chi and writes both (32).  Per voxel-iteration 16 + 44 + 16 + 32 = 108 B.
L1_3D_BYTES_PER_VOXEL_IT = 108.0
L1_3D_BYTES_PER_POINT = {"plane_column": 16.0, "z_transform": 44.0, "plane_row": 32.0}


def tv3_workload(nz=64, n=256, iters=500, reps=3, dz=2.0):
    """The weighted TV model in three dimensions (3-D gradient, 3-D dipole
    kernel) on nz slices of n x n: wall time per solve and each kernel
    class's HIP-event time and algorithmic bandwidth."""
    import torch
    import pd_inputs
    import paper_2006_09808_amd as pd
    dev = torch.device("cuda", 0)
    w = pd_inputs.tv_stack(6200, nz, n, n, max_iter=iters)
    # steps inside the 3-D bound: max|W| = max|M| = 1, max|D3| = 2/3, 4 + 4 + 4/dz^2
    w.tau = w.sigma = 0.95 / np.sqrt((2.0 / 3.0) ** 2 + 8.0 + 4.0 / dz ** 2)
    with pd.Solver(arena_bytes=8 << 30, device=0) as s:
        field = s.apply_kernel(torch.from_numpy(w.chi_true.astype(np.float32)).to(dev), kernel="dipole3d",
                               voxel_z=dz)
        d = torch.from_numpy(pd_inputs.make_delta(field.cpu().numpy().astype(np.float64), w.eta, w.rho)
                             .astype(np.float32)).to(dev)
        W = torch.from_numpy(w.weight.astype(np.float32)).to(dev)
        M = torch.from_numpy(w.mask.astype(np.float32)).to(dev)
        chi = torch.empty_like(d)
        sp = dict(w.solver_params(), model="tv", weight=W, mask=M, kernel="dipole3d", voxel_z=dz)
        best = None
        for i in range(reps + 2):
            t0 = pd.now()
            r = s.poll(s.submit([(d, chi, sp)])[0], -1)
            if r["status"] != pd.PD_OK or r["iterations"] != iters:
                raise RuntimeError("3-D TV solve failed: %r" % (r,))
            dt = pd.now() - t0
            if i >= 2:
                best = dt if best is None else min(best, dt)
    with pd.Solver(arena_bytes=8 << 30, device=0, time_kernels=True) as s:
        s.poll(s.submit([(d, chi, sp)])[0], -1)
        kt = {name: s.kernel_time(kind) for name, kind in
              (("plane_column", pd.KIND_TV_COLUMN), ("z_transform", pd.KIND_Z), ("tv_row", pd.KIND_TV_ROW))}
    vit = nz * n * n * iters
    out = {"workload": "weighted TV in three dimensions (3-D G, 3-D D), %d slices of %dx%d, %d iterations"
                       % (nz, n, n, iters),
           "ms": best * 1e3, "voxel_iterations_per_s": vit / best,
           "bytes_per_voxel_iteration": TV3_BYTES_PER_VOXEL_IT,
           "achieved_GBs_wall": TV3_BYTES_PER_VOXEL_IT * vit / best / 1e9, "kernels": {}}
    for name, (nl, ms, pts) in kt.items():
        if nl:
            bpp = TV3_BYTES_PER_POINT[name]
            out["kernels"][name] = {"launches": nl, "avg_ms": ms / nl, "GBs": bpp * pts / (ms * 1e-3) / 1e9,
                                    "bytes_per_launch": bpp * pts / nl}
    return out


def volume3d_workload(nz=64, n=256, iters=500, reps=3):
    """The 3-D dipole kernel (whole-volume operator, slices coupled) on nz
    slices of n x n: wall time per solve (steps replayed from HIP graphs) and
    the HIP-event time of its kernel classes on a second context."""
    import torch
    import pd_inputs
    import paper_2006_09808_amd as pd
    dev = torch.device("cuda", 0)
    w = pd_inputs.random_stack(6100, nz, n, n, lam=1e-3, max_iter=iters)
    sp = dict(w.solver_params(), kernel="dipole3d", voxel_z=2.0)
    with pd.Solver(arena_bytes=4 << 30, device=0) as s:
        field = s.apply_kernel(torch.from_numpy(w.chi_true.astype(np.float32)).to(dev), kernel="dipole3d",
                               voxel_z=2.0)
        d = torch.from_numpy(pd_inputs.make_delta(field.cpu().numpy().astype(np.float64), w.eta, w.rho)
                             .astype(np.float32)).to(dev)
        chi = torch.empty_like(d)
        best = None
        for i in range(reps + 2):
            t0 = pd.now()
            r = s.poll(s.submit([(d, chi, sp)])[0], -1)
            if r["status"] != pd.PD_OK or r["iterations"] != iters:
                raise RuntimeError("3-D solve failed: %r" % (r,))
            dt = pd.now() - t0
            if i >= 2:
                best = dt if best is None else min(best, dt)
    with pd.Solver(arena_bytes=4 << 30, device=0, time_kernels=True) as s:
        s.poll(s.submit([(d, chi, sp)])[0], -1)
        kt = {name: s.kernel_time(kind) for name, kind in
              (("plane_column", pd.KIND_COLUMN), ("plane_row", pd.KIND_ROW), ("z_transform", pd.KIND_Z))}
    vit = nz * n * n * iters
    out = {"workload": "3-D dipole kernel, %d slices of %dx%d, %d iterations" % (nz, n, n, iters),
           "ms": best * 1e3, "voxel_iterations_per_s": vit / best,
           "bytes_per_voxel_iteration": L1_3D_BYTES_PER_VOXEL_IT,
           "achieved_GBs_wall": L1_3D_BYTES_PER_VOXEL_IT * vit / best / 1e9, "kernels": {}}
    for name, (nl, ms, pts) in kt.items():
        if nl:
            bpp = L1_3D_BYTES_PER_POINT[name]
            out["kernels"][name] = {"launches": nl, "avg_ms": ms / nl, "GBs": bpp * pts / (ms * 1e-3) / 1e9,
                                    "bytes_per_launch": bpp * pts / nl}
    return out


def cpu_baseline(w, nslices, iters):
    """FP64 oracle on a bounded sample of the same workload (first `nslices`
    slices, `iters` iterations), on this host's cores."""
    import oracle
    import pd_inputs
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info() if i.get("user_api") == "blas"]
                      or [1])
    except Exception:
        threads = os.cpu_count() or 1
    chi = w.chi_true[:nslices]
    field = oracle.forward(chi)
    delta = pd_inputs.make_delta(field, w.eta[:nslices], w.rho).astype(np.float32).astype(np.float64)
    t0 = time.perf_counter()
    ref, _ = oracle.solve(delta, lam=w.lam, tau=w.tau, sigma=w.sigma, theta=w.theta, max_iter=iters)
    dt = time.perf_counter() - t0
    vit = nslices * NX * NY * iters
    out = {"value": vit / dt, "unit": "voxel-iterations/s", "cores": int(threads), "kind": "oracle",
           "sample": "%d of %d slices (256x256), %d of %d iterations, FP64 dense-DFT oracle, %.1f s"
                     % (nslices, NZ, iters, ITERS, dt),
           "host_cpus": os.cpu_count(), "blas_threads": int(threads),
           "threads_note": "the dense DFTs are BLAS matrix products on blas_threads threads; the "
                           "point-wise steps run on one"}
    # the same sample solved on the GPU (FP32, the autotuned launch
    # configuration of the bench shape), against the oracle's iterate
    import torch
    import paper_2006_09808_amd as pd
    with pd.Solver(arena_bytes=1 << 30, device=0) as s:
        s.tune(NX, NY, nslices, iters=50)
        got, info = s.solve(torch.from_numpy(delta.astype(np.float32)).to("cuda:0"), lam=w.lam, tau=w.tau,
                            sigma=w.sigma, theta=w.theta, max_iter=iters)
    got = got.cpu().numpy().astype(np.float64)
    out["parity"] = {"relL2": float(np.linalg.norm(got - ref) / np.linalg.norm(ref)),
                     "max_abs_ppm": float(np.abs(got - ref).max()), "tolerance": 1e-4,
                     "gpu": "FP32, %d iterations" % info["iterations"]}
    # the single 64x64 slice workload in full (200 iterations): small enough
    # for the oracle, so its GPU result is checked whole
    w1 = pd_inputs.config1()
    d1 = pd_inputs.make_delta(oracle.forward(w1.chi_true), w1.eta, w1.rho).astype(np.float32)
    t1 = time.perf_counter()
    ref1, _ = oracle.solve(d1.astype(np.float64), **w1.solver_params())
    t1 = time.perf_counter() - t1
    with pd.Solver(arena_bytes=256 << 20, device=0) as s:
        got1, info1 = s.solve(torch.from_numpy(d1).to("cuda:0"), **w1.solver_params())
    got1 = got1.cpu().numpy().astype(np.float64)
    out["parity_single_64x64x1_200it"] = {
        "relL2": float(np.linalg.norm(got1 - ref1) / np.linalg.norm(ref1)),
        "max_abs_ppm": float(np.abs(got1 - ref1).max()), "tolerance": 1e-4, "iterations": info1["iterations"]}
    out["per_config"] = oracle_per_config(t1, w1)
    return out


def oracle_per_config(t1, w1):
    """The oracle's rate on bounded samples of the other workloads (same
    host, same threads): the single 64x64 slice whole, one slice pair of each
    volume size of the uneven batch, two slices of the tilted-needle volume;
    fixed iteration counts (the oracle's cost per iteration does not depend on
    the stop rule)."""
    import oracle
    import pd_inputs
    res = {"single_64x64x1_200it": {"value": 64 * 64 * w1.max_iter / t1, "seconds": t1,
                                    "sample": "the whole workload"}}
    tot_v, tot_t, parts = 0.0, 0.0, []
    for w in pd_inputs.config3():
        nz, ny, nx = w.shape
        iters = 20 if nx <= 128 else 10
        d = pd_inputs.make_delta(oracle.forward(w.chi_true[:2]), w.eta[:2], w.rho)
        t0 = time.perf_counter()
        oracle.solve(d, lam=w.lam, tau=w.tau, sigma=w.sigma, theta=w.theta, max_iter=iters)
        dt = time.perf_counter() - t0
        tot_v += 2 * nx * ny * iters
        tot_t += dt
        parts.append("%dx%d: 2 slices x %d iterations" % (nx, ny, iters))
    res["uneven_128x32_256x48_384x24"] = {"value": tot_v / tot_t, "seconds": tot_t, "sample": "; ".join(parts)}
    w4 = pd_inputs.config4()
    d4 = pd_inputs.make_delta(oracle.forward(w4.chi_true[:2]), w4.eta[:2], w4.rho)
    t0 = time.perf_counter()
    oracle.solve(d4, **dict(w4.solver_params(), max_iter=20))
    dt = time.perf_counter() - t0
    res["precision_256x256x128"] = {"value": 2 * 256 * 256 * 20 / dt, "seconds": dt,
                                    "sample": "2 of 128 slices, 20 of 800 iterations"}
    for v in res.values():
        v["unit"] = "voxel-iterations/s"
    return res


def main():
    a = parse()
    if a.copy_probe:
        copy_probe(a.copy_probe)
        return
    if a.tv_only:
        print(json.dumps({"tv_256x256x64_500it": tv_workload()}), flush=True)
        return
    if a.volume3d_only:
        out = {}
        if a.volume3d_only in ("both", "tv"):
            out["tv3_256x256x64_500it"] = tv3_workload()
        if a.volume3d_only in ("both", "l1"):
            out["dipole3d_256x256x64_500it"] = volume3d_workload()
        print(json.dumps(out), flush=True)
        return
    if a.gpus != 1:
        print("bench.py runs on one GPU only: this solver has no multi-GPU path to measure "
              "(requests would be sharded across GPUs with no exchange inside a solve)", file=sys.stderr)
        sys.exit(2)
    import torch
    import pd_inputs
    import paper_2006_09808_amd as pd

    dev = torch.device("cuda", 0)
    w = pd_inputs.config2()
    sp = w.solver_params()

    with pd.Solver(arena_bytes=2 << 30, device=0, time_kernels=True) as s:
        # autotune the kernel configuration of this shape on this device
        # (200-iteration launches rank the variants as the 100-500-iteration
        # steps of a solve do; 50-iteration ones are dominated by launch cost)
        tune_table = s.tune(NX, NY, NZ, iters=200)
        if a.resident_variant >= 0:
            s.tune_set(NX, NY, a.resident_variant, 0, 0)
        tune_choice = s.tune_get(NX, NY)
        chi_true = torch.from_numpy(w.chi_true.astype(np.float32)).to(dev)
        field = s.apply_kernel(chi_true).cpu().numpy().astype(np.float64)
        delta = torch.from_numpy(pd_inputs.make_delta(field, w.eta, w.rho).astype(np.float32)).to(dev)
        chi = torch.empty_like(delta)
        torch.cuda.synchronize()

        def step():
            (t,) = s.submit([(delta, chi, sp)])
            info = s.poll(t, -1)
            if info["status"] != pd.PD_OK or info["iterations"] != ITERS:
                raise RuntimeError("solve failed: %r" % (info,))
            return info

        for _ in range(a.warmup):
            step()
        torch.cuda.synchronize()
        s.kernel_time_reset()
        t0 = time.perf_counter()
        for _ in range(a.steps):
            info = step()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        kt = {name: s.kernel_time(kind) for name, kind in
              (("column", pd.KIND_COLUMN), ("row", pd.KIND_ROW), ("resident", pd.KIND_RESIDENT))}

    per_slice = None
    per_slice_rel = None
    if not a.no_per_slice:
        chi_batched = chi.clone()
        # plain per-slice GPU loop: each slice solved alone, one after another,
        # two kernel launches per iteration (the paper's slice loop on the GPU)
        with pd.Solver(arena_bytes=1 << 30, device=0, resident=False) as s1:
            def slice_pass():
                for z in range(NZ):
                    (t,) = s1.submit([(delta[z:z + 1], chi[z:z + 1], sp)])
                    r = s1.poll(t, -1)
                    if r["status"] != pd.PD_OK:
                        raise RuntimeError("per-slice solve failed")
            slice_pass()
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            slice_pass()
            torch.cuda.synchronize()
            per_slice = time.perf_counter() - t1
        # same iterates up to rounding (a slice alone rides with a zero
        # partner instead of its neighbour)
        per_slice_rel = float(torch.linalg.vector_norm((chi - chi_batched).double()) /
                              torch.linalg.vector_norm(chi_batched.double()))

    vit = NZ * NX * NY * ITERS
    value = vit * a.steps / dt
    kernels = {}
    for name, (n, ms, pts) in kt.items():
        if n == 0:
            continue
        gbs = BYTES_PER_POINT[name] * pts / (ms * 1e-3) / 1e9
        kernels[name] = {"launches": n, "avg_ms": ms / n, "GBs": gbs,
                         "bytes_per_launch": BYTES_PER_POINT[name] * pts / n, "total_ms": ms}
    dom = max(kernels, key=lambda k: kernels[k]["total_ms"])
    achieved = kernels[dom]["GBs"]
    if dom == "resident":
        # state stays on chip: the measured traffic is a few percent of the
        # streaming model's bytes, so the kernel is rated on arithmetic
        n, ms, pts = kt["resident"]
        tflops = flops_per_voxel_iteration(NX) * 2 * pts / (ms * 1e-3) / 1e12
        variant = tune_choice["variant"]
        vrow = [t for t in tune_table if t["path"] == "resident" and t["variant"] == variant]
        traffic, traffic_src = measured_traffic(dom, variant)
        roofline = {"bound": "alu", "kernel": dom, "achieved": tflops, "peak": FP32_PEAK_TFLOPS,
                    "unit": "TFLOP/s", "frac": tflops / FP32_PEAK_TFLOPS,
                    "peak_note": "published FP32 vector peak (packed FP32, two FMAs per lane)",
                    "peak_nonpacked": FP32_NONPACKED_TFLOPS, "frac_nonpacked": tflops / FP32_NONPACKED_TFLOPS,
                    "peak_nonpacked_derivation": "256 CUs x 4 SIMD x 16 lanes x FMA x 2.4 GHz: the issue "
                                                 "ceiling of the non-packed FP32 this build emits",
                    "variant": variant,
                    "variant_shape": ({"workgroups_per_pair": vrow[0]["team"], "threads": vrow[0]["threads"]}
                                      if vrow else None),
                    "traffic": traffic,
                    "traffic_source": (None if traffic is None else
                                       "%s: rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE of this kernel and variant "
                                       "with the current sources, scaled by a 1 GiB copy; not measured in "
                                       "this run" % traffic_src),
                    "flops_per_voxel_iteration": flops_per_voxel_iteration(NX),
                    "avg_ms": kernels[dom]["avg_ms"],
                    "streaming_model": {
                        "bytes_per_voxel_iteration": 24,
                        "bytes_per_launch": kernels[dom]["bytes_per_launch"],
                        "equivalent_GBs": achieved,
                        "note": "bytes a kernel streaming its state through HBM every iteration would move "
                                "per second at this speed; this kernel keeps its state on chip, so it is "
                                "not a bandwidth measurement"},
                    "kernels": kernels}
    else:
        traffic, traffic_src = measured_traffic(dom)
        roofline = {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                    "traffic_source": None if traffic is None else "%s (not measured in this run)" % traffic_src,
                    "avg_ms": kernels[dom]["avg_ms"], "bytes_per_launch": kernels[dom]["bytes_per_launch"],
                    "kernels": kernels}
    out = {
        "metric": "voxel-iterations/s batched vs per-slice PD; p50/p99 solve latency at 1e-4",
        "value": value,
        "unit": "voxel-iterations/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": dt / a.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded needle/seed phantoms, 1% noise)",
        "config": {"workload": "batched PD, 64 slices of 256x256, 500 iterations, lambda 1e-3",
                   "slices": NZ, "nx": NX, "ny": NY, "iterations": ITERS, "parallelism": "single GPU"},
        "per_slice": None if per_slice is None else {
            "value": vit / per_slice, "unit": "voxel-iterations/s", "ms_per_solve": per_slice * 1e3,
            "speedup_batched": value / (vit / per_slice), "relL2_vs_batched": per_slice_rel},
        "roofline": roofline,
        "rel_gap": info["rel_gap"],
        "autotune": {"choice": tune_choice, "timings": tune_table},
    }
    if not a.no_workloads:
        out["workloads"] = other_workloads()
        out["workloads"]["tv_256x256x64_500it"] = tv_workload()
        out["workloads"]["dipole3d_256x256x64_500it"] = volume3d_workload()
        out["workloads"]["tv3_256x256x64_500it"] = tv3_workload()
    if a.serve_seconds > 0:
        out["serving"] = serving(a.serve_rate, a.serve_seconds, a.serve_arena_gb)
    if a.serve_seconds > 0 and a.serve_stress_seconds > 0:
        # admission under pressure: the same request mix with a 2 GB arena,
        # where requests wait for arena space
        out["serving_2GB_arena"] = serving(a.serve_rate, a.serve_stress_seconds, 2.0)
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, a.cpu_sample_slices, a.cpu_sample_iters)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

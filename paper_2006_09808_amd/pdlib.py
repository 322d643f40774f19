"""ctypes binding of the HIP primal-dual solver library (C ABI of include/pd.h).

Argument marshalling only: every step of the solve runs in the library's HIP
kernels.  PyTorch supplies device memory (the arena, the field map and the
output) and synchronisation with the caller's stream.  If the compiled
library is missing this module raises on import of the library, it never
falls back to another implementation.
"""

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpd_hip.so")

PD_OK, PD_PENDING = 0, 1
PD_ERR_ARG, PD_ERR_SIZE, PD_ERR_STEP, PD_ERR_BUDGET = -1, -2, -3, -4
PD_ERR_NONFINITE, PD_ERR_HIP, PD_ERR_CANCELLED, PD_ERR_TICKET, PD_ERR_NODEVICE = -5, -6, -7, -8, -9
PD_ERR_SCRATCH = -10
PD_STATIC_SCRATCH_BYTES = 64 << 20
PD_FP32, PD_FP64 = 0, 1
PD_KERNEL_DIPOLE, PD_KERNEL_IDENTITY, PD_KERNEL_DIPOLE_3D = 0, 1, 2
_KERNELS = {"dipole": PD_KERNEL_DIPOLE, "identity": PD_KERNEL_IDENTITY, "dipole3d": PD_KERNEL_DIPOLE_3D}
PD_MODEL_L1, PD_MODEL_TV = 0, 1
PD_FLAG_TIME_KERNELS, PD_FLAG_NO_RESIDENT, PD_FLAG_FENCED_EXCHANGE, PD_FLAG_NO_GRAPHS = 1, 2, 4, 8
PD_FLAG_TEST_BARRIER_GIVEUP = 16
KIND_COLUMN, KIND_ROW, KIND_RESIDENT, KIND_TV_COLUMN, KIND_TV_ROW, KIND_Z, KIND_MULTI, KIND_TV_RESIDENT = range(8)

# lengths with a direct FFT plan; any other length 2..MAX_BLUESTEIN runs
# through the Bluestein (chirp-z) engine
SUPPORTED_SIZES = (8, 16, 24, 32, 48, 64, 96, 128, 192, 256, 288, 384, 512, 576, 768)
MAX_BLUESTEIN = 384

EXPORTS = ("pd_create", "pd_solve_batch", "pd_poll", "pd_destroy", "pd_status_string",
           "pd_validate", "pd_kernel_norm", "pd_apply_kernel", "pd_now",
           "pd_kernel_time", "pd_kernel_time_reset", "pd_graph_stats", "pd_arena_usage",
           "pd_tune", "pd_tune_set", "pd_tune_get", "pd_recovery_stats", "pd_apply_kernel_noalloc")


class PdConfig(ctypes.Structure):
    _fields_ = [("device", ctypes.c_int), ("stream", ctypes.c_void_p),
                ("arena", ctypes.c_void_p), ("arena_bytes", ctypes.c_size_t),
                ("max_slots", ctypes.c_int), ("precision", ctypes.c_int),
                ("step_iters", ctypes.c_int), ("flags", ctypes.c_int), ("tune_cache", ctypes.c_char_p)]


class PdRequest(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
                ("b0", ctypes.c_double * 3), ("voxel", ctypes.c_double * 2),
                ("kernel", ctypes.c_int), ("lam", ctypes.c_double),
                ("tau", ctypes.c_double), ("sigma", ctypes.c_double),
                ("theta", ctypes.c_double), ("max_iter", ctypes.c_int),
                ("gap_tol", ctypes.c_double), ("check_every", ctypes.c_int),
                ("delta", ctypes.c_void_p), ("chi", ctypes.c_void_p),
                ("model", ctypes.c_int), ("weight", ctypes.c_void_p), ("mask", ctypes.c_void_p),
                ("voxel_z", ctypes.c_double)]


class PdTuneEntry(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int), ("iters", ctypes.c_int),
                ("path", ctypes.c_int), ("variant", ctypes.c_int), ("team", ctypes.c_int),
                ("threads", ctypes.c_int), ("rows", ctypes.c_int), ("cols", ctypes.c_int),
                ("plan", ctypes.c_int), ("ms", ctypes.c_double)]


class PdResult(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("iterations", ctypes.c_int),
                ("primal", ctypes.c_double), ("dual", ctypes.c_double),
                ("rel_gap", ctypes.c_double), ("t_submit", ctypes.c_double),
                ("t_start", ctypes.c_double), ("t_done", ctypes.c_double)]


_lib = None


def load_library(path=None):
    """Load libpd_hip.so (built by paper_2006_09808_amd.build).  Raises
    OSError if it is missing: there is no other implementation to fall back to."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise OSError("HIP library %s is not built; run `python -m paper_2006_09808_amd.build`" % p)
    lib = ctypes.CDLL(p)
    c = ctypes
    lib.pd_create.argtypes = [c.POINTER(PdConfig), c.POINTER(c.c_void_p)]
    lib.pd_solve_batch.argtypes = [c.c_void_p, c.POINTER(PdRequest), c.c_int, c.POINTER(c.c_uint64)]
    lib.pd_poll.argtypes = [c.c_void_p, c.c_uint64, c.POINTER(PdResult), c.c_int]
    lib.pd_destroy.argtypes = [c.c_void_p]
    lib.pd_status_string.argtypes = [c.c_int32]
    lib.pd_status_string.restype = c.c_char_p
    lib.pd_validate.argtypes = [c.POINTER(PdRequest), c.c_int, c.POINTER(c.c_size_t)]
    lib.pd_kernel_norm.argtypes = [c.POINTER(PdRequest), c.POINTER(c.c_double)]
    lib.pd_apply_kernel.argtypes = [c.c_void_p, c.POINTER(PdRequest)]
    lib.pd_apply_kernel_noalloc.argtypes = [c.c_void_p, c.POINTER(PdRequest)]
    lib.pd_now.argtypes = []
    lib.pd_now.restype = c.c_double
    lib.pd_kernel_time.argtypes = [c.c_void_p, c.c_int, c.POINTER(c.c_int64), c.POINTER(c.c_double),
                                   c.POINTER(c.c_double)]
    lib.pd_kernel_time_reset.argtypes = [c.c_void_p]
    lib.pd_arena_usage.argtypes = [c.c_void_p, c.POINTER(c.c_size_t), c.POINTER(c.c_int), c.POINTER(c.c_int)]
    lib.pd_graph_stats.argtypes = [c.c_void_p, c.POINTER(c.c_int64), c.POINTER(c.c_int64)]
    lib.pd_recovery_stats.argtypes = [c.c_void_p, c.POINTER(c.c_int64), c.POINTER(c.c_int64)]
    lib.pd_tune.argtypes = [c.c_void_p, c.c_int, c.c_int, c.c_int, c.c_int, c.POINTER(PdTuneEntry), c.c_int,
                            c.POINTER(c.c_int)]
    lib.pd_tune_set.argtypes = [c.c_void_p, c.c_int, c.c_int, c.c_int, c.c_int, c.c_int, c.c_int, c.c_int]
    lib.pd_tune_get.argtypes = [c.c_void_p, c.c_int, c.c_int, c.POINTER(c.c_int), c.POINTER(c.c_int),
                                c.POINTER(c.c_int), c.POINTER(c.c_int), c.POINTER(c.c_int)]
    for name in ("pd_create", "pd_solve_batch", "pd_poll", "pd_destroy", "pd_validate",
                 "pd_kernel_norm", "pd_apply_kernel", "pd_kernel_time", "pd_kernel_time_reset",
                 "pd_graph_stats", "pd_arena_usage", "pd_tune", "pd_tune_set", "pd_tune_get",
                 "pd_recovery_stats", "pd_apply_kernel_noalloc"):
        getattr(lib, name).restype = c.c_int32
    if path is None:
        _lib = lib
    return lib


class PdError(RuntimeError):
    def __init__(self, status, what=""):
        self.status = int(status)
        name = load_library().pd_status_string(self.status).decode()
        super().__init__("%s%s (status %d)" % (what + ": " if what else "", name, self.status))


def status_string(status):
    return load_library().pd_status_string(int(status)).decode()


def now():
    return load_library().pd_now()


def make_request(nx, ny, nz, delta_ptr=0, chi_ptr=0, lam=1e-3, tau=1.4, sigma=1.4, theta=1.0,
                 max_iter=200, gap_tol=0.0, check_every=10, b0=(0.0, 1.0, 0.0), voxel=(1.0, 1.0),
                 kernel="dipole", model="l1", weight_ptr=0, mask_ptr=0, voxel_z=1.0):
    r = PdRequest()
    r.nx, r.ny, r.nz = int(nx), int(ny), int(nz)
    r.b0 = (ctypes.c_double * 3)(*[float(v) for v in b0])
    r.voxel = (ctypes.c_double * 2)(*[float(v) for v in voxel])
    r.kernel = _KERNELS[kernel] if isinstance(kernel, str) else int(kernel)
    r.voxel_z = float(voxel_z)
    r.lam, r.tau, r.sigma, r.theta = float(lam), float(tau), float(sigma), float(theta)
    r.max_iter, r.gap_tol, r.check_every = int(max_iter), float(gap_tol), int(check_every)
    r.delta, r.chi = int(delta_ptr) or None, int(chi_ptr) or None
    r.model = {"l1": PD_MODEL_L1, "tv": PD_MODEL_TV}[model] if isinstance(model, str) else int(model)
    r.weight, r.mask = int(weight_ptr) or None, int(mask_ptr) or None
    return r


def validate(nx, ny, nz, precision="fp32", **params):
    """Host-only validation (no GPU): returns the arena bytes the request needs;
    raises PdError with the library's status otherwise."""
    r = make_request(nx, ny, nz, delta_ptr=params.pop("delta_ptr", 1), chi_ptr=params.pop("chi_ptr", 2),
                     **params)
    nbytes = ctypes.c_size_t(0)
    st = load_library().pd_validate(ctypes.byref(r), _prec(precision), ctypes.byref(nbytes))
    if st != PD_OK:
        raise PdError(st, "validate")
    return int(nbytes.value)


def kernel_norm(nx, ny, b0=(0.0, 1.0, 0.0), voxel=(1.0, 1.0), kernel="dipole", nz=1, voxel_z=1.0):
    r = make_request(nx, ny, nz, b0=b0, voxel=voxel, kernel=kernel, voxel_z=voxel_z)
    out = ctypes.c_double(0.0)
    st = load_library().pd_kernel_norm(ctypes.byref(r), ctypes.byref(out))
    if st != PD_OK:
        raise PdError(st, "kernel_norm")
    return out.value


def _prec(p):
    if isinstance(p, str):
        return {"fp32": PD_FP32, "fp64": PD_FP64}[p]
    return int(p)


def _result_dict(res):
    return {"status": int(res.status), "iterations": int(res.iterations), "primal": res.primal,
            "dual": res.dual, "rel_gap": res.rel_gap, "t_submit": res.t_submit,
            "t_start": res.t_start, "t_done": res.t_done}


class Solver:
    """A library context on one GPU: an arena (HBM budget) and a worker that
    iterates every admitted request together (continuous batching)."""

    def __init__(self, arena_bytes=1 << 30, device=0, max_slots=0, precision="fp32",
                 step_iters=0, time_kernels=False, resident=True, fenced_exchange=False, graphs=True,
                 stream=None, arena=None, tune_cache=None, barrier_giveup_test=False):
        import torch
        self._torch = torch
        self.lib = load_library()
        self.device = int(device)
        self.precision = _prec(precision)
        self.dtype = torch.float64 if self.precision == PD_FP64 else torch.float32
        dev = torch.device("cuda", self.device)
        self.arena = arena if arena is not None else torch.empty(int(arena_bytes), dtype=torch.uint8, device=dev)
        self._stream = stream
        cfg = PdConfig()
        cfg.device = self.device
        cfg.stream = int(stream.cuda_stream) if stream is not None else None
        cfg.arena = self.arena.data_ptr()
        cfg.arena_bytes = self.arena.numel() * self.arena.element_size()
        cfg.max_slots = int(max_slots)
        cfg.precision = self.precision
        cfg.step_iters = int(step_iters)
        cfg.flags = ((PD_FLAG_TIME_KERNELS if time_kernels else 0) | (0 if resident else PD_FLAG_NO_RESIDENT)
                     | (PD_FLAG_FENCED_EXCHANGE if fenced_exchange else 0) | (0 if graphs else PD_FLAG_NO_GRAPHS)
                     | (PD_FLAG_TEST_BARRIER_GIVEUP if barrier_giveup_test else 0))
        cfg.tune_cache = os.fsencode(tune_cache) if tune_cache else None
        self._ctx = ctypes.c_void_p()
        st = self.lib.pd_create(ctypes.byref(cfg), ctypes.byref(self._ctx))
        if st != PD_OK:
            raise PdError(st, "pd_create")
        self._keep = {}

    # -- submission --------------------------------------------------------
    def _check_tensor(self, t, name):
        torch = self._torch
        if not (t.is_cuda and t.device.index == self.device):
            raise ValueError("%s must live on cuda:%d" % (name, self.device))
        if t.dtype != self.dtype or t.dim() != 3 or not t.is_contiguous():
            raise ValueError("%s must be a contiguous [nz, ny, nx] %s tensor" % (name, self.dtype))
        return t

    def submit(self, jobs):
        """jobs: list of (delta, chi, params).  Returns tickets.  For the
        weighted TV model, params holds model="tv" and the device tensors
        weight (W) and mask (M) of delta's shape."""
        torch = self._torch
        reqs = (PdRequest * len(jobs))()
        keep = []
        for i, (delta, chi, params) in enumerate(jobs):
            self._check_tensor(delta, "delta")
            self._check_tensor(chi, "chi")
            if delta.shape != chi.shape:
                raise ValueError("delta and chi shapes differ")
            params = dict(params)
            extra = []
            for key in ("weight", "mask"):
                t = params.pop(key, None)
                if t is not None:
                    self._check_tensor(t, key)
                    if t.shape != delta.shape:
                        raise ValueError("%s and delta shapes differ" % key)
                    params[key + "_ptr"] = t.data_ptr()
                    extra.append(t)
            nz, ny, nx = delta.shape
            reqs[i] = make_request(nx, ny, nz, delta.data_ptr(), chi.data_ptr(), **params)
            keep.append((delta, chi) + tuple(extra))
        # inputs written by torch on the caller's stream must be complete
        torch.cuda.current_stream(self.device).synchronize()
        tickets = (ctypes.c_uint64 * len(jobs))()
        st = self.lib.pd_solve_batch(self._ctx, reqs, len(jobs), tickets)
        if st != PD_OK:
            raise PdError(st, "pd_solve_batch")
        out = [int(t) for t in tickets]
        for t, k in zip(out, keep):
            self._keep[t] = k
        return out

    def poll(self, ticket, timeout_ms=-1):
        """Result dict once finished, None while pending."""
        res = PdResult()
        st = self.lib.pd_poll(self._ctx, ctypes.c_uint64(ticket), ctypes.byref(res), int(timeout_ms))
        if st == PD_PENDING:
            return None
        if st == PD_ERR_TICKET:
            raise PdError(st, "pd_poll")
        self._keep.pop(ticket, None)
        return _result_dict(res)

    def solve(self, delta, chi=None, **params):
        """Blocking solve of one volume: returns (chi, info)."""
        if chi is None:
            chi = self._torch.empty_like(delta)
        (t,) = self.submit([(delta, chi, params)])
        info = self.poll(t, -1)
        if info["status"] not in (PD_OK,):
            raise PdError(info["status"], "solve")
        return chi, info

    def apply_kernel(self, x, out=None, b0=(0.0, 1.0, 0.0), voxel=(1.0, 1.0), kernel="dipole", voxel_z=1.0,
                     noalloc=False):
        """out = A x (the field map of susceptibility x): slice by slice, or
        over the whole volume for kernel="dipole3d".  noalloc=True calls
        pd_apply_kernel_noalloc, whose scratch is the library's fixed device
        array instead of the arena (out must then be given to allocate nothing)."""
        self._check_tensor(x, "x")
        if out is None:
            out = self._torch.empty_like(x)
        self._check_tensor(out, "out")
        nz, ny, nx = x.shape
        r = make_request(nx, ny, nz, x.data_ptr(), out.data_ptr(), b0=b0, voxel=voxel, kernel=kernel,
                         voxel_z=voxel_z)
        self._torch.cuda.current_stream(self.device).synchronize()
        fn = self.lib.pd_apply_kernel_noalloc if noalloc else self.lib.pd_apply_kernel
        st = fn(self._ctx, ctypes.byref(r))
        if st != PD_OK:
            raise PdError(st, "pd_apply_kernel_noalloc" if noalloc else "pd_apply_kernel")
        return out

    # -- introspection -----------------------------------------------------
    def kernel_time(self, kind):
        """(launches, summed HIP-event ms, summed iterations x slice-pair points)
        of one kernel class (KIND_COLUMN, KIND_ROW, KIND_RESIDENT)."""
        n = ctypes.c_int64(0)
        ms = ctypes.c_double(0.0)
        pts = ctypes.c_double(0.0)
        st = self.lib.pd_kernel_time(self._ctx, int(kind), ctypes.byref(n), ctypes.byref(ms), ctypes.byref(pts))
        if st != PD_OK:
            raise PdError(st, "pd_kernel_time")
        return int(n.value), float(ms.value), float(pts.value)

    def kernel_time_reset(self):
        self.lib.pd_kernel_time_reset(self._ctx)

    def tune(self, nx, ny, nz, iters=20):
        """Time every kernel configuration of the nx x ny shape and make the
        fastest the context's choice.  Returns the list of timings: path
        "resident" (variant, team, threads), "column" (cols, plan of the ny
        transforms) or "row" (rows, plan of the nx transforms)."""
        buf = (PdTuneEntry * 64)()
        n = ctypes.c_int(0)
        st = self.lib.pd_tune(self._ctx, int(nx), int(ny), int(nz), int(iters), buf, 64, ctypes.byref(n))
        if st != PD_OK:
            raise PdError(st, "pd_tune")
        out = []
        for e in buf[:n.value]:
            out.append({"path": ("resident", "column", "row")[e.path], "variant": e.variant,
                        "team": e.team, "threads": e.threads, "rows": e.rows, "cols": e.cols, "plan": e.plan,
                        "ms": e.ms, "nz": e.nz, "iters": e.iters})
        return out

    def tune_get(self, nx, ny):
        v, r, cl, px, py = (ctypes.c_int(0) for _ in range(5))
        st = self.lib.pd_tune_get(self._ctx, int(nx), int(ny), ctypes.byref(v), ctypes.byref(r), ctypes.byref(cl),
                                  ctypes.byref(px), ctypes.byref(py))
        if st != PD_OK:
            raise PdError(st, "pd_tune_get")
        return {"variant": v.value, "rows": r.value, "cols": cl.value, "plan_x": px.value, "plan_y": py.value}

    def tune_set(self, nx, ny, variant=-1, rows=0, cols=0, plan_x=0, plan_y=0):
        st = self.lib.pd_tune_set(self._ctx, int(nx), int(ny), int(variant), int(rows), int(cols), int(plan_x),
                                  int(plan_y))
        if st != PD_OK:
            raise PdError(st, "pd_tune_set")

    def save_tuning(self, path, shapes):
        """Write the choices of the given (nx, ny) shapes as JSON."""
        import json
        with open(path, "w") as f:
            json.dump({"%dx%d" % (nx, ny): self.tune_get(nx, ny) for nx, ny in shapes}, f, indent=1)

    def load_tuning(self, path):
        import json
        with open(path) as f:
            d = json.load(f)
        for k, v in d.items():
            nx, ny = (int(t) for t in k.split("x"))
            self.tune_set(nx, ny, v["variant"], v["rows"], v["cols"], v.get("plan_x", 0), v.get("plan_y", 0))

    def graph_stats(self):
        """(steps captured into HIP graphs, steps replayed from one)."""
        cap = ctypes.c_int64(0)
        rep = ctypes.c_int64(0)
        st = self.lib.pd_graph_stats(self._ctx, ctypes.byref(cap), ctypes.byref(rep))
        if st != PD_OK:
            raise PdError(st, "pd_graph_stats")
        return int(cap.value), int(rep.value)

    def recovery_stats(self):
        """(scheduling rounds whose resident launch gave up at a team barrier,
        requests restarted on the two-launch path because of it)."""
        ab = ctypes.c_int64(0)
        rs = ctypes.c_int64(0)
        st = self.lib.pd_recovery_stats(self._ctx, ctypes.byref(ab), ctypes.byref(rs))
        if st != PD_OK:
            raise PdError(st, "pd_recovery_stats")
        return int(ab.value), int(rs.value)

    def arena_usage(self):
        used = ctypes.c_size_t(0)
        res = ctypes.c_int(0)
        q = ctypes.c_int(0)
        self.lib.pd_arena_usage(self._ctx, ctypes.byref(used), ctypes.byref(res), ctypes.byref(q))
        return int(used.value), int(res.value), int(q.value)

    def close(self):
        if self._ctx:
            self.lib.pd_destroy(self._ctx)
            self._ctx = ctypes.c_void_p()
            self._keep.clear()

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

"""Seeded synthetic susceptibility phantoms for the positive-contrast workloads.

Shared by the oracle-side tests and the HIP-side tests/benchmark.  It holds
none of the solver's arithmetic: it draws ground-truth susceptibility maps
(metal devices over tissue) and standard-normal noise fields, and scales the
noise onto a field map computed elsewhere.  The field map A chi itself is
computed by whichever side is being exercised (the oracle's dense DFT, or
the library's own dipole forward operator).

The paper's datasets (stent, seeds in meat, needle in a copper-sulfate
phantom; Sec. III) are not available, so these stand in for them with the
same device types: needle cross-sections (discs), brachytherapy seeds
(small ellipses) and a tilted needle crossing a slice stack.

Conventions: geometry in voxel units, object centres at integer coordinates,
arrays are [nz, ny, nx] (x fastest), susceptibility in ppm.  Objects drawn
later overwrite earlier ones; every voxel no object covers carries tissue
noise N(0, 0.05^2) ppm.  B0 lies in-plane along y.  Each workload's noise
field eta is standard normal; the measured field map is
    delta = field + rho * max|field| * eta.
"""

from dataclasses import dataclass, field as dc_field
import math

import numpy as np

TISSUE_SD = 0.05          # ppm
B0_Y = (0.0, 1.0, 0.0)


@dataclass
class Workload:
    """One reconstruction request: ground truth, noise, and solver settings."""
    chi_true: np.ndarray            # float64 [nz, ny, nx], ppm
    eta: np.ndarray                 # float64 [nz, ny, nx], standard normal
    rho: float                      # noise level relative to max |field|
    lam: float = 1e-3
    tau: float = 1.4
    sigma: float = 1.4
    theta: float = 1.0
    max_iter: int = 200
    gap_tol: float = 0.0
    check_every: int = 10
    b0: tuple = B0_Y
    voxel: tuple = (1.0, 1.0)
    name: str = ""
    meta: dict = dc_field(default_factory=dict)

    @property
    def shape(self):
        return self.chi_true.shape

    def solver_params(self):
        return dict(lam=self.lam, tau=self.tau, sigma=self.sigma, theta=self.theta,
                    max_iter=self.max_iter, gap_tol=self.gap_tol,
                    check_every=self.check_every, b0=self.b0, voxel=self.voxel)


def make_delta(field, eta, rho):
    """Measured field map: field plus Gaussian noise at rho * max|field|."""
    field = np.asarray(field, dtype=np.float64)
    amp = float(np.max(np.abs(field))) if field.size else 0.0
    return field + rho * amp * np.asarray(eta, dtype=np.float64)


def _grid(ny, nx):
    yy, xx = np.meshgrid(np.arange(ny, dtype=np.float64),
                         np.arange(nx, dtype=np.float64), indexing="ij")
    return yy, xx


def _tissue(rng, shape):
    return rng.normal(0.0, TISSUE_SD, size=shape)


def device_slice(rng, ny, nx):
    """One slice of needle discs and seed ellipses; returns (values, covered)."""
    yy, xx = _grid(ny, nx)
    val = np.zeros((ny, nx))
    cov = np.zeros((ny, nx), dtype=bool)
    for _ in range(int(rng.integers(2, 7))):              # 2..6 needle discs
        r = int(rng.integers(2, 6))                         # radius 2..5
        r = max(1, min(r, (min(ny, nx) - 1) // 2))
        v = float(rng.uniform(150.0, 200.0))
        cy = int(rng.integers(r, ny - r))
        cx = int(rng.integers(r, nx - r))
        m = (yy - cy) ** 2 + (xx - cx) ** 2 <= r * r
        val[m] = v
        cov |= m
    for _ in range(int(rng.integers(0, 4))):              # 0..3 seeds
        a, b = (2.5, 1.5) if rng.integers(0, 2) == 0 else (1.5, 2.5)
        cy = int(rng.integers(min(3, ny // 2), max(ny - 3, ny // 2 + 1)))
        cx = int(rng.integers(min(3, nx // 2), max(nx - 3, nx // 2 + 1)))
        m = ((xx - cx) / a) ** 2 + ((yy - cy) / b) ** 2 <= 1.0
        val[m] = 100.0
        cov |= m
    return val, cov


def device_stack(rng, nz, ny, nx):
    """Ground truth for nz slices of discs/ellipses over tissue noise."""
    chi = _tissue(rng, (nz, ny, nx))
    for z in range(nz):
        val, cov = device_slice(rng, ny, nx)
        chi[z][cov] = val[cov]
    return chi


def needle_disc_slice(n=64, r=3, value=180.0, rng=None):
    """A single needle cross-section of radius r at the slice centre."""
    rng = np.random.default_rng(0) if rng is None else rng
    chi = _tissue(rng, (1, n, n))
    yy, xx = _grid(n, n)
    m = (yy - n // 2) ** 2 + (xx - n // 2) ** 2 <= r * r
    chi[0][m] = value
    return chi


def tilted_needle(rng, nz, ny, nx, r=3.0, value=180.0, tilt_deg=30.0):
    """A needle of radius r through the volume centre, tilted tilt_deg from
    B0 (y) towards z; every slice shows an ellipse drifting in y."""
    chi = _tissue(rng, (nz, ny, nx))
    c = np.array([nx // 2, ny // 2, nz // 2], dtype=np.float64)
    t = math.radians(tilt_deg)
    u = np.array([0.0, math.cos(t), math.sin(t)])
    yy, xx = _grid(ny, nx)
    for z in range(nz):
        px, py, pz = xx - c[0], yy - c[1], float(z) - c[2]
        proj = px * u[0] + py * u[1] + pz * u[2]
        d2 = px * px + py * py + pz * pz - proj * proj
        m = d2 <= r * r
        chi[z][m] = value
    return chi


# ---------------------------------------------------------------------------
# The five workloads (sizes and distributions of the positive-contrast
# experiments, scaled to the throughput/latency/precision questions asked)
# ---------------------------------------------------------------------------

def config1(seed=1000):
    """One 64x64 slice, needle disc r=3 at 180 ppm, 1% noise, 200 iterations."""
    rng = np.random.default_rng(seed)
    chi = needle_disc_slice(64, 3, 180.0, rng)
    eta = rng.standard_normal(chi.shape)
    return Workload(chi, eta, 0.01, lam=1e-3, max_iter=200, name="plain_64x64x1")


def config2(seed=2000, nz=64, n=256, max_iter=500):
    """nz slices of n x n with 2-6 needle discs and 0-3 seeds, 1% noise."""
    rng = np.random.default_rng(seed)
    chi = device_stack(rng, nz, n, n)
    eta = rng.standard_normal(chi.shape)
    return Workload(chi, eta, 0.01, lam=1e-3, max_iter=max_iter,
                    name="batched_%dx%dx%d" % (n, n, nz))


def config3(seed=3000, shapes=((128, 32), (256, 48), (384, 24)),
            gap_tol=1e-5, max_iter=1000):
    """Uneven batch: one volume per (n, nz), each stopping at its own gap."""
    out = []
    for i, (n, nz) in enumerate(shapes):
        rng = np.random.default_rng(seed + i)
        chi = device_stack(rng, nz, n, n)
        eta = rng.standard_normal(chi.shape)
        out.append(Workload(chi, eta, 0.01, lam=1e-3, max_iter=max_iter,
                            gap_tol=gap_tol, check_every=10,
                            name="uneven_%dx%dx%d" % (n, n, nz)))
    return out


def config4(seed=4000, nz=128, n=256, max_iter=800):
    """Tilted needle (30 deg to B0) across nz slices, 0.5% noise, lam=5e-4."""
    rng = np.random.default_rng(seed)
    chi = tilted_needle(rng, nz, n, n)
    eta = rng.standard_normal(chi.shape)
    return Workload(chi, eta, 0.005, lam=5e-4, max_iter=max_iter,
                    name="precision_%dx%dx%d" % (n, n, nz))


SERVING_SIZES = (128, 192, 256, 384)


def serving_schedule(seed=5000, rate=20.0, duration=60.0):
    """Open-loop Poisson arrivals: list of (t_arrival_s, n, nz, request_seed)."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    i = 0
    while True:
        t += float(rng.exponential(1.0 / rate))
        if t >= duration:
            break
        n = SERVING_SIZES[int(rng.integers(0, len(SERVING_SIZES)))]
        nz = int(rng.integers(16, 65))
        out.append((t, n, nz, seed + 1 + i))
        i += 1
    return out


def serving_request(request_seed, n, nz, gap_tol=1e-5, max_iter=1000):
    """One served reconstruction, generated as the batched workload."""
    rng = np.random.default_rng(request_seed)
    chi = device_stack(rng, nz, n, n)
    eta = rng.standard_normal(chi.shape)
    return Workload(chi, eta, 0.01, lam=1e-3, max_iter=max_iter, gap_tol=gap_tol,
                    check_every=10, name="serve_%dx%dx%d" % (n, n, nz))


def random_stack(seed, nz, ny, nx, rho=0.01, **params):
    """Device stack on an arbitrary (possibly rectangular) grid."""
    rng = np.random.default_rng(seed)
    chi = device_stack(rng, nz, ny, nx)
    eta = rng.standard_normal(chi.shape)
    return Workload(chi, eta, rho, name="stack_%dx%dx%d" % (nx, ny, nz), **params)


# ---------------------------------------------------------------------------
# Weighted-TV model inputs (Eq. (1)): weights W and a mask M beside the
# ground truth.  W stands in for a magnitude-derived weight (about 1 in
# tissue, lower inside each device's signal void); M is 1 inside an
# elliptical field of view covering most of the slice, 0 outside.
# ---------------------------------------------------------------------------

@dataclass
class TvWorkload:
    chi_true: np.ndarray            # float64 [nz, ny, nx], ppm
    eta: np.ndarray                 # float64 [nz, ny, nx], standard normal
    rho: float
    weight: np.ndarray              # float64 [nz, ny, nx], in [0.2, 1]
    mask: np.ndarray                # float64 [nz, ny, nx], 0 or 1
    lam: float = 100.0              # weight of the data term
    tau: float = 0.34
    sigma: float = 0.34
    theta: float = 1.0
    max_iter: int = 200
    b0: tuple = B0_Y
    voxel: tuple = (1.0, 1.0)
    name: str = ""

    @property
    def shape(self):
        return self.chi_true.shape

    def solver_params(self):
        """Scalar parameters; W and M travel as arrays beside them."""
        return dict(lam=self.lam, tau=self.tau, sigma=self.sigma, theta=self.theta,
                    max_iter=self.max_iter, b0=self.b0, voxel=self.voxel)


def weight_and_mask(chi_true, void_scale=2.0):
    """W = 1 - 0.8 exp(-d^2 / (2 s^2)) with d the distance to the nearest
    device voxel (|chi| > 50 ppm) in-plane and s = void_scale voxels; M = 1
    inside the ellipse with semi-axes 0.45 nx, 0.45 ny about the centre."""
    from scipy.ndimage import distance_transform_edt
    nz, ny, nx = chi_true.shape
    yy, xx = _grid(ny, nx)
    w = np.ones((nz, ny, nx))
    for z in range(nz):
        dev = np.abs(chi_true[z]) > 50.0
        if not dev.any():
            continue
        d = distance_transform_edt(~dev)
        w[z] = 1.0 - 0.8 * np.exp(-d * d / (2.0 * void_scale ** 2))
    ell = ((xx - (nx - 1) / 2.0) / (0.45 * nx)) ** 2 + ((yy - (ny - 1) / 2.0) / (0.45 * ny)) ** 2 <= 1.0
    m = np.broadcast_to(ell.astype(np.float64), (nz, ny, nx)).copy()
    return w, m


def tv_stack(seed, nz, ny, nx, rho=0.01, **params):
    """Device stack (as the batched workload) with its W and M."""
    rng = np.random.default_rng(seed)
    chi = device_stack(rng, nz, ny, nx)
    eta = rng.standard_normal(chi.shape)
    w, m = weight_and_mask(chi)
    return TvWorkload(chi, eta, rho, w, m, name="tv_%dx%dx%d" % (nx, ny, nz), **params)


# ---------------------------------------------------------------------------
# Serving requests drawn on the GPU: the same recipe as device_stack (tissue
# noise, 2-6 needle discs and 0-3 seed ellipses per slice, later objects
# over earlier ones), each request from its own seed, with the two noise
# fields drawn on the device so that a thousand independent requests can be
# made in seconds.  The object geometry is drawn on the host and painted
# into the device array in drawing order.
# ---------------------------------------------------------------------------

def device_objects(rng, nz, ny, nx):
    """(z, y, x, value) of every voxel the discs and ellipses of an nz-slice
    stack cover, in drawing order (a voxel listed twice takes its last
    value), as four numpy arrays."""
    zs, ys, xs, vs = [], [], [], []

    def paint(z, cy, cx, ry, rx, value, ellipse):
        y0, y1 = max(0, int(cy - ry) - 1), min(ny, int(cy + ry) + 2)
        x0, x1 = max(0, int(cx - rx) - 1), min(nx, int(cx + rx) + 2)
        yy, xx = np.meshgrid(np.arange(y0, y1), np.arange(x0, x1), indexing="ij")
        if ellipse:
            m = ((xx - cx) / rx) ** 2 + ((yy - cy) / ry) ** 2 <= 1.0
        else:
            m = (yy - cy) ** 2 + (xx - cx) ** 2 <= ry * ry
        k = int(m.sum())
        zs.append(np.full(k, z))
        ys.append(yy[m])
        xs.append(xx[m])
        vs.append(np.full(k, value))

    for z in range(nz):
        for _ in range(int(rng.integers(2, 7))):
            r = int(rng.integers(2, 6))
            r = max(1, min(r, (min(ny, nx) - 1) // 2))
            v = float(rng.uniform(150.0, 200.0))
            cy = int(rng.integers(r, ny - r))
            cx = int(rng.integers(r, nx - r))
            paint(z, cy, cx, r, r, v, False)
        for _ in range(int(rng.integers(0, 4))):
            a, b = (2.5, 1.5) if rng.integers(0, 2) == 0 else (1.5, 2.5)
            cy = int(rng.integers(min(3, ny // 2), max(ny - 3, ny // 2 + 1)))
            cx = int(rng.integers(min(3, nx // 2), max(nx - 3, nx // 2 + 1)))
            paint(z, cy, cx, b, a, 100.0, True)
    cat = lambda a: np.concatenate(a) if a else np.zeros(0)
    return cat(zs).astype(np.int64), cat(ys).astype(np.int64), cat(xs).astype(np.int64), cat(vs)


def serving_request_device(request_seed, n, nz, device):
    """One served request's ground truth chi (float32, on `device`) and a
    standard-normal noise field eta of the same shape, both from its own
    seed: tissue noise and eta drawn by a device generator seeded with it,
    the devices painted over the tissue in drawing order."""
    import torch
    rng = np.random.default_rng(request_seed)
    z, y, x, v = device_objects(rng, nz, n, n)
    g = torch.Generator(device=device)
    g.manual_seed(int(request_seed))
    chi = torch.randn((nz, n, n), generator=g, device=device, dtype=torch.float32) * TISSUE_SD
    eta = torch.randn((nz, n, n), generator=g, device=device, dtype=torch.float32)
    if v.size:
        # the last write to a voxel wins: keep each voxel's last object only
        flat = (z * n + y) * n + x
        _, last = np.unique(flat[::-1], return_index=True)
        keep = flat.size - 1 - last
        idx = torch.from_numpy(flat[keep]).to(device)
        chi.view(-1)[idx] = torch.from_numpy(v[keep].astype(np.float32)).to(device)
    return chi, eta

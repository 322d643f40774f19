"""FP64 CPU oracle for the primal-dual dipole deconvolution of
Wang, Cai et al., "Positive Contrast Susceptibility MR Imaging Using GPU-based
Primal-Dual Algorithm" (arXiv:2006.09808).

TEST INFRASTRUCTURE ONLY.  This is the plain, slow, obviously-correct reference
that the HIP solver is checked against.  Only the test-suite, the smoke check
and the benchmark's CPU-baseline leg may import it; the product path never
does.  It shares no code, constants or tables with the HIP library, and it
never takes an input or an expected value from the HIP path.

What it computes (Sec. II-A, Eq. (1) and the PD pseudocode), per 2-D slice:

    minimise over chi   1/2 || A chi - delta ||_2^2  +  lam || chi ||_1
    A = F^-1 diag(D) F,  D(k) = 1/3 - (k . b)^2 / |k|^2,  D(0) = 0

with the first-order primal-dual (Chambolle-Pock) iteration of the paper's
pseudocode, K = A, F*(y) = 1/2||y||^2 + <y, delta>, G(chi) = lam ||chi||_1:

    y      <- (y + sigma (A chibar - delta)) / (1 + sigma)        dual prox
    chi'   <- soft(chi - tau A y, tau lam)                          primal prox
    chibar <- chi' + theta (chi' - chi)                              over-relaxation

Readings of the paper used here (it is silent or ambiguous on these points):
  * lam weights the L1 term (Eq. (1) puts lam/2 on the data term; with the
    workloads' lam = 1e-3 that reading makes the threshold 1000 ppm and the
    solution identically zero), so the dual prox divides by (1 + sigma).
  * The regulariser is L1 on chi itself (M G -> identity) and W = I; the
    weighted TV form of Eq. (1) is not this path.
  * Slices are independent 2-D problems (Sec. II-C, strategy (2)); the kernel
    is the 2-D restriction (k_z = 0) of the dipole kernel, B0 direction given
    in voxel axes, frequencies on the unshifted DFT grid k_i = i/(n d) for
    i < ceil(n/2), else (i - n)/(n d).  Where an even grid's Nyquist line makes
    that formula not even in k (oblique in-plane B0), D is the mean of the
    formula at k and at -k, so A stays real and symmetric.
  * Step sizes must satisfy tau sigma max|D|^2 < 1 strictly (the pseudocode's
    tau = sigma = 1/L sits on the boundary of the convergence condition);
    theta must lie in [0, 1].
  * Exactly max_iter updates; the result is chi after the last update (not
    chibar, not an average).  With gap_tol > 0 the duality gap is evaluated on
    (chi_n, y_n) after every check_every-th update and after the last one, and
    the solve stops at the first check with relgap <= gap_tol.
  * Duality gap (the paper defines none; it stops on n >= N): per volume,
        P    = sum_slices 1/2||A chi - delta||^2 + lam ||chi||_1
        m    = max_slices ||A y||_inf,  s = min(1, lam / m)  (s = 1 if m = 0)
        Dual = sum_slices (-1/2 s^2 ||y||^2 - s <y, delta>)
        relgap = (P - Dual) / max(P, 1e-300)
    s y is feasible for the dual  max -1/2||y||^2 - <y,delta>  s.t.
    ||A y||_inf <= lam, so P - Dual >= 0 (weak duality).

The transform is a dense DFT matrix applied along each axis: no FFT
factorisation, no pairing of slices, and the dual stays in the image domain
(four transforms per iteration), on purpose different from the GPU path.

3-D kernel (kind="dipole3d"; the "all three dimensions" of Sec. II-A): the
same iteration with A = F3^-1 diag(D3) F3 over the whole volume,
D3(k) = 1/3 - (k . b)^2 / |k|^2 on the (kz, ky, kx) grid (kz with voxel size
voxel_z), D3(0) = 0, averaged between k and -k like the 2-D kernel.  It couples
the slices; the 2-D kernel is its kz = 0 plane.
"""

import numpy as np

__all__ = [
    "kgrid", "dipole_kernel", "kernel_norm", "check_steps",
    "dft_matrix", "dft2", "idft2", "apply_A", "forward",
    "dipole_kernel3", "dft3", "idft3", "apply_A3",
    "prox_l1", "prox_dual", "duality_gap", "solve",
]


# ---------------------------------------------------------------------------
# Dipole kernel (Eq. (1), operator D)
# ---------------------------------------------------------------------------

def kgrid(n, d=1.0):
    """Unshifted DFT frequency grid in cycles per unit length: i/(n d) for
    i < ceil(n/2), else (i - n)/(n d)."""
    n = int(n)
    half = (n + 1) // 2
    k = np.empty(n, dtype=np.float64)
    for i in range(n):
        k[i] = (i if i < half else i - n) / (n * float(d))
    return k


def _unit_b0(b0):
    b = np.asarray(b0, dtype=np.float64).reshape(3)
    nrm = float(np.sqrt(np.sum(b * b)))
    if not np.isfinite(nrm) or nrm == 0.0:
        raise ValueError("B0 direction must be a finite, non-zero 3-vector")
    return b / nrm


def dipole_kernel(nx, ny, b0=(0.0, 1.0, 0.0), voxel=(1.0, 1.0), kind="dipole"):
    """D on the (ny, nx) frequency grid (row index = k_y, column = k_x).

    kind="dipole":   D = 1/3 - (kx bx + ky by)^2 / (kx^2 + ky^2), D(0) = 0,
                     symmetrised between k and -k (only changes the Nyquist
                     lines of an even grid with oblique in-plane B0).
    kind="identity": D = 1 everywhere (A = I; used for closed-form checks).
    """
    nx, ny = int(nx), int(ny)
    if kind == "identity":
        return np.ones((ny, nx), dtype=np.float64)
    if kind != "dipole":
        raise ValueError("unknown kernel kind %r" % (kind,))
    b = _unit_b0(b0)
    kx = kgrid(nx, voxel[0])
    ky = kgrid(ny, voxel[1])

    def formula(fx, fy):
        k2 = fx * fx + fy * fy
        if k2 == 0.0:
            return 0.0
        kb = fx * b[0] + fy * b[1]
        return 1.0 / 3.0 - kb * kb / k2

    D = np.empty((ny, nx), dtype=np.float64)
    for j in range(ny):
        for i in range(nx):
            jm, im = (-j) % ny, (-i) % nx          # index of -k
            D[j, i] = 0.5 * (formula(kx[i], ky[j]) + formula(kx[im], ky[jm]))
    return D


def dipole_kernel3(nx, ny, nz, b0=(0.0, 1.0, 0.0), voxel=(1.0, 1.0), voxel_z=1.0):
    """3-D dipole kernel on the (nz, ny, nx) frequency grid:
    D = 1/3 - (k . b)^2 / |k|^2, D(0) = 0, symmetrised between k and -k."""
    nx, ny, nz = int(nx), int(ny), int(nz)
    b = _unit_b0(b0)
    kx = kgrid(nx, voxel[0])
    ky = kgrid(ny, voxel[1])
    kz = kgrid(nz, voxel_z)

    def formula(fx, fy, fz):
        k2 = fx * fx + fy * fy + fz * fz
        if k2 == 0.0:
            return 0.0
        kb = fx * b[0] + fy * b[1] + fz * b[2]
        return 1.0 / 3.0 - kb * kb / k2

    D = np.empty((nz, ny, nx), dtype=np.float64)
    for l in range(nz):
        lm = (-l) % nz
        for j in range(ny):
            jm = (-j) % ny
            for i in range(nx):
                im = (-i) % nx
                D[l, j, i] = 0.5 * (formula(kx[i], ky[j], kz[l]) + formula(kx[im], ky[jm], kz[lm]))
    return D


def kernel_norm(D):
    """||A||_2 = max |D| (A is normal with eigenvalues D)."""
    return float(np.max(np.abs(D)))


def check_steps(tau, sigma, theta, D):
    """Chambolle-Pock step condition tau*sigma*||A||^2 < 1, theta in [0, 1]."""
    L = kernel_norm(D)
    if not (tau > 0 and sigma > 0):
        raise ValueError("tau and sigma must be positive")
    if not (tau * sigma * L * L < 1.0):
        raise ValueError("step sizes violate tau*sigma*max|D|^2 < 1")
    if not (0.0 <= theta <= 1.0):
        raise ValueError("theta must lie in [0, 1]")


# ---------------------------------------------------------------------------
# Naive DFT: dense matrices, one per axis
# ---------------------------------------------------------------------------

def dft_matrix(n, inverse=False):
    """W[k, j] = exp(-+ 2 pi i ((k j) mod n) / n); no 1/n factor."""
    n = int(n)
    kj = np.outer(np.arange(n, dtype=np.int64), np.arange(n, dtype=np.int64)) % n
    sign = 1.0 if inverse else -1.0
    return np.exp(sign * 2j * np.pi * kj.astype(np.float64) / n)


def dft2(x):
    """Unnormalised forward 2-D DFT of the last two axes (ny, nx)."""
    x = np.asarray(x)
    ny, nx = x.shape[-2], x.shape[-1]
    Wy = dft_matrix(ny)
    Wx = dft_matrix(nx)
    return np.matmul(np.matmul(Wy, x.astype(np.complex128)), Wx.T)


def idft2(X):
    """Inverse 2-D DFT of the last two axes, with the 1/(nx ny) factor."""
    X = np.asarray(X)
    ny, nx = X.shape[-2], X.shape[-1]
    Wy = dft_matrix(ny, inverse=True)
    Wx = dft_matrix(nx, inverse=True)
    return np.matmul(np.matmul(Wy, X.astype(np.complex128)), Wx.T) / float(nx * ny)


def dft3(x):
    """Unnormalised forward 3-D DFT of the last three axes (nz, ny, nx)."""
    x = np.asarray(x).astype(np.complex128)
    nz = x.shape[-3]
    X = dft2(x)
    Wz = dft_matrix(nz)
    return np.einsum("kz,...zyx->...kyx", Wz, X)


def idft3(X):
    """Inverse 3-D DFT of the last three axes, with the 1/(nx ny nz) factor."""
    X = np.asarray(X).astype(np.complex128)
    nz = X.shape[-3]
    x = idft2(X)
    Wz = dft_matrix(nz, inverse=True)
    return np.einsum("kz,...zyx->...kyx", Wz, x) / float(nz)


def apply_A3(x, D3):
    """A x = Re F3^-1 (D3 . F3 x) over the whole [nz, ny, nx] volume."""
    x = np.asarray(x, dtype=np.float64)
    z = idft3(D3 * dft3(x))
    scale = max(float(np.max(np.abs(x))) if x.size else 0.0, 1e-300)
    if float(np.max(np.abs(z.imag))) > 1e-10 * scale:
        raise AssertionError("A x has a non-negligible imaginary part")
    return z.real


def apply_A(x, D):
    """A x = Re F^-1 (D . F x), slice by slice over leading axes."""
    x = np.asarray(x, dtype=np.float64)
    z = idft2(D * dft2(x))
    scale = max(float(np.max(np.abs(x))) if x.size else 0.0, 1e-300)
    if float(np.max(np.abs(z.imag))) > 1e-10 * scale:
        raise AssertionError("A x has a non-negligible imaginary part")
    return z.real


def _operator(shape, b0, voxel, kind, voxel_z):
    """(D, A) for a [nz, ny, nx] stack: the slice-wise 2-D kernel, or the
    3-D kernel over the whole volume (kind="dipole3d")."""
    nz, ny, nx = shape
    if kind == "dipole3d":
        D = dipole_kernel3(nx, ny, nz, b0, voxel, voxel_z)
        return D, (lambda x: apply_A3(x, D))
    D = dipole_kernel(nx, ny, b0, voxel, kind)
    return D, (lambda x: apply_A(x, D))


def forward(chi, b0=(0.0, 1.0, 0.0), voxel=(1.0, 1.0), kind="dipole", voxel_z=1.0):
    """Field map produced by a susceptibility stack chi[nz, ny, nx]: A chi."""
    chi = np.asarray(chi, dtype=np.float64)
    if chi.ndim == 2:
        chi = chi[None]
    _, A = _operator(chi.shape, b0, voxel, kind, voxel_z)
    return A(chi)


# ---------------------------------------------------------------------------
# Proximal maps
# ---------------------------------------------------------------------------

def prox_l1(v, t):
    """prox of t||.||_1: argmin_x 1/2 (x - v)^2 + t |x| = sign(v) max(|v|-t, 0)."""
    v = np.asarray(v, dtype=np.float64)
    return np.sign(v) * np.maximum(np.abs(v) - t, 0.0)


def prox_dual(w, delta, sigma):
    """prox of sigma F*, F*(y) = 1/2||y||^2 + <y, delta>:
    argmin_y sigma F*(y) + 1/2||y - w||^2 = (w - sigma delta) / (1 + sigma)."""
    return (np.asarray(w, dtype=np.float64) - sigma * np.asarray(delta, dtype=np.float64)) / (1.0 + sigma)


# ---------------------------------------------------------------------------
# Duality gap
# ---------------------------------------------------------------------------

def duality_gap(chi, y, Ay, delta, D, lam, A=None):
    """(P, Dual, relgap) for the whole stack at the pair (chi, y); Ay = A y.
    A is the operator (default: the slice-wise A with kernel grid D)."""
    r = (A(chi) if A is not None else apply_A(chi, D)) - delta
    P = 0.5 * float(np.sum(r * r)) + lam * float(np.sum(np.abs(chi)))
    m = float(np.max(np.abs(Ay))) if Ay.size else 0.0
    s = 1.0 if m == 0.0 else min(1.0, lam / m)
    Dual = -0.5 * s * s * float(np.sum(y * y)) - s * float(np.sum(y * delta))
    relgap = (P - Dual) / max(P, 1e-300)
    return P, Dual, relgap


# ---------------------------------------------------------------------------
# The primal-dual solve
# ---------------------------------------------------------------------------

def solve(delta, lam, tau=1.4, sigma=1.4, theta=1.0, max_iter=200,
          gap_tol=0.0, check_every=10, b0=(0.0, 1.0, 0.0), voxel=(1.0, 1.0),
          kind="dipole", history=None, voxel_z=1.0):
    """Primal-dual iteration of the paper's pseudocode on a stack delta[nz, ny, nx].

    Returns (chi, info) with info = {iterations, primal, dual, rel_gap, status}.
    status is "ok" or "nonfinite".  The gap in info is always that of the
    returned iterate.  If `history` is a list, (n, P, Dual, relgap) of every
    check is appended to it.
    """
    delta = np.asarray(delta, dtype=np.float64)
    if delta.ndim == 2:
        delta = delta[None]
    if delta.ndim != 3:
        raise ValueError("delta must be [nz, ny, nx]")
    nz, ny, nx = delta.shape
    D, A = _operator(delta.shape, b0, voxel, kind, voxel_z)
    check_steps(tau, sigma, theta, D)
    if max_iter < 0:
        raise ValueError("max_iter must be >= 0")
    if gap_tol > 0 and check_every < 1:
        raise ValueError("check_every must be >= 1 when gap_tol > 0")

    # initial values: chi_0 = y_0 = 0, chibar_0 = chi_0
    chi = np.zeros_like(delta)
    y = np.zeros_like(delta)
    chibar = chi.copy()
    Ay = np.zeros_like(delta)

    n = 0
    P = Dual = relgap = float("nan")
    status = "ok"
    while n < max_iter:
        y = prox_dual(y + sigma * A(chibar), delta, sigma)
        Ay = A(y)
        chi_new = prox_l1(chi - tau * Ay, tau * lam)
        chibar = chi_new + theta * (chi_new - chi)
        chi = chi_new
        n += 1
        if gap_tol > 0 and (n % check_every == 0 or n == max_iter):
            P, Dual, relgap = duality_gap(chi, y, Ay, delta, D, lam, A)
            if history is not None:
                history.append((n, P, Dual, relgap))
            if not (np.isfinite(P) and np.isfinite(Dual)):
                status = "nonfinite"
                break
            if relgap <= gap_tol:
                break
    if gap_tol <= 0 or n == 0:
        P, Dual, relgap = duality_gap(chi, y, Ay, delta, D, lam, A)
        if not (np.isfinite(P) and np.isfinite(Dual)):
            status = "nonfinite"
    return chi, {"iterations": n, "primal": P, "dual": Dual,
                 "rel_gap": relgap, "status": status}

"""FP64 CPU oracle for the weighted total-variation model of Eq. (1) of
Wang, Cai et al., "Positive Contrast Susceptibility MR Imaging Using GPU-based
Primal-Dual Algorithm" (arXiv:2006.09808).

TEST INFRASTRUCTURE ONLY.  Like pd_oracle, this is the plain reference the HIP
solver's TV model is checked against; only the test-suite, the smoke check and
the benchmark's CPU-baseline leg may import it.  It shares no code with the HIP
library and takes no input or expected value from it.

What it computes (Sec. II-A, Eq. (1) and the PD pseudocode), per 2-D slice:

    minimise over chi   lam/2 || W (D chi - delta) ||_2^2  +  || M G chi ||_1

It is the Chambolle-Pock primal-dual method of Sec. II-A applied to the
saddle-point form of that problem.  Stack the two linear maps into
K chi = (W D chi, M G chi) and write the problem as F(K chi) with
F(z, v) = F1(z) + F2(v), F1(z) = lam/2 ||z - W delta||^2 and F2(v) the sum
over voxels of the Euclidean norm of the gradient 2-vector v(r); chi has no
own term.  One iteration is then three maps, each written below from its
definition: a proximal step on the dual variable y = (p, q) for F* (which
splits into F1* acting on p and F2* acting on q), a plain gradient step on
chi along -K* y (the prox of the zero function is the identity), and the
over-relaxed point chibar at which the next dual step evaluates K.

Readings of the paper used here (it is silent or ambiguous on these points):
  * lam weights the data term, as Eq. (1) prints it and as the pseudocode's
    dual prox (division by 1 + sigma/lam) implies.  (The L1-prior path of
    pd_oracle puts lam on the L1 term instead; that path is a different model.)
  * The dual prox subtracts W delta: Eq. (1) weights the whole residual
    D chi - delta.  The pseudocode's line writes the field map unweighted; the
    two agree for W = I.
  * G is the in-plane (2-D) forward difference, divided by the voxel size
    (dx, dy), with the last difference along each axis set to zero (Neumann
    boundary); slices stay independent (Sec. II-C, strategy (2)).  G* is its
    exact adjoint.  The paper's "all three dimensions" is the 3-D variant,
    which couples slices and is not this model.
  * The L1 norm of the gradient field is the isotropic one (the Euclidean
    norm of (g_x, g_y) per voxel, summed): the pseudocode's q update divides
    the 2-vector by max(1, its norm), the projection onto that norm's dual
    ball.  M multiplies both components.
  * W and M are real, per-voxel (diagonal) operators; D is the dipole kernel
    of pd_oracle (real and even, so D* = D).
  * Step sizes: tau sigma L^2 < 1 strictly, with the bound
    L^2 <= max|W|^2 max|D|^2 + max|M|^2 (4/dx^2 + 4/dy^2) on ||K||^2.
  * Exactly max_iter updates; the result is chi after the last update.  The
    paper's stop rule is the iteration count; no gap is defined here.

The model in three dimensions (kind="dipole3d"): Eq. (1) with both D and G
taken over the whole volume, as Sec. II-A states for the paper's own model.
D is then the 3-D dipole kernel of pd_oracle (dipole_kernel3, apply_A3) and G
the 3-D forward difference (g_x, g_y, g_z), the z difference divided by the
slice thickness voxel_z and zero at the last slice (Neumann, as in-plane);
the norm is the Euclidean norm of the 3-vector per voxel, its dual ball the
unit ball in R^3.  The bound on ||K||^2 gains 4/dz^2.  The slices are then
one coupled problem.  grad_dims=3 with another kernel (the identity) is the
same gradient on a slice-wise operator; the pins use it for closed forms.
"""

import numpy as np

from .pd_oracle import apply_A, dipole_kernel, kernel_norm, _operator

__all__ = ["grad", "grad_adj", "grad_norm_bound", "check_steps_tv", "objective_tv",
           "prox_data_dual", "proj_unit_ball", "apply_K", "apply_K_adj", "prox_dual_tv", "solve_tv",
           "grad3", "grad3_adj", "grad3_norm_bound", "proj_unit_ball3", "check_steps_tv3", "objective_tv3",
           "apply_K3", "apply_K3_adj", "prox_dual_tv3", "solve_tv3"]


# ---------------------------------------------------------------------------
# In-plane gradient G and its adjoint G*
# ---------------------------------------------------------------------------

def grad(x, voxel=(1.0, 1.0)):
    """(g_x, g_y) of x[..., ny, nx]: forward differences divided by the voxel
    size; the last column of g_x and the last row of g_y are zero."""
    x = np.asarray(x, dtype=np.float64)
    dx, dy = float(voxel[0]), float(voxel[1])
    gx = np.zeros_like(x)
    gy = np.zeros_like(x)
    gx[..., :, :-1] = (x[..., :, 1:] - x[..., :, :-1]) / dx
    gy[..., :-1, :] = (x[..., 1:, :] - x[..., :-1, :]) / dy
    return gx, gy


def grad_adj(qx, qy, voxel=(1.0, 1.0)):
    """G* (qx, qy), the adjoint of grad: for each axis, element i receives
    +q[i-1] (if i-1 is a difference the gradient computes) and -q[i] (if i is
    one), divided by the voxel size along that axis."""
    qx = np.asarray(qx, dtype=np.float64)
    qy = np.asarray(qy, dtype=np.float64)
    dx, dy = float(voxel[0]), float(voxel[1])
    out = np.zeros(np.broadcast(qx, qy).shape)
    # x: differences i = 0 .. nx-2 touch elements i (weight -1) and i+1 (+1)
    out[..., :, :-1] -= qx[..., :, :-1] / dx
    out[..., :, 1:] += qx[..., :, :-1] / dx
    out[..., :-1, :] -= qy[..., :-1, :] / dy
    out[..., 1:, :] += qy[..., :-1, :] / dy
    return out


def grad_norm_bound(voxel=(1.0, 1.0)):
    """Upper bound 4/dx^2 + 4/dy^2 on ||G||^2 (each axis' difference operator
    has norm at most 2/d)."""
    dx, dy = float(voxel[0]), float(voxel[1])
    return 4.0 / (dx * dx) + 4.0 / (dy * dy)


def check_steps_tv(tau, sigma, theta, D, W, M, voxel=(1.0, 1.0)):
    """Chambolle-Pock condition tau sigma ||K||^2 < 1 with the bound above."""
    if not (tau > 0 and sigma > 0):
        raise ValueError("tau and sigma must be positive")
    if not (0.0 <= theta <= 1.0):
        raise ValueError("theta must lie in [0, 1]")
    wmax = float(np.max(np.abs(W))) if np.size(W) else 0.0
    mmax = float(np.max(np.abs(M))) if np.size(M) else 0.0
    L2 = wmax * wmax * kernel_norm(D) ** 2 + mmax * mmax * grad_norm_bound(voxel)
    if not (tau * sigma * L2 < 1.0):
        raise ValueError("step sizes violate tau*sigma*||K||^2 < 1")


def objective_tv(chi, delta, W, M, D, lam, voxel=(1.0, 1.0)):
    """lam/2 ||W (A chi - delta)||^2 + sum |M G chi|_2 over the whole stack."""
    r = np.asarray(W) * (apply_A(chi, D) - np.asarray(delta, dtype=np.float64))
    gx, gy = grad(chi, voxel)
    M = np.asarray(M, dtype=np.float64)
    return 0.5 * lam * float(np.sum(r * r)) + float(np.sum(np.sqrt((M * gx) ** 2 + (M * gy) ** 2)))


# ---------------------------------------------------------------------------
# Proximal maps of the two dual terms
# ---------------------------------------------------------------------------

def prox_data_dual(w, b, sigma, lam):
    """prox of sigma F1*, F1*(p) = 1/(2 lam)||p||^2 + <p, b> (b = W delta):
    argmin_p sigma F1*(p) + 1/2||p - w||^2 = (w - sigma b) / (1 + sigma / lam)."""
    return (np.asarray(w, dtype=np.float64) - sigma * np.asarray(b, dtype=np.float64)) / (1.0 + sigma / lam)


def proj_unit_ball(vx, vy):
    """Per-voxel projection of the 2-vector (vx, vy) onto the Euclidean unit
    ball: v / max(1, |v|) (prox of sigma F2* for any sigma)."""
    s = np.maximum(1.0, np.sqrt(vx * vx + vy * vy))
    return vx / s, vy / s


# ---------------------------------------------------------------------------
# The stacked operator K = [W D ; M G] and its adjoint
# ---------------------------------------------------------------------------

def apply_K(x, W, M, D, voxel=(1.0, 1.0)):
    """K x = (W D x, M g_x, M g_y): the data-term image and the masked
    gradient field of x."""
    gx, gy = grad(x, voxel)
    return W * apply_A(x, D), M * gx, M * gy


def apply_K_adj(p, qx, qy, W, M, D, voxel=(1.0, 1.0)):
    """K* (p, q) = D* W* p + G* M* q, with D, W and M real and diagonal in
    their own domains (D* = D since the kernel is real and even)."""
    return apply_A(W * p, D) + grad_adj(M * qx, M * qy, voxel)


def prox_dual_tv(p, qx, qy, b, sigma, lam):
    """prox of sigma F* at (p, q): F* is separable, so the data block takes
    prox_data_dual and every voxel's gradient 2-vector its unit-ball
    projection."""
    return (prox_data_dual(p, b, sigma, lam),) + proj_unit_ball(qx, qy)


# ---------------------------------------------------------------------------
# The primal-dual solve
# ---------------------------------------------------------------------------

def solve_tv(delta, weight, mask, lam, tau, sigma, theta=1.0, max_iter=200,
             b0=(0.0, 1.0, 0.0), voxel=(1.0, 1.0), kind="dipole", history=None,
             voxel_z=1.0, grad_dims=None):
    """The primal-dual iteration of Sec. II-A for Eq. (1) on a stack
    delta[nz, ny, nx] with weights W and mask M of the same shape.

    kind="dipole3d" (or grad_dims=3) solves the model in three dimensions
    (solve_tv3 below); otherwise every slice is its own 2-D problem.

    Returns (chi, info) with info = {iterations, objective}.  If `history` is a
    list, the objective after every update is appended to it.
    """
    dims = grad_dims if grad_dims is not None else (3 if kind == "dipole3d" else 2)
    if dims not in (2, 3):
        raise ValueError("grad_dims must be 2 or 3")
    if kind == "dipole3d" and dims != 3:
        raise ValueError("the 3-D dipole kernel goes with the 3-D gradient")
    if dims == 3:
        return solve_tv3(delta, weight, mask, lam, tau, sigma, theta, max_iter, b0, voxel, kind, history, voxel_z)
    delta = np.asarray(delta, dtype=np.float64)
    if delta.ndim == 2:
        delta = delta[None]
    if delta.ndim != 3:
        raise ValueError("delta must be [nz, ny, nx]")
    W = np.broadcast_to(np.asarray(weight, dtype=np.float64), delta.shape)
    M = np.broadcast_to(np.asarray(mask, dtype=np.float64), delta.shape)
    if not lam > 0:
        raise ValueError("lam must be positive")
    if max_iter < 0:
        raise ValueError("max_iter must be >= 0")
    nz, ny, nx = delta.shape
    D = dipole_kernel(nx, ny, b0, voxel, kind)
    check_steps_tv(tau, sigma, theta, D, W, M, voxel)

    b = W * delta
    # initial values: chi_0 = p_0 = q_0 = 0, chibar_0 = chi_0
    chi = np.zeros_like(delta)
    p = np.zeros_like(delta)
    qx = np.zeros_like(delta)
    qy = np.zeros_like(delta)
    chibar = chi.copy()
    for _ in range(max_iter):
        # dual: y <- prox_{sigma F*}(y + sigma K chibar)
        kp, kx, ky = apply_K(chibar, W, M, D, voxel)
        p, qx, qy = prox_dual_tv(p + sigma * kp, qx + sigma * kx, qy + sigma * ky, b, sigma, lam)
        # primal: chi <- chi - tau K* y (no own term for chi)
        chi_new = chi - tau * apply_K_adj(p, qx, qy, W, M, D, voxel)
        # over-relaxation
        chibar = chi_new + theta * (chi_new - chi)
        chi = chi_new
        if history is not None:
            history.append(objective_tv(chi, delta, W, M, D, lam, voxel))
    return chi, {"iterations": int(max_iter),
                 "objective": objective_tv(chi, delta, W, M, D, lam, voxel)}


# ---------------------------------------------------------------------------
# The model in three dimensions: 3-D gradient (and, for kind="dipole3d", the
# 3-D dipole kernel over the whole volume)
# ---------------------------------------------------------------------------

def grad3(x, voxel=(1.0, 1.0, 1.0)):
    """(g_x, g_y, g_z) of x[nz, ny, nx]: forward differences along each axis
    divided by that axis' voxel size (dx, dy, dz); the last difference along
    each axis is zero."""
    x = np.asarray(x, dtype=np.float64)
    if x.ndim != 3:
        raise ValueError("x must be [nz, ny, nx]")
    dx, dy, dz = (float(v) for v in voxel)
    g = [np.zeros_like(x) for _ in range(3)]
    g[0][:, :, :-1] = (x[:, :, 1:] - x[:, :, :-1]) / dx
    g[1][:, :-1, :] = (x[:, 1:, :] - x[:, :-1, :]) / dy
    g[2][:-1, :, :] = (x[1:, :, :] - x[:-1, :, :]) / dz
    return tuple(g)


def grad3_adj(qx, qy, qz, voxel=(1.0, 1.0, 1.0)):
    """G3* (qx, qy, qz), the adjoint of grad3: per axis, a difference taken
    between elements i and i+1 gives -q[i]/d to element i and +q[i]/d to
    element i+1."""
    qs = [np.asarray(q, dtype=np.float64) for q in (qx, qy, qz)]
    dx, dy, dz = (float(v) for v in voxel)
    out = np.zeros(qs[0].shape)
    out[:, :, :-1] -= qs[0][:, :, :-1] / dx
    out[:, :, 1:] += qs[0][:, :, :-1] / dx
    out[:, :-1, :] -= qs[1][:, :-1, :] / dy
    out[:, 1:, :] += qs[1][:, :-1, :] / dy
    out[:-1, :, :] -= qs[2][:-1, :, :] / dz
    out[1:, :, :] += qs[2][:-1, :, :] / dz
    return out


def grad3_norm_bound(voxel=(1.0, 1.0, 1.0)):
    """Upper bound 4/dx^2 + 4/dy^2 + 4/dz^2 on ||G3||^2."""
    return sum(4.0 / (float(d) * float(d)) for d in voxel)


def proj_unit_ball3(vx, vy, vz):
    """Per-voxel projection of the 3-vector (vx, vy, vz) onto the Euclidean
    unit ball (the prox of sigma F2* for the 3-D gradient's norm)."""
    s = np.maximum(1.0, np.sqrt(vx * vx + vy * vy + vz * vz))
    return vx / s, vy / s, vz / s


def check_steps_tv3(tau, sigma, theta, D, W, M, voxel=(1.0, 1.0, 1.0)):
    """tau sigma ||K||^2 < 1 with ||K||^2 <= max|W|^2 max|D|^2 + max|M|^2
    (4/dx^2 + 4/dy^2 + 4/dz^2)."""
    if not (tau > 0 and sigma > 0):
        raise ValueError("tau and sigma must be positive")
    if not (0.0 <= theta <= 1.0):
        raise ValueError("theta must lie in [0, 1]")
    wmax = float(np.max(np.abs(W))) if np.size(W) else 0.0
    mmax = float(np.max(np.abs(M))) if np.size(M) else 0.0
    L2 = wmax * wmax * kernel_norm(D) ** 2 + mmax * mmax * grad3_norm_bound(voxel)
    if not (tau * sigma * L2 < 1.0):
        raise ValueError("step sizes violate tau*sigma*||K||^2 < 1")


def objective_tv3(chi, delta, W, M, A, lam, voxel=(1.0, 1.0, 1.0)):
    """lam/2 ||W (A chi - delta)||^2 + sum over voxels |M G3 chi|_2, with A
    the operator as a function."""
    r = np.asarray(W) * (A(chi) - np.asarray(delta, dtype=np.float64))
    gx, gy, gz = grad3(chi, voxel)
    M = np.asarray(M, dtype=np.float64)
    return 0.5 * lam * float(np.sum(r * r)) + float(np.sum(M * np.sqrt(gx * gx + gy * gy + gz * gz)))


def apply_K3(x, W, M, A, voxel=(1.0, 1.0, 1.0)):
    """K x = (W A x, M g_x, M g_y, M g_z)."""
    gx, gy, gz = grad3(x, voxel)
    return W * A(x), M * gx, M * gy, M * gz


def apply_K3_adj(p, qx, qy, qz, W, M, A, voxel=(1.0, 1.0, 1.0)):
    """K* (p, q) = A* W p + G3* M q (A self-adjoint: its D is real and even)."""
    return A(W * p) + grad3_adj(M * qx, M * qy, M * qz, voxel)


def prox_dual_tv3(p, qx, qy, qz, b, sigma, lam):
    """prox of sigma F* at (p, q) for the 3-D gradient: the data block as in
    two dimensions, each voxel's 3-vector onto the unit ball."""
    return (prox_data_dual(p, b, sigma, lam),) + proj_unit_ball3(qx, qy, qz)


def solve_tv3(delta, weight, mask, lam, tau, sigma, theta=1.0, max_iter=200,
              b0=(0.0, 1.0, 0.0), voxel=(1.0, 1.0), kind="dipole3d", history=None, voxel_z=1.0):
    """The primal-dual iteration of Sec. II-A for Eq. (1) in three
    dimensions on the volume delta[nz, ny, nx]: K = [W A; M G3] with A the
    3-D dipole operator (kind="dipole3d") or the slice-wise one of `kind`."""
    delta = np.asarray(delta, dtype=np.float64)
    if delta.ndim == 2:
        delta = delta[None]
    if delta.ndim != 3:
        raise ValueError("delta must be [nz, ny, nx]")
    W = np.broadcast_to(np.asarray(weight, dtype=np.float64), delta.shape)
    M = np.broadcast_to(np.asarray(mask, dtype=np.float64), delta.shape)
    if not lam > 0:
        raise ValueError("lam must be positive")
    if max_iter < 0:
        raise ValueError("max_iter must be >= 0")
    if not (np.isfinite(voxel_z) and voxel_z > 0):
        raise ValueError("voxel_z must be positive")
    vox3 = (float(voxel[0]), float(voxel[1]), float(voxel_z))
    D, A = _operator(delta.shape, b0, voxel, kind, voxel_z)
    check_steps_tv3(tau, sigma, theta, D, W, M, vox3)

    b = W * delta
    chi = np.zeros_like(delta)
    y = [np.zeros_like(delta) for _ in range(4)]   # p, q_x, q_y, q_z
    chibar = chi.copy()
    for _ in range(max_iter):
        # dual: y <- prox_{sigma F*}(y + sigma K chibar)
        k = apply_K3(chibar, W, M, A, vox3)
        y = list(prox_dual_tv3(*[yi + sigma * ki for yi, ki in zip(y, k)], b, sigma, lam))
        # primal: plain step along -K* y, then over-relaxation
        chi_new = chi - tau * apply_K3_adj(*y, W, M, A, vox3)
        chibar = chi_new + theta * (chi_new - chi)
        chi = chi_new
        if history is not None:
            history.append(objective_tv3(chi, delta, W, M, A, lam, vox3))
    return chi, {"iterations": int(max_iter), "objective": objective_tv3(chi, delta, W, M, A, lam, vox3)}

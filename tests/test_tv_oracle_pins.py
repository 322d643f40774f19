"""Pins for the FP64 oracle of the weighted TV model (Eq. (1)) against facts
that do not come from the oracle: the gradient written out element by element,
its adjoint identity, the closed-form norm of the Neumann difference operator,
the projection's variational inequality, a dense-matrix run of the iteration,
and closed-form minimisers (1-D TV denoising of a step; the unregularised
weighted fit).  The model in three dimensions (3-D gradient, 3-D dipole
kernel) has the same pins along z, plus its reductions to the 2-D model on a
single slice and on a volume constant along z.  Planted mistakes at the end show that plausible slips in the
oracle fail these pins.
"""

import numpy as np
import pytest
from scipy import optimize

import oracle as O
from test_oracle_pins import dense_A_from_cosines, dense_A3_from_cosines


# ---------------------------------------------------------------------------
# helpers independent of the oracle
# ---------------------------------------------------------------------------

def dense_grad(nx, ny, voxel):
    """Dense G_x, G_y on an ny x nx slice from the definition: row r of G_x
    is (e_{r+1} - e_r)/dx unless r sits in the last column (then zero)."""
    dx, dy = voxel
    n = nx * ny
    Gx = np.zeros((n, n))
    Gy = np.zeros((n, n))
    for y in range(ny):
        for x in range(nx):
            r = y * nx + x
            if x + 1 < nx:
                Gx[r, r + 1] = 1.0 / dx
                Gx[r, r] = -1.0 / dx
            if y + 1 < ny:
                Gy[r, r + nx] = 1.0 / dy
                Gy[r, r] = -1.0 / dy
    return Gx, Gy


def dense_pd_tv(A, Gx, Gy, w, m, d, lam, tau, sigma, theta, iters):
    """The iteration on one slice with explicit matrices; the isotropic
    projection is written per voxel from its definition."""
    n = A.shape[0]
    W = np.diag(w)
    Mm = np.diag(m)
    chi = np.zeros(n)
    p = np.zeros(n)
    qx = np.zeros(n)
    qy = np.zeros(n)
    cb = chi.copy()
    for _ in range(iters):
        p = (p + sigma * (W @ (A @ cb) - W @ d)) / (1.0 + sigma / lam)
        vx = qx + sigma * (Mm @ (Gx @ cb))
        vy = qy + sigma * (Mm @ (Gy @ cb))
        for i in range(n):
            nrm = np.hypot(vx[i], vy[i])
            s = 1.0 if nrm <= 1.0 else nrm
            qx[i], qy[i] = vx[i] / s, vy[i] / s
        new = chi - tau * (A.T @ (W.T @ p)) - tau * (Gx.T @ (Mm.T @ qx) + Gy.T @ (Mm.T @ qy))
        cb = new + theta * (new - chi)
        chi = new
    return chi


# ---------------------------------------------------------------------------
# gradient and adjoint
# ---------------------------------------------------------------------------

def test_grad_matches_elementwise_definition():
    rng = np.random.default_rng(1)
    x = rng.normal(size=(2, 3, 4))
    dx, dy = 0.7, 1.3
    gx, gy = O.grad(x, (dx, dy))
    for z in range(2):
        for j in range(3):
            for i in range(4):
                ex = (x[z, j, i + 1] - x[z, j, i]) / dx if i < 3 else 0.0
                ey = (x[z, j + 1, i] - x[z, j, i]) / dy if j < 2 else 0.0
                assert gx[z, j, i] == pytest.approx(ex, abs=1e-15)
                assert gy[z, j, i] == pytest.approx(ey, abs=1e-15)


@pytest.mark.parametrize("shape", [(1, 5, 7), (3, 8, 8), (1, 1, 9), (2, 6, 1), (1, 16, 12)])
@pytest.mark.parametrize("voxel", [(1.0, 1.0), (0.72, 2.0)])
def test_grad_adjoint_identity(shape, voxel):
    rng = np.random.default_rng(2)
    x = rng.normal(size=shape)
    qx = rng.normal(size=shape)
    qy = rng.normal(size=shape)
    gx, gy = O.grad(x, voxel)
    lhs = np.sum(gx * qx) + np.sum(gy * qy)
    rhs = np.sum(x * O.grad_adj(qx, qy, voxel))
    assert lhs == pytest.approx(rhs, rel=1e-13, abs=1e-13)


def test_grad_equals_dense_definition_matrix():
    nx, ny, vox = 5, 4, (0.8, 1.3)
    Gx, Gy = dense_grad(nx, ny, vox)
    rng = np.random.default_rng(3)
    x = rng.normal(size=(ny, nx))
    gx, gy = O.grad(x, vox)
    np.testing.assert_allclose(gx.ravel(), Gx @ x.ravel(), atol=1e-14)
    np.testing.assert_allclose(gy.ravel(), Gy @ x.ravel(), atol=1e-14)
    qx, qy = rng.normal(size=(ny, nx)), rng.normal(size=(ny, nx))
    np.testing.assert_allclose(O.grad_adj(qx, qy, vox).ravel(), Gx.T @ qx.ravel() + Gy.T @ qy.ravel(), atol=1e-14)


@pytest.mark.parametrize("nx,ny,vox", [(6, 5, (0.8, 1.3)), (8, 8, (1.0, 1.0)), (3, 7, (2.0, 0.5))])
def test_grad_norm_closed_form(nx, ny, vox):
    # G*G = L_x/dx^2 (x) I + I (x) L_y/dy^2 with L the 1-D Neumann Laplacian,
    # whose eigenvalues are 4 sin^2(pi k / (2 n)), k = 0..n-1
    cols = []
    for r in range(nx * ny):
        e = np.zeros(nx * ny)
        e[r] = 1.0
        gx, gy = O.grad(e.reshape(ny, nx), vox)
        cols.append(np.concatenate([gx.ravel(), gy.ravel()]))
    G = np.array(cols).T
    top = np.linalg.eigvalsh(G.T @ G)[-1]
    dx, dy = vox
    expect = 4 * np.sin(np.pi * (nx - 1) / (2 * nx)) ** 2 / dx ** 2 + 4 * np.sin(np.pi * (ny - 1) / (2 * ny)) ** 2 / dy ** 2
    assert top == pytest.approx(expect, rel=1e-12)
    assert top <= O.grad_norm_bound(vox)


# ---------------------------------------------------------------------------
# proximal maps
# ---------------------------------------------------------------------------

def test_projection_is_the_euclidean_projection():
    rng = np.random.default_rng(4)
    vx, vy = rng.normal(size=200) * 2, rng.normal(size=200) * 2
    px, py = O.proj_unit_ball(vx, vy)
    nv = np.hypot(vx, vy)
    inside = nv <= 1
    np.testing.assert_allclose(px[inside], vx[inside], atol=0)
    np.testing.assert_allclose(np.hypot(px[~inside], py[~inside]), 1.0, rtol=1e-15)
    # variational inequality <v - P v, u - P v> <= 0 for every u in the ball
    for _ in range(20):
        ang = rng.uniform(0, 2 * np.pi, size=200)
        rad = np.sqrt(rng.uniform(0, 1, size=200))
        ux, uy = rad * np.cos(ang), rad * np.sin(ang)
        assert np.all((vx - px) * (ux - px) + (vy - py) * (uy - py) <= 1e-14)


@pytest.mark.parametrize("w,b,sigma,lam", [(1.0, 0.3, 0.3, 2.0), (-2.0, 1.0, 0.5, 0.1), (0.0, -4.0, 2.0, 50.0)])
def test_prox_data_dual_bruteforce(w, b, sigma, lam):
    # sigma F1*(p) + 1/2 (p - w)^2 with F1*(p) = p^2/(2 lam) + p b
    f = lambda p: sigma * (p * p / (2 * lam) + p * b) + 0.5 * (p - w) ** 2
    res = optimize.minimize_scalar(f, bounds=(-100, 100), method="bounded", options=dict(xatol=1e-12))
    assert O.prox_data_dual(w, b, sigma, lam) == pytest.approx(res.x, abs=1e-8)


def test_step_condition_uses_weight_mask_and_voxel():
    D = O.dipole_kernel(8, 8)
    W = np.full((1, 8, 8), 0.5)
    M = np.ones((1, 8, 8))
    L2 = 0.25 * (2.0 / 3.0) ** 2 + 8.0
    t = 1.0 / np.sqrt(L2)
    O.check_steps_tv(0.999 * t, t, 1.0, D, W, M)
    with pytest.raises(ValueError):
        O.check_steps_tv(1.001 * t, t, 1.0, D, W, M)
    # anisotropic voxel: bound 4/dx^2 + 4/dy^2
    L2v = 0.25 * (2.0 / 3.0) ** 2 + 4.0 / 0.25 + 4.0
    tv = 1.0 / np.sqrt(L2v)
    with pytest.raises(ValueError):
        O.check_steps_tv(1.001 * tv, tv, 1.0, D, W, M, voxel=(0.5, 1.0))
    with pytest.raises(ValueError):
        O.check_steps_tv(0.1, 0.1, 1.5, D, W, M)


# ---------------------------------------------------------------------------
# the iteration against a dense-matrix run
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("shape,b0,vox", [((4, 4), (0, 1, 0), (1.0, 1.0)), ((3, 5), (0.3, 0.5, 0.8), (0.8, 1.2)),
                                          ((6, 4), (1, 1, 0), (1.0, 0.7))])
@pytest.mark.parametrize("iters", [1, 6, 40])
def test_tv_pd_equals_dense_matrix_pd(shape, b0, vox, iters):
    ny, nx = shape
    rng = np.random.default_rng(10 + iters)
    d = rng.normal(size=(ny, nx)) * 3
    w = rng.uniform(0.2, 1.0, size=(ny, nx))
    m = (rng.uniform(size=(ny, nx)) > 0.3).astype(float) * rng.uniform(0.5, 1.0, size=(ny, nx))
    lam, tau, sigma, theta = 4.0, 0.25, 0.3, 1.0
    D = O.dipole_kernel(nx, ny, b0, vox)
    A = dense_A_from_cosines(D)
    Gx, Gy = dense_grad(nx, ny, vox)
    ref = dense_pd_tv(A, Gx, Gy, w.ravel(), m.ravel(), d.ravel(), lam, tau, sigma, theta, iters)
    chi, info = O.solve_tv(d[None], w[None], m[None], lam, tau, sigma, theta, iters, b0=b0, voxel=vox)
    assert info["iterations"] == iters
    np.testing.assert_allclose(chi[0].ravel(), ref, rtol=0, atol=1e-11 * max(1.0, np.max(np.abs(ref))))


def test_dense_case_exercises_the_projection():
    # the 40-iteration dense case reaches |q| = 1 (the projection binds)
    ny, nx = 3, 5
    rng = np.random.default_rng(10 + 40)
    d = rng.normal(size=(ny, nx)) * 3
    w = rng.uniform(0.2, 1.0, size=(ny, nx))
    m = (rng.uniform(size=(ny, nx)) > 0.3).astype(float) * rng.uniform(0.5, 1.0, size=(ny, nx))
    D = O.dipole_kernel(nx, ny, (0.3, 0.5, 0.8), (0.8, 1.2))
    Gx, Gy = dense_grad(nx, ny, (0.8, 1.2))
    A = dense_A_from_cosines(D)
    n = nx * ny
    chi = np.zeros(n); p = np.zeros(n); qx = np.zeros(n); qy = np.zeros(n); cb = chi.copy()
    bound = 0
    for _ in range(40):
        p = (p + 0.3 * (w.ravel() * (A @ cb) - w.ravel() * d.ravel())) / (1 + 0.3 / 4.0)
        vx = qx + 0.3 * m.ravel() * (Gx @ cb)
        vy = qy + 0.3 * m.ravel() * (Gy @ cb)
        nv = np.hypot(vx, vy)
        bound += int(np.sum(nv > 1))
        s = np.maximum(1, nv)
        qx, qy = vx / s, vy / s
        new = chi - 0.25 * (A.T @ (w.ravel() * p)) - 0.25 * (Gx.T @ (m.ravel() * qx) + Gy.T @ (m.ravel() * qy))
        cb = 2 * new - chi
        chi = new
    assert bound > 0


def test_tv_slices_are_independent():
    rng = np.random.default_rng(5)
    d = rng.normal(size=(3, 6, 8))
    w = rng.uniform(0.5, 1, size=d.shape)
    m = rng.uniform(0, 1, size=d.shape)
    chi, _ = O.solve_tv(d, w, m, 3.0, 0.3, 0.3, 1.0, 25)
    for z in range(3):
        cz, _ = O.solve_tv(d[z:z + 1], w[z:z + 1], m[z:z + 1], 3.0, 0.3, 0.3, 1.0, 25)
        np.testing.assert_allclose(chi[z], cz[0], atol=1e-14)


# ---------------------------------------------------------------------------
# closed-form minimisers
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("axis,d_step", [("x", 1.0), ("x", 0.5), ("y", 2.0)])
def test_tv_denoising_of_a_step_has_the_closed_form_plateaus(axis, d_step):
    # min lam/2 ||chi - delta||^2 + sum |chi_{i+1} - chi_i| / d  on a step of
    # heights (a, b) over (nL, nR) voxels: two plateaus a + 1/(lam d nL) and
    # b - 1/(lam d nR) while the jump stays positive.  Rows are identical, so
    # the isotropic norm reduces to |g| along the step's axis.
    nL, nR, a, b, lam = 5, 3, 0.0, 4.0, 1.0
    line = np.array([a] * nL + [b] * nR)
    reps = 3
    if axis == "x":
        delta = np.tile(line, (reps, 1))
        vox = (d_step, 1.3)
    else:
        delta = np.tile(line[:, None], (1, reps))
        vox = (1.3, d_step)
    ny, nx = delta.shape
    L2 = 1.0 + O.grad_norm_bound(vox)
    t = 0.99 / np.sqrt(L2)
    chi, _ = O.solve_tv(delta[None], 1.0, 1.0, lam, t, t, 1.0, 6000, voxel=vox, kind="identity")
    expect_line = np.array([a + 1 / (lam * d_step * nL)] * nL + [b - 1 / (lam * d_step * nR)] * nR)
    expect = np.tile(expect_line, (reps, 1)) if axis == "x" else np.tile(expect_line[:, None], (1, reps))
    np.testing.assert_allclose(chi[0], expect, atol=1e-7)


def test_unregularised_weighted_fit_recovers_the_field():
    # M = 0: min lam/2 ||W (chi - delta)||^2 with W > 0 is solved by chi = delta
    rng = np.random.default_rng(6)
    delta = rng.normal(size=(2, 6, 6))
    w = rng.uniform(0.5, 1.0, size=delta.shape)
    chi, info = O.solve_tv(delta, w, 0.0, 2.0, 0.9, 0.9, 1.0, 400, kind="identity")
    np.testing.assert_allclose(chi, delta, atol=1e-9)
    assert info["objective"] == pytest.approx(0.0, abs=1e-15)


def test_zero_iterations_give_zero():
    d = np.ones((1, 4, 4))
    chi, info = O.solve_tv(d, 1.0, 1.0, 1.0, 0.1, 0.1, 1.0, 0)
    assert np.all(chi == 0) and info["iterations"] == 0


# ---------------------------------------------------------------------------
# planted mistakes
# ---------------------------------------------------------------------------

def _plant(monkeypatch, name, fn):
    monkeypatch.setattr(O.pd_tv_oracle, name, fn)


def _dense_pin_passes():
    try:
        test_tv_pd_equals_dense_matrix_pd((3, 5), (0.3, 0.5, 0.8), (0.8, 1.2), 40)
        return True
    except AssertionError:
        return False


def _step_pin_passes():
    try:
        test_tv_denoising_of_a_step_has_the_closed_form_plateaus("x", 0.5)
        return True
    except AssertionError:
        return False


def test_planted_adjoint_sign_is_caught(monkeypatch):
    good = O.pd_tv_oracle.grad_adj
    _plant(monkeypatch, "grad_adj", lambda qx, qy, voxel=(1.0, 1.0): -good(qx, qy, voxel))
    assert not _dense_pin_passes()


def test_planted_unweighted_field_term_is_caught(monkeypatch):
    # subtracting delta instead of W delta in the data-term dual prox
    good = O.pd_tv_oracle.prox_data_dual
    _plant(monkeypatch, "prox_data_dual",
           lambda w, b, sigma, lam: good(w, b, sigma, lam) + 0.1 * sigma * b / (1.0 + sigma / lam))
    assert not _dense_pin_passes()


def test_planted_anisotropic_projection_is_caught(monkeypatch):
    _plant(monkeypatch, "proj_unit_ball", lambda vx, vy: (np.clip(vx, -1, 1), np.clip(vy, -1, 1)))
    assert not _dense_pin_passes()


def test_planted_swapped_voxel_axes_is_caught(monkeypatch):
    good = O.pd_tv_oracle.grad
    good_adj = O.pd_tv_oracle.grad_adj
    _plant(monkeypatch, "grad", lambda x, voxel=(1.0, 1.0): good(x, (voxel[1], voxel[0])))
    _plant(monkeypatch, "grad_adj", lambda qx, qy, voxel=(1.0, 1.0): good_adj(qx, qy, (voxel[1], voxel[0])))
    assert not _step_pin_passes()


def test_planted_missing_lam_in_dual_prox_is_caught(monkeypatch):
    good = O.pd_tv_oracle.prox_data_dual
    _plant(monkeypatch, "prox_data_dual", lambda w, b, sigma, lam: good(w, b, sigma, 1.0))
    assert not _dense_pin_passes()


# ---------------------------------------------------------------------------
# the model in three dimensions
# ---------------------------------------------------------------------------

def dense_grad3(nx, ny, nz, voxel3):
    """Dense G_x, G_y, G_z on an nz x ny x nx volume from the definition."""
    dx, dy, dz = voxel3
    n = nx * ny * nz
    G = [np.zeros((n, n)) for _ in range(3)]
    for z in range(nz):
        for y in range(ny):
            for x in range(nx):
                r = (z * ny + y) * nx + x
                for a, (ok, step, d) in enumerate(((x + 1 < nx, 1, dx), (y + 1 < ny, nx, dy),
                                                   (z + 1 < nz, nx * ny, dz))):
                    if ok:
                        G[a][r, r + step] = 1.0 / d
                        G[a][r, r] = -1.0 / d
    return G


def dense_pd_tv3(A, G, w, m, d, lam, tau, sigma, theta, iters):
    """The iteration on a volume with explicit matrices; the projection onto
    the unit ball of R^3 written per voxel."""
    n = A.shape[0]
    chi = np.zeros(n)
    p = np.zeros(n)
    q = [np.zeros(n) for _ in range(3)]
    cb = chi.copy()
    for _ in range(iters):
        p = (p + sigma * (w * (A @ cb) - w * d)) / (1.0 + sigma / lam)
        v = [q[a] + sigma * m * (G[a] @ cb) for a in range(3)]
        for i in range(n):
            nrm = np.sqrt(v[0][i] ** 2 + v[1][i] ** 2 + v[2][i] ** 2)
            s = max(1.0, nrm)
            for a in range(3):
                q[a][i] = v[a][i] / s
        new = chi - tau * (A.T @ (w * p)) - tau * sum(G[a].T @ (m * q[a]) for a in range(3))
        cb = new + theta * (new - chi)
        chi = new
    return chi


def test_grad3_matches_elementwise_definition():
    rng = np.random.default_rng(21)
    x = rng.normal(size=(3, 4, 5))
    vox = (0.7, 1.3, 2.1)
    gx, gy, gz = O.grad3(x, vox)
    for z in range(3):
        for j in range(4):
            for i in range(5):
                assert gx[z, j, i] == pytest.approx((x[z, j, i + 1] - x[z, j, i]) / 0.7 if i < 4 else 0.0, abs=1e-15)
                assert gy[z, j, i] == pytest.approx((x[z, j + 1, i] - x[z, j, i]) / 1.3 if j < 3 else 0.0, abs=1e-15)
                assert gz[z, j, i] == pytest.approx((x[z + 1, j, i] - x[z, j, i]) / 2.1 if z < 2 else 0.0, abs=1e-15)


@pytest.mark.parametrize("shape", [(1, 5, 7), (4, 3, 3), (9, 1, 1), (2, 6, 1), (5, 8, 6)])
@pytest.mark.parametrize("voxel3", [(1.0, 1.0, 1.0), (0.72, 2.0, 1.5)])
def test_grad3_adjoint_identity(shape, voxel3):
    rng = np.random.default_rng(22)
    x = rng.normal(size=shape)
    q = [rng.normal(size=shape) for _ in range(3)]
    g = O.grad3(x, voxel3)
    lhs = sum(np.sum(g[a] * q[a]) for a in range(3))
    rhs = np.sum(x * O.grad3_adj(*q, voxel3))
    assert lhs == pytest.approx(rhs, rel=1e-13, abs=1e-13)


def test_grad3_equals_dense_definition_matrix():
    nx, ny, nz, vox = 4, 3, 3, (0.8, 1.3, 1.9)
    G = dense_grad3(nx, ny, nz, vox)
    rng = np.random.default_rng(23)
    x = rng.normal(size=(nz, ny, nx))
    g = O.grad3(x, vox)
    for a in range(3):
        np.testing.assert_allclose(g[a].ravel(), G[a] @ x.ravel(), atol=1e-14)
    q = [rng.normal(size=(nz, ny, nx)) for _ in range(3)]
    np.testing.assert_allclose(O.grad3_adj(*q, vox).ravel(), sum(G[a].T @ q[a].ravel() for a in range(3)),
                               atol=1e-14)


@pytest.mark.parametrize("shape,vox", [((3, 4, 5), (0.8, 1.3, 2.0)), ((4, 4, 4), (1.0, 1.0, 1.0)),
                                       ((6, 2, 3), (2.0, 0.5, 0.7))])
def test_grad3_norm_closed_form(shape, vox):
    # G3*G3 is the sum over axes of the 1-D Neumann Laplacian / d^2 (Kronecker
    # sum), so its top eigenvalue is the sum of the axes' 4 sin^2(pi (n-1) / (2n)) / d^2
    nz, ny, nx = shape
    G = np.vstack(dense_grad3(nx, ny, nz, vox))
    top = np.linalg.eigvalsh(G.T @ G)[-1]
    expect = sum(4 * np.sin(np.pi * (n - 1) / (2 * n)) ** 2 / d ** 2 for n, d in zip((nx, ny, nz), vox))
    assert top == pytest.approx(expect, rel=1e-12)
    assert top <= O.grad3_norm_bound(vox)


def test_projection3_is_the_euclidean_projection():
    rng = np.random.default_rng(24)
    v = [rng.normal(size=300) * 2 for _ in range(3)]
    pr = O.proj_unit_ball3(*v)
    nv = np.sqrt(sum(c * c for c in v))
    inside = nv <= 1
    for a in range(3):
        np.testing.assert_allclose(pr[a][inside], v[a][inside], atol=0)
    np.testing.assert_allclose(np.sqrt(sum(c[~inside] ** 2 for c in pr)), 1.0, rtol=1e-15)
    for _ in range(20):
        u = rng.normal(size=(3, 300))
        u *= (rng.uniform(size=300) ** (1 / 3)) / np.linalg.norm(u, axis=0)
        assert np.all(sum((v[a] - pr[a]) * (u[a] - pr[a]) for a in range(3)) <= 1e-14)


def test_step_condition_3d_adds_the_z_term():
    D = O.dipole_kernel3(4, 4, 4)
    W = np.full((4, 4, 4), 0.5)
    M = np.ones((4, 4, 4))
    vox = (1.0, 1.0, 0.5)
    L2 = 0.25 * O.kernel_norm(D) ** 2 + 4.0 + 4.0 + 16.0
    t = 1.0 / np.sqrt(L2)
    O.check_steps_tv3(0.999 * t, t, 1.0, D, W, M, vox)
    with pytest.raises(ValueError):
        O.check_steps_tv3(1.001 * t, t, 1.0, D, W, M, vox)
    # the in-plane bound alone would admit these steps
    O.check_steps_tv(1.2 * t, t, 1.0, D, W, M, vox[:2])


def _tv3_case(shape, seed):
    rng = np.random.default_rng(seed)
    d = rng.normal(size=shape) * 3
    w = rng.uniform(0.2, 1.0, size=shape)
    m = (rng.uniform(size=shape) > 0.3).astype(float) * rng.uniform(0.5, 1.0, size=shape)
    return d, w, m


@pytest.mark.parametrize("shape,b0,vox,vz", [((2, 3, 4), (0.3, 0.5, 0.8), (1.0, 0.8), 1.6),
                                             ((3, 2, 3), (0.0, 0.0, 1.0), (1.0, 1.0), 1.0),
                                             ((4, 3, 2), (1.0, 1.0, 0.5), (0.9, 1.1), 0.7)])
@pytest.mark.parametrize("iters", [1, 6, 40])
def test_tv3_pd_equals_dense_matrix_pd(shape, b0, vox, vz, iters):
    nz, ny, nx = shape
    d, w, m = _tv3_case(shape, 30 + iters)
    lam, tau, sigma, theta = 4.0, 0.2, 0.25, 1.0
    D = O.dipole_kernel3(nx, ny, nz, b0, vox, vz)
    A = dense_A3_from_cosines(D)
    G = dense_grad3(nx, ny, nz, (vox[0], vox[1], vz))
    ref = dense_pd_tv3(A, G, w.ravel(), m.ravel(), d.ravel(), lam, tau, sigma, theta, iters)
    chi, info = O.solve_tv(d, w, m, lam, tau, sigma, theta, iters, b0=b0, voxel=vox, kind="dipole3d", voxel_z=vz)
    assert info["iterations"] == iters
    np.testing.assert_allclose(chi.ravel(), ref, rtol=0, atol=1e-11 * max(1.0, np.max(np.abs(ref))))


def test_tv3_dense_case_exercises_the_projection_with_z():
    # in the 40-iteration dense case the 3-vector projection binds, and z
    # carries part of the projected norm there
    d, w, m = _tv3_case((2, 3, 4), 70)
    D = O.dipole_kernel3(4, 3, 2, (0.3, 0.5, 0.8), (1.0, 0.8), 1.6)
    A = dense_A3_from_cosines(D)
    G = dense_grad3(4, 3, 2, (1.0, 0.8, 1.6))
    n = 24
    chi = np.zeros(n); cb = chi.copy(); p = np.zeros(n); q = [np.zeros(n) for _ in range(3)]
    bound_z = 0
    for _ in range(40):
        p = (p + 0.25 * (w.ravel() * (A @ cb) - w.ravel() * d.ravel())) / (1 + 0.25 / 4.0)
        v = [q[a] + 0.25 * m.ravel() * (G[a] @ cb) for a in range(3)]
        nv = np.sqrt(sum(c * c for c in v))
        bound_z += int(np.sum((nv > 1) & (np.abs(v[2]) > 1e-3)))
        q = [c / np.maximum(1, nv) for c in v]
        new = chi - 0.2 * (A @ (w.ravel() * p)) - 0.2 * sum(G[a].T @ (m.ravel() * q[a]) for a in range(3))
        cb = 2 * new - chi
        chi = new
    assert bound_z > 0


def test_tv3_single_slice_is_the_2d_model():
    # nz = 1: D3 is the 2-D kernel (its kz = 0 plane) and the z difference vanishes
    d, w, m = _tv3_case((1, 6, 8), 40)
    args = (d, w, m, 3.0, 0.2, 0.25, 1.0, 30)
    c3, _ = O.solve_tv(*args, b0=(0.3, 0.5, 0.8), voxel=(0.9, 1.2), kind="dipole3d", voxel_z=0.6)
    c2, _ = O.solve_tv(*args, b0=(0.3, 0.5, 0.8), voxel=(0.9, 1.2))
    np.testing.assert_allclose(c3, c2, atol=1e-12)


def test_tv3_on_z_constant_volume_is_the_2d_model():
    # delta, W and M constant along z: A3 acts as the slice operator on
    # z-constant volumes, G3 adds a zero z component, so every iterate stays
    # z-constant and equals the 2-D iterate of one slice
    d, w, m = _tv3_case((1, 6, 8), 41)
    D3 = np.broadcast_to(d, (4, 6, 8)).copy()
    W3 = np.broadcast_to(w, (4, 6, 8)).copy()
    M3 = np.broadcast_to(m, (4, 6, 8)).copy()
    c3, _ = O.solve_tv(D3, W3, M3, 3.0, 0.2, 0.25, 1.0, 30, b0=(0.3, 0.5, 0.8), kind="dipole3d", voxel_z=1.7)
    c2, _ = O.solve_tv(d, w, m, 3.0, 0.2, 0.25, 1.0, 30, b0=(0.3, 0.5, 0.8))
    for z in range(4):
        np.testing.assert_allclose(c3[z], c2[0], atol=1e-12)


@pytest.mark.parametrize("dz", [1.0, 0.5, 2.0])
def test_tv3_denoising_of_a_z_step_has_the_closed_form_plateaus(dz):
    # identity operator, chi constant in-plane and a step along z over
    # (nL, nR) slices: the plateaus a + 1/(lam dz nL), b - 1/(lam dz nR)
    nL, nR, a, b, lam = 4, 3, 0.0, 4.0, 1.0
    line = np.array([a] * nL + [b] * nR)
    delta = np.broadcast_to(line[:, None, None], (nL + nR, 3, 2)).copy()
    vox = (1.3, 0.9)
    L2 = 1.0 + O.grad3_norm_bound((vox[0], vox[1], dz))
    t = 0.99 / np.sqrt(L2)
    chi, _ = O.solve_tv(delta, 1.0, 1.0, lam, t, t, 1.0, 6000, voxel=vox, kind="identity", voxel_z=dz,
                        grad_dims=3)
    expect = np.array([a + 1 / (lam * dz * nL)] * nL + [b - 1 / (lam * dz * nR)] * nR)
    np.testing.assert_allclose(chi, np.broadcast_to(expect[:, None, None], chi.shape), atol=1e-7)


def test_tv3_couples_the_slices():
    # unlike the slice-wise model, changing one slice's field moves the others
    d, w, m = _tv3_case((3, 4, 4), 42)
    c0, _ = O.solve_tv(d, w, m, 3.0, 0.2, 0.25, 1.0, 10, kind="dipole3d")
    d2 = d.copy()
    d2[2] += 1.0
    c1, _ = O.solve_tv(d2, w, m, 3.0, 0.2, 0.25, 1.0, 10, kind="dipole3d")
    assert np.max(np.abs(c1[0] - c0[0])) > 1e-3


def _dense3_pin_passes():
    try:
        test_tv3_pd_equals_dense_matrix_pd((2, 3, 4), (0.3, 0.5, 0.8), (1.0, 0.8), 1.6, 40)
        return True
    except AssertionError:
        return False


def _zstep_pin_passes():
    try:
        test_tv3_denoising_of_a_z_step_has_the_closed_form_plateaus(0.5)
        return True
    except AssertionError:
        return False


def test_planted_z_adjoint_sign_is_caught(monkeypatch):
    good = O.pd_tv_oracle.grad3_adj
    def bad(qx, qy, qz, voxel=(1.0, 1.0, 1.0)):
        return good(qx, qy, 0 * qz, voxel) - (good(0 * qx, 0 * qy, qz, voxel))
    _plant(monkeypatch, "grad3_adj", bad)
    assert not _dense3_pin_passes()


def test_planted_in_plane_projection_in_3d_is_caught(monkeypatch):
    # projecting (q_x, q_y) and q_z separately instead of the 3-vector
    good2 = O.pd_tv_oracle.proj_unit_ball
    _plant(monkeypatch, "proj_unit_ball3",
           lambda vx, vy, vz: good2(vx, vy) + (np.clip(vz, -1, 1),))
    assert not _dense3_pin_passes()


def test_planted_ignored_slice_thickness_in_gradient_is_caught(monkeypatch):
    good = O.pd_tv_oracle.grad3
    good_adj = O.pd_tv_oracle.grad3_adj
    _plant(monkeypatch, "grad3", lambda x, voxel=(1.0, 1.0, 1.0): good(x, (voxel[0], voxel[1], 1.0)))
    _plant(monkeypatch, "grad3_adj",
           lambda qx, qy, qz, voxel=(1.0, 1.0, 1.0): good_adj(qx, qy, qz, (voxel[0], voxel[1], 1.0)))
    assert not _zstep_pin_passes()


def test_planted_slice_wise_kernel_in_3d_is_caught(monkeypatch):
    # the 2-D kernel per slice in place of the 3-D kernel over the volume
    import oracle.pd_oracle as L1
    good = L1._operator
    def slicewise(shape, b0, voxel, kind, voxel_z):
        return good(shape, b0, voxel, "dipole" if kind == "dipole3d" else kind, voxel_z)
    _plant(monkeypatch, "_operator", slicewise)
    assert not _dense3_pin_passes()
